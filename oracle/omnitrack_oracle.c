/*
 * omnitrack_oracle.c -- plain FP64 CPU reference of the pyramidal
 * Lucas-Kanade box-tracking path.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code
 * with the HIP library.  Written for clarity, not speed: every value is
 * recomputed from its definition in double precision, with no blocking or
 * reordering beyond what the definitions state.  Built with -O2
 * -ffp-contract=off and without fast-math.
 *
 * What it computes (OmniTrack, arXiv 1910.06017, Sec. V-A):
 *   preprocessing  -- each frame is reduced by a Gaussian pyramid;
 *   feature calc.  -- motion between the frames (here sparse pyramidal
 *                     Lucas-Kanade on point grids instead of the paper's
 *                     dense TV-L1 field of Sec. IV);
 *   prediction     -- each box moves by the motion of its points (the paper
 *                     averages; the median is the default here).
 * The Lucas-Kanade steps follow the published methods: Burt & Adelson 1983
 * (binomial reduce), Scharr 2000 (3x3 derivative), Shi & Tomasi 1994
 * (minimum-eigenvalue test), Lucas & Kanade 1981 with the coarse-to-fine
 * scheme of Bouguet 2000 (pyramidal Lucas-Kanade feature tracker).
 */
#include "omnitrack_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int32_t clampi(int32_t v, int32_t lo, int32_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

void orc_level_dims(int32_t W, int32_t H, int32_t levels, int32_t* w, int32_t* h) {
    w[0] = W;
    h[0] = H;
    for (int32_t l = 1; l < levels; ++l) {
        w[l] = (w[l - 1] + 1) / 2;
        h[l] = (h[l - 1] + 1) / 2;
    }
}

/* ---------------------------------------------------------------------------
 * Gaussian pyramid (paper Sec. V-A preprocessing; kernel per Burt-Adelson):
 * P_l(x,y) = round( sum_{i,j=-2..2} k_i k_j P_{l-1}(clamp(2x+i), clamp(2y+j)) / 256 )
 * with k = (1,4,6,4,1), rounding half up: (s + 128) >> 8 on the exact sum.
 * ------------------------------------------------------------------------- */
static const int32_t K5[5] = {1, 4, 6, 4, 1};

void orc_pyr_down(const uint8_t* src, int32_t sw, int32_t sh, int32_t spitch, uint8_t* dst) {
    int32_t dw = (sw + 1) / 2, dh = (sh + 1) / 2;
    for (int32_t y = 0; y < dh; ++y) {
        for (int32_t x = 0; x < dw; ++x) {
            int32_t s = 0;
            for (int32_t j = -2; j <= 2; ++j) {
                int32_t yy = clampi(2 * y + j, 0, sh - 1);
                int32_t row = 0;
                for (int32_t i = -2; i <= 2; ++i) {
                    int32_t xx = clampi(2 * x + i, 0, sw - 1);
                    row += K5[i + 2] * (int32_t)src[(size_t)yy * spitch + xx];
                }
                s += K5[j + 2] * row;
            }
            dst[(size_t)y * dw + x] = (uint8_t)((s + 128) >> 8);
        }
    }
}

void orc_pyr_down_direct(const uint8_t* src, int32_t sw, int32_t sh, int32_t spitch,
                         uint8_t* dst) {
    /* 5x5 weight table written out (outer product of the binomial row). */
    static const int32_t W55[5][5] = {{1, 4, 6, 4, 1},
                                      {4, 16, 24, 16, 4},
                                      {6, 24, 36, 24, 6},
                                      {4, 16, 24, 16, 4},
                                      {1, 4, 6, 4, 1}};
    int32_t dw = (sw + 1) / 2, dh = (sh + 1) / 2;
    for (int32_t y = 0; y < dh; ++y)
        for (int32_t x = 0; x < dw; ++x) {
            double s = 0.0;
            for (int32_t j = 0; j < 5; ++j)
                for (int32_t i = 0; i < 5; ++i) {
                    int32_t yy = clampi(2 * y + j - 2, 0, sh - 1);
                    int32_t xx = clampi(2 * x + i - 2, 0, sw - 1);
                    s += (double)W55[j][i] * (double)src[(size_t)yy * spitch + xx];
                }
            /* round half up of the exact rational s/256 */
            dst[(size_t)y * dw + x] = (uint8_t)floor(s / 256.0 + 0.5);
        }
}

void orc_pyramid(const uint8_t* frame, int32_t W, int32_t H, int32_t pitch, int32_t levels,
                 uint8_t* out) {
    int32_t w[32], h[32];
    orc_level_dims(W, H, levels, w, h);
    const uint8_t* src = frame;
    int32_t sp = pitch;
    uint8_t* dst = out;
    for (int32_t l = 1; l < levels; ++l) {
        orc_pyr_down(src, w[l - 1], h[l - 1], sp, dst);
        src = dst;
        sp = w[l];
        dst += (size_t)w[l] * h[l];
    }
}

/* ---------------------------------------------------------------------------
 * Scharr derivative (Scharr 2000): smoothing (3,10,3) across, central
 * difference along; dividing by 32 gives gray levels per pixel.
 * ------------------------------------------------------------------------- */
void orc_scharr(const uint8_t* img, int32_t w, int32_t h, int32_t* sx, int32_t* sy) {
    static const int32_t S3[3] = {3, 10, 3};
    for (int32_t y = 0; y < h; ++y)
        for (int32_t x = 0; x < w; ++x) {
            int32_t ax = 0, ay = 0;
            for (int32_t t = -1; t <= 1; ++t) {
                int32_t yt = clampi(y + t, 0, h - 1), xt = clampi(x + t, 0, w - 1);
                int32_t xl = clampi(x - 1, 0, w - 1), xr = clampi(x + 1, 0, w - 1);
                int32_t yu = clampi(y - 1, 0, h - 1), yd = clampi(y + 1, 0, h - 1);
                ax += S3[t + 1] * ((int32_t)img[(size_t)yt * w + xr] - (int32_t)img[(size_t)yt * w + xl]);
                ay += S3[t + 1] * ((int32_t)img[(size_t)yd * w + xt] - (int32_t)img[(size_t)yu * w + xt]);
            }
            sx[(size_t)y * w + x] = ax;
            sy[(size_t)y * w + x] = ay;
        }
}

/* ---------------------------------------------------------------------------
 * Bilinear interpolation: x0 = floor(x), a = x - x0 (same for y);
 * F = (1-a)(1-b) F00 + a(1-b) F10 + (1-a) b F01 + a b F11, taps clamped.
 * ------------------------------------------------------------------------- */
#define BILINEAR_BODY(T)                                                          \
    double fx = floor(x), fy = floor(y);                                          \
    double a = x - fx, b = y - fy;                                                \
    int32_t x0 = (int32_t)fmax(fmin(fx, 1e9), -1e9);                              \
    int32_t y0 = (int32_t)fmax(fmin(fy, 1e9), -1e9);                              \
    int32_t xa = clampi(x0, 0, w - 1), xb = clampi(x0 + 1, 0, w - 1);             \
    int32_t ya = clampi(y0, 0, h - 1), yb = clampi(y0 + 1, 0, h - 1);             \
    double f00 = (double)img[(size_t)ya * w + xa], f10 = (double)img[(size_t)ya * w + xb]; \
    double f01 = (double)img[(size_t)yb * w + xa], f11 = (double)img[(size_t)yb * w + xb]; \
    return (1 - a) * (1 - b) * f00 + a * (1 - b) * f10 + (1 - a) * b * f01 + a * b * f11;

double orc_bilinear_u8(const uint8_t* img, int32_t w, int32_t h, double x, double y) {
    BILINEAR_BODY(uint8_t)
}

double orc_bilinear_i32(const int32_t* img, int32_t w, int32_t h, double x, double y) {
    BILINEAR_BODY(int32_t)
}

double orc_min_eig(const double* G) {
    double m = 0.5 * (G[0] + G[2]);
    double d = 0.5 * (G[0] - G[2]);
    return m - sqrt(d * d + G[1] * G[1]);
}

double orc_structure_tensor(const uint8_t* img, int32_t w, int32_t h, double cx, double cy,
                            int32_t win, double* G) {
    int32_t r = win / 2;
    int32_t* sx = (int32_t*)malloc(sizeof(int32_t) * (size_t)w * h);
    int32_t* sy = (int32_t*)malloc(sizeof(int32_t) * (size_t)w * h);
    orc_scharr(img, w, h, sx, sy);
    G[0] = G[1] = G[2] = 0.0;
    for (int32_t oy = -r; oy <= r; ++oy)
        for (int32_t ox = -r; ox <= r; ++ox) {
            double X = orc_bilinear_i32(sx, w, h, cx + ox, cy + oy) / 32.0;
            double Y = orc_bilinear_i32(sy, w, h, cx + ox, cy + oy) / 32.0;
            G[0] += X * X;
            G[1] += X * Y;
            G[2] += Y * Y;
        }
    free(sx);
    free(sy);
    return orc_min_eig(G);
}

/* ---------------------------------------------------------------------------
 * Pyramidal Lucas-Kanade for one point (Bouguet 2000):
 *   g = 0 at the coarsest level; for level l = L-1 .. 0, c = u / 2^l:
 *     template A(o) = I(c+o), gradients X(o), Y(o) (bilinear, o in window)
 *     G = sum [X^2 XY; XY Y^2]; lost when lambda_min(G)/N < min_eig
 *     nu = 0; repeat up to `iters` times:
 *        B(o) = J(c + g + nu + o);  d = A - B;  b = sum d [X, Y]
 *        eta = G^{-1} b;  nu += eta;  stop once |eta|^2 < eps^2
 *     g = 2 (g + nu) when l > 0, else flow = g + nu
 *   next = u + flow; lost when non-finite or outside the frame.
 *   err = mean over the level-0 window of |I(u+o) - J(next+o)|.
 * ------------------------------------------------------------------------- */
typedef struct {
    const uint8_t* const* prev;
    const uint8_t* const* next;
    const int32_t* w;
    const int32_t* h;
    int32_t* const* sx;  /* Scharr of prev, per level */
    int32_t* const* sy;
    int32_t levels, win, iters;
    double eps, min_eig;
} lk_ctx;

static void lk_one_point(const lk_ctx* C, double ux, double uy, double* out_xy,
                         uint8_t* status, double* err, int32_t* it_out, double* lam_out,
                         int32_t* reason) {
    const int32_t L = C->levels, r = C->win / 2, N = C->win * C->win;
    const double W0 = C->w[0], H0 = C->h[0];
    double* A = (double*)malloc(sizeof(double) * 3 * (size_t)N);
    double* X = A + N;
    double* Y = X + N;
    for (int32_t l = 0; l < L; ++l) {
        if (it_out) it_out[l] = 0;
        if (lam_out) lam_out[l] = 0.0;
    }
    out_xy[0] = ux;
    out_xy[1] = uy;
    *status = 0;
    *err = -1.0;
    *reason = ORC_BAD_INPUT;
    if (!isfinite(ux) || !isfinite(uy) || ux < 0 || uy < 0 || ux > W0 - 1 || uy > H0 - 1) {
        free(A);
        return;
    }
    double gx = 0.0, gy = 0.0, fx = 0.0, fy = 0.0;
    for (int32_t l = L - 1; l >= 0; --l) {
        const int32_t w = C->w[l], h = C->h[l];
        const double scale = ldexp(1.0, l);
        const double cx = ux / scale, cy = uy / scale;
        double G0 = 0, G1 = 0, G2 = 0;
        int32_t k = 0;
        for (int32_t oy = -r; oy <= r; ++oy)
            for (int32_t ox = -r; ox <= r; ++ox, ++k) {
                A[k] = orc_bilinear_u8(C->prev[l], w, h, cx + ox, cy + oy);
                X[k] = orc_bilinear_i32(C->sx[l], w, h, cx + ox, cy + oy) / 32.0;
                Y[k] = orc_bilinear_i32(C->sy[l], w, h, cx + ox, cy + oy) / 32.0;
                G0 += X[k] * X[k];
                G1 += X[k] * Y[k];
                G2 += Y[k] * Y[k];
            }
        double Gm[3] = {G0, G1, G2};
        double lam = orc_min_eig(Gm) / N;
        if (lam_out) lam_out[l] = lam;
        if (!(lam >= C->min_eig)) {
            out_xy[0] = ux + gx * scale;
            out_xy[1] = uy + gy * scale;
            *reason = ORC_GATED;
            free(A);
            return;
        }
        const double det = G0 * G2 - G1 * G1;
        double nux = 0.0, nuy = 0.0;
        int32_t it = 0;
        while (it < C->iters) {
            double bx = 0.0, by = 0.0;
            k = 0;
            for (int32_t oy = -r; oy <= r; ++oy)
                for (int32_t ox = -r; ox <= r; ++ox, ++k) {
                    double B = orc_bilinear_u8(C->next[l], w, h, cx + gx + nux + ox,
                                               cy + gy + nuy + oy);
                    double d = A[k] - B;
                    bx += d * X[k];
                    by += d * Y[k];
                }
            double ex = (G2 * bx - G1 * by) / det;
            double ey = (G0 * by - G1 * bx) / det;
            nux += ex;
            nuy += ey;
            ++it;
            if (ex * ex + ey * ey < C->eps * C->eps) break;
        }
        if (it_out) it_out[l] = it;
        if (l > 0) {
            gx = 2.0 * (gx + nux);
            gy = 2.0 * (gy + nuy);
        } else {
            fx = gx + nux;
            fy = gy + nuy;
        }
    }
    const double nx = ux + fx, ny = uy + fy;
    out_xy[0] = nx;
    out_xy[1] = ny;
    if (!isfinite(nx) || !isfinite(ny) || nx < 0 || ny < 0 || nx > W0 - 1 || ny > H0 - 1) {
        *reason = ORC_OUT_OF_FRAME;
        free(A);
        return;
    }
    double e = 0.0;
    for (int32_t oy = -r; oy <= r; ++oy)
        for (int32_t ox = -r; ox <= r; ++ox)
            e += fabs(orc_bilinear_u8(C->prev[0], C->w[0], C->h[0], ux + ox, uy + oy) -
                      orc_bilinear_u8(C->next[0], C->w[0], C->h[0], nx + ox, ny + oy));
    *err = e / N;
    *status = 1;
    *reason = ORC_OK;
    free(A);
}

int32_t orc_lk_track(const uint8_t* const* prev, const uint8_t* const* next,
                     const int32_t* w, const int32_t* h, int32_t levels,
                     const float* pts, int32_t n, int32_t win, int32_t iters,
                     double eps, double min_eig,
                     double* next_pts, uint8_t* status, double* err,
                     int32_t* iters_out, double* lam_out, int32_t* reason,
                     int32_t nthreads) {
    if (levels < 1 || levels > 16 || win < 3 || (win & 1) == 0 || iters < 1 || n < 0)
        return -1;
    int32_t* sx[16];
    int32_t* sy[16];
    for (int32_t l = 0; l < levels; ++l) {
        sx[l] = (int32_t*)malloc(sizeof(int32_t) * (size_t)w[l] * h[l]);
        sy[l] = (int32_t*)malloc(sizeof(int32_t) * (size_t)w[l] * h[l]);
        orc_scharr(prev[l], w[l], h[l], sx[l], sy[l]);
    }
    lk_ctx C = {prev, next, w, h, sx, sy, levels, win, iters, eps, min_eig};
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads)
#endif
    for (int32_t i = 0; i < n; ++i) {
        int32_t rs;
        double e;
        uint8_t st;
        lk_one_point(&C, (double)pts[2 * i], (double)pts[2 * i + 1], next_pts + 2 * (size_t)i,
                     &st, &e, iters_out ? iters_out + (size_t)i * levels : NULL,
                     lam_out ? lam_out + (size_t)i * levels : NULL, &rs);
        status[i] = st;
        err[i] = e;
        if (reason) reason[i] = rs;
    }
    for (int32_t l = 0; l < levels; ++l) {
        free(sx[l]);
        free(sy[l]);
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Box prediction (paper Sec. V-A prediction phase): every box moves by the
 * motion of its own tracked points; the median of an even count is the mean
 * of the two middle values.
 * ------------------------------------------------------------------------- */
static int cmp_double(const void* a, const void* b) {
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

static double median_sorted(const double* v, int32_t c) {
    return (c & 1) ? v[c / 2] : 0.5 * (v[c / 2 - 1] + v[c / 2]);
}

void orc_box_update(const double* boxes, int32_t m, const int32_t* box_id,
                    const double* pts, const double* next_pts, const uint8_t* status,
                    int32_t n, int32_t use_mean, double* out_boxes, int32_t* out_count) {
    double* dx = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* dy = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int32_t b = 0; b < m; ++b) {
        int32_t c = 0;
        for (int32_t i = 0; i < n; ++i)
            if (box_id[i] == b && status[i] == 1) {
                dx[c] = next_pts[2 * (size_t)i] - pts[2 * (size_t)i];
                dy[c] = next_pts[2 * (size_t)i + 1] - pts[2 * (size_t)i + 1];
                ++c;
            }
        double mx = 0.0, my = 0.0;
        if (c > 0) {
            if (use_mean) {
                for (int32_t i = 0; i < c; ++i) {
                    mx += dx[i];
                    my += dy[i];
                }
                mx /= c;
                my /= c;
            } else {
                qsort(dx, (size_t)c, sizeof(double), cmp_double);
                qsort(dy, (size_t)c, sizeof(double), cmp_double);
                mx = median_sorted(dx, c);
                my = median_sorted(dy, c);
            }
        }
        out_boxes[4 * b + 0] = boxes[4 * b + 0] + mx;
        out_boxes[4 * b + 1] = boxes[4 * b + 1] + my;
        out_boxes[4 * b + 2] = boxes[4 * b + 2] + mx;
        out_boxes[4 * b + 3] = boxes[4 * b + 3] + my;
        out_count[b] = c;
    }
    free(dx);
    free(dy);
}

void orc_fb_gate(const double* pts, const double* back_pts, const uint8_t* st_fwd,
                 const uint8_t* st_bwd, int32_t n, double fb_max, double* fb_err,
                 uint8_t* status_out) {
    for (int32_t i = 0; i < n; ++i) {
        if (st_fwd[i] == 1 && st_bwd[i] == 1) {
            const double ex = pts[2 * (size_t)i] - back_pts[2 * (size_t)i];
            const double ey = pts[2 * (size_t)i + 1] - back_pts[2 * (size_t)i + 1];
            const double e = sqrt(ex * ex + ey * ey);
            fb_err[i] = e;
            status_out[i] = (e <= fb_max) ? 1 : 0;
        } else {
            fb_err[i] = -1.0;
            status_out[i] = 0;
        }
    }
}

void orc_box_update_scaled(const double* boxes, int32_t m, const int32_t* box_id,
                           const double* pts, const double* next_pts, const uint8_t* status,
                           int32_t n, double* out_boxes, int32_t* out_count, double* out_scale) {
    int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    double* dx = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* dy = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int32_t b = 0; b < m; ++b) {
        int32_t c = 0;
        for (int32_t i = 0; i < n; ++i)
            if (box_id[i] == b && status[i] == 1) {
                idx[c] = i;
                dx[c] = next_pts[2 * (size_t)i] - pts[2 * (size_t)i];
                dy[c] = next_pts[2 * (size_t)i + 1] - pts[2 * (size_t)i + 1];
                ++c;
            }
        double mx = 0.0, my = 0.0, s = 1.0;
        if (c > 0) {
            qsort(dx, (size_t)c, sizeof(double), cmp_double);
            qsort(dy, (size_t)c, sizeof(double), cmp_double);
            mx = median_sorted(dx, c);
            my = median_sorted(dy, c);
        }
        // scale: all pairs of the box's points
        const size_t np = (size_t)c * (size_t)(c > 0 ? c - 1 : 0) / 2;
        double* r = (double*)malloc(sizeof(double) * (np > 0 ? np : 1));
        int32_t nr = 0;
        for (int32_t a = 0; a < c; ++a)
            for (int32_t q = a + 1; q < c; ++q) {
                const int32_t i = idx[a], j = idx[q];
                const double ux = pts[2 * (size_t)i] - pts[2 * (size_t)j];
                const double uy = pts[2 * (size_t)i + 1] - pts[2 * (size_t)j + 1];
                const double du = sqrt(ux * ux + uy * uy);
                if (du == 0.0) continue;
                const double vx = next_pts[2 * (size_t)i] - next_pts[2 * (size_t)j];
                const double vy = next_pts[2 * (size_t)i + 1] - next_pts[2 * (size_t)j + 1];
                r[nr++] = sqrt(vx * vx + vy * vy) / du;
            }
        if (nr > 0) {
            qsort(r, (size_t)nr, sizeof(double), cmp_double);
            s = median_sorted(r, nr);
        }
        free(r);
        const double cx = 0.5 * (boxes[4 * b + 0] + boxes[4 * b + 2]) + mx;
        const double cy = 0.5 * (boxes[4 * b + 1] + boxes[4 * b + 3]) + my;
        const double hw = 0.5 * (boxes[4 * b + 2] - boxes[4 * b + 0]);
        const double hh = 0.5 * (boxes[4 * b + 3] - boxes[4 * b + 1]);
        if (c > 0) {
            out_boxes[4 * b + 0] = cx - s * hw;
            out_boxes[4 * b + 1] = cy - s * hh;
            out_boxes[4 * b + 2] = cx + s * hw;
            out_boxes[4 * b + 3] = cy + s * hh;
        } else {
            for (int k = 0; k < 4; ++k) out_boxes[4 * b + k] = boxes[4 * b + k];
        }
        out_count[b] = c;
        out_scale[b] = s;
    }
    free(idx);
    free(dx);
    free(dy);
}

int32_t orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
