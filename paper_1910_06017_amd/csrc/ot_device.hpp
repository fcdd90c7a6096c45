// ot_device.hpp -- gfx950 device code of the pyramidal Lucas-Kanade tracker:
// wave64 DPP reductions, the pyramid reduce tile, the per-point tracker and
// the per-box median.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ot_common.hpp"

namespace ot {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

__device__ __forceinline__ float uniform_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// One DPP move of a float across lanes (GFX9 DPP control codes); lanes whose
// source is outside the row, or rows masked off, read 0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xF, true));
}

// Sum over the 64 lanes of a wave; every lane gets the total.  Within a row
// of 16 lanes: two quad permutes, half-row mirror and row mirror leave the row
// total in every lane; row_bcast:15 and row_bcast:31 then fold the four row
// totals into lane 63, which is broadcast.  All 64 lanes must be active.
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_f<0xB1>(v);       // quad_perm [1,0,3,2]
    v += dpp_f<0x4E>(v);       // quad_perm [2,3,0,1]
    v += dpp_f<0x141>(v);      // row_half_mirror
    v += dpp_f<0x140>(v);      // row_mirror
    v += dpp_f<0x142, 0xA>(v); // row_bcast:15 -> rows 1, 3
    v += dpp_f<0x143, 0xC>(v); // row_bcast:31 -> rows 2, 3
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Workgroup b runs on XCD b % 8; hand each XCD one contiguous range of work
// items so neighbouring points share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int G) {
    const int X = 8;
    const int q = G / X, rem = G % X;
    const int xcd = b % X, k = b / X;
    return (xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q) + k;
}

// ---------------------------------------------------------------------------
// Gaussian pyramid reduce of one PYR_TW x PYR_TH output tile (binomial
// (1,4,6,4,1) in both directions, clamp-to-edge, exact integer sum rounded
// half up).  256 threads.
// ---------------------------------------------------------------------------
struct PyrSmem {
    uint8_t in[2 * PYR_TH + 3][2 * PYR_TW + 4];
    int32_t hs[2 * PYR_TH + 3][PYR_TW];
};

__device__ __forceinline__ void pyr_tile(const uint8_t* __restrict__ src, int sw, int sh, int sp,
                                         uint8_t* __restrict__ dst, int dw, int dh, int dp,
                                         int tx, int ty, PyrSmem& sm) {
    const int tid = threadIdx.x;
    const int ox0 = tx * PYR_TW, oy0 = ty * PYR_TH;
    const int ix0 = 2 * ox0 - 2, iy0 = 2 * oy0 - 2;
    constexpr int IR = 2 * PYR_TH + 3, IC = 2 * PYR_TW + 3;
    const bool interior = ix0 >= 0 && iy0 >= 0 && ix0 + IC <= sw && iy0 + IR <= sh;
    if (interior) {
        for (int e = tid; e < IR * IC; e += PYR_THREADS) {
            const int r = e / IC, c = e - r * IC;
            sm.in[r][c] = src[(size_t)(iy0 + r) * sp + ix0 + c];
        }
    } else {
        for (int e = tid; e < IR * IC; e += PYR_THREADS) {
            const int r = e / IC, c = e - r * IC;
            const int y = clampi(iy0 + r, 0, sh - 1), x = clampi(ix0 + c, 0, sw - 1);
            sm.in[r][c] = src[(size_t)y * sp + x];
        }
    }
    __syncthreads();
    for (int e = tid; e < IR * PYR_TW; e += PYR_THREADS) {
        const int r = e / PYR_TW, c = e - r * PYR_TW;
        const uint8_t* p = &sm.in[r][2 * c];
        sm.hs[r][c] = (int)p[0] + 4 * (int)p[1] + 6 * (int)p[2] + 4 * (int)p[3] + (int)p[4];
    }
    __syncthreads();
    for (int e = tid; e < PYR_TH * PYR_TW; e += PYR_THREADS) {
        const int r = e / PYR_TW, c = e - r * PYR_TW;
        const int y = oy0 + r, x = ox0 + c;
        if (y < dh && x < dw) {
            const int s = sm.hs[2 * r][c] + 4 * sm.hs[2 * r + 1][c] + 6 * sm.hs[2 * r + 2][c] +
                          4 * sm.hs[2 * r + 3][c] + sm.hs[2 * r + 4][c];
            dst[(size_t)y * dp + x] = (uint8_t)((s + 128) >> 8);
        }
    }
}

// ---------------------------------------------------------------------------
// Lucas-Kanade for one point, one wave64 per point.
//
// Lane mapping: the win x win window is split into win columns x nseg row
// segments; lane = seg * win + col owns the R consecutive window rows
// seg*R .. seg*R+R-1 of column col (lanes past win*nseg own nothing).  Each
// lane keeps its template, x- and y-gradient samples in registers, so a
// Lucas-Kanade iteration reads only the target image.
//
// LDS (per wave): during a level's set-up, the raw template patch (uint8)
// and the Scharr gradients at the bilinear tap grid; during iterations, the
// target region with a `margin` border, stored as (J[x], J[x+1]-J[x]) pairs
// so each bilinear row blend is one FMA.  Regions are restaged only when the
// estimate walks out of the margin.
// ---------------------------------------------------------------------------
struct LkGeom {
    int win, r, nseg, RR, TW, PW, M, SC, SR;
    __device__ LkGeom(int win_, int R, int margin) {
        win = win_;
        r = win >> 1;
        nseg = min(win, max(1, 64 / win));
        RR = nseg * R + 1;  // tap rows held (>= win + 1)
        TW = win + 1;       // tap columns
        PW = (TW + 2 + 3) & ~3;
        M = margin;
        SC = TW + 2 * M;
        SR = RR + 2 * M;
    }
};

struct LkResult {
    float nx, ny, err;
    int status;
};

template <int R, class PyrRef>
__device__ __forceinline__ LkResult lk_point(const PyrRef& P, const PyrRef& Q, float ux, float uy,
                                             int L, int iters, float eps2, float min_eig,
                                             const LkGeom& g, unsigned char* __restrict__ smem,
                                             uint8_t* iters_out, float* lam_out) {
    const int lane = threadIdx.x & 63;
    const int used = g.win * g.nseg;
    const bool lvalid = lane < used;
    const int col = lvalid ? lane % g.win : 0;
    const int seg = lvalid ? lane / g.win : 0;
    const int row0 = seg * R;
    const int nrows = lvalid ? max(0, min(R, g.win - row0)) : 0;
    const float N = (float)(g.win * g.win);

    LkResult res;
    res.nx = ux;
    res.ny = uy;
    res.err = -1.0f;
    res.status = 0;
    const int W0 = P.w[0], H0 = P.h[0];
    if (!(ux >= 0.0f && uy >= 0.0f && ux <= (float)(W0 - 1) && uy <= (float)(H0 - 1))) {
        if (lane == 0)
            for (int l = 0; l < L; ++l) {
                if (iters_out) iters_out[l] = 0;
                if (lam_out) lam_out[l] = 0.0f;
            }
        return res;  // also catches NaN
    }

    float A[R], X[R], Y[R];
    float gx = 0.0f, gy = 0.0f;
    float nux = 0.0f, nuy = 0.0f;
    float2* jr = reinterpret_cast<float2*>(smem);
    int sx0 = 0, sy0 = 0;  // origin of the staged target region (level coords)

    for (int l = L - 1; l >= 0; --l) {
        const uint8_t* __restrict__ Il = P.lvl[l];
        const uint8_t* __restrict__ Jl = Q.lvl[l];
        const int w = P.w[l], h = P.h[l], ip = P.pitch[l], jp = Q.pitch[l];
        const float sc = __builtin_ldexpf(1.0f, -l);
        const float cx = ux * sc, cy = uy * sc;
        const float flx = floorf(cx), fly = floorf(cy);
        const float ax = cx - flx, ay = cy - fly;
        const int x0 = (int)flx - g.r, y0 = (int)fly - g.r;  // top-left tap

        // ---- template patch (RR+2 rows x TW+2 cols, origin x0-1, y0-1), clamped reads
        uint8_t* patch = smem;
        float2* grad = reinterpret_cast<float2*>(smem + (((g.RR + 2) * g.PW + 15) & ~15));
        for (int e = lane; e < (g.RR + 2) * (g.TW + 2); e += 64) {
            const int pr = e / (g.TW + 2), pc = e - pr * (g.TW + 2);
            const int yy = clampi(y0 - 1 + pr, 0, h - 1), xx = clampi(x0 - 1 + pc, 0, w - 1);
            patch[pr * g.PW + pc] = Il[(size_t)yy * ip + xx];
        }
        __syncthreads();
        // ---- Scharr gradients at the tap grid: the gradient image is defined on
        // the level's pixels and read at clamped indices, so a tap outside the
        // level takes the gradient of the nearest edge pixel.
        for (int e = lane; e < g.RR * g.TW; e += 64) {
            const int ty = e / g.TW, tx = e - ty * g.TW;
            const int qx = clampi(x0 + tx, 0, w - 1), qy = clampi(y0 + ty, 0, h - 1);
            const int xl = max(qx - 1, 0) - (x0 - 1), xc = qx - (x0 - 1), xr = min(qx + 1, w - 1) - (x0 - 1);
            const int yu = max(qy - 1, 0) - (y0 - 1), yc = qy - (y0 - 1), yd = min(qy + 1, h - 1) - (y0 - 1);
            const int pul = patch[yu * g.PW + xl], puc = patch[yu * g.PW + xc], pur = patch[yu * g.PW + xr];
            const int pcl = patch[yc * g.PW + xl], pcr = patch[yc * g.PW + xr];
            const int pdl = patch[yd * g.PW + xl], pdc = patch[yd * g.PW + xc], pdr = patch[yd * g.PW + xr];
            const int sxv = 3 * (pur - pul) + 10 * (pcr - pcl) + 3 * (pdr - pdl);
            const int syv = 3 * (pdl - pul) + 10 * (pdc - puc) + 3 * (pdr - pur);
            grad[e] = make_float2((float)sxv * (1.0f / 32.0f), (float)syv * (1.0f / 32.0f));
        }
        __syncthreads();
        // ---- bilinear template and gradients of this lane's strip
        {
            float pi = 0.0f, px = 0.0f, py = 0.0f;
#pragma unroll
            for (int k = 0; k <= R; ++k) {
                const int ty = row0 + k;
                const float i0 = (float)patch[(ty + 1) * g.PW + col + 1];
                const float i1 = (float)patch[(ty + 1) * g.PW + col + 2];
                const float2 g0 = grad[ty * g.TW + col];
                const float2 g1 = grad[ty * g.TW + col + 1];
                const float ri = fmaf(ax, i1 - i0, i0);
                const float rx = fmaf(ax, g1.x - g0.x, g0.x);
                const float ry = fmaf(ax, g1.y - g0.y, g0.y);
                if (k > 0) {
                    const bool v = (k - 1) < nrows;
                    A[k - 1] = v ? fmaf(ay, ri - pi, pi) : 0.0f;
                    X[k - 1] = v ? fmaf(ay, rx - px, px) : 0.0f;
                    Y[k - 1] = v ? fmaf(ay, ry - py, py) : 0.0f;
                }
                pi = ri;
                px = rx;
                py = ry;
            }
        }
        float gxx = 0.0f, gxy = 0.0f, gyy = 0.0f;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            gxx = fmaf(X[k], X[k], gxx);
            gxy = fmaf(X[k], Y[k], gxy);
            gyy = fmaf(Y[k], Y[k], gyy);
        }
        gxx = wave_sum(gxx);
        gxy = wave_sum(gxy);
        gyy = wave_sum(gyy);
        const float hm = 0.5f * (gxx + gyy), hd = 0.5f * (gxx - gyy);
        const float lam = (hm - sqrtf(hd * hd + gxy * gxy)) / N;
        if (lane == 0 && lam_out) lam_out[l] = lam;
        if (!(lam >= min_eig)) {
            if (lane == 0)
                for (int k = l; k >= 0; --k) {
                    if (iters_out) iters_out[k] = 0;
                    if (lam_out && k < l) lam_out[k] = 0.0f;
                }
            const float s = __builtin_ldexpf(1.0f, l);
            res.nx = ux + gx * s;
            res.ny = uy + gy * s;
            return res;
        }
        const float idet = 1.0f / (gxx * gyy - gxy * gxy);
        __syncthreads();  // the set-up LDS is reused for the target region

        // ---- stage the target region around the level's initial estimate
        auto stage = [&](float fx, float fy) {
            sx0 = (int)fx - g.r - g.M;
            sy0 = (int)fy - g.r - g.M;
            for (int e = lane; e < g.SR * g.SC; e += 64) {
                const int rr = e / g.SC, cc = e - rr * g.SC;
                const int yy = clampi(sy0 + rr, 0, h - 1);
                const int xa = clampi(sx0 + cc, 0, w - 1), xb = clampi(sx0 + cc + 1, 0, w - 1);
                const float v0 = (float)Jl[(size_t)yy * jp + xa];
                const float v1 = (float)Jl[(size_t)yy * jp + xb];
                jr[e] = make_float2(v0, v1 - v0);
            }
            __syncthreads();
        };
        // Positions are clamped before the integer conversion; past the bounds
        // every tap already reads the level's edge, so the samples are unchanged.
        const float lo = -(float)(g.win + 8), hix = (float)(w + g.win + 8), hiy = (float)(h + g.win + 8);
        nux = 0.0f;
        nuy = 0.0f;
        {
            const float qx = fminf(fmaxf(cx + gx, lo), hix), qy = fminf(fmaxf(cy + gy, lo), hiy);
            stage(floorf(qx), floorf(qy));
        }
        int it = 0;
        while (it < iters) {
            const float qx = fminf(fmaxf(cx + gx + nux, lo), hix);
            const float qy = fminf(fmaxf(cy + gy + nuy, lo), hiy);
            const float fqx = floorf(qx), fqy = floorf(qy);
            const float bxw = qx - fqx, byw = qy - fqy;
            int ox = (int)fqx - g.r - sx0, oy = (int)fqy - g.r - sy0;
            if (ox < 0 || oy < 0 || ox > 2 * g.M || oy > 2 * g.M) {
                __syncthreads();
                stage(fqx, fqy);
                ox = g.M;
                oy = g.M;
            }
            const float2* __restrict__ jb = jr + (oy + row0) * g.SC + ox + col;
            float2 t = jb[0];
            float rp = fmaf(bxw, t.y, t.x);
            float bx = 0.0f, by = 0.0f;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                t = jb[(k + 1) * g.SC];
                const float rn = fmaf(bxw, t.y, t.x);
                const float d = A[k] - fmaf(byw, rn - rp, rp);
                bx = fmaf(d, X[k], bx);
                by = fmaf(d, Y[k], by);
                rp = rn;
            }
            bx = wave_sum(bx);
            by = wave_sum(by);
            const float ex = (gyy * bx - gxy * by) * idet;
            const float ey = (gxx * by - gxy * bx) * idet;
            nux += ex;
            nuy += ey;
            ++it;
            if (ex * ex + ey * ey < eps2) break;
        }
        if (lane == 0 && iters_out) iters_out[l] = (uint8_t)min(it, 255);
        if (l > 0) {
            gx = 2.0f * (gx + nux);
            gy = 2.0f * (gy + nuy);
        }
    }
    // level 0: flow = g + nu
    const float fx = gx + nux, fy = gy + nuy;
    const float nx = ux + fx, ny = uy + fy;
    res.nx = nx;
    res.ny = ny;
    if (!(nx >= 0.0f && ny >= 0.0f && nx <= (float)(W0 - 1) && ny <= (float)(H0 - 1))) return res;

    // ---- err: mean |I - J| over the level-0 window at the final position
    {
        const int w = P.w[0], h = P.h[0];
        const float fqx = floorf(nx), fqy = floorf(ny);
        const float bxw = nx - fqx, byw = ny - fqy;
        int ox = (int)fqx - g.r - sx0, oy = (int)fqy - g.r - sy0;
        if (ox < 0 || oy < 0 || ox > 2 * g.M || oy > 2 * g.M) {
            __syncthreads();
            const uint8_t* __restrict__ Jl = Q.lvl[0];
            const int jp = Q.pitch[0];
            sx0 = (int)fqx - g.r - g.M;
            sy0 = (int)fqy - g.r - g.M;
            for (int e = lane; e < g.SR * g.SC; e += 64) {
                const int rr = e / g.SC, cc = e - rr * g.SC;
                const int yy = clampi(sy0 + rr, 0, h - 1);
                const int xa = clampi(sx0 + cc, 0, w - 1), xb = clampi(sx0 + cc + 1, 0, w - 1);
                const float v0 = (float)Jl[(size_t)yy * jp + xa];
                const float v1 = (float)Jl[(size_t)yy * jp + xb];
                jr[e] = make_float2(v0, v1 - v0);
            }
            __syncthreads();
            ox = g.M;
            oy = g.M;
        }
        const float2* __restrict__ jb = jr + (oy + row0) * g.SC + ox + col;
        float2 t = jb[0];
        float rp = fmaf(bxw, t.y, t.x);
        float e = 0.0f;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            t = jb[(k + 1) * g.SC];
            const float rn = fmaf(bxw, t.y, t.x);
            const float d = A[k] - fmaf(byw, rn - rp, rp);
            e += (k < nrows) ? fabsf(d) : 0.0f;
            rp = rn;
        }
        res.err = wave_sum(e) / N;
    }
    res.status = 1;
    return res;
}

// ---------------------------------------------------------------------------
// Per-box median of point displacements: exact radix selection (four 8-bit
// passes over order-preserving integer keys), four selections at once
// (x and y at ranks (c-1)/2 and c/2).  256 threads.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t f2key(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key2f(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

struct BoxSmem {
    float dx[BOX_CAP];
    float dy[BOX_CAP];
    uint32_t hist[4][256];
    uint32_t prefix[4];
    uint32_t rank[4];
    int32_t count;
};

// Visit every selected point of the box as f(dx, dy).  In LDS mode the
// gathered values are visited; otherwise the job's points are re-scanned.
template <class F>
__device__ __forceinline__ void box_visit(bool in_lds, const BoxSmem& sm, int c, int b,
                                          const int32_t* __restrict__ box_id,
                                          const uint8_t* __restrict__ status,
                                          const float* __restrict__ pts,
                                          const float* __restrict__ next_pts, int n, F&& f) {
    if (in_lds) {
        for (int i = threadIdx.x; i < c; i += BOX_THREADS) f(sm.dx[i], sm.dy[i]);
    } else {
        for (int i = threadIdx.x; i < n; i += BOX_THREADS)
            if (box_id[i] == b && status[i] == 1)
                f(next_pts[2 * i] - pts[2 * i], next_pts[2 * i + 1] - pts[2 * i + 1]);
    }
}

__device__ __forceinline__ void box_median(const float* __restrict__ boxes, int b,
                                           const int32_t* __restrict__ box_id,
                                           const float* __restrict__ pts,
                                           const float* __restrict__ next_pts,
                                           const uint8_t* __restrict__ status, int n,
                                           float* __restrict__ out_boxes,
                                           int32_t* __restrict__ out_count, BoxSmem& sm) {
    const int tid = threadIdx.x;
    if (tid == 0) sm.count = 0;
    __syncthreads();
    for (int i = tid; i < n; i += BOX_THREADS) {
        if (box_id[i] == b && status[i] == 1) {
            const int k = atomicAdd(&sm.count, 1);
            if (k < BOX_CAP) {
                sm.dx[k] = next_pts[2 * i] - pts[2 * i];
                sm.dy[k] = next_pts[2 * i + 1] - pts[2 * i + 1];
            }
        }
    }
    __syncthreads();
    const int c = sm.count;
    const bool in_lds = c <= BOX_CAP;
    float mx = 0.0f, my = 0.0f;
    if (c > 0) {
        if (tid < 4) {
            sm.prefix[tid] = 0;
            sm.rank[tid] = (tid & 1) ? (uint32_t)(c / 2) : (uint32_t)((c - 1) / 2);
        }
        for (int pass = 3; pass >= 0; --pass) {
            const int shift = pass * 8;
            for (int e = tid; e < 4 * 256; e += BOX_THREADS) (&sm.hist[0][0])[e] = 0;
            __syncthreads();
            const uint32_t hmask = pass == 3 ? 0u : (0xFFFFFFFFu << (shift + 8));
            const uint32_t p0 = sm.prefix[0] & hmask, p1 = sm.prefix[1] & hmask;
            const uint32_t p2 = sm.prefix[2] & hmask, p3 = sm.prefix[3] & hmask;
            box_visit(in_lds, sm, c, b, box_id, status, pts, next_pts, n, [&](float vx, float vy) {
                const uint32_t kx = f2key(vx), ky = f2key(vy);
                const uint32_t dxk = (kx >> shift) & 255u, dyk = (ky >> shift) & 255u;
                if ((kx & hmask) == p0) atomicAdd(&sm.hist[0][dxk], 1u);
                if ((kx & hmask) == p1) atomicAdd(&sm.hist[1][dxk], 1u);
                if ((ky & hmask) == p2) atomicAdd(&sm.hist[2][dyk], 1u);
                if ((ky & hmask) == p3) atomicAdd(&sm.hist[3][dyk], 1u);
            });
            __syncthreads();
            const int wave = tid >> 6, lane = tid & 63;
            if (wave < 4) {
                // lane owns bins 4*lane .. 4*lane+3; inclusive scan over lanes
                const uint32_t* hs = sm.hist[wave];
                const uint32_t c0 = hs[4 * lane], c1 = hs[4 * lane + 1], c2 = hs[4 * lane + 2],
                               c3 = hs[4 * lane + 3];
                uint32_t tot = c0 + c1 + c2 + c3, incl = tot;
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t v = __shfl_up(incl, o, 64);
                    if (lane >= o) incl += v;
                }
                const uint32_t excl = incl - tot;
                const uint32_t k = sm.rank[wave];
                if (k >= excl && k < incl) {
                    uint32_t base = excl, bin = 4 * lane;
                    const uint32_t cs[4] = {c0, c1, c2, c3};
                    for (int j = 0; j < 4; ++j) {
                        if (k < base + cs[j]) {
                            bin = 4 * lane + j;
                            break;
                        }
                        base += cs[j];
                    }
                    sm.prefix[wave] |= bin << shift;
                    sm.rank[wave] = k - base;
                }
            }
            __syncthreads();
        }
        mx = 0.5f * (key2f(sm.prefix[0]) + key2f(sm.prefix[1]));
        my = 0.5f * (key2f(sm.prefix[2]) + key2f(sm.prefix[3]));
    }
    if (tid == 0) {
        out_boxes[4 * b + 0] = boxes[4 * b + 0] + mx;
        out_boxes[4 * b + 1] = boxes[4 * b + 1] + my;
        out_boxes[4 * b + 2] = boxes[4 * b + 2] + mx;
        out_boxes[4 * b + 3] = boxes[4 * b + 3] + my;
        out_count[b] = c;
    }
}

}  // namespace ot
