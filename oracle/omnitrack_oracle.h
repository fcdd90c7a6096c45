/*
 * omnitrack_oracle.h -- plain FP64 CPU reference of the pyramidal
 * Lucas-Kanade box-tracking path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path (the
 * HIP library and its Python binding) never calls it and shares no code,
 * header, table or helper with it.
 *
 * All pointers are host pointers.  Images are uint8, row-major.  Coordinates
 * are pixels with pixel centres at integers; level l pixel i sits at level-0
 * position 2^l * i.
 */
#ifndef OMNITRACK_ORACLE_H
#define OMNITRACK_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Level sizes: w[0]=W, w[l]=ceil(w[l-1]/2); same for h. */
void orc_level_dims(int32_t W, int32_t H, int32_t levels, int32_t* w, int32_t* h);

/* One pyramid step (Burt-Adelson binomial reduce): dst is ceil(sw/2) x ceil(sh/2),
 * tightly packed; src has row pitch `spitch` bytes. */
void orc_pyr_down(const uint8_t* src, int32_t sw, int32_t sh, int32_t spitch, uint8_t* dst);

/* Same value computed as a direct 5x5 double loop with a per-tap weight table. */
void orc_pyr_down_direct(const uint8_t* src, int32_t sw, int32_t sh, int32_t spitch,
                         uint8_t* dst);

/* Levels 1..levels-1 of a frame, concatenated tightly in level order. */
void orc_pyramid(const uint8_t* frame, int32_t W, int32_t H, int32_t pitch, int32_t levels,
                 uint8_t* out);

/* Integer 3x3 Scharr responses (32 x the gradient in gray levels per pixel),
 * clamp-to-edge reads.  sx, sy are w*h. */
void orc_scharr(const uint8_t* img, int32_t w, int32_t h, int32_t* sx, int32_t* sy);

/* Bilinear interpolation with clamp-to-edge taps. */
double orc_bilinear_u8(const uint8_t* img, int32_t w, int32_t h, double x, double y);
double orc_bilinear_i32(const int32_t* img, int32_t w, int32_t h, double x, double y);

/* Spatial-gradient matrix G = sum over the win x win window centred at (cx,cy)
 * of [Ix^2, IxIy, Iy^2] (gradients in gray levels per pixel, bilinear).
 * G[0]=Gxx, G[1]=Gxy, G[2]=Gyy.  Returns lambda_min(G). */
double orc_structure_tensor(const uint8_t* img, int32_t w, int32_t h, double cx, double cy,
                            int32_t win, double* G);

/* Smaller eigenvalue of the symmetric 2x2 matrix [G0 G1; G1 G2]. */
double orc_min_eig(const double* G);

/* Lost-point reasons written to `reason`. */
enum { ORC_OK = 0, ORC_BAD_INPUT = 1, ORC_GATED = 2, ORC_OUT_OF_FRAME = 3 };

/*
 * Pyramidal iterative Lucas-Kanade tracking of n points from the `prev`
 * pyramid to the `next` pyramid.  prev[l], next[l] are tight w[l] x h[l]
 * images.  pts is n x 2 float32 (x, y) in level-0 pixels.
 * Outputs: next_pts n x 2, status n (1 tracked, 0 lost), err n (mean absolute
 * level-0 window difference on the 0..255 scale, -1 when lost).
 * Optional (may be NULL): iters_out n x levels, lam_out n x levels
 * (lambda_min / win^2 per level, indexed by level), reason n.
 * nthreads <= 0 uses the OpenMP default.  Returns 0, or -1 on bad arguments.
 */
int32_t orc_lk_track(const uint8_t* const* prev, const uint8_t* const* next,
                     const int32_t* w, const int32_t* h, int32_t levels,
                     const float* pts, int32_t n, int32_t win, int32_t iters,
                     double eps, double min_eig,
                     double* next_pts, uint8_t* status, double* err,
                     int32_t* iters_out, double* lam_out, int32_t* reason,
                     int32_t nthreads);

/*
 * Box prediction: for box b, the component-wise median (or mean when
 * use_mean != 0) of next_pts - pts over the points with box_id == b and
 * status == 1; out = box + (mx, my, mx, my) and out_count[b] = that count.
 * A box without such points is copied unchanged with count 0.
 */
void orc_box_update(const double* boxes, int32_t m, const int32_t* box_id,
                    const double* pts, const double* next_pts, const uint8_t* status,
                    int32_t n, int32_t use_mean, double* out_boxes, int32_t* out_count);

/*
 * Forward-backward check (Kalal, Mikolajczyk & Matas 2010): back_pts are the
 * forward results tracked back to the first frame.  fb_err[i] = |pts_i -
 * back_pts_i| (Euclidean) when both tracks succeeded (status 1), else -1;
 * status_out[i] = 1 when both succeeded and fb_err[i] <= fb_max, else 0.
 */
void orc_fb_gate(const double* pts, const double* back_pts, const uint8_t* st_fwd,
                 const uint8_t* st_bwd, int32_t n, double fb_max, double* fb_err,
                 uint8_t* status_out);

/*
 * Median-Flow box update (Kalal et al. 2010) over the points with box_id == b
 * and status == 1 (count c): the displacement (mx, my) is the component-wise
 * median of next_pts - pts as in orc_box_update; the scale s is the median,
 * over the pairs i < j of those points with pts_i != pts_j, of
 * |next_i - next_j| / |pts_i - pts_j| (1 when there is no such pair).  The box
 * centre moves by (mx, my) and its half-extents are multiplied by s:
 * out = (cx - s*hw, cy - s*hh, cx + s*hw, cy + s*hh) with cx = (x0+x1)/2 + mx,
 * hw = (x1-x0)/2, and likewise in y.  A box without points is copied with
 * count 0 and scale 1.
 */
void orc_box_update_scaled(const double* boxes, int32_t m, const int32_t* box_id,
                           const double* pts, const double* next_pts, const uint8_t* status,
                           int32_t n, double* out_boxes, int32_t* out_count, double* out_scale);

/* Number of OpenMP threads a parallel region gets by default. */
int32_t orc_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
