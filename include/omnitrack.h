/*
 * omnitrack.h -- C ABI of the MI355X (gfx950) pyramidal Lucas-Kanade box
 * tracker.
 *
 * The operation is the tracking stage of OmniTrack (arXiv 1910.06017,
 * Sec. V-A): given two consecutive frames I_{t-1}, I_t and the boxes
 * S_{t-1} of the objects tracked so far, predict their boxes S_t.
 *   - preprocessing: each frame is reduced by a Gaussian pyramid
 *     (ot_pyramid_build);
 *   - feature calculation: the motion between the frames, here sparse
 *     coarse-to-fine iterative Lucas-Kanade on points inside the boxes
 *     (ot_lk_track) in place of the paper's dense TV-L1 field (Sec. IV);
 *   - prediction: every box moves by the (median) motion of its points
 *     (ot_box_update; the paper averages the motion vectors in the box).
 * The Lucas-Kanade steps follow Bouguet (2000), "Pyramidal implementation
 * of the Lucas-Kanade feature tracker"; gradients are 3x3 Scharr (2000);
 * the point gate is the Shi-Tomasi (1994) minimum eigenvalue.
 * Around that path: many streams in one batched, graph-capturable tick
 * (ot_batch_*); the working level of the preprocessing phase
 * (ot_working_level, ot_lk_opts.base_level); Median Flow's forward-backward
 * gate and scaled boxes (ot_fb_gate, ot_box_update_scaled); the matching and
 * update phases (ot_iou_matrix, ot_assign, ot_track_update); and the
 * paper's own dense engine, TV-L1 flow with the mean-flow box prediction
 * (ot_tvl1_flow, ot_tvl1_flow_async, ot_tvl1_texture, ot_tvl1_flow_tex,
 * ot_box_mean_flow).
 *
 * Conventions shared by every call
 *   - Pointers are DEVICE pointers unless marked (host).
 *   - Images are uint8, row-major, with a row pitch in bytes >= width.
 *   - Coordinates are level-0 pixels with pixel centres at integers; pixel i
 *     of level l sits at level-0 position 2^l * i.  Level sizes are
 *     w_l = ceil(w_{l-1} / 2), h_l = ceil(h_{l-1} / 2).
 *   - Every call validates its arguments on the host before it enqueues
 *     anything.  On an error nothing is enqueued and no output is written.
 *     Otherwise the call only enqueues kernels on `stream` (a hipStream_t
 *     passed as void*, NULL = the default stream) and returns without
 *     synchronising; device faults surface at the caller's next
 *     synchronisation.  No C++ exception crosses the ABI.
 *   - The library allocates no device memory, keeps no pointer after a call
 *     returns and has no global stream, handle or mutable state: calls are
 *     thread-safe and may run concurrently on different streams (each
 *     caller thread owns its own stream, the lesson of Sec. III-B).  Two
 *     exceptions: ot_box_update_scaled_noalloc, whose scratch is a static
 *     device array per GPU shared by all its calls (see there), and
 *     ot_tvl1_flow_async, which keeps a set of HIP events per GPU for its
 *     fork and join (created on first use, never freed; the enqueue sequence
 *     that uses them is serialised by a lock).
 *   - The caller owns every buffer and keeps it (and any frame a pyramid
 *     aliases as its level 0) alive until the enqueued work has finished.
 */
#ifndef OMNITRACK_H
#define OMNITRACK_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define OT_API __attribute__((visibility("default")))
#else
#define OT_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ot_err;
enum {
    OT_OK = 0,
    OT_E_INVAL = -1,       /* a pointer, count or parameter is invalid */
    OT_E_SHAPE = -2,       /* image or pyramid shapes do not agree */
    OT_E_WORKSPACE = -3,   /* a caller buffer is too small */
    OT_E_LAUNCH = -4,      /* the HIP runtime refused a launch or copy */
    OT_E_UNSUPPORTED = -5  /* valid request the library does not implement */
};

#define OT_MAX_LEVELS 8
#define OT_MAX_WIN 31
#define OT_MAX_DIM 16384
/* Row pitch limit in bytes (8 x OT_MAX_DIM): level offsets are 32-bit. */
#define OT_MAX_PITCH 131072

/* Gate default: lambda_min(G) / win^2 below this (gray levels per pixel,
 * squared; 1e-4 on a [0,1] intensity scale) marks a point lost. */
#define OT_DEFAULT_MIN_EIG 6.5025f

/* Pyramid flag: also materialize the Scharr responses of every level (0 ..
 * levels-1) in the workspace.  A tracker that reads such a pyramid as its
 * template (previous) pyramid takes the gradients from these planes instead
 * of computing them for every point and level; results are identical. */
#define OT_PYR_GRADS 1

/* (host) Descriptor of a device-resident pyramid.  level[0] may alias the
 * caller's frame; levels 1.. live in a workspace. */
typedef struct {
    const uint8_t* level[OT_MAX_LEVELS];
    int32_t w[OT_MAX_LEVELS];
    int32_t h[OT_MAX_LEVELS];
    int32_t pitch[OT_MAX_LEVELS];
    int32_t levels; /* number of levels including level 0 */
    int32_t flags;  /* 0 or OT_PYR_GRADS */
    /* With OT_PYR_GRADS, per level one int32 per pixel (row pitch gpitch
     * elements): bits 0-15 the signed Scharr sum Sx, bits 16-31 Sy, with
     * Sx(x,y) = sum_{j=-1..1} s_j (P(cx(x+1), cy(y+j)) - P(cx(x-1), cy(y+j))),
     * s = (3,10,3), cx/cy clamping to the level; the gradient is S/32 and
     * |S| <= 4080.  Sy likewise with x and y exchanged.  NULL / 0 otherwise. */
    const int32_t* grad[OT_MAX_LEVELS];
    int32_t gpitch[OT_MAX_LEVELS];
} ot_pyr;

/* Bytes of device workspace ot_pyramid_build needs for levels 1..levels-1
 * of a W x H frame (0 when levels == 1 and flags == 0), plus, with
 * OT_PYR_GRADS, the gradient planes of all levels.  Returns 0 for invalid
 * sizes or flags.  Each level and plane starts 256-byte aligned; level
 * pitches are rounded up to 64 bytes, plane pitches to 16 elements. */
OT_API size_t ot_pyramid_bytes(int32_t W, int32_t H, int32_t levels, int32_t flags);

/* (host) Fill *out with the layout ot_pyramid_build would produce, without
 * enqueuing anything (used to re-describe a resident pyramid). */
OT_API ot_err ot_pyramid_layout(const uint8_t* frame, int32_t W, int32_t H, int32_t pitch,
                         int32_t levels, void* workspace, size_t ws_bytes, int32_t flags,
                         ot_pyr* out);

/* Gaussian pyramid (Sec. V-A preprocessing; binomial reduce of Burt &
 * Adelson 1983): level l from level l-1 as
 *   P_l(x,y) = (S + 128) >> 8,  S = sum_{i,j=-2..2} k_i k_j P_{l-1}(cx(2x+i), cy(2y+j))
 * with k = (1,4,6,4,1) and cx, cy clamping to the level's edge -- exact
 * integer arithmetic, rounding half up.
 * frame: W x H, row pitch `pitch`; levels in [1, OT_MAX_LEVELS];
 * workspace: >= ot_pyramid_bytes(W, H, levels, flags) bytes, 256-aligned.
 * *out (host) receives the descriptor, level[0] = frame.
 * Errors: OT_E_INVAL (null pointers, W/H out of [1, OT_MAX_DIM], pitch < W
 * or > OT_MAX_PITCH, levels out of range, flags not 0 or OT_PYR_GRADS), OT_E_WORKSPACE
 * (ws_bytes too small or misaligned), OT_E_LAUNCH.  With OT_PYR_GRADS the
 * gradient planes (see ot_pyr) are written on the same stream after the
 * levels. */
OT_API ot_err ot_pyramid_build(const uint8_t* frame, int32_t W, int32_t H, int32_t pitch,
                        int32_t levels, void* workspace, size_t ws_bytes, int32_t flags,
                        ot_pyr* out, void* stream);

/* Optional controls of ot_lk_track_ex (host struct). */
typedef struct {
    float min_eig;      /* gate threshold on lambda_min/win^2 (OT_DEFAULT_MIN_EIG) */
    uint8_t* iters_out; /* device n x levels, iterations run per level, or NULL */
    float* lam_out;     /* device n x levels, lambda_min/win^2 per level, or NULL */
    int32_t margin;     /* LDS search margin in pixels, 0 = default (4), max 16 */
    int32_t base_level; /* working level (Sec. V-A preprocessing), 0 = full resolution:
                           levels base_level .. base_level+levels-1 of both pyramids are
                           tracked as a pyramid whose level 0 is base_level; pts and
                           next_pts stay level-0 pixels (scaled by 2^-base_level in and
                           2^base_level out, exactly), the in-frame test and err refer to
                           level base_level.  See ot_working_level. */
    const int32_t* order; /* device n, or NULL: the k-th wave tracks point order[k] instead
                             of point k, so the caller can start long tracks first (see
                             ot_lk_order); a permutation of 0..n-1 (entries outside [0, n)
                             are skipped).  Results stay at the points' own indices and do
                             not depend on the order. */
} ot_lk_opts;

/* A processing order for ot_lk_opts.order: the n points by descending total
 * iterations over `levels` levels of `iters` (device n x levels uint8, e.g.
 * ot_lk_opts.iters_out of an earlier pair of the same points, such as the
 * previous frame pair of a stream), ties in any order.  The cost of a point
 * changes little from one frame pair to the next, and a launch whose long
 * tracks start first ends sooner.  order: device n int32 (a permutation of
 * 0..n-1).  One workgroup.  n == 0 is a no-op.
 * Errors: OT_E_INVAL (n < 0 or > 2^24, levels outside 1..OT_MAX_LEVELS, null
 * pointers with n > 0), OT_E_LAUNCH. */
OT_API ot_err ot_lk_order(const uint8_t* iters, int32_t n, int32_t levels, int32_t* order,
                          void* stream);

/* (host) Working-level policy for a frame of W x H pixels: the smallest
 * level l >= 0 whose width w_l (w_0 = W, w_l = ceil(w_{l-1} / 2)) is at most
 * max_width; 720x576 gives 0, 2560x1280 gives 1, 3840x2160 gives 2 for
 * max_width 1280.  Returns -1 for W, H or max_width < 1. */
OT_API int32_t ot_working_level(int32_t W, int32_t H, int32_t max_width);

/* Pyramidal iterative Lucas-Kanade (Bouguet 2000) from prev_pyr to next_pyr.
 * For each point u (pts, n x 2 float32 interleaved x,y):
 *   g = 0; for l = levels-1 .. 0, with c = u / 2^l:
 *     A(o) = I_l(c+o), X(o), Y(o) = bilinear Scharr/32 gradients of I_l at c+o,
 *       o over the win x win integer offsets around c;
 *     G = sum [X^2 XY; XY Y^2]; the point is lost if lambda_min(G)/win^2 < min_eig;
 *     nu = 0; up to `iters` times: B(o) = J_l(c+g+nu+o), d = A - B,
 *       b = sum d [X, Y], eta = G^{-1} b, nu += eta, stop once |eta|^2 < eps^2;
 *     g = 2 (g + nu) for l > 0, else the flow is g + nu.
 *   next = u + flow.  Bilinear taps clamp to the level's edge.
 * Outputs: next_pts n x 2 float32; status n (1 tracked, 0 lost: non-finite or
 * out-of-frame input, failed gate, or final position non-finite or outside
 * [0,W-1] x [0,H-1]); err n float32 (mean |I-J| over the level-0 window on the
 * 0..255 scale, -1 when lost) or NULL.  next_pts of a lost point holds its last
 * estimate.  Arithmetic is FP32.
 * Arguments: win odd in [3, OT_MAX_WIN]; 1 <= levels <= both pyramids' levels;
 * iters >= 1; eps >= 0 and finite (0 runs exactly `iters` iterations per level);
 * level-0 shapes of both pyramids equal; n >= 0 (n == 0 is a no-op).
 * Errors: OT_E_INVAL, OT_E_SHAPE, OT_E_LAUNCH. */
OT_API ot_err ot_lk_track(const ot_pyr* prev_pyr, const ot_pyr* next_pyr, const float* pts, int32_t n,
                   int32_t win, int32_t levels, int32_t iters, float eps, float* next_pts,
                   uint8_t* status, float* err, void* stream);

/* ot_lk_track with optional controls; opts may be NULL (defaults). */
OT_API ot_err ot_lk_track_ex(const ot_pyr* prev_pyr, const ot_pyr* next_pyr, const float* pts,
                      int32_t n, int32_t win, int32_t levels, int32_t iters, float eps,
                      float* next_pts, uint8_t* status, float* err, const ot_lk_opts* opts,
                      void* stream);

/* Box prediction (Sec. V-A prediction phase): for box b in [0, m),
 * (mx, my) = component-wise median of next_pts - pts over the points with
 * box_id == b and status == 1 (the mean of the two middle values for an even
 * count); out_boxes[b] = boxes[b] + (mx, my, mx, my), out_count[b] = that count.
 * A box without such points is copied unchanged with count 0 (lost).
 * boxes, out_boxes m x 4 float32 (x0, y0, x1, y1); box_id n int32 (ids outside
 * [0, m) belong to no box); pts, next_pts n x 2, 8-byte aligned; status n.
 * Errors: OT_E_INVAL (negative counts, null pointers with m > 0), OT_E_LAUNCH. */
OT_API ot_err ot_box_update(const float* boxes, int32_t m, const int32_t* box_id, const float* pts,
                     const float* next_pts, const uint8_t* status, int32_t n, float* out_boxes,
                     int32_t* out_count, void* stream);

/* ------------------------------------------------------------------------
 * Median Flow (Kalal, Mikolajczyk and Matas 2010), a refinement of the
 * prediction phase: points are tracked forward (I_{t-1} -> I_t) and back
 * (I_t -> I_{t-1}) with ot_lk_track_fb (or ot_lk_track twice), points that
 * do not return to where they started are dropped, and each box both moves
 * and scales with its points.
 * ---------------------------------------------------------------------- */

/* Points per box the scaled update takes (all gathered on chip). */
#define OT_SCALE_MAX_POINTS 6144

/* Forward-backward gate: for point i, if st_fwd[i] == 1 and st_bwd[i] == 1,
 * e = |pts[i] - back_pts[i]| (Euclidean, float32), fb_err[i] = e and
 * status_out[i] = (e <= fb_max); otherwise fb_err[i] = -1 and status_out[i]
 * = 0.  pts are the points tracked forward, back_pts the result of tracking
 * their forward positions back to the first frame.  pts, back_pts n x 2,
 * 8-byte aligned; st_fwd, st_bwd, status_out n; fb_err n or NULL.
 * status_out may alias st_fwd or st_bwd.  n == 0 is a no-op.
 * Errors: OT_E_INVAL (n < 0, null pointers with n > 0, misalignment, fb_max
 * negative or NaN), OT_E_LAUNCH. */
OT_API ot_err ot_fb_gate(const float* pts, const float* back_pts, const uint8_t* st_fwd,
                  const uint8_t* st_bwd, int32_t n, float fb_max, float* fb_err,
                  uint8_t* status_out, void* stream);

/* Forward and backward tracking in one launch (Median Flow's forward-backward
 * check, Kalal et al. 2010; Sec. V-A feature calculation): next_pts, status
 * and err are exactly those of ot_lk_track_ex(prev_pyr, next_pyr, pts, ...,
 * opts), and back_pts, back_status exactly those of ot_lk_track_ex(next_pyr,
 * prev_pyr, next_pts, ..., opts) -- each point's wave tracks it forward and
 * then its forward result back, so the launch has one fill and one tail
 * instead of two.  The backward pass's residuals are not returned.  With
 * kept non-NULL the forward-backward gate follows in the same launch: kept
 * and fb_err are exactly ot_fb_gate(pts, back_pts, status, back_status, n,
 * fb_max, fb_err, kept).
 * Arguments as ot_lk_track_ex; back_pts n x 2 float32, back_status n, kept n,
 * fb_err n float32 (the caller's device buffers); err and fb_err may be NULL,
 * kept NULL skips the gate (fb_max is then ignored); opts may be NULL
 * (defaults; its base_level, margin and min_eig apply to both directions).
 * Errors: as ot_lk_track_ex, OT_E_INVAL for null back_pts/back_status with
 * n > 0, fb_max negative or NaN with kept set, or fb_err not 4-byte aligned;
 * OT_E_UNSUPPORTED when opts asks for iters_out, lam_out or order. */
OT_API ot_err ot_lk_track_fb(const ot_pyr* prev_pyr, const ot_pyr* next_pyr, const float* pts,
                      int32_t n, int32_t win, int32_t levels, int32_t iters, float eps,
                      float* next_pts, uint8_t* status, float* err, float* back_pts,
                      uint8_t* back_status, float fb_max, float* fb_err, uint8_t* kept,
                      const ot_lk_opts* opts, void* stream);

/* Scaled box prediction: for box b in [0, m), over its points with
 * box_id == b and status == 1 (count c): (mx, my) = component-wise median
 * of next_pts - pts, s = the median over all unordered pairs {i, j} of those
 * points with pts[i] != pts[j] of |next_pts[i] - next_pts[j]| /
 * |pts[i] - pts[j]| (s = 1 when there is no such pair); medians of an even
 * count are the mean of the two middle values.  With centre (cx, cy) and
 * half-extents (hw, hh) of boxes[b], out_boxes[b] = (cx + mx - s*hw,
 * cy + my - s*hh, cx + mx + s*hw, cy + my + s*hh), out_count[b] = c,
 * out_scale[b] = s.  A box with c == 0 is copied unchanged with scale 1.  A
 * box with c > OT_SCALE_MAX_POINTS gets NaN in out_boxes[b] and out_scale[b]
 * (its count is still written).  Ratios are formed in float32; pairs whose
 * squared first-frame distance is zero in float32 are skipped.  Layouts as in
 * ot_box_update; out_scale m float32.  Work per box grows with c^2; the
 * pairs of one box are spread over several workgroups.  ws: device scratch
 * of at least ot_box_scaled_bytes(m) bytes, 256-byte aligned, owned by the
 * caller; every call rewrites it from scratch and keeps nothing in it, but
 * two calls whose work overlaps in time (different streams) must not share
 * one.  m == 0 is a no-op.
 * Errors: OT_E_INVAL (negative counts, m > 2^24, null pointers with m > 0,
 * misalignment), OT_E_WORKSPACE (ws NULL, not 256-byte aligned or smaller
 * than ot_box_scaled_bytes(m)), OT_E_LAUNCH. */
OT_API ot_err ot_box_update_scaled(const float* boxes, int32_t m, const int32_t* box_id,
                            const float* pts, const float* next_pts, const uint8_t* status,
                            int32_t n, float* out_boxes, int32_t* out_count, float* out_scale,
                            void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes of ot_box_update_scaled for m boxes (0 if invalid). */
OT_API size_t ot_box_scaled_bytes(int32_t m);

/* Largest box count of ot_box_update_scaled_noalloc. */
#define OT_SCALED_NOALLOC_MAX_BOXES 64

/* ot_box_update_scaled for callers that cannot allocate device memory (code
 * under HIP graph capture, allocation-free serving loops): the same
 * arguments, results and errors without ws/ws_bytes.  The per-box scratch is
 * a static device array inside the library, OT_SCALED_NOALLOC_MAX_BOXES x
 * ot_box_scaled_bytes(1) bytes (8.1 MB), of which each GPU the library runs
 * on holds its own copy until the process ends; the call allocates nothing.
 * Its device address is looked up once per device, on the first call that
 * targets it (the device of `stream`, or the current device for NULL).
 * Every call rewrites the scratch it uses from scratch, but all calls on one
 * GPU share the one array: calls whose work overlaps in time on one GPU
 * (different streams, several host threads) race and must be serialised by
 * the caller.  Errors: as ot_box_update_scaled, plus OT_E_INVAL for m >
 * OT_SCALED_NOALLOC_MAX_BOXES (nothing enqueued) and OT_E_LAUNCH when the
 * scratch address cannot be obtained. */
OT_API ot_err ot_box_update_scaled_noalloc(const float* boxes, int32_t m, const int32_t* box_id,
                                           const float* pts, const float* next_pts,
                                           const uint8_t* status, int32_t n, float* out_boxes,
                                           int32_t* out_count, float* out_scale, void* stream);

/* ------------------------------------------------------------------------
 * Matching and update phases (Sec. V-A): the predicted scene objects S_t
 * are matched one-to-one against the detections D_t, globally optimally
 * (Hungarian method, Kuhn 1955) with intersection-over-union as the score;
 * unmatched objects are flagged lost, unmatched detections become new
 * objects.  The score matrix is built on the GPU, the assignment and the
 * update run on the host.
 * ---------------------------------------------------------------------- */

/* iou[i * k + j] = area(S_i & D_j) / area(S_i | D_j) (float32) for every
 * object i < m and detection j < k; area(x0, y0, x1, y1) = max(0, x1 - x0) *
 * max(0, y1 - y0); 0 when the union has no area, and 0 in the rows of
 * objects with active[i] == 0 (active may be NULL: all active).
 * S m x 4, D k x 4 float32 (x0, y0, x1, y1), 16-byte aligned; active m;
 * iou m x k.  Device pointers; m == 0 or k == 0 is a no-op.
 * Errors: OT_E_INVAL (negative sizes, null pointers, misalignment),
 * OT_E_LAUNCH. */
OT_API ot_err ot_iou_matrix(const float* S, int32_t m, const float* D, int32_t k,
                     const uint8_t* active, float* iou, void* stream);

/* (host) Optimal matching on an m x k score matrix (host, row-major): among
 * one-to-one matchings whose pairs all have iou >= iou_min, one with the
 * largest summed iou.  s2d[i] = matched detection of object i or -1, d2s[j]
 * = matched object of detection j or -1; score (may be NULL) = the summed
 * iou of the matched pairs, in double.  Where several matchings reach the
 * same sum any one of them is returned.  0 < iou_min <= 1 (so rows of
 * inactive objects never match).  Allocates O(m k) host memory; O(m k
 * min(m, k)) time; m * k <= 2^26.
 * Errors: OT_E_INVAL. */
OT_API ot_err ot_assign(const float* iou, int32_t m, int32_t k, float iou_min, int32_t* s2d,
                 int32_t* d2s, double* score);

/* (host) Track update: for every object i < m that is not lost, a match
 * s2d[i] = j replaces its box by det[j], no match sets lost[i] = 1; lost
 * objects are left unchanged.  Every detection j with d2s[j] == -1 is then
 * appended (in detection order) as a new object with id *next_id (which is
 * incremented) and lost = 0; *m_out receives the new object count.
 * boxes cap x 4, ids cap, lost cap (host, the first m entries valid on
 * entry); det k x 4, s2d m, d2s k (host).  s2d and d2s must be mutually
 * consistent (as ot_assign writes them).  Errors: OT_E_INVAL (sizes,
 * pointers, inconsistent matching, id overflow), OT_E_WORKSPACE (more than
 * cap objects would result; nothing is written). */
OT_API ot_err ot_track_update(float* boxes, int32_t* ids, uint8_t* lost, int32_t m, int32_t cap,
                       const float* det, int32_t k, const int32_t* s2d, const int32_t* d2s,
                       int32_t* next_id, int32_t* m_out);

/* ------------------------------------------------------------------------
 * Dense variant of the motion features (Sec. IV): TV-L1 optical flow with a
 * Huber-smoothed total variation, solved by projected steps on the dual
 * variable (Zach, Pock & Bischof 2007; Werlberger et al. 2009), on
 * structure-texture decomposed inputs (Wedel et al. 2009), coarse to fine
 * over the same uint8 pyramids as the sparse path; and the prediction of
 * Sec. V-A: every box moves by the mean of the dense field inside it.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t levels;   /* pyramid levels used, coarse to fine (1..OT_MAX_LEVELS) */
    int32_t warps;    /* linearisations of the data term per level (>= 1) */
    int32_t iters;    /* iterations per linearisation (>= 1) */
    float lam;        /* data weight, textures on the [0, 1] scale (> 0) */
    float theta;      /* coupling weight of the flow and its auxiliary (> 0) */
    float tau;        /* dual step (0 < tau <= 0.25) */
    float eps;        /* Huber smoothing of the total variation (>= 0) */
    float alpha;      /* texture = f - alpha * structure */
    float theta_s;    /* structure (ROF) fidelity weight (> 0) */
    float tau_s;      /* structure dual step (0 < tau_s <= 0.25) */
    int32_t iters_s;  /* structure iterations (>= 0; 0: structure = f) */
} ot_tvl1_params;

/* (host) The defaults: 5 levels, 5 warps, 30 iterations, lam 40, theta 0.3,
 * tau 0.25, eps 0.01, alpha 0.95, theta_s 0.1, tau_s 0.125, 50 structure
 * iterations. */
OT_API void ot_tvl1_default_params(ot_tvl1_params* p);

/* Workspace bytes of ot_tvl1_flow / ot_tvl1_flow_async for a W x H level 0
 * (0 if invalid): level-0 planes for the structure duals, the linearised
 * data term, the flow and its dual, and per level the two textures and the
 * second texture's gradient, for pyramids of up to OT_MAX_LEVELS levels of
 * the usual sizes. */
OT_API size_t ot_tvl1_bytes(int32_t W, int32_t H);

/* Dense flow from prev_pyr to next_pyr.  Every level l < p->levels (coarse
 * to fine) of both pyramids is scaled to f = I / 255 and split: structure =
 * argmin_s TV(s) + |s - f|^2 / (2 theta_s) by iters_s dual (Chambolle 2004)
 * steps from p = 0, texture = f - alpha * structure.  The flow starts at 0
 * on the coarsest level and enters each finer level as 2 u(x / 2) (bilinear,
 * clamped).  On each level, `warps` times: I1, its central-difference
 * gradient (clamped indices) are sampled bilinearly at x + u0 (position
 * clamped to the level), rho(u) = I1(x+u0) + g . (u - u0) - I0; then `iters`
 * times: v = the pointwise minimiser of |v - u|^2 / (2 theta) + lam |rho(v)|,
 * u = v + theta div p, p = projection onto |p| <= 1 of (p + (tau/theta) grad
 * u) / (1 + tau eps / theta) for each flow component (grad: forward
 * differences, 0 on the last column / row; div = -grad^T); p restarts at 0
 * on every level.  flow: W0 x H0 float32 pairs (u_x, u_y) per pixel of
 * level 0, row-major, dense, 8-byte aligned, in level-0 pixels.  ws:
 * ot_tvl1_bytes(W0, H0) bytes, 256-byte aligned, owned by the caller.
 * Arithmetic is FP32.  Errors: OT_E_INVAL (descriptors, parameters, null
 * pointers), OT_E_SHAPE (level sizes differ), OT_E_WORKSPACE, OT_E_LAUNCH. */
OT_API ot_err ot_tvl1_flow(const ot_pyr* prev_pyr, const ot_pyr* next_pyr,
                    const ot_tvl1_params* prm, void* ws, size_t ws_bytes, float* flow,
                    void* stream);

/* ot_tvl1_flow with the structure-texture split and the texture gradients of
 * every level enqueued on aux_stream, ahead of the flow on `stream` (Sec.
 * V-B: independent phases run side by side).  The split of level l depends
 * only on the frames, not on the flow of the coarser levels, so it runs while
 * the latency-bound coarse levels leave most of the GPU idle; level l's flow
 * waits for an event recorded on aux_stream after its planes.  aux_stream
 * starts after an event recorded on `stream` (all work enqueued there
 * before the call) and is joined back into `stream` before the call's last
 * launch, so the call also works under graph capture of `stream`.  Same
 * kernels and inputs: the flow is bit for bit that of ot_tvl1_flow.  Both
 * streams must belong to one device; aux_stream == stream is ot_tvl1_flow.
 * Errors: those of ot_tvl1_flow; OT_E_INVAL also for streams of different
 * devices, OT_E_LAUNCH if an event cannot be created or recorded. */
OT_API ot_err ot_tvl1_flow_async(const ot_pyr* prev_pyr, const ot_pyr* next_pyr,
                          const ot_tvl1_params* prm, void* ws, size_t ws_bytes, float* flow,
                          void* stream, void* aux_stream);

/* One video stream, frame by frame (Sec. V-B): a frame's structure-texture
 * split is the same whether it is the second frame of a pair or the first of
 * the next, so it can be computed once per frame, ahead of the flow (the
 * prefetch of the next frame's preprocessing).  ot_tvl1_texture_bytes: bytes
 * of one frame's texture buffer for a W x H level 0 (0 if invalid): the
 * split's scratch (two level-0 float2 planes) and, per level, the texture
 * (float) and its central-difference gradient (float2 pairs). */
OT_API size_t ot_tvl1_texture_bytes(int32_t W, int32_t H);

/* The structure-texture split of every level l < prm->levels of one frame's
 * pyramid (as ot_tvl1_flow does for each frame: iters_s dual steps from p = 0,
 * texture = f - alpha * structure) and the texture's clamped central-difference
 * gradient, into tex: ot_tvl1_texture_bytes(W0, H0) bytes, 256-byte aligned,
 * owned by the caller, opaque (read by ot_tvl1_flow_tex with the same levels
 * and level sizes).  Errors: OT_E_INVAL, OT_E_WORKSPACE, OT_E_LAUNCH. */
OT_API ot_err ot_tvl1_texture(const ot_pyr* pyr, const ot_tvl1_params* prm, void* tex,
                       size_t tex_bytes, void* stream);

/* ot_tvl1_flow from two frames' texture buffers (ot_tvl1_texture with the same
 * prm->levels, iters_s, theta_s, tau_s and alpha): prev_pyr and next_pyr give
 * the level sizes only.  The flow is bit for bit that of ot_tvl1_flow on the
 * two pyramids.  ws as ot_tvl1_flow.  Errors: those of ot_tvl1_flow, and
 * OT_E_WORKSPACE for a texture buffer that is not 256-byte aligned. */
OT_API ot_err ot_tvl1_flow_tex(const ot_pyr* prev_pyr, const ot_pyr* next_pyr,
                        const void* prev_tex, const void* next_tex,
                        const ot_tvl1_params* prm, void* ws, size_t ws_bytes, float* flow,
                        void* stream);

/* Box prediction from a dense field (Sec. V-A): for box b, (mx, my) = the
 * mean of flow over the pixels (x, y) with integer x in [ceil(x0),
 * floor(x1)] and y in [ceil(y0), floor(y1)], clipped to the W x H field
 * (sums in double); out_boxes[b] = boxes[b] + (mx, my, mx, my), out_count[b]
 * = the pixel count; a box without pixels is copied unchanged with count 0.
 * flow W x H float32 pairs (8-byte aligned), boxes/out_boxes m x 4, out_count
 * m.  Errors: OT_E_INVAL, OT_E_LAUNCH. */
OT_API ot_err ot_box_mean_flow(const float* flow, int32_t W, int32_t H, const float* boxes,
                        int32_t m, float* out_boxes, int32_t* out_count, void* stream);

/* ------------------------------------------------------------------------
 * Batched tick: many independent streams (frame pairs) in one launch per
 * stage.  Stage 1 builds every job's next pyramid (all jobs, one launch per
 * level), stage 2 tracks every job's points in one launch, stage 3 updates
 * every job's boxes in one launch.  Results equal the per-job calls.
 * The caller packs a descriptor table on the host (ot_batch_pack into a
 * pinned buffer of ot_batch_table_bytes), and ot_batch_run copies it to a
 * device buffer of the same size and launches the stages on `stream`.  The
 * work sizes are read from the device table, so a HIP graph captured around
 * ot_batch_run replays any later table of the same capacities.
 * ---------------------------------------------------------------------- */
typedef struct {
    ot_pyr prev;                /* resident pyramid of I_{t-1} */
    const uint8_t* next_frame;  /* level 0 of I_t */
    int32_t next_pitch;
    void* next_ws;              /* workspace for levels 1.. of I_t's pyramid */
    size_t next_ws_bytes;
    int32_t levels;             /* levels built and tracked (<= prev.levels) */
    const float* pts;           /* n x 2 */
    int32_t n;
    float* next_pts;            /* n x 2 */
    uint8_t* status;            /* n */
    float* err;                 /* n or NULL */
    const float* boxes;         /* m x 4 */
    int32_t m;
    const int32_t* box_id;      /* n */
    float* out_boxes;           /* m x 4 */
    int32_t* out_count;         /* m */
} ot_job;

typedef struct {
    int32_t win, iters;
    float eps, min_eig;
    int32_t margin;        /* as ot_lk_opts.margin */
    int32_t lk_waves;      /* persistent LK grid in waves; 0 = one wave per point */
    int32_t chunk;         /* points a persistent wave claims at a time (>= 1) */
    int32_t max_jobs;      /* table capacity in jobs */
    int32_t max_points;    /* capacity in points, sizes the non-persistent LK grid */
    int32_t max_boxes;     /* capacity in boxes */
    int32_t max_tiles;     /* capacity in pyramid tiles per fused launch (16x8 tiles of
                              the top level of each run of up to 3 levels) */
    int32_t max_levels;    /* levels launched for the pyramid stage */
    int32_t exact_grids;   /* nonzero: size every launch from the packed table's totals
                              (read from table_host) instead of the capacities -- for
                              eager ticks; a captured graph needs capacity-sized grids */
    int32_t lk_wpg;        /* waves per workgroup of the tracking stage (0 or 1, 2, 4) */
    int32_t lk_ppw;        /* points each wave tracks one after the other (0 or 1, 2, 4);
                              wpg or ppw above 1 need the 21 x 21 window at margin 4 or 6
                              and lk_waves == 0 (else OT_E_UNSUPPORTED) */
} ot_batch_cfg;

/* Bytes of the descriptor table for cfg's capacities (0 if invalid). */
OT_API size_t ot_batch_table_bytes(const ot_batch_cfg* cfg);

/* (host) Validate the jobs against cfg and write the table into table_host.
 * next_out (host, njobs entries, may be NULL) receives each job's next
 * pyramid descriptor.  Errors: OT_E_INVAL, OT_E_SHAPE, OT_E_WORKSPACE
 * (capacity exceeded or a job's workspace too small). */
OT_API ot_err ot_batch_pack(const ot_job* jobs, int32_t njobs, const ot_batch_cfg* cfg,
                     void* table_host, size_t table_bytes, ot_pyr* next_out);

/* Copy the packed table to table_dev and launch the three stages on stream.
 * table_host should be pinned memory for the copy to be asynchronous; it
 * must stay unchanged until the copy has executed.  The table holds the
 * persistent stage's work counter, which the stage returns to zero itself.
 * Errors: OT_E_INVAL, OT_E_WORKSPACE, OT_E_LAUNCH. */
OT_API ot_err ot_batch_run(const void* table_host, void* table_dev, size_t table_bytes,
                    const ot_batch_cfg* cfg, void* stream);

/* Stages of ot_batch_run_stages (bit mask). */
#define OT_STAGE_PYRAMID 1 /* copy the table to table_dev, build every job's next pyramid */
#define OT_STAGE_TRACK 2   /* track every job's points, update every job's boxes */

/* ot_batch_run split in two stages, so that a caller can run one tick's
 * preprocessing on one stream while an earlier tick is tracked on another
 * (the prefetch of Sec. V-B).  stages = OT_STAGE_PYRAMID | OT_STAGE_TRACK is
 * ot_batch_run.  OT_STAGE_TRACK alone reads the table that an earlier
 * OT_STAGE_PYRAMID call copied into the same table_dev; the caller orders
 * the two (e.g. an event recorded after the first and waited on the second
 * stream) and keeps table_host and table_dev unchanged until both stages
 * have run.  Arguments and errors as ot_batch_run, plus OT_E_INVAL for an
 * empty or unknown stage mask. */
OT_API ot_err ot_batch_run_stages(const void* table_host, void* table_dev, size_t table_bytes,
                                  const ot_batch_cfg* cfg, int32_t stages, void* stream);

/* Static text for an error code. */
OT_API const char* ot_strerror(ot_err e);

/* Library version (major * 10000 + minor * 100 + patch). */
OT_API int32_t ot_version(void);

#ifdef __cplusplus
}
#endif
#endif /* OMNITRACK_H */
