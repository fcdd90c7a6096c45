// ot_lk_fb.hip -- forward and backward Lucas-Kanade tracking of each point in
// one launch (Median Flow's forward-backward check, Kalal, Mikolajczyk and
// Matas 2010): the wave of point i tracks it from the first frame to the
// second, then tracks that result back to the first frame.  Each direction is
// the single-call tracker's per-point routine on the same inputs, so both
// results are bit for bit those of two ot_lk_track calls; one launch holds
// every point's whole chain, so the launch pays one fill and one tail where
// two launches pay two.  Optionally the forward-backward gate of each point
// follows, with the gate call's own arithmetic.
#include "ot_box.hpp"
#include "ot_launch.hpp"
#include "ot_lk_sched.hpp"

namespace ot {

template <int R, int WIN = 0, int MARGIN = 0>
__global__ __launch_bounds__(64) void k_lk_track_fb(DevPyr P, DevPyr Q, const float* __restrict__ pts,
                                                    int n, LkParams prm,
                                                    float* __restrict__ next_pts,
                                                    uint8_t* __restrict__ status,
                                                    float* __restrict__ err,
                                                    float* __restrict__ back_pts,
                                                    uint8_t* __restrict__ back_status,
                                                    float fb_max, float* __restrict__ fb_err,
                                                    uint8_t* __restrict__ kept) {
    extern __shared__ __align__(16) unsigned char lk_smem[];
    const int i = lk_item(blockIdx.x, gridDim.x);
    if (i >= n) return;
    const LkGeom g(WIN > 0 ? WIN : prm.win, R, MARGIN > 0 ? MARGIN : prm.margin);
    const int L = prm.levels;
    const float ux = uniform_f(pts[2 * i]) * prm.pscale, uy = uniform_f(pts[2 * i + 1]) * prm.pscale;
    // Issue priority by the work left (see lk_priority): the forward pass has
    // the whole backward pass still ahead of it, so it runs at the top
    // priority throughout; the backward pass ranks by level as a single call.
    __builtin_amdgcn_s_setprio(3);
    const LkResult f = lk_point<R, (WIN > 0), false, DevPyr, false, LK_PRIO_NONE>(
        P, Q, ux, uy, L, prm.iters, prm.eps2, prm.min_eig, g, lk_smem, nullptr, nullptr);
    // the forward result as the caller receives it, read back as the backward
    // call would read it (the scales are powers of two)
    const float fx = f.nx * prm.pscale_inv, fy = f.ny * prm.pscale_inv;
    if ((threadIdx.x & 63) == 0) {
        next_pts[2 * i] = fx;
        next_pts[2 * i + 1] = fy;
        status[i] = (uint8_t)f.status;
        if (err) err[i] = f.err;
    }
    __syncthreads();  // the backward pass restages the same LDS
    const LkResult b = lk_point<R, (WIN > 0), false, DevPyr, false, LK_PRIO_REMAINING>(
        Q, P, fx * prm.pscale, fy * prm.pscale, L, prm.iters, prm.eps2, prm.min_eig, g, lk_smem,
        nullptr, nullptr);
    if ((threadIdx.x & 63) == 0) {
        const float2 q = make_float2(b.nx * prm.pscale_inv, b.ny * prm.pscale_inv);
        back_pts[2 * i] = q.x;
        back_pts[2 * i + 1] = q.y;
        back_status[i] = (uint8_t)b.status;
        if (kept) {
            float e;
            uint8_t st;
            fb_gate_value(make_float2(pts[2 * i], pts[2 * i + 1]), q, (unsigned)f.status,
                          (unsigned)b.status, fb_max, e, st);
            kept[i] = st;
            if (fb_err) fb_err[i] = e;
        }
    }
}

hipError_t launch_lk_fb(const DevPyr& prev, const DevPyr& next, const float* pts, int n,
                        const LkParams& prm, float* next_pts, uint8_t* status, float* err,
                        float* back_pts, uint8_t* back_status, float fb_max, float* fb_err,
                        uint8_t* kept, hipStream_t stream) {
    const int R = lk_template_rows(prm.win);
    const size_t lds = lk_lds_bytes(prm.win, R, prm.margin);
#define OT_LAUNCH(...)                                                                           \
    hipLaunchKernelGGL((k_lk_track_fb<__VA_ARGS__>), dim3(n), dim3(64), lds, stream, prev, next, \
                       pts, n, prm, next_pts, status, err, back_pts, back_status, fb_max,   \
                       fb_err, kept)
    if (R == 7 && prm.win == 21 && (prm.margin == 4 || prm.margin == 6)) {
        if (prm.margin == 4) OT_LAUNCH(7, 21, 4); else OT_LAUNCH(7, 21, 6);
        return hipGetLastError();
    }
    switch (R) {
#define OT_CASE(RR)        \
    case RR:               \
        OT_LAUNCH(RR);     \
        break;
        OT_LK_ROWS(OT_CASE)
#undef OT_CASE
        default:
            return hipErrorInvalidValue;
    }
#undef OT_LAUNCH
    return hipGetLastError();
}

}  // namespace ot
