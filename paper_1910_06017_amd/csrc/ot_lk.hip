// ot_lk.hip -- the single-call Lucas-Kanade tracking kernel for gfx950: one
// wave64 per point over one pyramid pair.
#include "ot_launch.hpp"
#include "ot_lk_sched.hpp"

namespace ot {

template <int R, int WIN = 0, int MARGIN = 0, bool GRADS = false>
__global__ OT_LK_BOUNDS void k_lk_track(DevPyr P, DevPyr Q, const float* __restrict__ pts,
                                                 int n, LkParams prm, float* __restrict__ next_pts,
                                                 uint8_t* __restrict__ status,
                                                 float* __restrict__ err,
                                                 uint8_t* __restrict__ iters_out,
                                                 float* __restrict__ lam_out,
                                                 const int32_t* __restrict__ order) {
    extern __shared__ __align__(16) unsigned char lk_smem[];
    int i = lk_item(blockIdx.x, gridDim.x);
    if (i >= n) return;
    if (order) {
        i = order[i];
        if ((unsigned)i >= (unsigned)n) return;
    }
    const float ux = uniform_f(pts[2 * i]) * prm.pscale, uy = uniform_f(pts[2 * i + 1]) * prm.pscale;
    const LkGeom g(WIN > 0 ? WIN : prm.win, R, MARGIN > 0 ? MARGIN : prm.margin);
    const int L = prm.levels;
    const LkResult r = lk_point<R, (WIN > 0), GRADS, DevPyr, false, LK_PRIO_REMAINING>(P, Q, ux, uy, L, prm.iters, prm.eps2, prm.min_eig, g, lk_smem,
                                   iters_out ? iters_out + (size_t)i * L : nullptr,
                                   lam_out ? lam_out + (size_t)i * L : nullptr);
    if ((threadIdx.x & 63) == 0) {
        next_pts[2 * i] = r.nx * prm.pscale_inv;
        next_pts[2 * i + 1] = r.ny * prm.pscale_inv;
        status[i] = (uint8_t)r.status;
        if (err) err[i] = r.err;
    }
}

int lk_template_rows(int win) {
    const int need = lk_rows_needed(win);
    static const int rows[] = {1, 2, 4, 7, 8, 12, 16};
    for (int r : rows)
        if (r >= need) return r;
    return 0;
}

hipError_t launch_lk(const DevPyr& prev, const DevPyr& next, const float* pts, int n,
                     const LkParams& prm, float* next_pts, uint8_t* status, float* err,
                     uint8_t* iters_out, float* lam_out, const int32_t* order,
                     hipStream_t stream) {
    const int R = lk_template_rows(prm.win);
    const size_t lds = lk_lds_bytes(prm.win, R, prm.margin);
    const bool grads = (prev.flags & OT_PYR_GRADS) != 0;
#define OT_LAUNCH(...)                                                                           \
    hipLaunchKernelGGL((k_lk_track<__VA_ARGS__>), dim3(n), dim3(64), lds, stream, prev, next, pts, \
                       n, prm, next_pts, status, err, iters_out, lam_out, order)
    if (R == 7 && prm.win == 21 && (prm.margin == 4 || prm.margin == 6)) {
        if (prm.margin == 4) {
            if (grads) OT_LAUNCH(7, 21, 4, true); else OT_LAUNCH(7, 21, 4, false);
        } else {
            if (grads) OT_LAUNCH(7, 21, 6, true); else OT_LAUNCH(7, 21, 6, false);
        }
        return hipGetLastError();
    }
    switch (R) {
#define OT_CASE(RR)                                                 \
    case RR:                                                        \
        if (grads) OT_LAUNCH(RR, 0, 0, true); else OT_LAUNCH(RR, 0, 0, false); \
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
