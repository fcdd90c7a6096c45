// ot_lk.hip -- Lucas-Kanade tracking kernels for gfx950: one wave64 per point,
// single-pyramid-pair and batched (flattened multi-stream table) forms.
#include "ot_lk_dev.hpp"
#include "ot_launch.hpp"

// Optional occupancy target (waves per SIMD) for the tracking kernels.
#ifndef OT_LK_MIN_WAVES
#define OT_LK_MIN_WAVES 0
#endif
#if OT_LK_MIN_WAVES > 0
#define OT_LK_BOUNDS __launch_bounds__(64, OT_LK_MIN_WAVES)
#else
#define OT_LK_BOUNDS __launch_bounds__(64)
#endif

// Point order.  Workgroup b runs on XCD b % 8.  Points of one box cost
// alike, so giving each XCD one contiguous range of points (OT_LK_XCD_REMAP
// 1) leaves some XCDs with the expensive boxes.  The default (0) deals
// chunks of LK_CHUNK consecutive points to the XCDs round-robin: the XCDs
// get even shares of every box, while each chunk's outputs fill whole cache
// lines in one XCD's L2 and its neighbouring windows share that L2.  Each XCD
// then reads most of both pyramids (a few MB per frame pair), which costs far
// less than the imbalance it removes.
#ifndef OT_LK_XCD_REMAP
#define OT_LK_XCD_REMAP 0
#endif

namespace ot {

constexpr int LK_CHUNK = 16;

__device__ __forceinline__ int lk_item(int b, int G) {
    if (OT_LK_XCD_REMAP) return xcd_remap(b, G);
    constexpr int X = 8, S = X * LK_CHUNK;
    if (b >= G - G % S) return b;  // ragged tail in dispatch order
    const int x = b % X, k = b / X;
    return ((k / LK_CHUNK) * X + x) * LK_CHUNK + k % LK_CHUNK;
}

template <int R, int WIN = 0, int MARGIN = 0, bool GRADS = false>
__global__ OT_LK_BOUNDS void k_lk_track(DevPyr P, DevPyr Q, const float* __restrict__ pts,
                                                 int n, LkParams prm, float* __restrict__ next_pts,
                                                 uint8_t* __restrict__ status,
                                                 float* __restrict__ err,
                                                 uint8_t* __restrict__ iters_out,
                                                 float* __restrict__ lam_out) {
    extern __shared__ __align__(16) unsigned char lk_smem[];
    const int i = lk_item(blockIdx.x, gridDim.x);
    if (i >= n) return;
    const float ux = uniform_f(pts[2 * i]) * prm.pscale, uy = uniform_f(pts[2 * i + 1]) * prm.pscale;
    const LkGeom g(WIN > 0 ? WIN : prm.win, R, MARGIN > 0 ? MARGIN : prm.margin);
    const int L = prm.levels;
    const LkResult r = lk_point<R, (WIN > 0), GRADS>(P, Q, ux, uy, L, prm.iters, prm.eps2, prm.min_eig, g, lk_smem,
                                   iters_out ? iters_out + (size_t)i * L : nullptr,
                                   lam_out ? lam_out + (size_t)i * L : nullptr);
    if ((threadIdx.x & 63) == 0) {
        next_pts[2 * i] = r.nx * prm.pscale_inv;
        next_pts[2 * i + 1] = r.ny * prm.pscale_inv;
        status[i] = (uint8_t)r.status;
        if (err) err[i] = r.err;
    }
}

// Index of the job whose prefix range holds item i (prefix has njobs+1 entries).
__device__ __forceinline__ int find_job(const int32_t* __restrict__ prefix, int njobs, int i) {
    int lo = 0, hi = njobs;  // invariant: prefix[lo] <= i < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

template <int R, int WIN = 0, int MARGIN = 0>
__device__ __forceinline__ void lk_batch_item(const uint8_t* __restrict__ table,
                                              const TableLayout& T, const TableHdr& hd, int i,
                                              unsigned char* smem) {
    const int32_t* pt_prefix = reinterpret_cast<const int32_t*>(table + T.pt_prefix);
    const DevJob* jobs = reinterpret_cast<const DevJob*>(table + T.jobs);
    const int j = __builtin_amdgcn_readfirstlane(find_job(pt_prefix, hd.njobs, i));
    const DevJob& jb = jobs[j];
    const int li = i - pt_prefix[j];
    const float ux = uniform_f(jb.pts[2 * li]), uy = uniform_f(jb.pts[2 * li + 1]);
    const LkGeom g(WIN > 0 ? WIN : hd.lk.win, R, MARGIN > 0 ? MARGIN : hd.lk.margin);
    const LkResult r = lk_point<R, (WIN > 0), false>(jb.prev, jb.next, ux, uy, jb.levels, hd.lk.iters, hd.lk.eps2,
                                   hd.lk.min_eig, g, smem, nullptr, nullptr);
    if ((threadIdx.x & 63) == 0) {
        jb.next_pts[2 * li] = r.nx;
        jb.next_pts[2 * li + 1] = r.ny;
        jb.status[li] = (uint8_t)r.status;
        if (jb.err) jb.err[li] = r.err;
    }
}

// One wave per point over the flattened points of every job.
template <int R, int WIN = 0, int MARGIN = 0>
__global__ OT_LK_BOUNDS void k_lk_batch(const uint8_t* __restrict__ table, int cap) {
    extern __shared__ __align__(16) unsigned char lk_smem[];
    const TableLayout T = TableLayout::make(cap);
    const TableHdr& hd = *reinterpret_cast<const TableHdr*>(table);
    const int i = lk_item(blockIdx.x, gridDim.x);
    if (i >= hd.total_pts) return;
    lk_batch_item<R, WIN, MARGIN>(table, T, hd, i, lk_smem);
}

// Persistent form: a fixed grid of waves claims chunks of points from the
// table's work counter until the points run out.
template <int R, int WIN = 0, int MARGIN = 0>
__global__ OT_LK_BOUNDS void k_lk_batch_persistent(uint8_t* __restrict__ table, int cap) {
    extern __shared__ __align__(16) unsigned char lk_smem[];
    const TableLayout T = TableLayout::make(cap);
    TableHdr& hd = *reinterpret_cast<TableHdr*>(table);
    const int total = hd.total_pts;
    const int chunk = max(1, hd.chunk);
    for (;;) {
        int base = 0;
        if ((threadIdx.x & 63) == 0) base = (int)atomicAdd(&hd.counter, (uint32_t)chunk);
        base = __builtin_amdgcn_readfirstlane(base);
        if (base >= total) break;
        const int end = min(base + chunk, total);
        for (int i = base; i < end; ++i) lk_batch_item<R, WIN, MARGIN>(table, T, hd, i, lk_smem);
    }
}

#define OT_LK_ROWS(X) X(1) X(2) X(4) X(7) X(8) X(12) X(16)

int lk_template_rows(int win) {
    const int need = lk_rows_needed(win);
    static const int rows[] = {1, 2, 4, 7, 8, 12, 16};
    for (int r : rows)
        if (r >= need) return r;
    return 0;
}

hipError_t launch_lk(const DevPyr& prev, const DevPyr& next, const float* pts, int n,
                     const LkParams& prm, float* next_pts, uint8_t* status, float* err,
                     uint8_t* iters_out, float* lam_out, hipStream_t stream) {
    const int R = lk_template_rows(prm.win);
    const size_t lds = lk_lds_bytes(prm.win, R, prm.margin);
    const bool grads = (prev.flags & OT_PYR_GRADS) != 0;
#define OT_LAUNCH(...)                                                                           \
    hipLaunchKernelGGL((k_lk_track<__VA_ARGS__>), dim3(n), dim3(64), lds, stream, prev, next, pts, \
                       n, prm, next_pts, status, err, iters_out, lam_out)
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

hipError_t launch_batch_lk(const uint8_t* table, int cap, int win, int margin, int grid,
                           bool persistent, hipStream_t stream) {
    const int R = lk_template_rows(win);
    const size_t lds = lk_lds_bytes(win, R, margin);
    if (R == 7 && win == 21 && (margin == 4 || margin == 6)) {
#define OT_SPEC(MM)                                                                              \
    if (persistent)                                                                              \
        hipLaunchKernelGGL((k_lk_batch_persistent<7, 21, MM>), dim3(grid), dim3(64), lds, stream, \
                           const_cast<uint8_t*>(table), cap);                                    \
    else                                                                                         \
        hipLaunchKernelGGL((k_lk_batch<7, 21, MM>), dim3(grid), dim3(64), lds, stream, table, cap);
        if (margin == 4) {
            OT_SPEC(4)
        } else {
            OT_SPEC(6)
        }
#undef OT_SPEC
        return hipGetLastError();
    }
    switch (R) {
#define OT_CASE(RR)                                                                           \
    case RR:                                                                                  \
        if (persistent)                                                                       \
            hipLaunchKernelGGL(k_lk_batch_persistent<RR>, dim3(grid), dim3(64), lds, stream,  \
                               const_cast<uint8_t*>(table), cap);                             \
        else                                                                                  \
            hipLaunchKernelGGL(k_lk_batch<RR>, dim3(grid), dim3(64), lds, stream, table, cap); \
        break;
        OT_LK_ROWS(OT_CASE)
#undef OT_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ot
