// ot_lk_batch.hip -- batched Lucas-Kanade tracking kernels for gfx950 over a
// flattened multi-stream table: waves per workgroup and points per wave as
// template shapes, and a persistent work-claiming form.
#include "ot_launch.hpp"
#include "ot_lk_sched.hpp"

namespace ot {

// Index of the job whose prefix range holds item i (prefix has njobs+1 entries).
__device__ __forceinline__ int find_job(const int32_t* __restrict__ prefix, int njobs, int i) {
    int lo = 0, hi = njobs;  // invariant: prefix[lo] <= i < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

template <int R, int WIN = 0, int MARGIN = 0, bool WSYNC = false>
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
    const LkResult r = lk_point<R, (WIN > 0), false, DevPyr, WSYNC, LK_PRIO_ITERATIONS>(jb.prev, jb.next, ux, uy, jb.levels, hd.lk.iters, hd.lk.eps2,
                                   hd.lk.min_eig, g, smem, nullptr, nullptr);
    if ((threadIdx.x & 63) == 0) {
        jb.next_pts[2 * li] = r.nx;
        jb.next_pts[2 * li + 1] = r.ny;
        jb.status[li] = (uint8_t)r.status;
        if (jb.err) jb.err[li] = r.err;
    }
}

// The flattened points of every job: WPG waves per workgroup, each tracking
// PPW consecutive points one after the other (each wave with its own LDS
// slice of lds_wave bytes; the waves never synchronise with each other).
template <int R, int WIN = 0, int MARGIN = 0, int WPG = 1, int PPW = 1>
__global__ __launch_bounds__(64 * WPG) void k_lk_batch(const uint8_t* __restrict__ table, int cap) {
    extern __shared__ __align__(16) unsigned char lk_smem[];
    static_assert(WPG == 1 || (WIN > 0 && MARGIN > 0), "several waves need a fixed geometry");
    constexpr int LDSW = WIN > 0 ? (int)((lk_lds_bytes(WIN, R, MARGIN) + 15) & ~(size_t)15) : 0;
    const TableLayout T = TableLayout::make(cap);
    const TableHdr& hd = *reinterpret_cast<const TableHdr*>(table);
    const int wv = WPG > 1 ? (int)(threadIdx.x >> 6) : 0;
    const int first = (lk_item(blockIdx.x, gridDim.x) * WPG + wv) * PPW;
    unsigned char* smem = lk_smem + wv * LDSW;
#pragma unroll 1
    for (int j = 0; j < PPW; ++j) {
        const int i = first + j;
        if (i >= hd.total_pts) return;
        lk_batch_item<R, WIN, MARGIN, (WPG > 1)>(table, T, hd, i, smem);
    }
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

int batch_lk_shape_ok(int win, int margin, int wpg, int ppw) {
    if (wpg == 1 && ppw == 1) return 1;
    const bool fixed = lk_template_rows(win) == 7 && win == 21 && (margin == 4 || margin == 6);
    const bool w_ok = wpg == 1 || wpg == 2 || wpg == 4;
    const bool p_ok = ppw == 1 || ppw == 2 || ppw == 4;
    return fixed && w_ok && p_ok ? 1 : 0;
}

hipError_t launch_batch_lk(const uint8_t* table, int cap, int win, int margin, int npts,
                           int lk_waves, int wpg, int ppw, hipStream_t stream) {
    const int R = lk_template_rows(win);
    const size_t lds = (lk_lds_bytes(win, R, margin) + 15) & ~(size_t)15;
    const bool persistent = lk_waves > 0;
    if (!batch_lk_shape_ok(win, margin, wpg, ppw) || (persistent && (wpg != 1 || ppw != 1)))
        return hipErrorInvalidValue;
    if (R == 7 && win == 21 && (margin == 4 || margin == 6)) {
        if (persistent) {
            if (margin == 4)
                hipLaunchKernelGGL((k_lk_batch_persistent<7, 21, 4>), dim3(lk_waves), dim3(64), lds,
                                   stream, const_cast<uint8_t*>(table), cap);
            else
                hipLaunchKernelGGL((k_lk_batch_persistent<7, 21, 6>), dim3(lk_waves), dim3(64), lds,
                                   stream, const_cast<uint8_t*>(table), cap);
            return hipGetLastError();
        }
        const int per = wpg * ppw;
        const int grid = (npts + per - 1) / per;
#define OT_SHAPE(MM, WW, PP)                                                                  \
    if (margin == MM && wpg == WW && ppw == PP)                                               \
        hipLaunchKernelGGL((k_lk_batch<7, 21, MM, WW, PP>), dim3(grid), dim3(64 * WW), WW * lds, \
                           stream, table, cap);
#define OT_SHAPES(MM) \
    OT_SHAPE(MM, 1, 1) OT_SHAPE(MM, 1, 2) OT_SHAPE(MM, 1, 4) OT_SHAPE(MM, 2, 1) \
    OT_SHAPE(MM, 2, 2) OT_SHAPE(MM, 2, 4) OT_SHAPE(MM, 4, 1) OT_SHAPE(MM, 4, 2) OT_SHAPE(MM, 4, 4)
        OT_SHAPES(4)
        OT_SHAPES(6)
#undef OT_SHAPES
#undef OT_SHAPE
        return hipGetLastError();
    }
    switch (R) {
#define OT_CASE(RR)                                                                             \
    case RR:                                                                                    \
        if (persistent)                                                                         \
            hipLaunchKernelGGL(k_lk_batch_persistent<RR>, dim3(lk_waves), dim3(64), lds, stream, \
                               const_cast<uint8_t*>(table), cap);                               \
        else                                                                                    \
            hipLaunchKernelGGL(k_lk_batch<RR>, dim3(npts), dim3(64), lds, stream, table, cap);   \
        break;
        OT_LK_ROWS(OT_CASE)
#undef OT_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ot
