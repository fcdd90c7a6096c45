// ot_misc.hip -- pyramid reduce and box-median kernels for gfx950, single and
// batched forms.
#include "ot_device.hpp"
#include "ot_launch.hpp"

namespace ot {

__global__ __launch_bounds__(PYR_THREADS) void k_pyr_level(const uint8_t* __restrict__ src, int sw,
                                                           int sh, int sp, uint8_t* __restrict__ dst,
                                                           int dw, int dh, int dp) {
    __shared__ PyrSmem sm;
    pyr_tile(src, sw, sh, sp, dst, dw, dh, dp, blockIdx.x, blockIdx.y, sm);
}

hipError_t launch_pyr_level(const uint8_t* src, int sw, int sh, int sp, uint8_t* dst, int dw,
                            int dh, int dp, hipStream_t stream) {
    const dim3 grid((dw + PYR_TW - 1) / PYR_TW, (dh + PYR_TH - 1) / PYR_TH);
    hipLaunchKernelGGL(k_pyr_level, grid, dim3(PYR_THREADS), 0, stream, src, sw, sh, sp, dst, dw,
                       dh, dp);
    return hipGetLastError();
}

__device__ __forceinline__ int find_item(const int32_t* __restrict__ prefix, int njobs, int i) {
    int lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// Level `level` of every job's next pyramid: one workgroup per tile of the
// flattened tile list.
__global__ __launch_bounds__(PYR_THREADS) void k_batch_pyr(const uint8_t* __restrict__ table,
                                                           int cap, int level) {
    __shared__ PyrSmem sm;
    const TableLayout T = TableLayout::make(cap);
    const TableHdr& hd = *reinterpret_cast<const TableHdr*>(table);
    const int t = blockIdx.x;
    if (t >= hd.total_tiles[level]) return;
    const int32_t* tp = reinterpret_cast<const int32_t*>(table + T.tile_prefix) + (size_t)level * (cap + 1);
    const int32_t* tc = reinterpret_cast<const int32_t*>(table + T.tile_cols) + (size_t)level * cap;
    const int j = __builtin_amdgcn_readfirstlane(find_item(tp, hd.njobs, t));
    const DevJob& jb = reinterpret_cast<const DevJob*>(table + T.jobs)[j];
    const int lt = t - tp[j];
    const int cols = tc[j];
    const DevPyr& P = jb.next;
    pyr_tile(P.lvl[level - 1], P.w[level - 1], P.h[level - 1], P.pitch[level - 1],
             const_cast<uint8_t*>(P.lvl[level]), P.w[level], P.h[level], P.pitch[level],
             lt % cols, lt / cols, sm);
}

hipError_t launch_batch_pyr(const uint8_t* table, int cap, int level, int grid,
                            hipStream_t stream) {
    hipLaunchKernelGGL(k_batch_pyr, dim3(grid), dim3(PYR_THREADS), 0, stream, table, cap, level);
    return hipGetLastError();
}

__global__ __launch_bounds__(BOX_THREADS) void k_box(const float* __restrict__ boxes, int m,
                                                     const int32_t* __restrict__ box_id,
                                                     const float* __restrict__ pts,
                                                     const float* __restrict__ next_pts,
                                                     const uint8_t* __restrict__ status, int n,
                                                     float* __restrict__ out_boxes,
                                                     int32_t* __restrict__ out_count) {
    __shared__ BoxSmem sm;
    box_median(boxes, blockIdx.x, box_id, pts, next_pts, status, n, out_boxes, out_count, sm);
}

hipError_t launch_box(const float* boxes, int m, const int32_t* box_id, const float* pts,
                      const float* next_pts, const uint8_t* status, int n, float* out_boxes,
                      int32_t* out_count, hipStream_t stream) {
    hipLaunchKernelGGL(k_box, dim3(m), dim3(BOX_THREADS), 0, stream, boxes, m, box_id, pts,
                       next_pts, status, n, out_boxes, out_count);
    return hipGetLastError();
}

__global__ __launch_bounds__(BOX_THREADS) void k_batch_box(const uint8_t* __restrict__ table,
                                                           int cap) {
    __shared__ BoxSmem sm;
    const TableLayout T = TableLayout::make(cap);
    const TableHdr& hd = *reinterpret_cast<const TableHdr*>(table);
    const int t = blockIdx.x;
    if (t >= hd.total_boxes) return;
    const int32_t* bp = reinterpret_cast<const int32_t*>(table + T.box_prefix);
    const int j = __builtin_amdgcn_readfirstlane(find_item(bp, hd.njobs, t));
    const DevJob& jb = reinterpret_cast<const DevJob*>(table + T.jobs)[j];
    box_median(jb.boxes, t - bp[j], jb.box_id, jb.pts, jb.next_pts, jb.status, jb.n,
               jb.out_boxes, jb.out_count, sm);
}

hipError_t launch_batch_box(const uint8_t* table, int cap, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(k_batch_box, dim3(grid), dim3(BOX_THREADS), 0, stream, table, cap);
    return hipGetLastError();
}

}  // namespace ot
