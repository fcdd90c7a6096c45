// ot_misc.hip -- pyramid reduce and box-median kernels for gfx950, single and
// batched forms.
#include <mutex>

#include "ot_box.hpp"
#include "ot_pyr.hpp"
#include "ot_launch.hpp"

namespace ot {

__global__ __launch_bounds__(PYR_THREADS) void k_pyr_stage(DevPyr P, int l0, int K) {
    __shared__ PyrSmem sm;
    pyr_fused(P, l0, K, blockIdx.x, blockIdx.y, sm);
}

// Gradient planes of levels 0..levels-1: workgroup t takes tile t of the
// levels' tile lists laid end to end (tpre: first tile of each level).
struct GradLaunch {
    DevPyr P;
    int32_t tpre[OT_MAX_LEVELS + 1];
    int32_t cols[OT_MAX_LEVELS];
    int32_t levels;
};

__global__ __launch_bounds__(GRAD_THREADS) void k_grad(GradLaunch g) {
    __shared__ GradSmem sm;
    const int t = blockIdx.x;
    int l = 0;
    while (l + 1 < g.levels && t >= g.tpre[l + 1]) ++l;
    const int lt = t - g.tpre[l], cols = g.cols[l];
    grad_tile(g.P.lvl[l], g.P.w[l], g.P.h[l], g.P.pitch[l], const_cast<int32_t*>(g.P.grad[l]),
              g.P.gpitch[l], lt % cols, lt / cols, sm);
}

hipError_t launch_grad(const DevPyr& P, int levels, hipStream_t stream) {
    GradLaunch g;
    g.P = P;
    g.levels = levels;
    g.tpre[0] = 0;
    for (int l = 0; l < levels; ++l) {
        g.cols[l] = (P.w[l] + GRAD_TW - 1) / GRAD_TW;
        g.tpre[l + 1] = g.tpre[l] + g.cols[l] * ((P.h[l] + GRAD_TH - 1) / GRAD_TH);
    }
    hipLaunchKernelGGL(k_grad, dim3(g.tpre[levels]), dim3(GRAD_THREADS), 0, stream, g);
    return hipGetLastError();
}

hipError_t launch_pyr_stage(const DevPyr& P, int l0, int K, hipStream_t stream) {
    const int top = l0 + K;
    const dim3 grid((P.w[top] + PYR_FTW - 1) / PYR_FTW, (P.h[top] + PYR_FTH - 1) / PYR_FTH);
    hipLaunchKernelGGL(k_pyr_stage, grid, dim3(PYR_THREADS), 0, stream, P, l0, K);
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

// The fused stage starting at level l0 of every job's next pyramid: one
// workgroup per top-level tile of the flattened tile list (kept at index
// l0 + 1 of the table's per-level tile arrays).
__global__ __launch_bounds__(PYR_THREADS) void k_batch_pyr(const uint8_t* __restrict__ table,
                                                           int cap, int l0) {
    __shared__ PyrSmem sm;
    const TableLayout T = TableLayout::make(cap);
    const TableHdr& hd = *reinterpret_cast<const TableHdr*>(table);
    const int t = blockIdx.x;
    if (t >= hd.total_tiles[l0 + 1]) return;
    const int32_t* tp = reinterpret_cast<const int32_t*>(table + T.tile_prefix) + (size_t)(l0 + 1) * (cap + 1);
    const int32_t* tc = reinterpret_cast<const int32_t*>(table + T.tile_cols) + (size_t)(l0 + 1) * cap;
    const int j = __builtin_amdgcn_readfirstlane(find_item(tp, hd.njobs, t));
    const DevJob& jb = reinterpret_cast<const DevJob*>(table + T.jobs)[j];
    const int lt = t - tp[j];
    const int cols = tc[j];
    pyr_fused(jb.next, l0, pyr_stage_steps(jb.levels, l0), lt % cols, lt / cols, sm);
}

hipError_t launch_batch_pyr(const uint8_t* table, int cap, int l0, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(k_batch_pyr, dim3(grid), dim3(PYR_THREADS), 0, stream, table, cap, l0);
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

__global__ __launch_bounds__(BOX_THREADS) void k_scaled_prep(const float* __restrict__ boxes,
                                                             const int32_t* __restrict__ box_id,
                                                             const float* __restrict__ pts,
                                                             const float* __restrict__ next_pts,
                                                             const uint8_t* __restrict__ status, int n,
                                                             float* __restrict__ out_boxes,
                                                             int32_t* __restrict__ out_count,
                                                             float* __restrict__ out_scale,
                                                             ScaleWs* __restrict__ ws) {
    __shared__ ScaleSmem sm;
    const int b = blockIdx.x >> 1;
    scaled_prep(boxes, b, (int)(blockIdx.x & 1), box_id, pts, next_pts, status, n, out_boxes, out_count,
                out_scale, ws + b, sm);
}

__global__ __launch_bounds__(BOX_THREADS) void k_scaled_hist(ScaleWs* __restrict__ ws, int S) {
    __shared__ SliceSmem sm;
    scaled_hist(ws + blockIdx.x / S, (int)(blockIdx.x % S), S, sm);
}

__global__ __launch_bounds__(BOX_THREADS) void k_scaled_band(ScaleWs* __restrict__ ws, int S) {
    __shared__ SliceSmem sm;
    scaled_band(ws + blockIdx.x / S, (int)(blockIdx.x % S), S, sm);
}

__global__ __launch_bounds__(BOX_THREADS) void k_scaled_final(const float* __restrict__ boxes,
                                                              float* __restrict__ out_boxes,
                                                              int32_t* __restrict__ out_count,
                                                              float* __restrict__ out_scale,
                                                              const ScaleWs* __restrict__ ws) {
    __shared__ ScaleSmem sm;
    scaled_final(boxes, blockIdx.x, out_boxes, out_count, out_scale, ws + blockIdx.x, sm);
}

size_t box_scaled_ws_bytes(int m) { return (size_t)m * sizeof(ScaleWs); }

int box_scaled_slices(int m) { return m >= 256 ? 1 : min(64, 256 / m); }

hipError_t launch_box_scaled(const float* boxes, int m, const int32_t* box_id, const float* pts,
                             const float* next_pts, const uint8_t* status, int n, float* out_boxes,
                             int32_t* out_count, float* out_scale, void* ws, hipStream_t stream) {
    ScaleWs* w = static_cast<ScaleWs*>(ws);
    const int S = box_scaled_slices(m);
    hipLaunchKernelGGL(k_scaled_prep, dim3(2 * m), dim3(BOX_THREADS), 0, stream, boxes, box_id, pts,
                       next_pts, status, n, out_boxes, out_count, out_scale, w);
    hipLaunchKernelGGL(k_scaled_hist, dim3(m * S), dim3(BOX_THREADS), 0, stream, w, S);
    hipLaunchKernelGGL(k_scaled_band, dim3(m * S), dim3(BOX_THREADS), 0, stream, w, S);
    hipLaunchKernelGGL(k_scaled_final, dim3(m), dim3(BOX_THREADS), 0, stream, boxes, out_boxes,
                       out_count, out_scale, w);
    return hipGetLastError();
}

// Scratch of the allocation-free scaled update: a static device array (one
// copy per GPU).  Host code never passes `scratch` itself to a kernel -- on
// the host that name is only a stand-in for the symbol -- but the device
// address hipGetSymbolAddress returns for it, looked up once per device with
// that device current.
static __device__ __align__(256) ScaleWs scratch[OT_SCALED_NOALLOC_MAX_BOXES];

namespace {
constexpr int SCRATCH_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_addr[SCRATCH_DEVICES] = {};

hipError_t scratch_for_stream(hipStream_t stream, void** out) {
    hipDevice_t dev = -1;
    hipError_t e = hipStreamGetDevice(stream, &dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= SCRATCH_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_addr[dev]) {
        int cur = -1;
        if ((e = hipGetDevice(&cur)) != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_addr[dev] = p;
    }
    *out = scratch_addr[dev];
    return hipSuccess;
}
}  // namespace

hipError_t launch_box_scaled_noalloc(const float* boxes, int m, const int32_t* box_id,
                                     const float* pts, const float* next_pts,
                                     const uint8_t* status, int n, float* out_boxes,
                                     int32_t* out_count, float* out_scale, hipStream_t stream) {
    if (m < 1 || m > OT_SCALED_NOALLOC_MAX_BOXES) return hipErrorInvalidValue;
    void* ws = nullptr;
    const hipError_t e = scratch_for_stream(stream, &ws);
    if (e != hipSuccess) return e;
    // the kernels clear the per-box counters and histograms they use
    return launch_box_scaled(boxes, m, box_id, pts, next_pts, status, n, out_boxes, out_count,
                             out_scale, ws, stream);
}

// Points by descending total iterations: a counting sort in one workgroup.
// Key k = sum of a point's per-level counts (<= 8 * 255 < ORD_BINS); bin
// ORD_BINS-1-k holds key k, so an ascending scan of the bins lists the
// largest keys first.  Slots within a bin are taken with LDS atomics (ties in
// any order).  Each thread keeps the keys of its first ORD_KEEP points in
// registers between the two passes (points past that are read again).
constexpr int ORD_THREADS = 1024, ORD_BINS = 2048, ORD_KEEP = 16;

__device__ __forceinline__ int ord_key(const uint8_t* __restrict__ iters, int i, int levels) {
    const uint8_t* p = iters + (size_t)i * levels;
    int k = 0;
#pragma unroll
    for (int l = 0; l < OT_MAX_LEVELS; ++l)
        if (l < levels) k += p[l];
    return min(k, ORD_BINS - 1);
}

__global__ __launch_bounds__(ORD_THREADS) void k_lk_order(const uint8_t* __restrict__ iters, int n,
                                                          int levels, int32_t* __restrict__ order) {
    __shared__ uint32_t bin[ORD_BINS];
    __shared__ uint32_t wsum[ORD_THREADS / 64];
    const int tid = threadIdx.x;
    for (int b = tid; b < ORD_BINS; b += ORD_THREADS) bin[b] = 0u;
    int key[ORD_KEEP];
#pragma unroll
    for (int q = 0; q < ORD_KEEP; ++q) {
        const int i = tid + q * ORD_THREADS;
        key[q] = i < n ? ord_key(iters, i, levels) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < ORD_KEEP; ++q)
        if (tid + q * ORD_THREADS < n) atomicAdd(&bin[ORD_BINS - 1 - key[q]], 1u);
    for (int i = tid + ORD_KEEP * ORD_THREADS; i < n; i += ORD_THREADS)
        atomicAdd(&bin[ORD_BINS - 1 - ord_key(iters, i, levels)], 1u);
    __syncthreads();
    // exclusive scan of the bins: each thread owns two consecutive bins
    const uint32_t a = bin[2 * tid], b = bin[2 * tid + 1];
    const uint32_t incl = wave_incl_scan_u32(a + b);
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    uint32_t before = 0u;
    for (int k = 0; k < wv; ++k) before += wsum[k];
    const uint32_t ex = before + incl - (a + b);
    __syncthreads();
    bin[2 * tid] = ex;
    bin[2 * tid + 1] = ex + a;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < ORD_KEEP; ++q) {
        const int i = tid + q * ORD_THREADS;
        if (i < n) order[atomicAdd(&bin[ORD_BINS - 1 - key[q]], 1u)] = i;
    }
    for (int i = tid + ORD_KEEP * ORD_THREADS; i < n; i += ORD_THREADS)
        order[atomicAdd(&bin[ORD_BINS - 1 - ord_key(iters, i, levels)], 1u)] = i;
}

hipError_t launch_lk_order(const uint8_t* iters, int n, int levels, int32_t* order,
                           hipStream_t stream) {
    static_assert(2 * ORD_THREADS == ORD_BINS, "two bins per thread");
    hipLaunchKernelGGL(k_lk_order, dim3(1), dim3(ORD_THREADS), 0, stream, iters, n, levels, order);
    return hipGetLastError();
}

constexpr int FB_THREADS = 256;

__global__ __launch_bounds__(FB_THREADS) void k_fb_gate(const float* __restrict__ pts,
                                                        const float* __restrict__ back_pts,
                                                        const uint8_t* __restrict__ st_fwd,
                                                        const uint8_t* __restrict__ st_bwd, int n,
                                                        float fb_max, float* __restrict__ fb_err,
                                                        uint8_t* __restrict__ status_out) {
    const int i = blockIdx.x * FB_THREADS + threadIdx.x;
    if (i < n) fb_gate_point(pts, back_pts, st_fwd, st_bwd, i, fb_max, fb_err, status_out);
}

hipError_t launch_fb_gate(const float* pts, const float* back_pts, const uint8_t* st_fwd,
                          const uint8_t* st_bwd, int n, float fb_max, float* fb_err,
                          uint8_t* status_out, hipStream_t stream) {
    const int grid = (n + FB_THREADS - 1) / FB_THREADS;
    hipLaunchKernelGGL(k_fb_gate, dim3(grid), dim3(FB_THREADS), 0, stream, pts, back_pts, st_fwd,
                       st_bwd, n, fb_max, fb_err, status_out);
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
