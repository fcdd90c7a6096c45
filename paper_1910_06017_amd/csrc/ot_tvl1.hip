// ot_tvl1.hip -- dense TV-L1 optical flow for gfx950 (Sec. IV): Huber total
// variation, projected dual steps, structure-texture inputs, coarse-to-fine
// warps (Zach, Pock & Bischof 2007; Werlberger et al. 2009; Wedel et al.
// 2009); and the per-box mean of the dense field (Sec. V-A prediction).
//
// Every pass is a 2-D stencil over float planes.  The pointwise passes run
// one thread per pixel in 64 x 4 workgroups (a wave reads a row segment of
// every plane; neighbour reads hit the same lines in L1/L2).  The iterated
// passes (the structure dual and the TV-L1 iteration) run up to TV_K
// iterations per launch on LDS tiles with a TV_K-pixel halo.  Launches
// ping-pong between two buffers so no workgroup reads what another one
// writes in the same launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "omnitrack.h"

namespace ot {
namespace {

constexpr int TV_BX = 64, TV_BY = 4;

// grad u at (x, y): forward differences, 0 on the last column / row.
__device__ __forceinline__ float fwd_x(float c, float r, int x, int W) { return x + 1 < W ? r - c : 0.0f; }
__device__ __forceinline__ float fwd_y(float c, float d, int y, int H) { return y + 1 < H ? d - c : 0.0f; }

// div p at (x, y) from p at (x, y), (x-1, y) and (x, y-1): backward
// differences with p taken as 0 on the last column / row and before the
// first (the negative adjoint of the forward-difference gradient).
template <class GetX, class GetY>
__device__ __forceinline__ float div_at(int x, int y, int W, int H, GetX&& px, GetY&& py) {
    float d = 0.0f;
    if (x + 1 < W) d += px(x, y);
    if (x > 0) d -= px(x - 1, y);
    if (y + 1 < H) d += py(x, y);
    if (y > 0) d -= py(x, y - 1);
    return d;
}

// ---------------------------------------------------------------- structure
// texture = f - alpha * (f - theta div p), both frames (blockIdx.z).
__global__ __launch_bounds__(TV_BX* TV_BY) void k_texture(const uint8_t* __restrict__ img0, int pitch0,
                                                          const uint8_t* __restrict__ img1, int pitch1,
                                                          int W, int H, const float2* __restrict__ p0,
                                                          const float2* __restrict__ p1,
                                                          float* __restrict__ tex0,
                                                          float* __restrict__ tex1, float theta,
                                                          float alpha) {
    const int x = blockIdx.x * TV_BX + threadIdx.x, y = blockIdx.y * TV_BY + threadIdx.y;
    if (x >= W || y >= H) return;
    const bool second = blockIdx.z != 0;
    const uint8_t* __restrict__ img = second ? img1 : img0;
    const int pitch = second ? pitch1 : pitch0;
    const float2* __restrict__ p = second ? p1 : p0;
    float* __restrict__ tex = second ? tex1 : tex0;
    const float f = (float)img[(size_t)y * pitch + x] * (1.0f / 255.0f);
    auto pxf = [&](int xx, int yy) { return p[(size_t)yy * W + xx].x; };
    auto pyf = [&](int xx, int yy) { return p[(size_t)yy * W + xx].y; };
    const float s = f - theta * div_at(x, y, W, H, pxf, pyf);
    tex[(size_t)y * W + x] = f - alpha * s;
}

// (I(x+1) - I(x-1)) / 2 with clamped indices, both axes.
__global__ __launch_bounds__(TV_BX* TV_BY) void k_central_grad(const float* __restrict__ I, int W, int H,
                                                               float2* __restrict__ g) {
    const int x = blockIdx.x * TV_BX + threadIdx.x, y = blockIdx.y * TV_BY + threadIdx.y;
    if (x >= W || y >= H) return;
    const size_t r = (size_t)y * W;
    const float xp = I[r + min(x + 1, W - 1)], xm = I[r + max(x - 1, 0)];
    const float yp = I[(size_t)min(y + 1, H - 1) * W + x], ym = I[(size_t)max(y - 1, 0) * W + x];
    g[r + x] = make_float2(0.5f * (xp - xm), 0.5f * (yp - ym));
}

// Bilinear sample with the position clamped to the plane.
template <class T, class Get>
__device__ __forceinline__ T bilin(float x, float y, int W, int H, Get&& get) {
    x = fminf(fmaxf(x, 0.0f), (float)(W - 1));
    y = fminf(fmaxf(y, 0.0f), (float)(H - 1));
    const float fx = floorf(x), fy = floorf(y);
    const int x0 = (int)fx, y0 = (int)fy;
    const int x1 = min(x0 + 1, W - 1), y1 = min(y0 + 1, H - 1);
    const float a = x - fx, b = y - fy;
    return (1.0f - a) * (1.0f - b) * get(x0, y0) + a * (1.0f - b) * get(x1, y0) +
           (1.0f - a) * b * get(x0, y1) + a * b * get(x1, y1);
}

// Linearisation of the data term at pixel (x, y) and the current flow u0:
// data = (gx, gy, rho0, gx^2 + gy^2) with rho(u) = rho0 + g . u.
__device__ __forceinline__ float4 warp_data(const float* __restrict__ I0,
                                            const float* __restrict__ I1,
                                            const float2* __restrict__ G1, int W, int H, int x,
                                            int y, float2 u0) {
    const float wx = (float)x + u0.x, wy = (float)y + u0.y;
    const float I1w = bilin<float>(wx, wy, W, H, [&](int a, int b) { return I1[(size_t)b * W + a]; });
    const float gx = bilin<float>(wx, wy, W, H, [&](int a, int b) { return G1[(size_t)b * W + a].x; });
    const float gy = bilin<float>(wx, wy, W, H, [&](int a, int b) { return G1[(size_t)b * W + a].y; });
    const float rho0 = I1w - gx * u0.x - gy * u0.y - I0[(size_t)y * W + x];
    return make_float4(gx, gy, rho0, gx * gx + gy * gy);
}

// Flow of a finer level at (x, y) from the coarser one (Wc x Hc): 2 u(x / 2).
__device__ __forceinline__ float2 upsample_at(const float2* __restrict__ uc, int Wc, int Hc, int x,
                                              int y) {
    const float sx = 0.5f * (float)x, sy = 0.5f * (float)y;
    const float a = bilin<float>(sx, sy, Wc, Hc, [&](int i, int j) { return uc[(size_t)j * Wc + i].x; });
    const float b = bilin<float>(sx, sy, Wc, Hc, [&](int i, int j) { return uc[(size_t)j * Wc + i].y; });
    return make_float2(2.0f * a, 2.0f * b);
}

// Where the first launch of a warp takes the data term from: the textures and
// the gradient of the second (I0 == nullptr: read `data` as written before);
// and where the first launch of a level takes the flow from: init 0 reads
// u_in, 1 starts from zero (the coarsest level), 2 upsamples the coarser
// level's flow uc (Wc x Hc).
struct WarpSrc {
    const float* I0;
    const float* I1;
    const float2* G1;
    float4* data_out;  // the tile's own pixels' data, for the warp's later launches
    const float2* uc;
    int Wc, Hc, init;
};

// Pointwise L1 data step: v minimising |v - u|^2 / (2 theta) + lam |rho(v)|.
__device__ __forceinline__ float2 data_step(float2 u, float4 d, float lt) {
    const float rho = d.z + d.x * u.x + d.y * u.y;
    const float t = lt * d.w;
    float s;
    if (rho < -t) s = lt;
    else if (rho > t) s = -lt;
    else if (d.w > 0.0f) s = -rho * __builtin_amdgcn_rcpf(d.w);
    else s = 0.0f;
    return make_float2(u.x + s * d.x, u.y + s * d.y);
}

// ------------------------------------------------------ temporally blocked
// Up to K iterations in one launch: a workgroup owns a TX x TY tile and
// loads the state of the tile plus a K-pixel halo into LDS.  Each iteration
// has two phases separated by barriers, both in place: phase A needs the
// dual at the pixel and its left and upper neighbours, phase B the primal
// at the pixel and its right and lower neighbours, so every iteration
// invalidates one more ring of the region on each side and after n <= K
// iterations exactly the tile is exact.  Region pixels outside the frame are
// never used (the difference rules at the frame's edges do not reach past
// it); reads past the region's own edge fall in the invalid ring and take 0
// (dual) or the pixel's own value (primal).
#ifndef OT_TV_K
#define OT_TV_K 5
#endif

// Tile TX x TY outputs, NT threads; the region is the tile plus the halo.
template <int K, int TX, int TY, int NT>
struct TileGeom {
    static constexpr int RX = TX + 2 * K, RY = TY + 2 * K, RN = RX * RY;
    static constexpr int PER = (RN + NT - 1) / NT;  // region pixels per thread
};
// Large tiles for large levels; small ones where large tiles would leave
// most compute units idle (each workgroup's critical path is its region).
constexpr int TBL_X = 64, TBL_Y = 16, TBL_T = 1024;
// tiles of the TV-L1 iterations on large levels
#ifndef OT_TVF_X
#define OT_TVF_X 32
#endif
#ifndef OT_TVF_Y
#define OT_TVF_Y 32
#endif
#ifndef OT_TVF_K
#define OT_TVF_K 5
#endif
constexpr int TBF_X = OT_TVF_X, TBF_Y = OT_TVF_Y, TBF_T = 1024, TV_KF = OT_TVF_K;
#ifndef OT_TVS_T
#define OT_TVS_T 512
#endif
#ifndef OT_TVS_Y
#define OT_TVS_Y 8
#endif
#ifndef OT_TVS_X
#define OT_TVS_X 16
#endif
constexpr int TBS_X = OT_TVS_X, TBS_Y = OT_TVS_Y, TBS_T = OT_TVS_T;
// Levels whose small-tile grid would still leave most compute units idle
// (fewer than 256 workgroups) are bound by each launch's fixed cost (the
// loads, the stores, the dispatch): their TV-L1 iterations run OT_TV_KT per
// launch on the same tiles with an OT_TV_KT-pixel halo, one region pixel per
// thread.
#ifndef OT_TV_KT
#define OT_TV_KT 10
#endif
constexpr int TBT_T = 1024;
// Levels between: the TV-L1 iterations on wider tiles (less halo per output)
// when those still give 256 workgroups.
#ifndef OT_TVM_X
#define OT_TVM_X 16
#endif
#ifndef OT_TVM_Y
#define OT_TVM_Y 16
#endif
#ifndef OT_TVM_T
#define OT_TVM_T 676
#endif
constexpr int TBM_X = OT_TVM_X, TBM_Y = OT_TVM_Y, TBM_T = OT_TVM_T;

// n (<= K) TV-L1 iterations: v = data step of u, u = v + theta div p (both
// flow components), p = projection onto the unit ball of (p + (tau/theta)
// grad u) / (1 + tau eps / theta); p is (p1x, p1y, p2x, p2y) per pixel and
// taken as 0 when `first`.
// With ws.I0 set (the first launch of a warp) the data term of every region
// pixel is computed from the flow the launch reads, and the tile's own
// pixels' terms are stored for the warp's later launches.
template <int K, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_tvl1_block(const float4* __restrict__ data, WarpSrc ws,
                                                           const float2* __restrict__ u_in,
                                                           const float4* __restrict__ p_in,
                                                           float2* __restrict__ u_out,
                                                           float4* __restrict__ p_out, int W, int H,
                                                           float lt, float theta, float k,
                                                           float inv_shrink, int first, int n) {
    using G = TileGeom<K, TX, TY, NT>;
    __shared__ float2 su[G::RN];
    __shared__ float4 sp[G::RN];
    const int tid = threadIdx.x;
    const int ox = blockIdx.x * TX - K, oy = blockIdx.y * TY - K;
    float4 dat[G::PER];
#pragma unroll
    for (int q = 0; q < G::PER; ++q) {
        const int r = tid + q * NT;
        if (r >= G::RN) break;
        const int lx = r % G::RX, ly = r / G::RX, gx = ox + lx, gy = oy + ly;
        const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
        const size_t i = in ? (size_t)gy * W + gx : 0;
        float2 u0 = make_float2(0.0f, 0.0f);
        if (in && ws.init == 0) u0 = u_in[i];
        else if (in && ws.init == 2) u0 = upsample_at(ws.uc, ws.Wc, ws.Hc, gx, gy);
        su[r] = u0;
        sp[r] = (in && !first) ? p_in[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (ws.I0) {
            dat[q] = in ? warp_data(ws.I0, ws.I1, ws.G1, W, H, gx, gy, u0)
                        : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (in && lx >= K && lx < K + TX && ly >= K && ly < K + TY) ws.data_out[i] = dat[q];
        } else {
            dat[q] = in ? data[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
    }
    __syncthreads();
    for (int it = 0; it < n; ++it) {
        // phase A: u = data step of u + theta div p
#pragma unroll
        for (int q = 0; q < G::PER; ++q) {
            const int r = tid + q * NT;
            if (r >= G::RN) break;
            const int lx = r % G::RX, ly = r / G::RX, gx = ox + lx, gy = oy + ly;
            if (gx < 0 || gx >= W || gy < 0 || gy >= H) continue;
            const float2 v = data_step(su[r], dat[q], lt);
            const float4 pc = sp[r];
            const float4 pl = (gx > 0 && lx > 0) ? sp[r - 1] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            const float4 pu = (gy > 0 && ly > 0) ? sp[r - G::RX] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            float d1 = 0.0f, d2 = 0.0f;
            if (gx + 1 < W) {
                d1 += pc.x;
                d2 += pc.z;
            }
            if (gx > 0) {
                d1 -= pl.x;
                d2 -= pl.z;
            }
            if (gy + 1 < H) {
                d1 += pc.y;
                d2 += pc.w;
            }
            if (gy > 0) {
                d1 -= pu.y;
                d2 -= pu.w;
            }
            su[r] = make_float2(v.x + theta * d1, v.y + theta * d2);
        }
        __syncthreads();
        // phase B: dual step and projection
#pragma unroll
        for (int q = 0; q < G::PER; ++q) {
            const int r = tid + q * NT;
            if (r >= G::RN) break;
            const int lx = r % G::RX, ly = r / G::RX, gx = ox + lx, gy = oy + ly;
            if (gx < 0 || gx >= W || gy < 0 || gy >= H) continue;
            const float2 uc = su[r];
            const float2 ur = lx + 1 < G::RX ? su[r + 1] : uc;
            const float2 ud = ly + 1 < G::RY ? su[r + G::RX] : uc;
            const float4 p = sp[r];
            const float q1x = (p.x + k * fwd_x(uc.x, ur.x, gx, W)) * inv_shrink;
            const float q1y = (p.y + k * fwd_y(uc.x, ud.x, gy, H)) * inv_shrink;
            const float q2x = (p.z + k * fwd_x(uc.y, ur.y, gx, W)) * inv_shrink;
            const float q2y = (p.w + k * fwd_y(uc.y, ud.y, gy, H)) * inv_shrink;
            // projection: scale by min(1, 1/|q|) (|q| = 0 gives inf, so 1)
            const float s1 = fminf(1.0f, __builtin_amdgcn_rsqf(q1x * q1x + q1y * q1y));
            const float s2 = fminf(1.0f, __builtin_amdgcn_rsqf(q2x * q2x + q2y * q2y));
            sp[r] = make_float4(q1x * s1, q1y * s1, q2x * s2, q2y * s2);
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < G::PER; ++q) {
        const int r = tid + q * NT;
        if (r >= G::RN) break;
        const int lx = r % G::RX, ly = r / G::RX, gx = ox + lx, gy = oy + ly;
        if (lx < K || lx >= K + TX || ly < K || ly >= K + TY || gx >= W || gy >= H) continue;
        const size_t i = (size_t)gy * W + gx;
        u_out[i] = su[r];
        p_out[i] = sp[r];
    }
}

// n (<= K) dual steps of the structure (ROF) problem on f = img / 255:
// w = div p - f / theta, p <- (p + tau grad w) / (1 + tau |grad w|); p taken
// as 0 when `first`.
// The two frames of a pair, one per blockIdx.z.
struct FramePair {
    const uint8_t* img[2];
    int pitch[2];
    const float2* p_in[2];
    float2* p_out[2];
};

template <int K, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_rof_block(FramePair fp, int W, int H, float inv_theta,
                                                  float tau, int first, int n) {
    using G = TileGeom<K, TX, TY, NT>;
    const uint8_t* __restrict__ img = fp.img[blockIdx.z];
    const int pitch = fp.pitch[blockIdx.z];
    const float2* __restrict__ p_in = fp.p_in[blockIdx.z];
    float2* __restrict__ p_out = fp.p_out[blockIdx.z];
    __shared__ float2 sp[G::RN];
    __shared__ float sw[G::RN];
    const int tid = threadIdx.x;
    const int ox = blockIdx.x * TX - K, oy = blockIdx.y * TY - K;
    float fs[G::PER];
#pragma unroll
    for (int q = 0; q < G::PER; ++q) {
        const int r = tid + q * NT;
        if (r >= G::RN) break;
        const int gx = ox + r % G::RX, gy = oy + r / G::RX;
        const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
        sp[r] = (in && !first) ? p_in[(size_t)gy * W + gx] : make_float2(0.0f, 0.0f);
        fs[q] = in ? (float)img[(size_t)gy * pitch + gx] * (1.0f / 255.0f) * inv_theta : 0.0f;
    }
    __syncthreads();
    for (int it = 0; it < n; ++it) {
        // phase A: w = div p - f / theta
#pragma unroll
        for (int q = 0; q < G::PER; ++q) {
            const int r = tid + q * NT;
            if (r >= G::RN) break;
            const int lx = r % G::RX, ly = r / G::RX, gx = ox + lx, gy = oy + ly;
            if (gx < 0 || gx >= W || gy < 0 || gy >= H) continue;
            const float2 pc = sp[r];
            float d = 0.0f;
            if (gx + 1 < W) d += pc.x;
            if (gx > 0) d -= lx > 0 ? sp[r - 1].x : 0.0f;
            if (gy + 1 < H) d += pc.y;
            if (gy > 0) d -= ly > 0 ? sp[r - G::RX].y : 0.0f;
            sw[r] = d - fs[q];
        }
        __syncthreads();
        // phase B: p <- (p + tau grad w) / (1 + tau |grad w|)
#pragma unroll
        for (int q = 0; q < G::PER; ++q) {
            const int r = tid + q * NT;
            if (r >= G::RN) break;
            const int lx = r % G::RX, ly = r / G::RX, gx = ox + lx, gy = oy + ly;
            if (gx < 0 || gx >= W || gy < 0 || gy >= H) continue;
            const float wc = sw[r];
            const float gxv = gx + 1 < W ? (lx + 1 < G::RX ? sw[r + 1] : wc) - wc : 0.0f;
            const float gyv = gy + 1 < H ? (ly + 1 < G::RY ? sw[r + G::RX] : wc) - wc : 0.0f;
            const float inrm = __builtin_amdgcn_rcpf(1.0f + tau * sqrtf(gxv * gxv + gyv * gyv));
            const float2 p = sp[r];
            sp[r] = make_float2((p.x + tau * gxv) * inrm, (p.y + tau * gyv) * inrm);
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < G::PER; ++q) {
        const int r = tid + q * NT;
        if (r >= G::RN) break;
        const int lx = r % G::RX, ly = r / G::RX, gx = ox + lx, gy = oy + ly;
        if (lx < K || lx >= K + TX || ly < K || ly >= K + TY || gx >= W || gy >= H) continue;
        p_out[(size_t)gy * W + gx] = sp[r];
    }
}

// Zero flow (the coarsest level's start).
__global__ __launch_bounds__(256) void k_zero2(float2* __restrict__ u, size_t n) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) u[i] = make_float2(0.0f, 0.0f);
}

// ------------------------------------------------------------------ box mean
constexpr int BM_THREADS = 256;

// Mean of the flow over the pixel centres inside box b (edges included,
// clipped to the frame); the box moves by it.  Sums in double.
__global__ __launch_bounds__(BM_THREADS) void k_box_mean(const float2* __restrict__ flow, int W, int H,
                                                         const float* __restrict__ boxes,
                                                         float* __restrict__ out_boxes,
                                                         int32_t* __restrict__ out_count) {
    __shared__ double red[2][BM_THREADS / 64];
    const int b = blockIdx.x, tid = threadIdx.x;
    const float x0 = boxes[4 * b], y0 = boxes[4 * b + 1], x1 = boxes[4 * b + 2], y1 = boxes[4 * b + 3];
    // bounds in float, clamped before the conversion so it cannot overflow
    const int xa = (int)fmaxf(0.0f, ceilf(fminf(x0, (float)W))), xb = (int)fminf((float)(W - 1), floorf(fmaxf(x1, -1.0f)));
    const int ya = (int)fmaxf(0.0f, ceilf(fminf(y0, (float)H))), yb = (int)fminf((float)(H - 1), floorf(fmaxf(y1, -1.0f)));
    const bool any = xa <= xb && ya <= yb && x0 == x0 && y0 == y0 && x1 == x1 && y1 == y1;
    const int bw = any ? xb - xa + 1 : 0, bh = any ? yb - ya + 1 : 0;
    const long long npx = (long long)bw * bh;
    double s1 = 0.0, s2 = 0.0;
    for (long long q = tid; q < npx; q += BM_THREADS) {
        const int yy = ya + (int)(q / bw), xx = xa + (int)(q % bw);
        const float2 v = flow[(size_t)yy * W + xx];
        s1 += v.x;
        s2 += v.y;
    }
    for (int o = 32; o > 0; o >>= 1) {
        s1 += __shfl_xor(s1, o);
        s2 += __shfl_xor(s2, o);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = s1;
        red[1][tid >> 6] = s2;
    }
    __syncthreads();
    if (tid == 0) {
        double t1 = 0.0, t2 = 0.0;
        for (int w = 0; w < BM_THREADS / 64; ++w) {
            t1 += red[0][w];
            t2 += red[1][w];
        }
        float m1 = 0.0f, m2 = 0.0f;
        if (npx > 0) {
            m1 = (float)(t1 / (double)npx);
            m2 = (float)(t2 / (double)npx);
        }
        out_boxes[4 * b] = x0 + m1;
        out_boxes[4 * b + 1] = y0 + m2;
        out_boxes[4 * b + 2] = x1 + m1;
        out_boxes[4 * b + 3] = y1 + m2;
        out_count[b] = (int32_t)min(npx, (long long)INT32_MAX);
    }
}

// ------------------------------------------------------------------ host side
// iterations per blocked launch (the halo width)
constexpr int TV_K = OT_TV_K;
constexpr int TV_KT = OT_TV_KT;
static_assert(TileGeom<TV_KT, TBS_X, TBS_Y, TBT_T>::RN <= TBT_T, "one region pixel per thread");
static_assert(TileGeom<TV_K, TBM_X, TBM_Y, TBM_T>::RN <= TBM_T, "one region pixel per thread");

inline dim3 grid2(int W, int H) { return dim3((W + TV_BX - 1) / TV_BX, (H + TV_BY - 1) / TV_BY); }

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace: structure duals (2 x 2 x float2), data (float4), flow (2 x
// float2) and dual (2 x float4) sized for level 0 and reused by the coarser
// levels; then, per level, the two frames' textures (float) and the second
// texture's gradient (float2), so the structure-texture passes of every level
// can run ahead of the flow.
struct TvLayout {
    size_t r0, r1, r2, r3, d, u0, u1, p0, p1;
    size_t t0[OT_MAX_LEVELS], t1[OT_MAX_LEVELS], g[OT_MAX_LEVELS];
    size_t bytes;
    // w, h: sizes of levels 0 .. L-1
    static TvLayout make(const int32_t* w, const int32_t* h, int L) {
        const size_t n = (size_t)w[0] * h[0];
        TvLayout T{};
        size_t o = 0;
        auto take = [&](size_t b) {
            const size_t at = o;
            o += al256(b);
            return at;
        };
        T.r0 = take(n * 8);
        T.r1 = take(n * 8);
        T.r2 = take(n * 8);
        T.r3 = take(n * 8);
        T.d = take(n * 16);
        T.u0 = take(n * 8);
        T.u1 = take(n * 8);
        T.p0 = take(n * 16);
        T.p1 = take(n * 16);
        for (int l = 0; l < L; ++l) {
            const size_t nl = (size_t)w[l] * h[l];
            T.t0[l] = take(nl * 4);
            T.t1[l] = take(nl * 4);
            T.g[l] = take(nl * 8);
        }
        T.bytes = o;
        return T;
    }
    // the layout for a pyramid of OT_MAX_LEVELS levels of the usual sizes
    // (w_l = ceil(w_{l-1} / 2)), which covers every pyramid built for W x H
    static size_t bound(int32_t W, int32_t H) {
        int32_t w[OT_MAX_LEVELS], h[OT_MAX_LEVELS];
        w[0] = W;
        h[0] = H;
        for (int l = 1; l < OT_MAX_LEVELS; ++l) {
            w[l] = (w[l - 1] + 1) / 2;
            h[l] = (h[l - 1] + 1) / 2;
        }
        return make(w, h, OT_MAX_LEVELS).bytes;
    }
};

// Fork/join events of ot_tvl1_flow_async, one set per device, created on first
// use and kept; the enqueue sequence that records and waits on them holds the
// mutex, so concurrent callers cannot interleave on a shared event.
constexpr int TV_DEVICES = 64;
std::mutex tv_ev_mu;
hipEvent_t tv_ev[TV_DEVICES][OT_MAX_LEVELS + 1];
bool tv_ev_ready[TV_DEVICES];

hipError_t tv_events(int dev, hipEvent_t** out) {
    if (dev < 0 || dev >= TV_DEVICES) return hipErrorInvalidDevice;
    if (!tv_ev_ready[dev]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        int made = 0;
        for (; made <= OT_MAX_LEVELS && e == hipSuccess; ++made)
            e = hipEventCreateWithFlags(&tv_ev[dev][made], hipEventDisableTiming);
        if (e != hipSuccess)
            for (int i = 0; i < made - 1; ++i) (void)hipEventDestroy(tv_ev[dev][i]);
        if (cur != dev) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        tv_ev_ready[dev] = true;
    }
    *out = tv_ev[dev];
    return hipSuccess;
}

bool params_ok(const ot_tvl1_params* p) {
    return p && p->levels >= 1 && p->levels <= OT_MAX_LEVELS && p->warps >= 1 && p->iters >= 1 &&
           p->iters_s >= 0 && std::isfinite(p->lam) && p->lam > 0.0f && std::isfinite(p->theta) &&
           p->theta > 0.0f && std::isfinite(p->tau) && p->tau > 0.0f && p->tau <= 0.25f &&
           std::isfinite(p->eps) && p->eps >= 0.0f && std::isfinite(p->alpha) &&
           std::isfinite(p->theta_s) && p->theta_s > 0.0f && std::isfinite(p->tau_s) &&
           p->tau_s > 0.0f && p->tau_s <= 0.25f;
}

bool pyr_ok(const ot_pyr* p) {
    if (!p || p->levels < 1 || p->levels > OT_MAX_LEVELS) return false;
    for (int l = 0; l < p->levels; ++l)
        if (!p->level[l] || p->w[l] < 1 || p->h[l] < 1 || p->pitch[l] < p->w[l]) return false;
    return true;
}

}  // namespace
}  // namespace ot

using namespace ot;

extern "C" {

void ot_tvl1_default_params(ot_tvl1_params* p) {
    if (!p) return;
    p->levels = 5;
    p->warps = 5;
    p->iters = 30;
    p->lam = 40.0f;
    p->theta = 0.3f;
    p->tau = 0.25f;
    p->eps = 0.01f;
    p->alpha = 0.95f;
    p->theta_s = 0.1f;
    p->tau_s = 0.125f;
    p->iters_s = 50;
}

size_t ot_tvl1_bytes(int32_t W, int32_t H) {
    if (W < 1 || H < 1 || W > 16384 || H > 16384) return 0;
    return TvLayout::bound(W, H);
}

}  // extern "C"

namespace ot {
namespace {

// One frame's structure-texture pyramid for ot_tvl1_texture: the structure
// dual's ping-pong planes (level 0 sized) and, per level, the texture (float)
// and its central-difference gradient (float2).
struct TexLayout {
    size_t r0, r1;
    size_t t[OT_MAX_LEVELS], g[OT_MAX_LEVELS];
    size_t bytes;
    static TexLayout make(const int32_t* w, const int32_t* h, int L) {
        const size_t n = (size_t)w[0] * h[0];
        TexLayout T{};
        size_t o = 0;
        auto take = [&](size_t b) {
            const size_t at = o;
            o += al256(b);
            return at;
        };
        T.r0 = take(n * 8);
        T.r1 = take(n * 8);
        for (int l = 0; l < L; ++l) {
            const size_t nl = (size_t)w[l] * h[l];
            T.t[l] = take(nl * 4);
            T.g[l] = take(nl * 8);
        }
        T.bytes = o;
        return T;
    }
    static size_t bound(int32_t W, int32_t H) {
        int32_t w[OT_MAX_LEVELS], h[OT_MAX_LEVELS];
        w[0] = W;
        h[0] = H;
        for (int l = 1; l < OT_MAX_LEVELS; ++l) {
            w[l] = (w[l - 1] + 1) / 2;
            h[l] = (h[l - 1] + 1) / 2;
        }
        return make(w, h, OT_MAX_LEVELS).bytes;
    }
};

// The structure-texture split of level l of nf (1 or 2) frames, side by side
// in every launch (grid z): iters_s dual steps on the ping-pong planes R[f],
// the textures tex[f], and the central-difference gradient of the last
// frame's texture into grad.
hipError_t split_level(const ot_pyr* const* pyr, int nf, int l, const ot_tvl1_params* prm,
                       float2* const (*R)[2], float* const* tex, float2* grad, hipStream_t a) {
    const int W = pyr[0]->w[l], H = pyr[0]->h[l];
    const dim3 gr = grid2(W, H), bl(TV_BX, TV_BY);
    const dim3 gbl((W + TBL_X - 1) / TBL_X, (H + TBL_Y - 1) / TBL_Y);
    const dim3 gbs((W + TBS_X - 1) / TBS_X, (H + TBS_Y - 1) / TBS_Y);
    const bool large = gbl.x * gbl.y >= 256;
    // levels whose small-tile grid stays under 256 workgroups take OT_TV_KT
    // steps per launch
    const bool tiny_s = !large && gbs.x * gbs.y < 256;
    const int kr = tiny_s ? TV_KT : TV_K;
    int cr = 0;
    for (int it = 0; it < prm->iters_s; it += kr) {
        const int nb = prm->iters_s - it < kr ? prm->iters_s - it : kr;
        FramePair fp;
        for (int f = 0; f < 2; ++f) {
            const int ff = f < nf ? f : 0;
            fp.img[f] = pyr[ff]->level[l];
            fp.pitch[f] = pyr[ff]->pitch[l];
            fp.p_in[f] = R[ff][cr];
            fp.p_out[f] = R[ff][cr ^ 1];
        }
        if (large)
            hipLaunchKernelGGL((k_rof_block<TV_K, TBL_X, TBL_Y, TBL_T>), dim3(gbl.x, gbl.y, nf), dim3(TBL_T), 0,
                               a, fp, W, H, 1.0f / prm->theta_s, prm->tau_s, it == 0 ? 1 : 0, nb);
        else if (tiny_s)
            hipLaunchKernelGGL((k_rof_block<TV_KT, TBS_X, TBS_Y, TBT_T>), dim3(gbs.x, gbs.y, nf), dim3(TBT_T), 0,
                               a, fp, W, H, 1.0f / prm->theta_s, prm->tau_s, it == 0 ? 1 : 0, nb);
        else
            hipLaunchKernelGGL((k_rof_block<TV_K, TBS_X, TBS_Y, TBS_T>), dim3(gbs.x, gbs.y, nf), dim3(TBS_T), 0,
                               a, fp, W, H, 1.0f / prm->theta_s, prm->tau_s, it == 0 ? 1 : 0, nb);
        cr ^= 1;
    }
    if (prm->iters_s == 0) {
        // no structure iterations: p = 0
        for (int f = 0; f < nf; ++f)
            hipLaunchKernelGGL(k_zero2, dim3((unsigned)(((size_t)W * H + 255) / 256)), dim3(256), 0, a,
                               R[f][cr], (size_t)W * H);
    }
    const int f1 = nf - 1;
    hipLaunchKernelGGL(k_texture, dim3(gr.x, gr.y, nf), bl, 0, a, pyr[0]->level[l], pyr[0]->pitch[l],
                       pyr[f1]->level[l], pyr[f1]->pitch[l], W, H, R[0][cr], R[f1][cr], tex[0],
                       tex[f1], prm->theta_s, prm->alpha);
    hipLaunchKernelGGL(k_central_grad, gr, bl, 0, a, tex[f1], W, H, grad);
    return hipGetLastError();
}

// The flow of levels L-1 .. 0 on s from per-level planes: planes(l, I0, I1,
// G1) gives level l's first and second texture and the second's gradient.
// With ev, level l's flow first waits for ev[l].  ws holds the level-0 sized
// data term, flow and dual planes of T.
template <class Planes>
ot_err flow_levels(const ot_pyr* shape, const ot_tvl1_params* prm, uint8_t* base,
                   const TvLayout& T, Planes&& planes, float* flow, hipStream_t s,
                   const hipEvent_t* ev) {
    const int L = prm->levels;
    float4* D = reinterpret_cast<float4*>(base + T.d);
    float2* U[2] = {reinterpret_cast<float2*>(base + T.u0), reinterpret_cast<float2*>(base + T.u1)};
    float4* Pd[2] = {reinterpret_cast<float4*>(base + T.p0), reinterpret_cast<float4*>(base + T.p1)};
    const float lt = prm->lam * prm->theta, k = prm->tau / prm->theta;
    const float inv_shrink = 1.0f / (1.0f + prm->tau * prm->eps / prm->theta);
    int cu = 0;  // index of the current flow buffer
    for (int l = L - 1; l >= 0; --l) {
        const int W = shape->w[l], H = shape->h[l];
        const dim3 gbl((W + TBL_X - 1) / TBL_X, (H + TBL_Y - 1) / TBL_Y);
        const dim3 gbs((W + TBS_X - 1) / TBS_X, (H + TBS_Y - 1) / TBS_Y);
        const bool large = gbl.x * gbl.y >= 256;
        if (ev && hipStreamWaitEvent(s, ev[l], 0) != hipSuccess) return OT_E_LAUNCH;
        const float* I0 = nullptr;
        const float* I1 = nullptr;
        const float2* G1 = nullptr;
        planes(l, I0, I1, G1);
        // initial flow (in the level's first launch): zero at the coarsest
        // level, else the coarser flow doubled; U[cu] holds the coarser flow
        int cp = 0;
        bool first = true;
        const dim3 gbf((W + TBF_X - 1) / TBF_X, (H + TBF_Y - 1) / TBF_Y);
        const bool tiny = !large && gbs.x * gbs.y < 256;
        const dim3 gbm((W + TBM_X - 1) / TBM_X, (H + TBM_Y - 1) / TBM_Y);
        const bool mid = !large && !tiny && gbm.x * gbm.y >= 256;
        const int kb = tiny ? TV_KT : large ? TV_KF : TV_K;  // iterations per launch
        for (int wv = 0; wv < prm->warps; ++wv) {
            for (int it = 0; it < prm->iters; it += kb) {
                const int nb = prm->iters - it < kb ? prm->iters - it : kb;
                // the warp's first launch linearises the data term at the flow it reads
                WarpSrc wsrc{};
                if (it == 0) {
                    wsrc.I0 = I0;
                    wsrc.I1 = I1;
                    wsrc.G1 = G1;
                    wsrc.data_out = D;
                }
                if (wv == 0 && it == 0) {
                    wsrc.init = l == L - 1 ? 1 : 2;
                    wsrc.uc = U[cu];
                    wsrc.Wc = l + 1 < L ? shape->w[l + 1] : 0;
                    wsrc.Hc = l + 1 < L ? shape->h[l + 1] : 0;
                }
                // the last launch of level 0 writes the caller's flow
                const bool last = l == 0 && wv == prm->warps - 1 && it + kb >= prm->iters;
                float2* uo = last ? reinterpret_cast<float2*>(flow) : U[cu ^ 1];
                if (large)
                    hipLaunchKernelGGL((k_tvl1_block<TV_KF, TBF_X, TBF_Y, TBF_T>), gbf, dim3(TBF_T), 0, s, D,
                                       wsrc, U[cu], Pd[cp], uo, Pd[cp ^ 1], W, H, lt, prm->theta, k,
                                       inv_shrink, first ? 1 : 0, nb);
                else if (tiny)
                    hipLaunchKernelGGL((k_tvl1_block<TV_KT, TBS_X, TBS_Y, TBT_T>), gbs, dim3(TBT_T), 0, s, D,
                                       wsrc, U[cu], Pd[cp], uo, Pd[cp ^ 1], W, H, lt, prm->theta, k,
                                       inv_shrink, first ? 1 : 0, nb);
                else if (mid)
                    hipLaunchKernelGGL((k_tvl1_block<TV_K, TBM_X, TBM_Y, TBM_T>), gbm, dim3(TBM_T), 0, s, D,
                                       wsrc, U[cu], Pd[cp], uo, Pd[cp ^ 1], W, H, lt, prm->theta, k,
                                       inv_shrink, first ? 1 : 0, nb);
                else
                    hipLaunchKernelGGL((k_tvl1_block<TV_K, TBS_X, TBS_Y, TBS_T>), gbs, dim3(TBS_T), 0, s, D,
                                       wsrc, U[cu], Pd[cp], uo, Pd[cp ^ 1], W, H, lt, prm->theta, k,
                                       inv_shrink, first ? 1 : 0, nb);
                cu ^= 1;
                cp ^= 1;
                first = false;
            }
        }
    }
    if (hipGetLastError() != hipSuccess) return OT_E_LAUNCH;
    return OT_OK;
}

// Common checks of the flow calls: the parameters, the level sizes of the
// pyramids (equal on every level used) and the workspace.
ot_err flow_args(const ot_pyr* prev_pyr, const ot_pyr* next_pyr, const ot_tvl1_params* prm,
                 const void* ws, size_t ws_bytes, const float* flow, TvLayout* T) {
    if (!pyr_ok(prev_pyr) || !pyr_ok(next_pyr) || !params_ok(prm) || !flow || !ws) return OT_E_INVAL;
    const int L = prm->levels;
    if (L > prev_pyr->levels || L > next_pyr->levels) return OT_E_INVAL;
    for (int l = 0; l < L; ++l)
        if (prev_pyr->w[l] != next_pyr->w[l] || prev_pyr->h[l] != next_pyr->h[l]) return OT_E_SHAPE;
    const int W0 = prev_pyr->w[0], H0 = prev_pyr->h[0];
    if (W0 > 16384 || H0 > 16384) return OT_E_INVAL;
    *T = TvLayout::make(prev_pyr->w, prev_pyr->h, L);
    // the documented size, and what this pyramid's levels take
    if (ws_bytes < TvLayout::bound(W0, H0) || ws_bytes < T->bytes || ((uintptr_t)ws & 255) ||
        ((uintptr_t)flow & 7))
        return OT_E_WORKSPACE;
    return OT_OK;
}

// The structure-texture passes and gradients of every level (coarse to fine)
// on stream a, the flow on stream s; with a != s, level l's flow waits for an
// event recorded on a after level l's planes, and a starts after an event of
// s (everything the caller enqueued before).  The last wait joins a into s.
ot_err tvl1_run(const ot_pyr* prev_pyr, const ot_pyr* next_pyr, const ot_tvl1_params* prm,
                void* ws, size_t ws_bytes, float* flow, hipStream_t s, hipStream_t a) {
    TvLayout T;
    const ot_err e0 = flow_args(prev_pyr, next_pyr, prm, ws, ws_bytes, flow, &T);
    if (e0 != OT_OK) return e0;
    const int L = prm->levels;
    const bool two = a != s;
    hipEvent_t* ev = nullptr;
    std::unique_lock<std::mutex> lock(tv_ev_mu, std::defer_lock);
    if (two) {
        hipDevice_t ds = -1, da = -1;
        if (hipStreamGetDevice(s, &ds) != hipSuccess || hipStreamGetDevice(a, &da) != hipSuccess ||
            ds != da)
            return OT_E_INVAL;
        lock.lock();
        if (tv_events(ds, &ev) != hipSuccess) return OT_E_LAUNCH;
    }
    uint8_t* base = static_cast<uint8_t*>(ws);
    float2* const R[2][2] = {{reinterpret_cast<float2*>(base + T.r0), reinterpret_cast<float2*>(base + T.r1)},
                             {reinterpret_cast<float2*>(base + T.r2), reinterpret_cast<float2*>(base + T.r3)}};
    if (two) {
        if (hipEventRecord(ev[OT_MAX_LEVELS], s) != hipSuccess ||
            hipStreamWaitEvent(a, ev[OT_MAX_LEVELS], 0) != hipSuccess)
            return OT_E_LAUNCH;
    }
    // ---- structure-texture split and texture gradient of every level, on a
    const ot_pyr* const pyrs[2] = {prev_pyr, next_pyr};
    for (int l = L - 1; l >= 0; --l) {
        float* const tex[2] = {reinterpret_cast<float*>(base + T.t0[l]),
                               reinterpret_cast<float*>(base + T.t1[l])};
        if (split_level(pyrs, 2, l, prm, R, tex, reinterpret_cast<float2*>(base + T.g[l]), a) !=
            hipSuccess)
            return OT_E_LAUNCH;
        if (two && hipEventRecord(ev[l], a) != hipSuccess) return OT_E_LAUNCH;
    }
    // ---- flow, coarse to fine, on s
    return flow_levels(prev_pyr, prm, base, T,
                       [&](int l, const float*& I0, const float*& I1, const float2*& G1) {
                           I0 = reinterpret_cast<const float*>(base + T.t0[l]);
                           I1 = reinterpret_cast<const float*>(base + T.t1[l]);
                           G1 = reinterpret_cast<const float2*>(base + T.g[l]);
                       },
                       flow, s, two ? ev : nullptr);
}

}  // namespace
}  // namespace ot

extern "C" {

ot_err ot_tvl1_flow(const ot_pyr* prev_pyr, const ot_pyr* next_pyr, const ot_tvl1_params* prm,
                    void* ws, size_t ws_bytes, float* flow, void* stream) {
    const hipStream_t s = static_cast<hipStream_t>(stream);
    return tvl1_run(prev_pyr, next_pyr, prm, ws, ws_bytes, flow, s, s);
}

ot_err ot_tvl1_flow_async(const ot_pyr* prev_pyr, const ot_pyr* next_pyr,
                          const ot_tvl1_params* prm, void* ws, size_t ws_bytes, float* flow,
                          void* stream, void* aux_stream) {
    return tvl1_run(prev_pyr, next_pyr, prm, ws, ws_bytes, flow, static_cast<hipStream_t>(stream),
                    static_cast<hipStream_t>(aux_stream));
}

size_t ot_tvl1_texture_bytes(int32_t W, int32_t H) {
    if (W < 1 || H < 1 || W > 16384 || H > 16384) return 0;
    return TexLayout::bound(W, H);
}

ot_err ot_tvl1_texture(const ot_pyr* pyr, const ot_tvl1_params* prm, void* tex, size_t tex_bytes,
                       void* stream) {
    if (!pyr_ok(pyr) || !params_ok(prm) || !tex) return OT_E_INVAL;
    const int L = prm->levels;
    if (L > pyr->levels) return OT_E_INVAL;
    const int W0 = pyr->w[0], H0 = pyr->h[0];
    if (W0 > 16384 || H0 > 16384) return OT_E_INVAL;
    const TexLayout X = TexLayout::make(pyr->w, pyr->h, L);
    if (tex_bytes < TexLayout::bound(W0, H0) || tex_bytes < X.bytes || ((uintptr_t)tex & 255))
        return OT_E_WORKSPACE;
    uint8_t* base = static_cast<uint8_t*>(tex);
    float2* const R[1][2] = {{reinterpret_cast<float2*>(base + X.r0), reinterpret_cast<float2*>(base + X.r1)}};
    const ot_pyr* const pyrs[1] = {pyr};
    const hipStream_t s = static_cast<hipStream_t>(stream);
    for (int l = L - 1; l >= 0; --l) {
        float* const t[1] = {reinterpret_cast<float*>(base + X.t[l])};
        if (split_level(pyrs, 1, l, prm, R, t, reinterpret_cast<float2*>(base + X.g[l]), s) !=
            hipSuccess)
            return OT_E_LAUNCH;
    }
    return OT_OK;
}

ot_err ot_tvl1_flow_tex(const ot_pyr* prev_pyr, const ot_pyr* next_pyr, const void* prev_tex,
                        const void* next_tex, const ot_tvl1_params* prm, void* ws,
                        size_t ws_bytes, float* flow, void* stream) {
    TvLayout T;
    const ot_err e0 = flow_args(prev_pyr, next_pyr, prm, ws, ws_bytes, flow, &T);
    if (e0 != OT_OK) return e0;
    if (!prev_tex || !next_tex) return OT_E_INVAL;
    if (((uintptr_t)prev_tex | (uintptr_t)next_tex) & 255) return OT_E_WORKSPACE;
    const TexLayout X = TexLayout::make(prev_pyr->w, prev_pyr->h, prm->levels);
    const uint8_t* pb = static_cast<const uint8_t*>(prev_tex);
    const uint8_t* nb = static_cast<const uint8_t*>(next_tex);
    return flow_levels(prev_pyr, prm, static_cast<uint8_t*>(ws), T,
                       [&](int l, const float*& I0, const float*& I1, const float2*& G1) {
                           I0 = reinterpret_cast<const float*>(pb + X.t[l]);
                           I1 = reinterpret_cast<const float*>(nb + X.t[l]);
                           G1 = reinterpret_cast<const float2*>(nb + X.g[l]);
                       },
                       flow, static_cast<hipStream_t>(stream), nullptr);
}

ot_err ot_box_mean_flow(const float* flow, int32_t W, int32_t H, const float* boxes, int32_t m,
                        float* out_boxes, int32_t* out_count, void* stream) {
    if (m < 0 || W < 1 || H < 1) return OT_E_INVAL;
    if (m == 0) return OT_OK;
    if (!flow || !boxes || !out_boxes || !out_count || ((uintptr_t)flow & 7)) return OT_E_INVAL;
    hipLaunchKernelGGL(k_box_mean, dim3(m), dim3(BM_THREADS), 0, static_cast<hipStream_t>(stream),
                       reinterpret_cast<const float2*>(flow), W, H, boxes, out_boxes, out_count);
    return hipGetLastError() == hipSuccess ? OT_OK : OT_E_LAUNCH;
}

}  // extern "C"
