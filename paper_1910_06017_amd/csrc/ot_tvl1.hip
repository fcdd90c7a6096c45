// ot_tvl1.hip -- dense TV-L1 optical flow for gfx950 (Sec. IV): Huber total
// variation, projected dual steps, structure-texture inputs, coarse-to-fine
// warps (Zach, Pock & Bischof 2007; Werlberger et al. 2009; Wedel et al.
// 2009); and the per-box mean of the dense field (Sec. V-A prediction).
//
// Every pass is a 2-D stencil over float planes, one thread per pixel in
// 64 x 4 workgroups (a wave covers 64 consecutive pixels of a row, so every
// plane read is a coalesced row segment; the neighbour reads of a stencil
// hit the same lines in L1/L2).  Iterations ping-pong between two buffers so
// no workgroup reads what another one writes in the same launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

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
// One dual step of the structure (ROF) problem on f = img / 255:
// w = div p - f / theta at (x, y), (x+1, y), (x, y+1); p <- (p + tau grad w)
// / (1 + tau |grad w|).  p_in unused (taken as 0) when `first`.
__global__ __launch_bounds__(TV_BX* TV_BY) void k_rof_step(const uint8_t* __restrict__ img, int pitch,
                                                           int W, int H, const float2* __restrict__ p_in,
                                                           float2* __restrict__ p_out, float inv_theta,
                                                           float tau, int first) {
    const int x = blockIdx.x * TV_BX + threadIdx.x, y = blockIdx.y * TV_BY + threadIdx.y;
    if (x >= W || y >= H) return;
    auto f = [&](int xx, int yy) { return (float)img[(size_t)yy * pitch + xx] * (1.0f / 255.0f); };
    auto pxf = [&](int xx, int yy) { return first ? 0.0f : p_in[(size_t)yy * W + xx].x; };
    auto pyf = [&](int xx, int yy) { return first ? 0.0f : p_in[(size_t)yy * W + xx].y; };
    auto w = [&](int xx, int yy) { return div_at(xx, yy, W, H, pxf, pyf) - f(xx, yy) * inv_theta; };
    const float wc = w(x, y);
    const float gx = x + 1 < W ? w(x + 1, y) - wc : 0.0f;
    const float gy = y + 1 < H ? w(x, y + 1) - wc : 0.0f;
    const float nrm = 1.0f + tau * sqrtf(gx * gx + gy * gy);
    const float2 p = first ? make_float2(0.0f, 0.0f) : p_in[(size_t)y * W + x];
    p_out[(size_t)y * W + x] = make_float2((p.x + tau * gx) / nrm, (p.y + tau * gy) / nrm);
}

// texture = f - alpha * (f - theta div p)
__global__ __launch_bounds__(TV_BX* TV_BY) void k_texture(const uint8_t* __restrict__ img, int pitch,
                                                          int W, int H, const float2* __restrict__ p,
                                                          float* __restrict__ tex, float theta,
                                                          float alpha) {
    const int x = blockIdx.x * TV_BX + threadIdx.x, y = blockIdx.y * TV_BY + threadIdx.y;
    if (x >= W || y >= H) return;
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

// Linearisation of the data term at the current flow u0:
// data = (gx, gy, rho0, gx^2 + gy^2) with rho(u) = rho0 + g . u.
__global__ __launch_bounds__(TV_BX* TV_BY) void k_warp(const float* __restrict__ I0,
                                                       const float* __restrict__ I1,
                                                       const float2* __restrict__ G1, int W, int H,
                                                       const float2* __restrict__ u,
                                                       float4* __restrict__ data) {
    const int x = blockIdx.x * TV_BX + threadIdx.x, y = blockIdx.y * TV_BY + threadIdx.y;
    if (x >= W || y >= H) return;
    const size_t i = (size_t)y * W + x;
    const float2 u0 = u[i];
    const float wx = (float)x + u0.x, wy = (float)y + u0.y;
    const float I1w = bilin<float>(wx, wy, W, H, [&](int a, int b) { return I1[(size_t)b * W + a]; });
    const float gx = bilin<float>(wx, wy, W, H, [&](int a, int b) { return G1[(size_t)b * W + a].x; });
    const float gy = bilin<float>(wx, wy, W, H, [&](int a, int b) { return G1[(size_t)b * W + a].y; });
    const float rho0 = I1w - gx * u0.x - gy * u0.y - I0[i];
    data[i] = make_float4(gx, gy, rho0, gx * gx + gy * gy);
}

// Pointwise L1 data step: v minimising |v - u|^2 / (2 theta) + lam |rho(v)|.
__device__ __forceinline__ float2 data_step(float2 u, float4 d, float lt) {
    const float rho = d.z + d.x * u.x + d.y * u.y;
    const float t = lt * d.w;
    float s;
    if (rho < -t) s = lt;
    else if (rho > t) s = -lt;
    else if (d.w > 0.0f) s = -rho / d.w;
    else s = 0.0f;
    return make_float2(u.x + s * d.x, u.y + s * d.y);
}

// One TV-L1 iteration: v = data step of u_in, u = v + theta div p_in (both
// flow components), p = projection onto the unit ball of (p_in + (tau/theta)
// grad u) / (1 + tau eps / theta).  The thread also forms u at its right and
// lower neighbours (the gradient's other taps) from the same inputs.  p is
// (p1x, p1y, p2x, p2y) per pixel; p_in taken as 0 when `first`.
__global__ __launch_bounds__(TV_BX* TV_BY) void k_tvl1_iter(const float4* __restrict__ data,
                                                            const float2* __restrict__ u_in,
                                                            const float4* __restrict__ p_in,
                                                            float2* __restrict__ u_out,
                                                            float4* __restrict__ p_out, int W, int H,
                                                            float lt, float theta, float k,
                                                            float inv_shrink, int first) {
    const int x = blockIdx.x * TV_BX + threadIdx.x, y = blockIdx.y * TV_BY + threadIdx.y;
    if (x >= W || y >= H) return;
    auto P = [&](int xx, int yy) {
        return first ? make_float4(0.0f, 0.0f, 0.0f, 0.0f) : p_in[(size_t)yy * W + xx];
    };
    auto unew = [&](int xx, int yy) {
        const size_t j = (size_t)yy * W + xx;
        const float2 v = data_step(u_in[j], data[j], lt);
        const float d1 = div_at(xx, yy, W, H, [&](int a, int b) { return P(a, b).x; },
                                [&](int a, int b) { return P(a, b).y; });
        const float d2 = div_at(xx, yy, W, H, [&](int a, int b) { return P(a, b).z; },
                                [&](int a, int b) { return P(a, b).w; });
        return make_float2(v.x + theta * d1, v.y + theta * d2);
    };
    const float2 uc = unew(x, y);
    const float2 ur = x + 1 < W ? unew(x + 1, y) : uc;
    const float2 ud = y + 1 < H ? unew(x, y + 1) : uc;
    const size_t i = (size_t)y * W + x;
    const float4 p = P(x, y);
    float q1x = (p.x + k * fwd_x(uc.x, ur.x, x, W)) * inv_shrink;
    float q1y = (p.y + k * fwd_y(uc.x, ud.x, y, H)) * inv_shrink;
    float q2x = (p.z + k * fwd_x(uc.y, ur.y, x, W)) * inv_shrink;
    float q2y = (p.w + k * fwd_y(uc.y, ud.y, y, H)) * inv_shrink;
    const float n1 = fmaxf(1.0f, sqrtf(q1x * q1x + q1y * q1y));
    const float n2 = fmaxf(1.0f, sqrtf(q2x * q2x + q2y * q2y));
    u_out[i] = uc;
    p_out[i] = make_float4(q1x / n1, q1y / n1, q2x / n2, q2y / n2);
}

// Flow of a finer level (W x H) from the coarser one (Wc x Hc): 2 u(x / 2).
__global__ __launch_bounds__(TV_BX* TV_BY) void k_upsample(const float2* __restrict__ uc, int Wc, int Hc,
                                                           float2* __restrict__ uf, int W, int H) {
    const int x = blockIdx.x * TV_BX + threadIdx.x, y = blockIdx.y * TV_BY + threadIdx.y;
    if (x >= W || y >= H) return;
    const float sx = 0.5f * (float)x, sy = 0.5f * (float)y;
    const float a = bilin<float>(sx, sy, Wc, Hc, [&](int i, int j) { return uc[(size_t)j * Wc + i].x; });
    const float b = bilin<float>(sx, sy, Wc, Hc, [&](int i, int j) { return uc[(size_t)j * Wc + i].y; });
    uf[(size_t)y * W + x] = make_float2(2.0f * a, 2.0f * b);
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
inline dim3 grid2(int W, int H) { return dim3((W + TV_BX - 1) / TV_BX, (H + TV_BY - 1) / TV_BY); }

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace: textures T0, T1 (float), structure duals (2 x float2), image
// gradient (float2), data (float4), flow (2 x float2), dual (2 x float4),
// each sized for level 0 and reused by the coarser levels.
struct TvLayout {
    size_t t0, t1, r0, r1, g, d, u0, u1, p0, p1, bytes;
    static TvLayout make(int W, int H) {
        const size_t n = (size_t)W * H;
        TvLayout L;
        size_t o = 0;
        auto take = [&](size_t b) {
            const size_t at = o;
            o += al256(b);
            return at;
        };
        L.t0 = take(n * 4);
        L.t1 = take(n * 4);
        L.r0 = take(n * 8);
        L.r1 = take(n * 8);
        L.g = take(n * 8);
        L.d = take(n * 16);
        L.u0 = take(n * 8);
        L.u1 = take(n * 8);
        L.p0 = take(n * 16);
        L.p1 = take(n * 16);
        L.bytes = o;
        return L;
    }
};

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
    return TvLayout::make(W, H).bytes;
}

ot_err ot_tvl1_flow(const ot_pyr* prev_pyr, const ot_pyr* next_pyr, const ot_tvl1_params* prm,
                    void* ws, size_t ws_bytes, float* flow, void* stream) {
    if (!pyr_ok(prev_pyr) || !pyr_ok(next_pyr) || !params_ok(prm) || !flow || !ws) return OT_E_INVAL;
    const int L = prm->levels;
    if (L > prev_pyr->levels || L > next_pyr->levels) return OT_E_INVAL;
    for (int l = 0; l < L; ++l)
        if (prev_pyr->w[l] != next_pyr->w[l] || prev_pyr->h[l] != next_pyr->h[l]) return OT_E_SHAPE;
    const int W0 = prev_pyr->w[0], H0 = prev_pyr->h[0];
    if (W0 > 16384 || H0 > 16384) return OT_E_INVAL;
    const TvLayout T = TvLayout::make(W0, H0);
    if (ws_bytes < T.bytes || ((uintptr_t)ws & 255) || ((uintptr_t)flow & 7)) return OT_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint8_t* base = static_cast<uint8_t*>(ws);
    float* T0 = reinterpret_cast<float*>(base + T.t0);
    float* T1 = reinterpret_cast<float*>(base + T.t1);
    float2* R[2] = {reinterpret_cast<float2*>(base + T.r0), reinterpret_cast<float2*>(base + T.r1)};
    float2* G = reinterpret_cast<float2*>(base + T.g);
    float4* D = reinterpret_cast<float4*>(base + T.d);
    float2* U[2] = {reinterpret_cast<float2*>(base + T.u0), reinterpret_cast<float2*>(base + T.u1)};
    float4* Pd[2] = {reinterpret_cast<float4*>(base + T.p0), reinterpret_cast<float4*>(base + T.p1)};
    const float lt = prm->lam * prm->theta, k = prm->tau / prm->theta;
    const float inv_shrink = 1.0f / (1.0f + prm->tau * prm->eps / prm->theta);
    int cu = 0;  // index of the current flow buffer
    for (int l = L - 1; l >= 0; --l) {
        const int W = prev_pyr->w[l], H = prev_pyr->h[l];
        const dim3 gr = grid2(W, H), bl(TV_BX, TV_BY);
        // textures of both frames
        for (int f = 0; f < 2; ++f) {
            const ot_pyr* py = f == 0 ? prev_pyr : next_pyr;
            const uint8_t* img = py->level[l];
            const int pitch = py->pitch[l];
            int cr = 0;
            for (int it = 0; it < prm->iters_s; ++it) {
                hipLaunchKernelGGL(k_rof_step, gr, bl, 0, s, img, pitch, W, H, R[cr], R[cr ^ 1],
                                   1.0f / prm->theta_s, prm->tau_s, it == 0 ? 1 : 0);
                cr ^= 1;
            }
            if (prm->iters_s == 0) {
                // no structure iterations: p = 0
                hipLaunchKernelGGL(k_zero2, dim3((unsigned)(((size_t)W * H + 255) / 256)), dim3(256), 0,
                                   s, R[cr], (size_t)W * H);
            }
            hipLaunchKernelGGL(k_texture, gr, bl, 0, s, img, pitch, W, H, R[cr], f == 0 ? T0 : T1,
                               prm->theta_s, prm->alpha);
        }
        hipLaunchKernelGGL(k_central_grad, gr, bl, 0, s, T1, W, H, G);
        // initial flow: zero at the coarsest level, else the coarser flow doubled
        if (l == L - 1) {
            hipLaunchKernelGGL(k_zero2, dim3((unsigned)(((size_t)W * H + 255) / 256)), dim3(256), 0, s,
                               U[cu], (size_t)W * H);
        } else {
            hipLaunchKernelGGL(k_upsample, gr, bl, 0, s, U[cu], prev_pyr->w[l + 1], prev_pyr->h[l + 1],
                               U[cu ^ 1], W, H);
            cu ^= 1;
        }
        int cp = 0;
        bool first = true;
        for (int wv = 0; wv < prm->warps; ++wv) {
            hipLaunchKernelGGL(k_warp, gr, bl, 0, s, T0, T1, G, W, H, U[cu], D);
            for (int it = 0; it < prm->iters; ++it) {
                hipLaunchKernelGGL(k_tvl1_iter, gr, bl, 0, s, D, U[cu], Pd[cp], U[cu ^ 1], Pd[cp ^ 1], W,
                                   H, lt, prm->theta, k, inv_shrink, first ? 1 : 0);
                cu ^= 1;
                cp ^= 1;
                first = false;
            }
        }
    }
    if (hipGetLastError() != hipSuccess) return OT_E_LAUNCH;
    if (hipMemcpyAsync(flow, U[cu], (size_t)W0 * H0 * sizeof(float2), hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
        return OT_E_LAUNCH;
    return OT_OK;
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
