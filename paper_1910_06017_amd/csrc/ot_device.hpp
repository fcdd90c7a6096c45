// ot_device.hpp -- gfx950 device code of the pyramidal Lucas-Kanade tracker:
// wave64 DPP reductions, the pyramid reduce tile, the per-point tracker and
// the per-box median.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ot_common.hpp"

// Clamped-byte staging near level edges keeps this many loads per lane in
// flight (registers vs latency).
#ifndef OT_STAGE_BATCH
#define OT_STAGE_BATCH 4
#endif

namespace ot {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

__device__ __forceinline__ float uniform_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// One DPP move of a float across lanes (GFX9 DPP control codes); lanes whose
// source is outside the row, or rows masked off, read 0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xF, true));
}

// Sum over the 64 lanes of a wave; every lane gets the total.  Within a row
// of 16 lanes: two quad permutes, half-row mirror and row mirror leave the row
// total in every lane; row_bcast:15 and row_bcast:31 then fold the four row
// totals into lane 63, which is broadcast.  All 64 lanes must be active.
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_f<0xB1>(v);       // quad_perm [1,0,3,2]
    v += dpp_f<0x4E>(v);       // quad_perm [2,3,0,1]
    v += dpp_f<0x141>(v);      // row_half_mirror
    v += dpp_f<0x140>(v);      // row_mirror
    v += dpp_f<0x142, 0xA>(v); // row_bcast:15 -> rows 1, 3
    v += dpp_f<0x143, 0xC>(v); // row_bcast:31 -> rows 2, 3
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Workgroup b runs on XCD b % 8; hand each XCD one contiguous range of work
// items so neighbouring points share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int G) {
    const int X = 8;
    const int q = G / X, rem = G % X;
    const int xcd = b % X, k = b / X;
    return (xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q) + k;
}

// ---------------------------------------------------------------------------
// Gaussian pyramid reduce of one PYR_TW x PYR_TH output tile (binomial
// (1,4,6,4,1) in both directions, clamp-to-edge, exact integer sum rounded
// half up).  256 threads.
// ---------------------------------------------------------------------------
struct PyrSmem {
    // input rows start at the 4-byte aligned column below 2*ox0-2; `in_off`
    // is where that column sits in the row
    uint8_t in[2 * PYR_TH + 3][2 * PYR_TW + 8];
    int32_t hs[2 * PYR_TH + 3][PYR_TW];
};

__device__ __forceinline__ void pyr_tile(const uint8_t* __restrict__ src, int sw, int sh, int sp,
                                         uint8_t* __restrict__ dst, int dw, int dh, int dp,
                                         int tx, int ty, PyrSmem& sm) {
    const int tid = threadIdx.x;
    const int ox0 = tx * PYR_TW, oy0 = ty * PYR_TH;
    const int ix0 = 2 * ox0 - 2, iy0 = 2 * oy0 - 2;
    constexpr int IR = 2 * PYR_TH + 3, IC = 2 * PYR_TW + 3;
    const int a0 = ix0 & ~3, off = ix0 - a0;
    constexpr int ND = (IC + 3 + 3) / 4;  // dwords per row covering [a0, ix0 + IC)
    const bool fast = a0 >= 0 && iy0 >= 0 && a0 + 4 * ND <= sw && iy0 + IR <= sh &&
                      ((reinterpret_cast<uintptr_t>(src) | (uintptr_t)sp) & 3) == 0;
    if (fast) {
        // IR x ND aligned dwords, all loads in flight before the LDS writes
        constexpr int NT = IR * ND, PER = (NT + PYR_THREADS - 1) / PYR_THREADS;
        uint32_t v[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + k * PYR_THREADS;
            const int r = e / ND, c = e - r * ND;
            v[k] = e < NT ? *reinterpret_cast<const uint32_t*>(src + (size_t)(iy0 + r) * sp + a0 + 4 * c)
                          : 0u;
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + k * PYR_THREADS;
            const int r = e / ND, c = e - r * ND;
            if (e < NT) *reinterpret_cast<uint32_t*>(&sm.in[r][4 * c]) = v[k];
        }
    } else {
        constexpr int NT = IR * IC, PER = (NT + PYR_THREADS - 1) / PYR_THREADS;
        for (int k0 = 0; k0 < PER; k0 += 8) {
            uint32_t v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int e = tid + (k0 + k) * PYR_THREADS;
                const int r = e / IC, c = e - r * IC;
                const int y = clampi(iy0 + r, 0, sh - 1), x = clampi(ix0 + c, 0, sw - 1);
                v[k] = (k0 + k < PER && e < NT) ? src[(size_t)y * sp + x] : 0u;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int e = tid + (k0 + k) * PYR_THREADS;
                const int r = e / IC, c = e - r * IC;
                if (k0 + k < PER && e < NT) sm.in[r][off + c] = (uint8_t)v[k];
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < IR * PYR_TW; e += PYR_THREADS) {
        const int r = e / PYR_TW, c = e - r * PYR_TW;
        const uint8_t* p = &sm.in[r][off + 2 * c];
        sm.hs[r][c] = (int)p[0] + 4 * (int)p[1] + 6 * (int)p[2] + 4 * (int)p[3] + (int)p[4];
    }
    __syncthreads();
    // one thread per 4 horizontally adjacent outputs
    {
        const int r = tid / (PYR_TW / 4), c = (tid - r * (PYR_TW / 4)) * 4;
        const int y = oy0 + r, x = ox0 + c;
        if (y < dh) {
            uint32_t packed = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int s = sm.hs[2 * r][c + k] + 4 * sm.hs[2 * r + 1][c + k] +
                              6 * sm.hs[2 * r + 2][c + k] + 4 * sm.hs[2 * r + 3][c + k] +
                              sm.hs[2 * r + 4][c + k];
                packed |= (uint32_t)((s + 128) >> 8) << (8 * k);
            }
            uint8_t* o = dst + (size_t)y * dp + x;
            if (x + 4 <= dw && ((reinterpret_cast<uintptr_t>(o)) & 3) == 0) {
                *reinterpret_cast<uint32_t*>(o) = packed;
            } else {
                for (int k = 0; k < 4; ++k)
                    if (x + k < dw) o[k] = (uint8_t)(packed >> (8 * k));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Paired and quadruple wave sums using the gfx950 lane-swap instructions:
// v_permlane32_swap folds the upper half-wave of one value onto the lower
// half of another, v_permlane16_swap does the same for 16-lane rows, so two
// (or four) sums share one DPP row reduction.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned fbits(float v) { return __builtin_bit_cast(unsigned, v); }
__device__ __forceinline__ float ubits(unsigned v) { return __builtin_bit_cast(float, v); }

__device__ __forceinline__ float row_sum16(float t) {
    t += dpp_f<0xB1>(t);   // quad_perm [1,0,3,2]
    t += dpp_f<0x4E>(t);   // quad_perm [2,3,0,1]
    t += dpp_f<0x141>(t);  // row_half_mirror
    t += dpp_f<0x140>(t);  // row_mirror
    return t;
}

// (sum of a, sum of b) over the 64 lanes, wave-uniform.
__device__ __forceinline__ void wave_sum2(float a, float b, float& sa, float& sb) {
    const auto r = __builtin_amdgcn_permlane32_swap(fbits(a), fbits(b), false, false);
    const float s = ubits(r[0]) + ubits(r[1]);  // lanes 0-31: a, lanes 32-63: b
    const auto q = __builtin_amdgcn_permlane16_swap(fbits(s), fbits(s), false, false);
    const float t = row_sum16(ubits(q[0]) + ubits(q[1]));  // rows 0,1: a; rows 2,3: b
    sa = ubits(__builtin_amdgcn_readlane(fbits(t), 0));
    sb = ubits(__builtin_amdgcn_readlane(fbits(t), 32));
}

// Sums of a, b, c, d over the 64 lanes, wave-uniform.
__device__ __forceinline__ void wave_sum4(float a, float b, float c, float d, float& sa, float& sb,
                                          float& sc, float& sd) {
    const auto r1 = __builtin_amdgcn_permlane32_swap(fbits(a), fbits(b), false, false);
    const auto r2 = __builtin_amdgcn_permlane32_swap(fbits(c), fbits(d), false, false);
    const float s1 = ubits(r1[0]) + ubits(r1[1]);  // a | b
    const float s2 = ubits(r2[0]) + ubits(r2[1]);  // c | d
    const auto q = __builtin_amdgcn_permlane16_swap(fbits(s1), fbits(s2), false, false);
    const float t = row_sum16(ubits(q[0]) + ubits(q[1]));  // rows: a, c, b, d
    sa = ubits(__builtin_amdgcn_readlane(fbits(t), 0));
    sc = ubits(__builtin_amdgcn_readlane(fbits(t), 16));
    sb = ubits(__builtin_amdgcn_readlane(fbits(t), 32));
    sd = ubits(__builtin_amdgcn_readlane(fbits(t), 48));
}

// ---------------------------------------------------------------------------
// Lucas-Kanade for one point, one wave64 per point.
//
// Lane mapping: the win x win window is split into win columns x nseg row
// segments; lane = seg * win + col owns the R consecutive window rows
// seg*R .. seg*R+R-1 of column col (lanes past win*nseg own nothing).  Each
// lane keeps its template, x- and y-gradient samples in registers, so a
// Lucas-Kanade iteration reads only the target image.
//
// LDS (per wave): during a level's set-up, the raw template patch (uint8,
// rows starting at a 4-byte aligned column) and the Scharr gradients at the
// bilinear tap grid; during iterations, the target region with a `margin`
// border, stored as (J[x], J[x+1]-J[x]) pairs so each bilinear row blend is
// one FMA.  Regions are restaged only when the estimate leaves the margin.
// Global reads are issued in batches before their LDS writes, as aligned
// dwords when the region lies inside the level and as clamped bytes near
// its edges.
// ---------------------------------------------------------------------------
struct LkGeom {
    int win, r, nseg, RR, TW, PR, PW, M, SC, SR;
    __device__ LkGeom(int win_, int R, int margin) {
        win = win_;
        r = win >> 1;
        nseg = min(win, max(1, 64 / win));
        RR = nseg * R + 1;               // tap rows held (>= win + 1)
        TW = win + 1;                    // tap columns
        PR = RR + 2;                     // template patch rows
        PW = 4 * (((TW + 4) >> 2) + 1);  // template patch row bytes
        M = margin;
        SC = TW + 2 * M;
        SR = RR + 2 * M;
    }
};

// Target region: entry (rr, cc) = (J[y][x], J[y][x+1] - J[y][x]) with
// y = clamp(sy0 + rr), x = clamp(sx0 + cc), for rr < SR, cc < SC.
__device__ __forceinline__ void stage_target(const uint8_t* __restrict__ Jl, int w, int h, int jp,
                                             int sx0, int sy0, int SR, int SC,
                                             float2* __restrict__ jr, int lane) {
    const int a0 = sx0 & ~3;
    const int nd = ((sx0 + SC - a0) >> 2) + 1;  // dwords covering columns a0 .. sx0+SC
    const bool fast = a0 >= 0 && sy0 >= 0 && a0 + 4 * nd <= w && sy0 + SR <= h &&
                      ((reinterpret_cast<uintptr_t>(Jl) | (uintptr_t)jp) & 3) == 0;
    if (fast) {
        const int rps = 64 / nd;
        const int lr = lane / nd, kk = lane - lr * nd;
        const bool lane_ok = lr < rps;
        const int steps = (SR + rps - 1) / rps;
        const int c0 = a0 + 4 * kk - sx0;
        const uint8_t* __restrict__ base = Jl + (size_t)sy0 * jp + a0 + 4 * kk;
        for (int s0 = 0; s0 < steps; s0 += 8) {
            uint32_t v[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int rr = lr + (s0 + s) * rps;
                v[s] = (lane_ok && rr < SR)
                           ? *reinterpret_cast<const uint32_t*>(base + (size_t)rr * jp)
                           : 0u;
            }
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const uint32_t nx = __shfl_down(v[s], 1, 64);
                const int rr = lr + (s0 + s) * rps;
                if (lane_ok && rr < SR) {
                    const float b0 = (float)(v[s] & 255u), b1 = (float)((v[s] >> 8) & 255u);
                    const float b2 = (float)((v[s] >> 16) & 255u), b3 = (float)(v[s] >> 24);
                    const float b4 = (float)(nx & 255u);
                    float2* row = jr + rr * SC;
                    if (c0 >= 0 && c0 < SC) row[c0] = make_float2(b0, b1 - b0);
                    if (c0 + 1 >= 0 && c0 + 1 < SC) row[c0 + 1] = make_float2(b1, b2 - b1);
                    if (c0 + 2 >= 0 && c0 + 2 < SC) row[c0 + 2] = make_float2(b2, b3 - b2);
                    if (c0 + 3 >= 0 && c0 + 3 < SC) row[c0 + 3] = make_float2(b3, b4 - b3);
                }
            }
        }
    } else {
        const int dr = 64 / SC, dc = 64 - dr * SC;
        int r = lane / SC, c = lane - r * SC;
        const int nk = (SR * SC + 63) >> 6;
        for (int kb = 0; kb < nk; kb += OT_STAGE_BATCH) {
            int idx[OT_STAGE_BATCH];
            uint32_t p0[OT_STAGE_BATCH], p1[OT_STAGE_BATCH];
#pragma unroll
            for (int s = 0; s < OT_STAGE_BATCH; ++s) {
                idx[s] = -1;
                p0[s] = p1[s] = 0;
                if (kb + s < nk && r < SR) {
                    const uint8_t* row = Jl + (size_t)clampi(sy0 + r, 0, h - 1) * jp;
                    p0[s] = row[clampi(sx0 + c, 0, w - 1)];
                    p1[s] = row[clampi(sx0 + c + 1, 0, w - 1)];
                    idx[s] = r * SC + c;
                }
                c += dc;
                r += dr;
                if (c >= SC) {
                    c -= SC;
                    ++r;
                }
            }
#pragma unroll
            for (int s = 0; s < OT_STAGE_BATCH; ++s)
                if (idx[s] >= 0) {
                    const float f0 = (float)p0[s], f1 = (float)p1[s];
                    jr[idx[s]] = make_float2(f0, f1 - f0);
                }
        }
    }
}

// Template patch: rows y0-1 .. y0+PR-2, columns x0-1 .. x0+TW of the level
// (clamped), stored with its row starting at column a0p = (x0-1) & ~3, so
// patch[pr * PW + (x - a0p)] holds I[clamp(y0-1+pr)][clamp(x)].
__device__ __forceinline__ void stage_patch(const uint8_t* __restrict__ Il, int w, int h, int ip,
                                            int x0, int y0, const LkGeom& g,
                                            uint8_t* __restrict__ patch, int lane) {
    const int xs = x0 - 1, ys = y0 - 1;
    const int a0 = xs & ~3;
    const int nd = ((x0 + g.TW - a0) >> 2) + 1;  // dwords covering a0 .. x0+TW
    const bool fast = a0 >= 0 && ys >= 0 && a0 + 4 * nd <= w && ys + g.PR <= h &&
                      ((reinterpret_cast<uintptr_t>(Il) | (uintptr_t)ip) & 3) == 0;
    if (fast) {
        const int rps = 64 / nd;
        const int lr = lane / nd, kk = lane - lr * nd;
        const bool lane_ok = lr < rps;
        const int steps = (g.PR + rps - 1) / rps;
        const uint8_t* __restrict__ base = Il + (size_t)ys * ip + a0 + 4 * kk;
        for (int s0 = 0; s0 < steps; s0 += 8) {
            uint32_t v[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int rr = lr + (s0 + s) * rps;
                v[s] = (lane_ok && rr < g.PR)
                           ? *reinterpret_cast<const uint32_t*>(base + (size_t)rr * ip)
                           : 0u;
            }
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int rr = lr + (s0 + s) * rps;
                if (lane_ok && rr < g.PR)
                    *reinterpret_cast<uint32_t*>(patch + rr * g.PW + 4 * kk) = v[s];
            }
        }
    } else {
        const int cols = g.TW + 2, po = xs - a0;
        const int dr = 64 / cols, dc = 64 - dr * cols;
        int r = lane / cols, c = lane - r * cols;
        const int nk = (g.PR * cols + 63) >> 6;
        for (int kb = 0; kb < nk; kb += 8) {
            int idx[8];
            uint32_t p[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                idx[s] = -1;
                p[s] = 0;
                if (kb + s < nk && r < g.PR) {
                    p[s] = Il[(size_t)clampi(ys + r, 0, h - 1) * ip + clampi(xs + c, 0, w - 1)];
                    idx[s] = r * g.PW + po + c;
                }
                c += dc;
                r += dr;
                if (c >= cols) {
                    c -= cols;
                    ++r;
                }
            }
#pragma unroll
            for (int s = 0; s < 8; ++s)
                if (idx[s] >= 0) patch[idx[s]] = (uint8_t)p[s];
        }
    }
}

struct LkResult {
    float nx, ny, err;
    int status;
};

template <int R, class PyrRef>
__device__ __forceinline__ LkResult lk_point(const PyrRef& P, const PyrRef& Q, float ux, float uy,
                                             int L, int iters, float eps2, float min_eig,
                                             const LkGeom& g, unsigned char* __restrict__ smem,
                                             uint8_t* iters_out, float* lam_out) {
    const int lane = threadIdx.x & 63;
    const int used = g.win * g.nseg;
    const bool lvalid = lane < used;
    const int col = lvalid ? lane % g.win : 0;
    const int seg = lvalid ? lane / g.win : 0;
    const int row0 = seg * R;
    const int nrows = lvalid ? max(0, min(R, g.win - row0)) : 0;
    const float N = (float)(g.win * g.win);

    LkResult res;
    res.nx = ux;
    res.ny = uy;
    res.err = -1.0f;
    res.status = 0;
    const int W0 = P.w[0], H0 = P.h[0];
    if (!(ux >= 0.0f && uy >= 0.0f && ux <= (float)(W0 - 1) && uy <= (float)(H0 - 1))) {
        if (lane == 0)
            for (int l = 0; l < L; ++l) {
                if (iters_out) iters_out[l] = 0;
                if (lam_out) lam_out[l] = 0.0f;
            }
        return res;  // also catches NaN
    }

    float A[R], X[R], Y[R];
    float gx = 0.0f, gy = 0.0f;
    float nux = 0.0f, nuy = 0.0f;
    float2* jr = reinterpret_cast<float2*>(smem);
    uint8_t* patch = smem;
    float2* grad = reinterpret_cast<float2*>(smem + ((g.PR * g.PW + 15) & ~15));
    int sx0 = 0, sy0 = 0;  // origin of the staged target region (level coords)

    for (int l = L - 1; l >= 0; --l) {
        const uint8_t* __restrict__ Il = P.lvl[l];
        const uint8_t* __restrict__ Jl = Q.lvl[l];
        const int w = P.w[l], h = P.h[l], ip = P.pitch[l], jp = Q.pitch[l];
        const float sc = __builtin_ldexpf(1.0f, -l);
        const float cx = ux * sc, cy = uy * sc;
        const float flx = floorf(cx), fly = floorf(cy);
        const float ax = cx - flx, ay = cy - fly;
        const int x0 = (int)flx - g.r, y0 = (int)fly - g.r;  // top-left tap
        const int a0p = (x0 - 1) & ~3;

        // ---- template patch
        stage_patch(Il, w, h, ip, x0, y0, g, patch, lane);
        __syncthreads();
        // ---- Scharr gradients at the tap grid: the gradient image is defined on
        // the level's pixels and read at clamped indices, so a tap outside the
        // level takes the gradient of the nearest edge pixel.
        if (x0 >= 1 && x0 + g.TW <= w - 1 && y0 >= 1 && y0 + g.RR <= h - 1) {
            // interior: no clamping; each lane slides a 3x3 window down a
            // column of taps, so a tap costs three byte reads.  With
            // d = right - left and t = 3 left + 10 centre + 3 right per row:
            // Sx = 3 d(y-1) + 10 d(y) + 3 d(y+1),  Sy = t(y+1) - t(y-1).
            const int ncg = 64 / g.TW;
            const int GR = (g.RR + ncg - 1) / ncg;
            const int tx = lane % g.TW, rg = lane / g.TW;
            if (rg < ncg) {
                const int ty0 = rg * GR, ty1 = min(ty0 + GR, g.RR);
                const uint8_t* pp = patch + ty0 * g.PW + (x0 + tx - a0p);
                int vl = pp[-1], vc = pp[0], vr = pp[1];
                int d0 = vr - vl, t0 = 3 * (vl + vr) + 10 * vc;
                vl = pp[g.PW - 1], vc = pp[g.PW], vr = pp[g.PW + 1];
                int d1 = vr - vl, t1 = 3 * (vl + vr) + 10 * vc;
                for (int ty = ty0; ty < ty1; ++ty) {
                    const uint8_t* q = pp + (ty - ty0 + 2) * g.PW;
                    vl = q[-1], vc = q[0], vr = q[1];
                    const int d2 = vr - vl, t2 = 3 * (vl + vr) + 10 * vc;
                    const int sxv = 3 * (d0 + d2) + 10 * d1;
                    const int syv = t2 - t0;
                    grad[ty * g.TW + tx] = make_float2((float)sxv * (1.0f / 32.0f), (float)syv * (1.0f / 32.0f));
                    d0 = d1;
                    d1 = d2;
                    t0 = t1;
                    t1 = t2;
                }
            }
        } else {
            const int dr = 64 / g.TW, dc = 64 - dr * g.TW;
            int ty = lane / g.TW, tx = lane - ty * g.TW;
            const int ntap = g.RR * g.TW;
            for (int e = lane; e < ntap; e += 64) {
                const int qx = clampi(x0 + tx, 0, w - 1), qy = clampi(y0 + ty, 0, h - 1);
                const int xl = max(qx - 1, 0) - a0p, xc = qx - a0p, xr = min(qx + 1, w - 1) - a0p;
                const int yu = (max(qy - 1, 0) - (y0 - 1)) * g.PW;
                const int yc = (qy - (y0 - 1)) * g.PW;
                const int yd = (min(qy + 1, h - 1) - (y0 - 1)) * g.PW;
                const int pul = patch[yu + xl], puc = patch[yu + xc], pur = patch[yu + xr];
                const int pcl = patch[yc + xl], pcr = patch[yc + xr];
                const int pdl = patch[yd + xl], pdc = patch[yd + xc], pdr = patch[yd + xr];
                const int sxv = 3 * (pur - pul) + 10 * (pcr - pcl) + 3 * (pdr - pdl);
                const int syv = 3 * (pdl - pul) + 10 * (pdc - puc) + 3 * (pdr - pur);
                grad[e] = make_float2((float)sxv * (1.0f / 32.0f), (float)syv * (1.0f / 32.0f));
                tx += dc;
                ty += dr;
                if (tx >= g.TW) {
                    tx -= g.TW;
                    ++ty;
                }
            }
        }
        __syncthreads();
        // ---- bilinear template and gradients of this lane's strip
        {
            const int pcol = x0 + col - a0p;  // patch column of tap column `col`
            float pi = 0.0f, px = 0.0f, py = 0.0f;
#pragma unroll
            for (int k = 0; k <= R; ++k) {
                const int ty = row0 + k;
                const float i0 = (float)patch[(ty + 1) * g.PW + pcol];
                const float i1 = (float)patch[(ty + 1) * g.PW + pcol + 1];
                const float2 g0 = grad[ty * g.TW + col];
                const float2 g1 = grad[ty * g.TW + col + 1];
                const float ri = fmaf(ax, i1 - i0, i0);
                const float rx = fmaf(ax, g1.x - g0.x, g0.x);
                const float ry = fmaf(ax, g1.y - g0.y, g0.y);
                if (k > 0) {
                    const bool v = (k - 1) < nrows;
                    A[k - 1] = v ? fmaf(ay, ri - pi, pi) : 0.0f;
                    X[k - 1] = v ? fmaf(ay, rx - px, px) : 0.0f;
                    Y[k - 1] = v ? fmaf(ay, ry - py, py) : 0.0f;
                }
                pi = ri;
                px = rx;
                py = ry;
            }
        }
        float gxx = 0.0f, gxy = 0.0f, gyy = 0.0f;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            gxx = fmaf(X[k], X[k], gxx);
            gxy = fmaf(X[k], Y[k], gxy);
            gyy = fmaf(Y[k], Y[k], gyy);
        }
        {
            float unused;
            wave_sum4(gxx, gxy, gyy, 0.0f, gxx, gxy, gyy, unused);
        }
        const float hm = 0.5f * (gxx + gyy), hd = 0.5f * (gxx - gyy);
        const float lam = (hm - sqrtf(hd * hd + gxy * gxy)) / N;
        if (lane == 0 && lam_out) lam_out[l] = lam;
        if (!(lam >= min_eig)) {
            if (lane == 0)
                for (int k = l; k >= 0; --k) {
                    if (iters_out) iters_out[k] = 0;
                    if (lam_out && k < l) lam_out[k] = 0.0f;
                }
            const float s = __builtin_ldexpf(1.0f, l);
            res.nx = ux + gx * s;
            res.ny = uy + gy * s;
            return res;
        }
        const float idet = 1.0f / (gxx * gyy - gxy * gxy);
        __syncthreads();  // the set-up LDS is reused for the target region

        // Positions are clamped before the integer conversion; past the bounds
        // every tap already reads the level's edge, so the samples are unchanged.
        const float lo = -(float)(g.win + 8), hix = (float)(w + g.win + 8), hiy = (float)(h + g.win + 8);
        nux = 0.0f;
        nuy = 0.0f;
        {
            const float qx = fminf(fmaxf(cx + gx, lo), hix), qy = fminf(fmaxf(cy + gy, lo), hiy);
            sx0 = (int)floorf(qx) - g.r - g.M;
            sy0 = (int)floorf(qy) - g.r - g.M;
            stage_target(Jl, w, h, jp, sx0, sy0, g.SR, g.SC, jr, lane);
            __syncthreads();
        }
        int it = 0;
        while (it < iters) {
            const float qx = fminf(fmaxf(cx + gx + nux, lo), hix);
            const float qy = fminf(fmaxf(cy + gy + nuy, lo), hiy);
            const float fqx = floorf(qx), fqy = floorf(qy);
            const float bxw = qx - fqx, byw = qy - fqy;
            int ox = (int)fqx - g.r - sx0, oy = (int)fqy - g.r - sy0;
            if (ox < 0 || oy < 0 || ox > 2 * g.M || oy > 2 * g.M) {
                __syncthreads();
                sx0 += ox - g.M;
                sy0 += oy - g.M;
                stage_target(Jl, w, h, jp, sx0, sy0, g.SR, g.SC, jr, lane);
                __syncthreads();
                ox = g.M;
                oy = g.M;
            }
            const float2* __restrict__ jb = jr + (oy + row0) * g.SC + ox + col;
            float2 t = jb[0];
            float rp = fmaf(bxw, t.y, t.x);
            float bx = 0.0f, by = 0.0f;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                t = jb[(k + 1) * g.SC];
                const float rn = fmaf(bxw, t.y, t.x);
                const float d = A[k] - fmaf(byw, rn - rp, rp);
                bx = fmaf(d, X[k], bx);
                by = fmaf(d, Y[k], by);
                rp = rn;
            }
            wave_sum2(bx, by, bx, by);
            const float ex = (gyy * bx - gxy * by) * idet;
            const float ey = (gxx * by - gxy * bx) * idet;
            nux += ex;
            nuy += ey;
            ++it;
            if (ex * ex + ey * ey < eps2) break;
        }
        if (lane == 0 && iters_out) iters_out[l] = (uint8_t)min(it, 255);
        if (l > 0) {
            gx = 2.0f * (gx + nux);
            gy = 2.0f * (gy + nuy);
        }
    }
    // level 0: flow = g + nu
    const float fx = gx + nux, fy = gy + nuy;
    const float nx = ux + fx, ny = uy + fy;
    res.nx = nx;
    res.ny = ny;
    if (!(nx >= 0.0f && ny >= 0.0f && nx <= (float)(W0 - 1) && ny <= (float)(H0 - 1))) return res;

    // ---- err: mean |I - J| over the level-0 window at the final position
    {
        const float fqx = floorf(nx), fqy = floorf(ny);
        const float bxw = nx - fqx, byw = ny - fqy;
        int ox = (int)fqx - g.r - sx0, oy = (int)fqy - g.r - sy0;
        if (ox < 0 || oy < 0 || ox > 2 * g.M || oy > 2 * g.M) {
            __syncthreads();
            sx0 += ox - g.M;
            sy0 += oy - g.M;
            stage_target(Q.lvl[0], P.w[0], P.h[0], Q.pitch[0], sx0, sy0, g.SR, g.SC, jr, lane);
            __syncthreads();
            ox = g.M;
            oy = g.M;
        }
        const float2* __restrict__ jb = jr + (oy + row0) * g.SC + ox + col;
        float2 t = jb[0];
        float rp = fmaf(bxw, t.y, t.x);
        float e = 0.0f;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            t = jb[(k + 1) * g.SC];
            const float rn = fmaf(bxw, t.y, t.x);
            const float d = A[k] - fmaf(byw, rn - rp, rp);
            e += (k < nrows) ? fabsf(d) : 0.0f;
            rp = rn;
        }
        res.err = wave_sum(e) / N;
    }
    res.status = 1;
    return res;
}

// ---------------------------------------------------------------------------
// Per-box median of point displacements: exact radix selection (four 8-bit
// passes over order-preserving integer keys), four selections at once
// (x and y at ranks (c-1)/2 and c/2).  256 threads.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t f2key(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key2f(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

struct BoxSmem {
    float dx[BOX_CAP];
    float dy[BOX_CAP];
    uint32_t hist[4][256];
    uint32_t prefix[4];
    uint32_t rank[4];
    int32_t count;
};

// Visit every selected point of the box as f(dx, dy).  In LDS mode the
// gathered values are visited; otherwise the job's points are re-scanned.
template <class F>
__device__ __forceinline__ void box_visit(bool in_lds, const BoxSmem& sm, int c, int b,
                                          const int32_t* __restrict__ box_id,
                                          const uint8_t* __restrict__ status,
                                          const float* __restrict__ pts,
                                          const float* __restrict__ next_pts, int n, F&& f) {
    if (in_lds) {
        for (int i = threadIdx.x; i < c; i += BOX_THREADS) f(sm.dx[i], sm.dy[i]);
    } else {
        for (int i = threadIdx.x; i < n; i += BOX_THREADS)
            if (box_id[i] == b && status[i] == 1)
                f(next_pts[2 * i] - pts[2 * i], next_pts[2 * i + 1] - pts[2 * i + 1]);
    }
}

// Exact k-th smallest keys by radix selection (four 8-bit passes), four
// selections at once: x and y at ranks (c-1)/2 and c/2.
__device__ __forceinline__ void box_radix_select(bool in_lds, BoxSmem& sm, int c, int b,
                                                 const int32_t* __restrict__ box_id,
                                                 const uint8_t* __restrict__ status,
                                                 const float* __restrict__ pts,
                                                 const float* __restrict__ next_pts, int n) {
    const int tid = threadIdx.x;
    if (tid < 4) {
        sm.prefix[tid] = 0;
        sm.rank[tid] = (tid & 1) ? (uint32_t)(c / 2) : (uint32_t)((c - 1) / 2);
    }
    for (int pass = 3; pass >= 0; --pass) {
        const int shift = pass * 8;
        for (int e = tid; e < 4 * 256; e += BOX_THREADS) (&sm.hist[0][0])[e] = 0;
        __syncthreads();
        const uint32_t hmask = pass == 3 ? 0u : (0xFFFFFFFFu << (shift + 8));
        const uint32_t p0 = sm.prefix[0] & hmask, p1 = sm.prefix[1] & hmask;
        const uint32_t p2 = sm.prefix[2] & hmask, p3 = sm.prefix[3] & hmask;
        box_visit(in_lds, sm, c, b, box_id, status, pts, next_pts, n, [&](float vx, float vy) {
            const uint32_t kx = f2key(vx), ky = f2key(vy);
            const uint32_t dxk = (kx >> shift) & 255u, dyk = (ky >> shift) & 255u;
            if ((kx & hmask) == p0) atomicAdd(&sm.hist[0][dxk], 1u);
            if ((kx & hmask) == p1) atomicAdd(&sm.hist[1][dxk], 1u);
            if ((ky & hmask) == p2) atomicAdd(&sm.hist[2][dyk], 1u);
            if ((ky & hmask) == p3) atomicAdd(&sm.hist[3][dyk], 1u);
        });
        __syncthreads();
        const int wave = tid >> 6, lane = tid & 63;
        if (wave < 4) {
            // lane owns bins 4*lane .. 4*lane+3; inclusive scan over lanes
            const uint32_t* hs = sm.hist[wave];
            const uint32_t c0 = hs[4 * lane], c1 = hs[4 * lane + 1], c2 = hs[4 * lane + 2],
                           c3 = hs[4 * lane + 3];
            const uint32_t tot = c0 + c1 + c2 + c3;
            uint32_t incl = tot;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t v = __shfl_up(incl, o, 64);
                if (lane >= o) incl += v;
            }
            const uint32_t excl = incl - tot;
            const uint32_t k = sm.rank[wave];
            if (k >= excl && k < incl) {
                uint32_t base = excl, bin = 4 * lane;
                const uint32_t cs[4] = {c0, c1, c2, c3};
                for (int j = 0; j < 4; ++j) {
                    if (k < base + cs[j]) {
                        bin = 4 * lane + j;
                        break;
                    }
                    base += cs[j];
                }
                sm.prefix[wave] |= bin << shift;
                sm.rank[wave] = k - base;
            }
        }
        __syncthreads();
    }
}

// Ascending bitonic sort of dx[0..np2) and dy[0..np2) in LDS (np2 a power of two).
__device__ __forceinline__ void box_bitonic(BoxSmem& sm, int np2) {
    const int tid = threadIdx.x;
    for (int k = 2; k <= np2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = tid; t < (np2 >> 1); t += BOX_THREADS) {
                const int i = 2 * t - (t & (j - 1)), p = i + j;
                const bool up = (i & k) == 0;
                const float a = sm.dx[i], bb = sm.dx[p];
                if ((a > bb) == up) {
                    sm.dx[i] = bb;
                    sm.dx[p] = a;
                }
                const float c = sm.dy[i], d = sm.dy[p];
                if ((c > d) == up) {
                    sm.dy[i] = d;
                    sm.dy[p] = c;
                }
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ void box_median(const float* __restrict__ boxes, int b,
                                           const int32_t* __restrict__ box_id,
                                           const float* __restrict__ pts,
                                           const float* __restrict__ next_pts,
                                           const uint8_t* __restrict__ status, int n,
                                           float* __restrict__ out_boxes,
                                           int32_t* __restrict__ out_count, BoxSmem& sm) {
    const int tid = threadIdx.x, lane = tid & 63;
    if (tid == 0) sm.count = 0;
    __syncthreads();
    // gather: 16 consecutive ids and statuses per thread in flight (vector
    // loads when aligned), then wave-ballot compaction of the matches into LDS
    const float2* __restrict__ p2 = reinterpret_cast<const float2*>(pts);
    const float2* __restrict__ n2 = reinterpret_cast<const float2*>(next_pts);
    const bool vec = ((reinterpret_cast<uintptr_t>(box_id) | reinterpret_cast<uintptr_t>(status)) & 15) == 0;
    constexpr int PT = 16;
    for (int base = 0; base < n; base += PT * BOX_THREADS) {
        const int i0 = base + tid * PT;
        int32_t id[PT];
        uint32_t st[PT];
        if (vec && i0 + PT <= n) {
#pragma unroll
            for (int q = 0; q < PT / 4; ++q) {
                const int4 v = reinterpret_cast<const int4*>(box_id + i0)[q];
                id[4 * q] = v.x;
                id[4 * q + 1] = v.y;
                id[4 * q + 2] = v.z;
                id[4 * q + 3] = v.w;
            }
            const uint4 sv = *reinterpret_cast<const uint4*>(status + i0);
            const uint32_t sw[4] = {sv.x, sv.y, sv.z, sv.w};
#pragma unroll
            for (int j = 0; j < PT; ++j) st[j] = (sw[j >> 2] >> (8 * (j & 3))) & 255u;
        } else {
#pragma unroll
            for (int j = 0; j < PT; ++j) {
                const int i = i0 + j;
                id[j] = i < n ? box_id[i] : -1;
                st[j] = i < n ? status[i] : 0u;
            }
        }
        // at most PT matches per thread; their point loads are issued together
        float2 pa[PT], pb[PT];
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            const bool match = id[j] == b && st[j] == 1u;
            if (match) {
                pa[j] = p2[i0 + j];
                pb[j] = n2[i0 + j];
            }
        }
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            const bool match = id[j] == b && st[j] == 1u;
            const uint64_t mask = __ballot(match);
            const int cnt = __popcll(mask);
            int off = 0;
            if (lane == 0 && cnt) off = atomicAdd(&sm.count, cnt);
            off = __builtin_amdgcn_readfirstlane(off);
            if (match) {
                const int k = off + __popcll(mask & ((1ull << lane) - 1ull));
                if (k < BOX_CAP) {
                    sm.dx[k] = pb[j].x - pa[j].x;
                    sm.dy[k] = pb[j].y - pa[j].y;
                }
            }
        }
    }
    __syncthreads();
    const int c = sm.count;
    float mx = 0.0f, my = 0.0f;
    if (c > 0 && c <= BOX_SORT_MAX) {
        int np2 = 64;
        while (np2 < c) np2 <<= 1;
        for (int i = c + tid; i < np2; i += BOX_THREADS) {
            sm.dx[i] = __builtin_inff();
            sm.dy[i] = __builtin_inff();
        }
        __syncthreads();
        box_bitonic(sm, np2);
        mx = 0.5f * (sm.dx[(c - 1) / 2] + sm.dx[c / 2]);
        my = 0.5f * (sm.dy[(c - 1) / 2] + sm.dy[c / 2]);
    } else if (c > 0) {
        box_radix_select(c <= BOX_CAP, sm, c, b, box_id, status, pts, next_pts, n);
        mx = 0.5f * (key2f(sm.prefix[0]) + key2f(sm.prefix[1]));
        my = 0.5f * (key2f(sm.prefix[2]) + key2f(sm.prefix[3]));
    }
    if (tid == 0) {
        out_boxes[4 * b + 0] = boxes[4 * b + 0] + mx;
        out_boxes[4 * b + 1] = boxes[4 * b + 1] + my;
        out_boxes[4 * b + 2] = boxes[4 * b + 2] + mx;
        out_boxes[4 * b + 3] = boxes[4 * b + 3] + my;
        out_count[b] = c;
    }
}

}  // namespace ot
