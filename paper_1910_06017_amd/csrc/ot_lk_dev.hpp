// ot_lk_dev.hpp -- gfx950 device code of the per-point pyramidal Lucas-Kanade
// tracker (one wave64 per point) and its paired wave reductions.
#pragma once
#include "ot_device.hpp"

// Clamped-byte staging near level edges keeps this many loads per lane in
// flight (registers vs latency).
#ifndef OT_STAGE_BATCH
#define OT_STAGE_BATCH 4
#endif
// Rows of the target region each lane loads per batch on the in-frame path.
#ifndef OT_TARGET_BATCH
#define OT_TARGET_BATCH 4
#endif

namespace ot {

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
    int win, r, nseg, RR, TW, PR, PW, M, SC, SR, SP, AO;
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
        SP = 4 * (((SC + 3) >> 2) + 1);  // target row entries (16-byte rows)
        AO = (int)lk_lds_a_offset(win, R, margin);  // level-0 template samples
    }
};

// Target region, stored as packed half pairs (J[y][x], J[y][x+1] - J[y][x]):
// both are integers of magnitude <= 255, exact in binary16, and a bilinear
// row blend is then one mixed-precision FMA on the pair.  Rows start at the
// 4-byte aligned column a0 = sx0 & ~3 and hold SP entries; entry
// (rr, (sx0 & 3) + cc) covers y = clamp(sy0 + rr), x = clamp(sx0 + cc) for
// rr < SR, cc < SC (SP >= 4 * (((SC + 3) >> 2) + 1)).
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_pair(float j, float dj) {
    return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(j, dj));
}

// Horizontal blend J[x] + bx * (J[x+1] - J[x]) of one packed entry.
__device__ __forceinline__ float blend_pair(uint32_t e, float bx) {
    const half2_t h = __builtin_bit_cast(half2_t, e);
    return fmaf(bx, (float)h.y, (float)h.x);
}

// Bilinear blend of window sums at fractional offset (fx, fy), bb = fx * fy:
// (1-fy) (S_J0 + fx S_D0) + fy (S_J1 + fx S_D1) expanded as
// S_J0 + fx S_D0 + fy (S_J1 - S_J0) + fx fy (S_D1 - S_D0).  The template and
// target terms both go through this one function, so equal inputs give
// equal results (identical frames give b == 0 exactly).
__device__ __forceinline__ float blend_sums(float j0, float d0, float jd, float dd, float fx,
                                            float fy, float bb) {
    return fmaf(bb, dd, fmaf(fy, jd, fmaf(fx, d0, j0)));
}

__device__ __forceinline__ void stage_target(const uint8_t* __restrict__ Jl, int w, int h, int jp,
                                             int sx0, int sy0, int SR, int SC, int SP,
                                             uint32_t* __restrict__ jr, int lane) {
    const plane_t J = plane_rsrc(Jl, (uint32_t)jp * (uint32_t)h);
    const int a0 = sx0 & ~3;
    const int nd = ((sx0 + SC - a0) >> 2) + 1;  // dwords covering columns a0 .. sx0+SC
    const bool fast = a0 >= 0 && sy0 >= 0 && a0 + 4 * nd <= w && sy0 + SR <= h &&
                      ((reinterpret_cast<uintptr_t>(Jl) | (uintptr_t)jp) & 3) == 0;
    if (fast) {
        // one dword (4 pixels) per lane and row; the fifth pixel of the last
        // entry comes from the next lane (junk for the row's last dword, whose
        // last entry lies past column SC - 1 and is never read).  Loads of rows
        // past the region are not predicated: they stay inside the plane or
        // read 0, and are never stored.
        const int rps = udiv_small(64, nd);
        const int lr = udiv_small(lane, nd), kk = lane - lr * nd;
        const bool lane_ok = lr < rps;
        const int steps = udiv_small(SR + rps - 1, rps);
        const uint32_t dstep = (uint32_t)(rps * jp);
        uint32_t off = (uint32_t)((sy0 + lr) * jp + a0 + 4 * kk);
        uint32_t* __restrict__ dst = jr + lr * SP + 4 * kk;
constexpr int TB = OT_TARGET_BATCH;
#pragma unroll 1
        for (int s0 = 0; s0 < steps; s0 += TB) {
            uint32_t v[TB];
#pragma unroll
            for (int s = 0; s < TB; ++s) v[s] = plane_dword(J, off + (uint32_t)s * dstep);
#pragma unroll
            for (int s = 0; s < TB; ++s) {
                const uint32_t nx = __shfl_down(v[s], 1, 64);
                const int rr = lr + (s0 + s) * rps;
                if (lane_ok && rr < SR) {
                    const float b0 = (float)(v[s] & 255u), b1 = (float)((v[s] >> 8) & 255u);
                    const float b2 = (float)((v[s] >> 16) & 255u), b3 = (float)(v[s] >> 24);
                    const float b4 = (float)(nx & 255u);
                    uint4 q;
                    q.x = pack_pair(b0, b1 - b0);
                    q.y = pack_pair(b1, b2 - b1);
                    q.z = pack_pair(b2, b3 - b2);
                    q.w = pack_pair(b3, b4 - b3);
                    *reinterpret_cast<uint4*>(dst + (s0 + s) * rps * SP) = q;
                }
            }
            off += (uint32_t)TB * dstep;
        }
    } else {
        const int off = sx0 - a0;
        const int dr = udiv_small(64, SC), dc = 64 - dr * SC;
        int r = udiv_small(lane, SC), c = lane - r * SC;
        const int nk = (SR * SC + 63) >> 6;
#pragma unroll 1
        for (int kb = 0; kb < nk; kb += OT_STAGE_BATCH) {
            int idx[OT_STAGE_BATCH];
            uint32_t p0[OT_STAGE_BATCH], p1[OT_STAGE_BATCH];
#pragma unroll
            for (int s = 0; s < OT_STAGE_BATCH; ++s) {
                idx[s] = -1;
                // clamped (always in-plane) offsets, loaded unpredicated
                const uint32_t row = (uint32_t)(clampi(sy0 + r, 0, h - 1) * jp);
                p0[s] = plane_byte(J, row + (uint32_t)clampi(sx0 + c, 0, w - 1));
                p1[s] = plane_byte(J, row + (uint32_t)clampi(sx0 + c + 1, 0, w - 1));
                if (kb + s < nk && r < SR) idx[s] = r * SP + off + c;
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
                    jr[idx[s]] = pack_pair(f0, f1 - f0);
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
    const plane_t I = plane_rsrc(Il, (uint32_t)ip * (uint32_t)h);
    const int xs = x0 - 1, ys = y0 - 1;
    const int a0 = xs & ~3;
    const int nd = ((x0 + g.TW - a0) >> 2) + 1;  // dwords covering a0 .. x0+TW
    const bool fast = a0 >= 0 && ys >= 0 && a0 + 4 * nd <= w && ys + g.PR <= h &&
                      ((reinterpret_cast<uintptr_t>(Il) | (uintptr_t)ip) & 3) == 0;
    if (fast) {
        const int rps = udiv_small(64, nd);
        const int lr = udiv_small(lane, nd), kk = lane - lr * nd;
        const bool lane_ok = lr < rps;
        const int steps = udiv_small(g.PR + rps - 1, rps);
        const uint32_t dstep = (uint32_t)(rps * ip);
        uint32_t off = (uint32_t)((ys + lr) * ip + a0 + 4 * kk);
#pragma unroll 1
        for (int s0 = 0; s0 < steps; s0 += 4) {
            uint32_t v[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) v[s] = plane_dword(I, off + (uint32_t)s * dstep);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int rr = lr + (s0 + s) * rps;
                if (lane_ok && rr < g.PR)
                    *reinterpret_cast<uint32_t*>(patch + rr * g.PW + 4 * kk) = v[s];
            }
            off += 4u * dstep;
        }
    } else {
        const int cols = g.TW + 2, po = xs - a0;
        const int dr = udiv_small(64, cols), dc = 64 - dr * cols;
        int r = udiv_small(lane, cols), c = lane - r * cols;
        const int nk = (g.PR * cols + 63) >> 6;
#pragma unroll 1
        for (int kb = 0; kb < nk; kb += 8) {
            int idx[8];
            uint32_t p[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                idx[s] = -1;
                p[s] = plane_byte(I, (uint32_t)(clampi(ys + r, 0, h - 1) * ip +
                                                clampi(xs + c, 0, w - 1)));
                if (kb + s < nk && r < g.PR) idx[s] = r * g.PW + po + c;
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

// Issue priority of a wave (s_setprio), which changes only which ready wave
// of a SIMD issues first, never a result.
//  LK_PRIO_REMAINING: by the work the wave has left.  A launch holds more
//   points than the chip has wave slots, and a point's cost is not known
//   before it is tracked, so the launch ends with a tail of long waves.
//   Waves on the coarse levels (most of their work still ahead) outrank those
//   on the fine ones, and a level's iterations (a chain of dependent
//   wave-uniform steps) outrank the set-up work of the same level.
//  LK_PRIO_ITERATIONS: only the iterations are raised, for launches of many
//   rounds of waves, where the tail is a small part and the throughput of the
//   rounds is what counts.
enum LkPrio { LK_PRIO_NONE = 0, LK_PRIO_REMAINING = 1, LK_PRIO_ITERATIONS = 2 };

__device__ __forceinline__ void lk_priority(int p) {
    switch (p) {
        case 0: __builtin_amdgcn_s_setprio(0); break;
        case 1: __builtin_amdgcn_s_setprio(1); break;
        case 2: __builtin_amdgcn_s_setprio(2); break;
        default: __builtin_amdgcn_s_setprio(3); break;
    }
}

// Orders a wave's LDS writes before its later reads of them (the region a
// wave stages is private to it).  With several waves per workgroup (WSYNC)
// the order is kept within the wave only: the waves track different points
// with different iteration counts and never wait on each other.  A
// one-wave workgroup uses the workgroup barrier, which is the same thing.
template <bool WSYNC>
__device__ __forceinline__ void lk_sync() {
    if constexpr (WSYNC) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Positions are carried as an exact integer anchor plus a small float
// offset: a level coordinate of ~2000 px held in one float has a spacing of
// 1.2e-4 px, which a non-contracting iterate amplifies, while an offset of a
// few pixels keeps ~1e-7 px.  split_pos gives the integer floor and the
// fraction of anchor + t.  The offset is bounded to +-2^20 px so the integer
// cannot overflow; a position past the level's edge needs no other bound,
// since every tap of a region staged there reads the edge (the staging
// clamps each index), the value the oracle's clamped taps give as well.
__device__ __forceinline__ void split_pos(int anchor, float t, int& ip, float& f) {
    t = __builtin_amdgcn_fmed3f(t, -1048576.0f, 1048576.0f);
    const float ft = floorf(t);
    ip = anchor + (int)ft;
    f = t - ft;
}

// g <- 2 (g + nu) on the split form g = gi + gf, gf in [0, 1): the doubling
// and the floor are exact, only gf + nu rounds (at the magnitude of nu).
__device__ __forceinline__ void carry_level(int& gi, float& gf, float nu) {
    const float t = 2.0f * __builtin_amdgcn_fmed3f(gf + nu, -1048576.0f, 1048576.0f);
    const float ft = floorf(t);
    gi = 2 * gi + (int)ft;
    gf = t - ft;
}

// FIXED: the geometry g is a compile-time constant (the caller's window and
// margin are template arguments), so fixed-count loops are unrolled.
// GRADS: the template pyramid carries materialized Scharr sums, which are
// read (at clamped indices) instead of computed.
// PRIO: the wave's issue-priority rule (LkPrio).
template <int R, bool FIXED, bool GRADS, class PyrRef, bool WSYNC = false, int PRIO = LK_PRIO_NONE>
__device__ __forceinline__ LkResult lk_point(const PyrRef& P, const PyrRef& Q, float ux, float uy,
                                             int L, int iters, float eps2, float min_eig,
                                             const LkGeom& g, unsigned char* __restrict__ smem,
                                             uint8_t* iters_out, float* lam_out) {
    const int lane = threadIdx.x & 63;
    const int used = g.win * g.nseg;
    const bool lvalid = lane < used;
    const int seg = lvalid ? udiv_small(lane, g.win) : 0;
    const int col = lvalid ? lane - seg * g.win : 0;
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

    float X[R], Y[R];
    float* __restrict__ aA = reinterpret_cast<float*>(smem + g.AO);  // [R][64], level 0 only
    // guess g = (gix + gfx, giy + gfy) in the current level's pixels
    int gix = 0, giy = 0;
    float gfx = 0.0f, gfy = 0.0f;
    float nux = 0.0f, nuy = 0.0f;
    uint32_t* jr = reinterpret_cast<uint32_t*>(smem);
    uint8_t* patch = smem;
    float2* grad = reinterpret_cast<float2*>(smem + ((g.PR * g.PW + 15) & ~15));
    int sx0 = 0, sy0 = 0;  // origin of the staged target region (level coords)
    int soff = 0;          // sx0 & 3: column of sx0 in a staged row

    for (int l = L - 1; l >= 0; --l) {
        if constexpr (PRIO == LK_PRIO_REMAINING) lk_priority(min(l, 2));
        if constexpr (PRIO == LK_PRIO_ITERATIONS) lk_priority(0);
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
        lk_sync<WSYNC>();
        // ---- Scharr gradients at the tap grid: the gradient image is defined on
        // the level's pixels and read at clamped indices, so a tap outside the
        // level takes the gradient of the nearest edge pixel.  The responses are
        // kept as the integer sums (32x the gradient); the factor is exact and
        // is taken out in the tensor, the gate and the solve.
        if constexpr (GRADS) {
            // the planes hold the sums of every level pixel; a tap outside the
            // level reads the nearest edge pixel's sums
            const int32_t* __restrict__ Gl = P.grad[l];
            const int gp = P.gpitch[l];
            const bool inside = x0 >= 0 && x0 + g.TW <= w && y0 >= 0 && y0 + g.RR <= h;
            const int dr = udiv_small(64, g.TW), dc = 64 - dr * g.TW;
            int ty = udiv_small(lane, g.TW), tx = lane - ty * g.TW;
            const int ntap = g.RR * g.TW;
            auto tap = [&](int e) {
                if (e < ntap) {
                    const int qx = inside ? x0 + tx : clampi(x0 + tx, 0, w - 1);
                    const int qy = inside ? y0 + ty : clampi(y0 + ty, 0, h - 1);
                    const int32_t v = Gl[(size_t)qy * gp + qx];
                    grad[e] = make_float2((float)(int16_t)(v & 0xFFFF), (float)(v >> 16));
                }
                tx += dc;
                ty += dr;
                if (tx >= g.TW) {
                    tx -= g.TW;
                    ++ty;
                }
            };
            const int nk = (ntap + 63) >> 6;
#pragma unroll 2
            for (int k = 0; k < nk; ++k) tap(lane + 64 * k);
        } else if (x0 >= 1 && x0 + g.TW <= w - 1 && y0 >= 1 && y0 + g.RR <= h - 1) {
            // interior: no clamping; ncg groups of TW lanes each slide a 3x3
            // window down GR consecutive taps of a column, so a tap costs three
            // byte reads.  With d = right - left and t = 3 left + 10 centre +
            // 3 right per row: Sx = 3 d(y-1) + 10 d(y) + 3 d(y+1),
            // Sy = t(y+1) - t(y-1).  Groups run past row RR - 1 when ncg does
            // not divide RR; those taps land in LDS rows nobody reads.
            const int ncg = udiv_small(64, g.TW);
            const int GR = udiv_small(g.RR + ncg - 1, ncg);
            const int rg = udiv_small(lane, g.TW), tx = lane - rg * g.TW;
            if (rg < ncg) {
                const int ty0 = rg * GR;
                const uint8_t* pp = patch + ty0 * g.PW + (x0 + tx - a0p);
                float2* gp = grad + ty0 * g.TW + tx;
                int vl = pp[-1], vc = pp[0], vr = pp[1];
                int d0 = vr - vl, t0 = 3 * (vl + vr) + 10 * vc;
                vl = pp[g.PW - 1], vc = pp[g.PW], vr = pp[g.PW + 1];
                int d1 = vr - vl, t1 = 3 * (vl + vr) + 10 * vc;
                auto tap = [&](int k) {
                    const uint8_t* q = pp + (k + 2) * g.PW;
                    vl = q[-1], vc = q[0], vr = q[1];
                    const int d2 = vr - vl, t2 = 3 * (vl + vr) + 10 * vc;
                    gp[k * g.TW] = make_float2((float)(3 * (d0 + d2) + 10 * d1), (float)(t2 - t0));
                    d0 = d1;
                    d1 = d2;
                    t0 = t1;
                    t1 = t2;
                };
                if constexpr (FIXED) {
#pragma unroll
                    for (int k = 0; k < GR; ++k) tap(k);
                } else {
#pragma unroll 1
                    for (int k = 0; k < GR; ++k) tap(k);
                }
            }
        } else {
            const int dr = udiv_small(64, g.TW), dc = 64 - dr * g.TW;
            int ty = udiv_small(lane, g.TW), tx = lane - ty * g.TW;
            const int ntap = g.RR * g.TW;
#pragma unroll 1
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
                grad[e] = make_float2((float)sxv, (float)syv);
                tx += dc;
                ty += dr;
                if (tx >= g.TW) {
                    tx -= g.TW;
                    ++ty;
                }
            }
        }
        lk_sync<WSYNC>();
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
                    if (l == 0) aA[(k - 1) * 64 + lane] = v ? fmaf(ay, ri - pi, pi) : 0.0f;
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
        // sum(A grad) through the same window sums and blend the iterations use
        // for the target (below), so identical frames give b == 0 exactly
        float cax, cay;
        {
            const uint8_t* pr = patch + (row0 + 1) * g.PW + x0 + col - a0p;
            float p0 = 0.0f, p1 = 0.0f, p2 = 0.0f, p3 = 0.0f;
            float q0 = 0.0f, q1 = 0.0f, q2 = 0.0f, q3 = 0.0f;
            float i0 = (float)pr[0], di0 = (float)pr[1] - i0;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const float i1 = (float)pr[(k + 1) * g.PW], di1 = (float)pr[(k + 1) * g.PW + 1] - i1;
                p0 = fmaf(i0, X[k], p0);
                p1 = fmaf(di0, X[k], p1);
                p2 = fmaf(i1, X[k], p2);
                p3 = fmaf(di1, X[k], p3);
                q0 = fmaf(i0, Y[k], q0);
                q1 = fmaf(di0, Y[k], q1);
                q2 = fmaf(i1, Y[k], q2);
                q3 = fmaf(di1, Y[k], q3);
                i0 = i1;
                di0 = di1;
            }
            float tj0x, td0x, tj1x, td1x, tj0y, td0y, tj1y, td1y;
            wave_sum4(p0, p1, p2, p3, tj0x, td0x, tj1x, td1x);
            wave_sum4(q0, q1, q2, q3, tj0y, td0y, tj1y, td1y);
            cax = blend_sums(tj0x, td0x, tj1x - tj0x, td1x - td0x, ax, ay, ax * ay);
            cay = blend_sums(tj0y, td0y, tj1y - tj0y, td1y - td0y, ax, ay, ax * ay);
        }
        // the sums are 1024x the tensor of the true gradients (exactly)
        const float hm = 0.5f * (gxx + gyy), hd = 0.5f * (gxx - gyy);
        const float lam = ((hm - sqrtf(hd * hd + gxy * gxy)) / N) * (1.0f / 1024.0f);
        if (lane == 0 && lam_out) lam_out[l] = lam;
        if (!(lam >= min_eig)) {
            if (lane == 0)
                for (int k = l; k >= 0; --k) {
                    if (iters_out) iters_out[k] = 0;
                    if (lam_out && k < l) lam_out[k] = 0.0f;
                }
            const double s = __builtin_ldexp(1.0, l);
            res.nx = (float)((double)ux + ((double)gix + (double)gfx) * s);
            res.ny = (float)((double)uy + ((double)giy + (double)gfy) * s);
            return res;
        }
        // b comes out 32x and the tensor 1024x: 32 / det(1024 G) gives eta
        const float idet = 32.0f / (gxx * gyy - gxy * gxy);
        lk_sync<WSYNC>();  // the set-up LDS is reused for the target region

        // Positions are clamped before the integer conversion; past the bounds
        // every tap already reads the level's edge, so the samples are unchanged.
        // target position c + g + nu = (floor(c) + gi) + (frac(c) + gf + nu)
        const int ancx = (int)flx + gix, ancy = (int)fly + giy;
        const float f0x = ax + gfx, f0y = ay + gfy;
        nux = 0.0f;
        nuy = 0.0f;
        {
            int qx, qy;
            float unusedx, unusedy;
            split_pos(ancx, f0x, qx, unusedx);
            split_pos(ancy, f0y, qy, unusedy);
            sx0 = qx - g.r - g.M;
            sy0 = qy - g.r - g.M;
            stage_target(Jl, w, h, jp, sx0, sy0, g.SR, g.SC, g.SP, jr, lane);
            soff = sx0 & 3;
            lk_sync<WSYNC>();
        }
        // The bilinear target at position floor + (fx, fy) blends four whole-
        // pixel samples with weights that depend only on (fx, fy), so
        //   sum_p J(p + d) grad_p = (1-fy) (S_J0 + fx S_D0) + fy (S_J1 + fx S_D1)
        // with S_J0 = sum J(row k) grad, S_D0 = sum (J(x+1) - J(x))(row k) grad
        // and S_J1, S_D1 the same one row down.  These eight window sums are
        // recomputed only when the floor position changes; an iteration that
        // stays on the same pixel costs a handful of wave-uniform operations.
        // The sums are kept as (S_J0, S_D0, S_J1 - S_J0, S_D1 - S_D0), the form
        // blend_sums takes, which the template term above uses as well.
        int sfx = INT32_MIN, sfy = INT32_MIN;  // floor position of the sums
        float sj0x = 0.0f, sd0x = 0.0f, sjdx = 0.0f, sddx = 0.0f;
        float sj0y = 0.0f, sd0y = 0.0f, sjdy = 0.0f, sddy = 0.0f;
        int it = 0;
        if constexpr (PRIO == LK_PRIO_REMAINING) lk_priority(min(l, 2) + 1);
        if constexpr (PRIO == LK_PRIO_ITERATIONS) lk_priority(2);
        while (it < iters) {
            int ifx, ify;
            float bxw, byw;
            split_pos(ancx, f0x + nux, ifx, bxw);
            split_pos(ancy, f0y + nuy, ify, byw);
            int ox = ifx - g.r - sx0, oy = ify - g.r - sy0;
            if (ox < 0 || oy < 0 || ox > 2 * g.M || oy > 2 * g.M) {
                lk_sync<WSYNC>();
                sx0 += ox - g.M;
                sy0 += oy - g.M;
                stage_target(Jl, w, h, jp, sx0, sy0, g.SR, g.SC, g.SP, jr, lane);
                soff = sx0 & 3;
                lk_sync<WSYNC>();
                ox = g.M;
                oy = g.M;
            }
            if (ifx != sfx || ify != sfy) {
                const uint32_t* __restrict__ jb = jr + (oy + row0) * g.SP + soff + ox + col;
                float p0 = 0.0f, p1 = 0.0f, p2 = 0.0f, p3 = 0.0f;
                float q0 = 0.0f, q1 = 0.0f, q2 = 0.0f, q3 = 0.0f;
                half2_t e = __builtin_bit_cast(half2_t, jb[0]);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const half2_t en = __builtin_bit_cast(half2_t, jb[(k + 1) * g.SP]);
                    p0 = fmaf((float)e.x, X[k], p0);
                    p1 = fmaf((float)e.y, X[k], p1);
                    p2 = fmaf((float)en.x, X[k], p2);
                    p3 = fmaf((float)en.y, X[k], p3);
                    q0 = fmaf((float)e.x, Y[k], q0);
                    q1 = fmaf((float)e.y, Y[k], q1);
                    q2 = fmaf((float)en.x, Y[k], q2);
                    q3 = fmaf((float)en.y, Y[k], q3);
                    e = en;
                }
                float sj1x, sd1x, sj1y, sd1y;
                wave_sum4(p0, p1, p2, p3, sj0x, sd0x, sj1x, sd1x);
                wave_sum4(q0, q1, q2, q3, sj0y, sd0y, sj1y, sd1y);
                sjdx = sj1x - sj0x;
                sddx = sd1x - sd0x;
                sjdy = sj1y - sj0y;
                sddy = sd1y - sd0y;
                sfx = ifx;
                sfy = ify;
            }
            const float bb = bxw * byw;
            const float bx = cax - blend_sums(sj0x, sd0x, sjdx, sddx, bxw, byw, bb);
            const float by = cay - blend_sums(sj0y, sd0y, sjdy, sddy, bxw, byw, bb);
            const float ex = (gyy * bx - gxy * by) * idet;
            const float ey = (gxx * by - gxy * bx) * idet;
            nux += ex;
            nuy += ey;
            ++it;
            if (ex * ex + ey * ey < eps2) break;
        }
        if (lane == 0 && iters_out) iters_out[l] = (uint8_t)min(it, 255);
        if (l > 0) {
            carry_level(gix, gfx, nux);
            carry_level(giy, gfy, nuy);
        }
    }
    // level 0: next = u + g + nu = floor(u) + gi + (frac(u) + gf + nu), one rounding
    const float fu0x = floorf(ux), fu0y = floorf(uy);
    const int fix0 = (int)fu0x + gix, fiy0 = (int)fu0y + giy;
    const float ffx0 = ((ux - fu0x) + gfx) + nux, ffy0 = ((uy - fu0y) + gfy) + nuy;
    const float nx = (float)((double)fix0 + (double)ffx0);
    const float ny = (float)((double)fiy0 + (double)ffy0);
    res.nx = nx;
    res.ny = ny;
    if (!(nx >= 0.0f && ny >= 0.0f && nx <= (float)(W0 - 1) && ny <= (float)(H0 - 1))) return res;

    // ---- err: mean |I - J| over the level-0 window at the final position
    {
        int qx, qy;
        float bxw, byw;
        split_pos(fix0, ffx0, qx, bxw);
        split_pos(fiy0, ffy0, qy, byw);
        int ox = qx - g.r - sx0, oy = qy - g.r - sy0;
        if (ox < 0 || oy < 0 || ox > 2 * g.M || oy > 2 * g.M) {
            lk_sync<WSYNC>();
            sx0 += ox - g.M;
            sy0 += oy - g.M;
            stage_target(Q.lvl[0], P.w[0], P.h[0], Q.pitch[0], sx0, sy0, g.SR, g.SC, g.SP, jr, lane);
            soff = sx0 & 3;
            lk_sync<WSYNC>();
            ox = g.M;
            oy = g.M;
        }
        const uint32_t* __restrict__ jb = jr + (oy + row0) * g.SP + soff + ox + col;
        float rp = blend_pair(jb[0], bxw);
        float e = 0.0f;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const float rn = blend_pair(jb[(k + 1) * g.SP], bxw);
            const float d = aA[k * 64 + lane] - fmaf(byw, rn - rp, rp);
            e += (k < nrows) ? fabsf(d) : 0.0f;
            rp = rn;
        }
        res.err = wave_sum(e) / N;
    }
    res.status = 1;
    return res;
}

}  // namespace ot
