// ot_pyr.hpp -- gfx950 device code of the fused Gaussian pyramid reduce.
#pragma once
#include "ot_device.hpp"

namespace ot {

// ---------------------------------------------------------------------------
// Gaussian pyramid: K <= PYR_FUSE consecutive reduce steps (binomial
// (1,4,6,4,1) in both directions, clamp-to-edge, exact integer sum rounded
// half up) in one launch.  A workgroup owns a PYR_FTW x PYR_FTH tile of the
// top level l0+K and the tile's footprint (2^d times larger) at the level d
// steps below it.  It stages the level-l0 region that footprint depends on
// and reduces it level by level in LDS.  The region at each level extends
// past the footprint by the filter support; a region position outside the
// level holds the level's value at the clamped position, which is exactly
// what the next reduction reads under the clamp-to-edge rule.  Every output
// pixel is written by one workgroup and equals the level-by-level result.
// ---------------------------------------------------------------------------
constexpr int pyr_fc(int d) { return d == 0 ? PYR_FTW : 2 * pyr_fc(d - 1) + 3; }
constexpr int pyr_fr(int d) { return d == 0 ? PYR_FTH : 2 * pyr_fr(d - 1) + 3; }
constexpr int PYR_IN_P = 4 * ((pyr_fc(PYR_FUSE) + 6) / 4);  // staged row bytes
constexpr int PYR_MID_R = pyr_fr(PYR_FUSE - 1), PYR_MID_P = pyr_fc(PYR_FUSE - 1);

struct PyrSmem {
    // level-l0 region; rows start at the 4-byte aligned column at or below
    // the region's first column
    uint8_t in[pyr_fr(PYR_FUSE)][PYR_IN_P];
    uint16_t hs[pyr_fr(PYR_FUSE)][PYR_MID_P];  // horizontal pass
    uint8_t mid[2][PYR_MID_R][PYR_MID_P];      // intermediate levels
};

// Step k (level l0+k, d = K-k steps below the top): reduce the region at
// distance d+1 (the staged input for k = 1, else an intermediate region) to
// the region at distance d; store it for the next step and write the owned
// footprint to the level.
template <int K, int k>
__device__ __forceinline__ void pyr_step(const DevPyr& P, int l0, const int (&X)[K + 1],
                                         const int (&Y)[K + 1], int in_off, int tx, int ty,
                                         PyrSmem& sm) {
    constexpr int d = K - k;
    constexpr int RL = pyr_fr(d + 1), CU = pyr_fc(d), RU = pyr_fr(d);
    const int tid = threadIdx.x;
    const int l = l0 + k;
    const int w = P.w[l], h = P.h[l];
    const uint8_t* lo;
    int lo_p, lo_off;
    if constexpr (k == 1) {
        lo = &sm.in[0][0];
        lo_p = PYR_IN_P;
        lo_off = in_off;
    } else {
        lo = &sm.mid[(k - 2) & 1][0][0];
        lo_p = PYR_MID_P;
        lo_off = 0;
    }
    lo_off -= X[d + 1] + 2;
    for (int e = tid; e < RL * CU; e += PYR_THREADS) {
        const int i = e / CU, j = e - i * CU;
        const int xc = clampi(X[d] + j, 0, w - 1);
        const uint8_t* p = lo + i * lo_p + lo_off + 2 * xc;
        sm.hs[i][j] = (uint16_t)((int)p[0] + 4 * (int)p[1] + 6 * (int)p[2] + 4 * (int)p[3] + (int)p[4]);
    }
    __syncthreads();
    uint8_t* __restrict__ dst = const_cast<uint8_t*>(P.lvl[l]);
    const int dp = P.pitch[l];
    const int fx0 = tx * (PYR_FTW << d), fy0 = ty * (PYR_FTH << d);
    const int fx1 = min(fx0 + (PYR_FTW << d), w), fy1 = min(fy0 + (PYR_FTH << d), h);
    for (int e = tid; e < RU * CU; e += PYR_THREADS) {
        const int i = e / CU, j = e - i * CU;
        const int r = 2 * clampi(Y[d] + i, 0, h - 1) - 2 - Y[d + 1];
        const int s = (int)sm.hs[r][j] + 4 * (int)sm.hs[r + 1][j] + 6 * (int)sm.hs[r + 2][j] +
                      4 * (int)sm.hs[r + 3][j] + (int)sm.hs[r + 4][j];
        const uint8_t v = (uint8_t)((s + 128) >> 8);
        if constexpr (k < K) sm.mid[(k - 1) & 1][i][j] = v;
        const int x = X[d] + j, y = Y[d] + i;
        if (x >= fx0 && x < fx1 && y >= fy0 && y < fy1) dst[(size_t)y * dp + x] = v;
    }
    if constexpr (k < K) {
        __syncthreads();
        pyr_step<K, k + 1>(P, l0, X, Y, in_off, tx, ty, sm);
    }
}

// Levels l0+1 .. l0+K of P for top-level tile (tx, ty).  PYR_THREADS threads.
template <int K>
__device__ __forceinline__ void pyr_fused_tile(const DevPyr& P, int l0, int tx, int ty,
                                               PyrSmem& sm) {
    const int tid = threadIdx.x;
    int X[K + 1], Y[K + 1];  // region origins, d steps below the top, in that level's pixels
    X[0] = tx * PYR_FTW;
    Y[0] = ty * PYR_FTH;
#pragma unroll
    for (int d = 1; d <= K; ++d) {
        X[d] = 2 * X[d - 1] - 2;
        Y[d] = 2 * Y[d - 1] - 2;
    }
    const uint8_t* __restrict__ src = P.lvl[l0];
    const int sw = P.w[l0], sh = P.h[l0], sp = P.pitch[l0];
    constexpr int IR = pyr_fr(K), IC = pyr_fc(K);
    const int ix0 = X[K], iy0 = Y[K];
    const int a0 = ix0 & ~3, off = ix0 - a0;
    constexpr int ND = (IC + 6) / 4;  // dwords covering [a0, ix0 + IC) for any off
    const bool fast = a0 >= 0 && iy0 >= 0 && a0 + 4 * ND <= sw && iy0 + IR <= sh &&
                      ((reinterpret_cast<uintptr_t>(src) | (uintptr_t)sp) & 3) == 0;
    if (fast) {
        constexpr int NT = IR * ND, PER = (NT + PYR_THREADS - 1) / PYR_THREADS;
        uint32_t v[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * PYR_THREADS;
            const int r = e / ND, c = e - r * ND;
            v[q] = e < NT ? *reinterpret_cast<const uint32_t*>(src + (size_t)(iy0 + r) * sp + a0 + 4 * c)
                          : 0u;
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * PYR_THREADS;
            const int r = e / ND, c = e - r * ND;
            if (e < NT) *reinterpret_cast<uint32_t*>(&sm.in[r][4 * c]) = v[q];
        }
    } else {
        constexpr int NT = IR * IC, PER = (NT + PYR_THREADS - 1) / PYR_THREADS;
        for (int q0 = 0; q0 < PER; q0 += 8) {
            uint32_t v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = tid + (q0 + q) * PYR_THREADS;
                const int r = e / IC, c = e - r * IC;
                const int y = clampi(iy0 + r, 0, sh - 1), x = clampi(ix0 + c, 0, sw - 1);
                v[q] = (q0 + q < PER && e < NT) ? src[(size_t)y * sp + x] : 0u;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = tid + (q0 + q) * PYR_THREADS;
                const int r = e / IC, c = e - r * IC;
                if (q0 + q < PER && e < NT) sm.in[r][off + c] = (uint8_t)v[q];
            }
        }
    }
    __syncthreads();
    pyr_step<K, 1>(P, l0, X, Y, off, tx, ty, sm);
}

// Runtime step count (uniform per workgroup).
__device__ __forceinline__ void pyr_fused(const DevPyr& P, int l0, int K, int tx, int ty,
                                          PyrSmem& sm) {
    switch (K) {
        case 1: pyr_fused_tile<1>(P, l0, tx, ty, sm); break;
        case 2: pyr_fused_tile<2>(P, l0, tx, ty, sm); break;
        default: pyr_fused_tile<3>(P, l0, tx, ty, sm); break;
    }
}

// ---------------------------------------------------------------------------
// Materialized Scharr sums of one level: one GRAD_THREADS workgroup per
// GRAD_TW x GRAD_TH tile stages the tile plus a one-pixel halo (clamped to
// the level, so border pixels see their clamped neighbours) in LDS and
// writes (Sx & 0xFFFF) | (Sy << 16) per pixel.
// ---------------------------------------------------------------------------
constexpr int GRAD_TW = 64, GRAD_TH = 16, GRAD_THREADS = 256;

struct GradSmem {
    uint8_t in[GRAD_TH + 2][GRAD_TW + 4];
};

__device__ __forceinline__ void grad_tile(const uint8_t* __restrict__ src, int w, int h, int sp,
                                          int32_t* __restrict__ dst, int gp, int tx, int ty,
                                          GradSmem& sm) {
    const int tid = threadIdx.x;
    const int x0 = tx * GRAD_TW - 1, y0 = ty * GRAD_TH - 1;
    constexpr int IR = GRAD_TH + 2, IC = GRAD_TW + 2;
    for (int e = tid; e < IR * IC; e += GRAD_THREADS) {
        const int r = e / IC, c = e - r * IC;
        sm.in[r][c] = src[(size_t)clampi(y0 + r, 0, h - 1) * sp + clampi(x0 + c, 0, w - 1)];
    }
    __syncthreads();
    // one thread per 4 horizontally adjacent pixels
    const int r = tid / (GRAD_TW / 4), c0 = (tid - r * (GRAD_TW / 4)) * 4;
    const int y = ty * GRAD_TH + r;
    if (y >= h) return;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = c0 + k, x = tx * GRAD_TW + c;
        if (x >= w) break;
        const uint8_t* u = &sm.in[r][c];  // (x-1, y-1)
        const uint8_t* m = u + (GRAD_TW + 4);
        const uint8_t* d = m + (GRAD_TW + 4);
        const int sx = 3 * ((int)u[2] - (int)u[0]) + 10 * ((int)m[2] - (int)m[0]) +
                       3 * ((int)d[2] - (int)d[0]);
        const int sy = 3 * ((int)d[0] - (int)u[0]) + 10 * ((int)d[1] - (int)u[1]) +
                       3 * ((int)d[2] - (int)u[2]);
        dst[(size_t)y * gp + x] = (int32_t)(((uint32_t)sx & 0xFFFFu) | ((uint32_t)sy << 16));
    }
}

}  // namespace ot
