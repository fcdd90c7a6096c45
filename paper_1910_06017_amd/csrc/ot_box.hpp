// ot_box.hpp -- gfx950 device code of the per-box median displacement.
#pragma once
#include "ot_device.hpp"

namespace ot {

// ---------------------------------------------------------------------------
// Per-box median of point displacements, one BOX_THREADS workgroup per box.
// The box's tracked displacements are gathered into LDS; the x and y values
// at ranks (c-1)/2 and c/2 then come from a one-wave register sort per axis
// (c <= BOX_WAVE_SORT) or, for larger boxes, an exact radix selection (four
// 8-bit passes over order-preserving integer keys, four selections at once).
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
    float med[2];
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

// Ascending bitonic sort of 512 values held 8 per lane (value i in lane i/8,
// register i%8) by one wave: the compare distances of 8 and more are lane
// exchanges, the smaller ones stay inside a lane's registers.
template <int J>
__device__ __forceinline__ void sort8_inlane(float (&x)[8], int k, int lane) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        if ((r & J) == 0) {
            const bool up = ((8 * lane + r) & k) == 0;
            const float a = x[r], b = x[r + J];
            x[r] = up ? fminf(a, b) : fmaxf(a, b);
            x[r + J] = up ? fmaxf(a, b) : fminf(a, b);
        }
    }
}

__device__ __forceinline__ void wave_sort512(float (&x)[8], int lane) {
    for (int k = 2; k <= 512; k <<= 1) {
        for (int j = k >> 1; j >= 8; j >>= 1) {
            const int lj = j >> 3;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int i = 8 * lane + r;
                const bool keep_min = ((i & j) == 0) == ((i & k) == 0);
                const float o = __shfl_xor(x[r], lj, 64);
                x[r] = keep_min ? fminf(x[r], o) : fmaxf(x[r], o);
            }
        }
        if (k >= 8) sort8_inlane<4>(x, k, lane);
        if (k >= 4) sort8_inlane<2>(x, k, lane);
        sort8_inlane<1>(x, k, lane);
    }
}

// Values at ranks k1 and k2 of v[0..c) (c <= 512) by one wave; every lane
// gets both.
__device__ __forceinline__ void wave_ranks512(const float* __restrict__ v, int c, int k1, int k2,
                                              int lane, float& r1, float& r2) {
    float x[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int i = 8 * lane + r;
        x[r] = i < c ? v[i] : __builtin_inff();
    }
    wave_sort512(x, lane);
    float a = 0.0f, b = 0.0f;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int i = 8 * lane + r;
        if (i == k1) a = x[r];
        if (i == k2) b = x[r];
    }
    r1 = __shfl(a, k1 >> 3, 64);
    r2 = __shfl(b, k2 >> 3, 64);
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
        // the order of the gathered values does not matter: one wave-wide
        // exclusive scan of the per-thread match counts and one LDS atomic
        // per wave reserve the slots
        int mine = 0;
#pragma unroll
        for (int j = 0; j < PT; ++j) mine += (id[j] == b && st[j] == 1u) ? 1 : 0;
        int incl = mine;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        const int wtot = __shfl(incl, 63, 64);
        int off = 0;
        if (lane == 0 && wtot) off = atomicAdd(&sm.count, wtot);
        int k = __shfl(off, 0, 64) + incl - mine;
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            if (id[j] == b && st[j] == 1u) {
                if (k < BOX_CAP) {
                    sm.dx[k] = pb[j].x - pa[j].x;
                    sm.dy[k] = pb[j].y - pa[j].y;
                }
                ++k;
            }
        }
    }
    __syncthreads();
    const int c = sm.count;
    float mx = 0.0f, my = 0.0f;
    if (c > 0 && c <= BOX_WAVE_SORT) {
        // wave 0 sorts x, wave 1 sorts y, in registers; the others are done
        const int wave = tid >> 6;
        if (wave < 2) {
            float r1, r2;
            wave_ranks512(wave == 0 ? sm.dx : sm.dy, c, (c - 1) / 2, c / 2, lane, r1, r2);
            if (lane == 0) sm.med[wave] = 0.5f * (r1 + r2);
        }
        __syncthreads();
        mx = sm.med[0];
        my = sm.med[1];
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
