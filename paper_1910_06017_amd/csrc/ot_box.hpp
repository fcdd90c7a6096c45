// ot_box.hpp -- gfx950 device code of the per-box median displacement.
#pragma once
#include "ot_device.hpp"

namespace ot {

// ---------------------------------------------------------------------------
// Per-box median of point displacements, one BOX_THREADS workgroup per box.
// The box's tracked displacements are gathered into LDS (boxes with more than
// BOX_CAP are re-read from memory on every pass instead).  The x and y values
// at ranks (c-1)/2 and c/2 are then selected exactly on order-preserving
// integer keys: each round histograms the keys of the range still holding
// both ranks into BOX_NB buckets of equal key width; if the two ranks fall in
// different buckets they are the largest key of the lower bucket and the
// smallest of the upper one, if they share a bucket of at most BOX_CAND keys
// one wave ranks those keys, and otherwise the next round narrows the range
// to that bucket's keys.  The first round's buckets are linear in the value
// (one round is the common case); later rounds shrink the key range by
// BOX_NB and a bucket one key wide is its own answer, so at most five rounds
// run.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t f2key(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key2f(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

constexpr int BOX_NB = 1024;   // buckets per round
constexpr int BOX_CAND = 64;   // a shared bucket this small is ranked by one wave

struct BoxSmem {
    float dx[BOX_CAP];
    float dy[BOX_CAP];
    uint32_t hist[2][BOX_NB];
    uint32_t klo[2], khi[2];    // per axis: key range holding both targets
    uint32_t rank[2][2];        // the targets' ranks among the keys in that range
    int32_t bkt[2][2];          // the targets' buckets this round
    int32_t mode[2];            // 0 done, 1 two buckets, 2 rank candidates, 3 narrow
    uint32_t red[2][4];         // max of bucket 0, min of bucket 1, min and max of bucket 0
    uint32_t ncand[2];
    uint32_t cand[2][BOX_CAND];
    uint32_t res[2][2];         // selected keys
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

// Bucket map of one axis for one round: linear in the value over [lo, hi]
// (the first round, so a tight cluster spreads over many buckets even when
// outliers stretch the range), or linear in the key with a power-of-two width
// (later rounds, and whenever the value span is not a usable float).  Both
// are non-decreasing in the key, so buckets partition the keys in order.
struct BoxMap {
    uint32_t lo, hi;
    float vlo, scale;
    int sh;
    bool lin;
    __device__ __forceinline__ bool in(uint32_t k) const { return k >= lo && k <= hi; }
    __device__ __forceinline__ int bucket(uint32_t k, float v) const {
        return lin ? min(BOX_NB - 1, (int)((v - vlo) * scale)) : (int)((k - lo) >> sh);
    }
};

__device__ __forceinline__ BoxMap box_map(uint32_t lo, uint32_t hi, bool linear) {
    BoxMap m;
    m.lo = lo;
    m.hi = hi;
    const uint32_t span = hi - lo;
    const int bits = span == 0u ? 0 : 32 - __clz((int)span);
    m.sh = max(0, bits - 10);  // (hi - lo) >> sh < BOX_NB
    m.vlo = key2f(lo);
    const float vspan = key2f(hi) - m.vlo;
    m.scale = (float)BOX_NB / vspan;
    m.lin = linear && vspan > 0.0f && __builtin_isfinite(vspan) && __builtin_isfinite(m.scale) &&
            m.scale > 0.0f;
    return m;
}

// Keys of x and y at ranks (c-1)/2 and c/2 (c > 0) into sm.res.  On entry
// sm.klo/khi hold each axis' smallest and largest key, sm.rank the two ranks
// and sm.hist is zero (all written before a barrier that precedes the first
// read).
__device__ __forceinline__ void box_select(bool in_lds, BoxSmem& sm, int c, int b,
                                           const int32_t* __restrict__ box_id,
                                           const uint8_t* __restrict__ status,
                                           const float* __restrict__ pts,
                                           const float* __restrict__ next_pts, int n) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int round = 0; round < 8; ++round) {
        const int mode0 = round == 0 ? 3 : sm.mode[0], mode1 = round == 0 ? 3 : sm.mode[1];
        if (mode0 == 0 && mode1 == 0) break;
        const BoxMap m0 = box_map(sm.klo[0], sm.khi[0], round == 0);
        const BoxMap m1 = box_map(sm.klo[1], sm.khi[1], round == 0);
        box_visit(in_lds, sm, c, b, box_id, status, pts, next_pts, n, [&](float vx, float vy) {
            const uint32_t kx = f2key(vx), ky = f2key(vy);
            if (mode0 != 0 && m0.in(kx)) atomicAdd(&sm.hist[0][m0.bucket(kx, vx)], 1u);
            if (mode1 != 0 && m1.in(ky)) atomicAdd(&sm.hist[1][m1.bucket(ky, vy)], 1u);
        });
        __syncthreads();
        if (wave < 2 && (wave == 0 ? mode0 : mode1) != 0) {
            // lane owns buckets 16*lane .. 16*lane+15; find the targets' buckets
            const uint4* hs = reinterpret_cast<const uint4*>(&sm.hist[wave][16 * lane]);
            uint32_t cnt[16];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint4 v = hs[q];
                cnt[4 * q] = v.x;
                cnt[4 * q + 1] = v.y;
                cnt[4 * q + 2] = v.z;
                cnt[4 * q + 3] = v.w;
            }
            uint32_t tot = 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) tot += cnt[j];
            const uint32_t incl = wave_incl_scan_u32(tot);
            const uint32_t excl = incl - tot;
            int bk[2];
            uint32_t rr[2], nb = 0;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const uint32_t k = sm.rank[wave][t];
                const bool mine = k >= excl && k < incl;
                // bucket j holds rank k when base_j <= k < base_j + cnt[j]
                int bin = 16 * lane;
                uint32_t base = excl, acc = excl, nbin = 0;
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const bool past = k >= acc + cnt[j];
                    acc += cnt[j];
                    if (past) {
                        bin = 16 * lane + j + 1;
                        base = acc;
                    }
                }
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    if (bin == 16 * lane + j) nbin = cnt[j];
                const int src = __ffsll((unsigned long long)__ballot(mine)) - 1;
                bk[t] = __builtin_amdgcn_readlane(bin, src);
                rr[t] = k - (uint32_t)__builtin_amdgcn_readlane((int)base, src);
                if (t == 0) nb = (uint32_t)__builtin_amdgcn_readlane((int)nbin, src);
            }
            if (lane == 0) {
                const BoxMap& m = wave == 0 ? m0 : m1;
                int md;
                if (m.lo == m.hi) {
                    md = 0;
                    sm.res[wave][0] = sm.res[wave][1] = m.lo;
                } else if (!m.lin && m.sh == 0) {
                    // key buckets one key wide: the buckets are the keys
                    md = 0;
                    sm.res[wave][0] = m.lo + (uint32_t)bk[0];
                    sm.res[wave][1] = m.lo + (uint32_t)bk[1];
                } else if (bk[0] != bk[1]) {
                    md = 1;
                } else if (nb <= (uint32_t)BOX_CAND) {
                    md = 2;
                } else {
                    md = 3;
                }
                sm.mode[wave] = md;
                sm.bkt[wave][0] = bk[0];
                sm.bkt[wave][1] = bk[1];
                sm.rank[wave][0] = rr[0];
                sm.rank[wave][1] = rr[1];
                sm.red[wave][0] = 0u;
                sm.red[wave][1] = 0xFFFFFFFFu;
                sm.red[wave][2] = 0xFFFFFFFFu;
                sm.red[wave][3] = 0u;
                sm.ncand[wave] = 0u;
            }
        }
        __syncthreads();
        // one pass for what each axis needs from its target buckets
        {
            const int md0 = sm.mode[0], md1 = sm.mode[1];
            const int b00 = sm.bkt[0][0], b01 = sm.bkt[0][1], b10 = sm.bkt[1][0], b11 = sm.bkt[1][1];
            uint32_t acc[2][4] = {{0u, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u}, {0u, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u}};
            auto take = [&](int a, int md, uint32_t k, float v, const BoxMap& m, int bA, int bB) {
                if (md == 0 || !m.in(k)) return;
                const int bu = m.bucket(k, v);
                if (md == 1) {
                    if (bu == bA) acc[a][0] = max(acc[a][0], k);
                    if (bu == bB) acc[a][1] = min(acc[a][1], k);
                } else if (bu == bA) {
                    if (md == 2) {
                        const uint32_t s = atomicAdd(&sm.ncand[a], 1u);
                        if (s < (uint32_t)BOX_CAND) sm.cand[a][s] = k;
                    } else {
                        acc[a][2] = min(acc[a][2], k);
                        acc[a][3] = max(acc[a][3], k);
                    }
                }
            };
            box_visit(in_lds, sm, c, b, box_id, status, pts, next_pts, n, [&](float vx, float vy) {
                take(0, md0, f2key(vx), vx, m0, b00, b01);
                take(1, md1, f2key(vy), vy, m1, b10, b11);
            });
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int md = a == 0 ? md0 : md1;
                if (md == 1) {
                    const uint32_t r0 = wave_max_u32(acc[a][0]), r1 = wave_min_u32(acc[a][1]);
                    if (lane == 0) {
                        atomicMax(&sm.red[a][0], r0);
                        atomicMin(&sm.red[a][1], r1);
                    }
                } else if (md == 3) {
                    const uint32_t r2 = wave_min_u32(acc[a][2]), r3 = wave_max_u32(acc[a][3]);
                    if (lane == 0) {
                        atomicMin(&sm.red[a][2], r2);
                        atomicMax(&sm.red[a][3], r3);
                    }
                }
            }
        }
        __syncthreads();
        // results, the next round's ranges, and a cleared histogram
        for (int e = tid; e < 2 * BOX_NB; e += BOX_THREADS) (&sm.hist[0][0])[e] = 0u;
        if (wave < 2) {
            const int a = wave, md = sm.mode[a];
            if (md == 1) {
                if (lane == 0) {
                    sm.res[a][0] = sm.red[a][0];
                    sm.res[a][1] = sm.red[a][1];
                    sm.mode[a] = 0;
                }
            } else if (md == 2) {
                // rank the shared bucket's keys (ties broken by slot)
                const uint32_t nc = min(sm.ncand[a], (uint32_t)BOX_CAND);
                const uint32_t kj = (uint32_t)lane < nc ? sm.cand[a][lane] : 0xFFFFFFFFu;
                uint32_t rk = 0;
                for (uint32_t i = 0; i < nc; ++i) {
                    const uint32_t ki = (uint32_t)__builtin_amdgcn_readlane((int)kj, (int)i);
                    rk += (ki < kj || (ki == kj && i < (uint32_t)lane)) ? 1u : 0u;
                }
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const bool hit = (uint32_t)lane < nc && rk == sm.rank[a][t];
                    const int src = __ffsll((unsigned long long)__ballot(hit)) - 1;
                    const uint32_t v = (uint32_t)__builtin_amdgcn_readlane((int)kj, src);
                    if (lane == 0) sm.res[a][t] = v;
                }
                if (lane == 0) sm.mode[a] = 0;
            } else if (md == 3) {
                if (lane == 0) {
                    sm.klo[a] = sm.red[a][2];
                    sm.khi[a] = sm.red[a][3];
                }
            }
        }
        __syncthreads();
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
    if (tid < 2) {
        sm.klo[tid] = 0xFFFFFFFFu;
        sm.khi[tid] = 0u;
    }
    for (int e = tid; e < 2 * BOX_NB; e += BOX_THREADS) (&sm.hist[0][0])[e] = 0u;
    __syncthreads();
    uint32_t kmin[2] = {0xFFFFFFFFu, 0xFFFFFFFFu}, kmax[2] = {0u, 0u};
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
        const int incl = (int)wave_incl_scan_u32((uint32_t)mine);
        const int wtot = __builtin_amdgcn_readlane(incl, 63);
        int off = 0;
        if (lane == 0 && wtot) off = atomicAdd(&sm.count, wtot);
        int k = __builtin_amdgcn_readlane(off, 0) + incl - mine;
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            if (id[j] == b && st[j] == 1u) {
                const float vx = pb[j].x - pa[j].x, vy = pb[j].y - pa[j].y;
                if (k >= 0 && k < BOX_CAP) {
                    sm.dx[k] = vx;
                    sm.dy[k] = vy;
                }
                ++k;
                const uint32_t kx = f2key(vx), ky = f2key(vy);
                kmin[0] = min(kmin[0], kx);
                kmax[0] = max(kmax[0], kx);
                kmin[1] = min(kmin[1], ky);
                kmax[1] = max(kmax[1], ky);
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const uint32_t lo = wave_min_u32(kmin[a]), hi = wave_max_u32(kmax[a]);
        if (lane == 0 && lo <= hi) {
            atomicMin(&sm.klo[a], lo);
            atomicMax(&sm.khi[a], hi);
        }
    }
    __syncthreads();
    const int c = sm.count;
    float mx = 0.0f, my = 0.0f;
    if (c > 0) {
        if (tid < 2) {
            sm.rank[tid][0] = (uint32_t)((c - 1) / 2);
            sm.rank[tid][1] = (uint32_t)(c / 2);
        }
        box_select(c <= BOX_CAP, sm, c, b, box_id, status, pts, next_pts, n);
        mx = 0.5f * (key2f(sm.res[0][0]) + key2f(sm.res[0][1]));
        my = 0.5f * (key2f(sm.res[1][0]) + key2f(sm.res[1][1]));
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
