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

// Selection state for NA axes (one selection of two ranks per axis).
template <int NA>
struct SelSmem {
    uint32_t hist[NA][BOX_NB];
    uint32_t klo[NA], khi[NA];  // per axis: key range holding both targets
    uint32_t rank[NA][2];       // the targets' ranks among the keys in that range
    int32_t bkt[NA][2];         // the targets' buckets this round
    int32_t mode[NA];           // 0 done, 1 two buckets, 2 rank candidates, 3 narrow
    uint32_t red[NA][4];        // max of bucket 0, min of bucket 1, min and max of bucket 0
    uint32_t ncand[NA];
    uint32_t cand[NA][BOX_CAND];
    uint32_t res[NA][2];        // selected keys
};

struct BoxSmem {
    float dx[BOX_CAP];
    float dy[BOX_CAP];
    SelSmem<2> sel;
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

// Keys at ranks sel.rank[a][0..1] of every axis a < NA of the elements that
// visit() presents (visit(f) calls f(v) with float v[NA] once per element, all
// threads of the workgroup taking part) into sel.res.  On entry sel.klo/khi
// hold each axis' smallest and largest key, sel.rank the two ranks and
// sel.hist is zero, all written before a barrier that precedes the call.
// The two ranks of an axis must be equal or adjacent (two targets in
// different buckets are taken as the largest key of the lower bucket and the
// smallest of the upper one).
// Every axis must hold at least one element, and visit() must present the
// same multiset with the same values on every call.  value_linear selects
// value-linear buckets for the first round (else key-linear).  Waves 0..NA-1 do the per-axis
// bookkeeping, so NA <= BOX_THREADS / 64.
template <int NA, class Visit>
__device__ __forceinline__ void select_ranks(SelSmem<NA>& sm, bool value_linear, Visit&& visit) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int round = 0; round < 8; ++round) {
        int mode[NA];
        bool any = false;
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            mode[a] = round == 0 ? 3 : sm.mode[a];
            any = any || mode[a] != 0;
        }
        if (!any) break;
        BoxMap mp[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) mp[a] = box_map(sm.klo[a], sm.khi[a], value_linear && round == 0);
        // runs of equal buckets are counted in registers and added once: a
        // tight cluster would otherwise serialise on one LDS address
        int cur[NA];
        uint32_t run[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            cur[a] = 0;
            run[a] = 0u;
        }
        visit([&](const float (&v)[NA]) {
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const uint32_t k = f2key(v[a]);
                if (mode[a] != 0 && mp[a].in(k)) {
                    const int bu = mp[a].bucket(k, v[a]);
                    if (bu != cur[a]) {
                        if (run[a]) atomicAdd(&sm.hist[a][cur[a]], run[a]);
                        cur[a] = bu;
                        run[a] = 0u;
                    }
                    ++run[a];
                }
            }
        });
#pragma unroll
        for (int a = 0; a < NA; ++a)
            if (run[a]) atomicAdd(&sm.hist[a][cur[a]], run[a]);
        __syncthreads();
        // per-wave copies by selection rather than by a dynamic index into
        // register arrays (which would spill them to scratch)
        int mw = 0;
        BoxMap mwp = mp[0];
#pragma unroll
        for (int a = 0; a < NA; ++a)
            if (wave == a) {
                mw = mode[a];
                mwp = mp[a];
            }
        if (wave < NA && mw != 0) {
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
                const BoxMap& m = mwp;
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
            int md[NA], bA[NA], bB[NA];
            uint32_t acc[NA][4];
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                md[a] = sm.mode[a];
                bA[a] = sm.bkt[a][0];
                bB[a] = sm.bkt[a][1];
                acc[a][0] = 0u;
                acc[a][1] = 0xFFFFFFFFu;
                acc[a][2] = 0xFFFFFFFFu;
                acc[a][3] = 0u;
            }
            visit([&](const float (&v)[NA]) {
#pragma unroll
                for (int a = 0; a < NA; ++a) {
                    const uint32_t k = f2key(v[a]);
                    if (md[a] == 0 || !mp[a].in(k)) continue;
                    const int bu = mp[a].bucket(k, v[a]);
                    if (md[a] == 1) {
                        if (bu == bA[a]) acc[a][0] = max(acc[a][0], k);
                        if (bu == bB[a]) acc[a][1] = min(acc[a][1], k);
                    } else if (bu == bA[a]) {
                        if (md[a] == 2) {
                            const uint32_t sl = atomicAdd(&sm.ncand[a], 1u);
                            if (sl < (uint32_t)BOX_CAND) sm.cand[a][sl] = k;
                        } else {
                            acc[a][2] = min(acc[a][2], k);
                            acc[a][3] = max(acc[a][3], k);
                        }
                    }
                }
            });
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                if (md[a] == 1) {
                    const uint32_t r0 = wave_max_u32(acc[a][0]), r1 = wave_min_u32(acc[a][1]);
                    if (lane == 0) {
                        atomicMax(&sm.red[a][0], r0);
                        atomicMin(&sm.red[a][1], r1);
                    }
                } else if (md[a] == 3) {
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
        for (int e = tid; e < NA * BOX_NB; e += BOX_THREADS) (&sm.hist[0][0])[e] = 0u;
        if (wave < NA) {
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

// Gather the points of box b with status 1: store(k, p, q) receives slot k
// (0 <= k < CAP; points beyond CAP are counted but not stored) with the
// point's position p in the first frame and q in the second, count receives
// the number of points, and sel.klo/khi the range of the displacement keys
// q - p per axis (sel.klo/khi initialised to the empty range and count to 0
// before a barrier that precedes the call).  16 consecutive ids and statuses
// per thread are in flight (vector loads when aligned); a wave-wide scan of
// the per-thread match counts and one LDS atomic per wave reserve the slots,
// so the slots' order is arbitrary.
template <int CAP, class Store>
__device__ __forceinline__ void box_gather(int b, const int32_t* __restrict__ box_id,
                                           const float* __restrict__ pts,
                                           const float* __restrict__ next_pts,
                                           const uint8_t* __restrict__ status, int n,
                                           int32_t& count, SelSmem<2>& sel, Store&& store) {
    const int tid = threadIdx.x, lane = tid & 63;
    uint32_t kmin[2] = {0xFFFFFFFFu, 0xFFFFFFFFu}, kmax[2] = {0u, 0u};
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
        int mine = 0;
#pragma unroll
        for (int j = 0; j < PT; ++j) mine += (id[j] == b && st[j] == 1u) ? 1 : 0;
        const int incl = (int)wave_incl_scan_u32((uint32_t)mine);
        const int wtot = __builtin_amdgcn_readlane(incl, 63);
        int off = 0;
        if (lane == 0 && wtot) off = atomicAdd(&count, wtot);
        int k = __builtin_amdgcn_readlane(off, 0) + incl - mine;
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            if (id[j] == b && st[j] == 1u) {
                if (k >= 0 && k < CAP) store(k, pa[j], pb[j]);
                ++k;
                const uint32_t kx = f2key(pb[j].x - pa[j].x), ky = f2key(pb[j].y - pa[j].y);
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
            atomicMin(&sel.klo[a], lo);
            atomicMax(&sel.khi[a], hi);
        }
    }
}

// Selection state set-up: empty key ranges and a zero histogram.
template <int NA>
__device__ __forceinline__ void sel_init(SelSmem<NA>& sel) {
    const int tid = threadIdx.x;
    if (tid < NA) {
        sel.klo[tid] = 0xFFFFFFFFu;
        sel.khi[tid] = 0u;
    }
    for (int e = tid; e < NA * BOX_NB; e += BOX_THREADS) (&sel.hist[0][0])[e] = 0u;
}

__device__ __forceinline__ void box_median(const float* __restrict__ boxes, int b,
                                           const int32_t* __restrict__ box_id,
                                           const float* __restrict__ pts,
                                           const float* __restrict__ next_pts,
                                           const uint8_t* __restrict__ status, int n,
                                           float* __restrict__ out_boxes,
                                           int32_t* __restrict__ out_count, BoxSmem& sm) {
    const int tid = threadIdx.x;
    if (tid == 0) sm.count = 0;
    sel_init(sm.sel);
    __syncthreads();
    box_gather<BOX_CAP>(b, box_id, pts, next_pts, status, n, sm.count, sm.sel,
                        [&](int k, float2 p, float2 q) {
                            sm.dx[k] = q.x - p.x;
                            sm.dy[k] = q.y - p.y;
                        });
    __syncthreads();
    const int c = sm.count;
    float mx = 0.0f, my = 0.0f;
    if (c > 0) {
        if (tid < 2) {
            sm.sel.rank[tid][0] = (uint32_t)((c - 1) / 2);
            sm.sel.rank[tid][1] = (uint32_t)(c / 2);
        }
        const bool in_lds = c <= BOX_CAP;
        select_ranks<2>(sm.sel, true, [&](auto&& f) {
            box_visit(in_lds, sm, c, b, box_id, status, pts, next_pts, n, [&](float vx, float vy) {
                const float v[2] = {vx, vy};
                f(v);
            });
        });
        mx = 0.5f * (key2f(sm.sel.res[0][0]) + key2f(sm.sel.res[0][1]));
        my = 0.5f * (key2f(sm.sel.res[1][0]) + key2f(sm.sel.res[1][1]));
    }
    if (tid == 0) {
        out_boxes[4 * b + 0] = boxes[4 * b + 0] + mx;
        out_boxes[4 * b + 1] = boxes[4 * b + 1] + my;
        out_boxes[4 * b + 2] = boxes[4 * b + 2] + mx;
        out_boxes[4 * b + 3] = boxes[4 * b + 3] + my;
        out_count[b] = c;
    }
}

// ---------------------------------------------------------------------------
// Median-Flow box update (Kalal, Mikolajczyk and Matas 2010): the box's
// centre moves by the component-wise median displacement of its tracked
// points and its half-extents scale by the median, over all unordered pairs
// of those points at distinct first-frame positions, of the ratio of the
// pair's distance in the second frame to its distance in the first.  Up to
// SCALE_CAP points per box are gathered.  The pair ratios are never stored:
// every pass walks the pairs, keyed by the squared ratio (monotone in the
// ratio), and the two middle squared ratios are square-rooted at the end.
// ---------------------------------------------------------------------------
constexpr int SCALE_BAND = 6144;    // keys around the median held for the final selection
constexpr int SCALE_SAMPLE = 4096;  // sampled pairs (in the band's storage, used first)
constexpr int SCALE_SHB_LOG2 = 14;  // buckets of the sample's histogram: 2^14
constexpr int SCALE_SHB = 1 << SCALE_SHB_LOG2;

struct ScaleSmem {
    float4 pu[SCALE_CAP];      // (x, y) in the first frame, (x, y) in the second
    uint32_t band[SCALE_BAND];  // sampled keys, then the keys of the band
    SelSmem<2> sel;            // displacement medians, the bracket
    SelSmem<1> rsel;           // ratio median
    int32_t count;
    uint32_t nsample;
};
static_assert(SCALE_SHB * sizeof(uint32_t) <= sizeof(float4) * SCALE_CAP, "sample histogram in the points' LDS");
static_assert(SCALE_SHB % BOX_THREADS == 0 && SCALE_SHB % 4 == 0, "sample histogram split over the threads");

// Key of the pair (a, e): the order-preserving key of the squared distance
// ratio; false when the squared first-frame distance is 0.  Every pass goes
// through this one function (explicit FMAs, the hardware reciprocal), so a
// pair gets the same key every time.
__device__ __forceinline__ bool pair_key(const float4& a, const float4& e, uint32_t& key) {
    const float ux = a.x - e.x, uy = a.y - e.y, vx = a.z - e.z, vy = a.w - e.w;
    const float du2 = __builtin_fmaf(ux, ux, uy * uy);
    const float dv2 = __builtin_fmaf(vx, vx, vy * vy);
    key = f2key(dv2 * __builtin_amdgcn_rcpf(du2));
    return du2 > 0.0f;
}

// A fixed bijective mixing of 32-bit integers (xor-shift and odd-multiply
// rounds), used to draw sample indices.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Slot for each active lane with pred set, reserved with one atomic per wave
// on *counter (LDS or global; lanes may be inactive; slots follow lane order).
__device__ __forceinline__ uint32_t wave_append(bool pred, uint32_t* counter) {
    const unsigned long long m = __ballot(pred);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    const int leader = __ffsll(__ballot(1)) - 1;
    uint32_t base = 0u;
    if ((int)(threadIdx.x & 63) == leader && m) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
    return base + below;
}

// Pair q of the c * floor((c-1)/2) + (c even ? c/2 : 0) unordered pairs is
// (i, (i + d) mod c) with i = q mod c and d = q / c + 1: every circular
// distance d below c/2 pairs all c points, and for even c the distance c/2
// pairs only the first half.  The sample draws pairs through this numbering.
__device__ __forceinline__ uint32_t pair_total(int c) {
    const uint32_t uc = (uint32_t)c;
    return uc * ((uc - 1u) / 2u) + ((uc & 1u) ? 0u : uc / 2u);
}

// The passes walk the same pairs as items that share their first point: item
// t < G*c (G = ceil(floor((c-1)/2) / PAIR_K)) is point i = t mod c with the
// distances 1 + PAIR_K*g .. PAIR_K*(g+1) below c/2, g = t / c (the last
// group may hold fewer); for even c, item G*c + i (i < c/2) is the pair
// (i, i + c/2).  One load of point i serves PAIR_K pairs.
constexpr uint32_t PAIR_K = 4;

__device__ __forceinline__ uint32_t pair_items(int c) {
    if (c < 2) return 0u;
    const uint32_t uc = (uint32_t)c, df = (uc - 1u) / 2u;
    return ((df + PAIR_K - 1u) / PAIR_K) * uc + ((uc & 1u) ? 0u : uc / 2u);
}

// Visit every unordered pair {i, j} of the c gathered points in the items
// [t0, t1) once as f(key, ok), key that of the squared distance ratio
// (pair_key) and ok false for a pair whose squared first-frame distance is
// zero (its key is then meaningless and the pair is skipped).  The callback
// runs for every pair so that it can be branch-free.  Each thread steps its
// item by BOX_THREADS with an incremental (g, i) update.
template <class F>
__device__ __forceinline__ void visit_pairs_range(const float4* __restrict__ pu, int c, uint32_t t0,
                                                  uint32_t t1, F&& f) {
    if (c < 2) return;
    const uint32_t uc = (uint32_t)c, df = (uc - 1u) / 2u;
    const uint32_t gc = ((df + PAIR_K - 1u) / PAIR_K) * uc, half = uc / 2u;
    uint32_t t = t0 + threadIdx.x;
    if (t >= t1) return;
    uint32_t g = t / uc, i = t - g * uc;
    const uint32_t sg = (uint32_t)BOX_THREADS / uc, si = (uint32_t)BOX_THREADS - sg * uc;
    for (; t < t1; t += BOX_THREADS) {
        if (t < gc) {
            const float4 a = pu[i];
            const uint32_t d0 = g * PAIR_K;
            uint32_t j = i + d0 + 1u;
            if (j >= uc) j -= uc;
#pragma unroll
            for (uint32_t k = 0; k < PAIR_K; ++k) {
                if (d0 + k < df) {
                    uint32_t key;
                    const bool ok = pair_key(a, pu[j], key);
                    f(key, ok);
                }
                ++j;
                if (j >= uc) j -= uc;
            }
        } else {
            const uint32_t ih = t - gc;  // < c/2, even c only
            uint32_t key;
            const bool ok = pair_key(pu[ih], pu[ih + half], key);
            f(key, ok);
        }
        i += si;
        g += sg;
        if (i >= uc) {
            i -= uc;
            ++g;
        }
    }
}

template <class F>
__device__ __forceinline__ void visit_pairs(const float4* __restrict__ pu, int c, F&& f) {
    visit_pairs_range(pu, c, 0u, pair_items(c), f);
}

// ---------------------------------------------------------------------------
// The scaled update runs in four launches so that the pair passes of one box
// spread over many compute units (a box of 5000 points has 12.5 M pairs):
//   prep   (two workgroups per box): gather; one selects the displacement
//          medians, the other draws the sample bracket [A, B] and writes the
//          points, the state and a zero histogram to the box's workspace;
//   hist   (S workgroups per box, each a slice of the pair walk): pass one,
//          counts and the histogram of [A, B], merged with global atomics;
//   band   (S per box): each workgroup reads the merged histogram, finds the
//          bucket(s) of both middle ranks and appends its slice's keys there;
//   final  (one per box): the exact selection on the band (or, if a middle
//          rank fell outside [A, B] or the band overflowed, on all pairs),
//          then the box.
// ---------------------------------------------------------------------------
struct ScaleState {
    int32_t c;            // kept points; 0 or > SCALE_CAP: the box is done after prep
    uint32_t A, B;        // bracket keys
    uint32_t nsample;     // valid sampled pairs (0: no bracket)
    float mx, my;         // displacement medians
    uint32_t npairs, nbelow, nabove, kmin, kmax;  // pass one
    uint32_t nband;       // pass two
    uint32_t pad[4];
};
struct ScaleWs {
    ScaleState st;
    uint32_t hist[BOX_NB];
    uint32_t band[SCALE_BAND];
    float4 pu[SCALE_CAP];
};

__device__ __forceinline__ int bracket_shift(uint32_t A, uint32_t B) {
    const uint32_t span = B - A;
    return max(0, (span == 0u ? 0 : 32 - __clz((int)span)) - 10);
}

__device__ __forceinline__ void scaled_write(const float* __restrict__ boxes, int b, int c, float mx,
                                             float my, float s, float* __restrict__ out_boxes,
                                             int32_t* __restrict__ out_count,
                                             float* __restrict__ out_scale) {
    const float x0 = boxes[4 * b + 0], y0 = boxes[4 * b + 1], x1 = boxes[4 * b + 2], y1 = boxes[4 * b + 3];
    if (c > 0) {
        const float cx = 0.5f * (x0 + x1) + mx, cy = 0.5f * (y0 + y1) + my;
        const float hw = 0.5f * (x1 - x0), hh = 0.5f * (y1 - y0);
        out_boxes[4 * b + 0] = cx - s * hw;
        out_boxes[4 * b + 1] = cy - s * hh;
        out_boxes[4 * b + 2] = cx + s * hw;
        out_boxes[4 * b + 3] = cy + s * hh;
    } else {
        out_boxes[4 * b + 0] = x0;
        out_boxes[4 * b + 1] = y0;
        out_boxes[4 * b + 2] = x1;
        out_boxes[4 * b + 3] = y1;
    }
    out_count[b] = c;
    out_scale[b] = s;
}

// Zero the sample histogram (SCALE_SHB buckets in LDS).
__device__ __forceinline__ void shist_zero(uint32_t* hs) {
    for (int e = threadIdx.x; e < SCALE_SHB / 4; e += BOX_THREADS)
        reinterpret_cast<uint4*>(hs)[e] = make_uint4(0u, 0u, 0u, 0u);
}

// The buckets of ranks r0 and r1 (both below the histogram's total) in the
// SCALE_SHB-bucket histogram hs: out[t] = {bucket, keys before it, keys in
// it}.  Thread i owns buckets PER*i .. PER*i+PER-1; wtot holds the waves'
// totals.  All threads call; out is valid after the closing barrier.
template <class Out>
__device__ __forceinline__ void shist_find(const uint32_t* hs, uint32_t r0, uint32_t r1,
                                           uint32_t* wtot, Out& out) {
    constexpr int PER = SCALE_SHB / BOX_THREADS;
    const int tid = threadIdx.x, lane = tid & 63;
    uint32_t cnt[PER];
    uint32_t tot = 0u;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        cnt[j] = hs[PER * tid + j];
        tot += cnt[j];
    }
    const uint32_t incl = wave_incl_scan_u32(tot);
    if (lane == 63) wtot[tid >> 6] = incl;
    __syncthreads();
    uint32_t base = 0u;
    for (int w = 0; w < (tid >> 6); ++w) base += wtot[w];
    const uint32_t excl = base + incl - tot;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const uint32_t r = t == 0 ? r0 : r1;
        if (r >= excl && r < excl + tot) {
            uint32_t acc = excl, before = excl, in = cnt[0];
            int bk = PER * tid;
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                if (r >= acc + cnt[j]) {
                    bk = PER * tid + j + 1;
                    before = acc + cnt[j];
                    in = j + 1 < PER ? cnt[j + 1] : 0u;
                }
                acc += cnt[j];
            }
            out[t][0] = (uint32_t)bk;
            out[t][1] = before;
            out[t][2] = in;
        }
    }
    __syncthreads();
}

// Phase 1, two workgroups per box that both gather the box's points.  Role 0
// keeps the points and draws the sample: at most SCALE_SAMPLE pairs drawn by
// a hashed index (neighbouring pairs of the walk share their points, so an
// evenly strided sample is far from random); A and B are its quantiles 14
// standard deviations of the sample median's rank either side of the median.
// Role 1 selects the displacement medians at the same time.
__device__ __forceinline__ void scaled_prep(const float* __restrict__ boxes, int b, int role,
                                            const int32_t* __restrict__ box_id,
                                            const float* __restrict__ pts,
                                            const float* __restrict__ next_pts,
                                            const uint8_t* __restrict__ status, int n,
                                            float* __restrict__ out_boxes,
                                            int32_t* __restrict__ out_count,
                                            float* __restrict__ out_scale, ScaleWs* __restrict__ ws,
                                            ScaleSmem& sm) {
    const int tid = threadIdx.x, lane = tid & 63;
    if (tid == 0) {
        sm.count = 0;
        sm.nsample = 0u;
    }
    sel_init(sm.sel);
    __syncthreads();
    box_gather<SCALE_CAP>(b, box_id, pts, next_pts, status, n, sm.count, sm.sel,
                          [&](int k, float2 p, float2 q) { sm.pu[k] = make_float4(p.x, p.y, q.x, q.y); });
    __syncthreads();
    const int c = sm.count;
    ScaleState& st = ws->st;
    if (role == 1) {
        if (c > SCALE_CAP || c == 0) return;
        if (tid < 2) {
            sm.sel.rank[tid][0] = (uint32_t)((c - 1) / 2);
            sm.sel.rank[tid][1] = (uint32_t)(c / 2);
        }
        select_ranks<2>(sm.sel, true, [&](auto&& f) {
            for (int i = tid; i < c; i += BOX_THREADS) {
                const float4 p = sm.pu[i];
                const float v[2] = {p.z - p.x, p.w - p.y};
                f(v);
            }
        });
        if (tid == 0) {
            st.mx = 0.5f * (key2f(sm.sel.res[0][0]) + key2f(sm.sel.res[0][1]));
            st.my = 0.5f * (key2f(sm.sel.res[1][0]) + key2f(sm.sel.res[1][1]));
        }
        return;
    }
    for (int e = tid; e < BOX_NB; e += BOX_THREADS) ws->hist[e] = 0u;
    if (c > SCALE_CAP || c == 0) {
        // too many points for the pair passes (no result), or none
        if (tid == 0) {
            st.c = c;
            if (c == 0) {
                scaled_write(boxes, b, 0, 0.0f, 0.0f, 1.0f, out_boxes, out_count, out_scale);
            } else {
                const float nan = __builtin_nanf("");
                for (int k = 0; k < 4; ++k) out_boxes[4 * b + k] = nan;
                out_count[b] = c;
                out_scale[b] = nan;
            }
        }
        return;
    }
    for (int i = tid; i < c; i += BOX_THREADS) ws->pu[i] = sm.pu[i];
    const uint32_t uc = (uint32_t)c, total = pair_total(c);
    const uint32_t ns = min(total, (uint32_t)SCALE_SAMPLE);
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    for (uint32_t t = tid; t < ns; t += BOX_THREADS) {
        const uint32_t q = (uint32_t)(((uint64_t)mix32(t) * total) >> 32), d = q / uc, i = q - d * uc;
        uint32_t j = i + d + 1u;
        if (j >= uc) j -= uc;
        uint32_t key;
        const bool ok = pair_key(sm.pu[i], sm.pu[j], key);
        const uint32_t slot = wave_append(ok, &sm.nsample);
        if (ok) {
            sm.band[slot] = key;
            lo = min(lo, key);
            hi = max(hi, key);
        }
    }
    lo = wave_min_u32(lo);
    hi = wave_max_u32(hi);
    // The bracket only has to contain the two sample quantiles (any A <= B
    // gives the exact result; a wider one only widens the band), so two
    // histogram rounds of the sample replace an exact selection: round one
    // over the sample's key range in SCALE_SHB key-linear buckets, round two
    // over the two buckets that hold the quantiles, SCALE_SHB / 2 finer
    // buckets each.  A is the lower edge of the lower quantile's final
    // bucket, B the upper edge of the upper one's.  The gathered points are
    // no longer needed in LDS (they are in the workspace), so the histogram
    // takes their place.
    if (tid == 0) {
        sm.sel.klo[0] = 0xFFFFFFFFu;
        sm.sel.khi[0] = 0u;
    }
    __syncthreads();
    uint32_t* hs = reinterpret_cast<uint32_t*>(sm.pu);
    shist_zero(hs);
    if (lane == 0 && lo <= hi) {
        atomicMin(&sm.sel.klo[0], lo);
        atomicMax(&sm.sel.khi[0], hi);
    }
    __syncthreads();
    const uint32_t msmp = sm.nsample;
    uint32_t A = 0u, B = 0xFFFFFFFFu;
    if (msmp > 0u) {
        const uint32_t klo = sm.sel.klo[0], khi = sm.sel.khi[0];
        const uint32_t span = khi - klo;
        const int sh = max(0, (span == 0u ? 0 : 32 - __clz((int)span)) - SCALE_SHB_LOG2);
        for (uint32_t t = tid; t < msmp; t += BOX_THREADS) atomicAdd(&hs[(sm.band[t] - klo) >> sh], 1u);
        __syncthreads();
        const uint32_t h = 2u + (uint32_t)ceilf(7.0f * sqrtf((float)msmp));
        const uint32_t rc = (msmp - 1u) / 2u;
        const uint32_t r0 = rc > h ? rc - h : 0u, r1 = min(msmp - 1u, msmp / 2u + h);
        shist_find(hs, r0, r1, sm.sel.hist[0], sm.sel.red);
        const uint32_t bk0 = sm.sel.red[0][0], base0 = sm.sel.red[0][1], n0 = sm.sel.red[0][2];
        const uint32_t bk1 = sm.sel.red[1][0], base1 = sm.sel.red[1][1];
        const uint32_t lo0 = klo + (bk0 << sh), lo1 = klo + (bk1 << sh);
        uint32_t s0 = 0u, s1 = 0u;
        int sh2 = 0;
        if (sh > 0) {
            sh2 = max(0, sh - (SCALE_SHB_LOG2 - 1));
            __syncthreads();  // every thread has read round one's result
            shist_zero(hs);
            __syncthreads();
            for (uint32_t t = tid; t < msmp; t += BOX_THREADS) {
                const uint32_t key = sm.band[t], bk = (key - klo) >> sh;
                if (bk == bk0) atomicAdd(&hs[(key - lo0) >> sh2], 1u);
                if (bk == bk1) atomicAdd(&hs[SCALE_SHB / 2 + ((key - lo1) >> sh2)], 1u);
            }
            __syncthreads();
            shist_find(hs, r0 - base0, n0 + (r1 - base1), sm.sel.hist[0], sm.sel.red);
            s0 = sm.sel.red[0][0];
            s1 = sm.sel.red[1][0] - (uint32_t)(SCALE_SHB / 2);
        }
        A = lo0 + (s0 << sh2);
        const uint64_t b1 = (uint64_t)lo1 + ((uint64_t)(s1 + 1u) << sh2) - 1u;
        B = (uint32_t)min(b1, (uint64_t)khi);
    }
    if (tid == 0) {
        st.c = c;
        st.A = A;
        st.B = B;
        st.nsample = msmp;
        st.npairs = st.nbelow = st.nabove = st.nband = 0u;
        st.kmin = 0xFFFFFFFFu;
        st.kmax = 0u;
    }
}

// Loads the box's points into LDS (c <= SCALE_CAP).
__device__ __forceinline__ void load_points(const ScaleWs* __restrict__ ws, int c, float4* pu) {
    for (int i = threadIdx.x; i < c; i += BOX_THREADS) pu[i] = ws->pu[i];
    __syncthreads();
}

__device__ __forceinline__ void slice_range(int c, int slice, int S, uint32_t& q0, uint32_t& q1) {
    const uint64_t total = pair_items(c);
    q0 = (uint32_t)(total * (uint64_t)slice / (uint64_t)S);
    q1 = (uint32_t)(total * (uint64_t)(slice + 1) / (uint64_t)S);
}

struct SliceSmem {
    float4 pu[SCALE_CAP];
    uint32_t hist[BOX_NB];
    uint32_t dec[8];   // the band decision: inside, klo, khi
    uint32_t stat[5];  // the slice's pairs, below, above, smallest and largest key
};

// Phase 2: pass one over a slice of the pairs.
__device__ __forceinline__ void scaled_hist(ScaleWs* __restrict__ ws, int slice, int S, SliceSmem& sm) {
    const int tid = threadIdx.x, lane = tid & 63;
    ScaleState& st = ws->st;
    const int c = st.c;
    if (c <= 0 || c > SCALE_CAP) return;
    const uint32_t A = st.A, B = st.B;
    const int sh = bracket_shift(A, B);
    for (int e = tid; e < BOX_NB; e += BOX_THREADS) sm.hist[e] = 0u;
    if (tid == 0) {
        sm.stat[0] = sm.stat[1] = sm.stat[2] = sm.stat[4] = 0u;
        sm.stat[3] = 0xFFFFFFFFu;
    }
    load_points(ws, c, sm.pu);
    uint32_t q0, q1;
    slice_range(c, slice, S, q0, q1);
    uint32_t np = 0u, nbelow = 0u, nabove = 0u, lo = 0xFFFFFFFFu, hi = 0u, run = 0u;
    int cur = 0;
    visit_pairs_range(sm.pu, c, q0, q1, [&](uint32_t key, bool ok) {
        // selects instead of branches; runs of equal buckets are added once
        np += ok ? 1u : 0u;
        lo = ok ? min(lo, key) : lo;
        hi = ok ? max(hi, key) : hi;
        const bool below = ok && key < A, above = ok && key > B;
        nbelow += below ? 1u : 0u;
        nabove += above ? 1u : 0u;
        const bool in = ok && !below && !above;
        const int bu = (int)((key - A) >> sh);
        const bool fresh = in && bu != cur;
        if (fresh && run) atomicAdd(&sm.hist[cur], run);
        cur = fresh ? bu : cur;
        run = fresh ? 1u : run + (in ? 1u : 0u);
    });
    if (run) atomicAdd(&sm.hist[cur], run);
    lo = wave_min_u32(lo);
    hi = wave_max_u32(hi);
    np = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan_u32(np), 63);
    nbelow = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan_u32(nbelow), 63);
    nabove = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan_u32(nabove), 63);
    // the waves' counts meet in LDS; the workgroup adds them to the box once
    if (lane == 0 && np > 0u) {
        atomicAdd(&sm.stat[0], np);
        atomicAdd(&sm.stat[1], nbelow);
        atomicAdd(&sm.stat[2], nabove);
        atomicMin(&sm.stat[3], lo);
        atomicMax(&sm.stat[4], hi);
    }
    __syncthreads();
    if (tid == 0 && sm.stat[0] > 0u) {
        atomicAdd(&st.npairs, sm.stat[0]);
        atomicAdd(&st.nbelow, sm.stat[1]);
        atomicAdd(&st.nabove, sm.stat[2]);
        atomicMin(&st.kmin, sm.stat[3]);
        atomicMax(&st.kmax, sm.stat[4]);
    }
    for (int e = tid; e < BOX_NB; e += BOX_THREADS) {
        const uint32_t v = sm.hist[e];
        if (v) atomicAdd(&ws->hist[e], v);
    }
}

// The bucket(s) of both middle ranks among the keys in [A, B], by wave 0:
// dec = {inside, first key, last key of those buckets, keys below them}.
__device__ __forceinline__ void scaled_decide(const ScaleWs* __restrict__ ws, uint32_t* dec) {
    const int tid = threadIdx.x, lane = tid & 63;
    const ScaleState& st = ws->st;
    const uint32_t npairs = st.npairs, below = st.nbelow, above = st.nabove;
    const uint32_t A = st.A, B = st.B;
    const int sh = bracket_shift(A, B);
    const uint32_t t0 = npairs > 0u ? (npairs - 1u) / 2u : 0u, t1 = npairs / 2u;
    const bool inside = npairs > 0u && st.nsample > 0u && below <= t0 && t1 < npairs - above;
    if (tid < 64) {
        if (!inside) {
            if (lane == 0) dec[0] = 0u;
        } else {
            uint32_t cnt[16];
            uint32_t tot = 0u;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                cnt[j] = ws->hist[16 * lane + j];
                tot += cnt[j];
            }
            const uint32_t incl = wave_incl_scan_u32(tot), excl = incl - tot;
            int bk[2];
            uint32_t base0 = 0u;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const uint32_t k = (t == 0 ? t0 : t1) - below;
                const bool mine = k >= excl && k < incl;
                int bin = 16 * lane;
                uint32_t acc = excl, bse = excl;
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    if (k >= acc + cnt[j]) {
                        bin = 16 * lane + j + 1;
                        bse = acc + cnt[j];
                    }
                    acc += cnt[j];
                }
                const int src = __ffsll((unsigned long long)__ballot(mine)) - 1;
                bk[t] = __builtin_amdgcn_readlane(bin, src);
                if (t == 0) base0 = (uint32_t)__builtin_amdgcn_readlane((int)bse, src);
            }
            if (lane == 0) {
                const uint64_t khi64 = (uint64_t)A + ((uint64_t)(bk[1] + 1) << sh) - 1u;
                dec[0] = 1u;
                dec[1] = A + ((uint32_t)bk[0] << sh);
                dec[2] = (uint32_t)min(khi64, (uint64_t)B);
                dec[3] = below + base0;
            }
        }
    }
    __syncthreads();
}

// Phase 3: pass two over a slice: the keys of the target buckets.
__device__ __forceinline__ void scaled_band(ScaleWs* __restrict__ ws, int slice, int S, SliceSmem& sm) {
    ScaleState& st = ws->st;
    const int c = st.c;
    if (c <= 0 || c > SCALE_CAP) return;
    scaled_decide(ws, sm.dec);
    if (sm.dec[0] == 0u) return;
    const uint32_t bl = sm.dec[1], bh = sm.dec[2];
    load_points(ws, c, sm.pu);
    uint32_t q0, q1;
    slice_range(c, slice, S, q0, q1);
    visit_pairs_range(sm.pu, c, q0, q1, [&](uint32_t key, bool ok) {
        const bool in = ok && key >= bl && key <= bh;
        if (__ballot(in)) {  // band keys are rare: most waves skip the append
            const uint32_t slot = wave_append(in, &st.nband);
            if (in && slot < (uint32_t)SCALE_BAND) ws->band[slot] = key;
        }
    });
}

// Phase 4: the ratio median and the box.
__device__ __forceinline__ void scaled_final(const float* __restrict__ boxes, int b,
                                             float* __restrict__ out_boxes,
                                             int32_t* __restrict__ out_count,
                                             float* __restrict__ out_scale,
                                             const ScaleWs* __restrict__ ws, ScaleSmem& sm) {
    const int tid = threadIdx.x;
    const ScaleState& st = ws->st;
    const int c = st.c;
    if (c <= 0 || c > SCALE_CAP) return;
    const uint32_t npairs = st.npairs;
    float s = 1.0f;
    if (npairs > 0u) {
        sel_init(sm.rsel);
        uint32_t* dec = reinterpret_cast<uint32_t*>(&sm.sel.res[0][0]);
        scaled_decide(ws, dec);
        const uint32_t t0 = (npairs - 1u) / 2u, t1 = npairs / 2u;
        const uint32_t nband = st.nband;
        const bool fast = dec[0] != 0u && nband <= (uint32_t)SCALE_BAND;
        if (tid == 0) {
            if (fast) {
                sm.rsel.klo[0] = dec[1];
                sm.rsel.khi[0] = dec[2];
                sm.rsel.rank[0][0] = t0 - dec[3];
                sm.rsel.rank[0][1] = t1 - dec[3];
            } else {
                sm.rsel.klo[0] = st.kmin;
                sm.rsel.khi[0] = st.kmax;
                sm.rsel.rank[0][0] = t0;
                sm.rsel.rank[0][1] = t1;
            }
        }
        // key-linear first rounds: ratio outliers would squeeze the bulk
        // into a few value-linear buckets
        if (fast) {
            for (uint32_t t = tid; t < nband; t += BOX_THREADS) sm.band[t] = ws->band[t];
            __syncthreads();
            select_ranks<1>(sm.rsel, false, [&](auto&& f) {
                for (uint32_t t = tid; t < nband; t += BOX_THREADS) {
                    const float v[1] = {key2f(sm.band[t])};
                    f(v);
                }
            });
        } else {
            load_points(ws, c, sm.pu);
            select_ranks<1>(sm.rsel, false, [&](auto&& f) {
                visit_pairs(sm.pu, c, [&](uint32_t key, bool ok) {
                    if (ok) {
                        const float v[1] = {key2f(key)};
                        f(v);
                    }
                });
            });
        }
        s = 0.5f * (__builtin_sqrtf(key2f(sm.rsel.res[0][0])) + __builtin_sqrtf(key2f(sm.rsel.res[0][1])));
    }
    if (tid == 0) scaled_write(boxes, b, c, st.mx, st.my, s, out_boxes, out_count, out_scale);
}

// Forward-backward gate (Kalal et al. 2010): a point keeps status 1 when it
// was tracked forward and back and lands within fb_max of where it started.
// The gate of one point from its start p, its backward result q and the two
// statuses: the forward-backward error e (-1 unless both passes tracked it)
// and whether it is kept.
__device__ __forceinline__ void fb_gate_value(float2 p, float2 q, unsigned sf, unsigned sb,
                                              float fb_max, float& e, uint8_t& st) {
    e = -1.0f;
    st = 0;
    if (sf == 1 && sb == 1) {
        const float ex = p.x - q.x, ey = p.y - q.y;
        e = __builtin_sqrtf(__builtin_fmaf(ex, ex, ey * ey));
        st = e <= fb_max ? 1 : 0;
    }
}

__device__ __forceinline__ void fb_gate_point(const float* __restrict__ pts,
                                              const float* __restrict__ back_pts,
                                              const uint8_t* __restrict__ st_fwd,
                                              const uint8_t* __restrict__ st_bwd, int i,
                                              float fb_max, float* __restrict__ fb_err,
                                              uint8_t* __restrict__ status_out) {
    const float2 p = reinterpret_cast<const float2*>(pts)[i];
    const float2 q = reinterpret_cast<const float2*>(back_pts)[i];
    float e;
    uint8_t st;
    fb_gate_value(p, q, st_fwd[i], st_bwd[i], fb_max, e, st);
    if (fb_err) fb_err[i] = e;
    status_out[i] = st;
}

}  // namespace ot
