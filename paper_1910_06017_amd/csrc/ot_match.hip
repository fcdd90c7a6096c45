// ot_match.hip -- matching and update phases (Sec. V-A): the IoU score matrix
// of predicted scene objects against detections on the GPU, the globally
// optimal assignment (Kuhn 1955) and the track update on the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <limits>
#include <vector>

#include "omnitrack.h"

namespace ot {

constexpr int IOU_THREADS = 256;

// IoU of one (object, detection) pair per thread; pairs laid out row-major
// (object-major), so a wave covers consecutive detections of one object.
__global__ __launch_bounds__(IOU_THREADS) void k_iou(const float4* __restrict__ S, int m,
                                                     const float4* __restrict__ D, int k,
                                                     const uint8_t* __restrict__ active,
                                                     float* __restrict__ out) {
    const long long t = (long long)blockIdx.x * IOU_THREADS + threadIdx.x;
    if (t >= (long long)m * k) return;
    const int i = (int)(t / k), j = (int)(t - (long long)i * k);
    float r = 0.0f;
    if (!active || active[i]) {
        const float4 a = S[i], b = D[j];
        const float ix = fmaxf(0.0f, fminf(a.z, b.z) - fmaxf(a.x, b.x));
        const float iy = fmaxf(0.0f, fminf(a.w, b.w) - fmaxf(a.y, b.y));
        const float inter = ix * iy;
        const float aa = fmaxf(0.0f, a.z - a.x) * fmaxf(0.0f, a.w - a.y);
        const float ab = fmaxf(0.0f, b.z - b.x) * fmaxf(0.0f, b.w - b.y);
        const float uni = aa + ab - inter;
        r = uni > 0.0f ? inter / uni : 0.0f;
    }
    out[t] = r;
}

// Maximum-gain assignment of the rows of an n x w gain matrix (n <= w) to
// distinct columns, every row assigned: shortest augmenting paths over
// reduced costs c(i, j) - u(i) - v(j) >= 0 with c = -gain (Kuhn-Munkres with
// dual potentials).  Rows are added one at a time; each addition grows a tree
// of tight edges from the new row with Dijkstra-like label updates until it
// reaches a free column, then flips the path.  O(n^2 w).
static void assign_rows(const std::vector<double>& gain, int n, int w, std::vector<int>& row_col) {
    const double INF = std::numeric_limits<double>::infinity();
    // column 0 is a virtual root; col_row[c] = row owning column c (1-based), 0 = free
    std::vector<double> u(n + 1, 0.0), v(w + 1, 0.0), dist(w + 1);
    std::vector<int> col_row(w + 1, 0), prev_col(w + 1, 0);
    std::vector<char> done(w + 1);
    auto cost = [&](int r, int c) { return -gain[(size_t)(r - 1) * w + (c - 1)]; };
    for (int r = 1; r <= n; ++r) {
        col_row[0] = r;
        int c0 = 0;
        std::fill(dist.begin(), dist.end(), INF);
        std::fill(done.begin(), done.end(), 0);
        while (true) {
            done[c0] = 1;
            const int r0 = col_row[c0];
            double step = INF;
            int c_next = -1;
            for (int c = 1; c <= w; ++c) {
                if (done[c]) continue;
                const double red = cost(r0, c) - u[r0] - v[c];
                if (red < dist[c]) {
                    dist[c] = red;
                    prev_col[c] = c0;
                }
                if (dist[c] < step) {
                    step = dist[c];
                    c_next = c;
                }
            }
            for (int c = 0; c <= w; ++c) {
                if (done[c]) {
                    u[col_row[c]] += step;
                    v[c] -= step;
                } else {
                    dist[c] -= step;
                }
            }
            c0 = c_next;
            if (col_row[c0] == 0) break;  // reached a free column
        }
        // flip the alternating path back to the root
        while (c0 != 0) {
            const int cp = prev_col[c0];
            col_row[c0] = col_row[cp];
            c0 = cp;
        }
    }
    row_col.assign(n, -1);
    for (int c = 1; c <= w; ++c)
        if (col_row[c] > 0) row_col[col_row[c] - 1] = c - 1;
}

}  // namespace ot

using namespace ot;

extern "C" {

ot_err ot_iou_matrix(const float* S, int32_t m, const float* D, int32_t k, const uint8_t* active,
                     float* iou, void* stream) {
    if (m < 0 || k < 0) return OT_E_INVAL;
    if (m == 0 || k == 0) return OT_OK;
    if (!S || !D || !iou) return OT_E_INVAL;
    if (((uintptr_t)S | (uintptr_t)D) & 15) return OT_E_INVAL;
    if ((uintptr_t)iou & 3) return OT_E_INVAL;
    const long long total = (long long)m * k;
    if (total > (long long)INT32_MAX * IOU_THREADS / 2) return OT_E_INVAL;
    const int grid = (int)((total + IOU_THREADS - 1) / IOU_THREADS);
    hipLaunchKernelGGL(k_iou, dim3(grid), dim3(IOU_THREADS), 0, static_cast<hipStream_t>(stream),
                       reinterpret_cast<const float4*>(S), m, reinterpret_cast<const float4*>(D), k,
                       active, iou);
    return hipGetLastError() == hipSuccess ? OT_OK : OT_E_LAUNCH;
}

ot_err ot_assign(const float* iou, int32_t m, int32_t k, float iou_min, int32_t* s2d, int32_t* d2s,
                 double* score) {
    if (m < 0 || k < 0 || !(iou_min > 0.0f && iou_min <= 1.0f)) return OT_E_INVAL;
    if ((m > 0 && !s2d) || (k > 0 && !d2s) || (m > 0 && k > 0 && !iou)) return OT_E_INVAL;
    if ((long long)m * k > (1LL << 26)) return OT_E_INVAL;
    for (int i = 0; i < m; ++i) s2d[i] = -1;
    for (int j = 0; j < k; ++j) d2s[j] = -1;
    double tot = 0.0;
    if (m > 0 && k > 0) {
        // gain of a pair below the threshold is 0: assigning it is worth
        // exactly as much as leaving both unmatched, and it is dropped below
        const bool tr = m > k;  // rows must be the smaller side
        const int n = tr ? k : m, w = tr ? m : k;
        std::vector<double> gain((size_t)n * w);
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < w; ++c) {
                const float g = tr ? iou[(size_t)c * k + r] : iou[(size_t)r * k + c];
                gain[(size_t)r * w + c] = g >= iou_min ? (double)g : 0.0;
            }
        std::vector<int> row_col;
        assign_rows(gain, n, w, row_col);
        for (int r = 0; r < n; ++r) {
            const int c = row_col[r];
            if (c < 0 || gain[(size_t)r * w + c] <= 0.0) continue;
            const int i = tr ? c : r, j = tr ? r : c;
            s2d[i] = j;
            d2s[j] = i;
            tot += (double)iou[(size_t)i * k + j];
        }
    }
    if (score) *score = tot;
    return OT_OK;
}

ot_err ot_track_update(float* boxes, int32_t* ids, uint8_t* lost, int32_t m, int32_t cap,
                       const float* det, int32_t k, const int32_t* s2d, const int32_t* d2s,
                       int32_t* next_id, int32_t* m_out) {
    if (m < 0 || k < 0 || cap < m || !next_id || !m_out) return OT_E_INVAL;
    if (cap > 0 && (!boxes || !ids || !lost)) return OT_E_INVAL;
    if ((m > 0 && !s2d) || (k > 0 && (!det || !d2s))) return OT_E_INVAL;
    int fresh = 0;
    for (int i = 0; i < m; ++i) {
        const int j = s2d[i];
        if (j < -1 || j >= k || (j >= 0 && d2s[j] != i)) return OT_E_INVAL;
    }
    for (int j = 0; j < k; ++j) {
        const int i = d2s[j];
        if (i < -1 || i >= m || (i >= 0 && s2d[i] != j)) return OT_E_INVAL;
        fresh += i < 0 ? 1 : 0;
    }
    if ((long long)m + fresh > cap) return OT_E_WORKSPACE;
    if ((long long)*next_id + fresh > INT32_MAX) return OT_E_INVAL;
    for (int i = 0; i < m; ++i) {
        if (lost[i]) continue;
        const int j = s2d[i];
        if (j >= 0) {
            for (int q = 0; q < 4; ++q) boxes[4 * i + q] = det[4 * j + q];
        } else {
            lost[i] = 1;
        }
    }
    int o = m;
    for (int j = 0; j < k; ++j) {
        if (d2s[j] >= 0) continue;
        for (int q = 0; q < 4; ++q) boxes[4 * o + q] = det[4 * j + q];
        ids[o] = (*next_id)++;
        lost[o] = 0;
        ++o;
    }
    *m_out = o;
    return OT_OK;
}

}  // extern "C"
