// ot_lk_sched.hpp -- launch shape shared by the single-call and batched
// tracking kernels: occupancy bounds and the order in which workgroups take
// points (XCD-aware).
#pragma once
#include "ot_lk_dev.hpp"

// Optional occupancy target (waves per SIMD) for the tracking kernels.
#ifndef OT_LK_MIN_WAVES
#define OT_LK_MIN_WAVES 0
#endif
#if OT_LK_MIN_WAVES > 0
#define OT_LK_BOUNDS __launch_bounds__(64, OT_LK_MIN_WAVES)
#else
#define OT_LK_BOUNDS __launch_bounds__(64)
#endif

// Point order.  Workgroup b runs on XCD b % 8.  Points of one box cost
// alike, so giving each XCD one contiguous range of points (OT_LK_XCD_REMAP
// 1) leaves some XCDs with the expensive boxes.  The default (0) deals
// chunks of LK_CHUNK consecutive points to the XCDs round-robin: the XCDs
// get even shares of every box, while each chunk's outputs fill whole cache
// lines in one XCD's L2 and its neighbouring windows share that L2.  Each XCD
// then reads most of both pyramids (a few MB per frame pair), which costs far
// less than the imbalance it removes.
#ifndef OT_LK_XCD_REMAP
#define OT_LK_XCD_REMAP 0
#endif

namespace ot {

constexpr int LK_CHUNK = 16;

__device__ __forceinline__ int lk_item(int b, int G) {
    if (OT_LK_XCD_REMAP) return xcd_remap(b, G);
    constexpr int X = 8, S = X * LK_CHUNK;
    if (b >= G - G % S) return b;  // ragged tail in dispatch order
    const int x = b % X, k = b / X;
    return ((k / LK_CHUNK) * X + x) * LK_CHUNK + k % LK_CHUNK;
}

}  // namespace ot

// Template row counts of the generic (any odd window) tracking kernels.
#define OT_LK_ROWS(X) X(1) X(2) X(4) X(7) X(8) X(12) X(16)
