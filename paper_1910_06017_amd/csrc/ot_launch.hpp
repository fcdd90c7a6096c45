// ot_launch.hpp -- internal host launchers (one per kernel family).  Each
// enqueues on `stream` and returns hipGetLastError() of its launches.
#pragma once
#include <hip/hip_runtime.h>

#include "ot_common.hpp"

namespace ot {

// Levels l0+1 .. l0+K (K <= PYR_FUSE) of a pyramid from level l0.
hipError_t launch_pyr_stage(const DevPyr& P, int l0, int K, hipStream_t stream);

// Scharr gradient planes of levels 0..levels-1 (P.grad must be set).
hipError_t launch_grad(const DevPyr& P, int levels, hipStream_t stream);

// Template row count the tracker uses for a window (0 = unsupported).
int lk_template_rows(int win);

hipError_t launch_lk(const DevPyr& prev, const DevPyr& next, const float* pts, int n,
                     const LkParams& prm, float* next_pts, uint8_t* status, float* err,
                     uint8_t* iters_out, float* lam_out, const int32_t* order,
                     hipStream_t stream);

// Forward then backward tracking of every point in one launch (next_pts,
// status, err as launch_lk(prev, next); back_pts, back_status as
// launch_lk(next, prev) on next_pts), then, with kept set, the
// forward-backward gate (kept, fb_err as launch_fb_gate).
hipError_t launch_lk_fb(const DevPyr& prev, const DevPyr& next, const float* pts, int n,
                        const LkParams& prm, float* next_pts, uint8_t* status, float* err,
                        float* back_pts, uint8_t* back_status, float fb_max, float* fb_err,
                        uint8_t* kept, hipStream_t stream);

// Points by descending total iteration count (one workgroup, counting sort).
hipError_t launch_lk_order(const uint8_t* iters, int n, int levels, int32_t* order,
                           hipStream_t stream);

hipError_t launch_box(const float* boxes, int m, const int32_t* box_id, const float* pts,
                      const float* next_pts, const uint8_t* status, int n, float* out_boxes,
                      int32_t* out_count, hipStream_t stream);

// Median-Flow box update (centre by the median displacement, extents by the
// median pairwise distance ratio) and the forward-backward point gate.
hipError_t launch_box_scaled(const float* boxes, int m, const int32_t* box_id, const float* pts,
                             const float* next_pts, const uint8_t* status, int n, float* out_boxes,
                             int32_t* out_count, float* out_scale, void* ws, hipStream_t stream);
// Workspace of the scaled update for m boxes (one block per box).
size_t box_scaled_ws_bytes(int m);
// The scaled update on the library's static per-device scratch
// (m <= OT_SCALED_NOALLOC_MAX_BOXES, checked by the caller).
hipError_t launch_box_scaled_noalloc(const float* boxes, int m, const int32_t* box_id,
                                     const float* pts, const float* next_pts,
                                     const uint8_t* status, int n, float* out_boxes,
                                     int32_t* out_count, float* out_scale, hipStream_t stream);
hipError_t launch_fb_gate(const float* pts, const float* back_pts, const uint8_t* st_fwd,
                          const uint8_t* st_bwd, int n, float fb_max, float* fb_err,
                          uint8_t* status_out, hipStream_t stream);

// Batched stages over a device table (layout TableLayout::make(cap)).
hipError_t launch_batch_pyr(const uint8_t* table, int cap, int l0, int grid, hipStream_t stream);
// Tracking stage: a persistent grid of lk_waves waves (lk_waves > 0), else
// npts points in workgroups of wpg waves tracking ppw points each.
hipError_t launch_batch_lk(const uint8_t* table, int cap, int win, int margin, int npts,
                           int lk_waves, int wpg, int ppw, hipStream_t stream);
// 1 if the tracking stage has an instantiation for this window, margin and
// (wpg, ppw) (1 x 1 always; 2 and 4 for the 21 x 21 window at margins 4, 6).
int batch_lk_shape_ok(int win, int margin, int wpg, int ppw);
hipError_t launch_batch_box(const uint8_t* table, int cap, int grid, hipStream_t stream);

}  // namespace ot
