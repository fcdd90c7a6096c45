// ot_common.hpp -- layouts shared by the host layer and the gfx950 kernels of
// the pyramidal Lucas-Kanade tracker (device descriptors, batched table).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "omnitrack.h"

#if defined(__HIPCC__)
#define OT_HD __host__ __device__
#else
#define OT_HD
#endif

namespace ot {

// Pyramid: one launch reduces up to PYR_FUSE levels; a PYR_THREADS workgroup
// owns a PYR_FTW x PYR_FTH tile of the launch's top level and that tile's
// footprint at the levels below it.
#ifndef OT_PYR_FTW
#define OT_PYR_FTW 16
#endif
#ifndef OT_PYR_FTH
#define OT_PYR_FTH 8
#endif
#ifndef OT_PYR_THREADS
#define OT_PYR_THREADS 1024
#endif
constexpr int PYR_FUSE = 3;
constexpr int PYR_FTW = OT_PYR_FTW;
constexpr int PYR_FTH = OT_PYR_FTH;
constexpr int PYR_THREADS = OT_PYR_THREADS;

// Steps of the fused launch starting at level l0 for a pyramid of `levels`.
OT_HD inline int pyr_stage_steps(int levels, int l0) {
    const int k = levels - 1 - l0;
    return k < 0 ? 0 : (k > PYR_FUSE ? PYR_FUSE : k);
}

// Box median: one BOX_THREADS workgroup per box; up to BOX_CAP point
// displacements are gathered in LDS, larger boxes are re-scanned from memory.
#ifndef OT_BOX_THREADS
#define OT_BOX_THREADS 1024
#endif
constexpr int BOX_THREADS = OT_BOX_THREADS;
constexpr int BOX_CAP = 6144;
// Median-Flow box update: points per box it can take (all gathered in LDS,
// 16 bytes each).
constexpr int SCALE_CAP = OT_SCALE_MAX_POINTS;

constexpr int LK_DEFAULT_MARGIN = 4;
constexpr int LK_MAX_MARGIN = 16;
constexpr size_t LK_MAX_LDS = 64 * 1024;

// Device view of a pyramid (copied by value into kernel arguments or into
// the batched table).
struct DevPyr {
    const uint8_t* lvl[OT_MAX_LEVELS];
    const int32_t* grad[OT_MAX_LEVELS];  // packed Scharr sums (Sx low, Sy high), or null
    int32_t w[OT_MAX_LEVELS];
    int32_t h[OT_MAX_LEVELS];
    int32_t pitch[OT_MAX_LEVELS];
    int32_t gpitch[OT_MAX_LEVELS];
    int32_t levels;
    int32_t flags;
};

struct LkParams {
    int32_t win;
    int32_t levels;  // single-call launches; batched jobs carry their own
    int32_t iters;
    float eps2;
    float min_eig;
    int32_t margin;
    float pscale;      // point coordinates are multiplied by pscale on entry
    float pscale_inv;  // and results by pscale_inv (powers of two: a working level)
};

// One stream's frame pair in the batched table.
struct DevJob {
    DevPyr prev;
    DevPyr next;
    const float* pts;
    float* next_pts;
    uint8_t* status;
    float* err;
    const float* boxes;
    const int32_t* box_id;
    float* out_boxes;
    int32_t* out_count;
    int32_t n, m, levels, pad0;
};

// Batched table header.  The whole table is rewritten by each host->device
// copy, which also returns the persistent stage's work counter to zero.
struct TableHdr {
    int32_t njobs;
    int32_t total_pts;
    int32_t total_boxes;
    int32_t max_level;                  // highest pyramid level built
    int32_t total_tiles[OT_MAX_LEVELS]; // fused pyramid stage from level l-1 at index l
    LkParams lk;
    int32_t chunk;
    uint32_t counter;                   // persistent LK work counter
    uint32_t pad[4];
};

// Table layout for capacities (njobs_cap): header | pt_prefix | box_prefix |
// tile_prefix[levels][njobs_cap + 1] | tile_cols[levels][njobs_cap] | jobs.
struct TableLayout {
    size_t jobs, pt_prefix, box_prefix, tile_prefix, tile_cols, bytes;
    // The job records come last, so an eager tick copies the header, the
    // prefix sums and only the records of its packed jobs.
    OT_HD static TableLayout make(int32_t cap) {
        TableLayout t;
        size_t off = (sizeof(TableHdr) + 255) & ~size_t(255);
        t.pt_prefix = off;
        off += sizeof(int32_t) * (size_t)(cap + 1);
        t.box_prefix = off;
        off += sizeof(int32_t) * (size_t)(cap + 1);
        t.tile_prefix = off;
        off += sizeof(int32_t) * (size_t)(cap + 1) * OT_MAX_LEVELS;
        t.tile_cols = off;
        off += sizeof(int32_t) * (size_t)cap * OT_MAX_LEVELS;
        t.jobs = (off + 15) & ~size_t(15);
        off = t.jobs + sizeof(DevJob) * (size_t)cap;
        t.bytes = (off + 255) & ~size_t(255);
        return t;
    }
    // Bytes a tick of njobs jobs reads: everything up to its last job record.
    OT_HD size_t used(int32_t njobs) const { return jobs + sizeof(DevJob) * (size_t)njobs; }
};

// Rows per lane strip for a window: the wave's 64 lanes cover the window as
// win columns x nseg row segments of `rows` rows.
OT_HD constexpr int lk_nseg(int win) {
    int s = 64 / win;
    return s < 1 ? 1 : (s > win ? win : s);
}
OT_HD constexpr int lk_rows_needed(int win) {
    int s = lk_nseg(win);
    return (win + s - 1) / s;
}

// LDS of one tracking wave: the larger of the set-up stage (uint8 template
// patch + float2 gradient tap grid, both with the rows the Scharr groups run
// past the tap grid) and the iteration stage (packed half-pair target region
// with a margin on every side, rows padded to whole 16-byte groups from the
// 4-byte aligned column at or below the region), followed by the level-0
// template samples (R floats per lane, kept for the residual).
OT_HD constexpr size_t lk_lds_a_offset(int win, int R, int margin) {
    const int nseg = lk_nseg(win);
    const int RR = nseg * R + 1, TW = win + 1, PW = 4 * (((TW + 4) >> 2) + 1);
    const int ncg = 64 / TW, GR = (RR + ncg - 1) / ncg, GRR = ncg * GR;  // GRR >= RR
    const int PR = GRR + 2;
    const int SC = TW + 2 * margin, SP = 4 * (((SC + 3) >> 2) + 1);
    const size_t setup = (size_t)((PR * PW + 15) & ~15) + (size_t)GRR * TW * 8;
    const size_t iter = (size_t)(RR + 2 * margin) * SP * 4;
    return ((setup > iter ? setup : iter) + 15) & ~(size_t)15;
}
OT_HD constexpr size_t lk_lds_bytes(int win, int R, int margin) {
    return lk_lds_a_offset(win, R, margin) + (size_t)64 * R * 4;
}

}  // namespace ot
