// ot_api.hip -- the C ABI (include/omnitrack.h): argument validation,
// pyramid layout, single-call launches and the batched tick.
#include <math.h>
#include <string.h>

#include <hip/hip_runtime.h>

#include "ot_common.hpp"
#include "ot_launch.hpp"

using namespace ot;

namespace {

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool level_dims(int32_t W, int32_t H, int32_t levels, int32_t* w, int32_t* h) {
    if (W < 1 || H < 1 || W > OT_MAX_DIM || H > OT_MAX_DIM || levels < 1 || levels > OT_MAX_LEVELS)
        return false;
    w[0] = W;
    h[0] = H;
    for (int l = 1; l < levels; ++l) {
        w[l] = (w[l - 1] + 1) / 2;
        h[l] = (h[l - 1] + 1) / 2;
    }
    return true;
}

size_t level_pitch(int32_t w) { return align_up((size_t)w, 64); }
size_t grad_pitch(int32_t w) { return align_up((size_t)w, 16); }  // int32 elements

size_t pyr_bytes(const int32_t* w, const int32_t* h, int32_t levels, int32_t flags) {
    size_t total = 0;
    for (int l = 1; l < levels; ++l) total += align_up(level_pitch(w[l]) * (size_t)h[l], 256);
    if (flags & OT_PYR_GRADS)
        for (int l = 0; l < levels; ++l) total += align_up(grad_pitch(w[l]) * (size_t)h[l] * 4, 256);
    return total;
}

bool flags_valid(int32_t flags) { return flags == 0 || flags == OT_PYR_GRADS; }

ot_err layout(const uint8_t* frame, int32_t W, int32_t H, int32_t pitch, int32_t levels,
              void* workspace, size_t ws_bytes, int32_t flags, ot_pyr* out) {
    int32_t w[OT_MAX_LEVELS], h[OT_MAX_LEVELS];
    if (!frame || !out || !flags_valid(flags) || pitch < W || pitch > OT_MAX_PITCH ||
        !level_dims(W, H, levels, w, h))
        return OT_E_INVAL;
    const size_t need = pyr_bytes(w, h, levels, flags);
    if (need > 0 && (!workspace || ws_bytes < need || ((uintptr_t)workspace & 255) != 0))
        return OT_E_WORKSPACE;
    ot_pyr p;
    memset(&p, 0, sizeof(p));
    p.levels = levels;
    p.level[0] = frame;
    p.w[0] = W;
    p.h[0] = H;
    p.pitch[0] = pitch;
    size_t off = 0;
    for (int l = 1; l < levels; ++l) {
        p.level[l] = static_cast<const uint8_t*>(workspace) + off;
        p.w[l] = w[l];
        p.h[l] = h[l];
        p.pitch[l] = (int32_t)level_pitch(w[l]);
        off += align_up((size_t)p.pitch[l] * h[l], 256);
    }
    p.flags = flags;
    if (flags & OT_PYR_GRADS)
        for (int l = 0; l < levels; ++l) {
            p.grad[l] = reinterpret_cast<const int32_t*>(static_cast<const uint8_t*>(workspace) + off);
            p.gpitch[l] = (int32_t)grad_pitch(w[l]);
            off += align_up((size_t)p.gpitch[l] * h[l] * 4, 256);
        }
    *out = p;
    return OT_OK;
}

// A descriptor the caller hands back must be self-consistent.
bool pyr_valid(const ot_pyr* p) {
    if (!p || p->levels < 1 || p->levels > OT_MAX_LEVELS) return false;
    int32_t w[OT_MAX_LEVELS], h[OT_MAX_LEVELS];
    if (!level_dims(p->w[0], p->h[0], p->levels, w, h)) return false;
    for (int l = 0; l < p->levels; ++l)
        if (!p->level[l] || p->w[l] != w[l] || p->h[l] != h[l] || p->pitch[l] < w[l] ||
            p->pitch[l] > OT_MAX_PITCH)
            return false;
    if (!flags_valid(p->flags)) return false;
    if (p->flags & OT_PYR_GRADS)
        for (int l = 0; l < p->levels; ++l)
            if (!p->grad[l] || p->gpitch[l] < w[l] || ((uintptr_t)p->grad[l] & 3) != 0) return false;
    return true;
}

// Device descriptor of levels base.. of p (base 0: the whole pyramid).
DevPyr to_dev(const ot_pyr& p, int base = 0) {
    DevPyr d;
    memset(&d, 0, sizeof(d));
    for (int l = 0; l + base < p.levels; ++l) {
        d.lvl[l] = p.level[l + base];
        d.w[l] = p.w[l + base];
        d.h[l] = p.h[l + base];
        d.pitch[l] = p.pitch[l + base];
        if (p.flags & OT_PYR_GRADS) {
            d.grad[l] = p.grad[l + base];
            d.gpitch[l] = p.gpitch[l + base];
        }
    }
    d.levels = p.levels - base;
    d.flags = p.flags;
    return d;
}

ot_err lk_params(int32_t win, int32_t levels, int32_t iters, float eps, float min_eig,
                 int32_t margin, LkParams* prm) {
    if (win < 3 || win > OT_MAX_WIN || (win & 1) == 0 || iters < 1 || !(eps >= 0.0f) ||
        !isfinite(eps) || !isfinite(min_eig) || levels < 1 || levels > OT_MAX_LEVELS ||
        margin < 0 || margin > LK_MAX_MARGIN)
        return OT_E_INVAL;
    const int m = margin == 0 ? LK_DEFAULT_MARGIN : margin;
    const int R = lk_template_rows(win);
    if (R == 0 || lk_lds_bytes(win, R, m) > LK_MAX_LDS) return OT_E_UNSUPPORTED;
    prm->win = win;
    prm->levels = levels;
    prm->iters = iters;
    prm->eps2 = eps * eps;
    prm->min_eig = min_eig;
    prm->margin = m;
    prm->pscale = 1.0f;
    prm->pscale_inv = 1.0f;
    return OT_OK;
}

}  // namespace

extern "C" {

size_t ot_pyramid_bytes(int32_t W, int32_t H, int32_t levels, int32_t flags) {
    int32_t w[OT_MAX_LEVELS], h[OT_MAX_LEVELS];
    if (!flags_valid(flags) || !level_dims(W, H, levels, w, h)) return 0;
    return pyr_bytes(w, h, levels, flags);
}

ot_err ot_pyramid_layout(const uint8_t* frame, int32_t W, int32_t H, int32_t pitch,
                         int32_t levels, void* workspace, size_t ws_bytes, int32_t flags,
                         ot_pyr* out) {
    return layout(frame, W, H, pitch, levels, workspace, ws_bytes, flags, out);
}

ot_err ot_pyramid_build(const uint8_t* frame, int32_t W, int32_t H, int32_t pitch,
                        int32_t levels, void* workspace, size_t ws_bytes, int32_t flags,
                        ot_pyr* out, void* stream) {
    ot_pyr p;
    const ot_err e = layout(frame, W, H, pitch, levels, workspace, ws_bytes, flags, &p);
    if (e != OT_OK) return e;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const DevPyr d = to_dev(p);
    for (int l0 = 0; l0 < levels - 1; l0 += PYR_FUSE)
        if (launch_pyr_stage(d, l0, pyr_stage_steps(levels, l0), s) != hipSuccess)
            return OT_E_LAUNCH;
    if ((flags & OT_PYR_GRADS) && launch_grad(d, levels, s) != hipSuccess) return OT_E_LAUNCH;
    *out = p;
    return OT_OK;
}

ot_err ot_lk_track_ex(const ot_pyr* prev_pyr, const ot_pyr* next_pyr, const float* pts,
                      int32_t n, int32_t win, int32_t levels, int32_t iters, float eps,
                      float* next_pts, uint8_t* status, float* err, const ot_lk_opts* opts,
                      void* stream) {
    if (n < 0) return OT_E_INVAL;
    if (!pyr_valid(prev_pyr) || !pyr_valid(next_pyr)) return OT_E_INVAL;
    const int base = opts ? opts->base_level : 0;
    if (base < 0 || base >= OT_MAX_LEVELS || levels > OT_MAX_LEVELS ||
        levels + base > prev_pyr->levels || levels + base > next_pyr->levels)
        return OT_E_INVAL;
    if (prev_pyr->w[0] != next_pyr->w[0] || prev_pyr->h[0] != next_pyr->h[0]) return OT_E_SHAPE;
    LkParams prm;
    const float min_eig = opts ? opts->min_eig : OT_DEFAULT_MIN_EIG;
    const ot_err e = lk_params(win, levels, iters, eps, min_eig, opts ? opts->margin : 0, &prm);
    if (e != OT_OK) return e;
    prm.pscale = ldexpf(1.0f, -base);
    prm.pscale_inv = ldexpf(1.0f, base);
    if (n == 0) return OT_OK;
    if (!pts || !next_pts || !status) return OT_E_INVAL;
    if (launch_lk(to_dev(*prev_pyr, base), to_dev(*next_pyr, base), pts, n, prm, next_pts, status, err,
                  opts ? opts->iters_out : nullptr, opts ? opts->lam_out : nullptr,
                  opts ? opts->order : nullptr, static_cast<hipStream_t>(stream)) != hipSuccess)
        return OT_E_LAUNCH;
    return OT_OK;
}

ot_err ot_lk_track(const ot_pyr* prev_pyr, const ot_pyr* next_pyr, const float* pts, int32_t n,
                   int32_t win, int32_t levels, int32_t iters, float eps, float* next_pts,
                   uint8_t* status, float* err, void* stream) {
    return ot_lk_track_ex(prev_pyr, next_pyr, pts, n, win, levels, iters, eps, next_pts, status,
                          err, nullptr, stream);
}

ot_err ot_lk_track_fb(const ot_pyr* prev_pyr, const ot_pyr* next_pyr, const float* pts,
                      int32_t n, int32_t win, int32_t levels, int32_t iters, float eps,
                      float* next_pts, uint8_t* status, float* err, float* back_pts,
                      uint8_t* back_status, float fb_max, float* fb_err, uint8_t* kept,
                      const ot_lk_opts* opts, void* stream) {
    if (n < 0) return OT_E_INVAL;
    if (kept && !(fb_max >= 0.0f)) return OT_E_INVAL;  // also NaN
    if (!pyr_valid(prev_pyr) || !pyr_valid(next_pyr)) return OT_E_INVAL;
    const int base = opts ? opts->base_level : 0;
    if (base < 0 || base >= OT_MAX_LEVELS || levels > OT_MAX_LEVELS ||
        levels + base > prev_pyr->levels || levels + base > next_pyr->levels)
        return OT_E_INVAL;
    if (prev_pyr->w[0] != next_pyr->w[0] || prev_pyr->h[0] != next_pyr->h[0]) return OT_E_SHAPE;
    if (opts && (opts->iters_out || opts->lam_out || opts->order)) return OT_E_UNSUPPORTED;
    LkParams prm;
    const float min_eig = opts ? opts->min_eig : OT_DEFAULT_MIN_EIG;
    const ot_err e = lk_params(win, levels, iters, eps, min_eig, opts ? opts->margin : 0, &prm);
    if (e != OT_OK) return e;
    prm.pscale = ldexpf(1.0f, -base);
    prm.pscale_inv = ldexpf(1.0f, base);
    if (n == 0) return OT_OK;
    if (!pts || !next_pts || !status || !back_pts || !back_status) return OT_E_INVAL;
    if (((uintptr_t)fb_err & 3) != 0) return OT_E_INVAL;
    if (launch_lk_fb(to_dev(*prev_pyr, base), to_dev(*next_pyr, base), pts, n, prm, next_pts,
                     status, err, back_pts, back_status, fb_max, fb_err, kept,
                     static_cast<hipStream_t>(stream)) != hipSuccess)
        return OT_E_LAUNCH;
    return OT_OK;
}

ot_err ot_lk_order(const uint8_t* iters, int32_t n, int32_t levels, int32_t* order,
                   void* stream) {
    if (n < 0 || n > (1 << 24) || levels < 1 || levels > OT_MAX_LEVELS) return OT_E_INVAL;
    if (n == 0) return OT_OK;
    if (!iters || !order) return OT_E_INVAL;
    if (launch_lk_order(iters, n, levels, order, static_cast<hipStream_t>(stream)) != hipSuccess)
        return OT_E_LAUNCH;
    return OT_OK;
}

int32_t ot_working_level(int32_t W, int32_t H, int32_t max_width) {
    if (W < 1 || H < 1 || max_width < 1) return -1;
    int32_t l = 0, w = W;
    while (w > max_width) {
        w = (w + 1) / 2;
        ++l;
    }
    return l;
}

ot_err ot_box_update(const float* boxes, int32_t m, const int32_t* box_id, const float* pts,
                     const float* next_pts, const uint8_t* status, int32_t n, float* out_boxes,
                     int32_t* out_count, void* stream) {
    if (m < 0 || n < 0) return OT_E_INVAL;
    if (m == 0) return OT_OK;
    if (!boxes || !out_boxes || !out_count) return OT_E_INVAL;
    if (n > 0 && (!box_id || !pts || !next_pts || !status)) return OT_E_INVAL;
    if (((uintptr_t)pts | (uintptr_t)next_pts) & 7) return OT_E_INVAL;
    if (launch_box(boxes, m, box_id, pts, next_pts, status, n, out_boxes, out_count,
                   static_cast<hipStream_t>(stream)) != hipSuccess)
        return OT_E_LAUNCH;
    return OT_OK;
}

ot_err ot_fb_gate(const float* pts, const float* back_pts, const uint8_t* st_fwd,
                  const uint8_t* st_bwd, int32_t n, float fb_max, float* fb_err,
                  uint8_t* status_out, void* stream) {
    if (n < 0 || !(fb_max >= 0.0f)) return OT_E_INVAL;
    if (n == 0) return OT_OK;
    if (!pts || !back_pts || !st_fwd || !st_bwd || !status_out) return OT_E_INVAL;
    if (((uintptr_t)pts | (uintptr_t)back_pts) & 7) return OT_E_INVAL;
    if (fb_err && ((uintptr_t)fb_err & 3)) return OT_E_INVAL;
    if (launch_fb_gate(pts, back_pts, st_fwd, st_bwd, n, fb_max, fb_err, status_out,
                       static_cast<hipStream_t>(stream)) != hipSuccess)
        return OT_E_LAUNCH;
    return OT_OK;
}

size_t ot_box_scaled_bytes(int32_t m) {
    if (m < 0 || m > (1 << 24)) return 0;
    return box_scaled_ws_bytes(m);
}

ot_err ot_box_update_scaled(const float* boxes, int32_t m, const int32_t* box_id,
                            const float* pts, const float* next_pts, const uint8_t* status,
                            int32_t n, float* out_boxes, int32_t* out_count, float* out_scale,
                            void* ws, size_t ws_bytes, void* stream) {
    if (m < 0 || n < 0 || m > (1 << 24)) return OT_E_INVAL;
    if (m == 0) return OT_OK;
    if (!boxes || !out_boxes || !out_count || !out_scale) return OT_E_INVAL;
    if (n > 0 && (!box_id || !pts || !next_pts || !status)) return OT_E_INVAL;
    if (((uintptr_t)pts | (uintptr_t)next_pts) & 7) return OT_E_INVAL;
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < box_scaled_ws_bytes(m)) return OT_E_WORKSPACE;
    if (launch_box_scaled(boxes, m, box_id, pts, next_pts, status, n, out_boxes, out_count,
                          out_scale, ws, static_cast<hipStream_t>(stream)) != hipSuccess)
        return OT_E_LAUNCH;
    return OT_OK;
}

ot_err ot_box_update_scaled_noalloc(const float* boxes, int32_t m, const int32_t* box_id,
                                    const float* pts, const float* next_pts, const uint8_t* status,
                                    int32_t n, float* out_boxes, int32_t* out_count,
                                    float* out_scale, void* stream) {
    if (m < 0 || n < 0 || m > OT_SCALED_NOALLOC_MAX_BOXES) return OT_E_INVAL;
    if (m == 0) return OT_OK;
    if (!boxes || !out_boxes || !out_count || !out_scale) return OT_E_INVAL;
    if (n > 0 && (!box_id || !pts || !next_pts || !status)) return OT_E_INVAL;
    if (((uintptr_t)pts | (uintptr_t)next_pts) & 7) return OT_E_INVAL;
    if (launch_box_scaled_noalloc(boxes, m, box_id, pts, next_pts, status, n, out_boxes,
                                  out_count, out_scale,
                                  static_cast<hipStream_t>(stream)) != hipSuccess)
        return OT_E_LAUNCH;
    return OT_OK;
}

// ------------------------------------------------------------------ batched
static bool cfg_valid(const ot_batch_cfg* c) {
    return c && c->max_jobs >= 1 && c->max_points >= 0 && c->max_boxes >= 0 &&
           c->max_tiles >= 0 && c->max_levels >= 1 && c->max_levels <= OT_MAX_LEVELS &&
           c->lk_waves >= 0 && c->chunk >= 0 && c->lk_wpg >= 0 && c->lk_ppw >= 0;
}

size_t ot_batch_table_bytes(const ot_batch_cfg* cfg) {
    if (!cfg_valid(cfg)) return 0;
    return TableLayout::make(cfg->max_jobs).bytes;
}

ot_err ot_batch_pack(const ot_job* jobs, int32_t njobs, const ot_batch_cfg* cfg,
                     void* table_host, size_t table_bytes, ot_pyr* next_out) {
    if (!cfg_valid(cfg) || njobs < 0 || (njobs > 0 && !jobs) || !table_host) return OT_E_INVAL;
    if (njobs > cfg->max_jobs) return OT_E_WORKSPACE;
    const TableLayout T = TableLayout::make(cfg->max_jobs);
    if (table_bytes < T.bytes) return OT_E_WORKSPACE;
    LkParams prm;
    ot_err e = lk_params(cfg->win, 1, cfg->iters, cfg->eps, cfg->min_eig, cfg->margin, &prm);
    if (e != OT_OK) return e;

    uint8_t* tb = static_cast<uint8_t*>(table_host);
    TableHdr hd;
    memset(&hd, 0, sizeof(hd));
    int32_t* ptp = reinterpret_cast<int32_t*>(tb + T.pt_prefix);
    int32_t* bxp = reinterpret_cast<int32_t*>(tb + T.box_prefix);
    int32_t* tlp = reinterpret_cast<int32_t*>(tb + T.tile_prefix);
    int32_t* tlc = reinterpret_cast<int32_t*>(tb + T.tile_cols);
    DevJob* dj = reinterpret_cast<DevJob*>(tb + T.jobs);
    int64_t pts_total = 0, boxes_total = 0;
    int64_t tiles[OT_MAX_LEVELS] = {0};
    int max_level = 0;
    // validate everything before writing anything
    for (int j = 0; j < njobs; ++j) {
        const ot_job& J = jobs[j];
        if (!pyr_valid(&J.prev) || J.levels < 1 || J.levels > J.prev.levels) return OT_E_INVAL;
        if (J.n < 0 || J.m < 0) return OT_E_INVAL;
        if (J.n > 0 && (!J.pts || !J.next_pts || !J.status)) return OT_E_INVAL;
        if (J.m > 0 && (!J.boxes || !J.out_boxes || !J.out_count || (J.n > 0 && !J.box_id)))
            return OT_E_INVAL;
        if (((uintptr_t)J.pts | (uintptr_t)J.next_pts) & 7) return OT_E_INVAL;
        ot_pyr np;
        e = layout(J.next_frame, J.prev.w[0], J.prev.h[0], J.next_pitch, J.levels, J.next_ws,
                   J.next_ws_bytes, 0, &np);
        if (e != OT_OK) return e;
        pts_total += J.n;
        boxes_total += J.m;
        for (int l0 = 0; l0 < J.levels - 1; l0 += PYR_FUSE) {
            const int top = l0 + pyr_stage_steps(J.levels, l0);
            tiles[l0 + 1] += (int64_t)((np.w[top] + PYR_FTW - 1) / PYR_FTW) *
                             ((np.h[top] + PYR_FTH - 1) / PYR_FTH);
        }
        if (J.levels - 1 > max_level) max_level = J.levels - 1;
    }
    if (pts_total > cfg->max_points && cfg->lk_waves == 0) return OT_E_WORKSPACE;
    if (pts_total > INT32_MAX / 2 || boxes_total > cfg->max_boxes) return OT_E_WORKSPACE;
    if (max_level > cfg->max_levels - 1) return OT_E_WORKSPACE;
    for (int l = 1; l < OT_MAX_LEVELS; ++l)
        if (tiles[l] > cfg->max_tiles) return OT_E_WORKSPACE;

    memset(tb, 0, T.bytes);
    int32_t pacc = 0, bacc = 0;
    int32_t tacc[OT_MAX_LEVELS] = {0};
    for (int j = 0; j < njobs; ++j) {
        const ot_job& J = jobs[j];
        ot_pyr np;
        layout(J.next_frame, J.prev.w[0], J.prev.h[0], J.next_pitch, J.levels, J.next_ws,
               J.next_ws_bytes, 0, &np);
        if (next_out) next_out[j] = np;
        DevJob d;
        memset(&d, 0, sizeof(d));
        d.prev = to_dev(J.prev);
        d.next = to_dev(np);
        d.pts = J.pts;
        d.next_pts = J.next_pts;
        d.status = J.status;
        d.err = J.err;
        d.boxes = J.boxes;
        d.box_id = J.box_id;
        d.out_boxes = J.out_boxes;
        d.out_count = J.out_count;
        d.n = J.n;
        d.m = J.m;
        d.levels = J.levels;
        memcpy(&dj[j], &d, sizeof(d));
        ptp[j] = pacc;
        bxp[j] = bacc;
        pacc += J.n;
        bacc += J.m;
        // fused pyramid stages start at levels 0, PYR_FUSE, ...; stage l0's
        // tile list lives at per-level index l0 + 1
        for (int l = 1; l < OT_MAX_LEVELS; ++l) {
            tlp[(size_t)l * (cfg->max_jobs + 1) + j] = tacc[l];
            const int l0 = l - 1;
            if (l0 % PYR_FUSE == 0 && l0 < J.levels - 1) {
                const int top = l0 + pyr_stage_steps(J.levels, l0);
                const int cols = (np.w[top] + PYR_FTW - 1) / PYR_FTW;
                tlc[(size_t)l * cfg->max_jobs + j] = cols;
                tacc[l] += cols * ((np.h[top] + PYR_FTH - 1) / PYR_FTH);
            } else {
                tlc[(size_t)l * cfg->max_jobs + j] = 1;
            }
        }
    }
    ptp[njobs] = pacc;
    bxp[njobs] = bacc;
    for (int l = 1; l < OT_MAX_LEVELS; ++l) tlp[(size_t)l * (cfg->max_jobs + 1) + njobs] = tacc[l];
    hd.njobs = njobs;
    hd.total_pts = pacc;
    hd.total_boxes = bacc;
    hd.max_level = max_level;
    for (int l = 0; l < OT_MAX_LEVELS; ++l) hd.total_tiles[l] = tacc[l];
    hd.lk = prm;
    hd.chunk = cfg->chunk > 0 ? cfg->chunk : 1;
    hd.counter = 0;
    memcpy(tb, &hd, sizeof(hd));
    return OT_OK;
}

ot_err ot_batch_run_stages(const void* table_host, void* table_dev, size_t table_bytes,
                           const ot_batch_cfg* cfg, int32_t stages, void* stream) {
    if (!cfg_valid(cfg) || !table_host || !table_dev) return OT_E_INVAL;
    if (stages < 1 || stages > (OT_STAGE_PYRAMID | OT_STAGE_TRACK)) return OT_E_INVAL;
    const TableLayout T = TableLayout::make(cfg->max_jobs);
    if (table_bytes < T.bytes || ((uintptr_t)table_dev & 255) != 0) return OT_E_WORKSPACE;
    LkParams prm;
    const ot_err e = lk_params(cfg->win, 1, cfg->iters, cfg->eps, cfg->min_eig, cfg->margin, &prm);
    if (e != OT_OK) return e;
    const int wpg = cfg->lk_wpg > 0 ? cfg->lk_wpg : 1, ppw = cfg->lk_ppw > 0 ? cfg->lk_ppw : 1;
    if (!batch_lk_shape_ok(prm.win, prm.margin, wpg, ppw) ||
        (cfg->lk_waves > 0 && (wpg != 1 || ppw != 1)))
        return OT_E_UNSUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint8_t* tdev = static_cast<const uint8_t*>(table_dev);
    // grid sizes: the capacities (graph-capturable), or the packed totals
    TableHdr hd;
    memcpy(&hd, table_host, sizeof(hd));
    const bool exact = cfg->exact_grids != 0;
    if (stages & OT_STAGE_PYRAMID) {
        // an eager tick copies what it packed; a graph-capturable one the whole table
        const size_t nb = exact && hd.njobs >= 0 && hd.njobs <= cfg->max_jobs ? T.used(hd.njobs)
                                                                                 : T.bytes;
        if (hipMemcpyAsync(table_dev, table_host, nb, hipMemcpyHostToDevice, s) != hipSuccess)
            return OT_E_LAUNCH;
        for (int l0 = 0; l0 < cfg->max_levels - 1; l0 += PYR_FUSE) {
            const int grid = exact ? hd.total_tiles[l0 + 1] : cfg->max_tiles;
            if (grid > 0 && launch_batch_pyr(tdev, cfg->max_jobs, l0, grid, s) != hipSuccess)
                return OT_E_LAUNCH;
        }
    }
    if (stages & OT_STAGE_TRACK) {
        const bool persistent = cfg->lk_waves > 0;
        const int npts = exact ? hd.total_pts : cfg->max_points;
        const int lk_waves = persistent && !(exact && hd.total_pts == 0) ? cfg->lk_waves : 0;
        if ((persistent ? lk_waves : npts) > 0 &&
            launch_batch_lk(tdev, cfg->max_jobs, prm.win, prm.margin, npts, lk_waves, wpg, ppw,
                            s) != hipSuccess)
            return OT_E_LAUNCH;
        const int grid = exact ? hd.total_boxes : cfg->max_boxes;
        if (grid > 0 && launch_batch_box(tdev, cfg->max_jobs, grid, s) != hipSuccess)
            return OT_E_LAUNCH;
    }
    return OT_OK;
}

ot_err ot_batch_run(const void* table_host, void* table_dev, size_t table_bytes,
                    const ot_batch_cfg* cfg, void* stream) {
    return ot_batch_run_stages(table_host, table_dev, table_bytes, cfg,
                               OT_STAGE_PYRAMID | OT_STAGE_TRACK, stream);
}

const char* ot_strerror(ot_err e) {
    switch (e) {
        case OT_OK: return "ok";
        case OT_E_INVAL: return "invalid argument";
        case OT_E_SHAPE: return "shape mismatch";
        case OT_E_WORKSPACE: return "workspace or capacity too small";
        case OT_E_LAUNCH: return "HIP launch failed";
        case OT_E_UNSUPPORTED: return "unsupported configuration";
        default: return "unknown error";
    }
}

int32_t ot_version(void) { return 100; }

}  // extern "C"
