"""The C ABI library on the CPU: it loads, exports every symbol the header
declares, and its host-side validation and table packing behave as the
header states.  No kernel is launched (fake device addresses are never
dereferenced because every case here fails validation or only packs a host
table)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1910_06017_amd import ops

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "omnitrack.h")

FAKE = 0x7F0000000000  # 256-aligned, never dereferenced


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ops.LIB_PATH):
        pytest.skip("libomnitrack.so not built")
    return ops.lib()


def declared_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"OT_API\s+[\w\s\*]*?\b(ot_\w+)\s*\(", txt)))


def test_header_symbols_exported(L):
    syms = declared_symbols()
    assert len(syms) == 30
    assert syms == sorted(ops.EXPORTS)
    for s in syms:
        assert hasattr(L, s), s


def test_pyramid_bytes(L):
    # levels 1..3 of 720x576: pitches 384/192/128 (64-byte rounding), 256-aligned sizes
    want = 384 * 288 + 192 * 144 + 128 * 72
    assert ops.pyramid_bytes(720, 576, 4) == want
    assert ops.pyramid_bytes(720, 576, 1) == 0
    for bad in [(0, 5, 2), (5, 0, 2), (5, 5, 0), (5, 5, 9), (20000, 5, 2)]:
        assert ops.pyramid_bytes(*bad) == 0
    assert L.ot_pyramid_bytes(64, 64, 2, 2) == 0  # unknown flag
    # OT_PYR_GRADS adds one int32 per pixel of levels 0..3, pitches rounded to 16
    # elements, planes 256-aligned: 720, 368 (360), 192 (180), 96 (90)
    al = lambda v: (v + 255) // 256 * 256
    planes = al(720 * 576 * 4) + al(368 * 288 * 4) + al(192 * 144 * 4) + al(96 * 72 * 4)
    assert ops.pyramid_bytes(720, 576, 4, ops.OT_PYR_GRADS) == want + planes
    assert ops.pyramid_bytes(720, 576, 1, ops.OT_PYR_GRADS) == al(720 * 576 * 4)


def layout(L, W=720, H=576, pitch=720, levels=4, ws=FAKE + 4096, wsb=10**7, flags=0):
    d = ops.OtPyr()
    rc = L.ot_pyramid_layout(FAKE, W, H, pitch, levels, ws, wsb, flags, C.byref(d))
    return rc, d


def test_pyramid_layout(L):
    rc, d = layout(L)
    assert rc == 0 and d.levels == 4
    assert list(d.w)[:4] == [720, 360, 180, 90] and list(d.h)[:4] == [576, 288, 144, 72]
    assert d.level[0] == FAKE and d.level[1] == FAKE + 4096
    assert d.level[2] == FAKE + 4096 + 384 * 288
    assert all(d.level[l] % 256 == 0 for l in range(1, 4))
    assert layout(L, pitch=719)[0] == ops_err("OT_E_INVAL")
    # row pitches are bounded so that the kernels' 32-bit offsets into a level
    # (row x pitch + column) cannot overflow
    assert layout(L, pitch=131072, levels=1, ws=0, wsb=0)[0] == 0
    assert layout(L, pitch=131073, levels=1, ws=0, wsb=0)[0] == ops_err("OT_E_INVAL")
    _, Q = layout(L)
    bad = ops.OtPyr()
    C.memmove(C.byref(bad), C.byref(Q), C.sizeof(Q))
    bad.pitch[0] = 131073
    assert lk_call(L, bad, Q) == ops_err("OT_E_INVAL")
    assert layout(L, ws=FAKE + 4096 + 8)[0] == ops_err("OT_E_WORKSPACE")
    assert layout(L, wsb=1000)[0] == ops_err("OT_E_WORKSPACE")
    assert layout(L, levels=1, ws=0, wsb=0)[0] == 0
    assert layout(L, flags=2)[0] == ops_err("OT_E_INVAL")
    assert d.flags == 0 and all(d.grad[l] is None for l in range(4))


def test_pyramid_layout_grads(L):
    G = ops.OT_PYR_GRADS
    rc, d = layout(L, flags=G)
    assert rc == 0 and d.flags == G
    base = FAKE + 4096 + 384 * 288 + 192 * 144 + 128 * 72   # after the uint8 levels
    assert d.grad[0] == base
    assert list(d.gpitch)[:4] == [720, 368, 192, 96]
    assert d.grad[1] == base + 720 * 576 * 4
    assert all(d.grad[l] % 256 == 0 for l in range(4))
    need = ops.pyramid_bytes(720, 576, 4, G)
    assert layout(L, flags=G, wsb=need)[0] == 0
    assert layout(L, flags=G, wsb=need - 1)[0] == ops_err("OT_E_WORKSPACE")
    # a single-level pyramid with planes needs a workspace
    assert layout(L, levels=1, ws=0, wsb=0, flags=G)[0] == ops_err("OT_E_WORKSPACE")
    # the tracker rejects a descriptor claiming planes it does not have
    _, P = layout(L, flags=G)
    _, Q = layout(L)
    bad = ops.OtPyr()
    C.memmove(C.byref(bad), C.byref(P), C.sizeof(P))
    bad.grad[2] = None
    assert lk_call(L, bad, Q) == ops_err("OT_E_INVAL")
    bad.grad[2] = P.grad[2]
    bad.gpitch[1] = 100
    assert lk_call(L, bad, Q) == ops_err("OT_E_INVAL")
    bad.gpitch[1] = P.gpitch[1]
    bad.flags = 3
    assert lk_call(L, bad, Q) == ops_err("OT_E_INVAL")


def ops_err(name):
    return {v: k for k, v in ops.ERRORS.items()}[name]


def lk_call(L, P, Q, n=10, win=21, levels=4, iters=30, eps=0.01, pts=FAKE, out=FAKE, st=FAKE):
    return L.ot_lk_track(C.byref(P), C.byref(Q), pts, n, win, levels, iters, eps, out, st, None,
                         None)


def test_lk_validation(L):
    _, P = layout(L)
    _, Q = layout(L)
    E, S, U = ops_err("OT_E_INVAL"), ops_err("OT_E_SHAPE"), ops_err("OT_E_UNSUPPORTED")
    assert lk_call(L, P, Q, win=20) == E          # even window
    assert lk_call(L, P, Q, win=1) == E
    assert lk_call(L, P, Q, win=33) == E         # above OT_MAX_WIN
    assert lk_call(L, P, Q, levels=5) == E        # more levels than the pyramids hold
    assert lk_call(L, P, Q, levels=0) == E
    assert lk_call(L, P, Q, iters=0) == E
    assert lk_call(L, P, Q, eps=-1.0) == E
    assert lk_call(L, P, Q, eps=float("nan")) == E
    assert lk_call(L, P, Q, eps=float("inf")) == E
    assert lk_call(L, P, Q, n=-1) == E
    assert lk_call(L, P, Q, pts=None) == E        # null pointer with n > 0
    assert lk_call(L, P, Q, out=None) == E
    assert lk_call(L, P, Q, n=0, pts=None, out=None, st=None) == 0  # no-op
    _, Q2 = layout(L, W=640)
    assert lk_call(L, P, Q2) == S
    bad = ops.OtPyr()
    C.memmove(C.byref(bad), C.byref(P), C.sizeof(P))
    bad.w[1] = 361                                # inconsistent descriptor
    assert lk_call(L, bad, Q) == E
    for base, lv in ((1, 4), (-1, 2), (4, 1), (8, 1)):   # base + levels beyond the pyramids
        opts = ops.OtLkOpts(6.5, None, None, 0, base)
        assert L.ot_lk_track_ex(C.byref(P), C.byref(Q), FAKE, 10, 21, lv, 30, 0.01, FAKE, FAKE,
                                None, C.byref(opts), None) == E
    opts = ops.OtLkOpts(6.5, None, None, 17)      # margin above the maximum
    assert L.ot_lk_track_ex(C.byref(P), C.byref(Q), FAKE, 10, 21, 4, 30, 0.01, FAKE, FAKE,
                            None, C.byref(opts), None) == E
    del U


def test_lk_fb_validation(L):
    """ot_lk_track_fb validates as ot_lk_track_ex, needs both outputs of the
    backward pass and, with the gate, a threshold as ot_fb_gate does; it has
    no per-point diagnostics or order."""
    _, P = layout(L)
    _, Q = layout(L)
    E, S, U = ops_err("OT_E_INVAL"), ops_err("OT_E_SHAPE"), ops_err("OT_E_UNSUPPORTED")

    def fb(P=P, Q=Q, n=10, win=21, levels=4, back=FAKE, bst=FAKE, opts=None, pts=FAKE,
           fb_max=1.0, fb_err=None, kept=None):
        return L.ot_lk_track_fb(C.byref(P), C.byref(Q), pts, n, win, levels, 30, 0.01, FAKE,
                                FAKE, None, back, bst, fb_max, fb_err, kept,
                                C.byref(opts) if opts else None, None)

    assert fb(n=-1) == E
    assert fb(win=20) == E
    assert fb(levels=5) == E
    assert fb(back=None) == E
    assert fb(bst=None) == E
    assert fb(pts=None) == E
    assert fb(n=0, back=None, bst=None, pts=None) == 0      # no-op
    _, Q2 = layout(L, W=640)
    assert fb(Q=Q2) == S
    for field in ("iters_out", "lam_out", "order"):
        opts = ops.OtLkOpts(6.5, None, None, 0, 0, None)
        setattr(opts, field, FAKE)
        assert fb(opts=opts) == U, field
    opts = ops.OtLkOpts(6.5, None, None, 0, 1)             # base + levels beyond the pyramids
    assert fb(opts=opts) == E
    # the gate's threshold is checked only when the gate runs
    assert fb(fb_max=-1.0, kept=FAKE) == E
    assert fb(fb_max=float("nan"), kept=FAKE) == E
    assert fb(kept=FAKE, fb_err=FAKE + 2) == E              # fb_err not 4-aligned
    assert fb(n=0, back=None, bst=None, pts=None, fb_max=-1.0) == 0


def test_box_validation(L):
    E = ops_err("OT_E_INVAL")
    assert L.ot_box_update(FAKE, -1, FAKE, FAKE, FAKE, FAKE, 5, FAKE, FAKE, None) == E
    assert L.ot_box_update(FAKE, 3, FAKE, FAKE, FAKE, FAKE, -5, FAKE, FAKE, None) == E
    assert L.ot_box_update(None, 3, FAKE, FAKE, FAKE, FAKE, 5, FAKE, FAKE, None) == E
    assert L.ot_box_update(FAKE, 3, None, FAKE, FAKE, FAKE, 5, FAKE, FAKE, None) == E
    assert L.ot_box_update(None, 0, None, None, None, None, 5, None, None, None) == 0
    assert L.ot_box_update(FAKE, 3, FAKE, FAKE + 4, FAKE, FAKE, 5, FAKE, FAKE, None) == E  # pts not 8-aligned


def test_fb_gate_validation(L):
    E = ops_err("OT_E_INVAL")
    g = L.ot_fb_gate
    assert g(FAKE, FAKE, FAKE, FAKE, -1, 1.0, FAKE, FAKE, None) == E
    assert g(FAKE, FAKE, FAKE, FAKE, 5, -0.5, FAKE, FAKE, None) == E          # negative threshold
    assert g(FAKE, FAKE, FAKE, FAKE, 5, float("nan"), FAKE, FAKE, None) == E
    assert g(None, FAKE, FAKE, FAKE, 5, 1.0, FAKE, FAKE, None) == E
    assert g(FAKE, FAKE, FAKE, None, 5, 1.0, FAKE, FAKE, None) == E
    assert g(FAKE, FAKE, FAKE, FAKE, 5, 1.0, FAKE, None, None) == E           # no status output
    assert g(FAKE, FAKE + 4, FAKE, FAKE, 5, 1.0, FAKE, FAKE, None) == E       # back_pts not 8-aligned
    assert g(FAKE, FAKE, FAKE, FAKE, 5, 1.0, FAKE + 2, FAKE, None) == E       # fb_err not 4-aligned
    assert g(None, None, None, None, 0, 1.0, None, None, None) == 0           # n == 0: no-op


def test_box_scaled_validation(L):
    E = ops_err("OT_E_INVAL")
    Wk = ops_err("OT_E_WORKSPACE")
    u = L.ot_box_update_scaled
    need = L.ot_box_scaled_bytes(3)
    assert need > 0 and L.ot_box_scaled_bytes(6) == 2 * need and L.ot_box_scaled_bytes(-1) == 0
    ws = FAKE + (1 << 20)
    assert u(FAKE, -1, FAKE, FAKE, FAKE, FAKE, 5, FAKE, FAKE, FAKE, ws, need, None) == E
    assert u(FAKE, 3, FAKE, FAKE, FAKE, FAKE, -5, FAKE, FAKE, FAKE, ws, need, None) == E
    assert u(FAKE, 3, FAKE, FAKE, FAKE, FAKE, 5, FAKE, FAKE, None, ws, need, None) == E  # no scale output
    assert u(FAKE, 3, None, FAKE, FAKE, FAKE, 5, FAKE, FAKE, FAKE, ws, need, None) == E
    assert u(FAKE, 3, FAKE, FAKE, FAKE + 4, FAKE, 5, FAKE, FAKE, FAKE, ws, need, None) == E  # misaligned
    assert u(FAKE, 3, FAKE, FAKE, FAKE, FAKE, 5, FAKE, FAKE, FAKE, ws, need - 1, None) == Wk
    assert u(FAKE, 3, FAKE, FAKE, FAKE, FAKE, 5, FAKE, FAKE, FAKE, ws + 16, need, None) == Wk
    assert u(FAKE, 3, FAKE, FAKE, FAKE, FAKE, 5, FAKE, FAKE, FAKE, None, need, None) == Wk
    assert u(None, 0, None, None, None, None, 5, None, None, None, None, 0, None) == 0


def test_lk_order_validation(L):
    E = ops_err("OT_E_INVAL")
    o = L.ot_lk_order
    assert o(FAKE, -1, 4, FAKE, None) == E
    assert o(FAKE, 10, 0, FAKE, None) == E
    assert o(FAKE, 10, 9, FAKE, None) == E
    assert o(None, 10, 4, FAKE, None) == E
    assert o(FAKE, 10, 4, None, None) == E
    assert o(None, 0, 4, None, None) == 0


def test_box_scaled_noalloc_validation(L):
    """Argument errors of the allocation-free form return before any device
    call: too many boxes for the static scratch, negative counts, nulls,
    misalignment; m == 0 is a no-op."""
    E = ops_err("OT_E_INVAL")
    u = L.ot_box_update_scaled_noalloc
    mx = ops.SCALED_NOALLOC_MAX_BOXES
    txt = open(HEADER).read()
    assert re.search(r"#define OT_SCALED_NOALLOC_MAX_BOXES (\d+)", txt).group(1) == str(mx)
    assert u(FAKE, mx + 1, FAKE, FAKE, FAKE, FAKE, 5, FAKE, FAKE, FAKE, None) == E
    assert u(FAKE, -1, FAKE, FAKE, FAKE, FAKE, 5, FAKE, FAKE, FAKE, None) == E
    assert u(FAKE, 3, FAKE, FAKE, FAKE, FAKE, -5, FAKE, FAKE, FAKE, None) == E
    assert u(FAKE, 3, FAKE, FAKE, FAKE, FAKE, 5, FAKE, FAKE, None, None) == E
    assert u(FAKE, 3, None, FAKE, FAKE, FAKE, 5, FAKE, FAKE, FAKE, None) == E
    assert u(FAKE, 3, FAKE, FAKE, FAKE + 4, FAKE, 5, FAKE, FAKE, FAKE, None) == E
    assert u(None, 0, None, None, None, None, 5, None, None, None, None) == 0


def test_scale_cap_matches_header():
    txt = open(HEADER).read()
    assert re.search(r"#define OT_SCALE_MAX_POINTS (\d+)", txt).group(1) == str(ops.SCALE_MAX_POINTS)


def make_cfg(**kw):
    c = ops.OtBatchCfg(win=21, iters=30, eps=0.01, min_eig=6.5025, margin=0, lk_waves=0,
                       chunk=1, max_jobs=4, max_points=5000, max_boxes=64, max_tiles=4096,
                       max_levels=5, exact_grids=0)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def make_job(L, W, H, levels, n, m, base):
    _, prev = layout(L, W=W, H=H, pitch=W, levels=levels)
    j = ops.OtJob()
    j.prev = prev
    j.next_frame = base
    j.next_pitch = W
    j.next_ws = base + (1 << 24)
    j.next_ws_bytes = ops.pyramid_bytes(W, H, levels)
    j.levels = levels
    j.pts, j.n, j.next_pts, j.status, j.err = base + 256, n, base + 512, base + 768, 0
    j.boxes, j.m, j.box_id = base + 1024, m, base + 1280
    j.out_boxes, j.out_count = base + 1536, base + 1792
    return j


def test_batch_pack_table(L):
    cfg = make_cfg()
    nb = L.ot_batch_table_bytes(C.byref(cfg))
    assert nb > 0 and nb % 256 == 0
    jobs = (ops.OtJob * 3)(make_job(L, 720, 576, 4, 100, 3, FAKE),
                           make_job(L, 1920, 1080, 5, 0, 0, FAKE + (1 << 28)),
                           make_job(L, 1280, 720, 4, 2500, 7, FAKE + (2 << 28)))
    buf = np.zeros(nb, np.uint8)
    nxt = (ops.OtPyr * 3)()
    rc = L.ot_batch_pack(jobs, 3, C.byref(cfg), buf.ctypes.data, nb, nxt)
    assert rc == 0
    hdr = buf[:64].view(np.int32)
    assert hdr[0] == 3 and hdr[1] == 2600 and hdr[2] == 10 and hdr[3] == 4
    # fused pyramid stage from level 0 (index 1): 16x8 tiles of level 3 of each job,
    # ceil(90/16)*ceil(72/8) + ceil(240/16)*ceil(135/8) + ceil(160/16)*ceil(90/8);
    # stage from level 3 (index 4): level 4 of the 5-level job only, ceil(120/16)*ceil(68/8)
    assert hdr[4 + 1] == 6 * 9 + 15 * 17 + 10 * 12
    assert hdr[4 + 2] == 0 and hdr[4 + 3] == 0
    assert hdr[4 + 4] == 8 * 9
    assert nxt[1].levels == 5 and nxt[1].level[0] == FAKE + (1 << 28)
    assert nxt[2].w[3] == 160
    # capacity and validation errors leave nothing half-written
    buf2 = np.full(nb, 7, np.uint8)
    small = make_cfg(max_points=1000)
    assert L.ot_batch_pack(jobs, 3, C.byref(small), buf2.ctypes.data, nb, None) == ops_err("OT_E_WORKSPACE")
    assert np.all(buf2 == 7)
    assert L.ot_batch_pack(jobs, 5, C.byref(make_cfg()), buf2.ctypes.data, nb, None) == ops_err("OT_E_WORKSPACE")
    jobs[0].next_ws_bytes = 10
    assert L.ot_batch_pack(jobs, 3, C.byref(cfg), buf2.ctypes.data, nb, None) == ops_err("OT_E_WORKSPACE")
    assert np.all(buf2 == 7)
    persistent = make_cfg(max_points=0, lk_waves=1024, chunk=4)
    jobs[0].next_ws_bytes = ops.pyramid_bytes(720, 576, 4)
    assert L.ot_batch_pack(jobs, 3, C.byref(persistent), buf.ctypes.data, nb, None) == 0


def test_batch_run_validation(L):
    cfg = make_cfg()
    nb = L.ot_batch_table_bytes(C.byref(cfg))
    buf = np.zeros(nb, np.uint8)
    assert L.ot_batch_run(buf.ctypes.data, FAKE + 16, nb, C.byref(cfg), None) == ops_err("OT_E_WORKSPACE")
    assert L.ot_batch_run(buf.ctypes.data, FAKE, nb - 256, C.byref(cfg), None) == ops_err("OT_E_WORKSPACE")
    assert L.ot_batch_run(None, FAKE, nb, C.byref(cfg), None) == ops_err("OT_E_INVAL")
    assert L.ot_batch_table_bytes(C.byref(make_cfg(max_jobs=0))) == 0
    rs = L.ot_batch_run_stages
    for bad in (0, 4, -1):
        assert rs(buf.ctypes.data, FAKE, nb, C.byref(cfg), bad, None) == ops_err("OT_E_INVAL")
    assert rs(buf.ctypes.data, FAKE + 16, nb, C.byref(cfg), 1, None) == ops_err("OT_E_WORKSPACE")
    assert rs(None, FAKE, nb, C.byref(cfg), 2, None) == ops_err("OT_E_INVAL")


def test_strerror(L):
    for code in ops.ERRORS:
        assert ops.strerror(code)
    assert ops.version() >= 100


def test_working_level_policy(L):
    import oracle
    for W in list(range(1, 5000, 13)) + [720, 1280, 1281, 2560, 2561, 3840]:
        assert L.ot_working_level(W, 10, 1280) == oracle.working_level(W, 10, 1280)
    assert L.ot_working_level(0, 10, 1280) == -1 and L.ot_working_level(10, 10, 0) == -1


def test_tvl1_validation(L):
    E, Wk = ops_err("OT_E_INVAL"), ops_err("OT_E_WORKSPACE")
    p = ops.OtTvl1Params()
    L.ot_tvl1_default_params(C.byref(p))
    assert (p.levels, p.warps, p.iters, p.iters_s) == (5, 5, 30, 50)
    n = 720 * 576
    al = lambda v: (v + 255) // 256 * 256
    # level-0 planes (4 structure duals, data, 2 flows, 2 flow duals), then per
    # level of an 8-level pyramid two textures and a gradient
    per_level, w, h = 0, 720, 576
    for _ in range(8):
        per_level += 2 * al(4 * w * h) + al(8 * w * h)
        w, h = (w + 1) // 2, (h + 1) // 2
    assert L.ot_tvl1_bytes(720, 576) == 4 * al(8 * n) + al(16 * n) + 2 * al(8 * n) + 2 * al(16 * n) + per_level
    assert L.ot_tvl1_bytes(0, 5) == 0
    _, P = layout(L, levels=5)
    need = L.ot_tvl1_bytes(720, 576)
    call = lambda prm, ws=FAKE, wsb=need, flow=FAKE: L.ot_tvl1_flow(C.byref(P), C.byref(P), C.byref(prm), ws,
                                                                    wsb, flow, None)
    for k, v in (("levels", 0), ("levels", 6), ("warps", 0), ("iters", 0), ("tau", 0.3),
                 ("lam", float("nan")), ("theta", 0.0), ("tau_s", 0.0), ("iters_s", -1)):
        q = ops.OtTvl1Params()
        C.memmove(C.byref(q), C.byref(p), C.sizeof(p))
        setattr(q, k, v)
        assert call(q) == E, k
    assert call(p, wsb=need - 1) == Wk
    assert call(p, ws=FAKE + 16) == Wk
    assert call(p, flow=None) == E
    # the async form validates the same way before it touches either stream
    acall = lambda prm, ws=FAKE, wsb=need, flow=FAKE: L.ot_tvl1_flow_async(
        C.byref(P), C.byref(P), C.byref(prm), ws, wsb, flow, None, None)
    q = ops.OtTvl1Params()
    C.memmove(C.byref(q), C.byref(p), C.sizeof(p))
    q.levels = 0
    assert acall(q) == E
    assert acall(p, wsb=need - 1) == Wk
    assert acall(p, flow=None) == E
    # one frame's texture buffer and the flow from two of them
    tb = L.ot_tvl1_texture_bytes(720, 576)
    per_level, w, h = 0, 720, 576
    for _ in range(8):
        per_level += al(4 * w * h) + al(8 * w * h)
        w, h = (w + 1) // 2, (h + 1) // 2
    assert tb == 2 * al(8 * n) + per_level
    assert L.ot_tvl1_texture_bytes(0, 3) == 0
    tcall = lambda prm, tex=FAKE, tbytes=tb: L.ot_tvl1_texture(C.byref(P), C.byref(prm), tex,
                                                              tbytes, None)
    assert tcall(q) == E                     # levels 0
    q.levels = 6                             # more levels than the pyramid holds
    assert tcall(q) == E
    assert tcall(p, tex=None) == E
    assert tcall(p, tbytes=tb - 1) == Wk
    assert tcall(p, tex=FAKE + 64) == Wk
    fcall = lambda prm, pt=FAKE, nt=FAKE, ws=FAKE, wsb=need, flow=FAKE: L.ot_tvl1_flow_tex(
        C.byref(P), C.byref(P), pt, nt, C.byref(prm), ws, wsb, flow, None)
    assert fcall(q) == E
    assert fcall(p, pt=None) == E
    assert fcall(p, nt=FAKE + 16) == Wk
    assert fcall(p, wsb=need - 1) == Wk
    assert fcall(p, flow=None) == E
    assert L.ot_box_mean_flow(FAKE, 10, 10, FAKE, -1, FAKE, FAKE, None) == E
    assert L.ot_box_mean_flow(FAKE + 4, 10, 10, FAKE, 3, FAKE, FAKE, None) == E
    assert L.ot_box_mean_flow(None, 10, 10, None, 0, None, None, None) == 0


class _FakeDev:
    """Stands in for a device tensor: an address, a shape and a row stride
    (ot_batch_pack reads only these and never dereferences them)."""

    def __init__(self, addr, shape, stride0=1, nbytes=None):
        self.addr, self.shape, self._s0 = addr, shape, stride0
        self._numel = nbytes if nbytes is not None else int(np.prod(shape))

    def data_ptr(self):
        return self.addr

    def stride(self, i):
        return self._s0

    def numel(self):
        return self._numel


def test_fit_capacities_finds_the_smallest_tiles(L):
    """batch.fit_capacities: totals for jobs, points and boxes, and the
    smallest tile capacity the fused pyramid stages fit (bisection with
    ot_batch_pack): the same three jobs as above need 54 + 255 + 120 = 429
    tiles in their first stage and 72 in the second."""
    from types import SimpleNamespace
    from paper_1910_06017_amd import batch

    def job(W, H, levels, n, m, base):
        _, prev = layout(L, W=W, H=H, pitch=W, levels=levels)
        return batch.Job(prev=SimpleNamespace(desc=prev),
                         next_frame=_FakeDev(base, (H, W), W),
                         next_ws=_FakeDev(base + (1 << 24), (1,),
                                          nbytes=ops.pyramid_bytes(W, H, levels)),
                         levels=levels, pts=_FakeDev(base + 256, (n, 2)),
                         next_pts=_FakeDev(base + 512, (n, 2)), status=_FakeDev(base + 768, (n,)),
                         err=None, boxes=_FakeDev(base + 1024, (m, 4)),
                         box_id=_FakeDev(base + 1280, (n,)), out_boxes=_FakeDev(base + 1536, (m, 4)),
                         out_count=_FakeDev(base + 1792, (m,)))

    jobs = [job(720, 576, 4, 100, 3, FAKE), job(1920, 1080, 5, 0, 0, FAKE + (1 << 28)),
            job(1280, 720, 4, 2500, 7, FAKE + (2 << 28))]
    cfg = batch.fit_capacities(batch.BatchConfig(max_tiles=1 << 15), jobs)
    assert (cfg.max_jobs, cfg.max_points, cfg.max_boxes, cfg.max_tiles) == (3, 2600, 10, 429)
    with pytest.raises(ValueError):
        batch.fit_capacities(batch.BatchConfig(max_tiles=400), jobs)
