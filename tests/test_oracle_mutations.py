"""Planted mistakes in a copy of the oracle must each fail at least one pin.

Each case edits one expression of the oracle's C source (a dropped term, a
wrong sign, a swapped operand, a wrong constant), compiles the copy with the
oracle's own flags into a temporary library, and runs the pins against it.
CPU only; the real oracle is untouched.
"""
import os

import pytest

import oracle
import oracle_pins as P

SRC = os.path.join(os.path.dirname(oracle.__file__), "omnitrack_oracle.c")

MUTATIONS = {
    "mismatch_sign": ("double d = A[k] - B;", "double d = B - A[k];"),
    "b_uses_wrong_gradient": ("bx += d * X[k];", "bx += d * Y[k];"),
    "inverse_offdiag_sign": ("(G2 * bx - G1 * by)", "(G2 * bx + G1 * by)"),
    "coarse_to_fine_no_doubling_x": ("gx = 2.0 * (gx + nux);", "gx = (gx + nux);"),
    "coarse_to_fine_no_doubling_y": ("gy = 2.0 * (gy + nuy);", "gy = (gy + nuy);"),
    "level_scale": ("const double cx = ux / scale", "const double cx = ux / (scale + 0.5)"),
    "window_template_offset": ("A[k] = orc_bilinear_u8(C->prev[l], w, h, cx + ox, cy + oy);",
                               "A[k] = orc_bilinear_u8(C->prev[l], w, h, cx + oy, cy + ox);"),
    "pyramid_rounding": ("(uint8_t)((s + 128) >> 8)", "(uint8_t)((s + 127) >> 8)"),
    "pyramid_kernel": ("K5[5] = {1, 4, 6, 4, 1}", "K5[5] = {1, 4, 6, 4, 2}"),
    "scharr_weights": ("S3[3] = {3, 10, 3}", "S3[3] = {3, 10, 4}"),
    "bilinear_weights_swapped": ("a * (1 - b) * f10 + (1 - a) * b * f01",
                                 "(1 - a) * b * f10 + a * (1 - b) * f01"),
    "gradient_scale": ("/ 32.0;\n                Y[k]", "/ 16.0;\n                Y[k]"),
    "gate_divisor": ("double lam = orc_min_eig(Gm) / N;", "double lam = orc_min_eig(Gm) / (N + 1);"),
    "gate_ignored": ("if (!(lam >= C->min_eig))", "if (!(lam >= 0.0))"),
    "eigen_sign": ("return m - sqrt(d * d + G[1] * G[1]);", "return m + sqrt(d * d + G[1] * G[1]);"),
    "err_normaliser": ("*err = e / N;", "*err = e / (N - 1);"),
    "even_median": ("0.5 * (v[c / 2 - 1] + v[c / 2])", "v[c / 2]"),
    "box_lost_points_counted": ("box_id[i] == b && status[i] == 1", "box_id[i] == b"),
    "out_of_frame_check": ("nx > W0 - 1 || ny > H0 - 1)", "nx > W0 + 5 || ny > H0 + 5)"),
    "convergence_test": ("if (ex * ex + ey * ey < C->eps * C->eps) break;",
                         "if (ex * ex + ey * ey < C->eps) break;"),
    "fb_threshold_exclusive": ("status_out[i] = (e <= fb_max) ? 1 : 0;",
                               "status_out[i] = (e < fb_max) ? 1 : 0;"),
    "fb_error_manhattan": ("const double e = sqrt(ex * ex + ey * ey);",
                           "const double e = fabs(ex) + fabs(ey);"),
    "fb_ignores_backward_status": ("if (st_fwd[i] == 1 && st_bwd[i] == 1) {",
                                   "if (st_fwd[i] == 1) {"),
    "scale_ratio_inverted": ("r[nr++] = sqrt(vx * vx + vy * vy) / du;",
                             "r[nr++] = du / sqrt(vx * vx + vy * vy);"),
    "scale_keeps_coincident_pairs": ("if (du == 0.0) continue;", "(void)0;"),
    "scale_skips_adjacent_pairs": ("for (int32_t q = a + 1; q < c; ++q) {",
                                   "for (int32_t q = a + 2; q < c; ++q) {"),
    "scale_about_corner": ("out_boxes[4 * b + 0] = cx - s * hw;",
                           "out_boxes[4 * b + 0] = cx - hw;"),
}


def _run_pins():
    failed = []
    for chk in P.ALL + [lambda: P.check_pyr_down_library(direct=True)]:
        try:
            chk()
        except AssertionError:
            failed.append(getattr(chk, "__name__", "pin"))
    return failed


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(orc, tmp_path, name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old!r}"
    mutated = tmp_path / "mut.c"
    mutated.write_text(src.replace(old, new, 1))
    lib = oracle.compile_to(str(mutated), str(tmp_path / "libmut.so"))
    with oracle.use_library(lib):
        failed = _run_pins()
    assert failed, f"no pin caught the planted mistake {name}"


# Planted mistakes in a copy of the matching/update oracle (Python source).
MATCH_SRC = os.path.join(os.path.dirname(oracle.__file__), "matching.py")
GREEDY = '''

def _greedy(gain):
    g = gain.copy()
    rows, cols = [], []
    while g.size and g.max() > 0:
        r, c = divmod(int(g.argmax()), g.shape[1])
        rows.append(r)
        cols.append(c)
        g[r, :] = 0
        g[:, c] = 0
    return rows, cols
'''

MATCH_MUTATIONS = {
    "iou_union_keeps_intersection": ("box_area(a) + box_area(b) - inter", "box_area(a) + box_area(b)", ""),
    "iou_intersection_uses_max": ("ix = max(0.0, min(float(a[2]), float(b[2]))",
                                  "ix = max(0.0, max(float(a[2]), float(b[2]))", ""),
    "iou_negative_overlap": ("iy = max(0.0, ", "iy = abs(", ""),
    "area_from_x_only": ("* max(0.0, float(b[3]) - float(b[1]))", "* max(0.0, float(b[2]) - float(b[0]))", ""),
    "assign_greedy": ("rows, cols = scipy.optimize.linear_sum_assignment(gain, maximize=True)",
                      "rows, cols = _greedy(gain)", GREEDY),
    "assign_minimizes": ("maximize=True", "maximize=False", ""),
    "assign_threshold_exclusive": ("if w[r, c] >= iou_min:", "if w[r, c] > iou_min:", ""),
    "assign_ignores_threshold": ("gain = np.where(w >= iou_min, w, 0.0)", "gain = w", ""),
    "update_no_lost_flag": ("            lost[i] = 1", "            pass", ""),
    "update_no_new_objects": ("if d2s[j] < 0:", "if False:", ""),
    "update_keeps_predicted_box": ("boxes[i] = det[s2d[i]].copy()", "pass", ""),
    "update_revives_lost": ("        if lost[i]:\n            continue\n", "", ""),
}


def _python_mutant_caught(tmp_path, src_path, names, old, new, extra, pins):
    """Load a mutated copy of an oracle Python module, route the oracle's
    functions `names` to it, and report whether any pin fails."""
    import importlib.util
    src = open(src_path).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old!r}"
    path = tmp_path / "oracle_mut.py"
    path.write_text(src.replace(old, new, 1) + extra)
    spec = importlib.util.spec_from_file_location("oracle_mut", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    saved = {n: getattr(oracle, n) for n in names}
    failed = []
    try:
        for n in names:
            setattr(oracle, n, getattr(mod, n))
        for chk in pins:
            try:
                chk()
            except AssertionError:
                failed.append(chk.__name__)
    finally:
        for n, f in saved.items():
            setattr(oracle, n, f)
    return failed


@pytest.mark.parametrize("name", sorted(MATCH_MUTATIONS))
def test_planted_matching_mistake_is_caught(tmp_path, name):
    old, new, extra = MATCH_MUTATIONS[name]
    failed = _python_mutant_caught(tmp_path, MATCH_SRC, ["iou", "iou_matrix", "assign", "track_update"],
                                   old, new, extra, P.MATCHING)
    assert failed, f"no pin caught the planted mistake {name}"


WORKING_SRC = os.path.join(os.path.dirname(oracle.__file__), "working.py")
WORKING_MUTATIONS = {
    "halving_floors": ("w = -(-w // 2)", "w = w // 2"),
    "first_level_over": ("while w > max_width:", "while w >= max_width:"),
    "points_not_scaled_in": ("np.asarray(pts, np.float32) * s", "np.asarray(pts, np.float32)"),
    "results_not_scaled_out": ("r.next_pts = r.next_pts * 2.0 ** base", "r.next_pts = r.next_pts"),
    "wrong_level_slice": ("oracle.pyramid(frame1, base + levels)[base:]",
                          "oracle.pyramid(frame1, base + levels + 1)[base + 1:]"),
}


@pytest.mark.parametrize("name", sorted(WORKING_MUTATIONS))
def test_planted_working_level_mistake_is_caught(orc, tmp_path, name):
    old, new = WORKING_MUTATIONS[name]
    failed = _python_mutant_caught(tmp_path, WORKING_SRC, ["working_level", "lk_track_working"],
                                   old, new, "", P.WORKING)
    assert failed, f"no pin caught the planted mistake {name}"


TVL1_SRC = os.path.join(os.path.dirname(oracle.__file__), "tvl1.py")
TVL1_MUTATIONS = {
    "grad_backward": ("gx[:, :-1] = u[:, 1:] - u[:, :-1]", "gx[:, 1:] = u[:, 1:] - u[:, :-1]"),
    "div_keeps_last_column": ("qx[:, -1] = 0.0", "pass"),
    "rof_sign": ("return f - theta * div(px, py)", "return f + theta * div(px, py)"),
    "texture_ignores_alpha": ("f - prm.alpha * rof(", "f - rof("),
    "threshold_sign": ("s[lo] = lam_theta", "s[lo] = -lam_theta"),
    "projection_sign": ("s[mid] = -rho[mid] / g2[mid]", "s[mid] = rho[mid] / g2[mid]"),
    "no_dual_projection": ("n = np.maximum(1.0, np.sqrt(qx * qx + qy * qy))", "n = 1.0"),
    "warp_sign": ("wx = xs + u1", "wx = xs - u1"),
    "upsample_no_doubling": ("return 2.0 * bilinear_clamped", "return bilinear_clamped"),
    "primal_sign": ("u1 = v1 + prm.theta * div(p[0], p[1])", "u1 = v1 - prm.theta * div(p[0], p[1])"),
    "linearisation_sign": ("rho0 = I1w - gx * u1 - gy * u2 - I0", "rho0 = I1w + gx * u1 + gy * u2 - I0"),
    "central_gradient_no_half": ("return 0.5 * (xp - xm), 0.5 * (yp - ym)", "return (xp - xm), (yp - ym)"),
    "central_gradient_x_no_half": ("return 0.5 * (xp - xm), 0.5 * (yp - ym)", "return (xp - xm), 0.5 * (yp - ym)"),
    "central_gradient_forward": ("return 0.5 * (xp - xm), 0.5 * (yp - ym)", "return (xp - img), (yp - img)"),
    "central_gradient_axes_swapped": ("return 0.5 * (xp - xm), 0.5 * (yp - ym)", "return 0.5 * (yp - ym), 0.5 * (xp - xm)"),
    "central_gradient_wraps": ("xp = np.concatenate([img[:, 1:], img[:, -1:]], axis=1)", "xp = np.roll(img, -1, axis=1)"),
    "box_excludes_right_edge": ("min(W - 1, int(np.floor(x1)))", "min(W - 1, int(np.floor(x1)) - 1)"),
}


@pytest.mark.parametrize("name", sorted(TVL1_MUTATIONS))
def test_planted_tvl1_mistake_is_caught(orc, tmp_path, name):
    import importlib.util
    old, new = TVL1_MUTATIONS[name]
    src = open(TVL1_SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old!r}"
    path = tmp_path / "tvl1_mut.py"
    path.write_text(src.replace(old, new, 1))
    import sys
    spec = importlib.util.spec_from_file_location("tvl1_mut", str(path))
    mod = importlib.util.module_from_spec(spec)
    sys.modules["tvl1_mut"] = mod          # dataclasses look their module up
    try:
        spec.loader.exec_module(mod)
    finally:
        sys.modules.pop("tvl1_mut", None)
    saved = oracle.tvl1
    failed = []
    try:
        oracle.tvl1 = mod
        for chk in P.TVL1:
            try:
                chk()
            except AssertionError:
                failed.append(chk.__name__)
    finally:
        oracle.tvl1 = saved
    assert failed, f"no pin caught the planted mistake {name}"
