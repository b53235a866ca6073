"""The C ABI on the host: the library loads, exports every declared symbol, and
rejects bad arguments before any GPU work (no device needed, no kernel launched)."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "scene_gather.h")
HEADERS = [os.path.join(ROOT, "include", n) for n in sorted(os.listdir(os.path.join(ROOT, "include")))
           if n.endswith(".h")]


@pytest.fixture(scope="module")
def native():
    from paper_2102_03011_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        from paper_2102_03011_amd import build
        build.build()
    return _native, _native.load()


def _declared_functions(path):
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if not n.startswith("SCENE")))


def test_header_functions_are_exported(native):
    mod, lib = native
    assert len(HEADERS) == 4
    names = [n for h in HEADERS for n in _declared_functions(h)]
    assert len(names) >= 16
    assert {"scene_depth_workspace_size", "scene_estimate_depth"} <= set(names)
    assert {"scene_frustum_workspace_size", "scene_frustum_count", "scene_frustum_scatter"} <= set(names)
    assert {"scene_frame_sharpness", "scene_filter_frames", "scene_inpaint", "scene_box_mask"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
        assert n in mod.SIGNATURES, n


def test_header_constants_match_binding_and_bound_the_gather_reads():
    """The binding's copies of the header's limits and layout constants agree, and
    the apron holds every block the gather reads: a projection is kept when its
    block centre is at most r outside the image, so blocks reach 2r beyond it on
    every side."""
    from paper_2102_03011_amd import _native
    text = open(HEADER).read()
    defs = {k: int(v, 0) for k, v in re.findall(r"^#define (SG_[A-Z_]+) \(?([0-9x]+)", text, flags=re.M)}
    for name in ("SG_APRON", "SG_APRON_RIGHT", "SG_MAX_RADIUS", "SG_MAX_WINDOW", "SG_ID_SHIFT"):
        assert getattr(_native, name) == defs[name], name
    ftext = open(os.path.join(ROOT, "include", "scene_filters.h")).read()
    assert _native.SG_MAX_INPAINT_STEPS == int(re.search(r"#define SG_MAX_INPAINT_STEPS (\d+)", ftext).group(1))
    for r in range(defs["SG_MAX_RADIUS"] + 1):
        assert defs["SG_APRON"] >= 2 * r, r
        # rightmost centre x = W - 1 + r; its block's last column lies 2r past the image
        assert defs["SG_APRON_RIGHT"] >= 2 * r, r


def test_version_and_status_strings(native):
    mod, lib = native
    assert lib.sg_version() == 1
    assert lib.sg_status_string(0) == b"ok"
    assert lib.sg_status_string(mod.SG_E_INVALID) == b"invalid argument"
    assert lib.sg_status_string(99) == b"unknown status"


def _clip(mod, w=64, h=32, n=10, fx=50.0):
    # fake, never dereferenced device addresses: every call below fails validation first
    return mod.SgClip(w, h, n, 0, 0x10000, 0x20000, 0x30000, fx, fx, (w - 1) / 2, (h - 1) / 2)


def _sets(mod, cap=0):
    return mod.SgSampleSets(0x40000, 0x50000 if cap else None, 0x60000 if cap else None, cap, 0x70000)


def test_workspace_size(native):
    mod, lib = native
    c = _clip(mod)
    out = ctypes.c_size_t(0)
    p = mod.SgGatherParams(3, 1, 0.01, 0.01)
    assert lib.scene_gather_workspace_size(ctypes.byref(c), 0, 10, ctypes.byref(p), ctypes.byref(out)) == 0
    big = out.value
    assert big >= 10 * 7 * 16 * 4
    assert lib.scene_gather_workspace_size(ctypes.byref(c), 0, 1, ctypes.byref(p), ctypes.byref(out)) == 0
    assert 0 < out.value < big


@pytest.mark.parametrize("case,expect", [
    ("null_clip", 1), ("f_empty", 1), ("f_past_end", 1), ("neg_window", 1), ("neg_radius", 1),
    ("big_window", 4), ("big_radius", 4), ("tol_zero", 1), ("tol_nan", 1), ("znear_neg", 1),
    ("too_many_pixels", 4), ("zero_fx", 1), ("null_sets", 1), ("null_ws", 1), ("small_ws", 1),
    ("neg_capacity", 1), ("null_arena", 1), ("null_rgbd", 1), ("rgbd_unaligned", 1), ("depth_unaligned", 1),
])
def test_gather_rejects_bad_arguments(native, case, expect):
    mod, lib = native
    c = _clip(mod)
    p = mod.SgGatherParams(3, 1, 0.01, 0.01)
    s = _sets(mod, 100)
    f0, f1, ws, wsb = 2, 4, 0x80000, 1 << 20
    cp = ctypes.byref(c)
    if case == "null_clip":
        cp = None
    elif case == "f_empty":
        f1 = f0
    elif case == "f_past_end":
        f1 = 11
    elif case == "neg_window":
        p.window = -1
    elif case == "neg_radius":
        p.radius = -1
    elif case == "big_window":
        p.window = 512
    elif case == "big_radius":
        p.radius = 4
    elif case == "tol_zero":
        p.tol = 0.0
    elif case == "tol_nan":
        p.tol = math.nan
    elif case == "znear_neg":
        p.z_near = -0.01
    elif case == "too_many_pixels":
        c.width, c.height = 4097, 1024
    elif case == "zero_fx":
        c.fx = 0.0
    elif case == "null_sets":
        s = None
    elif case == "null_ws":
        ws = None
    elif case == "small_ws":
        wsb = 16
    elif case == "neg_capacity":
        s.capacity = -1
    elif case == "null_arena":
        s.ids = None
    elif case == "null_rgbd":
        c.rgbd = None
    elif case == "rgbd_unaligned":      # 8-byte pixels
        c.rgbd = 0x10004
    elif case == "depth_unaligned":     # 32-bit row-pair words
        c.depth = 0x20002
    sp = ctypes.byref(s) if s is not None else None
    for fn in (lib.scene_gather, lib.scene_gather_scatter):
        assert fn(cp, f0, f1, ctypes.byref(p), sp, ws, wsb, None) == expect, (case, fn)
    if case not in ("neg_capacity", "null_arena"):
        assert lib.scene_gather_count(cp, f0, f1, ctypes.byref(p), sp, ws, wsb, None) == expect, case


@pytest.mark.parametrize("case", ["neg_window", "sigma_zero", "sigma_nan", "null_out", "null_sets", "bad_range"])
def test_filter_rejects_bad_arguments(native, case):
    mod, lib = native
    c = _clip(mod)
    s = _sets(mod, 100)
    fp = mod.SgFilterParams(0.01, math.inf, math.inf, 0.0)
    w, out, f0, f1 = 3, 0x90000, 0, 2
    sp = ctypes.byref(s)
    if case == "neg_window":
        w = -1
    elif case == "sigma_zero":
        fp.sigma_d = 0.0
    elif case == "sigma_nan":
        fp.sigma_c = math.nan
    elif case == "null_out":
        out = None
    elif case == "null_sets":
        sp = None
    elif case == "bad_range":
        f1 = 0
    assert lib.scene_filter(ctypes.byref(c), f0, f1, w, sp, ctypes.byref(fp), out, None) == 1


@pytest.mark.parametrize("case", ["null_clip", "bad_range", "big_radius", "null_fparams", "sigma_zero", "null_out",
                                  "null_ws", "small_ws"])
def test_gather_filter_rejects_bad_arguments(native, case):
    mod, lib = native
    c = _clip(mod)
    p = mod.SgGatherParams(3, 1, 0.01, 0.01)
    fp = mod.SgFilterParams(0.01, math.inf, math.inf, 0.0)
    f0, f1 = 0, 2
    need = ctypes.c_size_t(0)
    assert lib.scene_gather_workspace_size(ctypes.byref(c), f0, f1, ctypes.byref(p), ctypes.byref(need)) == 0
    cp, fpp, out, ws, wsb, expect = ctypes.byref(c), ctypes.byref(fp), 0x90000, 0xA0000, need.value, 1
    if case == "null_clip":
        cp = None
    elif case == "bad_range":
        f1 = 0
    elif case == "big_radius":
        p.radius, expect = 4, 4
    elif case == "null_fparams":
        fpp = None
    elif case == "sigma_zero":
        fp.sigma_d = 0.0
    elif case == "null_out":
        out = None
    elif case == "null_ws":
        ws = None
    elif case == "small_ws":
        wsb -= 1
    assert lib.scene_gather_filter(cp, f0, f1, ctypes.byref(p), fpp, out, ws, wsb, None) == expect, case


def test_range_beyond_the_int_grid_is_unsupported(native):
    # 1 x 2^22 frames: 2^20 tiles of 64 x 4 per output frame, so 2047 output frames
    # fit an int-indexed grid and 2048 (2^31 tiles) do not
    mod, lib = native
    c = _clip(mod, w=1, h=1 << 22, n=4096)
    p = mod.SgGatherParams(1, 1, 0.01, 0.01)
    fp = mod.SgFilterParams(0.01, math.inf, math.inf, 0.0)
    need = ctypes.c_size_t(0)
    assert lib.scene_gather_workspace_size(ctypes.byref(c), 0, 2047, ctypes.byref(p), ctypes.byref(need)) == 0
    assert lib.scene_gather_workspace_size(ctypes.byref(c), 0, 2048, ctypes.byref(p), ctypes.byref(need)) == 4
    assert lib.scene_gather_filter(ctypes.byref(c), 0, 2048, ctypes.byref(p), ctypes.byref(fp), 0x90000, 0xA0000,
                                   1 << 40, None) == 4


def test_frame_sharpness_rejects_bad_arguments(native):
    mod, lib = native
    c = _clip(mod)
    assert lib.scene_frame_sharpness(None, 0x90000, None) == 1
    assert lib.scene_frame_sharpness(ctypes.byref(c), None, None) == 1
    c.rgbd = None
    assert lib.scene_frame_sharpness(ctypes.byref(c), 0x90000, None) == 1
    c = _clip(mod, w=4097, h=1024)
    assert lib.scene_frame_sharpness(ctypes.byref(c), 0x90000, None) == 4


@pytest.mark.parametrize("case,expect", [
    ("ok_but_null_table", 1), ("null_sets", 1), ("null_out", 1), ("bad_range", 1), ("neg_window", 1),
    ("big_window", 4), ("sigma_zero", 1), ("null_params", 1), ("null_ids", 1), ("null_crho", 1),
    ("neg_capacity", 1),
])
def test_filter_frames_rejects_bad_arguments(native, case, expect):
    mod, lib = native
    c = _clip(mod)
    s = _sets(mod, 100)
    fp = mod.SgFilterParams(0.01, math.inf, math.inf, 0.0)
    f0, f1, w, table, out = 0, 2, 3, 0xB0000, 0x90000
    pp = ctypes.byref(fp)
    if case == "ok_but_null_table":
        table = None
    elif case == "null_sets":
        s = None
    elif case == "null_out":
        out = None
    elif case == "bad_range":
        f1 = 11
    elif case == "neg_window":
        w = -1
    elif case == "big_window":
        w = 512
    elif case == "sigma_zero":
        fp.sigma_d = 0.0
    elif case == "null_params":
        pp = None
    elif case == "null_ids":
        s.ids = None
    elif case == "null_crho":
        s.crho = None
    elif case == "neg_capacity":
        s.capacity = -1
    sp = ctypes.byref(s) if s is not None else None
    assert lib.scene_filter_frames(ctypes.byref(c), f0, f1, w, sp, pp, table, out, None) == expect, case


@pytest.mark.parametrize("case,expect", [
    ("null_mask", 1), ("sigma_zero", 1), ("sigma_nan", 1), ("sigma_inf", 1), ("steps_zero", 1),
    ("steps_big", 4), ("null_ids", 1), ("bad_range", 1), ("null_out", 1),
])
def test_inpaint_rejects_bad_arguments(native, case, expect):
    mod, lib = native
    c = _clip(mod)
    s = _sets(mod, 100)
    f0, f1, w, mask, sigma, steps, out = 0, 2, 3, 0xB0000, 0.2, 2, 0x90000
    if case == "null_mask":
        mask = None
    elif case == "sigma_zero":
        sigma = 0.0
    elif case == "sigma_nan":
        sigma = math.nan
    elif case == "sigma_inf":
        sigma = math.inf
    elif case == "steps_zero":
        steps = 0
    elif case == "steps_big":
        steps = mod.SG_MAX_INPAINT_STEPS + 1
    elif case == "null_ids":
        s.ids = None
    elif case == "bad_range":
        f0 = -1
    elif case == "null_out":
        out = None
    assert lib.scene_inpaint(ctypes.byref(c), f0, f1, w, ctypes.byref(s), mask, sigma, steps, out, None) == expect, \
        case


def test_box_mask_rejects_bad_arguments(native):
    mod, lib = native
    box = (ctypes.c_double * 6)(-1.0, -1.0, 0.5, 1.0, 1.0, 3.0)
    c = _clip(mod)
    assert lib.scene_box_mask(None, box, 0x90000, None) == 1
    assert lib.scene_box_mask(ctypes.byref(c), None, 0x90000, None) == 1
    assert lib.scene_box_mask(ctypes.byref(c), box, None, None) == 1
    for k in range(6):
        bad = (ctypes.c_double * 6)(*box)
        bad[k] = math.nan if k % 2 else math.inf
        assert lib.scene_box_mask(ctypes.byref(c), bad, 0x90000, None) == 1, k
    c.depth = None
    assert lib.scene_box_mask(ctypes.byref(c), box, 0x90000, None) == 1


@pytest.mark.parametrize("case,expect", [
    ("null_clip", 1), ("f_neg", 1), ("f_past_end", 1), ("neg_window", 1), ("big_window", 4), ("l_zero", 1),
    ("l_nan", 1), ("l_big", 4), ("near_zero", 1), ("far_below_near", 1), ("far_inf", 1), ("null_params", 1),
    ("null_depth", 1), ("null_sets", 1), ("null_status", 1), ("null_ws", 1), ("small_ws", 1),
])
def test_frustum_rejects_bad_arguments(native, case, expect):
    mod, lib = native
    c = _clip(mod)
    p = mod.SgFrustumParams(2, 3.0, 0.01, 1000.0)
    need = ctypes.c_size_t(0)
    assert lib.scene_frustum_workspace_size(ctypes.byref(c), 4, ctypes.byref(p), ctypes.byref(need)) == 0
    assert need.value > 5 * 64 * 32 * 20
    s = _sets(mod, 100)
    f, ws, wsb = 4, 0x80000, need.value
    cp, pp = ctypes.byref(c), ctypes.byref(p)
    if case == "null_clip":
        cp = None
    elif case == "f_neg":
        f = -1
    elif case == "f_past_end":
        f = 10
    elif case == "neg_window":
        p.window = -1
    elif case == "big_window":
        p.window = 512
    elif case == "l_zero":
        p.l = 0.0
    elif case == "l_nan":
        p.l = math.nan
    elif case == "l_big":
        p.l = 7.5
    elif case == "near_zero":
        p.near_z = 0.0
    elif case == "far_below_near":
        p.far_z = 0.005
    elif case == "far_inf":
        p.far_z = math.inf
    elif case == "null_params":
        pp = None
    elif case == "null_depth":
        c.depth = None
    elif case == "null_sets":
        s = None
    elif case == "null_status":
        s.status = None
    elif case == "null_ws":
        ws = None
    elif case == "small_ws":
        wsb -= 1
    sp = ctypes.byref(s) if s is not None else None
    for fn in (lib.scene_frustum_count, lib.scene_frustum_scatter):
        assert fn(cp, f, pp, sp, ws, wsb, None) == expect, (case, fn)


@pytest.mark.parametrize("case,expect", [
    ("null_clip", 1), ("f_neg", 1), ("f_past_end", 1), ("neg_window", 1), ("big_window", 4), ("null_hyp", 1),
    ("zero_hyp", 1), ("many_hyp", 4), ("null_out", 1), ("null_ws", 1), ("small_ws", 1), ("null_rgbd", 1),
])
def test_depth_rejects_bad_arguments(native, case, expect):
    mod, lib = native
    c = _clip(mod)
    need = ctypes.c_size_t(0)
    assert lib.scene_depth_workspace_size(ctypes.byref(c), 4, 2, ctypes.byref(need)) == 0
    assert need.value == 5 * 16 * 4
    f, w, hyp, n_hyp, out, ws, wsb = 4, 2, 0xB0000, 8, 0x90000, 0xA0000, need.value
    cp = ctypes.byref(c)
    if case == "null_clip":
        cp = None
    elif case == "f_neg":
        f = -1
    elif case == "f_past_end":
        f = 10
    elif case == "neg_window":
        w = -1
    elif case == "big_window":
        w = 512
    elif case == "null_hyp":
        hyp = None
    elif case == "zero_hyp":
        n_hyp = 0
    elif case == "many_hyp":
        n_hyp = mod.SG_MAX_DEPTH_HYPOTHESES + 1
    elif case == "null_out":
        out = None
    elif case == "null_ws":
        ws = None
    elif case == "small_ws":
        wsb -= 1
    elif case == "null_rgbd":
        c.rgbd = None
    assert lib.scene_estimate_depth(cp, f, w, hyp, n_hyp, out, None, ws, wsb, None) == expect, case


def test_stage_rejects_bad_arguments(native):
    mod, lib = native
    assert lib.scene_stage(None, 0x1000, 10, 64, 32, 0x2000, 0x3000, None) == 1
    assert lib.scene_stage(0x1000, 0x1000, -1, 64, 32, 0x2000, 0x3000, None) == 1
    assert lib.scene_stage(0x1000, 0x1000, 2, 0, 32, 0x2000, 0x3000, None) == 1
    assert lib.scene_stage(0x1000, 0x1000, 2, 64, 32, None, 0x3000, None) == 1
    assert lib.scene_stage(0x1000, 0x1000, 2, 4097, 1024, 0x2000, 0x3000, None) == 4
    assert lib.scene_stage(0x1000, 0x1000, 70000, 64, 32, 0x2000, 0x3000, None) == 4
    # stored planes must be aligned for the gather's reads: rgbd 8 bytes, depth 4
    assert lib.scene_stage(0x1000, 0x1000, 2, 64, 32, 0x2004, 0x3000, None) == 1
    assert lib.scene_stage(0x1000, 0x1000, 2, 64, 32, 0x2000, 0x3002, None) == 1


def _mlp(mod):
    return mod.SgMlp(0xA0000, 0xB0000)


def _train_state(mod):
    return mod.SgMlpTrain(0xC0000, 0xC1000, 0xC2000, 0xC3000, 0xC4000, 0xC5000, 0xC6000)


@pytest.mark.parametrize("case", ["null_clip", "bad_range", "neg_window", "null_sets", "null_mlp", "null_w",
                                  "null_out", "null_ws", "small_ws"])
def test_learned_filter_rejects_bad_arguments(native, case):
    mod, lib = native
    c = _clip(mod)
    p = mod.SgGatherParams(3, 1, 0.01, 0.01)
    s = _sets(mod, 100)
    m = _mlp(mod)
    cp, sp, mp = ctypes.byref(c), ctypes.byref(s), ctypes.byref(m)
    f0, f1, ws, wsb, out = 2, 4, 0x80000, 1 << 20, 0x90000
    if case == "null_clip":
        cp = None
    elif case == "bad_range":
        f1 = 1
    elif case == "neg_window":
        p.window = -2
    elif case == "null_sets":
        sp = None
    elif case == "null_mlp":
        mp = None
    elif case == "null_w":
        m.w = None
    elif case == "null_out":
        out = None
    elif case == "null_ws":
        ws = None
    elif case == "small_ws":
        wsb = 8
    assert lib.scene_filter_learned(cp, f0, f1, ctypes.byref(p), sp, mp, ws, wsb, out, None) == 1, case


@pytest.mark.parametrize("case", ["null_state", "null_master", "neg_pixels", "null_idx", "t_zero", "lr_zero",
                                  "lr_nan", "null_clean", "small_ws"])
def test_train_step_rejects_bad_arguments(native, case):
    mod, lib = native
    c = _clip(mod)
    p = mod.SgGatherParams(3, 1, 0.01, 0.01)
    s = _sets(mod, 100)
    st = _train_state(mod)
    stp = ctypes.byref(st)
    idx, n, clean, lr, t, ws, wsb = 0xD0000, 64, 0xE0000, 1e-3, 1, 0x80000, 1 << 20
    if case == "null_state":
        stp = None
    elif case == "null_master":
        st.master = None
    elif case == "neg_pixels":
        n = -1
    elif case == "null_idx":
        idx = None
    elif case == "t_zero":
        t = 0
    elif case == "lr_zero":
        lr = 0.0
    elif case == "lr_nan":
        lr = math.nan
    elif case == "null_clean":
        clean = None
    elif case == "small_ws":
        wsb = 8
    assert lib.scene_mlp_train_step(ctypes.byref(c), 2, 4, ctypes.byref(p), ctypes.byref(s), idx, n, clean, stp,
                                    lr, t, ws, wsb, None) == 1, case


def test_batch_entry_points_reject_bad_arguments(native):
    mod, lib = native
    c = _clip(mod)
    p = (mod.SgGatherParams * 2)(mod.SgGatherParams(3, 1, 0.01, 0.01), mod.SgGatherParams(3, 2, 0.01, 0.01))
    fp = (mod.SgFilterParams * 2)(mod.SgFilterParams(0.01, math.inf, math.inf, 0.0),
                                   mod.SgFilterParams(0.01, math.inf, math.inf, 0.0))
    clips = (mod.SgClip * 2)(c, c)
    n_out = (ctypes.c_int32 * 2)(1, 1)
    h = ctypes.c_void_p()
    assert lib.sg_batch_create(None, clips, 2, p, fp, n_out) == 1
    assert lib.sg_batch_create(ctypes.byref(h), clips, 0, p, fp, n_out) == 1
    assert lib.sg_batch_create(ctypes.byref(h), None, 2, p, fp, n_out) == 1
    assert lib.sg_batch_create(ctypes.byref(h), clips, 5000, p, fp, n_out) == 4
    # all clips of a batch share one radius
    assert lib.sg_batch_create(ctypes.byref(h), clips, 2, p, fp, n_out) == 4
    bad_n = (ctypes.c_int32 * 2)(1, 0)
    p[1].radius = 1
    assert lib.sg_batch_create(ctypes.byref(h), clips, 2, p, fp, bad_n) == 1
    fp[1].sigma_d = 0.0
    assert lib.sg_batch_create(ctypes.byref(h), clips, 2, p, fp, n_out) == 1
    assert h.value is None
    io = mod.SgBatchIo(0x1000, 0x2000, 0x3000, 10, 0x4000, None)
    assert lib.scene_gather_batched(None, ctypes.byref(io), None) == 1
    assert lib.sg_batch_count(None, ctypes.byref(io), None) == 1
    assert lib.sg_batch_capture(None, ctypes.byref(io), None) == 1
    assert lib.sg_batch_autotune(None, ctypes.byref(io), None, None) == 1
    assert lib.sg_batch_set_frames(None, n_out) == 1
    assert lib.sg_batch_set_config(None, 4, 1, 4) == 1
    assert lib.sg_batch_get_config(None, n_out) == 1
    assert lib.sg_batch_pixel_base(None, 0) == -1
    lib.sg_batch_destroy(None)


@pytest.mark.parametrize("case,expect", [
    ("null_clip", 1), ("f_past_end", 1), ("big_window", 4), ("null_sets", 1), ("null_arena", 1),
    ("null_rgbd", 1), ("scratch_too_small", 4),
])
def test_noalloc_gather_rejects_on_the_host(native, case, expect):
    """scene_gather_noalloc makes every host check of scene_gather before any HIP
    call, and refuses a call whose workspace exceeds its static scratch."""
    mod, lib = native
    c = _clip(mod)
    p = mod.SgGatherParams(3, 1, 0.01, 0.01)
    s = _sets(mod, 100)
    f0, f1 = 2, 4
    cp, sp = ctypes.byref(c), ctypes.byref(s)
    if case == "null_clip":
        cp = None
    elif case == "f_past_end":
        f1 = 11
    elif case == "big_window":
        p.window = 512
    elif case == "null_sets":
        sp = None
    elif case == "null_arena":
        s.ids = None
    elif case == "null_rgbd":
        c.rgbd = None
    elif case == "scratch_too_small":
        # 1000 output frames x 1023 window slots x 64 B of relative maps > 4 MiB
        c.num_frames, f0, f1, p.window = 1000, 0, 1000, 511
        need = ctypes.c_size_t(0)
        assert lib.scene_gather_workspace_size(cp, f0, f1, ctypes.byref(p), ctypes.byref(need)) == 0
        assert need.value > mod.SG_NOALLOC_SCRATCH_BYTES
    assert lib.scene_gather_noalloc(cp, f0, f1, ctypes.byref(p), sp, None) == expect, case


def test_noalloc_scratch_size_matches_header():
    from paper_2102_03011_amd import _native
    text = open(HEADER).read()
    m = re.search(r"#define SG_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m and _native.SG_NOALLOC_SCRATCH_BYTES == int(m.group(1)) << int(m.group(2))


def test_header_states_the_erf_gelu_the_oracle_and_kernels_use():
    """The MLP contract in the header is the exact erf form GELU(z) = z Phi(z), the
    function the oracle evaluates (GELU(1) = Phi(1) = 0.8413447460685429...)."""
    from oracle import learned
    text = open(HEADER).read()
    assert "GELU(z) = z Phi(z)" in text and "0.044715" not in text
    assert abs(float(learned.gelu(1.0)) - 0.8413447460685429) < 1e-15
    assert abs(float(learned.gelu(-1.0)) + (1.0 - 0.8413447460685429)) < 1e-15


def test_standardise_rejects_null_pointers(native):
    mod, lib = native
    assert lib.scene_mlp_standardise(None, 0x1000, None) == mod.SG_E_INVALID
    assert lib.scene_mlp_standardise(0x1000, None, None) == mod.SG_E_INVALID


@pytest.mark.parametrize("case", ["null_clip", "bad_range", "null_gparams", "null_sets", "null_params", "null_out",
                                  "null_ws", "small_ws", "sigma_xyz_zero", "sigma_xyz_nan", "sigma_d_zero"])
def test_filter_xyz_rejects_bad_arguments(native, case):
    mod, lib = native
    c = _clip(mod)
    g = mod.SgGatherParams(3, 1, 0.01, 0.01)
    s = _sets(mod, 100)
    fp = mod.SgFilterParams(0.01, math.inf, math.inf, 0.0)
    f0, f1, sx = 0, 2, 0.1
    need = ctypes.c_size_t(0)
    assert lib.scene_gather_workspace_size(ctypes.byref(c), f0, f1, ctypes.byref(g), ctypes.byref(need)) == 0
    cp, gp, sp, fpp, out, ws, wsb = ctypes.byref(c), ctypes.byref(g), ctypes.byref(s), ctypes.byref(fp), 0x90000, \
        0xA0000, need.value
    if case == "null_clip":
        cp = None
    elif case == "bad_range":
        f1 = 0
    elif case == "null_gparams":
        gp = None
    elif case == "null_sets":
        sp = None
    elif case == "null_params":
        fpp = None
    elif case == "null_out":
        out = None
    elif case == "null_ws":
        ws = None
    elif case == "small_ws":
        wsb -= 1
    elif case == "sigma_xyz_zero":
        sx = 0.0
    elif case == "sigma_xyz_nan":
        sx = math.nan
    elif case == "sigma_d_zero":
        fp.sigma_d = 0.0
    assert lib.scene_filter_xyz(cp, f0, f1, gp, sp, fpp, sx, None, ws, wsb, out, None) == mod.SG_E_INVALID, case


@pytest.mark.parametrize("case", ["sigma_ref_zero", "sigma_ref_nan", "sigma_rgb_inf", "null_mask", "steps_zero"])
def test_semi_transparent_rejects_bad_arguments(native, case):
    mod, lib = native
    c = _clip(mod)
    s = _sets(mod, 100)
    mask, srgb, sref, steps = 0xB0000, 0.2, 0.3, 2
    if case == "sigma_ref_zero":
        sref = 0.0
    elif case == "sigma_ref_nan":
        sref = math.nan
    elif case == "sigma_rgb_inf":
        srgb = math.inf
    elif case == "null_mask":
        mask = None
    elif case == "steps_zero":
        steps = 0
    assert lib.scene_semi_transparent(ctypes.byref(c), 0, 2, 3, ctypes.byref(s), mask, srgb, sref, steps, 0x90000,
                                      None) == mod.SG_E_INVALID, case
