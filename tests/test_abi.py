"""The C ABI library loads, exports every function the header declares, and
rejects bad arguments on the host (no GPU needed for any of this)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gs_coreset.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2607_02721_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2607_02721_amd import build
        build.build()
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("gs_sensitivity", "gs_sample_coreset", "gs_render_objective"):
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    the C compiler gives the header's struct (a field added on one side only
    shows up here, without a GPU)."""
    import shutil
    import subprocess
    from paper_2607_02721_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pairs = {"gs_scene": _lib.Scene, "gs_views": _lib.Views, "gs_params": _lib.Params, "gs_stats": _lib.Stats,
             "gs_plan_config": _lib.PlanConfig, "gs_plan_info": _lib.PlanInfo, "gs_peaks": _lib.Peaks,
             "gs_render_diag": _lib.RenderDiag}
    lines, want = [], []
    for cname, py in pairs.items():
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        want.append(C.sizeof(py))
        for f, _ in py._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
            want.append(getattr(py, f).offset)
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "gs_coreset.h"\nint main(void) {\n' +
                   "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == want


def test_library_has_no_oracle_dependency():
    from paper_2607_02721_amd import _lib
    data = open(_lib.LIB_PATH, "rb").read()
    assert b"ora_sensitivity" not in data and b"libgs_oracle" not in data


def test_status_strings(lib):
    assert lib.gs_status_string(0) == b"ok"
    assert lib.gs_status_string(4) == b"no positive sensitivity"


def _views(w=64, h=64):
    from paper_2607_02721_amd import _lib
    import synth
    v = synth.make_tiny_views(w, h)
    return _lib.HostViews(v.world_to_cam, v.intrinsics, v.size)


def _scene(n=10, deg=0, fmt=0, null=False):
    from paper_2607_02721_amd import _lib
    fake = 0 if null else 0x1000
    return _lib.Scene(n, deg, fmt, fake, fake, fake, fake, fake)


def _call_sens(lib, scene, views, params, out=0x1000):
    return lib.gs_sensitivity(C.byref(scene), C.byref(views.c) if views is not None else None,
                              C.byref(params) if params is not None else None, C.c_void_p(out), None, None)


@pytest.mark.parametrize("case,status", [
    ("n0", 1), ("deg4", 1), ("fmt7", 1), ("nullplane", 1), ("nullviews", 1), ("nullparams", 1),
    ("sigma0", 1), ("mode9", 1), ("nullout", 1), ("huge_n", 2), ("too_many_tiles", 2), ("bad_size", 1),
    ("neg_floor", 1), ("agg7", 1), ("agg_neg", 1), ("agg_pairs", 2), ("mode4", 1), ("channel_agg", 2),
])
def test_sensitivity_argument_errors(lib, case, status):
    from paper_2607_02721_amd import _lib
    sc, vw, p, out = _scene(), _views(), _lib.default_params(), 0x1000
    if case == "n0": sc = _scene(n=0)
    if case == "deg4": sc = _scene(deg=4)
    if case == "fmt7": sc = _scene(fmt=7)
    if case == "nullplane": sc = _scene(null=True)
    if case == "nullviews": vw = None
    if case == "nullparams": p = None
    if case == "sigma0": p.footprint_sigma = 0.0
    if case == "mode9": p.query_mode = 9
    if case == "nullout": out = 0
    if case == "huge_n": sc = _scene(n=1 << 28)
    if case == "too_many_tiles": vw = _views(4096, 4096)
    if case == "bad_size": vw = _views(0, 64)
    if case == "neg_floor": p.share_floor = -1.0
    if case == "agg7": p.aggregate = 7
    if case == "agg_neg": p.aggregate = -1
    if case == "mode4": p.query_mode = 4
    if case == "channel_agg":
        p.query_mode = _lib.QUERY_CHANNEL
        p.aggregate = _lib.AGG_IMAGE
    if case == "agg_pairs":
        p.aggregate = _lib.AGG_TILE
        p.flags = _lib.FLAG_COUNT_PAIRS
    assert _call_sens(lib, sc, vw, p, out) == status
    assert lib.gs_last_error()


def test_sampler_argument_errors(lib):
    f = lib.gs_sample_coreset
    ok = C.c_void_p(0x1000)
    assert f(ok, 0, 5, 0, ok, ok, ok, None) == 1
    assert f(ok, 10, 0, 0, ok, ok, ok, None) == 1
    assert f(None, 10, 5, 0, ok, ok, ok, None) == 1
    assert f(ok, 1 << 24, 5, 0, ok, ok, ok, None) == 2


def test_objective_argument_errors(lib):
    from paper_2607_02721_amd import _lib
    sc, vw, p = _scene(), _views(), _lib.default_params()
    f = lib.gs_render_objective
    assert f(C.byref(sc), C.byref(vw.c), C.byref(p), None, 1, None, None, None, None) == 1  # weights needed
    assert f(C.byref(sc), C.byref(vw.c), C.byref(p), None, 5, None, None, None, None) == 1  # objective
    p.query_mode = _lib.QUERY_CHANNEL
    assert f(C.byref(sc), C.byref(vw.c), C.byref(p), None, 0, None, None, None, None) == 2  # one query per ray


def test_default_params(lib):
    from paper_2607_02721_amd import _lib
    p = _lib.default_params()
    assert p.footprint_sigma == 3.0 and abs(p.dilation - 0.3) < 1e-7 and abs(p.z_near - 0.2) < 1e-7
    assert abs(p.share_floor - 1e-12) < 1e-18 and p.query_mode == 0 and p.ray_mask is None
    assert p.aggregate == _lib.AGG_RAY


def test_plan_argument_errors(lib):
    from paper_2607_02721_amd import _lib
    sc, vw, p = _scene(), _views(), _lib.default_params()
    scenes = (_lib.Scene * 1)(sc)
    views = (_lib.Views * 1)(vw.c)
    h = C.c_void_p(0x1234)
    f = lib.gs_plan_create
    assert f(scenes, views, 0, C.byref(p), C.byref(h), None) == 1 and h.value is None
    assert f(scenes, views, 1, C.byref(p), None, None) == 1
    assert f(None, views, 1, C.byref(p), C.byref(h), None) == 1
    p.ray_mask = 0x1000
    assert f(scenes, views, 1, C.byref(p), C.byref(h), None) == 2      # no ray masks in plans
    p = _lib.default_params()
    p.flags = 1
    assert f(scenes, views, 1, C.byref(p), C.byref(h), None) == 2      # no pair counting in plans
    p = _lib.default_params()
    p.aggregate = _lib.AGG_IMAGE
    assert f(scenes, views, 1, C.byref(p), C.byref(h), None) == 2      # per-ray queries only
    p = _lib.default_params()
    p.query_mode = _lib.QUERY_CHANNEL
    assert f(scenes, views, 1, C.byref(p), C.byref(h), None) == 2      # one query per ray
    p = _lib.default_params()
    bad = (_lib.Scene * 1)(_scene(n=0))
    assert f(bad, views, 1, C.byref(p), C.byref(h), None) == 1
    cfg = _lib.PlanConfig(0, 1)
    assert lib.gs_plan_set_config(None, C.byref(cfg)) == 1
    assert lib.gs_plan_sensitivity(None, None, None) == 1
    assert lib.gs_plan_tune(None, None, 3, None, None, None) == 1
    assert lib.gs_plan_get_info(None, None) == 1
    assert lib.gs_plan_status(None, None) == 1
    lib.gs_plan_destroy(None)


def test_learned_helper_argument_errors(lib):
    ok = C.c_void_p(0x1000)
    assert lib.gs_proposal_mixture(ok, 0, C.c_float(0.1), ok, None) == 1
    assert lib.gs_proposal_mixture(ok, 10, C.c_float(0.0), ok, None) == 1
    assert lib.gs_proposal_mixture(None, 10, C.c_float(0.1), ok, None) == 1
    assert lib.gs_log_targets(ok, 10, C.c_float(-1.0), ok, None) == 1
    assert lib.gs_log_targets(ok, 10, C.c_float(1e-6), None, None) == 1
