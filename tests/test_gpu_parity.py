"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Floating point: |s_gpu - s_oracle| <= 1e-5 s_oracle + 1e-12 for every
Gaussian, and per-ray A within 1e-5 relative, on the rays neither side flags
as ambiguous (the oracle: a pair within 1e-5 r^2 of the footprint cutoff, or
an order key within 2^-40 of a float32 rounding midpoint; the GPU: a pair
within 1e-5 r^2 of the cutoff in its own float32 arithmetic); both sides
score exactly the same unflagged rays through the ray mask.  Sampling: bit-exact
counts, weights and support given the same float32 sensitivities.
"""
import math

import numpy as np
import pytest

import parity_util
import synth

pytestmark = pytest.mark.gpu

REL, ABS = 1e-5, 1e-12


@pytest.fixture(scope="module")
def gs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_02721_amd as gs
    gs.load()
    return gs


_mask_tensor = parity_util.mask_tensor


def _parity(gs, ora, sc, vw, label, **kw):
    """Both sides score the rays outside the union of the oracle's and the
    GPU's ambiguity flags."""
    oprm = ora.default_params(**{k: v for k, v in kw.items() if k in ("query_mode", "dilation")})
    dsc = gs.DeviceScene.from_scene(sc)
    bits, oflag, gflag = parity_util.union_mask(gs, ora, sc, vw, dsc, oprm, **kw)
    ref = ora.sensitivity(sc, vw, oprm, bits)
    s, st = gs.sensitivity(dsc, vw, ray_mask=_mask_tensor(bits), stats=True, count_pairs=True, **kw)
    s = s.cpu().numpy().astype(np.float64)
    excess = np.abs(s - ref["s"]) - (REL * ref["s"] + ABS)
    worst = int(np.argmax(excess))
    print(f"[{label}] n={sc.n} flagged rays: oracle {int(oflag.sum())}, gpu {int(gflag.sum())}, "
          f"gpu only {int((gflag & ~oflag).sum())} of {vw.n_rays}; sort passes {st['sort_passes']} "
          f"max rel err={np.max(np.abs(s - ref['s']) / np.maximum(ref['s'], 1e-30)):.2e} "
          f"worst excess={excess[worst]:.2e} (s_ref={ref['s'][worst]:.3e})", flush=True)
    assert excess.max() <= 0, f"{label}: Gaussian {worst}: gpu {s[worst]!r} oracle {ref['s'][worst]!r}"
    return s, ref, st, bits


def test_tiny_scene_sensitivity_parity(gs, ora):
    sc, vw, _, _ = synth.make_config("tiny")
    s, ref, st, _ = _parity(gs, ora, sc, vw, "tiny")
    assert st["n_rays_positive"] == ref["rays_positive"]
    assert abs(st["total_sensitivity"] - ref["s"].sum()) <= 1e-5 * ref["s"].sum()


def _ragged():
    sc = synth.make_cluster_scene(20_000, 7, 3)
    vw = synth.make_orbit_views(3, 17, 200, 136)
    return sc, vw


def test_tiny_scene_sorts_in_three_passes(gs, ora):
    """Orbit views of the tiny scene see depths within a factor of four, so
    every view's keys span under 2^24 and the depth sort takes 3 passes."""
    sc, vw, _, _ = synth.make_config("tiny")
    _, st = gs.sensitivity(gs.DeviceScene.from_scene(sc), vw, stats=True)
    assert st["sort_passes"] == 3


@pytest.mark.parametrize("eye", [(1.3, 0.35, 0.25), (0.2, -0.1, 0.05)])
def test_four_pass_depth_sort_parity(gs, ora, eye):
    """A camera close to the cloud, or inside it, sees depths from z_near to
    several units: the keys span more than 2^24, the depth sort takes four
    8-bit passes, and the sensitivities still meet the bar."""
    sc, _, _, _ = synth.make_config("tiny")
    vw = synth.make_camera_set([eye, (3.0, 0.2, 0.4)], [(0.0, 0.0, 0.0), (0.0, 0.0, 0.0)], 96, 72, 70.0)
    pr = ora.project(sc, vw)
    z = pr["z"][0][pr["present"][0]]
    print(f"[4-pass {eye}] depths {z.min():.3f}..{z.max():.3f}, visible {z.size}", flush=True)
    s, ref, st, _ = _parity(gs, ora, sc, vw, f"4-pass {eye}")
    assert st["sort_passes"] == 4
    assert float(np.max(ref["s"])) > 0.5


def test_ragged_cluster_scene_parity(gs, ora):
    """Several tiles with a ragged right/bottom edge (200x136 is 12.5 x 8.5
    tiles of 16), SH degree 3, clustered means."""
    sc, vw = _ragged()
    _parity(gs, ora, sc, vw, "ragged")


def test_nocolor_mode_parity(gs, ora):
    sc, vw = _ragged()
    _parity(gs, ora, sc, vw, "nocolor", query_mode=gs.QUERY_NOCOLOR)


def test_pair_count_matches_without_stop(gs, ora):
    """share_floor = 0 evaluates every pair: in-footprint pair counts agree."""
    sc, vw, _, _ = synth.make_config("tiny")
    s, ref, st, _ = _parity(gs, ora, sc, vw, "tiny-nostop", share_floor=0.0)
    assert st["n_pairs"] == ref["pairs"]


def test_live_pair_count_close_to_oracle(gs, ora):
    """Pairs a ray still needs (T c_max >= floor A): float32 vs float64 prefix
    transmittance decide only a handful of boundary pairs differently."""
    sc, vw, _, _ = synth.make_config("tiny")
    s, ref, st, _ = _parity(gs, ora, sc, vw, "tiny-live")
    assert abs(st["n_live_pairs"] - ref["live_pairs"]) <= 1e-4 * ref["live_pairs"] + 5


def test_determinism_and_chunking(gs):
    sc, vw = _ragged()
    dsc = gs.DeviceScene.from_scene(sc)
    a, _ = gs.sensitivity(dsc, vw)
    b, _ = gs.sensitivity(dsc, vw)
    c, _ = gs.sensitivity(dsc, vw, max_views_per_chunk=1)
    a, b, c = (x.cpu().numpy().view(np.uint32) for x in (a, b, c))
    assert np.array_equal(a, b)
    assert np.array_equal(a, c)


def test_many_views_in_view_groups(gs, ora):
    """61 views in one call: the projection takes each block of Gaussians
    through three groups of views (20, 20 and 21); every ray against the
    oracle, and bit-identical to calls of 7 views (one group each)."""
    sc = synth.make_cluster_scene(3000, 23, 2)
    vw = synth.make_orbit_views(61, 29, 64, 48)
    _parity(gs, ora, sc, vw, "61 views")
    dsc = gs.DeviceScene.from_scene(sc)
    a, _ = gs.sensitivity(dsc, vw)
    c, _ = gs.sensitivity(dsc, vw, max_views_per_chunk=7)
    assert np.array_equal(a.cpu().numpy().view(np.uint32), c.cpu().numpy().view(np.uint32))


def test_stats_over_view_chunks(gs):
    """Counters are summed over view chunks of different sizes (3 views in
    chunks of 2 and 1), equal those of one chunk, and stay right on repeated
    calls; a non-finite Gaussian is counted once however many chunks there are."""
    import re
    import torch
    sc, vw = _ragged()
    dsc = gs.DeviceScene.from_scene(sc)
    _, one = gs.sensitivity(dsc, vw, stats=True, count_pairs=True)
    keys = ("n_projected", "n_entries", "n_pairs", "n_live_pairs", "n_rays_positive", "n_lane_pairs",
            "n_invalid_gaussians")
    for _ in range(3):
        # leave unrelated values in the work arena between the calls
        gs.sensitivity(dsc, vw, max_views_per_chunk=1)
        _, two = gs.sensitivity(dsc, vw, stats=True, count_pairs=True, max_views_per_chunk=2)
        torch.cuda.synchronize()
        assert {k: two[k] for k in keys} == {k: one[k] for k in keys}
    bad = synth.Scene(sc.mean.copy(), sc.log_scale, sc.quat, sc.opacity, sc.sh, sc.sh_degree)
    bad.mean[0, 17] = np.nan
    with pytest.raises(gs.GsError) as e:
        gs.sensitivity(gs.DeviceScene.from_scene(bad), vw, stats=True, max_views_per_chunk=1)
    assert e.value.status == 5
    assert re.search(r"\b1 Gaussians have non-finite", str(e.value)), str(e.value)


@pytest.mark.parametrize("room", ["none", "quarter", "tenth"])
def test_compaction_room_in_ranges(gs, monkeypatch, room):
    """Pass 2 reads the quadrant lists pass 1 left in a room; a room that
    holds a quarter or a tenth of them makes the call composite tile ranges
    one after another, and no room makes pass 2 filter the tile lists
    itself.  Sensitivities and the live-pair counts are identical in every case."""
    import torch
    sc, vw = _ragged()
    dsc = gs.DeviceScene.from_scene(sc)
    ref, st = gs.sensitivity(dsc, vw, stats=True, count_pairs=True)
    frac = {"none": 0.0, "quarter": 0.25, "tenth": 0.1}[room]
    monkeypatch.setenv("GS_COMPACT_POOL_GB", repr(16 * st["n_entries"] * frac / 2**30))
    s, st2 = gs.sensitivity(dsc, vw, stats=True, count_pairs=True)
    monkeypatch.delenv("GS_COMPACT_POOL_GB")
    torch.cuda.synchronize()
    assert torch.equal(s, ref)
    # (pairs evaluated past a ray's stop depend on where slices end, so only
    # the counters that do not are compared)
    keys = ("n_live_pairs", "n_rays_positive", "n_entries")
    assert {k: st2[k] for k in keys} == {k: st[k] for k in keys}


def test_render_full_matches_oracle(gs, ora):
    sc, vw = _ragged()
    ref = ora.sensitivity(sc, vw)
    out = gs.render_objective(gs.DeviceScene.from_scene(sc), vw)
    A = out["per_ray"].cpu().numpy().astype(np.float64)
    ok = ~ref["flag"]
    err = np.abs(A[ok] - ref["A"][ok]) - REL * ref["A"][ok]
    assert err.max() <= 1e-30, f"max A excess {err.max():.3e}"
    assert np.array_equal(A[ok] > 0, ref["A"][ok] > 0)


@pytest.mark.parametrize("n,m,seed", [(2000, 200, 0), (100_000, 10_000, 123456789012345),
                                      (257, 5000, 2 ** 63 + 11), (1_000_000, 100_000, 0)])
def test_sampler_bit_exact(gs, ora, n, m, seed):
    import torch
    rng = np.random.default_rng(n)
    s = rng.uniform(0, 1, n).astype(np.float32)
    s[rng.uniform(size=n) < 0.2] = 0
    s[:3] = [1.0, 2.0 ** -40, 3 * 2.0 ** -40]
    ref = ora.sample(s, m, seed)
    counts, w, sup = gs.sample_coreset(torch.as_tensor(s).cuda(), m, seed)
    assert np.array_equal(counts.cpu().numpy().view(np.uint32), ref["counts"])
    assert np.array_equal(w.cpu().numpy().view(np.uint64), ref["weights"].view(np.uint64))
    assert int(sup.item()) == ref["support"]


def test_sampler_small_integer_cdf(gs, ora):
    import torch
    k = np.array([1, 2, 0, 3, 1, 4], np.float64)
    s = (k * 2.0 ** -40).astype(np.float32)
    ref = ora.sample(s, 4000, 5)
    counts, w, sup = gs.sample_coreset(torch.as_tensor(s).cuda(), 4000, 5)
    assert np.array_equal(counts.cpu().numpy().view(np.uint32), ref["counts"])
    assert np.array_equal(w.cpu().numpy(), ref["weights"])


def test_sampler_rejects_all_zero(gs):
    import torch
    with pytest.raises(gs.GsError) as e:
        gs.sample_coreset(torch.zeros(100, device="cuda"), 10, 0)
    assert e.value.status == 4


def test_sampler_rejects_values_outside_unit_interval(gs, ora):
    """A sensitivity is a largest share, so it lies in [0, 1] up to float32
    rounding; a value above 1 + 2^-10 (which could overflow the 64-bit CDF),
    NaN or a negative value is rejected with the outputs zeroed, as the
    oracle does; 1 and values an ulp above it are drawn as usual."""
    import torch
    rng = np.random.default_rng(77)
    base = rng.uniform(0, 1, 5000).astype(np.float32)
    for v in (np.float32(1.001), np.float32(2.0 ** 30), np.float32(np.nan),
              np.float32(-1e-30), np.float32(np.inf)):
        x = base.copy()
        x[1234] = v
        assert ora.sample(x, 100, 1)["status"] == 5
        with pytest.raises(gs.GsError) as e:
            counts, w, sup = gs.sample_coreset(torch.as_tensor(x).cuda(), 100, 1)
        assert e.value.status == 5
    x = base.copy()
    x[:100] = 1.0
    x[100] = np.nextafter(np.float32(1), np.float32(2))
    x[101] = np.float32(1 + 2.0 ** -10)
    ref = ora.sample(x, 300, 2)
    counts, w, sup = gs.sample_coreset(torch.as_tensor(x).cuda(), 300, 2)
    assert ref["status"] == 0
    assert np.array_equal(counts.cpu().numpy().view(np.uint32), ref["counts"])
    assert np.array_equal(w.cpu().numpy().view(np.uint64), ref["weights"].view(np.uint64))


def test_coreset_error_kernel(gs):
    """gs_coreset_error against its definition on per-view sums, views with
    A = 0 left out."""
    import torch
    rng = np.random.default_rng(5)
    pv = rng.uniform(0.5, 2.0, (333, 3))
    pv[7, 0] = 0.0
    pv[7, 1] = 50.0
    on = pv[:, 0] > 0
    want0 = np.max(np.abs(pv[on, 1] - pv[on, 0]) / pv[on, 0])
    want1 = np.max(np.abs(pv[on, 2] - pv[on, 0]) / pv[on, 0])
    t = torch.as_tensor(pv).cuda()
    assert gs.coreset_error(t) == want0
    assert gs.coreset_error(t, reduced=True) == want1


def test_objective_parity(gs, ora):
    import torch
    sc, vw = _ragged()
    ref_s = ora.sensitivity(sc, vw)
    bits = synth.pack_bits(~ref_s["flag"])
    dsc = gs.DeviceScene.from_scene(sc)
    s, _ = gs.sensitivity(dsc, vw)
    w_ref = ora.sample(s.cpu().numpy(), sc.n // 10, 3)["weights"]
    w = torch.as_tensor(w_ref).cuda()
    ob = ora.objective(sc, vw, w_ref, None, bits)
    # the true reduced render's FP32 error grows with 1 / |1 - w rho| of the
    # earlier pairs (factors near 0 when w rho is near 1): the oracle's
    # rounding scale E bounds the change of A_w per unit relative error of
    # every rho, and float32 rho carries at most ~3e-6 (the exponent's
    # rounding times ln 2), so 1e-5 E is its share of the tolerance
    E = ora.objective_true_scale(sc, vw, w_ref, ray_mask=bits)
    for obj, key in ((gs.OBJ_FULL, "A"), (gs.OBJ_FIXED, "A_fixed"), (gs.OBJ_TRUE, "A_true")):
        out = gs.render_objective(dsc, vw, w, obj, ray_mask=_mask_tensor(bits))
        got = out["per_ray"].cpu().numpy().astype(np.float64)
        want = ob[key]
        scale = np.maximum(np.abs(want), ob["A"])
        tol = 1e-5 * scale + (1e-5 * E if obj == gs.OBJ_TRUE else 0.0)
        err = np.abs(got - want) / np.maximum(scale, 1e-30)
        excess = np.abs(got - want) - tol
        print(f"[objective {key}] max rel err {err.max():.3e}, p99.9 {np.quantile(err, 0.999):.3e}, "
              f"worst excess over the bound {excess.max():.3e}; pairs with w rho >= 1: {ob['n_invalid']}",
              flush=True)
        assert excess.max() <= 0.0, f"{key}: max rel err {err.max():.3e}"
        pv = out["per_view"].cpu().numpy()
        if obj != gs.OBJ_TRUE:
            # the full and fixed objectives stop a ray once later terms are
            # below 1e-9 A, so only their own columns are complete
            assert np.allclose(pv[:, :2], ob["view_sums"][:, :2], rtol=1e-5)
            continue
        assert np.allclose(pv[:, :2], ob["view_sums"][:, :2], rtol=1e-5)
        base = 0
        for v in range(vw.n_views):
            n = int(vw.size[v, 0]) * int(vw.size[v, 1])
            bound = 1e-5 * abs(ob["view_sums"][v, 2]) + tol[base:base + n].sum()
            assert abs(pv[v, 2] - ob["view_sums"][v, 2]) <= bound, v
            base += n
        assert out["n_invalid_pairs"] == ob["n_invalid"]
        if ob["gamma"] > 0:
            assert abs(out["gamma_max"] - ob["gamma"]) <= 1e-4 * ob["gamma"] + 1e-5


def test_single_gaussian_scores_one(gs):
    sc = synth.make_explicit_scene([(0.0, 0.0, 0.0)], [math.log(0.02)] * 3, (1, 0, 0, 0), 0.8,
                                   [[0.3, 0.6, 0.2]])
    vw = synth.make_camera_set([(-4.0, 0.0, 0.0)], [(0.0, 0.0, 0.0)], 37, 29, 60.0)
    s, st = gs.sensitivity(gs.DeviceScene.from_scene(sc), vw, stats=True)
    assert abs(float(s[0]) - 1.0) <= 2e-7
    assert st["n_projected"] == 1


def test_nothing_visible(gs):
    """All Gaussians behind the camera: s = 0 and sampling reports it."""
    sc, vw, _, _ = synth.make_config("tiny")
    far = synth.make_camera_set([(0.0, 0.0, 5.0)], [(0.0, 0.0, 10.0)], 64, 64, 60.0, up=(1, 0, 0))
    s, st = gs.sensitivity(gs.DeviceScene.from_scene(sc), far, stats=True)
    assert float(s.abs().max()) == 0.0 and st["n_projected"] == 0
    with pytest.raises(gs.GsError):
        gs.sample_coreset(s, 10, 0)


def test_masking_every_ray_gives_zero(gs):
    sc, vw, _, _ = synth.make_config("tiny")
    bits = synth.pack_bits(np.zeros(vw.n_rays, bool))
    s, _ = gs.sensitivity(gs.DeviceScene.from_scene(sc), vw, ray_mask=_mask_tensor(bits))
    assert float(s.abs().max()) == 0.0


def test_nan_attribute_reported(gs):
    sc, vw, _, _ = synth.make_config("tiny")
    sc.mean[0, 5] = np.nan
    with pytest.raises(gs.GsError) as e:
        gs.sensitivity(gs.DeviceScene.from_scene(sc), vw, stats=True)
    assert e.value.status == 5


def test_mixed_view_sizes_in_one_call(gs, ora):
    sc = synth.make_cluster_scene(5000, 9, 1)
    vw = synth.make_orbit_views(4, 21, resolutions=[(64, 48), (97, 61), (33, 130)])
    _parity(gs, ora, sc, vw, "mixed-sizes")


def _dequantized(sc):
    """The scene exactly as the mixed-precision planes hold it (bf16 mean,
    log-scale and SH; f16 quaternion and opacity), widened to float32."""
    import torch
    q = lambda a, dt: torch.as_tensor(a).to(dt).to(torch.float32).numpy()
    return synth.Scene(q(sc.mean, torch.bfloat16), q(sc.log_scale, torch.bfloat16),
                       q(sc.quat, torch.float16), q(sc.opacity, torch.float16),
                       q(sc.sh, torch.bfloat16), sc.sh_degree)


def test_mixed16_parity_on_dequantized_scene(gs, ora):
    """Mixed-precision storage changes only what is loaded: against the oracle
    run on the dequantized scene the bar is the float32 one."""
    sc, vw = _ragged()
    dq = _dequantized(sc)
    ref_all = ora.sensitivity(dq, vw)
    bits = synth.pack_bits(~ref_all["flag"])
    ref = ora.sensitivity(dq, vw, None, bits)
    d16 = gs.DeviceScene.from_scene(sc, fmt=gs.ATTR_MIXED16)
    assert d16.attribute_bytes() * 2 == gs.DeviceScene.from_scene(sc).attribute_bytes()
    s, _ = gs.sensitivity(d16, vw, ray_mask=_mask_tensor(bits))
    s = s.cpu().numpy().astype(np.float64)
    excess = np.abs(s - ref["s"]) - (REL * ref["s"] + ABS)
    assert excess.max() <= 0
    # error against the float32 source scene: reported, not gated
    src = ora.sensitivity(sc, vw, None, bits)
    big = src["s"] > 1e-3
    rel = np.abs(s[big] - src["s"][big]) / src["s"][big]
    print(f"[mixed16] vs float32 source: median rel {np.median(rel):.2e} p99 {np.quantile(rel, 0.99):.2e} "
          f"max {rel.max():.2e} (Gaussians with s > 1e-3)", flush=True)
