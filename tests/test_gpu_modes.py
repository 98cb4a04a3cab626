"""Score variants of the HIP path against the FP64 oracle, through the C ABI
(Section 3.5: the L2 contribution c^2 rho^2 T^2 with the three channel terms
summed per pixel, and Algorithm 1's per-channel queries c_k rho T; the
nocolor variant is covered with the per-ray parity tests).

Same bar as the per-ray parity tests: |s_gpu - s_oracle| <= 1e-5 s_oracle +
1e-12 on every Gaussian, both sides scoring the rays the oracle does not flag
as ambiguous; with the share-floor stop off the in-footprint pair counts
agree exactly; per-ray L2 objectives within 1e-5 relative."""
import numpy as np
import pytest

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


def _mask_tensor(bits):
    import torch
    return torch.as_tensor(np.ascontiguousarray(bits, np.uint32).view(np.int32)).cuda()


def _ragged():
    return synth.make_cluster_scene(20_000, 7, 3), synth.make_orbit_views(3, 17, 200, 136)


def _scene(which):
    return synth.make_config("tiny")[:2] if which == "tiny" else _ragged()


def _check(label, s, ref):
    excess = np.abs(s - ref) - (REL * ref + ABS)
    worst = int(np.argmax(excess))
    big = ref > 1e-9
    print(f"[{label}] s>0 on {int((ref > 0).sum())}, max rel err (s > 1e-9) "
          f"{np.max(np.abs(s[big] - ref[big]) / ref[big]):.2e}, worst excess {excess[worst]:.2e}", flush=True)
    assert excess.max() <= 0, f"{label}: Gaussian {worst}: gpu {s[worst]!r} oracle {ref[worst]!r}"


@pytest.mark.parametrize("which", ["tiny", "ragged"])
@pytest.mark.parametrize("mode", ["l2", "channel"])
def test_variant_parity(gs, ora, which, mode):
    qm = {"l2": gs.QUERY_L2, "channel": gs.QUERY_CHANNEL}[mode]
    sc, vw = _scene(which)
    prm = ora.default_params(query_mode=qm)
    bits = synth.pack_bits(~ora.sensitivity(sc, vw, prm)["flag"])
    ref = ora.sensitivity(sc, vw, prm, bits)
    s, st = gs.sensitivity(gs.DeviceScene.from_scene(sc), vw, query_mode=qm, ray_mask=_mask_tensor(bits),
                           stats=True, count_pairs=True)
    _check(f"{which}/{mode}", s.double().cpu().numpy(), ref["s"])
    assert st["n_rays_positive"] == ref["rays_positive"]


@pytest.mark.parametrize("mode", ["l2", "channel"])
def test_variant_pair_count_without_stop(gs, ora, mode):
    """share_floor = 0: every pair is evaluated and counted as the oracle does."""
    qm = {"l2": gs.QUERY_L2, "channel": gs.QUERY_CHANNEL}[mode]
    sc, vw = _scene("tiny")
    prm = ora.default_params(query_mode=qm)
    bits = synth.pack_bits(~ora.sensitivity(sc, vw, prm)["flag"])
    ref = ora.sensitivity(sc, vw, prm, bits)
    s, st = gs.sensitivity(gs.DeviceScene.from_scene(sc), vw, query_mode=qm, ray_mask=_mask_tensor(bits),
                           share_floor=0.0, stats=True, count_pairs=True)
    assert st["n_pairs"] == ref["pairs"]
    _check(f"nostop/{mode}", s.double().cpu().numpy(), ref["s"])


@pytest.mark.parametrize("mode", ["rgbsum", "l2", "channel"])
def test_sparse_mask_parity(gs, ora, mode):
    """A sparse ray mask (six 8x8 pixel blocks per view, well under a quarter
    of the quadrants) makes the library composite only the listed quadrants,
    one wave each, instead of the region launches that the dense masks of the
    other tests take; the same bar against the oracle on the same rays."""
    qm = {"rgbsum": gs.QUERY_RGBSUM, "l2": gs.QUERY_L2, "channel": gs.QUERY_CHANNEL}[mode]
    sc, vw = _ragged()
    prm = ora.default_params(query_mode=qm)
    flag = ora.sensitivity(sc, vw, prm)["flag"]
    W, H = 200, 136
    rng = np.random.default_rng(11)
    sel = np.zeros(3 * W * H, bool)
    for v in range(3):
        for _ in range(6):
            bx, by = int(rng.integers(0, W // 8)), int(rng.integers(0, H // 8))
            for y in range(8 * by, 8 * by + 8):
                sel[v * W * H + y * W + 8 * bx: v * W * H + y * W + 8 * bx + 8] = True
    bits = synth.pack_bits(sel & ~flag)
    ref = ora.sensitivity(sc, vw, prm, bits)
    s, st = gs.sensitivity(gs.DeviceScene.from_scene(sc), vw, query_mode=qm, ray_mask=_mask_tensor(bits),
                           stats=True, count_pairs=True)
    _check(f"sparse/{mode}", s.double().cpu().numpy(), ref["s"])
    assert st["n_rays_positive"] == ref["rays_positive"]


def test_channel_at_least_rgbsum(gs):
    """A pixel's RGB-sum share is a weighted mean of its channel shares, so
    the per-channel sensitivities bound the RGB-sum ones from above."""
    sc, vw = _ragged()
    d = gs.DeviceScene.from_scene(sc)
    a = gs.sensitivity(d, vw)[0].double().cpu().numpy()
    b = gs.sensitivity(d, vw, query_mode=gs.QUERY_CHANNEL)[0].double().cpu().numpy()
    assert np.all(b >= a * (1 - 2e-6))
    assert np.mean(b > a * (1 + 1e-4)) > 0.5


def test_l2_objectives_match_oracle(gs, ora):
    """Per-ray L2 objectives: the full render, the fixed relaxation and the
    reduced render with the retained scene's transmittance."""
    import torch
    sc, vw = _ragged()
    prm = ora.default_params(query_mode=gs.QUERY_L2)
    ref_s = ora.sensitivity(sc, vw, prm)
    bits = synth.pack_bits(~ref_s["flag"])
    d = gs.DeviceScene.from_scene(sc)
    s, _ = gs.sensitivity(d, vw, query_mode=gs.QUERY_L2)
    w_ref = ora.sample(s.cpu().numpy(), sc.n // 10, 4)["weights"]
    w = torch.as_tensor(w_ref).cuda()
    ob = ora.objective(sc, vw, w_ref, prm, bits)
    # reduced render: the oracle's rounding scale E (as in test_objective_parity)
    E = ora.objective_true_scale(sc, vw, w_ref, prm, ray_mask=bits)
    for obj, key in ((gs.OBJ_FULL, "A"), (gs.OBJ_FIXED, "A_fixed"), (gs.OBJ_TRUE, "A_true")):
        out = gs.render_objective(d, vw, w, obj, query_mode=gs.QUERY_L2, ray_mask=_mask_tensor(bits))
        got = out["per_ray"].cpu().numpy().astype(np.float64)
        want = ob[key]
        scale = np.maximum(np.abs(want), ob["A"])
        tol = 1e-5 * scale + (1e-5 * E if obj == gs.OBJ_TRUE else 0.0)
        err = np.abs(got - want) / np.maximum(scale, 1e-30)
        print(f"[l2 objective {key}] max rel err {err.max():.2e}, worst excess over the bound "
              f"{(np.abs(got - want) - tol).max():.2e}", flush=True)
        assert np.all(np.abs(got - want) <= tol), key


@pytest.mark.parametrize("level", ["tile", "image", "scene"])
def test_l2_aggregated_parity(gs, ora, level):
    sc, vw = _scene("ragged")
    prm = ora.default_params(query_mode=gs.QUERY_L2)
    bits = synth.pack_bits(~ora.sensitivity(sc, vw, prm)["flag"])
    lv = {"tile": gs.AGG_TILE, "image": gs.AGG_IMAGE, "scene": gs.AGG_SCENE}[level]
    ref = ora.sensitivity_agg(sc, vw, lv, prm, bits)
    s, _ = gs.sensitivity(gs.DeviceScene.from_scene(sc), vw, query_mode=gs.QUERY_L2, aggregate=lv,
                          ray_mask=_mask_tensor(bits))
    _check(f"l2/{level}", s.double().cpu().numpy(), ref)


def test_unsupported_combinations(gs):
    sc, vw = _scene("tiny")
    d = gs.DeviceScene.from_scene(sc)
    with pytest.raises(gs.GsError) as e:
        gs.sensitivity(d, vw, query_mode=gs.QUERY_CHANNEL, aggregate=gs.AGG_TILE)
    assert e.value.status == 2
    with pytest.raises(gs.GsError) as e:
        gs.render_objective(d, vw, None, gs.OBJ_FULL, query_mode=gs.QUERY_CHANNEL)
    assert e.value.status == 2
    with pytest.raises(gs.GsError) as e:
        gs.Plan([d], [vw], query_mode=gs.QUERY_CHANNEL)
    assert e.value.status == 2


def test_l2_plan_matches_per_scene_calls(gs):
    """Plans take the L2 mode: bit-identical to gs_sensitivity in every launch shape."""
    import torch
    specs = [(20_000, 11, 3, 6, 160, 96), (7_001, 12, 1, 3, 200, 136)]
    batch = [(gs.DeviceScene.from_scene(synth.make_cluster_scene(n, sd, deg)),
              synth.make_orbit_views(nv, sd + 100, W, H)) for n, sd, deg, nv, W, H in specs]
    ref = [gs.sensitivity(d, v, query_mode=gs.QUERY_L2)[0].clone() for d, v in batch]
    plan = gs.Plan([d for d, _ in batch], [v for _, v in batch], query_mode=gs.QUERY_L2)
    for persistent, xcd in ((0, 1), (1, 0)):
        plan.set_config(persistent, xcd)
        outs = plan.run()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o, r), (persistent, xcd)
    plan.close()
