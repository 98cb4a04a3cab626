"""Aggregated sensitivities (Section 3.5: queries that are 16x16 tiles, whole
views or the whole scene) of the HIP path against the FP64 oracle, through
the C ABI.

Both sides score the same rays: the oracle's ambiguous rays (a pair within
1e-5 r^2 of the footprint cutoff, or an order key near a float32 rounding
midpoint) are removed from every query through the ray mask.  The bar is the
per-ray one, |s_gpu - s_oracle| <= 1e-5 s_oracle + 1e-12: the GPU's shares
are float32 per ray, summed over a wave in float32 (at most 6 roundings of
positive terms, < 4e-7 relative), then in exact 64-bit fixed point with unit
2^-60 of the query's A; the share floor drops less than 1e-12 A(Q) per
query.  Properties at any size: the per-scene sensitivities sum to 1, the
levels are ordered (scene <= image <= tile <= ray) and every granularity is
deterministic (bit-identical on a second call)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

REL, ABS = 1e-5, 1e-12
LEVELS = ("tile", "image", "scene")


@pytest.fixture(scope="module")
def gs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_02721_amd as gs
    gs.load()
    return gs


def _level(gs, name):
    return {"ray": gs.AGG_RAY, "tile": gs.AGG_TILE, "image": gs.AGG_IMAGE, "scene": gs.AGG_SCENE}[name]


def _mask_tensor(bits):
    import torch
    return torch.as_tensor(np.ascontiguousarray(bits, np.uint32).view(np.int32)).cuda()


def _ragged():
    # 200x136 is 12.5 x 8.5 tiles: ragged right and bottom tiles in every view
    return synth.make_cluster_scene(20_000, 7, 3), synth.make_orbit_views(3, 17, 200, 136)


def _case(ora, sc, vw):
    flag = ora.sensitivity(sc, vw)["flag"]
    return synth.pack_bits(~flag), int(flag.sum())


def _check(label, s, ref):
    excess = np.abs(s - ref) - (REL * ref + ABS)
    worst = int(np.argmax(excess))
    big = ref > 1e-9
    rel = np.max(np.abs(s[big] - ref[big]) / ref[big]) if big.any() else 0.0
    print(f"[{label}] s>0 on {int((ref > 0).sum())}, max rel err (s > 1e-9) {rel:.2e}, "
          f"worst excess {excess[worst]:.2e}", flush=True)
    assert excess.max() <= 0, f"{label}: Gaussian {worst}: gpu {s[worst]!r} oracle {ref[worst]!r}"


@pytest.mark.parametrize("level", LEVELS)
@pytest.mark.parametrize("which", ["tiny", "ragged"])
def test_aggregated_parity(gs, ora, which, level):
    sc, vw = synth.make_config("tiny")[:2] if which == "tiny" else _ragged()
    bits, n_flag = _case(ora, sc, vw)
    ref = ora.sensitivity_agg(sc, vw, getattr(ora, "AGG_" + level.upper()), ray_mask=bits)
    d = gs.DeviceScene.from_scene(sc)
    s, _ = gs.sensitivity(d, vw, ray_mask=_mask_tensor(bits), aggregate=_level(gs, level))
    print(f"[{which}/{level}] flagged rays {n_flag}/{vw.n_rays}", flush=True)
    _check(f"{which}/{level}", s.double().cpu().numpy(), ref)


@pytest.mark.parametrize("level", LEVELS)
def test_sparse_mask_aggregated_parity(gs, ora, level):
    """A mask that selects one row of 8x8 quadrants per view (1 of 17) takes
    the quadrant-list form of both passes (per-tile queries: per-entry
    accumulators and a separate maximum); the other tests' dense masks take
    the region form (per-tile queries: the maximum in the region waves).
    Both score the same rays as the oracle."""
    sc, vw = _ragged()
    flag = ora.sensitivity(sc, vw)["flag"]
    sel = np.zeros((3, 136, 200), bool)
    sel[:, 16:24, :] = True
    bits = synth.pack_bits(sel.reshape(-1) & ~flag)
    ref = ora.sensitivity_agg(sc, vw, getattr(ora, "AGG_" + level.upper()), ray_mask=bits)
    assert (ref > 0).any()
    d = gs.DeviceScene.from_scene(sc)
    s, _ = gs.sensitivity(d, vw, ray_mask=_mask_tensor(bits), aggregate=_level(gs, level))
    _check(f"sparse/{level}", s.double().cpu().numpy(), ref)


@pytest.mark.parametrize("tile", [(16, 32), (32, 16), (32, 32)])
def test_tile_queries_on_larger_binning_tiles(gs, ora, tile):
    """Per-tile queries binned at 16x32, 32x16 or 32x32: each 16x16 region of
    a binning tile is one query, composited by its own wave; bit-identical to
    16x16 binning, dense or sparse mask (the sparse one takes the region
    form here, the quadrant-list form at 16x16), and the sparse run against
    the oracle."""
    import torch
    sc, vw = _ragged()
    d = gs.DeviceScene.from_scene(sc)
    flag = ora.sensitivity(sc, vw)["flag"]
    sel = np.zeros((3, 136, 200), bool)
    sel[:, 16:24, :] = True
    for bits in (synth.pack_bits(~flag), synth.pack_bits(sel.reshape(-1) & ~flag)):
        m = _mask_tensor(bits)
        s16, _ = gs.sensitivity(d, vw, ray_mask=m, aggregate=gs.AGG_TILE, tile=(16, 16))
        s, _ = gs.sensitivity(d, vw, ray_mask=m, aggregate=gs.AGG_TILE, tile=tile)
        torch.cuda.synchronize()
        assert torch.equal(s, s16), tile
    ref = ora.sensitivity_agg(sc, vw, ora.AGG_TILE, ray_mask=bits)
    _check(f"tile queries at {tile[0]}x{tile[1]}", s.double().cpu().numpy(), ref)


def test_views_in_several_chunks(gs, ora):
    """One view per launch: tile and image queries never straddle launches,
    so they are bit-identical to one launch; the per-scene sums are carried
    across launches in FP64 and still match the oracle."""
    import torch
    sc, vw = _ragged()
    bits, _ = _case(ora, sc, vw)
    d = gs.DeviceScene.from_scene(sc)
    m = _mask_tensor(bits)
    for level in LEVELS:
        one, _ = gs.sensitivity(d, vw, ray_mask=m, aggregate=_level(gs, level))
        per_view, _ = gs.sensitivity(d, vw, ray_mask=m, aggregate=_level(gs, level), max_views_per_chunk=1)
        torch.cuda.synchronize()
        if level != "scene":
            assert torch.equal(one, per_view), level
        else:
            ref = ora.sensitivity_agg(sc, vw, ora.AGG_SCENE, ray_mask=bits)
            _check("chunks/scene", per_view.double().cpu().numpy(), ref)


def test_invariants_and_determinism(gs):
    """Unmasked, on the ragged scene: per-scene shares sum to 1; each level is
    at most the finer one (up to float32 rounding of both); a second call is
    bit-identical at every granularity."""
    import torch
    sc, vw = _ragged()
    d = gs.DeviceScene.from_scene(sc)
    out = {}
    for level in ("ray",) + LEVELS:
        a, st = gs.sensitivity(d, vw, aggregate=_level(gs, level), stats=True)
        b, _ = gs.sensitivity(d, vw, aggregate=_level(gs, level))
        torch.cuda.synchronize()
        assert torch.equal(a, b), level
        assert bool((a >= 0).all()) and bool((a <= 1.0 + 1e-6).all())
        out[level] = (a.double().cpu().numpy(), st["total_sensitivity"])
    S_scene = out["scene"][1]
    print(f"[invariants] S per level: " + ", ".join(f"{k}={v[1]:.6f}" for k, v in out.items()), flush=True)
    assert abs(S_scene - 1.0) <= 1e-5
    for fine, coarse in (("ray", "tile"), ("tile", "image"), ("image", "scene")):
        f, c = out[fine][0], out[coarse][0]
        assert np.all(c <= f * (1 + 2e-6) + 1e-12), (fine, coarse, float(np.max(c - f)))
    assert out["ray"][1] >= out["tile"][1] >= out["image"][1] >= S_scene * (1 - 1e-6)


def test_per_scene_sampling_has_zero_variance(gs):
    """Per-scene sensitivities sampled on the GPU reproduce the scene's total
    objective at every seed (sum over views of A^th_w = sum of A) up to the
    2^-40 quantisation of the probabilities and float32 shares."""
    import torch
    sc, vw = _ragged()
    d = gs.DeviceScene.from_scene(sc)
    s, _ = gs.sensitivity(d, vw, aggregate=gs.AGG_SCENE)
    full = gs.render_objective(d, vw, None, gs.OBJ_FULL, per_ray=False, diag=False)["per_view"][:, 0]
    A = float(full.sum())
    errs = []
    for seed in range(3):
        _, w, _ = gs.sample_coreset(s, 2000, seed)
        pv = gs.render_objective(d, vw, w, gs.OBJ_FIXED, per_ray=False, diag=False)["per_view"]
        torch.cuda.synchronize()
        errs.append(abs(float(pv[:, 1].sum()) - A) / A)
    print(f"[zero variance] relative errors {errs}", flush=True)
    assert max(errs) < 1e-5
