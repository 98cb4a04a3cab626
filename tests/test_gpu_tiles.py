"""Binning tiles of every supported shape (8, 16 or 32 pixels per side).

The tile only decides which lists a Gaussian enters: the pairs that count
(d^2 <= r^2 at a pixel centre), their depth order and every per-ray sum are
the same for all shapes, so per-ray sensitivities, A and the objectives must
be bit-identical to the 16 x 16 pass, and every shape meets the oracle bar
of the parity tests.  Aggregated image and scene queries sum A over tiles in
a different order, so they agree to FP64 rounding only.
"""
import numpy as np
import pytest

import parity_util
import synth

pytestmark = pytest.mark.gpu

SHAPES = [(8, 8), (8, 16), (16, 8), (8, 32), (32, 8), (16, 32), (32, 16), (32, 32)]


@pytest.fixture(scope="module")
def gs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_02721_amd as gs
    gs.load()
    return gs


@pytest.fixture(scope="module")
def ragged():
    # 200 x 136 is ragged for every shape (25 x 17 tiles of 8, 6.25 x 4.25 of 32)
    sc = synth.make_cluster_scene(20_000, 7, 3)
    vw = synth.make_orbit_views(3, 17, 200, 136)
    return sc, vw


@pytest.fixture(scope="module")
def base16(gs, ragged):
    sc, vw = ragged
    d = gs.DeviceScene.from_scene(sc)
    s, st = gs.sensitivity(d, vw, stats=True, count_pairs=True)
    return d, s.clone(), st


@pytest.mark.parametrize("tile", SHAPES)
def test_shape_bit_identical_to_16x16(gs, ragged, base16, tile):
    import torch
    d, s16, st16 = base16
    s, st = gs.sensitivity(d, ragged[1], stats=True, count_pairs=True, tile=tile)
    print(f"[tile {tile}] entries {st['n_entries']} (16x16: {st16['n_entries']}), live pairs "
          f"{st['n_live_pairs']}", flush=True)
    assert torch.equal(s, s16), float((s - s16).abs().max())
    assert st["n_rays_positive"] == st16["n_rays_positive"]
    assert st["n_live_pairs"] == st16["n_live_pairs"]
    assert st["n_pairs"] == st16["n_pairs"]
    assert st["n_ambiguous_pairs"] == st16["n_ambiguous_pairs"]


@pytest.mark.parametrize("tile", [(8, 8), (32, 16), (32, 32)])
def test_shape_parity_with_oracle(gs, ora, ragged, tile):
    sc, vw = ragged
    dsc = gs.DeviceScene.from_scene(sc)
    oprm = ora.default_params()
    bits, oflag, gflag = parity_util.union_mask(gs, ora, sc, vw, dsc, oprm, tile=tile)
    ref = ora.sensitivity(sc, vw, oprm, bits)
    s, _ = gs.sensitivity(dsc, vw, ray_mask=parity_util.mask_tensor(bits), tile=tile)
    s = s.cpu().numpy().astype(np.float64)
    excess = np.abs(s - ref["s"]) - (1e-5 * ref["s"] + 1e-12)
    print(f"[tile {tile} vs oracle] flagged oracle {int(oflag.sum())} gpu {int(gflag.sum())}, worst excess "
          f"{excess.max():.3e}", flush=True)
    assert excess.max() <= 0


@pytest.mark.parametrize("tile", [(8, 16), (32, 32)])
def test_masked_shape_matches_16x16(gs, ragged, tile):
    """A random ray mask exercises the per-quadrant activity bits (up to 16
    quadrants per tile) and the quadrant lists."""
    import torch
    sc, vw = ragged
    rng = np.random.default_rng(5)
    keep = rng.random(vw.n_rays) < 0.03
    keep[:vw.n_rays // 3] = False   # the first view scores nothing
    m = parity_util.mask_tensor(synth.pack_bits(keep))
    d = gs.DeviceScene.from_scene(sc)
    s16, st16 = gs.sensitivity(d, vw, ray_mask=m, stats=True)
    s, st = gs.sensitivity(d, vw, ray_mask=m, stats=True, tile=tile)
    assert float(s16.max()) > 0
    assert torch.equal(s, s16)
    assert st["n_rays_positive"] == st16["n_rays_positive"]


@pytest.mark.parametrize("agg", ["image", "scene"])
def test_aggregated_queries_across_shapes(gs, ragged, base16, agg):
    import torch
    d, _, _ = base16
    a = gs.AGG_IMAGE if agg == "image" else gs.AGG_SCENE
    s16, _ = gs.sensitivity(d, ragged[1], aggregate=a)
    s32, _ = gs.sensitivity(d, ragged[1], aggregate=a, tile=(32, 32))
    s8, _ = gs.sensitivity(d, ragged[1], aggregate=a, tile=(8, 8))
    for s in (s32, s8):
        assert torch.allclose(s, s16, rtol=1e-6, atol=1e-30)


def test_objectives_across_shapes(gs, ragged, base16):
    import torch
    d, s16, _ = base16
    sc, vw = ragged
    w = torch.zeros(sc.n, dtype=torch.float64, device="cuda")
    w[::7] = 7.0
    for obj in (gs.OBJ_FULL, gs.OBJ_FIXED, gs.OBJ_TRUE):
        ref = gs.render_objective(d, vw, w, obj)
        for tile in ((8, 8), (32, 32), (16, 32)):
            out = gs.render_objective(d, vw, w, obj, tile=tile)
            assert torch.equal(out["per_ray"], ref["per_ray"]), (obj, tile)
            assert torch.allclose(out["per_view"], ref["per_view"], rtol=1e-12, atol=0.0), (obj, tile)
            assert out["n_invalid_pairs"] == ref["n_invalid_pairs"]


def test_plan_with_wide_tiles(gs):
    import torch
    specs = [(20_000, 11, 3, 6, 160, 96), (7_001, 12, 1, 3, 200, 136)]
    batch = []
    for n, seed, deg, nv, W, H in specs:
        sc = synth.make_cluster_scene(n, seed, deg)
        batch.append((gs.DeviceScene.from_scene(sc), synth.make_orbit_views(nv, seed + 100, W, H)))
    ref = [gs.sensitivity(dd, vv)[0].clone() for dd, vv in batch]
    for tile in ((32, 32), (8, 8)):
        plan = gs.Plan([dd for dd, _ in batch], [vv for _, vv in batch], tile=tile)
        outs = plan.run()
        torch.cuda.synchronize()
        plan.status()
        info = plan.info()
        print(f"[plan tile {tile}]", info, flush=True)
        assert info["n_compact_launches"] >= 1
        for o, r in zip(outs, ref):
            assert torch.equal(o, r)
        plan.close()


def test_tuner_returns_a_shape_and_result_is_unchanged(gs, ragged, base16):
    import torch
    d, s16, _ = base16
    best, table = gs.tune_tile(d, ragged[1], reps=1)
    print("[tile tuner]", best, {k: round(v, 3) for k, v in table.items()}, flush=True)
    assert best in table and len(table) == 9
    assert table[best] == min(table.values())
    s, _ = gs.sensitivity(d, ragged[1], tile=best)
    assert torch.equal(s, s16)
    # per-tile queries: the shapes with sides of 16 or 32 only
    best_t, table_t = gs.tune_tile(d, ragged[1], reps=1, aggregate=gs.AGG_TILE)
    assert set(table_t) == {(16, 16), (16, 32), (32, 16), (32, 32)} and best_t in table_t


def test_shape_errors(gs, ragged, base16):
    d, _, _ = base16
    vw = ragged[1]
    with pytest.raises(gs.GsError, match="8, 16 or 32"):
        gs.sensitivity(d, vw, tile=(12, 16))
    with pytest.raises(gs.GsError, match="16 or 32 pixels per side"):
        gs.sensitivity(d, vw, tile=(8, 16), aggregate=gs.AGG_TILE)
    big = synth.make_orbit_views(1, 3, 3840, 2160)
    with pytest.raises(gs.GsError, match="tiles of 8x8"):
        gs.sensitivity(d, big, tile=(8, 8))


def test_auto_tile_takes_the_tuned_shape(gs):
    """tile="auto" takes the shape the tuner chose for the same size class
    (seen in the entry count, which depends on the shape), and 16x16 for a
    size class it has not tuned; the sensitivities are the same."""
    import torch
    sc = synth.make_cluster_scene(30_000, 41, 1)
    vw = synth.make_orbit_views(2, 42, 320, 240)
    d = gs.DeviceScene.from_scene(sc)
    best, _ = gs.tune_tile(d, vw, reps=1)
    s_b, st_b = gs.sensitivity(d, vw, stats=True, tile=best)
    s_a, st_a = gs.sensitivity(d, vw, stats=True, tile="auto")
    assert st_a["n_entries"] == st_b["n_entries"]
    assert torch.equal(s_a, s_b)
    # another size class (4x the pixels): no tuned shape, so 16x16
    vw2 = synth.make_orbit_views(2, 43, 640, 480)
    _, st16 = gs.sensitivity(d, vw2, stats=True, tile=(16, 16))
    _, st2 = gs.sensitivity(d, vw2, stats=True, tile="auto")
    assert st2["n_entries"] == st16["n_entries"]
    # a plan with tile "auto" takes the same shape
    plan = gs.Plan([d], [vw], tile="auto")
    out = plan.run()
    torch.cuda.synchronize()
    plan.status()
    assert torch.equal(out[0], s_b)
    plan.close()


def test_auto_tile_widens_for_large_views(gs):
    """With no tuned shape for the size class, tile="auto" takes 16x32 for a
    view whose 16x16 tiles exceed the per-view limit (5120x2880: 58 101 cells
    of 16x16, 29 211 of 16x32) instead of rejecting it; the result is the
    explicit 16x32 run's, bit for bit."""
    import torch
    sc = synth.make_cluster_scene(8_000, 45, 1)
    vw = synth.make_orbit_views(1, 46, 5120, 2880)
    d = gs.DeviceScene.from_scene(sc)
    with pytest.raises(gs.GsError, match="tiles of 16x16"):
        gs.sensitivity(d, vw, tile=(16, 16))
    s_w, st_w = gs.sensitivity(d, vw, stats=True, tile=(16, 32))
    s_a, st_a = gs.sensitivity(d, vw, stats=True, tile="auto")
    assert st_a["n_entries"] == st_w["n_entries"]
    assert torch.equal(s_a, s_w)


def test_large_view_at_16x16(gs):
    """A 3840x2160 view at 16x16 tiles (32 776 cells: a 128 KiB difference
    array in the counting kernel's LDS) gives the same sensitivities as at
    32x32, bit for bit."""
    import torch
    sc = synth.make_cluster_scene(8_000, 47, 1)
    vw = synth.make_orbit_views(1, 48, 3840, 2160)
    d = gs.DeviceScene.from_scene(sc)
    s16, _ = gs.sensitivity(d, vw, tile=(16, 16))
    s32, _ = gs.sensitivity(d, vw, tile=(32, 32))
    assert torch.equal(s16, s32)
    assert float(s16.max()) > 0.0
