"""Batched plans (several scenes in one captured sequence) against the FP64
oracle (element by element, per scene) and against the per-scene entry
point: every scene's sensitivities must be bit-identical to gs_sensitivity
with the same parameters, for every launch shape, on graph replays, after
in-place attribute updates, and across scene groups.  The list-capacity and
depth-span guards are exercised by changing attributes in place."""
import pytest

import parity_util
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_02721_amd as gs
    gs.load()
    return gs


SPECS = [  # (n, seed, sh degree, views, width, height)
    (20_000, 11, 3, 6, 160, 96),
    (7_001, 12, 1, 3, 200, 136),
    (33_333, 13, 3, 9, 128, 128),
]


def _batch(gs, specs=SPECS):
    out = []
    for n, seed, deg, nv, W, H in specs:
        sc = synth.make_cluster_scene(n, seed, deg)
        vw = synth.make_orbit_views(nv, seed + 100, W, H)
        out.append((gs.DeviceScene.from_scene(sc), vw))
    return out


def _reference(gs, batch):
    return [gs.sensitivity(d, vw)[0].clone() for d, vw in batch]


def _same(a, b):
    import torch
    return torch.equal(a, b)


@pytest.fixture(scope="module")
def batch(gs):
    return _batch(gs)


@pytest.fixture(scope="module")
def ref(gs, batch):
    return _reference(gs, batch)


def test_plan_matches_per_scene_calls(gs, batch, ref):
    import torch
    plan = gs.Plan([d for d, _ in batch], [v for _, v in batch])
    outs = plan.run()
    torch.cuda.synchronize()
    info = plan.info()
    print("[plan]", info)
    assert info["n_scenes"] == 3 and info["n_groups"] == 1
    assert info["n_launches"] == 1 and info["n_compact_launches"] == 1 and info["compact_bytes"] > 0
    plan.status()
    for k, (o, r) in enumerate(zip(outs, ref)):
        assert float(r.max()) > 0.0
        assert _same(o, r), (k, float((o - r).abs().max()))
    plan.close()


def test_plan_matches_oracle(gs, ora):
    """Each scene of a plan against the FP64 oracle, element by element:
    three orbit scenes of mixed sizes and SH degrees, and one whose first
    camera sits close to the cloud (its keys span more than 2^24, so the plan
    sorts that scene with four passes).  Plans take no ray mask, so the
    Gaussians a flagged ray touches are left out (see parity_util)."""
    import torch
    specs = SPECS[:2] + [(4_000, 14, 2, 2, 96, 80)]
    batch = _batch(gs, specs)
    close_sc = synth.make_tiny_scene(3_000, 15)
    close_vw = synth.make_camera_set([(1.3, 0.35, 0.25), (0.0, 3.0, 0.5)], [(0.0, 0.0, 0.0)] * 2, 112, 80, 70.0)
    batch.append((gs.DeviceScene.from_scene(close_sc), close_vw))
    scenes = [synth.make_cluster_scene(n, seed, deg) for n, seed, deg, _, _, _ in specs] + [close_sc]
    plan = gs.Plan([d for d, _ in batch], [v for _, v in batch])
    info = plan.info()
    print("[plan vs oracle]", info, flush=True)
    assert info["n_sort3_scenes"] == len(batch) - 1
    outs = plan.run()
    torch.cuda.synchronize()
    plan.status()
    for k, ((d, vw), sc, o) in enumerate(zip(batch, scenes, outs)):
        ref = ora.sensitivity(sc, vw)
        gflag = parity_util.gpu_flags(gs, d, vw)[0]
        flag = ref["flag"] | gflag
        touched = parity_util.touched_by_flagged(ora, sc, vw, flag)
        worst, compared = parity_util.compare_unmasked(o.cpu().numpy(), ref["s"], touched)
        print(f"[plan vs oracle] scene {k}: n={sc.n} flagged rays {int(flag.sum())}, Gaussians compared "
              f"{compared}, worst excess {worst:.3e}", flush=True)
        assert worst <= 0.0, k
        assert compared >= 0.6 * sc.n
    plan.close()


def test_graph_replays_equal_eager(gs, batch, ref):
    """Each replay, with unrelated eager work and synchronisations between
    replays, reproduces the per-scene results; new output tensors re-capture."""
    import torch
    plan = gs.Plan([d for d, _ in batch], [v for _, v in batch])
    for rep in range(4):
        outs = plan.run()
        x = torch.randn(1 << 20, device="cuda")
        y = (x * 2).sum()            # eager work between replays
        torch.cuda.synchronize()
        assert y.isfinite()
        for k, (o, r) in enumerate(zip(outs, ref)):
            assert _same(o, r), (rep, k)
    assert plan.info()["graph_captured"] == 1
    fresh = [torch.full((d.n,), -1.0, device="cuda") for d, _ in batch]
    plan.run(fresh)
    torch.cuda.synchronize()
    for o, r in zip(fresh, ref):
        assert _same(o, r)
    plan.status()
    plan.close()


@pytest.mark.parametrize("persistent,xcd", [(0, 1), (0, 0), (1, 0), (1, 1)])
def test_launch_shapes_agree(gs, batch, ref, persistent, xcd):
    import torch
    plan = gs.Plan([d for d, _ in batch], [v for _, v in batch])
    plan.set_config(persistent, xcd)
    outs = plan.run()
    outs = plan.run()
    torch.cuda.synchronize()
    for o, r in zip(outs, ref):
        assert _same(o, r)
    plan.close()


def test_tuner_picks_a_shape(gs, batch, ref):
    import torch
    plan = gs.Plan([d for d, _ in batch], [v for _, v in batch])
    best, ms = plan.tune(reps=2)
    print("[tune]", best, ms)
    assert best in ({"persistent": 0, "xcd_remap": 1}, {"persistent": 0, "xcd_remap": 0},
                    {"persistent": 1, "xcd_remap": 0})
    assert all(t > 0 for t in ms)
    info = plan.info()
    assert (info["persistent"], info["xcd_remap"]) == (best["persistent"], best["xcd_remap"])
    outs = plan.run()
    torch.cuda.synchronize()
    for o, r in zip(outs, ref):
        assert _same(o, r)
    plan.close()


def test_in_place_attribute_update(gs):
    """Opacities change in place (same addresses, same footprints): the next
    run sees the new values."""
    import torch
    batch = _batch(gs, SPECS[:2])
    plan = gs.Plan([d for d, _ in batch], [v for _, v in batch])
    plan.run()
    batch[0][0].opacity.mul_(0.5)
    outs = plan.run()
    torch.cuda.synchronize()
    ref = _reference(gs, batch)
    for o, r in zip(outs, ref):
        assert _same(o, r)
    plan.status()
    plan.close()


def test_capacity_guard(gs):
    """Larger footprints than at creation overflow the list capacity of one
    scene: its output is zero, the other scene is unaffected, and the plan's
    status reports it."""
    import torch
    batch = _batch(gs, SPECS[:2])
    plan = gs.Plan([d for d, _ in batch], [v for _, v in batch])
    plan.run()
    torch.cuda.synchronize()
    plan.status()
    batch[0][0].log_scale.add_(1.0)     # e-times larger axes: many more tile entries
    outs = plan.run()
    torch.cuda.synchronize()
    with pytest.raises(gs.GsError) as e:
        plan.status()
    assert e.value.status == 5
    assert "more tile-list entries" in str(e.value) and "depth keys" not in str(e.value)
    assert float(outs[0].abs().max()) == 0.0
    ref1 = gs.sensitivity(*batch[1])[0]
    assert _same(outs[1], ref1)
    plan.close()


def test_depth_span_guard(gs):
    """Scenes whose depth keys span little enough take a three-pass sort; a
    Gaussian moved in place to half a unit in front of a camera stretches
    that view's keys past what three passes order: that scene's output is
    zero, the other scene is unaffected, and the status reports it."""
    import torch
    batch = _batch(gs, SPECS[:2])
    plan = gs.Plan([d for d, _ in batch], [v for _, v in batch])
    info = plan.info()
    print("[span]", info, flush=True)
    assert info["n_sort3_scenes"] == 2
    ref0 = plan.run()[0].clone()
    torch.cuda.synchronize()
    plan.status()
    assert _same(ref0, gs.sensitivity(*batch[0])[0])
    d0, v0 = batch[0]
    M = v0.world_to_cam[0].reshape(3, 4)
    eye = -M[:, :3].T @ M[:, 3]
    d0.mean[:, 0] = torch.as_tensor(eye + 0.5 * M[2, :3], dtype=torch.float32, device="cuda")
    outs = plan.run()
    torch.cuda.synchronize()
    with pytest.raises(gs.GsError) as e:
        plan.status()
    assert e.value.status == 5
    assert "depth keys spanned" in str(e.value) and "tile-list entries" not in str(e.value)
    assert float(outs[0].abs().max()) == 0.0
    assert _same(outs[1], gs.sensitivity(*batch[1])[0])
    plan.close()


def test_scenes_split_into_groups(gs, monkeypatch):
    """With a small scratch budget the plan packs the scenes into several
    groups (one compositing launch each); results are unchanged."""
    import torch
    monkeypatch.setenv("GS_SCRATCH_GB", "0.25")
    specs = [(100_000, 21, 3, 12, 96, 64), (100_000, 22, 3, 12, 96, 64), (5_000, 23, 0, 2, 64, 64)]
    batch = _batch(gs, specs)
    plan = gs.Plan([d for d, _ in batch], [v for _, v in batch])
    info = plan.info()
    print("[groups]", info)
    assert info["n_groups"] >= 2
    outs = plan.run()
    torch.cuda.synchronize()
    monkeypatch.delenv("GS_SCRATCH_GB")
    ref = _reference(gs, batch)
    for o, r in zip(outs, ref):
        assert _same(o, r)
    plan.close()


def _expected_launches(regions, budget):
    """Scenes in order into launches whose compacted regions fit the budget;
    a scene larger than the budget alone, uncompacted: (launches, compacting)."""
    launches, compact, used, last_compact = 0, 0, 0, False
    for r in regions:
        if r > budget:
            launches, used, last_compact = launches + 1, 0, False
            continue
        if not last_compact or used + r > budget:
            launches, compact, used, last_compact = launches + 1, compact + 1, 0, True
        used += r
    return launches, compact


@pytest.mark.parametrize("pool", ["none", "smallest", "all"])
def test_compaction_pool_splits_launches(gs, batch, ref, monkeypatch, pool):
    """The compaction pool bounds which scenes composite together: no pool
    (one launch per scene on the plain lists), a pool that holds only the
    smallest scene's compacted lists (mixed launches), and one that holds all
    three.  Every form gives the per-scene results bit for bit, in both
    launch shapes."""
    import torch
    regions = []
    for d, vw in batch:
        n = gs.sensitivity(d, vw, stats=True)[1]["n_entries"]
        cap = n + n // 64 + 1024
        regions.append((16 * cap + 255) // 256 * 256)
    budget = {"none": 0, "smallest": min(regions), "all": sum(regions)}[pool]
    monkeypatch.setenv("GS_COMPACT_POOL_GB", repr(budget / 2**30))
    plan = gs.Plan([d for d, _ in batch], [v for _, v in batch])
    monkeypatch.delenv("GS_COMPACT_POOL_GB")
    info = plan.info()
    want = _expected_launches(regions, budget)
    print("[pool]", pool, regions, info, flush=True)
    assert (info["n_launches"], info["n_compact_launches"]) == want
    if pool == "none":
        assert want == (3, 0) and info["compact_bytes"] == 0
    if pool == "all":
        assert want == (1, 1) and info["compact_bytes"] == sum(regions)
    for persistent, xcd in ((0, 1), (1, 0)):
        plan.set_config(persistent, xcd)
        outs = plan.run()
        torch.cuda.synchronize()
        for k, (o, r) in enumerate(zip(outs, ref)):
            assert _same(o, r), (pool, persistent, k)
    plan.close()
