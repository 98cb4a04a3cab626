"""The C ABI's allocator hook and ambiguity reporting on the GPU: scratch
arenas and plan buffers taken from torch's caching allocator give the same
bits as hipMalloc'd ones and go back to torch when the hook is removed; the
GPU's own ambiguity flags and counters are consistent with the oracle's."""
import numpy as np
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


def _work(gs, d, vw, plan_batch):
    import torch
    s, st = gs.sensitivity(d, vw, stats=True)
    c, w, sup = gs.sample_coreset(s, 500, 3)
    plan = gs.Plan([b for b, _ in plan_batch], [v for _, v in plan_batch])
    outs = [o.clone() for o in plan.run()]
    torch.cuda.synchronize()
    plan.close()
    return [s.clone(), c.clone(), w.clone(), sup.clone()] + outs


def test_torch_allocator_gives_same_bits(gs):
    import torch
    sc = synth.make_cluster_scene(20_000, 41, 3)
    vw = synth.make_orbit_views(4, 42, 160, 96)
    d = gs.DeviceScene.from_scene(sc)
    batch = [(gs.DeviceScene.from_scene(synth.make_cluster_scene(7_000, 43, 1)), synth.make_orbit_views(3, 44, 96, 64)),
             (d, vw)]
    ref = _work(gs, d, vw, batch)
    gs.release_workspace()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    gs.use_torch_allocator(True)
    try:
        got = _work(gs, d, vw, batch)
        torch.cuda.synchronize()
        held = torch.cuda.memory_allocated() - base
        print(f"[allocator] library memory held through torch: {held / 2**20:.1f} MiB", flush=True)
        assert held > 0 and held > sum(t.numel() * t.element_size() for t in got)
        same = all(torch.equal(a, b) for a, b in zip(ref, got))
        del got
        assert same
    finally:
        gs.use_torch_allocator(False)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
    # and the default allocator works again afterwards
    again = _work(gs, d, vw, batch)
    for a, b in zip(ref, again):
        assert torch.equal(a, b)


def test_allocator_argument_errors(gs):
    import ctypes as C
    from paper_2607_02721_amd import _lib
    fn = C.cast(C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)(lambda *a: None), C.c_void_p)
    assert _lib.load().gs_set_allocator(fn, None, None) == 1


def test_gpu_ambiguity_flags_and_counts(gs, ora):
    """The GPU flags a ray when one of its pairs lies within 1e-5 r^2 of the
    cutoff in its own arithmetic; those rays are (almost all) the oracle's
    flagged rays too, the pair counter matches the flagged rays, and depth
    keys near a float32 midpoint are counted."""
    sc = synth.make_cluster_scene(20_000, 7, 3)
    vw = synth.make_orbit_views(3, 17, 200, 136)
    d = gs.DeviceScene.from_scene(sc)
    gflag, st = parity_util.gpu_flags(gs, d, vw)
    ref = ora.sensitivity(sc, vw)
    both = int((gflag & ref["flag"]).sum())
    print(f"[ambiguity] gpu {int(gflag.sum())} oracle {int(ref['flag'].sum())} both {both}; pairs "
          f"{st['n_ambiguous_pairs']}, keys {st['n_ambiguous_keys']}", flush=True)
    assert st["n_ambiguous_pairs"] >= int(gflag.sum()) > 0
    assert both >= 0.9 * int(gflag.sum())
    # keys are counted for the Gaussians on screen: between the oracle's
    # ambiguous keys whose footprint box certainly meets the image and those
    # whose box meets it within a pixel
    pr = ora.project(sc, vw)
    W, H = vw.size[:, 0][:, None], vw.size[:, 1][:, None]
    mx, my = pr["mean2d"][..., 0], pr["mean2d"][..., 1]
    rx, ry = pr["radius"][..., 0], pr["radius"][..., 1]
    def on_screen(pad):
        return (pr["present"] & (mx + rx + pad >= 0.5) & (mx - rx - pad <= W - 0.5)
                & (my + ry + pad >= 0.5) & (my - ry - pad <= H - 0.5))
    amb = pr["key_ambiguous"]
    lo, hi = int((amb & on_screen(-1.0)).sum()), int((amb & on_screen(1.0)).sum())
    assert lo <= st["n_ambiguous_keys"] <= hi
    import torch
    with pytest.raises(gs.GsError):
        gs.sensitivity(d, vw, ambiguous_rays=torch.zeros(10, dtype=torch.int32, device="cuda"))
