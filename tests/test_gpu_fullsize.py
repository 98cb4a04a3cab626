"""Parity at the benchmark's full size: 1 000 000 Gaussians (64 clusters +
10% uniform background, SH degree 3) seen from 100 jittered-orbit views at
1280x720, in the launch configuration bench.py times (all 100 views in one
call).  The FP64 oracle cannot composite all 9.2e7 rays in a test, so it
scores a sample of them: three whole 64x64 pixel blocks in three views and
200 random rays in each of ten views (minus the rays it flags as ambiguous).
On that sample the GPU's sensitivities (same ray mask) and its per-ray A
must match the oracle element by element; over all rays, properties that
hold at any size are checked (s in [0, 1], 1 <= S <= rays with A > 0, and
unmasked s >= masked s exactly, since both runs compute the same per-ray
shares)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

REL, ABS = 1e-5, 1e-12
W, H = 1280, 720


@pytest.fixture(scope="module")
def gs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_02721_amd as gs
    gs.load()
    return gs


def _sample_rays(n_rays):
    keep = np.zeros(n_rays, bool)
    for v, (x0, y0) in ((0, (608, 328)), (37, (0, 0)), (99, (1216, 656))):
        base = v * W * H
        for y in range(y0, y0 + 64):
            keep[base + y * W + x0: base + y * W + x0 + 64] = True
    rng = np.random.default_rng(5)
    for v in rng.choice(100, 10, replace=False):
        keep[v * W * H + rng.choice(W * H, 200, replace=False)] = True
    return keep


def _mask_tensor(keep):
    import torch
    return torch.as_tensor(synth.pack_bits(keep).view(np.int32)).cuda()


def test_scene1m_full_size_sampled_parity(gs, ora):
    import torch
    sc = synth.make_cluster_scene(1_000_000, 1, 3)
    vw = synth.make_orbit_views(100, 101)
    assert vw.n_rays == 100 * W * H
    keep = _sample_rays(vw.n_rays)
    params = ora.default_params()
    flagged = ora.sensitivity(sc, vw, params, synth.pack_bits(keep))["flag"]
    keep &= ~flagged
    ref = ora.sensitivity(sc, vw, params, synth.pack_bits(keep))
    print(f"[scene1m] sampled rays {int(keep.sum())} (flagged {int(flagged.sum())}), "
          f"oracle pairs {ref['pairs']}", flush=True)

    d = gs.DeviceScene.from_scene(sc)
    s_full, st = gs.sensitivity(d, vw, stats=True)
    s_mask, _ = gs.sensitivity(d, vw, ray_mask=_mask_tensor(keep))
    ob = gs.render_objective(d, vw, None, gs.OBJ_FULL, per_ray=True, per_view=False, diag=False)
    torch.cuda.synchronize()

    # sensitivities over the sampled rays, every Gaussian
    s = s_mask.double().cpu().numpy()
    excess = np.abs(s - ref["s"]) - (REL * ref["s"] + ABS)
    worst = int(np.argmax(excess))
    big = ref["s"] > 1e-9
    print(f"[scene1m] s>0 on {int((ref['s'] > 0).sum())} Gaussians; max rel err where s > 1e-9: "
          f"{np.max(np.abs(s[big] - ref['s'][big]) / ref['s'][big]):.2e}", flush=True)
    assert excess.max() <= 0, (worst, s[worst], ref["s"][worst])

    # per-ray A on the sampled rays (from the unmasked full-scene objective)
    A_gpu = ob["per_ray"].double().cpu().numpy()[keep]
    A_ref = ref["A"][keep]
    assert np.all(np.abs(A_gpu - A_ref) <= REL * A_ref + 1e-30)

    # properties over all rays
    sf = s_full.cpu()
    sm = s_mask.cpu()
    assert bool((sf >= 0).all()) and bool((sf <= 1).all())
    assert bool((sf >= sm).all())
    S = st["total_sensitivity"]
    n_pos = int((ob["per_ray"] > 0).sum().item())
    assert 1.0 <= S <= n_pos
    print(f"[scene1m] S = {S:.1f} over {n_pos} rays with A > 0", flush=True)


def _dequantized(sc):
    """The scene exactly as the mixed-precision planes hold it (bf16 mean,
    log-scale and SH; f16 quaternion and opacity), widened to float32."""
    import torch
    q = lambda a, dt: torch.as_tensor(a).to(dt).to(torch.float32).numpy()
    return synth.Scene(q(sc.mean, torch.bfloat16), q(sc.log_scale, torch.bfloat16),
                       q(sc.quat, torch.float16), q(sc.opacity, torch.float16),
                       q(sc.sh, torch.bfloat16), sc.sh_degree)


def _sample_rays_1080(n_rays, views=200, Wd=1920, Hd=1080):
    keep = np.zeros(n_rays, bool)
    for v, (x0, y0) in ((0, (928, 508)), (67, (0, 0)), (199, (1856, 1016))):
        base = v * Wd * Hd
        for y in range(y0, y0 + 64):
            keep[base + y * Wd + x0: base + y * Wd + x0 + 64] = True
    # 200 random rays in each of 5 views, drawn from 8 random rows per view
    # (the oracle's cost grows with the number of 16-row bands it visits)
    rng = np.random.default_rng(6)
    for v in rng.choice(views, 5, replace=False):
        rows = rng.choice(Hd, 8, replace=False)
        for y in rows:
            keep[v * Wd * Hd + y * Wd + rng.choice(Wd, 25, replace=False)] = True
    return keep


def test_precision3m_full_size_sampled_parity(gs, ora):
    """The precision workload at full size: 3 000 000 Gaussians (SH degree 3)
    stored as bf16 means, log-scales and SH with f16 quaternions and
    opacities, seen from 200 orbit views at 1920x1080, all views in one call.
    The oracle scores three 64x64 blocks and 1 000 random rays on 40 random
    rows (minus the rays it flags as ambiguous on either scene).  Gated: the mixed16 pass against
    the oracle on the dequantized scene and the float32 pass against the
    oracle on the float32 scene, both at the float32 bar.  Reported: the
    mixed16 sensitivities against the float32 scene's (quantisation error) and
    the coreset error of a mixed16 draw at m = 10% N."""
    import time
    import torch
    sc, vw, m, seed = synth.make_config("precision3m")
    assert sc.n == 3_000_000 and vw.n_views == 200 and tuple(vw.size[0]) == (1920, 1080)
    dq = _dequantized(sc)
    keep = _sample_rays_1080(vw.n_rays)
    params = ora.default_params()
    t0 = time.perf_counter()
    flagged = ora.sensitivity(dq, vw, params, synth.pack_bits(keep))["flag"]
    flagged |= ora.sensitivity(sc, vw, params, synth.pack_bits(keep))["flag"]
    keep &= ~flagged
    bits = synth.pack_bits(keep)
    ref_dq = ora.sensitivity(dq, vw, params, bits)
    ref_sc = ora.sensitivity(sc, vw, params, bits)
    print(f"[precision3m] sampled rays {int(keep.sum())} (flagged {int(flagged.sum())}), oracle "
          f"{time.perf_counter() - t0:.1f} s", flush=True)

    d16 = gs.DeviceScene.from_scene(sc, fmt=gs.ATTR_MIXED16)
    d32 = gs.DeviceScene.from_scene(sc)
    mask = _mask_tensor(keep)
    s16, st16 = gs.sensitivity(d16, vw, ray_mask=mask, stats=True)
    s32, _ = gs.sensitivity(d32, vw, ray_mask=mask)
    torch.cuda.synchronize()
    print(f"[precision3m] mixed16 masked pass: entries {st16['n_entries']}, stages "
          f"{ {k: round(v, 1) for k, v in st16.items() if k.startswith('ms_')} }", flush=True)
    for label, s, ref in (("mixed16 vs dequantized", s16, ref_dq["s"]), ("float32 vs float32", s32, ref_sc["s"])):
        s = s.double().cpu().numpy()
        excess = np.abs(s - ref) - (REL * ref + ABS)
        worst = int(np.argmax(excess))
        big = ref > 1e-9
        print(f"[precision3m] {label}: s>0 on {int((ref > 0).sum())}, max rel err where s > 1e-9 "
              f"{np.max(np.abs(s[big] - ref[big]) / ref[big]):.2e}", flush=True)
        assert excess.max() <= 0, (label, worst, s[worst], ref[worst])
    s = s16.double().cpu().numpy()
    big = ref_sc["s"] > 1e-3
    rel = np.abs(s[big] - ref_sc["s"][big]) / ref_sc["s"][big]
    print(f"[precision3m] mixed16 vs float32 scene (quantisation): median rel {np.median(rel):.2e}, "
          f"p99 {np.quantile(rel, 0.99):.2e} on {int(big.sum())} Gaussians with s > 1e-3", flush=True)

    # unmasked passes: properties at any size, and a coreset drawn from mixed16
    full16, st = gs.sensitivity(d16, vw, stats=True)
    torch.cuda.synchronize()
    print(f"[precision3m] mixed16 full pass {sum(v for k, v in st.items() if k.startswith('ms_')):.1f} ms of "
          f"stages, S = {st['total_sensitivity']:.1f}", flush=True)
    sf = full16.cpu()
    assert bool((sf >= 0).all()) and bool((sf <= 1).all())
    assert bool((sf >= s16.cpu()).all())
    assert st["total_sensitivity"] >= 1.0
    _, w, _ = gs.sample_coreset(full16, m, seed)
    judge = torch.as_tensor(synth.block_subsample_mask(vw, 3).view(np.int32)).cuda()
    pv = gs.render_objective(d32, vw, w, gs.OBJ_FIXED, ray_mask=judge, per_ray=False, diag=False)["per_view"]
    print(f"[precision3m] coreset error of the mixed16 draw on the float32 scene (m = {m}): "
          f"{gs.coreset_error(pv):.4f}", flush=True)
