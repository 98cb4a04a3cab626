"""Compact-region extension on the GPU (gs_region_bound) against the FP64
region oracle: the same representatives, the same kept pixels (up to float32
decisions at the floor), Lipschitz estimates, eps_0 and Theorem 4's eps_reg,
and the bound holding at every sampled query."""
import numpy as np
import pytest

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


@pytest.mark.parametrize("objective", ["true", "fixed"])
def test_region_bound_matches_oracle(gs, ora, objective):
    import torch
    from oracle import region
    sc, vw, m, seed = synth.make_config("tiny")
    K = 24
    w2c = synth.make_pose_region(vw.world_to_cam[0], K, 0.05, 0.03, seed=5)
    views = synth.Views(np.stack(w2c), np.repeat(vw.intrinsics[:1], K, 0), np.repeat(vw.size[:1], K, 0))
    d = gs.DeviceScene.from_scene(sc)
    s, _ = gs.sensitivity(d, vw)
    _, w, _ = gs.sample_coreset(s, 1500, seed)
    full = gs.render_objective(d, views, None, gs.OBJ_FULL, per_view=False, diag=False)["per_ray"]
    obj = gs.OBJ_TRUE if objective == "true" else gs.OBJ_FIXED
    red = gs.render_objective(d, views, w, obj, per_view=False, diag=False)["per_ray"]
    P = int(vw.size[0, 0] * vw.size[0, 1])
    rep, net = gs.region_bound(views.world_to_cam, full.reshape(K, P).contiguous(), red.reshape(K, P).contiguous(),
                               lam=1.0, rho_target=0.04, a_floor=1e-3)
    ob = ora.objective(sc, views, w.cpu().numpy())
    A = ob["A"].reshape(K, P)
    Aw = (ob["A_true"] if objective == "true" else ob["A_fixed"]).reshape(K, P)
    keep = np.all(A > 1e-3, axis=0)
    D = region.distance_matrix(w2c, 1.0)
    net_ref, rho_ref = region.rho_net(D, 0.04)
    ref = region.region_bound(A, Aw, D, net_ref, keep)
    print(f"[region {objective}] gpu {rep}; oracle "
          f"{ {k: v for k, v in ref.items() if k != 'err_per_pose'} }; kept {int(keep.sum())}", flush=True)
    assert sorted(np.nonzero(net)[0].tolist()) == sorted(net_ref)
    assert abs(rep["rho"] - rho_ref) <= 1e-12
    assert abs(rep["n_pixels"] - int(keep.sum())) <= 2
    for k in ("L_full", "L_w", "A_min", "eps_0", "max_err"):
        assert abs(rep[k] - ref[k]) <= 2e-3 * abs(ref[k]) + 1e-9, k
    assert abs(rep["eps_reg"] - ref["eps_reg"]) <= 5e-3 * ref["eps_reg"]
    # Theorem 4 at every sampled query, on the GPU's own values
    assert rep["eps_0"] <= rep["max_err"] <= rep["eps_reg"]
    # the reduced render of a weight-1 scene is the full one: eps_0 = 0 and the
    # bound reduces to the cover term
    ones = torch.ones(sc.n, dtype=torch.float64, device="cuda")
    same = gs.render_objective(d, views, ones, obj, per_view=False, diag=False)["per_ray"]
    rep1, _ = gs.region_bound(views.world_to_cam, full.reshape(K, P).contiguous(), same.reshape(K, P).contiguous(),
                              lam=1.0, rho_target=0.04, a_floor=1e-3)
    assert rep1["eps_0"] <= 1e-5 and rep1["max_err"] <= 1e-5
    assert abs(rep1["L_w"] - rep1["L_full"]) <= 1e-4 * rep1["L_full"]
