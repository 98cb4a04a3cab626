"""Learned proposal on the GPU: MFMA MLP forward/gradient against the FP64
reference (same bf16-rounded weights and inputs; the FP32 mode of the same
kernels at 1e-5), the Adam step against the FP64 reference, deterministic
training, neighbour sets bit-exact and all 64 features against the oracle,
training, the gain over uniform sampling, and the fallback."""
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


@pytest.fixture(scope="module")
def L(gs):
    from paper_2607_02721_amd import learned
    return learned


def _bf16(t):
    import torch
    return t.to(torch.bfloat16).to(torch.float32)


def _ref_inputs(prop, feat):
    """Parameters and standardised inputs exactly as the BF16 kernels see them."""
    import torch
    from oracle import mlp_ref  # noqa: F401
    P = prop.params.detach().clone()
    for a, b in ((0, 16384), (16640, 82176), (82432, 147968), (148224, 148480)):
        P[a:b] = _bf16(P[a:b])
    X = _bf16((feat - prop.norm[0]) * prop.norm[1])
    return P.double().cpu().numpy(), X.double().cpu().numpy()


def _random_batch(n, seed=0):
    import torch
    g = torch.Generator().manual_seed(seed)
    feat = (torch.randn(n, 64, generator=g) * 2 + 0.5).cuda()
    y = torch.randn(n, generator=g).cuda() * 3 - 5
    return feat, y


def test_forward_matches_reference(gs, L):
    from oracle import mlp_ref
    feat, _ = _random_batch(1000)
    prop = L.Proposal(seed=3)
    prop.set_norm(L.feature_stats(feat))
    got = prop.predict(feat).double().cpu().numpy()
    P, X = _ref_inputs(prop, feat)
    want = mlp_ref.forward(P, X)[0]
    err = np.abs(got - want)
    print(f"[mlp fwd] max abs {err.max():.3e} (output std {want.std():.3e})")
    assert err.max() <= 2e-2 * max(want.std(), 1e-3) + 1e-3


def test_gradient_matches_reference(gs, L):
    from oracle import mlp_ref
    feat, y = _random_batch(4096, seed=1)
    prop = L.Proposal(seed=5)
    prop.set_norm(L.feature_stats(feat))
    loss, grad = prop.gradient(feat, y)
    P, X = _ref_inputs(prop, feat)
    l_ref, g_ref = mlp_ref.loss_and_grad(P, X, y.double().cpu().numpy())
    g = grad.double().cpu().numpy()
    cos = float(g @ g_ref / (np.linalg.norm(g) * np.linalg.norm(g_ref)))
    rel = float(np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref))
    print(f"[mlp grad] loss {float(loss.item()):.6f} vs {l_ref:.6f}; cos {cos:.6f} rel-L2 {rel:.3e}")
    assert abs(float(loss.item()) - l_ref) <= 1e-3 * l_ref
    assert cos >= 0.999 and rel <= 1e-2
    # per-block checks: every layer's gradient agrees, not only the total
    for a, b in ((0, 16384), (16640, 82176), (82432, 147968), (148224, 148480)):
        r = np.linalg.norm(g[a:b] - g_ref[a:b]) / np.linalg.norm(g_ref[a:b])
        assert r <= 2e-2, (a, b, r)


def test_gradient_fp32_mode_matches_reference(gs, L):
    """The FP32 mode of the same kernels (FP32 operands on
    v_mfma_f32_16x16x4_f32, FP32 activations) against the FP64 reference on
    the same FP32 parameters and standardised inputs: loss and every layer's
    gradient within 1e-5 relative (L2)."""
    from oracle import mlp_ref
    feat, y = _random_batch(4096, seed=2)
    prop = L.Proposal(seed=6)
    prop.set_norm(L.feature_stats(feat))
    loss, grad = prop.gradient(feat, y, fp32=True)
    P = prop.params.double().cpu().numpy()
    X = ((feat - prop.norm[0]) * prop.norm[1]).double().cpu().numpy()
    l_ref, g_ref = mlp_ref.loss_and_grad(P, X, y.double().cpu().numpy())
    g = grad.double().cpu().numpy()
    rels = []
    for a, b in ((0, 16384), (16384, 16640), (16640, 82176), (82176, 82432), (82432, 147968),
                 (147968, 148224), (148224, 148481)):
        rels.append(float(np.linalg.norm(g[a:b] - g_ref[a:b]) / np.linalg.norm(g_ref[a:b])))
    print(f"[mlp grad fp32] loss {float(loss.item()):.8f} vs {l_ref:.8f}; rel-L2 per block "
          + " ".join(f"{r:.2e}" for r in rels), flush=True)
    assert abs(float(loss.item()) - l_ref) <= 1e-5 * l_ref
    assert max(rels) <= 1e-5


def test_adam_step_matches_reference(gs, L):
    """Two training steps: the parameters and both moments after each equal
    the FP64 Adam step applied to the gradient the kernels computed (the
    update itself is checked, the gradient is checked above)."""
    import torch
    from oracle import mlp_ref
    feat, y = _random_batch(2048, seed=4)
    prop = L.Proposal(seed=8)
    prop.set_norm(L.feature_stats(feat))
    P = prop.params.double().cpu().numpy()
    m = np.zeros_like(P)
    v = np.zeros_like(P)
    for step, lr in ((1, 1e-3), (2, 3e-3)):
        g = torch.empty_like(prop.params)
        prop.train_step(feat, y, lr=lr, grad=g)
        torch.cuda.synchronize()
        P, m, v = mlp_ref.adam_step(P, m, v, g.double().cpu().numpy(), step, lr)
        got_P = prop.params.double().cpu().numpy()
        got_m = prop.adam[:prop.P].double().cpu().numpy()
        got_v = prop.adam[prop.P:].double().cpu().numpy()
        scale = np.abs(m).max()
        assert np.all(np.abs(got_m - m) <= 1e-6 * np.abs(m) + 1e-7 * scale), step
        assert np.all(np.abs(got_v - v) <= 1e-6 * np.abs(v) + 1e-30), step
        # the step is at most lr per parameter: compare it to lr, and the
        # parameters to their float32 rounding
        assert np.all(np.abs(got_P - P) <= 2e-6 * lr + 2e-7 * np.abs(P)), step
        P = got_P.copy()    # continue from the float32 parameters the kernels hold


def test_training_is_deterministic(gs, L):
    """Two runs of the same training steps give bit-identical parameters."""
    import torch
    feat, y = _random_batch(20_000, seed=9)
    outs = []
    for _ in range(2):
        prop = L.Proposal(seed=2)
        prop.set_norm(L.feature_stats(feat))
        for k in range(3):
            prop.train_step(feat[k * 5000:(k + 2) * 5000].contiguous(), y[k * 5000:(k + 2) * 5000].contiguous(),
                            lr=1e-3)
        torch.cuda.synchronize()
        outs.append(prop.params.clone())
    assert torch.equal(outs[0], outs[1])


def _dequantized(sc):
    """The float32 values of a mixed16 scene (bf16 mean, log-scale, SH; f16
    quaternion and opacity), exactly as the kernels widen them."""
    import torch
    q = lambda a, dt: np.ascontiguousarray(torch.as_tensor(np.asarray(a, np.float32)).to(dt).float().numpy())
    return synth.Scene(q(sc.mean, torch.bfloat16), q(sc.log_scale, torch.bfloat16),
                       q(sc.quat, torch.float16), q(sc.opacity, torch.float16),
                       q(sc.sh, torch.bfloat16), sc.sh_degree)


def _knn_check(gs, L, ora, sc, label, fmt=None):
    """Neighbour indices and float32 squared distances bit-exact against the
    oracle's brute force; every feature column against the FP64 features."""
    import torch
    d = gs.DeviceScene.from_scene(sc) if fmt is None else gs.DeviceScene.from_scene(sc, fmt=fmt)
    if fmt is not None:     # the oracle sees the dequantized scene the kernels read
        sc = _dequantized(sc)
    idx, d2 = L.knn(d)
    f = L.features(d)
    torch.cuda.synchronize()
    ref_f, ref_idx, ref_d2 = ora.features(sc)
    gi = idx.cpu().numpy().view(np.uint32)
    gd = d2.cpu().numpy()
    bad = np.nonzero(np.any(gi != ref_idx, axis=1))[0]
    print(f"[knn {label}] n={sc.n} rows with other neighbours: {bad.size}", flush=True)
    assert bad.size == 0, (bad[:5], gi[bad[:1]], ref_idx[bad[:1]])
    assert np.array_equal(gd.view(np.uint32), ref_d2.view(np.uint32))
    g = f.cpu().numpy().astype(np.float64)
    exact = list(range(0, 6)) + list(range(11, 59)) + [62]
    assert np.array_equal(g[:, exact], ref_f[:, exact])
    tol = {6: 1e-6, 7: 1e-6, 8: 1e-6, 9: 1e-6, 10: 1e-5, 59: 1e-5, 60: 1e-5, 61: 1e-6, 63: 1e-5}
    for c, t in tol.items():
        err = np.abs(g[:, c] - ref_f[:, c]) / np.maximum(1.0, np.abs(ref_f[:, c]))
        assert err.max() <= t, (label, c, float(err.max()))


def test_knn_features_match_oracle(gs, L, ora):
    sc = synth.make_cluster_scene(20_000, 11, 3)
    _knn_check(gs, L, ora, sc, "cluster20k")


def test_knn_features_edge_cases(gs, L, ora):
    """Fewer points than neighbours, a lattice full of distance ties (ties go
    by index), coincident means, and mixed16 storage."""
    rng = np.random.default_rng(12)
    for n in (1, 2, 9, 17):
        sc = synth.make_explicit_scene(rng.uniform(-1, 1, (n, 3)), np.full((n, 3), -3.0),
                                       np.tile([1.0, 0, 0, 0], (n, 1)), rng.uniform(0.1, 0.9, n),
                                       colours=np.full((n, 3), 0.5))
        _knn_check(gs, L, ora, sc, f"n={n}")
    g = np.arange(9, dtype=np.float64) * 0.125
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    pts = np.concatenate([pts, pts[:50]])           # 50 coincident pairs
    n = pts.shape[0]
    sc = synth.make_explicit_scene(pts, np.full((n, 3), -3.0), rng.standard_normal((n, 4)),
                                   rng.uniform(0.1, 0.9, n), colours=rng.uniform(0, 1, (n, 3)))
    _knn_check(gs, L, ora, sc, "lattice")
    _knn_check(gs, L, ora, synth.make_cluster_scene(5_000, 13, 2), "mixed16", fmt=gs.ATTR_MIXED16)


def _train_scenes(n_scenes=3, n=60_000, views=20):
    out = []
    for k in range(n_scenes):
        sc = synth.make_cluster_scene(n, 500 + k, 3)
        vw = synth.make_orbit_views(views, 600 + k, 320, 180)
        out.append((sc, vw))
    return out


@pytest.fixture(scope="module")
def trained(gs, L):
    import torch
    feats, targets = [], []
    for sc, vw in _train_scenes():
        d = gs.DeviceScene.from_scene(sc)
        s, _ = gs.sensitivity(d, vw)
        feats.append(L.features(d))
        targets.append(L.log_targets(s))
    prop = L.Proposal(seed=0)
    losses = prop.fit(feats, targets, epochs=12, batch=8192, lr=2e-3)
    torch.cuda.synchronize()
    return prop, losses


def test_training_reduces_loss(trained):
    prop, losses = trained
    print("[train] losses", [round(x, 3) for x in losses])
    assert losses[-1] < 0.6 * losses[0]


def test_learned_proposal_beats_uniform(gs, L, trained):
    """Held-out scene, equal m: the MLP mixture has a smaller coreset-objective
    error than uniform sampling (averaged over seeds)."""
    import torch
    prop, _ = trained
    sc = synth.make_cluster_scene(60_000, 777, 3)
    vw = synth.make_orbit_views(20, 778, 320, 180)
    d = gs.DeviceScene.from_scene(sc)
    feat = L.features(d)
    scores = L.mixture(prop.predict(feat))
    uni = torch.ones(sc.n, device="cuda")
    s_exact, _ = gs.sensitivity(d, vw)
    m = sc.n // 10
    errs = {"learned": [], "uniform": [], "exact": []}
    for seed in range(4):
        for name, sc_ in (("learned", scores), ("uniform", uni), ("exact", s_exact)):
            _, w, _ = gs.sample_coreset(sc_, m, seed)
            ob = gs.render_objective(d, vw, w, gs.OBJ_FIXED, per_ray=False, diag=False)
            errs[name].append(gs.coreset_error(ob["per_view"]))
    mean = {k: float(np.mean(v)) for k, v in errs.items()}
    print("[gain] mean E", mean)
    assert mean["learned"] < mean["uniform"]


def test_fallback_runs_exact_pass(gs, L, trained):
    prop, _ = trained
    sc = synth.make_cluster_scene(30_000, 901, 3)
    vw = synth.make_orbit_views(8, 902, 160, 96)
    d = gs.DeviceScene.from_scene(sc)
    mask = None
    out = L.sample_with_fallback(d, vw, sc.n // 10, 1, prop, mask, err_bound=0.0)
    assert out["fallback"] and "E_exact" in out
    s, _ = gs.sensitivity(d, vw)
    _, w_exact, _ = gs.sample_coreset(s, sc.n // 10, 1)
    assert np.array_equal(out["weights"].cpu().numpy(), w_exact.cpu().numpy())
    out2 = L.sample_with_fallback(d, vw, sc.n // 10, 1, prop, mask, err_bound=1e9)
    assert not out2["fallback"]


def test_mixture_and_targets_match_numpy(gs, L):
    import torch
    g = torch.Generator().manual_seed(7)
    y = (torch.randn(100_003, generator=g) * 4 - 6)
    p = L.mixture(y.cuda(), 0.1).double().cpu().numpy()
    yd = y.double().numpy()
    e = np.exp(yd - yd.max())
    want = 0.9 * e / e.sum() + 0.1 / yd.size
    assert np.allclose(p, want, rtol=1e-6, atol=0)
    assert abs(p.sum() - 1.0) < 1e-5 and p.min() >= 0.1 / yd.size * (1 - 1e-6)
    s = torch.rand(50_000, generator=g) ** 4
    s[::7] = 0.0
    t = L.log_targets(s.cuda()).cpu().numpy()
    ref = np.log(np.maximum(s.double().numpy(), np.float32(L.LOG_FLOOR).astype(np.float64))).astype(np.float32)
    assert np.array_equal(t, ref)


def test_learned_workload_full_size(gs, L, ora, trained):
    """The learned-proposal workload at full size: a held-out scene of
    5 000 000 Gaussians seen from 300 views at 1280x720.  Checked on samples
    the CPU references can afford: kNN features of 2 000 Gaussians against a
    k-d tree over all 5M means, the MLP on 4 096 rows against the FP64
    reference, the mixture's normalisation and floor, the exact pass (the
    fallback) and the fixed objective the judge evaluates on three 64x64
    blocks against the FP64 oracle (with w = 1 the fixed objective is A).
    The judge runs on 1% of the 8x8 blocks of all 300 views; when it sends
    the draw to the fallback, the weights must equal the exact pass's draw."""
    import time
    import torch
    from scipy.spatial import cKDTree
    from oracle import mlp_ref
    prop, _ = trained
    sc = synth.make_cluster_scene(5_000_000, 4200, 3)
    vw = synth.make_orbit_views(300, 4201)
    d = gs.DeviceScene.from_scene(sc)
    feat = L.features(d)
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)

    # kNN features on a sample, against a k-d tree over every mean
    pts = sc.mean.T.astype(np.float64)
    qi = rng.choice(sc.n, 2000, replace=False)
    dist, idx = cKDTree(pts).query(pts[qi], k=17)
    dist, idx = dist[:, 1:], idx[:, 1:]
    f = feat[torch.as_tensor(qi).cuda()].double().cpu().numpy()
    assert np.allclose(f[:, 59], np.log(dist.mean(1)), atol=1e-4)
    assert np.allclose(f[:, 60], np.log(dist[:, -1]), atol=1e-4)
    ok = np.abs(f[:, 61] - sc.opacity.astype(np.float64)[idx].mean(1)) < 1e-5
    assert ok.mean() > 0.995
    print(f"[learned5m] kNN features agree on {ok.mean():.4f} of 2000 sampled Gaussians", flush=True)

    # MLP forward on sampled rows
    rows = torch.as_tensor(rng.choice(sc.n, 4096, replace=False)).cuda()
    got = prop.predict(feat[rows].contiguous()).double().cpu().numpy()
    P, X = _ref_inputs(prop, feat[rows].contiguous())
    want = mlp_ref.forward(P, X)[0]
    assert np.abs(got - want).max() <= 2e-2 * max(want.std(), 1e-3) + 1e-3

    # proposal: a distribution with the uniform floor
    scores = L.mixture(prop.predict(feat))
    ps = scores.double()
    assert abs(float(ps.sum()) - 1.0) < 1e-4 and float(ps.min()) >= 0.1 / sc.n * (1 - 1e-5)

    # draw, judge on 1% of the 8x8 blocks, fall back to the exact pass when E > 1%
    judge = torch.as_tensor(synth.block_subsample_mask(vw, 4202).view(np.int32)).cuda()
    m = sc.n // 10
    out = L.sample_with_fallback(d, vw, m, 0, prop, judge, feat=feat)
    print(f"[learned5m] E learned {out['E_learned']:.4f}, propose {out['ms_propose']:.1f} ms, judge "
          f"{out['ms_judge']:.1f} ms, fallback {out['fallback']}", flush=True)
    if out["fallback"]:
        s, _ = gs.sensitivity(d, vw)
        _, w_exact, _ = gs.sample_coreset(s, m, 0)
        assert torch.equal(out["weights"], w_exact)
        print(f"[learned5m] exact fallback E {out['E_exact']:.4f} in {out['ms_fallback']:.1f} ms", flush=True)

    # the exact pass and the fixed objective against the oracle on three blocks
    W, H = 1280, 720
    keep = np.zeros(vw.n_rays, bool)
    for v, (x0, y0) in ((0, (608, 328)), (150, (0, 0)), (299, (1216, 656))):
        for y in range(y0, y0 + 64):
            keep[v * W * H + y * W + x0: v * W * H + y * W + x0 + 64] = True
    params = ora.default_params()
    t0 = time.perf_counter()
    keep &= ~ora.sensitivity(sc, vw, params, synth.pack_bits(keep))["flag"]
    ref = ora.sensitivity(sc, vw, params, synth.pack_bits(keep))
    print(f"[learned5m] oracle on {int(keep.sum())} rays in {time.perf_counter() - t0:.1f} s", flush=True)
    mask = torch.as_tensor(synth.pack_bits(keep).view(np.int32)).cuda()
    s_m, _ = gs.sensitivity(d, vw, ray_mask=mask)
    s_m = s_m.double().cpu().numpy()
    excess = np.abs(s_m - ref["s"]) - (1e-5 * ref["s"] + 1e-12)
    assert excess.max() <= 0, int(np.argmax(excess))
    ones = torch.ones(sc.n, dtype=torch.float64, device="cuda")
    ob = gs.render_objective(d, vw, ones, gs.OBJ_FIXED, ray_mask=mask, per_view=False, diag=False)
    A_gpu = ob["per_ray"][torch.as_tensor(np.flatnonzero(keep)).cuda()].double().cpu().numpy()
    A_ref = ref["A"][keep]
    assert np.all(np.abs(A_gpu - A_ref) <= 1e-5 * A_ref + 1e-30)
