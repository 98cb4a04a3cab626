"""Pins of the FP64 MLP reference: analytic gradient vs central differences,
forward values and gradients vs torch.nn layers and autograd, the Adam step
by hand and vs torch.optim.Adam,
and a hand-computed one-hidden-unit case of SiLU's derivative."""
import numpy as np

from oracle import mlp_ref


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    P = rng.normal(0, 0.08, 148481)
    X = rng.normal(0, 1, (12, 64))
    y = rng.normal(0, 1, 12)
    loss, g = mlp_ref.loss_and_grad(P, X, y)
    idx = np.concatenate([rng.choice(16384, 6), 16384 + rng.choice(256, 3), 16640 + rng.choice(65536, 6),
                          82432 + rng.choice(65536, 6), 147968 + rng.choice(256, 3),
                          148224 + rng.choice(256, 4), [148480]])
    h = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (mlp_ref.loss_and_grad(Pp, X, y)[0] - mlp_ref.loss_and_grad(Pm, X, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_silu_derivative_closed_form():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (mlp_ref.silu(z + h) - mlp_ref.silu(z - h)) / (2 * h)
    assert np.allclose(mlp_ref.silu_grad(z), fd, atol=1e-9)
    assert mlp_ref.silu(0.0) == 0.0 and abs(mlp_ref.silu_grad(0.0) - 0.5) < 1e-15


def _torch_net(P):
    """The same network built from torch.nn layers on the CPU in float64: an
    implementation independent of the NumPy reference."""
    import torch
    layers, w4, b4 = mlp_ref.unpack(P)
    mods = []
    for W, b in layers:
        lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.as_tensor(W))
            lin.bias.copy_(torch.as_tensor(b))
        mods += [lin, torch.nn.SiLU()]
    head = torch.nn.Linear(256, 1).double()
    with torch.no_grad():
        head.weight.copy_(torch.as_tensor(w4).reshape(1, 256))
        head.bias.copy_(torch.as_tensor([b4]))
    return torch.nn.Sequential(*mods, head)


def test_forward_and_gradient_match_torch_layers():
    """Forward values and the gradient of the mean squared error against
    torch.nn.Linear / SiLU layers and autograd (float64, CPU)."""
    import torch
    rng = np.random.default_rng(3)
    P = rng.normal(0, 0.1, 148481)
    X = rng.normal(0, 1, (37, 64))
    y = rng.normal(0, 1, 37)
    net = _torch_net(P)
    out = net(torch.as_tensor(X)).reshape(-1)
    yhat = mlp_ref.forward(P, X)[0]
    assert np.allclose(out.detach().numpy(), yhat, rtol=1e-12, atol=1e-12)
    loss_t = torch.mean((out - torch.as_tensor(y)) ** 2)
    loss_t.backward()
    g_t = []
    for mod in net:
        if isinstance(mod, torch.nn.Linear):
            g_t += [mod.weight.grad.numpy().ravel(), mod.bias.grad.numpy().ravel()]
    g_t = np.concatenate(g_t)
    loss, g = mlp_ref.loss_and_grad(P, X, y)
    assert abs(loss - float(loss_t.detach())) <= 1e-12 * max(1.0, loss)
    assert np.allclose(g, g_t, rtol=1e-10, atol=1e-13)


def test_adam_two_steps_by_hand():
    """Two Adam steps on one parameter, written out from Kingma & Ba's
    update: after step 1 the bias-corrected moments are g1 and g1^2, so the
    step is lr g1 / (|g1| + eps)."""
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    g1, g2 = 0.5, -2.0
    P1, m1, v1 = mlp_ref.adam_step(np.array([1.0]), np.zeros(1), np.zeros(1), np.array([g1]), 1, lr)
    assert abs(m1[0] - 0.05) < 1e-15 and abs(v1[0] - 0.00025) < 1e-15
    assert abs(P1[0] - (1.0 - lr * 0.5 / (0.5 + eps))) < 1e-15
    P2, m2, v2 = mlp_ref.adam_step(P1, m1, v1, np.array([g2]), 2, lr)
    m2_hand = 0.9 * 0.05 + 0.1 * g2                 # -0.155
    v2_hand = 0.999 * 0.00025 + 0.001 * g2 * g2     # 0.00424975
    step2 = lr * (m2_hand / (1 - b1 ** 2)) / (np.sqrt(v2_hand / (1 - b2 ** 2)) + eps)
    assert abs(m2[0] - m2_hand) < 1e-15 and abs(v2[0] - v2_hand) < 1e-15
    assert abs(P2[0] - (P1[0] - step2)) < 1e-15


def test_adam_matches_torch_optimizer():
    """Five steps against torch.optim.Adam (float64, CPU) on random gradients."""
    import torch
    rng = np.random.default_rng(7)
    P0 = rng.normal(0, 1, 300)
    grads = [rng.normal(0, 1, 300) * 10.0 ** rng.uniform(-4, 1, 300) for _ in range(5)]
    p = torch.nn.Parameter(torch.as_tensor(P0.copy()))
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    P, m, v = P0.copy(), np.zeros(300), np.zeros(300)
    for t, g in enumerate(grads, start=1):
        p.grad = torch.as_tensor(g.copy())
        opt.step()
        P, m, v = mlp_ref.adam_step(P, m, v, g, t, 3e-3)
        assert np.allclose(P, p.detach().numpy(), rtol=0, atol=1e-14)
    st = opt.state[p]
    assert np.allclose(m, st["exp_avg"].numpy(), rtol=1e-14, atol=0)
    assert np.allclose(v, st["exp_avg_sq"].numpy(), rtol=1e-14, atol=0)
