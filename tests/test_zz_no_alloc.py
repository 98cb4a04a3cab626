"""The allocation-free sampler (gs_sample_coreset_noalloc) against
gs_sample_coreset through the C ABI: bit-identical counts, weights and
support on two calls in a row, the second with fewer Gaussians (the fixed
scratch keeps the first call's contents), and the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_02721_amd as gs
    gs.load()
    return gs


def _draw(gs, s, m, seed, noalloc):
    import torch
    c, w, sup = gs.sample_coreset(s, m, seed, noalloc=noalloc)
    torch.cuda.synchronize()
    return c.cpu().numpy().view(np.uint32), w.cpu().numpy().view(np.uint64), int(sup.item())


def test_noalloc_matches_allocating_sampler_twice(gs):
    import torch
    rng = np.random.default_rng(31)
    for n, m, seed in ((1_000_000, 100_000, 0), (70_001, 9_000, 2 ** 40 + 3)):
        x = rng.uniform(0, 1, n).astype(np.float32)
        x[rng.uniform(size=n) < 0.3] = 0.0
        s = torch.as_tensor(x).cuda()
        a = _draw(gs, s, m, seed, False)
        b = _draw(gs, s, m, seed, True)
        print(f"[noalloc] n={n} m={m} support={b[2]}", flush=True)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_noalloc_errors(gs):
    import torch
    big = torch.zeros((1 << 23) + 1, dtype=torch.float32, device="cuda")
    with pytest.raises(gs.GsError) as e:
        gs.sample_coreset(big, 10, 0, noalloc=True)
    assert e.value.status == 2 and "exceeds" in str(e.value)
    with pytest.raises(gs.GsError) as e:
        gs.sample_coreset(torch.zeros(100, device="cuda"), 10, 0, noalloc=True)
    assert e.value.status == 4
    bad = torch.full((100,), 0.5, device="cuda")
    bad[3] = 1.5
    with pytest.raises(gs.GsError) as e:
        gs.sample_coreset(bad, 10, 0, noalloc=True)
    assert e.value.status == 5
    # a good call after the errors is still right
    ok = torch.rand(5000, device="cuda")
    a = _draw(gs, ok, 400, 9, False)
    b = _draw(gs, ok, 400, 9, True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
