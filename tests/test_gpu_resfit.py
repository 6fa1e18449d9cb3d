"""The residual-model regression (voldor_residual_fit) against the FP64 oracle
(oracle/resfit.py), through the C ABI: per-bin counts exactly, the FP64 sums
to 1e-12 relative (the same float inputs, FP64 arithmetic, summed in another
order), and the fitted laws to 1e-9."""
import numpy as np
import pytest
import scipy.stats

from oracle import resfit

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def vo():
    import paper_2104_06789_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _sample(n, seed, laws=(0.02, 0.07, -0.004, 1.3)):
    a1, a2, b1, b2 = laws
    rng = np.random.default_rng(seed)
    v = rng.uniform(0.2, 45.0, n)
    ang = rng.uniform(0, 2 * np.pi, n)
    X = np.stack([v * np.cos(ang), v * np.sin(ang)], axis=1)
    x = np.atleast_1d(scipy.stats.fisk.rvs(c=b1 * v + b2, scale=a1 * np.exp(a2 * v), size=n, random_state=rng))
    phi = rng.uniform(0, 2 * np.pi, n)
    G = X - np.sqrt(x)[:, None] * np.stack([np.cos(phi), np.sin(phi)], axis=1)
    X, G = X.astype(np.float32), G.astype(np.float32)
    X[::997] = np.nan   # skipped items
    return X, G


@pytest.mark.parametrize("n", [1, 1000, 333_333])
def test_residual_bins_and_laws(vo, torch, n):
    X, G = _sample(n, n)
    nb, vmax = 40, 40.0
    if n < 1000:
        with pytest.raises(vo.VoldorError):
            vo.residual_fit(torch.from_numpy(X).cuda(), torch.from_numpy(G).cuda(), nb, vmax)
        return
    laws, bins = vo.residual_fit(torch.from_numpy(X).cuda(), torch.from_numpy(G).cuda(), nb, vmax,
                                 min_count=8)
    ref = resfit.bin_stats(X, G, nb, vmax)
    assert np.array_equal(bins[:, 0], ref[:, 0])
    assert np.allclose(bins[:, 1:], ref[:, 1:], rtol=1e-12, atol=1e-9)
    (a1, a2, b1, b2), _ = resfit.fit(ref, min_count=8)
    assert np.allclose(laws, [a1, a2, b1, b2], rtol=1e-9, atol=1e-12)
    if n > 100_000:
        assert laws[0] == pytest.approx(0.02, rel=0.05) and laws[3] == pytest.approx(1.3, rel=0.02)


def test_residual_fit_rejects_bad_arguments(vo, torch):
    X = torch.zeros((100, 2), device="cuda")
    for kw in [dict(nbins=1), dict(nbins=300), dict(v_max=0.0), dict(min_count=1)]:
        with pytest.raises(vo.VoldorError):
            vo.residual_fit(X, X, **{**dict(nbins=40, v_max=40.0, min_count=64), **kw})


@pytest.mark.parametrize("nb", [2, 64, 65, 256])
def test_residual_bins_every_register_slot(vo, torch, nb):
    # bin counts that fill one, two and four register slots per lane (b = 64 k
    # + lane), the maximum included; flows over the whole range and beyond
    # v_max, a ragged tail of a wave and of a workgroup
    n = 3 * 512 * 1024 + 77
    X, G = _sample(n, 1000 + nb)
    vmax = 37.5
    bins = vo.residual_bins(torch.from_numpy(X).cuda(), torch.from_numpy(G).cuda(), nb, vmax).cpu().numpy()
    ref = resfit.bin_stats(X, G, nb, vmax)
    assert np.array_equal(bins[:, 0], ref[:, 0])
    assert np.allclose(bins[:, 1:], ref[:, 1:], rtol=1e-12, atol=1e-9)


def test_binding_rejects_bad_shapes_before_any_launch(vo, torch):
    X = torch.zeros((100, 2), device="cuda")
    with pytest.raises(ValueError):
        vo.residual_bins(X, torch.zeros((99, 2), device="cuda"))
    with pytest.raises(TypeError):
        vo.residual_bins(X, torch.zeros((100, 2), device="cuda", dtype=torch.float64))
    with pytest.raises(TypeError):
        vo.residual_bins(X, torch.zeros((2, 100), device="cuda").t())
    with pytest.raises(TypeError):
        vo.residual_bins(X, X, work=torch.zeros(3, dtype=torch.float64, device="cuda"))
    n = vo.Net(3, 1, 16, 16)
    with pytest.raises(ValueError):
        n.forward(torch.zeros((1, 4, 16, 16, 2), device="cuda"))      # T of another net
    with pytest.raises(ValueError):
        n.forward(torch.zeros((1, 3, 16, 16, 2), device="cuda"), depth=torch.zeros((1, 16, 15), device="cuda"))
    with pytest.raises(ValueError):
        n.train_step(torch.zeros((1, 3, 16, 16, 2), device="cuda"), torch.zeros((1, 16, 16), device="cuda"),
                     torch.zeros((1, 2, 16, 16), device="cuda"), 1e-3)
    n.close()
    s = vo.Solver(3, 16, 16, 64)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):
        s.window_init(torch.zeros((3, 16, 16, 2), device="cuda"), (10.0, 10.0, 8.0, 8.0), vo.default_params(),
                      torch.ones((16, 17), device="cuda"), torch.ones((3, 16, 16), device="cuda"),
                      vo.Batch.outputs(3, 16, 16), st[0])
    s.close()
