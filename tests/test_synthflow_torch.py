"""The torch form of the planes-scene generator (synthflow.torchgen) against
the numpy one: with the per-pixel noise drawn from the window's numpy
generator the windows are the same, and with torch's generator the noise has
the same log-logistic law.  Runs on the CPU."""
import numpy as np
import pytest
import torch

import synthflow
from synthflow.torchgen import make_window_torch


@pytest.mark.parametrize("name,kw", [("small", {}), ("small", dict(T=6, H=240, W=320)),
                                     ("indoor", dict(T=3, H=120, W=160))])
def test_same_window_as_numpy(name, kw):
    a = synthflow.make_window(name, 7, **kw)
    b = make_window_torch(name, 7, "cpu", noise_rng="numpy", **kw)
    fa, fb = a["flows"], b["flows"].numpy()
    assert fa.shape == fb.shape and fb.dtype == np.float32
    d = np.abs(fa - fb)
    # the same FP64 arithmetic up to the device's rounding, cast to FP32
    assert d.max() <= 1e-4 and np.mean(d > 1e-6) <= 1e-4
    assert np.abs(a["depth"] - b["depth"].numpy()).max() <= 1e-9
    assert np.array_equal(a["outlier"], b["outlier"].numpy())
    assert a["K"] == b["K"]
    for (Ra, ta), (Rb, tb) in zip(a["poses"], b["poses"]):
        assert np.array_equal(Ra, Rb) and np.array_equal(ta, tb)


def test_torch_noise_law():
    # the noise magnitude over alpha = c1 |f| + c0 is log-logistic with median 1
    # and shape beta: P(e / alpha <= x) = 1 / (1 + x^-beta)
    kw = dict(T=2, H=120, W=160)
    clean = make_window_torch("small", 5, "cpu", noise=False, **kw)["flows"].double()
    noisy = make_window_torch("small", 5, "cpu", **kw)["flows"].double()
    spec = synthflow.resolve_spec("small", **kw)
    alpha = spec.noise_c1 * torch.linalg.vector_norm(clean, dim=-1) + spec.noise_c0
    x = (torch.linalg.vector_norm(noisy - clean, dim=-1) / alpha).reshape(-1).numpy()
    n = x.size
    for q in (0.5, 1.0, 2.0):
        cdf = 1.0 / (1.0 + q ** -spec.noise_beta)
        assert abs(np.mean(x <= q) - cdf) < 5 * np.sqrt(cdf * (1 - cdf) / n)
    # and differs from the numpy draws (a stream of its own)
    ref = synthflow.make_window("small", 5, **kw)["flows"]
    assert not np.allclose(noisy.numpy(), ref)


def test_rejects_driving_scene():
    with pytest.raises(ValueError):
        make_window_torch("driving", 0, "cpu", T=2, H=60, W=120)
