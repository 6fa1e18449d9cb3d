"""Pins of the FP64 oracle of the residual-model regression (oracle/resfit.py):
recovery of the laws of Eq. 6-7 from residuals drawn from them with scipy, and
the binning against brute force."""
import numpy as np
import pytest

def test_resfit_recovers_the_laws_of_eq6_7():
    # residuals drawn exactly from Fisk(A(v), B(v)) with the paper's laws: the
    # regression gives back a1, a2, b1, b2 within the sampling error
    import scipy.stats
    from oracle import resfit
    rng = np.random.default_rng(0)
    a1, a2, b1, b2 = 0.02, 0.07, -0.004, 1.3
    n = 400_000
    v = rng.uniform(0.5, 40.0, n)
    ang = rng.uniform(0, 2 * np.pi, n)
    X = np.stack([v * np.cos(ang), v * np.sin(ang)], axis=1)
    x = scipy.stats.fisk.rvs(c=b1 * v + b2, scale=a1 * np.exp(a2 * v), random_state=rng)
    phi = rng.uniform(0, 2 * np.pi, n)
    G = X - np.sqrt(x)[:, None] * np.stack([np.cos(phi), np.sin(phi)], axis=1)
    st = resfit.bin_stats(X, G, 40, 40.0)
    (fa1, fa2, fb1, fb2), per_bin = resfit.fit(st)
    assert fa1 == pytest.approx(a1, rel=0.05) and fa2 == pytest.approx(a2, abs=2e-3)
    assert fb1 == pytest.approx(b1, abs=5e-4) and fb2 == pytest.approx(b2, rel=0.02)


def test_resfit_bins_brute_force():
    from oracle import resfit
    X = np.array([[1.0, 0.0], [0.0, 2.5], [3.0, 4.0], [np.nan, 0.0], [9.0, 9.0]])
    G = np.array([[0.5, 0.0], [0.0, 2.5], [3.0, 3.0], [0.0, 0.0], [0.0, 0.0]])
    st = resfit.bin_stats(X, G, 4, 8.0, x_floor=1e-12)
    # |v| = 1, 2.5, 5, (nan), 12.7 -> bins 0, 1, 2, skipped, beyond
    assert st[:, 0].tolist() == [1, 1, 1, 0]
    assert st[0, 1] == 1.0 and st[1, 1] == 2.5 and st[2, 1] == 5.0
    assert st[0, 2] == pytest.approx(np.log(0.25)) and st[1, 2] == pytest.approx(np.log(1e-12))
    assert st[2, 3] == pytest.approx(np.log(1.0) ** 2)
