"""Pins of the FP64 oracle against things other than itself.

Each test checks an oracle function against a closed form, a library routine,
brute force, or an invariant that the paper's definitions fix, chosen so that a
dropped term, a sign error or a transposed operand fails at least one test.
"""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.stats
from scipy.integrate import quad
from scipy.spatial.transform import Rotation

import oracle
import synthflow

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ---------------------------------------------------------------- Philox
def test_philox_known_answers():
    n = 0
    with open(os.path.join(GOLDEN, "philox4x64_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            out = oracle.philox(v[0:4], v[4:6])
            assert [int(x) for x in out] == v[6:10]
            n += 1
    assert n >= 2


def test_philox_matches_numpy():
    # numpy's Philox is 4x64-10 and advances its counter before each block:
    # block i of Philox(counter=c) is philox(c + 1 + i).
    rng = np.random.default_rng(1)
    for _ in range(50):
        key = rng.integers(0, 2**63, 2, dtype=np.uint64)
        ctr = rng.integers(0, 2**63, 4, dtype=np.uint64)
        bg = np.random.Philox(key=key, counter=ctr)
        ref = bg.random_raw(4)
        c1 = ctr.copy()
        c1[0] += np.uint64(1)
        assert np.array_equal(oracle.philox(c1, key), ref)


def test_depth_sample_log_uniform():
    lo, hi = 0.5, 40.0
    v = np.array([oracle.depth_sample(7, 3, 0, x, y, lo, hi) for y in range(8) for x in range(2500)])
    assert v.min() >= lo and v.max() <= hi
    u = (np.log(v) - math.log(lo)) / (math.log(hi) - math.log(lo))
    assert scipy.stats.kstest(u, "uniform").pvalue > 1e-3
    # the eight pixels that share a block draw different words
    assert len(set(v[:8].tolist())) == 8


def test_depth_sample_words_of_numpy_philox():
    # pixel (x, y) of a sweep draws word a mod 8 (hi before lo of each 64-bit
    # output) of the block with key (seed, 1) and counter (gsweep, b, a // 8, 0),
    # a / b = coordinate along / across the sweep axis; numpy's Philox4x64-10
    # supplies the block
    lo, hi = 0.25, 64.0
    rng = np.random.default_rng(5)
    for _ in range(40):
        seed, gs = int(rng.integers(0, 2**40)), int(rng.integers(0, 2**20))
        d, x, y = int(rng.integers(4)), int(rng.integers(300)), int(rng.integers(300))
        a, b = (y, x) if d & 1 else (x, y)
        ctr = np.array([gs - 1 if gs > 0 else 2**64 - 1, b, a // 8, 0], dtype=np.uint64)
        block = np.random.Philox(key=np.array([seed, 1], dtype=np.uint64), counter=ctr).random_raw(4)
        w = int(block[(a % 8) // 2])
        word = (w >> 32) if a % 2 == 0 else (w & 0xFFFFFFFF)
        u = (word + 0.5) / 2.0**32
        want = math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))
        assert oracle.depth_sample(seed, gs, d, x, y, lo, hi) == pytest.approx(want, rel=1e-14)
    # the draw depends on the pixel and the sweep's axis, not on its sense
    assert oracle.depth_sample(3, 9, 0, 17, 5, lo, hi) == oracle.depth_sample(3, 9, 2, 17, 5, lo, hi)
    assert oracle.depth_sample(3, 9, 1, 17, 5, lo, hi) == oracle.depth_sample(3, 9, 3, 17, 5, lo, hi)
    assert oracle.depth_sample(3, 9, 0, 17, 5, lo, hi) != oracle.depth_sample(3, 9, 1, 17, 5, lo, hi)


# ---------------------------------------------------------------- Fisk (Eq. 5)
@pytest.mark.parametrize("alpha,beta", [(0.01, 1.0), (0.3, 0.9), (2.5, 0.5), (1e3, 0.05), (0.7, 3.0)])
def test_fisk_matches_scipy(alpha, beta):
    xs = np.logspace(-10, 8, 200)
    ref = scipy.stats.fisk(c=beta, scale=alpha).logpdf(xs)
    got = np.array([oracle.fisk_logpdf(x, math.log(alpha), beta) for x in xs])
    ok = np.isfinite(ref)
    assert np.allclose(got[ok], ref[ok], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("alpha,beta", [(0.5, 0.8), (3.0, 2.0)])
def test_fisk_normalised_and_median(alpha, beta):
    f = lambda x: math.exp(oracle.fisk_logpdf(x, math.log(alpha), beta))
    tot = quad(f, 0, alpha)[0] + quad(f, alpha, np.inf, limit=400)[0]
    assert abs(tot - 1) < 1e-7
    assert abs(quad(f, 0, alpha)[0] - 0.5) < 1e-8   # CDF(alpha) = 1/2


# ------------------------------------------------- Gaussian residual model
@pytest.mark.parametrize("alpha", [1e-4, 0.01, 0.7, 40.0])
def test_gauss_model_is_squared_gaussian_error(alpha):
    # squared EPE of an isotropic 2-D Gaussian error with per-axis variance
    # sigma^2 is sigma^2 chi^2_2; the model's median must be the Fisk's alpha
    sigma2 = alpha / (2.0 * math.log(2.0))
    ref = scipy.stats.chi2(df=2, scale=sigma2)
    xs = np.logspace(-12, 4, 120) * alpha
    got = np.array([oracle.gauss_logpdf(x, math.log(alpha)) for x in xs])
    want = ref.logpdf(xs)
    ok = np.isfinite(want)
    assert np.allclose(got[ok], want[ok], rtol=1e-12, atol=1e-12)
    assert ref.median() == pytest.approx(alpha, rel=1e-12)
    # and by sampling: squared norms of Gaussian pairs (K-S)
    e = np.random.default_rng(5).normal(0.0, math.sqrt(sigma2), (20000, 2))
    assert scipy.stats.kstest((e ** 2).sum(1), ref.cdf).pvalue > 1e-3


def test_emission_gauss_model_against_scipy():
    p = oracle.params(residual_model=1)
    u_obs = 20.0
    alpha = p.a1 * math.exp(p.a2 * u_obs)
    g = scipy.stats.chi2(df=2, scale=alpha / (2.0 * math.log(2.0)))
    prev = None
    # residuals around lambda |v| = 3 px (far below it r is 1 in double)
    for xi in [22.5, 22.9, 23.0, 23.1, 23.5]:
        K, M, fl, th = _translation_world(u_obs, xi)
        r, ell, lr, lm, obs = oracle.emission_map(th, fl, K, p, M)
        x = max((xi - u_obs) ** 2, p.x_floor)
        m = (p.lam * u_obs) ** 2
        assert np.allclose(lr, g.logpdf(x), rtol=1e-10)
        assert np.allclose(lm, g.logpdf(m), rtol=1e-10)
        rr = 1.0 / (1.0 + math.exp(g.logpdf(m) - g.logpdf(x)))
        assert np.allclose(r, rr, rtol=1e-9, atol=1e-300)
        if prev is not None:
            assert r[0, 0, 0] < prev
        prev = r[0, 0, 0]
    # r = 1/2 where the residual equals the outlier argument lambda |v|
    K, M, fl, th = _translation_world(u_obs, u_obs + p.lam * u_obs)
    r, ell, lr, lm, obs = oracle.emission_map(th, fl, K, p, M)
    assert np.allclose(r, 0.5, atol=1e-9)
    assert oracle.window(fl, K, oracle.params(residual_model=2))[0] != 0   # invalid model


# ---------------------------------------------------------------- lookup / emission
def test_bilinear_exact_on_affine_field():
    H, W = 20, 30
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    A = np.array([[0.3, -0.2], [0.15, 0.05]])
    b = np.array([1.5, -2.0])
    fl = np.zeros((2, H, W, 2), np.float32)
    fl[1, ..., 0] = A[0, 0] * xs + A[0, 1] * ys + b[0]
    fl[1, ..., 1] = A[1, 0] * xs + A[1, 1] * ys + b[1]
    fl = fl.astype(np.float32)
    rng = np.random.default_rng(0)
    for _ in range(200):
        px, py = rng.uniform(0, W - 1), rng.uniform(0, H - 1)
        got = oracle.lookup(fl, 2, px, py)
        exp = A @ np.array([px, py]) + b
        assert np.allclose(got, exp, atol=2e-5)   # fp32 storage of the taps
    assert oracle.lookup(fl, 2, W - 1, H - 1) is not None       # closed domain
    assert oracle.lookup(fl, 2, W - 1 + 1e-9, 3.0) is None
    assert oracle.lookup(fl, 2, -1e-9, 3.0) is None
    fl2 = fl.copy()
    fl2[1, 5, 7, 0] = np.nan
    assert oracle.lookup(fl2, 2, 7.5, 5.5) is None               # a missing tap


def _translation_world(u_obs, xi, H=16, W=24, f=100.0, theta=5.0):
    """T=1, camera translating along x so the rigid flow is xi everywhere."""
    K = (f, f, W / 2, H / 2)
    tx = xi * theta / f
    M = np.zeros((2, 12))
    M[0, [0, 4, 8]] = 1
    M[1, [0, 4, 8]] = 1
    M[1, 9] = tx
    fl = np.zeros((1, H, W, 2), np.float32)
    fl[0, ..., 0] = u_obs
    return K, M, fl, np.full((H, W), theta)


@pytest.mark.parametrize("u_obs", [3.0, 12.0, 60.0, 300.0])
def test_rigidness_half_at_lambda(u_obs):
    # Eq. 8: mu is the Fisk density at EPE = lambda |v|, so r = 1/2 there.
    p = oracle.params()
    xi = u_obs * (1 + p.lam)
    K, M, fl, th = _translation_world(u_obs, xi)
    r, ell, lr, lm, obs = oracle.emission_map(th, fl, K, p, M)
    assert obs.all()
    assert np.allclose(r, 0.5, atol=1e-9)
    assert np.allclose(lr, lm, atol=1e-9)


def test_emission_against_scipy_and_monotone():
    p = oracle.params()
    u_obs = 20.0
    prev = None
    for xi in [20.0, 20.5, 21.0, 22.0, 25.0, 30.0, 40.0]:
        K, M, fl, th = _translation_world(u_obs, xi)
        r, ell, lr, lm, obs = oracle.emission_map(th, fl, K, p, M)
        x = max((xi - u_obs) ** 2, p.x_floor)
        alpha = p.a1 * math.exp(p.a2 * u_obs)
        beta = max(p.b1 * u_obs + p.b2, p.beta_min)
        fk = scipy.stats.fisk(c=beta, scale=alpha)
        assert np.allclose(lr, fk.logpdf(x), rtol=1e-10)
        assert np.allclose(lm, fk.logpdf((p.lam * u_obs) ** 2), rtol=1e-10)
        rr = fk.pdf(x) / (fk.pdf(x) + fk.pdf((p.lam * u_obs) ** 2))
        assert np.allclose(r, rr, rtol=1e-9)
        assert np.allclose(ell, np.log(rr), rtol=1e-9, atol=1e-12)
        if prev is not None:
            assert r[0, 0, 0] < prev       # r decreases with the residual (beta <= 1)
        prev = r[0, 0, 0]


def test_emission_missing_cases():
    p = oracle.params()
    K, M, fl, th = _translation_world(10.0, 10.0)
    # behind the camera in frame t
    M2 = M.copy()
    M2[1, 11] = -10.0
    r, ell, lr, lm, obs = oracle.emission_map(th, fl, K, p, M2)
    assert not obs.any() and np.allclose(r, 0.5) and np.allclose(ell, math.log(0.5))
    fl2 = fl.copy()
    fl2[0, 3, 4] = np.inf
    r, ell, lr, lm, obs = oracle.emission_map(th, fl2, K, p, M)
    assert not obs[0, 3, 4] and not obs[0, 2, 3] and obs[0, 10, 10]


def _three_frame_world(f=100.0, W=24, H=16, shift=6.0, theta=5.0):
    """T=3, camera translating along x by `shift` px of disparity per frame at
    depth theta, identity rotation; constant observed flows (exact bilinear)."""
    K = (f, f, W / 2, H / 2)
    M = np.zeros((4, 12))
    M[:, [0, 4, 8]] = 1
    M[:, 9] = np.arange(4) * shift * theta / f
    u = np.array([5.0, 7.5, 4.0])
    fl = np.zeros((3, H, W, 2), np.float32)
    for t in range(3):
        fl[t, ..., 0] = u[t]
        fl[t, ..., 1] = 0.5 * t
    return K, M, fl, u


@pytest.mark.parametrize("crit", [0, 1])
def test_depth_objective_against_scipy(crit):
    # Eq. 9 (MLE): sum_t q log rho + (1 - q) log mu over observed frames; Eq. 10
    # (MIE): sum_t q log(rho / (rho + mu)), log 1/2 where missing.  The rigid flow
    # is restated from the pinhole projection, the densities come from scipy.
    p = oracle.params(criterion=crit)
    K, M, fl, u = _three_frame_world()
    f, cx = K[0], K[2]
    rng = np.random.default_rng(5)
    q = rng.uniform(0.05, 0.95, (3, 16, 24))
    for x, y, th in [(5, 4, 5.0), (10, 7, 5.0), (14, 3, 5.0), (9, 8, 3.7), (2, 12, 9.0)]:
        got = oracle.depth_score(q, fl, K, p, M, x, y, th)
        want = 0.0
        for t in range(1, 4):
            prev_u = x + f * M[t - 1, 9] / th          # pi_{t-1}: lookup location of X_t
            xi = f * (M[t, 9] - M[t - 1, 9]) / th      # rigid flow pi_t - pi_{t-1} along x
            qt = q[t - 1, y, x]
            if not (0 <= prev_u <= 23):
                want += 0.0 if crit == 1 else qt * math.log(0.5)
                continue
            v = np.array([u[t - 1], 0.5 * (t - 1)])
            x2 = max((xi - v[0]) ** 2 + v[1] ** 2, p.x_floor)
            vn = np.linalg.norm(v)
            fk = scipy.stats.fisk(c=max(p.b1 * vn + p.b2, p.beta_min), scale=p.a1 * math.exp(p.a2 * vn))
            lr, lm = fk.logpdf(x2), fk.logpdf((p.lam * vn) ** 2)
            if crit == 1:
                want += qt * lr + (1 - qt) * lm
            else:
                want += qt * (lr - np.logaddexp(lr, lm))
        assert got == pytest.approx(want, rel=1e-10, abs=1e-12), (x, y, th)


def test_mle_objective_peaks_at_ground_truth():
    # noise-free flow, q = 1: log rho is largest at zero residual (B(v) <= 1
    # makes the Fisk density decreasing), so the true depth beats scaled depths
    # at every pixel.  Frame 1 only: X_1 is looked up at the pixel itself, with
    # no interpolation across depth edges (frames t >= 2 sample X_t at
    # pi_{t-1}, where bilinear interpolation leaves a residual at the truth)
    w = synthflow.make_window("small", 2, noise=False, outliers=False, T=1, H=40, W=56)
    R, t = w["poses"][0]
    M = oracle.cumulative(np.concatenate([R.ravel(), t])[None])
    p = oracle.params(criterion=1)
    q = np.ones((1, 40, 56))
    rng = np.random.default_rng(1)
    for _ in range(25):
        x, y = int(rng.integers(4, 52)), int(rng.integers(4, 36))
        g = float(w["depth"][y, x])
        s0 = oracle.depth_score(q, w["flows"], w["K"], p, M, x, y, g)
        for k in (0.8, 0.95, 0.99, 1.01, 1.05, 1.25):
            assert oracle.depth_score(q, w["flows"], w["K"], p, M, x, y, g * k) < s0


def test_identity_projection_and_gt_flow():
    # pi_0 is the pixel itself, and the generator's ground-truth flow equals the
    # rigid flow pi_1 - pi_0 at ground-truth depth and pose.
    w = synthflow.make_window("small", 3, noise=False, outliers=False, T=1)
    p = oracle.params()
    R, t = w["poses"][0]
    M = oracle.cumulative(np.concatenate([R.ravel(), t])[None])
    r, ell, lr, lm, obs = oracle.emission_map(w["depth"], w["flows"], w["K"], p, M)
    # zero residual up to float32 rounding of the stored flow: r must equal the
    # zero-residual value rho(x_floor) / (rho(x_floor) + mu) of Eq. 4-8
    assert obs.all()
    v = np.linalg.norm(w["flows"][0].astype(np.float64), axis=-1)
    alpha = p.a1 * np.exp(p.a2 * v)
    beta = np.maximum(p.b1 * v + p.b2, p.beta_min)
    f0 = scipy.stats.fisk(c=beta, scale=alpha).pdf(np.full_like(v, 1e-12))
    fm = scipy.stats.fisk(c=beta, scale=alpha).pdf((p.lam * v) ** 2)
    r0 = f0 / (f0 + fm)
    assert np.median(np.abs(r[0] - r0) / (1 - r0)) < 0.2
    assert np.all(r[0] <= r0 + 1e-12)          # any residual can only lower r


# ---------------------------------------------------------------- forward-backward (Eq. 11-14)
def _fb_brute(r, gamma):
    L = len(r)
    num = np.zeros(L)
    Z = 0.0
    for path in itertools.product((0, 1), repeat=L):
        pr = 0.5
        for k, s in enumerate(path):
            if k > 0:
                pr *= gamma if s == path[k - 1] else 1 - gamma
            pr *= r[k] if s == 1 else 1 - r[k]
        Z += pr
        num += pr * np.array(path)
    return num / Z


@pytest.mark.parametrize("L", [1, 2, 5, 11])
def test_fb_brute_force(L):
    rng = np.random.default_rng(L)
    for _ in range(5):
        r = rng.uniform(0.01, 0.99, L)
        gamma = rng.uniform(0.5, 0.99)
        assert np.allclose(oracle.fb_chain(r, gamma), _fb_brute(r, gamma), atol=1e-12)


def test_fb_special_cases():
    rng = np.random.default_rng(0)
    r = rng.uniform(0.01, 0.99, 40)
    assert np.allclose(oracle.fb_chain(r, 0.5), r, atol=1e-14)      # no coupling
    q = oracle.fb_chain(r, 1 - 1e-12)                              # full coupling
    assert np.ptp(q) < 1e-6
    # full coupling: the posterior of the all-1 path over the all-0 path
    a, b = np.prod(r), np.prod(1 - r)
    assert abs(q[0] - a / (a + b)) < 1e-6


def test_fb_map_chains():
    rng = np.random.default_rng(2)
    r = rng.uniform(0.05, 0.95, (2, 6, 7))
    qh = oracle.fb_map(r, 0, 0.8)
    qv = oracle.fb_map(r, 1, 0.8)
    assert np.allclose(qh[1, 3], oracle.fb_chain(r[1, 3], 0.8))
    assert np.allclose(qv[0, :, 4], oracle.fb_chain(r[0, :, 4], 0.8))
    assert np.allclose(oracle.fb_map(r, 2, 0.8), qh)    # posterior does not depend on direction
    assert np.allclose(oracle.fb_map(r, 3, 0.8), qv)


# ---------------------------------------------------------------- linear algebra, SE(3)
def test_sym_eig_and_svd():
    rng = np.random.default_rng(0)
    for n in (3, 9):
        A = rng.normal(size=(n, n))
        A = A + A.T
        w, V = oracle.sym_eig(A)
        assert np.allclose(w, np.linalg.eigvalsh(A), atol=1e-10)
        assert np.allclose(A @ V, V * w, atol=1e-9)
    A = rng.normal(size=(3, 3))
    U, S, V = oracle.svd3(A)
    assert np.allclose(S, np.linalg.svd(A, compute_uv=False), atol=1e-10)
    assert np.allclose(U[:, :2] * S[:2] @ V[:, :2].T + S[2] * np.outer(U[:, 2], V[:, 2]) * np.sign(np.linalg.det(A)), A, atol=1e-9)
    assert abs(np.linalg.det(U) - 1) < 1e-10 and abs(np.linalg.det(V) - 1) < 1e-10
    E = U @ np.diag([1.3, 0.7, 0]) @ V.T                   # rank 2 round trip
    U2, S2, V2 = oracle.svd3(E)
    assert np.allclose(U2[:, :2] * S2[:2] @ V2[:, :2].T, E, atol=1e-10)


def test_null_vector_matches_svd():
    rng = np.random.default_rng(9)
    for _ in range(20):
        A = rng.normal(size=(8, 9))
        e = oracle.null_vector_8x9(A)
        ref = np.linalg.svd(A)[2][-1]
        assert abs(abs(e @ ref) - 1) < 1e-12
        assert np.abs(A @ e).max() < 1e-12


def _twist(p):
    X = np.zeros((4, 4))
    X[:3, :3] = np.array([[0, -p[5], p[4]], [p[5], 0, -p[3]], [-p[4], p[3], 0]])
    X[:3, 3] = p[:3]
    return X


@pytest.mark.parametrize("scale", [1e-9, 1e-4, 0.3, 2.0, math.pi - 1e-7])
def test_se3_exp_log(scale):
    rng = np.random.default_rng(int(scale * 1e3) % 1000)
    for _ in range(20):
        ax = rng.normal(size=3)
        ax /= np.linalg.norm(ax)
        p = np.concatenate([rng.normal(size=3), ax * scale])
        R, t = oracle.se3_exp(p)
        G = scipy.linalg.expm(_twist(p))
        assert np.allclose(R, G[:3, :3], atol=1e-12)
        assert np.allclose(t, G[:3, 3], atol=1e-11)
        q = oracle.se3_log(R, t)
        assert np.allclose(q[3:], Rotation.from_matrix(R).as_rotvec(), atol=1e-7)
        if scale < math.pi - 1e-3:
            assert np.allclose(q, p, atol=1e-9)


# ---------------------------------------------------------------- P3P (Eq. 17)
def test_p3p_recovers_known_poses():
    rng = np.random.default_rng(5)
    hits = 0
    for trial in range(300):
        R = Rotation.from_rotvec(rng.normal(size=3) * 0.5).as_matrix()
        t = rng.normal(size=3)
        Q = np.column_stack([rng.uniform(-2, 2, 3), rng.uniform(-2, 2, 3), rng.uniform(3, 10, 3)])
        Pw = (Q - t) @ R                                  # world points: Q = R P + t
        f = Q / np.linalg.norm(Q, axis=1, keepdims=True)
        sols = oracle.p3p(Pw, f)
        assert len(sols) <= 4
        best = min((np.abs(Rs - R).max() + np.abs(ts - t).max() for Rs, ts in sols), default=np.inf)
        hits += best < 1e-9
        for Rs, ts in sols:                              # every root satisfies the bearings
            Qs = Pw @ Rs.T + ts
            Qs /= np.linalg.norm(Qs, axis=1, keepdims=True)
            assert np.allclose(np.abs(np.sum(Qs * f, axis=1)), 1, atol=1e-7)
            assert abs(np.linalg.det(Rs) - 1) < 1e-9
    # every draw, near-degenerate ones included: the roots are refined on the
    # law-of-cosines equations themselves
    assert hits == 300


# ---------------------------------------------------------------- mean-shift (Eq. 18-19)
def test_meanshift_identical_samples_exact():
    p = np.array([0.1, -0.2, 0.3, 0.01, 0.02, -0.03])
    S = np.tile(p, (10, 1))
    out, it = oracle.meanshift(S, np.ones(10), p + 0.05, 0.1, 0.004)
    assert np.allclose(out, p, atol=1e-15)


def test_meanshift_heavier_cluster_and_stationarity():
    rng = np.random.default_rng(3)
    a = np.array([0.0, 0, 1, 0, 0, 0])
    b = np.array([2.0, 0, 0, 0.5, 0, 0])
    S = np.vstack([a + 0.01 * rng.normal(size=(60, 6)), b + 0.01 * rng.normal(size=(40, 6))])
    w = rng.uniform(0.5, 1, 100)
    out, _ = oracle.meanshift(S, w, S[70], 0.1, 0.004)    # start in the lighter cluster
    assert np.linalg.norm(out - b) < 0.05                # local mode of the cluster it starts in
    out2, _ = oracle.meanshift(S, w, S[0], 0.1, 0.004)
    assert np.linalg.norm(out2 - a) < 0.05
    # stationarity: gradient of the weighted Gaussian KDE is zero at the mode
    Si = np.array([0.1] * 3 + [0.004] * 3)
    d = S - out2
    k = w * np.exp(-0.5 * np.sum(d * d / Si, axis=1))
    assert np.abs((k[:, None] * d / Si).sum(0)).max() < 1e-8 * k.sum()
    # seed scoring: the heavier cluster has the larger density
    assert oracle.kde(S, w, a, 0.1, 0.004) > oracle.kde(S, w, b, 0.1, 0.004)


def test_meanshift_zero_weights_ignored():
    rng = np.random.default_rng(4)
    S = rng.normal(size=(30, 6)) * 0.01
    w = np.ones(30)
    far = np.vstack([S, np.full((5, 6), 0.02)])
    wf = np.concatenate([w, np.zeros(5)])
    o1, _ = oracle.meanshift(S, w, S[0], 0.1, 0.004)
    o2, _ = oracle.meanshift(far, wf, S[0], 0.1, 0.004)
    assert np.allclose(o1, o2, atol=1e-15)


# ---------------------------------------------------------------- bootstrap (Sec. 5.3)
def test_allpixel_scores_are_rigidness_weighted_ell_sums():
    # each candidate's score is sum_j W_t^j ell_t^j over every pixel at
    # M_t = T_c o M_{t-1}: restated from the emission map (pinned to scipy above)
    w = synthflow.make_window("small", 6, T=3, H=24, W=32)
    R, t = w["poses"][0]
    rel = np.array([np.concatenate([R_.ravel(), t_ / np.linalg.norm(t)]) for R_, t_ in w["poses"]])
    M = oracle.cumulative(rel)
    th = w["depth"] / np.linalg.norm(t)
    rig = np.random.default_rng(2).uniform(0.1, 1.0, (3, 24, 32))
    p = oracle.params(n_pose_groups=24, pose_start=1)
    t_ = 2
    sc, _ = oracle.pose_scores(th, rig, w["flows"], w["K"], p, M, t_, 1, prevT=rel[t_ - 1])
    _, smp, diag = oracle.pose_step(th, rig, w["flows"], w["K"], p, M, t_, 1, prevT=rel[t_ - 1], want_samples=True)
    valid = smp[smp[:, 7] > 0]
    assert len(sc) == 1 + len(valid) == 1 + diag[0]
    cands = [rel[t_ - 1]] + [np.concatenate([a.ravel(), b]) for a, b in (oracle.se3_exp(v[:6]) for v in valid)]
    for i in range(0, len(cands), max(1, len(cands) // 8)):
        Rc, tc = cands[i][:9].reshape(3, 3), cands[i][9:]
        Rm, tm = M[t_ - 1][:9].reshape(3, 3), M[t_ - 1][9:]
        Mi = M.copy()
        Mi[t_] = np.concatenate([(Rc @ Rm).ravel(), Rc @ tm + tc])
        r, ell, lr, lm, obs = oracle.emission_map(th, w["flows"], w["K"], p, Mi)
        assert sc[i] == pytest.approx(float(np.sum(rig[t_ - 1] * ell[t_ - 1])), rel=1e-12), i


def test_allpixel_score_peaks_at_true_pose():
    # noise-free X_1, W = 1: the true pose scores above every perturbed one
    w = synthflow.make_window("small", 3, noise=False, outliers=False, T=1, H=40, W=56)
    R, t = w["poses"][0]
    gt = np.concatenate([R.ravel(), t])
    M = oracle.cumulative(gt[None])
    p = oracle.params(n_pose_groups=8, pose_start=1)
    s0 = oracle.pose_scores(w["depth"], None, w["flows"], w["K"], p, M, 1, 0, prevT=gt)[0][0]
    rng = np.random.default_rng(4)
    for _ in range(8):
        dR = Rotation.from_rotvec(rng.normal(0, 2e-3, 3)).as_matrix()
        cand = np.concatenate([(dR @ R).ravel(), t + rng.normal(0, 2e-3, 3)])
        s1 = oracle.pose_scores(w["depth"], None, w["flows"], w["K"], p, M, 1, 0, prevT=cand)[0][0]
        assert s1 < s0


def test_window_noise_free_recovery_allpixel_start():
    w = synthflow.make_window("small", 0, noise=False, outliers=False, T=3, H=48, W=64)
    st, poses, depth, rig, ll, diag = oracle.window(w["flows"], w["K"],
                                                    oracle.params(n_iters=2, n_pose_groups=32, pose_start=1))
    assert st == 0
    rot, tdir, s = _pose_errors(poses, w["poses"])
    assert rot.max() < 1e-3 and tdir.max() < 2e-2
    assert np.median(np.abs(depth * s - w["depth"]) / w["depth"]) < 1e-2


def test_bootstrap_noise_free_recovers_pose_and_depth():
    w = synthflow.make_window("small", 1, noise=False, outliers=False, T=1)
    p = oracle.params()
    st, rel, th, rng, info = oracle.bootstrap(w["flows"], w["K"], p)
    assert st == 0
    R, t = w["poses"][0]
    s = np.linalg.norm(t)
    # float32 flows limit the exactness to ~1e-7 relative
    assert np.abs(rel[:9].reshape(3, 3) - R).max() < 1e-5
    assert np.abs(rel[9:] - t / s).max() < 1e-4
    rel_err = np.abs(th * s - w["depth"]) / w["depth"]
    assert np.median(rel_err) < 1e-5
    assert info[1] < 1e-9                     # median Sampson residual (px^2)


def test_bootstrap_with_outliers_and_noise():
    w = synthflow.make_window("small", 2, noise=True, outliers=True, T=1)
    p = oracle.params()
    st, rel, th, rng, info = oracle.bootstrap(w["flows"], w["K"], p)
    assert st == 0
    R, t = w["poses"][0]
    ang = Rotation.from_matrix(rel[:9].reshape(3, 3) @ R.T).magnitude()
    cosang = rel[9:] @ t / np.linalg.norm(t)
    assert ang < 0.03 and cosang > 0.9        # 8-point on noisy flow: coarse start
    assert rng[0] > 0 and rng[1] > rng[0]


def test_bootstrap_degenerate():
    fl = np.full((1, 20, 20, 2), np.nan, np.float32)
    st, *_ = oracle.bootstrap(fl, (50, 50, 10, 10), oracle.params())
    assert st == -4


# ---------------------------------------------------------------- sweep (Eq. 10, Fig. 5)
def _sweep_world(seed=4, T=3, H=40, W=56, noise=True):
    w = synthflow.make_window("small", seed, noise=noise, outliers=noise, T=T, H=H, W=W)
    R, t = w["poses"][0]
    s = np.linalg.norm(t)
    rel = np.array([np.concatenate([R_.ravel(), t_ / s]) for R_, t_ in w["poses"]])
    return w, oracle.cumulative(rel), w["depth"] / s


def test_sweep_monotone_and_candidates():
    w, M, gt = _sweep_world()
    p = oracle.params()
    rng = np.random.default_rng(0)
    theta = gt * np.exp(rng.normal(0, 0.2, gt.shape))
    d_lo, d_hi = 0.5 * gt.min(), 2 * gt.max()
    for d in range(4):
        new, q, ch = oracle.sweep(theta, w["flows"], w["K"], p, M, d_lo, d_hi, 5 + d, d)
        _, ell_old, *_ = oracle.emission_map(theta, w["flows"], w["K"], p, M)
        _, ell_new, *_ = oracle.emission_map(new, w["flows"], w["K"], p, M)
        s_old = (q * ell_old).sum(0)
        s_new = (q * ell_new).sum(0)
        assert np.all(s_new >= s_old - 1e-12 * np.abs(s_old))   # MIE never decreases per pixel
        assert np.all(new[ch == 0] == theta[ch == 0])
        assert (ch == 1).any() and (ch == 2).any()
        st, _ = oracle.sweep_check(theta, new, w["flows"], w["K"], p, M, d_lo, d_hi, 5 + d, d,
                                   vtol=0, stol=0)
        assert (st == 0).all()
        # first position of every chain has no neighbour candidate
        first = {0: new[:, 0], 1: new[0, :], 2: new[:, -1], 3: new[-1, :]}[d]
        chf = {0: ch[:, 0], 1: ch[0, :], 2: ch[:, -1], 3: ch[-1, :]}[d]
        assert (chf != 1).all()
        theta = new


def test_sweep_ground_truth_is_fixed_point():
    # single flow, no noise: the ground-truth depth has (near) zero residual
    w, M, gt = _sweep_world(seed=6, T=1, noise=False)
    p = oracle.params()
    new, q, ch = oracle.sweep(gt, w["flows"], w["K"], p, M, 0.5 * gt.min(), 2 * gt.max(), 0, 0)
    assert np.mean(new == gt) > 0.999


def test_sweep_check_detects_wrong_choice():
    w, M, gt = _sweep_world(seed=7)
    p = oracle.params()
    theta = gt * 1.1
    d_lo, d_hi = 0.5 * gt.min(), 2 * gt.max()
    new, q, ch = oracle.sweep(theta, w["flows"], w["K"], p, M, d_lo, d_hi, 2, 1)
    bad = new.copy()
    i = np.argwhere(ch == 2)[0]
    bad[tuple(i)] = theta[tuple(i)]            # keep previous where the sample won
    st, _ = oracle.sweep_check(theta, bad, w["flows"], w["K"], p, M, d_lo, d_hi, 2, 1, 1e-9, 0)
    assert st[tuple(i)] == 3
    bad[tuple(i)] = 123.0                      # value outside the candidate set
    st, _ = oracle.sweep_check(theta, bad, w["flows"], w["K"], p, M, d_lo, d_hi, 2, 1, 1e-9, 0)
    assert st[tuple(i)] == 2


# ---------------------------------------------------------------- whole window (Table 1)
def _pose_errors(poses, gt):
    s = np.linalg.norm(gt[0][1])
    rot, tdir = [], []
    for k, (R, t) in enumerate(gt):
        Re = poses[k, :9].reshape(3, 3)
        te = poses[k, 9:]
        rot.append(Rotation.from_matrix(Re @ R.T).magnitude())
        tdir.append(math.acos(np.clip(te @ t / np.linalg.norm(te) / np.linalg.norm(t), -1, 1)))
    return np.array(rot), np.array(tdir), s


def test_window_noise_free_recovery():
    w = synthflow.make_window("small", 0, noise=False, outliers=False)
    st, poses, depth, rig, ll, diag = oracle.window(w["flows"], w["K"], oracle.params(n_iters=2))
    assert st == 0
    rot, tdir, s = _pose_errors(poses, w["poses"])
    assert abs(np.linalg.norm(poses[0, 9:]) - 1) < 1e-12          # gauge
    # limits: float32 flows and bilinear interpolation of the flow fields
    assert rot.max() < 1e-3 and tdir.max() < 2e-2
    rel = np.abs(depth * s - w["depth"]) / w["depth"]
    assert np.median(rel) < 1e-2
    assert np.median(rig) > 0.99


def test_window_noise_free_recovery_mle():
    # the maximum-likelihood depth criterion (Eq. 9) recovers the same truth
    w = synthflow.make_window("small", 0, noise=False, outliers=False)
    st, poses, depth, rig, ll, diag = oracle.window(w["flows"], w["K"], oracle.params(n_iters=2, criterion=1))
    assert st == 0
    rot, tdir, s = _pose_errors(poses, w["poses"])
    assert rot.max() < 1e-3 and tdir.max() < 2e-2
    rel = np.abs(depth * s - w["depth"]) / w["depth"]
    assert np.median(rel) < 1e-2
    assert np.median(rig) > 0.99


def test_window_noise_free_recovery_gauss_model():
    # the Gaussian residual model recovers the truth on noise-free flow, less
    # closely than the Fisk model (rot 5.7e-4, tdir 1.2e-2, median depth 1.4 %
    # after 2 iterations, against 2.0e-4, 5.3e-3 and 0.46 %): its light tail
    # weighs the float32 and bilinear errors of the flows more
    w = synthflow.make_window("small", 0, noise=False, outliers=False)
    st, poses, depth, rig, ll, diag = oracle.window(w["flows"], w["K"], oracle.params(n_iters=2, residual_model=1))
    assert st == 0
    rot, tdir, s = _pose_errors(poses, w["poses"])
    assert rot.max() < 2e-3 and tdir.max() < 3e-2
    rel = np.abs(depth * s - w["depth"]) / w["depth"]
    assert np.median(rel) < 3e-2
    assert np.median(rig) > 0.99


def test_bootstrap_seeded_matches_bootstrap_and_truth():
    # given the LMedS T_1, the seeded bootstrap is the bootstrap; given the true
    # T_1 (any scale) on noise-free flow, the depth is the truth in the unit gauge
    w = synthflow.make_window("small", 4, noise=False, outliers=False, T=2, H=48, W=64)
    p = oracle.params()
    st, rel, th, rng, info = oracle.bootstrap(w["flows"], w["K"], p)
    st2, rel2, th2, rng2 = oracle.bootstrap_seeded(w["flows"], w["K"], p, rel * np.r_[np.ones(9), 3.0 * np.ones(3)])
    assert st == st2 == 0
    assert np.allclose(rel2, rel, atol=1e-15) and np.allclose(th2, th, rtol=1e-13) and np.allclose(rng2, rng)
    R, t = w["poses"][0]
    st3, rel3, th3, _ = oracle.bootstrap_seeded(w["flows"], w["K"], p, np.concatenate([R.ravel(), 7.0 * t]))
    assert st3 == 0 and np.allclose(rel3[9:], t / np.linalg.norm(t), atol=1e-15)
    ok = (th3 > rng2[0] * 1.0001) & (th3 < rng2[1] * 0.9999)
    rel_err = np.abs(th3 * np.linalg.norm(t) - w["depth"]) / w["depth"]
    assert np.median(rel_err[ok]) < 1e-4
    assert oracle.bootstrap_seeded(w["flows"], w["K"], p, np.r_[R.ravel(), 0, 0, 0])[0] == -4


def test_window_starts():
    assert oracle.window_starts(12, 5, 1) == [0, 1, 2, 3, 4, 5, 6, 7]
    assert oracle.window_starts(12, 5, 3) == [0, 3, 6, 7]
    assert oracle.window_starts(5, 5, 2) == [0]
    assert oracle.window_starts(9, 4, 5) == [0, 5]


@pytest.mark.parametrize("stride", [1, 2])
def test_vo_sequence_noise_free_trajectory(stride):
    # noise-free flows over a 9-frame sequence whose per-frame speed varies by
    # 3x, so that every window has its own scale: each step of the chained
    # trajectory is the true relative pose in the first window's scale.  The
    # bounds are a few times the single-window noise-free limits (float32
    # flows, bilinear lookup, 96x128 pixels), since each window inherits the
    # previous one's T_1; dropping or inverting the chaining factor moves the
    # steps' lengths by tens of percent
    N, T = 9, 4
    w = synthflow.make_window("small", 5, noise=False, outliers=False, T=N, H=96, W=128, speed_range=(0.5, 1.5))
    p = oracle.params(n_iters=2, n_pose_groups=128)
    st, M, wp = oracle.vo_sequence(w["flows"], w["K"], p, T, stride)
    assert st == 0 and M.shape == (N + 1, 12)
    scale = np.linalg.norm(w["poses"][0][1])
    for k in range(N):
        Ra = M[k + 1][:9].reshape(3, 3) @ M[k][:9].reshape(3, 3).T
        ta = M[k + 1][9:] - Ra @ M[k][9:]
        Rg, tg = w["poses"][k][0], w["poses"][k][1] / scale
        ang = math.acos(max(-1.0, min(1.0, (np.trace(Ra @ Rg.T) - 1) / 2)))
        assert ang < 6e-3, (k, ang)
        assert np.linalg.norm(ta - tg) < 0.1 * np.linalg.norm(tg), (k, ta, tg)


def test_window_outliers_flagged():
    w = synthflow.make_window("small", 0, noise=True, outliers=True)
    st, poses, depth, rig, ll, diag = oracle.window(w["flows"], w["K"], oracle.params(n_iters=3))
    assert st == 0
    rot, tdir, s = _pose_errors(poses, w["poses"])
    assert rot.max() < 5e-3 and tdir.max() < 0.2
    out = w["outlier"]
    assert np.mean(rig[out] < 0.5) > 0.8           # moving regions get low rigidness
    assert np.mean(rig[~out] > 0.5) > 0.8
    assert ll[1] >= abs(ll[0])


def test_window_invalid_arguments():
    w = synthflow.make_window("small", 0, T=1, H=20, W=20)
    p = oracle.params()
    p.struct_size = 3
    assert oracle.window(w["flows"], w["K"], p)[0] == -1
    assert oracle.window(w["flows"], (0, 1, 1, 1), oracle.params())[0] == -1
    assert oracle.window(w["flows"], w["K"], oracle.params(criterion=2))[0] == -1
    assert oracle.window(w["flows"], w["K"], oracle.params(pose_start=2))[0] == -1
    assert oracle.window(w["flows"], w["K"], oracle.params(gamma=1.0))[0] == -1
    small = np.zeros((1, 8, 8, 2), np.float32)
    assert oracle.window(small, w["K"], oracle.params())[0] == -1


def test_window_init_selection():
    # the proposal competes with the bootstrap's state after one pass of pose
    # steps each, by window log-likelihood
    w = synthflow.make_window("small", 4, T=3, H=48, W=64)
    p = oracle.params(n_iters=2, n_pose_groups=128)
    T, H, W = 3, 48, 64
    st, op, od, orig, oll, _ = oracle.window(w["flows"], w["K"], p)
    assert st == 0
    sb, rel, th, rng, info = oracle.bootstrap(w["flows"], w["K"], p)
    # the bootstrap's own state proposed: equal likelihoods, the bootstrap is kept
    # and the result is the plain window's
    r = oracle.window_init(w["flows"], w["K"], p, th, np.ones((T, H, W)))
    assert r[0] == 0 and r[6] == 0
    assert np.array_equal(r[1], op) and np.array_equal(r[2], od) and np.array_equal(r[3], orig)
    # an implausible proposal loses
    r = oracle.window_init(w["flows"], w["K"], p, np.full((H, W), 1e3), np.ones((T, H, W)))
    assert r[6] == 0 and np.array_equal(r[1], op)
    # the converged state of a longer solve wins, and the window it ends in is
    # at least as likely as the plain one
    st4, op4, od4, orig4, oll4, _ = oracle.window(w["flows"], w["K"], oracle.params(n_iters=4, n_pose_groups=128))
    r = oracle.window_init(w["flows"], w["K"], p, od4, orig4)
    assert r[0] == 0 and r[6] == 1
    assert r[4][0] >= oll[0]
