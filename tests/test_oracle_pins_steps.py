"""More pins of the FP64 oracle: the pose step's inputs (Sec. 5.2, Eq. 17 and
Eq. 19), the window log-likelihood (Eq. 3), the bootstrap's depth range
(Sec. 5.3) and the beta_min clamp of the shape law (Eq. 7).

Every expected value here is recomputed from the paper's definitions with
numpy / scipy code written in this file (its own Philox counters, projection,
bilinear lookup and Fisk density), never from another oracle routine.
"""
import math

import numpy as np
import pytest
import scipy.spatial.transform
import scipy.stats

import oracle
import synthflow

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

POSE_KEY = 2   # key word 1 of the pose-group draws


def _philox_block(key, ctr):
    """Philox4x64-10 block of counter `ctr` (4 words) from numpy, whose
    generator advances its 256-bit counter by one before each block."""
    c = [int(v) for v in ctr]
    v = sum(w << (64 * i) for i, w in enumerate(c)) - 1
    v %= 1 << 256
    prev = np.array([(v >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    return np.random.Philox(key=np.array(key, dtype=np.uint64), counter=prev).random_raw(4)


def _group_pixels(seed, it, t, g, HW):
    """The three pixels of pose group g (Sec. 5.2: random pixel triples): up to
    eight attempts of three indices from the high words of one Philox block."""
    for a in range(8):
        o = _philox_block([seed, POSE_KEY], [it, t, g, a])
        j = [(int(o[k]) >> 32) * HW >> 32 for k in range(3)]
        if len(set(j)) == 3:
            return j
    return None


def _bilinear(field, px, py):
    """Bilinear lookup with pixel centres at integers (own implementation)."""
    H, W = field.shape[:2]
    if not (0 <= px <= W - 1 and 0 <= py <= H - 1):
        return None
    x0, y0 = min(int(math.floor(px)), W - 2), min(int(math.floor(py)), H - 2)
    ax, ay = px - x0, py - y0
    f = field.astype(np.float64)
    top = (1 - ax) * f[y0, x0] + ax * f[y0, x0 + 1]
    bot = (1 - ax) * f[y0 + 1, x0] + ax * f[y0 + 1, x0 + 1]
    v = (1 - ay) * top + ay * bot
    return v if np.all(np.isfinite(v)) else None


def _row_world(T=2, H=48, W=64, f=100.0, Z0=5.0):
    """Translating camera, identity rotation, depth constant along each image
    row (Z0, 2 Z0 or 4 Z0 by row), translations chosen so that every flow is a
    whole number of pixels: each lookup point pi_{t-1} of a frame-0 pixel is a
    pixel, where the bilinear lookup is exact.  Frame 1 moves along x only, so
    rows keep their depth in every frame and the flow X_t at a frame-(t-1)
    pixel is the motion of the row's depth."""
    K = (f, f, W / 2.0, H / 2.0)
    ys = np.arange(H)
    Z = Z0 * np.array([1.0, 2.0, 4.0])[ys % 3]
    depth = np.repeat(Z[:, None], W, axis=1)
    # relative translations in pixels of disparity at depth Z0
    steps = [(4.0, 0.0), (8.0, -4.0)][:T]
    rel = []
    flows = np.zeros((T, H, W, 2), np.float32)
    for t, (sx, sy) in enumerate(steps):
        tv = np.array([sx * Z0 / f, sy * Z0 / f, 0.0])
        rel.append(np.concatenate([np.eye(3).ravel(), tv]))
        flows[t, ..., 0] = (f * tv[0] / Z)[:, None]
        flows[t, ..., 1] = (f * tv[1] / Z)[:, None]
    return K, np.array(rel), flows, depth


@pytest.mark.parametrize("t", [1, 2])
def test_pose_step_weights_are_products_of_rigidness(t):
    # Eq. 19: a sample's weight is the product of W_t over the group's three
    # pixels (W of frame t, Sec. 5.2), each group drawn from its own Philox block
    K, rel, flows, depth = _row_world(T=2)
    T, H, W, _ = flows.shape
    HW = H * W
    rng = np.random.default_rng(3)
    Wmap = rng.uniform(0.05, 1.0, size=(T, H, W))
    p = oracle.params(n_pose_groups=200, seed=11)
    M = oracle.cumulative(rel)
    it = 1
    Tout, samples, diag = oracle.pose_step(depth, Wmap, flows, K, p, M, t, it, prevT=rel[t - 1],
                                           want_samples=True)
    S = p.n_pose_groups
    checked = 0
    for g in range(S):
        j = _group_pixels(p.seed, it, t, g, HW)
        slots = samples[4 * g:4 * g + 4]
        have = slots[:, 7] == 1
        if j is None:
            assert not have.any()
            continue
        want = Wmap[t - 1].ravel()[j[0]] * Wmap[t - 1].ravel()[j[1]] * Wmap[t - 1].ravel()[j[2]]
        for s in slots[have]:
            assert s[6] == pytest.approx(want, rel=1e-14), (g, j)
            checked += 1
        # any other frame's map gives another product
        other = Wmap[2 - t].ravel()
        assert not np.isclose(want, other[j[0]] * other[j[1]] * other[j[2]], rtol=1e-9)
    assert checked >= S // 2


@pytest.mark.parametrize("t", [1, 2])
def test_pose_step_correspondences_give_the_true_pose(t):
    # Sec. 5.2, Eq. 17: P_k = M_{t-1}(theta r_k) and y_k = pi_{t-1} + X_t(pi_{t-1}).
    # At the true depth and the true M_{t-1} on exact flow, every valid group has
    # a P3P root at the true T_t; which groups are valid follows from the
    # lookup domain of pi_{t-1}
    K, rel, flows, depth = _row_world(T=2)
    T, H, W, _ = flows.shape
    HW = H * W
    fx, fy, cx, cy = K
    p = oracle.params(n_pose_groups=300, seed=5)
    M = oracle.cumulative(rel)
    it = 0
    Tout, samples, diag = oracle.pose_step(depth, None, flows, K, p, M, t, it, prevT=None, want_samples=True)
    truth = oracle.se3_log(rel[t - 1][:9].reshape(3, 3), rel[t - 1][9:])
    Mp = M[t - 1]
    Rm, tm = Mp[:9].reshape(3, 3), Mp[9:]
    n_valid = 0
    for g in range(p.n_pose_groups):
        j = _group_pixels(p.seed, it, t, g, HW)
        slots = samples[4 * g:4 * g + 4]
        have = slots[:, 7] == 1
        ok = j is not None
        pts = []
        if ok:
            for jj in j:
                y, x = divmod(jj, W)
                P = Rm @ (depth[y, x] * np.array([(x - cx) / fx, (y - cy) / fy, 1.0])) + tm
                pts.append(P)
                px, py = (x, y) if t == 1 else (fx * P[0] / P[2] + cx, fy * P[1] / P[2] + cy)
                ok = ok and P[2] > 0 and _bilinear(flows[t - 1], px, py) is not None
        if not ok:
            assert not have.any(), g
            continue
        e1, e2 = pts[1] - pts[0], pts[2] - pts[0]
        if np.linalg.norm(np.cross(e1, e2)) < 1e-6 * np.linalg.norm(e1) * np.linalg.norm(e2):
            continue            # three collinear points: P3P has no unique answer
        n_valid += 1
        assert have.any(), g
        err = np.abs(slots[have, :6] - truth).max(axis=1)
        assert err.min() < 1e-8, (g, err)
    assert n_valid >= 100
    # the step's estimate is near the true pose: the spurious roots of the
    # groups that lie within the kernel's width (variances 0.1 and 0.004) pull
    # the mode by up to a few 1e-4
    assert np.abs(Tout - rel[t - 1]).max() < 2e-3


def test_pose_step_samples_follow_the_projection_of_the_previous_frame():
    # a wrong M (M_t in place of M_{t-1}) moves the 3-D points and the lookup:
    # the true pose is then no longer a root of most groups
    K, rel, flows, depth = _row_world(T=2)
    p = oracle.params(n_pose_groups=100, seed=5)
    M = oracle.cumulative(rel)
    Mwrong = M.copy()
    Mwrong[1] = M[2]
    truth = oracle.se3_log(np.eye(3), rel[1][9:])
    _, samples, _ = oracle.pose_step(depth, None, flows, K, p, Mwrong, 2, 0, want_samples=True)
    have = samples[:, 7] == 1
    err = np.abs(samples[have, :6] - truth).max(axis=1)
    assert np.mean(err < 1e-7) < 0.5


def _fisk_logpdf(x, alpha, beta):
    return scipy.stats.fisk(c=beta, scale=alpha).logpdf(x)


def test_window_loglik_is_eq3_at_the_final_state():
    # Eq. 3 with the final W (Table 1: W is the unsmoothed rigidness of the final
    # depth): L = sum over observed (t, j) of W log rho + (1 - W) log mu, its L1
    # mass beside it.  Every term is recomputed here with an own projection,
    # bilinear lookup and scipy's Fisk density.
    w = synthflow.make_window("small", 3, T=3, H=40, W=56)
    p = oracle.params(n_iters=2, n_pose_groups=128)
    st, poses, depth, rig, (L, mass), diag = oracle.window(w["flows"], w["K"], p)
    assert st == 0
    T, H, W, _ = w["flows"].shape
    fx, fy, cx, cy = w["K"]
    M = [np.eye(4)]
    for r in poses:
        A = np.eye(4)
        A[:3, :3] = r[:9].reshape(3, 3)
        A[:3, 3] = r[9:]
        M.append(A @ M[-1])
    acc, l1, n_obs = 0.0, 0.0, 0
    r_map = np.full((T, H, W), 0.5)
    for y in range(H):
        for x in range(W):
            ray = np.array([(x - cx) / fx, (y - cy) / fy, 1.0, 1.0 / depth[y, x]]) * depth[y, x]
            P = [Mt @ ray for Mt in M]
            for t in range(1, T + 1):
                if not (P[t - 1][2] > 0 and P[t][2] > 0):
                    continue
                u0, v0 = (x, y) if t == 1 else (fx * P[t - 1][0] / P[t - 1][2] + cx,
                                                fy * P[t - 1][1] / P[t - 1][2] + cy)
                v = _bilinear(w["flows"][t - 1], u0, v0)
                if v is None:
                    continue
                u1, v1 = fx * P[t][0] / P[t][2] + cx, fy * P[t][1] / P[t][2] + cy
                xres = max((u1 - u0 - v[0]) ** 2 + (v1 - v0 - v[1]) ** 2, p.x_floor)
                vn = math.hypot(v[0], v[1])
                alpha = p.a1 * math.exp(p.a2 * vn)
                beta = max(p.b1 * vn + p.b2, p.beta_min)
                lr = _fisk_logpdf(xres, alpha, beta)
                lm = _fisk_logpdf(max((p.lam * vn) ** 2, p.x_floor), alpha, beta)
                r = 1.0 / (1.0 + math.exp(lm - lr))
                r_map[t - 1, y, x] = r
                term = r * lr + (1 - r) * lm
                acc += term
                l1 += abs(term)
                n_obs += 1
    assert n_obs > 0.8 * T * H * W
    # the output rigidness is r at the final depth and poses
    assert np.abs(rig - r_map).max() < 1e-9
    assert L == pytest.approx(acc, rel=1e-10)
    assert mass == pytest.approx(l1, rel=1e-10)
    # the mu terms matter: without them (W = 1 everywhere) L would differ
    assert mass >= abs(L)


def _random_pose_world(H=48, W=64, f=80.0, seed=0):
    """One flow field from a general rigid motion at hand-made depths: the
    flow at every (integer) pixel is exact, so the triangulated depth is the
    true depth in the unit gauge |t_1| = 1."""
    rng = np.random.default_rng(seed)
    K = (f, f, W / 2.0, H / 2.0)
    n = H * W
    # well separated values (steps of 0.05) in random order
    vals = 2.0 + 0.05 * rng.permutation(n)
    depth = vals.reshape(H, W)
    ax = rng.normal(size=3)
    R = scipy.spatial.transform.Rotation.from_rotvec(0.02 * ax / np.linalg.norm(ax)).as_matrix()
    t = np.array([0.6, -0.25, 0.1])
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    rays = np.stack([(xs - K[2]) / f, (ys - K[3]) / f, np.ones_like(xs)], -1) * depth[..., None]
    P = rays @ R.T + t
    flows = np.zeros((1, H, W, 2), np.float32)
    flows[0, ..., 0] = f * P[..., 0] / P[..., 2] + K[2] - xs
    flows[0, ..., 1] = f * P[..., 1] / P[..., 2] + K[3] - ys
    return K, flows, depth, R, t


def test_bootstrap_depth_range_is_half_p1_and_twice_p99():
    # Sec. 5.3 / Table 1: the sampling range is [P1 / 2, 2 P99] of the valid
    # triangulated depths, percentiles by rank (the lower value at
    # floor(q (n - 1)) of the sorted depths); pixels without a depth take the
    # median, and every depth is clamped to the range
    K, flows, depth, R, t = _random_pose_world()
    H, W = depth.shape
    flat = depth.ravel().copy()
    order = np.argsort(flat)
    # the 20 nearest points pulled in far below P1 / 2, the 20 farthest pushed
    # far beyond 2 P99 (rank 30 and rank n - 1 - 30 stay as they were)
    near, far = order[:20], order[-20:]
    flat[near] = 0.05
    flat[far] = 500.0
    depth = flat.reshape(H, W)
    f = K[0]
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    rays = np.stack([(xs - K[2]) / f, (ys - K[3]) / f, np.ones_like(xs)], -1) * depth[..., None]
    P = rays @ R.T + t
    flows[0, ..., 0] = f * P[..., 0] / P[..., 2] + K[2] - xs
    flows[0, ..., 1] = f * P[..., 1] / P[..., 2] + K[3] - ys
    missing = [(3, 5), (20, 40), (47, 63)]
    for y, x in missing:
        flows[0, y, x] = np.nan
    st, rel, th, rng, info = oracle.bootstrap(flows, K, oracle.params())
    assert st == 0
    s = np.linalg.norm(t)
    assert np.abs(rel[9:] - t / s).max() < 1e-5
    valid = np.ones((H, W), bool)
    for y, x in missing:
        valid[y, x] = False
    v = np.sort(depth[valid] / s)
    n = v.size
    P1, P50, P99 = v[int(math.floor(0.01 * (n - 1)))], v[int(math.floor(0.5 * (n - 1)))], v[int(math.floor(0.99 * (n - 1)))]
    assert rng[0] == pytest.approx(0.5 * P1, rel=1e-5)
    assert rng[1] == pytest.approx(2.0 * P99, rel=1e-5)
    # a neighbouring rank or an interpolated percentile would be 0.05 / s away
    assert abs(rng[0] - 0.5 * v[int(math.floor(0.01 * (n - 1))) + 1]) > 1e-3
    for y, x in missing:
        assert th[y, x] == pytest.approx(P50, rel=1e-5)
    assert np.allclose(th.ravel()[near], rng[0], rtol=1e-12)
    assert np.allclose(th.ravel()[far], rng[1], rtol=1e-12)
    inside = valid & (depth / s > rng[0]) & (depth / s < rng[1])
    assert (np.abs(th[inside] * s - depth[inside]) / depth[inside]).max() < 1e-5


@pytest.mark.parametrize("u_obs", [480.0, 600.0, 900.0])
def test_emission_beta_min_clamp(u_obs):
    # Eq. 7 with the paper's constants gives B = b1 |v| + b2 <= 0 beyond
    # |v| = 454.5 px; the shape is then beta_min.  The emission follows the
    # Fisk density with that shape, and r = 1/2 still holds at EPE = lambda |v|
    p = oracle.params()
    B = p.b1 * u_obs + p.b2
    assert B <= 0
    H, W, f, theta = 16, 24, 100.0, 5.0
    K = (f, f, W / 2, H / 2)
    alpha = p.a1 * math.exp(p.a2 * u_obs)
    for xi in [u_obs * (1 + p.lam), u_obs + 1.0, u_obs + 40.0, u_obs]:
        M = np.zeros((2, 12))
        M[:, [0, 4, 8]] = 1
        M[1, 9] = xi * theta / f
        fl = np.zeros((1, H, W, 2), np.float32)
        fl[0, ..., 0] = u_obs
        r, ell, lr, lm, obs = oracle.emission_map(np.full((H, W), theta), fl, K, p, M)
        assert obs.all()
        x = max((xi - u_obs) ** 2, p.x_floor)
        fk = scipy.stats.fisk(c=p.beta_min, scale=alpha)
        assert np.allclose(lr, fk.logpdf(x), rtol=1e-9)
        assert np.allclose(lm, fk.logpdf((p.lam * u_obs) ** 2), rtol=1e-9)
        rr = 1.0 / (1.0 + math.exp(fk.logpdf((p.lam * u_obs) ** 2) - fk.logpdf(x)))
        assert np.allclose(r, rr, rtol=1e-9, atol=1e-15)
        if xi == u_obs * (1 + p.lam):
            assert np.allclose(r, 0.5, atol=1e-9)
    # a larger beta_min moves log rho: the clamp is what sets the shape
    p2 = oracle.params(beta_min=0.05)
    M = np.zeros((2, 12))
    M[:, [0, 4, 8]] = 1
    M[1, 9] = (u_obs + 1.0) * theta / f
    fl = np.zeros((1, H, W, 2), np.float32)
    fl[0, ..., 0] = u_obs
    _, _, lr2, _, _ = oracle.emission_map(np.full((H, W), theta), fl, K, p2, M)
    assert np.allclose(lr2, scipy.stats.fisk(c=0.05, scale=alpha).logpdf(1.0), rtol=1e-9)


def test_f32_range_hook_only_zeroes_posteriors_below_the_fp32_range():
    # the test hook under which the oracle takes the depth argmax with the
    # posterior in FP32's range: a posterior below 2^-126 becomes 0, nothing
    # else changes (log densities and ell of every item, larger posteriors)
    w = synthflow.make_window("small", 6, T=2, H=32, W=40)
    R, t = w["poses"][0]
    s = np.linalg.norm(t)
    rel = np.array([np.concatenate([R_.ravel(), t_ / s]) for R_, t_ in w["poses"]])
    M = oracle.cumulative(rel)
    theta = w["depth"] / s * np.exp(np.random.default_rng(0).normal(0, 0.3, w["depth"].shape))
    p = oracle.params(residual_model=1)
    a = oracle.emission_map(theta, w["flows"], w["K"], p, M)
    with oracle.f32_range():
        b = oracle.emission_map(theta, w["flows"], w["K"], p, M)
    c = oracle.emission_map(theta, w["flows"], w["K"], p, M)     # off again
    tiny = a[0] < 2.0 ** -126
    assert (a[0][tiny] > 0).sum() > 10            # FP64 keeps them (some underflow there too)
    assert np.all(b[0][tiny] == 0) and np.array_equal(b[0][~tiny], a[0][~tiny])
    for k in (1, 2, 3, 4):
        assert np.array_equal(a[k], b[k])
    assert all(np.array_equal(x, y) for x, y in zip(a, c))


def test_window_from_state_continues_the_window_exactly():
    # the window's iterations from the state an earlier, shorter window ends
    # in (its poses, depth, rigidness and depth range) are the longer window's
    # last iterations, bit for bit: the random draws depend only on the
    # iteration index, and the state is everything an iteration reads
    w = synthflow.make_window("small", 8, T=3, H=40, W=56)
    p2, p3 = oracle.params(n_iters=2, n_pose_groups=96), oracle.params(n_iters=3, n_pose_groups=96)
    st, P2, D2, R2, L2, diag2 = oracle.window(w["flows"], w["K"], p2)
    st3, P3, D3, R3, L3, diag3 = oracle.window(w["flows"], w["K"], p3)
    assert st == 0 and st3 == 0
    sf, Pf, Df, Rf, Lf = oracle.window_from_state(w["flows"], w["K"], p3, 2, P2, D2, R2, diag2[2:4])
    assert sf == 0
    assert np.array_equal(Pf, P3) and np.array_equal(Df, D3) and np.array_equal(Rf, R3)
    assert Lf == L3
    # a state from the wrong iteration (other random draws) gives another window
    sf, Pg, *_ = oracle.window_from_state(w["flows"], w["K"], oracle.params(n_iters=4, n_pose_groups=96), 3,
                                          P2, D2, R2, diag2[2:4])
    assert not np.array_equal(Pg, P3)
