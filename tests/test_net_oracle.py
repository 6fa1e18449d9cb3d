"""Pins of the FP64 oracle of the learned proposal (oracle/net.py): convolution
against brute force and scipy, every gradient against central finite
differences, Adam against its closed-form first step and a convex problem."""
import numpy as np
import pytest
import scipy.signal

from oracle import net

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _brute_conv(x, w, b):
    N, H, W, Ci = x.shape
    Co = w.shape[3]
    y = np.zeros((N, H, W, Co))
    for n in range(N):
        for yy in range(H):
            for xx in range(W):
                for o in range(Co):
                    s = b[o]
                    for dy in range(3):
                        for dx in range(3):
                            sy, sx = yy + dy - 1, xx + dx - 1
                            if 0 <= sy < H and 0 <= sx < W:
                                for i in range(Ci):
                                    s += w[dy, dx, i, o] * x[n, sy, sx, i]
                    y[n, yy, xx, o] = s
    return y


def test_conv_brute_force_and_scipy():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 4, 5, 3))
    w = rng.normal(size=(3, 3, 3, 2))
    b = rng.normal(size=2)
    y = net.conv3x3(x, w, b)
    assert np.allclose(y, _brute_conv(x, w, b), atol=1e-12)
    # the same as scipy's 2-D correlation summed over input channels
    for n in range(2):
        for o in range(2):
            ref = b[o] + sum(scipy.signal.correlate2d(x[n, :, :, i], w[:, :, i, o], mode="same")
                             for i in range(3))
            assert np.allclose(y[n, :, :, o], ref, atol=1e-12)


def test_conv_backward_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 4, 4, 3))
    w = rng.normal(size=(3, 3, 3, 2))
    b = rng.normal(size=2)
    gy = rng.normal(size=(1, 4, 4, 2))
    gx, gw, gb = net.conv3x3_backward(x, w, gy)
    f = lambda x_, w_, b_: np.sum(gy * net.conv3x3(x_, w_, b_))
    h = 1e-6
    for idx in [(0, 0, 0, 0), (0, 3, 2, 1), (0, 1, 3, 2)]:
        e = np.zeros_like(x)
        e[idx] = h
        assert (f(x + e, w, b) - f(x - e, w, b)) / (2 * h) == pytest.approx(gx[idx], rel=1e-7, abs=1e-9)
    for idx in [(0, 0, 0, 0), (2, 1, 2, 1), (1, 1, 1, 0)]:
        e = np.zeros_like(w)
        e[idx] = h
        assert (f(x, w + e, b) - f(x, w - e, b)) / (2 * h) == pytest.approx(gw[idx], rel=1e-7, abs=1e-9)
    for o in range(2):
        e = np.zeros_like(b)
        e[o] = h
        assert (f(x, w, b + e) - f(x, w, b - e)) / (2 * h) == pytest.approx(gb[o], rel=1e-7)


def _tiny_problem(seed=2, T=3, H=5, W=4):
    rng = np.random.default_rng(seed)
    params = net.init_params(T, seed)
    # non-zero biases so that every ReLU sees both signs
    params = [(w, rng.normal(0, 0.1, b.shape)) for w, b in params]
    flows = rng.normal(0, 8, (1, T, H, W, 2))
    flows[0, 1, 2, 1, 0] = np.nan   # a missing flow enters as 0
    x = net.net_input(flows)
    logd = rng.normal(1.0, 0.5, (1, H, W))
    wt = rng.uniform(0, 1, (1, T, H, W))
    return params, x, logd, wt, T


def test_net_input_layout():
    T, H, W = 2, 3, 4
    flows = np.arange(T * H * W * 2, dtype=np.float64).reshape(1, T, H, W, 2)
    flows[0, 1, 0, 0, 1] = np.inf
    x = net.net_input(flows)
    assert x.shape == (1, H, W, net.C_IN)
    assert x[0, 2, 3, 2] == flows[0, 1, 2, 3, 0] / net.IN_SCALE
    assert x[0, 0, 0, 3] == 0.0 and np.all(x[..., 2 * T:] == 0.0)


def test_net_gradient_finite_differences():
    params, x, logd, wt, T = _tiny_problem()
    z, acts = net.forward(params, x)
    loss, gz = net.loss_and_grad(z, T, logd, wt)
    grads = net.backward(params, acts, gz)

    def total(ps):
        zz, _ = net.forward(ps, x)
        return net.loss_and_grad(zz, T, logd, wt)[0]

    h = 1e-6
    rng = np.random.default_rng(3)
    for k in range(net.N_LAYERS):
        w, b = params[k]
        ci_real = 2 * T if k == 0 else w.shape[2]
        co_real = 1 + T if k == net.N_LAYERS - 1 else w.shape[3]
        for _ in range(3):
            idx = (rng.integers(3), rng.integers(3), rng.integers(ci_real), rng.integers(co_real))
            wp = w.copy(); wp[idx] += h
            wm = w.copy(); wm[idx] -= h
            pp = list(params); pp[k] = (wp, b)
            pm = list(params); pm[k] = (wm, b)
            fd = (total(pp) - total(pm)) / (2 * h)
            assert fd == pytest.approx(grads[k][0][idx], rel=1e-5, abs=1e-9)
        o = int(rng.integers(co_real))
        bp = b.copy(); bp[o] += h
        bm = b.copy(); bm[o] -= h
        pp = list(params); pp[k] = (w, bp)
        pm = list(params); pm[k] = (w, bm)
        assert (total(pp) - total(pm)) / (2 * h) == pytest.approx(grads[k][1][o], rel=1e-5, abs=1e-9)


def test_loss_closed_forms():
    # z_0 = log theta* and logits at +-inf towards W* in {0, 1}: zero loss and gradient
    T, N, H, W = 2, 1, 2, 3
    logd = np.full((N, H, W), 0.7)
    wt = np.zeros((N, T, H, W))
    wt[:, 1] = 1.0
    z = np.zeros((N, H, W, net.C_OUT6))
    z[..., 0] = 0.7
    z[..., 1] = -60.0
    z[..., 2] = 60.0
    loss, gz = net.loss_and_grad(z, T, logd, wt)
    assert loss == pytest.approx(0.0, abs=1e-25)
    assert np.abs(gz).max() < 1e-26
    # all logits 0, targets 1/2: loss = log 2, gradient 0
    z[..., 1:3] = 0.0
    loss, gz = net.loss_and_grad(z, T, logd, np.full((N, T, H, W), 0.5))
    assert loss == pytest.approx(np.log(2.0), rel=1e-14)
    assert np.abs(gz).max() == 0.0


def test_adam_first_step_and_convergence():
    g = np.array([3.0, -2e-3, 0.5])
    p, m, v = net.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    # bias-corrected first step is lr * g / |g|
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-12)
    # a convex quadratic converges to its minimum
    target = np.array([1.0, -2.0, 0.25])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for s in range(1, 4001):
        p, m, v = net.adam_step(p, 2 * (p - target), m, v, s, lr=0.01)
    assert np.allclose(p, target, atol=1e-3)

