"""FP64 numpy oracle of the learned depth/rigidness proposal.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use it.

The paper's method has no network; the proposal is an extension that only
replaces the initial state of Table 1 (depth theta and rigidness W) and is
judged by the plain EM afterwards.  Its definition here:

  * input: the 2T flow channels (u_t, v_t), t = 1..T, divided by IN_SCALE,
    non-finite values as 0, zero-padded to C_IN channels;
  * six 3x3 convolutions, stride 1, zero padding; layers 1..5 have 32 output
    channels and a ReLU, layer 6 has 1 + T outputs (padded to C_OUT6);
  * output channel 0 is log theta, channels 1..T the logits of W_t;
  * loss = mean over pixels of (z_0 - log theta*)^2
         + mean over pixels and frames of BCE(sigmoid(z_t), W*_t),
    BCE written with logits: softplus(z) - W* z;
  * Adam (Kingma & Ba, ICLR 2015) with bias correction.

Tensors are NHWC float64; weights are [3][3][C_in][C_out] (dy, dx, in, out).
"""
from __future__ import annotations

import numpy as np

C_IN = 32           # input channels after padding (2T <= 16 real ones)
C_HID = 32          # hidden width
C_OUT6 = 16         # output channels of layer 6 after padding (1 + T <= 9 real ones)
N_LAYERS = 6
IN_SCALE = 16.0     # pixels per input unit


def layer_shapes():
    """(C_in, C_out, relu) of the six layers."""
    out = []
    for k in range(N_LAYERS):
        ci = C_IN if k == 0 else C_HID
        co = C_OUT6 if k == N_LAYERS - 1 else C_HID
        out.append((ci, co, k < N_LAYERS - 1))
    return out


def net_input(flows):
    """flows [N][T][H][W][2] -> x [N][H][W][C_IN]: channel 2(t-1)+c is component c of X_t."""
    f = np.asarray(flows, dtype=np.float64)
    N, T, H, W, _ = f.shape
    x = np.zeros((N, H, W, C_IN))
    g = np.where(np.isfinite(f), f, 0.0) / IN_SCALE
    for t in range(T):
        x[..., 2 * t] = g[:, t, :, :, 0]
        x[..., 2 * t + 1] = g[:, t, :, :, 1]
    return x


def conv3x3(x, w, b):
    """y[n,y,x,o] = b[o] + sum_{dy,dx,i} w[dy,dx,i,o] x[n, y+dy-1, x+dx-1, i] (zero outside)."""
    N, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    y = np.broadcast_to(b, (N, H, W, w.shape[3])).astype(np.float64).copy()
    for dy in range(3):
        for dx in range(3):
            y += xp[:, dy:dy + H, dx:dx + W, :] @ w[dy, dx]
    return y


def conv3x3_backward(x, w, gy):
    """Gradients of sum(gy * conv3x3(x, w, b)) with respect to x, w and b."""
    N, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for dy in range(3):
        for dx in range(3):
            win = xp[:, dy:dy + H, dx:dx + W, :]
            gw[dy, dx] = np.einsum("nhwi,nhwo->io", win, gy)
            gxp[:, dy:dy + H, dx:dx + W, :] += gy @ w[dy, dx].T
    gb = gy.sum(axis=(0, 1, 2))
    return gxp[:, 1:H + 1, 1:W + 1, :], gw, gb


def forward(params, x):
    """params: list of (w, b).  Returns (z, acts) with acts[k] = input of layer k."""
    acts = [x]
    h = x
    for k, ((w, b), (_, _, relu)) in enumerate(zip(params, layer_shapes())):
        h = conv3x3(h, w, b)
        if relu:
            h = np.maximum(h, 0.0)
        if k < N_LAYERS - 1:
            acts.append(h)
    return h, acts


def loss_and_grad(z, T, logd_target, w_target):
    """Loss of the outputs z [N][H][W][C_OUT6] against log theta* [N][H][W] and
    W* [N][T][H][W]; returns (loss, dloss/dz)."""
    N, H, W, _ = z.shape
    npx = N * H * W
    gz = np.zeros_like(z)
    d = z[..., 0] - logd_target
    loss = np.sum(d * d) / npx
    gz[..., 0] = 2.0 * d / npx
    for t in range(T):
        s = z[..., 1 + t]
        wt = w_target[:, t]
        # softplus(s) - wt s, stably
        loss += np.sum(np.maximum(s, 0.0) + np.log1p(np.exp(-np.abs(s))) - wt * s) / (npx * T)
        gz[..., 1 + t] = (1.0 / (1.0 + np.exp(-s)) - wt) / (npx * T)
    return loss, gz


def backward(params, acts, gz):
    """Gradients [(gw, gb)] of the loss through the six layers, given dloss/dz."""
    grads = [None] * N_LAYERS
    g = gz
    for k in range(N_LAYERS - 1, -1, -1):
        w, b = params[k]
        x = acts[k]
        gx, gw, gb = conv3x3_backward(x, w, g)
        grads[k] = (gw, gb)
        if k > 0:
            g = gx * (acts[k] > 0.0)   # ReLU of layer k-1: acts[k] is its output
    return grads


def adam_step(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(T, seed=0):
    """He-normal weights (std sqrt(2 / (9 C_in_real))), zero biases; padded input
    channels and padded output channels of layer 6 are zero."""
    rng = np.random.default_rng(seed)
    params = []
    for k, (ci, co, _) in enumerate(layer_shapes()):
        ci_real = 2 * T if k == 0 else ci
        co_real = 1 + T if k == N_LAYERS - 1 else co
        w = np.zeros((3, 3, ci, co))
        w[:, :, :ci_real, :co_real] = rng.normal(0.0, np.sqrt(2.0 / (9 * ci_real)), (3, 3, ci_real, co_real))
        params.append((w, np.zeros(co)))
    return params
