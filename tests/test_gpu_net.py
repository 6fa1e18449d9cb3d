"""The learned proposal's HIP kernels (voldor_net_*) against the FP64 oracle
(oracle/net.py), through the C ABI.

Tolerances follow from BF16 (8 significant bits, unit roundoff u = 2^-9):
  * one layer on exact BF16 inputs and weights: the GPU accumulates in FP32 and
    rounds the output once to BF16, so |d| <= 2u |y| + 1e-5 max|y| (FP32 sums of
    288 terms sit far below that); the FP32 output of layer 6 to 1e-5 max|y|;
  * whole network: every hidden activation and every back-propagated gradient
    is rounded to BF16 once per layer (twelve roundings of relative size u on
    the longest path) -> relative L2 error of loss, outputs and each layer's
    gradient <= 12 u ~ 2.4 % with cosine >= 0.999;
  * Adam: FP32 arithmetic on the GPU's own gradient, 1e-6 relative.
"""
import numpy as np
import pytest

from oracle import net as onet

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

U = 2.0 ** -9


@pytest.fixture(scope="module")
def vo():
    import paper_2104_06789_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _bf16(torch, a):
    """Round to BF16 (round to nearest even) and back to float64."""
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _pack(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params]).astype(np.float32)


def _unpack(flat, like):
    out, o = [], 0
    for w, b in like:
        nw = w.size
        out.append((flat[o:o + nw].reshape(w.shape).astype(np.float64), flat[o + nw:o + nw + b.size].astype(np.float64)))
        o += nw + b.size
    return out


def _params(T, seed):
    rng = np.random.default_rng(seed + 100)
    ps = onet.init_params(T, seed)
    out = []
    for k, (w, b) in enumerate(ps):
        co_real = 1 + T if k == onet.N_LAYERS - 1 else b.size
        bb = np.zeros_like(b)
        bb[:co_real] = rng.normal(0, 0.1, co_real)
        out.append((w, bb))
    return out


def _net(vo, T, N, H, W, seed=0):
    n = vo.Net(T, N, H, W)
    ps = _params(T, seed)
    flat = _pack(ps)
    assert flat.size == n.n_params
    n.set_params(flat)
    return n, _unpack(flat, ps)   # the FP32 values the GPU holds


@pytest.mark.parametrize("k", [0, 2, 5])
def test_layer_forward_exact_inputs(vo, torch, k):
    T, N, H, W = 3, 2, 13, 37
    n, ps = _net(vo, T, N, H, W, seed=k)
    rng = np.random.default_rng(k)
    x = rng.normal(0, 1, (N, H, W, 32)).astype(np.float32)
    if k > 0:
        x = np.maximum(x, 0)
    xt = torch.from_numpy(x).to(torch.bfloat16).cuda()
    out = torch.empty((N, H, W, 16 if k == 5 else 32), dtype=torch.float32 if k == 5 else torch.bfloat16,
                      device="cuda")
    n.layer(k, xt, out)
    torch.cuda.synchronize()
    w, b = ps[k]
    ref = onet.conv3x3(xt.cpu().to(torch.float64).numpy(), _bf16(torch, w), b)
    if k < 5:
        ref = np.maximum(ref, 0)
    got = out.cpu().to(torch.float64).numpy()
    scale = np.abs(ref).max()
    tol = (1e-5 * scale) if k == 5 else (2 * U * np.abs(ref) + 1e-5 * scale)
    assert np.all(np.abs(got - ref) <= tol), float(np.abs(got - ref).max())


@pytest.mark.parametrize("k", [1, 3, 5])
def test_layer_backward_exact_inputs(vo, torch, k):
    T, N, H, W = 3, 2, 11, 35
    n, ps = _net(vo, T, N, H, W, seed=k)
    rng = np.random.default_rng(10 + k)
    co = 16 if k == 5 else 32
    dy = np.zeros((N, H, W, 32), np.float32)
    dy[..., :co] = rng.normal(0, 1, (N, H, W, co))
    if k == 5:
        dy[..., 1 + T:] = 0.0
    mask = np.maximum(rng.normal(0, 1, (N, H, W, 32)), 0).astype(np.float32)
    dyt = torch.from_numpy(dy).to(torch.bfloat16).cuda()
    mt = torch.from_numpy(mask).to(torch.bfloat16).cuda()
    out = torch.empty((N, H, W, 32), dtype=torch.bfloat16, device="cuda")
    n.layer(k, dyt, out, mask=mt, backward=True)
    torch.cuda.synchronize()
    w, _ = ps[k]
    dy64 = dyt.cpu().to(torch.float64).numpy()[..., :co]
    gx, _, _ = onet.conv3x3_backward(np.zeros((N, H, W, 32)), _bf16(torch, w), dy64)
    ref = gx * (mask > 0)
    got = out.cpu().to(torch.float64).numpy()
    scale = np.abs(ref).max()
    assert np.all(np.abs(got - ref) <= 2 * U * np.abs(ref) + 1e-5 * scale), float(np.abs(got - ref).max())


def _window_batch(T, N, H, W, seed):
    rng = np.random.default_rng(seed)
    flows = rng.normal(0, 8, (N, T, H, W, 2)).astype(np.float32)
    flows[0, 1, 3, 5] = np.nan
    depth = np.exp(rng.normal(1.0, 0.4, (N, H, W))).astype(np.float32)
    rig = rng.uniform(0.05, 0.95, (N, T, H, W)).astype(np.float32)
    return flows, depth, rig


def test_network_gradient_parity(vo, torch):
    T, N, H, W = 3, 2, 24, 40   # ragged against 16- and 32-pixel tiles
    n, ps = _net(vo, T, N, H, W, seed=7)
    flows, depth, rig = _window_batch(T, N, H, W, 7)
    ft, dt, rt = (torch.from_numpy(a).cuda() for a in (flows, depth, rig))
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    grad = torch.zeros(n.n_params, dtype=torch.float32, device="cuda")
    z = torch.zeros((N, H, W, 16), dtype=torch.float32, device="cuda")
    n.forward(ft, z=z)
    n.gradient(ft, dt, rt, loss=loss, grad=grad)
    torch.cuda.synchronize()
    # oracle on the BF16 weights the GPU multiplies with, FP64 everywhere else
    pq = [(_bf16(torch, w), b) for w, b in ps]
    x = onet.net_input(flows.astype(np.float64))
    zr, acts = onet.forward(pq, _bf16(torch, x))
    lr_, gz = onet.loss_and_grad(zr, T, np.log(depth.astype(np.float64)), rig.astype(np.float64))
    grads = onet.backward(pq, acts, gz)
    zg = z.cpu().numpy().astype(np.float64)[..., :1 + T]
    assert np.linalg.norm(zg - zr[..., :1 + T]) <= 12 * U * np.linalg.norm(zr[..., :1 + T])
    assert float(loss) == pytest.approx(lr_, rel=12 * U)
    g = grad.cpu().numpy().astype(np.float64)
    o = 0
    for k, (gw, gb) in enumerate(grads):
        ref = np.concatenate([gw.ravel(), gb.ravel()])
        got = g[o:o + ref.size]
        o += ref.size
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        cos = float(got @ ref / (np.linalg.norm(got) * np.linalg.norm(ref)))
        print(k, rel, cos)
        assert rel <= 12 * U and cos >= 0.999, (k, rel, cos)


@pytest.mark.parametrize("N,H,W", [(2, 37, 71), (1, 5, 9), (1, 48, 96)])
def test_fused_forward_equals_layers(vo, torch, N, H, W):
    # the one-launch forward pass (all six layers on LDS tiles of 16 x 32
    # output pixels with a 6-pixel halo) against the six single-layer launches,
    # bit for bit: ragged tiles, an image smaller than one tile, whole tiles
    T = 3
    n, ps = _net(vo, T, N, H, W, seed=3)
    flows, _, _ = _window_batch(T, N, H, W, 3)
    ft = torch.from_numpy(flows).cuda()
    z = torch.zeros((N, H, W, 16), dtype=torch.float32, device="cuda")
    n.forward(ft, z=z)
    x = torch.from_numpy(onet.net_input(flows.astype(np.float64)).astype(np.float32)).to(torch.bfloat16).cuda()
    for k in range(5):
        y = torch.empty((N, H, W, 32), dtype=torch.bfloat16, device="cuda")
        n.layer(k, x.contiguous(), y)
        x = y
    zl = torch.empty((N, H, W, 16), dtype=torch.float32, device="cuda")
    n.layer(5, x.contiguous(), zl)
    torch.cuda.synchronize()
    assert torch.equal(z, zl), float((z - zl).abs().max())


def test_adam_step_and_training_descends(vo, torch):
    T, N, H, W = 2, 2, 20, 33
    n, ps = _net(vo, T, N, H, W, seed=3)
    flows, depth, rig = _window_batch(T, N, H, W, 3)
    ft, dt, rt = (torch.from_numpy(a).cuda() for a in (flows, depth, rig))
    p0 = n.get_params().astype(np.float64)
    grad = torch.zeros(n.n_params, dtype=torch.float32, device="cuda")
    n.gradient(ft, dt, rt, grad=grad)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    n.train_step(ft, dt, rt, 1e-3, loss=loss)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    want, _, _ = onet.adam_step(p0, g, np.zeros_like(g), np.zeros_like(g), 1, lr=1e-3)
    got = n.get_params().astype(np.float64)
    assert np.allclose(got, want, rtol=1e-6, atol=1e-9)
    losses = [float(loss)]
    for _ in range(30):
        n.train_step(ft, dt, rt, 3e-3, loss=loss)
        losses.append(float(loss))
    torch.cuda.synchronize()
    assert losses[-1] < 0.7 * losses[0], losses
