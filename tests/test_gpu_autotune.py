"""Sweep widths (threads per chain), look-ahead caps and the autotuner, through
the C ABI.

Every width (256, 512, 768, 1024 threads per chain) and every look-ahead cap of the
propagation rounds computes each item with the same FP32 function and the
propagation's first losses exactly, so the depth of a sweep, and a whole
window, must be the same bit for bit at every setting; the autotuner only
picks the fastest, per chain class.
"""
import numpy as np
import pytest

import synthflow

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


@pytest.mark.parametrize("criterion", [0, 1])
def test_sweep_widths_bit_identical(vo, torch, criterion):
    # ragged 45x83 chains (shorter than every width), 4 frames, every direction
    T, H, W = 4, 45, 83
    w = synthflow.make_window("small", 20, T=T, H=H, W=W)
    R, t = w["poses"][0]
    rel = np.array([np.concatenate([R_.ravel(), t_ / np.linalg.norm(t)]) for R_, t_ in w["poses"]])
    M = [np.concatenate([np.eye(3).ravel(), np.zeros(3)])]
    for r in rel:
        Rr, tr = r[:9].reshape(3, 3), r[9:]
        Rm, tm = M[-1][:9].reshape(3, 3), M[-1][9:]
        M.append(np.concatenate([(Rr @ Rm).ravel(), Rr @ tm + tr]))
    M = np.array(M)
    gt = w["depth"] / np.linalg.norm(t)
    theta = torch.from_numpy((gt * np.exp(np.random.default_rng(1).normal(0, 0.15, gt.shape))).astype(np.float32)).cuda()
    fl = torch.from_numpy(w["flows"]).cuda()
    p = vo.default_params(criterion=criterion)
    s = vo.Solver(T, H, W, 256)
    d_lo, d_hi = 0.5 * float(gt.min()), 2.0 * float(gt.max())
    ref = {}
    for nt, cap in ((512, 0), (256, 0), (768, 0), (1024, 0), (512, 1), (256, 3), (768, 2), (1024, 16)):
        s.set_sweep_threads(nt, nt)
        s.set_sweep_lookahead(cap, cap)
        assert s.sweep_threads() == (nt, nt) and s.sweep_lookahead() == (cap, cap)
        for direction in range(4):
            out, q = s.sweep(theta, fl, w["K"], p, M, d_lo, d_hi, 3 + direction, direction, want_q=True)
            torch.cuda.synchronize()
            if (nt, cap) == (512, 0):
                ref[direction] = (out.clone(), q.clone())
            else:
                assert torch.equal(out, ref[direction][0]), (nt, cap, direction)
                assert torch.equal(q, ref[direction][1]), (nt, cap, direction)


def test_window_widths_and_autotune(vo, torch):
    w = synthflow.make_window("small", 0)
    spec = w["spec"]
    T, H, W = spec.T, spec.H, spec.W
    p = vo.default_params(n_iters=spec.n_iters, n_pose_groups=spec.n_groups)
    fl = torch.from_numpy(w["flows"]).cuda()
    s = vo.Solver(T, H, W, 256)
    ref = [x.clone() for x in s.window(fl, w["K"], p)]
    for rows, cols in [(256, 1024), (1024, 256)]:
        s.set_sweep_threads(rows, cols)
        out = s.window(fl, w["K"], p)
        for a, b in zip(out, ref):
            assert torch.equal(a, b), (rows, cols)
    s.set_sweep_lookahead(2, 5)
    out = s.window(fl, w["K"], p)
    for a, b in zip(out, ref):
        assert torch.equal(a, b)
    rows, cols = s.autotune(fl, w["K"], p)
    assert rows in (256, 512, 768, 1024) and cols in (256, 512, 768, 1024)
    tab = s.sweep_tuning()
    print(tab)
    assert (W, T, rows) == tab[0][:3] and (H, T, cols) == tab[1][:3]
    assert tab[0][3] in (0, 2, 4, 8, 16, 32) and tab[1][3] in (0, 2, 4, 8, 16, 32)
    out = s.window(fl, w["K"], p)
    for a, b in zip(out, ref):
        assert torch.equal(a, b)
    with pytest.raises(vo.VoldorError):
        s.set_sweep_threads(384, 512)
    with pytest.raises(vo.VoldorError):
        s.set_sweep_lookahead(-1, 0)
    s.set_sweep_threads(0, 0)
    assert s.sweep_threads() == (512, 512) and s.sweep_tuning() == []


def test_batch_autotune_keeps_results(vo, torch):
    # per-window P3P groups and the batch autotuner: results equal the single
    # windows solved with those groups, before and after tuning
    wins = [synthflow.make_window("small", sd, T=T, H=H, W=W) for sd, T, H, W in
            ((1, 3, 48, 64), (2, 4, 40, 72), (3, 3, 48, 64))]
    groups = (96, 128, 64)
    p = vo.default_params(n_iters=2, n_pose_groups=200)
    flows = [torch.from_numpy(w["flows"]).cuda() for w in wins]
    refs = []
    for f, w, g in zip(flows, wins, groups):
        T, H, W = f.shape[:3]
        s = vo.Solver(T, H, W, 256)
        refs.append([x.clone() for x in s.window(f, w["K"], vo.default_params(n_iters=2, n_pose_groups=g))])
        s.close()
    b = vo.Batch(2, 4, 48, 72, 256, graph=True)
    outs = [vo.Batch.outputs(*f.shape[:3]) for f in flows]
    items = [(f, w["K"], o, None, g) for f, w, o, g in zip(flows, wins, outs, groups)]
    st = torch.full((3,), -9, dtype=torch.int32, device="cuda")
    stream = torch.cuda.Stream()
    for tune in (False, True):
        if tune:
            b.autotune(items, p, stream=stream)
        with torch.cuda.stream(stream):
            b.solve(items, p, st, stream=stream)
        torch.cuda.synchronize()
        assert st.cpu().tolist() == [0, 0, 0]
        for o, r in zip(outs, refs):
            for a, c in zip(o, r):
                assert torch.equal(a, c), tune
    b.close()
