"""Batches of windows of uneven shape and T (voldor_window_batch) against the
single-window solver, through the C ABI.  Every window of a batch runs the same
kernels on the same inputs as voldor_window, so the results must agree bit for
bit, whatever lane a window lands on, with or without graph capture and replay,
and in lockstep mode, where one launch serves the pose-step kernels, sweeps and
rigidness passes of all the windows of a lane.
"""
import numpy as np
import pytest

import synthflow

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

# (generator, seed, T, H, W): uneven shapes and T, ragged sizes
MIX = [("small", 11, 3, 48, 64), ("driving", 12, 4, 40, 124), ("small", 13, 2, 64, 48),
       ("small", 14, 5, 56, 72), ("driving", 15, 3, 32, 100)]
S = 128


@pytest.fixture(scope="module")
def vo():
    import paper_2104_06789_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


@pytest.fixture(scope="module")
def case(vo, torch):
    wins = [synthflow.make_window(g, sd, T=T, H=H, W=W) for g, sd, T, H, W in MIX]
    flows = [torch.from_numpy(w["flows"]).cuda() for w in wins]
    p = vo.default_params(n_iters=2, n_pose_groups=S)
    Tm = max(m[2] for m in MIX)
    Hm = max(m[3] for m in MIX)
    Wm = max(m[4] for m in MIX)
    solver = vo.Solver(Tm, Hm, Wm, S)
    ref = [tuple(x.clone() for x in solver.window(f, w["K"], p)) for f, w in zip(flows, wins)]
    return dict(wins=wins, flows=flows, p=p, ref=ref, dims=(Tm, Hm, Wm), solver=solver)


def _outs(vo, case, idx):
    outs = []
    for i in idx:
        T, H, W, _ = case["flows"][i].shape
        o = vo.Batch.outputs(T, H, W)
        for x in o:
            x.fill_(float("nan"))
        outs.append(o)
    return outs


def _check(torch, case, idx, outs, status, expect_status=None):
    st = status[:len(idx)].cpu().tolist()
    for k, i in enumerate(idx):
        want = 0 if expect_status is None else expect_status[k]
        assert st[k] == want, (k, i, st)
        if want == 0:
            for a, b in zip(outs[k], case["ref"][i]):
                assert torch.equal(a, b), (k, i)


@pytest.mark.parametrize("lockstep", [False, True])
@pytest.mark.parametrize("lanes", [1, 3, 4])
def test_batch_equals_single_windows(vo, torch, case, lanes, lockstep):
    idx = list(range(len(MIX)))
    b = vo.Batch(lanes, *case["dims"], S, lockstep=lockstep)
    outs = _outs(vo, case, idx)
    status = torch.full((len(idx),), -99, dtype=torch.int32, device="cuda")
    b.solve([(case["flows"][i], case["wins"][i]["K"], outs[k]) for k, i in enumerate(idx)], case["p"], status)
    torch.cuda.synchronize()
    _check(torch, case, idx, outs, status)


@pytest.mark.parametrize("lockstep", [False, True])
def test_batch_graph_replays_and_recaptures(vo, torch, case, lockstep):
    s = torch.cuda.Stream()
    b = vo.Batch(3, *case["dims"], S, graph=True, lockstep=lockstep)
    idx = list(range(len(MIX)))
    outs = _outs(vo, case, idx)
    status = torch.full((len(idx),), -99, dtype=torch.int32, device="cuda")
    items = [(case["flows"][i], case["wins"][i]["K"], outs[k]) for k, i in enumerate(idx)]
    for rep in range(3):
        # eager work between replays: scrub the outputs, solve one window alone
        for o in outs:
            for x in o:
                x.fill_(float("nan"))
        status.fill_(-99)
        torch.cuda.synchronize()
        case["solver"].window(case["flows"][0], case["wins"][0]["K"], case["p"])
        with torch.cuda.stream(s):
            b.solve(items, case["p"], status, stream=s)
        s.synchronize()
        _check(torch, case, idx, outs, status)
    # a different (smaller) call captures a new graph
    idx2 = [3, 1]
    outs2 = _outs(vo, case, idx2)
    status2 = torch.full((2,), -99, dtype=torch.int32, device="cuda")
    with torch.cuda.stream(s):
        b.solve([(case["flows"][i], case["wins"][i]["K"], outs2[k]) for k, i in enumerate(idx2)], case["p"],
                status2, stream=s)
    s.synchronize()
    _check(torch, case, idx2, outs2, status2)


@pytest.mark.parametrize("lockstep", [False, True])
def test_batch_degenerate_window_reports_alone(vo, torch, case, lockstep):
    # every flow of window 2 missing: only its status says so
    idx = list(range(len(MIX)))
    bad = torch.full_like(case["flows"][2], float("nan"))
    outs = _outs(vo, case, idx)
    status = torch.full((len(idx),), -99, dtype=torch.int32, device="cuda")
    items = [(bad if i == 2 else case["flows"][i], case["wins"][i]["K"], outs[k]) for k, i in enumerate(idx)]
    vo.Batch(2, *case["dims"], S, lockstep=lockstep).solve(items, case["p"], status)
    torch.cuda.synchronize()
    _check(torch, case, idx, outs, status, expect_status=[0, 0, -4, 0, 0])


def test_batch_rejects_bad_descriptor_before_enqueue(vo, torch, case):
    b = vo.Batch(2, *case["dims"], S)
    big = torch.zeros((2, case["dims"][1] + 8, 32, 2), device="cuda")   # taller than the workspace
    outs = _outs(vo, case, [0, 1])
    status = torch.full((2,), -99, dtype=torch.int32, device="cuda")
    with pytest.raises(vo.VoldorError) as e:
        b.solve([(case["flows"][0], case["wins"][0]["K"], outs[0]), (big, case["wins"][1]["K"], outs[1])],
                case["p"], status)
    assert e.value.code == vo.EINVAL
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [-99, -99]   # nothing ran


def test_lockstep_per_window_groups_and_repeat_calls(vo, torch, case):
    # P3P groups per frame differ by window (the pose-step launches cover
    # windows of different block counts); a second call with other windows
    # rebuilds the plan, a third repeats the first
    groups = [96, 128, 64, 128, 80]
    solver = case["solver"]
    ref = []
    for i, g in enumerate(groups):
        p = vo.default_params(n_iters=2, n_pose_groups=g)
        ref.append(tuple(x.clone() for x in solver.window(case["flows"][i], case["wins"][i]["K"], p)))
    b = vo.Batch(2, *case["dims"], S, lockstep=True)
    for idx in ([0, 1, 2, 3, 4], [4, 2], [0, 1, 2, 3, 4]):
        outs = _outs(vo, case, idx)
        status = torch.full((len(idx),), -99, dtype=torch.int32, device="cuda")
        b.solve([(case["flows"][i], case["wins"][i]["K"], outs[k], None, groups[i]) for k, i in enumerate(idx)],
                case["p"], status)
        torch.cuda.synchronize()
        assert status.cpu().tolist() == [0] * len(idx)
        for k, i in enumerate(idx):
            for a, r in zip(outs[k], ref[i]):
                assert torch.equal(a, r), (idx, k, i)


def test_lockstep_rejects_allpixel_start_and_proposals(vo, torch, case):
    b = vo.Batch(2, *case["dims"], S, lockstep=True)
    outs = _outs(vo, case, [0])
    status = torch.full((1,), -99, dtype=torch.int32, device="cuda")
    item = (case["flows"][0], case["wins"][0]["K"], outs[0])
    with pytest.raises(vo.VoldorError) as e:
        b.solve([item], vo.default_params(n_iters=2, n_pose_groups=S, pose_start=1), status)
    assert e.value.code == vo.EINVAL
    T, H, W, _ = case["flows"][0].shape
    init = (torch.ones((H, W), device="cuda"), torch.ones((T, H, W), device="cuda"), None)
    with pytest.raises(vo.VoldorError) as e:
        b.solve([item + (init,)], case["p"], status)
    assert e.value.code == vo.EINVAL
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [-99]   # nothing ran
