"""What the trained proposal gains: the network (voldor_net_*) is trained on
the GPU by the library's own forward, backward and Adam kernels on windows
that the plain EM labels, then on held-out windows the EM started from the
proposal (where it wins the likelihood test against the bootstrap's state) is
compared with the EM started from the bootstrap, both capped at the same two
iterations, by pose error against the synthetic ground truth.  A small split
of the CPU-sized workload (T=5, 160x120) keeps it to seconds."""
import math

import numpy as np
import pytest

import synthflow

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

T, H, W = 5, 120, 160
N_TRAIN, N_EVAL, BATCH = 96, 48, 8
PLAIN_ITERS, SHORT_ITERS, GROUPS = 4, 2, 256


def _he_params(seed):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(6):
        ci, co = 32, (16 if k == 5 else 32)
        ci_real = 2 * T if k == 0 else ci
        co_real = 1 + T if k == 5 else co
        w = np.zeros((3, 3, ci, co), np.float32)
        w[:, :, :ci_real, :co_real] = rng.normal(0.0, math.sqrt(2.0 / (9 * ci_real)), (3, 3, ci_real, co_real))
        out += [w.ravel(), np.zeros(co, np.float32)]
    return np.concatenate(out)


def _pose_error(poses, gt):
    rot, tdir = [], []
    for k, (R, t) in enumerate(gt):
        Re, te = poses[k, :9].reshape(3, 3), poses[k, 9:]
        rot.append(math.acos(max(-1.0, min(1.0, (np.trace(Re @ R.T) - 1) / 2))))
        tdir.append(math.acos(max(-1.0, min(1.0, te @ t / (np.linalg.norm(te) * np.linalg.norm(t))))))
    return float(np.mean(rot)), float(np.mean(tdir))


@pytest.mark.timeout(600)
def test_trained_proposal_beats_the_bootstrap_at_two_iterations():
    import torch

    import paper_2104_06789_amd as vo
    train = [synthflow.make_window("small", 7000 + i) for i in range(N_TRAIN)]
    held = [synthflow.make_window("small", 9000 + i) for i in range(N_EVAL)]
    dev = torch.device("cuda")
    stream = torch.cuda.Stream()

    def solve(wins, iters, props=None):
        p = vo.default_params(n_iters=iters, n_pose_groups=GROUPS)
        flows = [torch.from_numpy(w["flows"]).to(dev) for w in wins]
        outs = [vo.Batch.outputs(T, H, W) for _ in wins]
        st = torch.full((len(wins),), -1, dtype=torch.int32, device=dev)
        ch = torch.full((len(wins),), -1, dtype=torch.int32, device=dev)
        items = [(f, w["K"], o) if props is None else (f, w["K"], o, (props[0][k], props[1][k], ch[k:k + 1]))
                 for k, (f, w, o) in enumerate(zip(flows, wins, outs))]
        b = vo.Batch(4, T, H, W, GROUPS)
        with torch.cuda.stream(stream):
            b.solve(items, p, st, stream=stream)
        torch.cuda.synchronize()
        b.close()
        assert all(int(x) == 0 for x in st.cpu().tolist())
        return outs, ch.cpu().numpy()

    labels, _ = solve(train, PLAIN_ITERS)
    net = vo.Net(T, BATCH, H, W)
    net.set_params(_he_params(0))
    tflows = torch.stack([torch.from_numpy(w["flows"]) for w in train]).to(dev)
    tdepth = torch.stack([o[1] for o in labels]).contiguous()
    trig = torch.stack([o[2] for o in labels]).contiguous()
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    rng = np.random.default_rng(0)
    losses = []
    for ep in range(40):
        order = rng.permutation(N_TRAIN)
        el = []
        for i in range(0, N_TRAIN - BATCH + 1, BATCH):
            idx = torch.from_numpy(order[i:i + BATCH]).to(dev)
            net.train_step(tflows[idx].contiguous(), tdepth[idx].contiguous(), trig[idx].contiguous(), 2e-3,
                           loss=loss)
            el.append(float(loss))
        losses.append(float(np.mean(el)))
    print("training loss by epoch", [round(x, 4) for x in losses[::5]], losses[-1])
    assert losses[-1] < 0.5 * losses[0]

    hflows = torch.stack([torch.from_numpy(w["flows"]) for w in held]).to(dev)
    pdepth = torch.empty((N_EVAL, H, W), device=dev)
    prig = torch.empty((N_EVAL, T, H, W), device=dev)
    for i in range(0, N_EVAL, BATCH):
        net.forward(hflows[i:i + BATCH].contiguous(), depth=pdepth[i:i + BATCH], rig=prig[i:i + BATCH])
    torch.cuda.synchronize()
    net.close()
    learned, choice = solve(held, SHORT_ITERS, props=(pdepth, prig))
    boot, _ = solve(held, SHORT_ITERS)
    plain, _ = solve(held, PLAIN_ITERS)
    e_l = np.array([_pose_error(o[0].cpu().numpy(), w["poses"]) for o, w in zip(learned, held)])
    e_b = np.array([_pose_error(o[0].cpu().numpy(), w["poses"]) for o, w in zip(boot, held)])
    e_p = np.array([_pose_error(o[0].cpu().numpy(), w["poses"]) for o, w in zip(plain, held)])
    used = float(np.mean(choice == 1))
    print(f"proposal used in {used:.2f} of the held-out windows")
    print("mean rotation / translation-direction error (rad): proposal + 2 it", e_l.mean(axis=0),
          "bootstrap + 2 it", e_b.mean(axis=0), "plain 4 it", e_p.mean(axis=0))
    assert used > 0.0
    # where it is used the proposal helps, and over all windows the start from
    # the proposal is no worse than the bootstrap's at the same iteration count
    sel = choice == 1
    print("on the windows that use it:", e_l[sel].mean(axis=0), "vs", e_b[sel].mean(axis=0))
    assert e_l[sel].mean(axis=0).sum() < e_b[sel].mean(axis=0).sum()
    assert e_l.mean(axis=0)[0] <= e_b.mean(axis=0)[0] * 1.02 and e_l.mean(axis=0)[1] <= e_b.mean(axis=0)[1] * 1.02
