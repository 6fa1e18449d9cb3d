"""ctypes wrapper of the FP64 CPU oracle (``voldor_oracle.c``).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(``paper_2104_06789_amd``) never imports, links or runs it.

All arrays are numpy; depth/rigidness/poses come back as float64.  Poses are
12-vectors: row-major R (9) followed by t (3), with P_cam = R P + t.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "voldor_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

DEFAULTS = dict(
    n_iters=3, sweeps_per_iter=4, n_pose_groups=256, n_seeds=64, ms_max_iters=100,
    lmeds_hypotheses=512, lmeds_eval_pixels=16384, ms_tol=1e-5,
    a1=0.01, a2=0.09, b1=-0.0022, b2=1.0, lam=0.15, gamma=0.9,
    sigma2_trans=0.1, sigma2_rot=0.004, beta_min=0.01, x_floor=1e-12,
    depth_lo=0.0, depth_hi=0.0, seed=0, criterion=0, pose_start=0, residual_model=0,
)


class Params(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("n_iters", C.c_int32), ("sweeps_per_iter", C.c_int32),
        ("n_pose_groups", C.c_int32), ("n_seeds", C.c_int32), ("ms_max_iters", C.c_int32),
        ("lmeds_hypotheses", C.c_int32), ("lmeds_eval_pixels", C.c_int32),
        ("ms_tol", C.c_double), ("a1", C.c_double), ("a2", C.c_double), ("b1", C.c_double),
        ("b2", C.c_double), ("lam", C.c_double), ("gamma", C.c_double),
        ("sigma2_trans", C.c_double), ("sigma2_rot", C.c_double), ("beta_min", C.c_double),
        ("x_floor", C.c_double), ("depth_lo", C.c_double), ("depth_hi", C.c_double),
        ("seed", C.c_uint64), ("criterion", C.c_int32), ("pose_start", C.c_int32),
        ("residual_model", C.c_int32), ("pad", C.c_int32),
    ]


def build(force=False):
    """Compile the oracle with gcc -O2 (no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-Wall",
                               "-Wno-unused-function", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        d, i, u8, i8, f = (C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_uint8),
                           C.POINTER(C.c_int8), C.POINTER(C.c_float))
        P = C.POINTER(Params)
        u64p = C.POINTER(C.c_uint64)
        sig = {
            "or_params_size": (C.c_int, []),
            "or_philox4x64": (None, [u64p, u64p, u64p]),
            "or_depth_sample": (C.c_double, [C.c_uint64, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_double,
                                             C.c_double]),
            "or_fisk_logpdf": (C.c_double, [C.c_double, C.c_double, C.c_double]),
            "or_gauss_logpdf": (C.c_double, [C.c_double, C.c_double]),
            "or_sym_eig": (None, [i, d, d, d]),
            "or_svd3": (None, [d, d, d, d]),
            "or_se3_exp": (None, [d, d, d]),
            "or_se3_log": (None, [d, d, d]),
            "or_emission_map": (None, [d, f, i, i, i, d, P, d, d, d, d, d, u8]),
            "or_fb_chain": (None, [d, i, C.c_double, d]),
            "or_fb_map": (None, [d, i, i, i, i, C.c_double, d]),
            "or_sweep": (None, [d, d, f, i, i, i, d, P, d, C.c_double, C.c_double, C.c_int64, i, d, i8]),
            "or_sweep_check": (None, [d, d, f, i, i, i, d, P, d, C.c_double, C.c_double, C.c_int64,
                                      i, C.c_double, C.c_double, i8, d]),
            "or_p3p": (C.c_int, [d, d, d, d]),
            "or_kde": (C.c_double, [d, d, i, d, C.c_double, C.c_double]),
            "or_depth_score": (C.c_double, [d, f, i, i, i, d, P, d, i, i, C.c_double]),
            "or_meanshift": (C.c_int, [d, d, i, d, C.c_double, C.c_double, C.c_double, i, d]),
            "or_pose_step": (C.c_int, [d, d, f, i, i, i, d, P, d, i, i, d, d, d, C.POINTER(C.c_int)]),
            "or_pose_step_scores": (C.c_int, [d, d, f, i, i, i, d, P, d, i, i, d, d, d, C.POINTER(C.c_int)]),
            "or_bootstrap": (C.c_int, [f, i, i, i, d, P, d, d, d, d]),
            "or_window": (C.c_int, [f, i, i, i, d, P, d, d, d, d, d]),
            "or_window_seeded": (C.c_int, [f, i, i, i, d, P, d, d, d, d, d, d]),
            "or_bootstrap_seeded": (C.c_int, [f, i, i, i, d, P, d, d, d, d]),
            "or_window_init": (C.c_int, [f, i, i, i, d, P, d, d, d, d, d, d, d, C.POINTER(C.c_int)]),
            "or_lookup": (C.c_int, [f, i, i, i, i, C.c_double, C.c_double, d]),
            "or_null_vector_8x9": (None, [d, d]),
            "or_set_f32_range": (None, [i]),
            "or_window_from_state": (C.c_int, [f, i, i, i, d, P, i, d, d, d, d, d, d, d, d]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        assert L.or_params_size() == C.sizeof(Params)
        _lib = L
    return _lib


def params(**kw):
    v = dict(DEFAULTS)
    for k, val in kw.items():
        if k not in v:
            raise KeyError(k)
        v[k] = val
    p = Params()
    p.struct_size = C.sizeof(Params)
    for k, val in v.items():
        setattr(p, k, val)
    return p


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, ct=C.c_double):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


def _flows(f):
    f = np.ascontiguousarray(f, dtype=np.float32)
    assert f.ndim == 4 and f.shape[3] == 2
    return f


# ---------------------------------------------------------------------------
def philox(ctr, key):
    c = np.array(ctr, dtype=np.uint64)
    k = np.array(key, dtype=np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64(_ptr(c, C.c_uint64), _ptr(k, C.c_uint64), _ptr(o, C.c_uint64))
    return o


def depth_sample(seed, global_sweep, direction, x, y, d_lo, d_hi):
    return lib().or_depth_sample(seed, global_sweep, direction, x, y, d_lo, d_hi)


def fisk_logpdf(x, log_alpha, beta):
    return lib().or_fisk_logpdf(float(x), float(log_alpha), float(beta))


def gauss_logpdf(x, log_alpha):
    """Log density of the squared EPE under the Gaussian residual model: the
    exponential with mean s = alpha / ln 2 (the Fisk's median alpha)."""
    return lib().or_gauss_logpdf(float(x), float(log_alpha))


def sym_eig(A):
    A = _d(A)
    n = A.shape[0]
    w = np.zeros(n)
    V = np.zeros((n, n))
    lib().or_sym_eig(n, _ptr(A), _ptr(w), _ptr(V))
    return w, V


def null_vector_8x9(A):
    A = _d(A)
    e = np.zeros(9)
    lib().or_null_vector_8x9(_ptr(A), _ptr(e))
    return e


def svd3(A):
    A = _d(A)
    U, S, V = np.zeros((3, 3)), np.zeros(3), np.zeros((3, 3))
    lib().or_svd3(_ptr(A), _ptr(U), _ptr(S), _ptr(V))
    return U, S, V


def se3_exp(p):
    p = _d(p)
    R, t = np.zeros((3, 3)), np.zeros(3)
    lib().or_se3_exp(_ptr(p), _ptr(R), _ptr(t))
    return R, t


def se3_log(R, t):
    R, t = _d(R), _d(t)
    p = np.zeros(6)
    lib().or_se3_log(_ptr(R), _ptr(t), _ptr(p))
    return p


def cumulative(rel):
    """M_0..M_T (T+1, 12) from relative poses (T, 12)."""
    rel = np.asarray(rel, dtype=np.float64).reshape(-1, 12)
    M = [np.concatenate([np.eye(3).ravel(), np.zeros(3)])]
    for r in rel:
        R, t = r[:9].reshape(3, 3), r[9:]
        Rm, tm = M[-1][:9].reshape(3, 3), M[-1][9:]
        M.append(np.concatenate([(R @ Rm).ravel(), R @ tm + t]))
    return np.array(M)


class f32_range:
    """Context: the posterior r below the smallest normal FP32 number is 0
    inside it (a test hook of the oracle; see or_set_f32_range), so that the
    depth M-step's argmax is taken with the posterior in FP32's range."""

    def __enter__(self):
        lib().or_set_f32_range(1)
        return self

    def __exit__(self, *exc):
        lib().or_set_f32_range(0)


def emission_map(theta, flows, K, p, M):
    flows = _flows(flows)
    T, H, W, _ = flows.shape
    theta, K, M = _d(theta), _d(K), _d(M)
    r, ell, lr, lm = (np.zeros((T, H, W)) for _ in range(4))
    obs = np.zeros((T, H, W), np.uint8)
    lib().or_emission_map(_ptr(theta), _ptr(flows, C.c_float), T, H, W, _ptr(K), C.byref(p), _ptr(M),
                          _ptr(r), _ptr(ell), _ptr(lr), _ptr(lm), _ptr(obs, C.c_uint8))
    return r, ell, lr, lm, obs.astype(bool)


def lookup(flows, t, px, py):
    flows = _flows(flows)
    T, H, W, _ = flows.shape
    out = np.zeros(2)
    ok = lib().or_lookup(_ptr(flows, C.c_float), T, H, W, t, px, py, _ptr(out))
    return (out if ok else None)


def fb_chain(r, gamma):
    r = _d(r)
    q = np.zeros_like(r)
    lib().or_fb_chain(_ptr(r), len(r), gamma, _ptr(q))
    return q


def fb_map(r, direction, gamma):
    r = _d(r)
    T, H, W = r.shape
    q = np.zeros_like(r)
    lib().or_fb_map(_ptr(r), T, H, W, direction, gamma, _ptr(q))
    return q


def depth_score(q, flows, K, p, M, x, y, theta):
    """Depth M-step objective sum_t term_t at pixel (x, y) for candidate depth
    theta, q [T][H][W] (criterion from p: 0 MIE, 1 MLE)."""
    flows = _flows(flows)
    T, H, W, _ = flows.shape
    return lib().or_depth_score(_ptr(_d(q)), _ptr(flows, C.c_float), T, H, W, _ptr(_d(K)), C.byref(p),
                                _ptr(_d(M)), x, y, theta)


def sweep(theta, flows, K, p, M, d_lo, d_hi, global_sweep, direction):
    flows = _flows(flows)
    T, H, W, _ = flows.shape
    th = _d(theta).copy()
    out = np.zeros_like(th)
    q = np.zeros((T, H, W))
    ch = np.zeros((H, W), np.int8)
    lib().or_sweep(_ptr(th), _ptr(out), _ptr(flows, C.c_float), T, H, W, _ptr(_d(K)), C.byref(p),
                   _ptr(_d(M)), d_lo, d_hi, global_sweep, direction, _ptr(q), _ptr(ch, C.c_int8))
    return out, q, ch


def sweep_check(theta_in, theta_cand, flows, K, p, M, d_lo, d_hi, global_sweep, direction,
                vtol=2e-6, stol=1e-5):
    flows = _flows(flows)
    T, H, W, _ = flows.shape
    a, b = _d(theta_in), _d(theta_cand)
    st = np.zeros((H, W), np.int8)
    gap = np.zeros((H, W))
    lib().or_sweep_check(_ptr(a), _ptr(b), _ptr(flows, C.c_float), T, H, W, _ptr(_d(K)), C.byref(p),
                         _ptr(_d(M)), d_lo, d_hi, global_sweep, direction, vtol, stol,
                         _ptr(st, C.c_int8), _ptr(gap))
    return st, gap


def p3p(Pw, f):
    Pw, f = _d(Pw), _d(f)
    Rs, ts = np.zeros((4, 3, 3)), np.zeros((4, 3))
    n = lib().or_p3p(_ptr(Pw), _ptr(f), _ptr(Rs), _ptr(ts))
    return [(Rs[i], ts[i]) for i in range(n)]


def kde(samples, w, at, s2t, s2r):
    s, w, at = _d(samples), _d(w), _d(at)
    return lib().or_kde(_ptr(s), _ptr(w), len(w), _ptr(at), s2t, s2r)


def meanshift(samples, w, start, s2t, s2r, tol=1e-12, max_iters=1000):
    s, w, st = _d(samples), _d(w), _d(start)
    out = np.zeros(6)
    it = lib().or_meanshift(_ptr(s), _ptr(w), len(w), _ptr(st), s2t, s2r, tol, max_iters, _ptr(out))
    return out, it


def pose_step(theta, Wmap, flows, K, p, M, t, it, prevT=None, want_samples=False):
    flows = _flows(flows)
    T, H, W, _ = flows.shape
    out = np.zeros(12)
    S = p.n_pose_groups
    samples = np.zeros((4 * S, 8)) if want_samples else None
    diag = (C.c_int * 4)()
    Wm = _d(Wmap) if Wmap is not None else None
    pv = _d(prevT) if prevT is not None else None
    lib().or_pose_step(_ptr(_d(theta)), _ptr(Wm), _ptr(flows, C.c_float), T, H, W, _ptr(_d(K)),
                       C.byref(p), _ptr(_d(M)), t, it, _ptr(pv), _ptr(out), _ptr(samples), diag)
    return out, samples, list(diag)


def pose_scores(theta, Wmap, flows, K, p, M, t, it, prevT=None):
    """All-pixel scores of the pose-step candidates: ([0] previous pose or -inf,
    [1..n] valid samples in (group, root) order) and the step's T_t."""
    flows = _flows(flows)
    T, H, W, _ = flows.shape
    out = np.zeros(12)
    sc = np.zeros(1 + 4 * p.n_pose_groups)
    n = C.c_int(0)
    Wm = _d(Wmap) if Wmap is not None else None
    pv = _d(prevT) if prevT is not None else None
    lib().or_pose_step_scores(_ptr(_d(theta)), _ptr(Wm), _ptr(flows, C.c_float), T, H, W, _ptr(_d(K)),
                              C.byref(p), _ptr(_d(M)), t, it, _ptr(pv), _ptr(out), _ptr(sc), C.byref(n))
    return sc[:n.value], out


def bootstrap(flows, K, p):
    flows = _flows(flows)
    T, H, W, _ = flows.shape
    rel = np.zeros(12)
    th = np.zeros((H, W))
    rng = np.zeros(2)
    info = np.zeros(4)
    st = lib().or_bootstrap(_ptr(flows, C.c_float), T, H, W, _ptr(_d(K)), C.byref(p), _ptr(rel),
                            _ptr(th), _ptr(rng), _ptr(info))
    return st, rel, th, rng, info


def window(flows, K, p):
    """Returns (status, poses [T,12], depth [H,W], rigidness [T,H,W], (L, L1 mass), diag[8])."""
    flows = _flows(flows)
    T, H, W, _ = flows.shape
    poses = np.zeros((T, 12))
    depth = np.zeros((H, W))
    rig = np.zeros((T, H, W))
    ll = np.zeros(2)
    diag = np.zeros(8)
    st = lib().or_window(_ptr(flows, C.c_float), T, H, W, _ptr(_d(K)), C.byref(p), _ptr(poses),
                         _ptr(depth), _ptr(rig), _ptr(ll), _ptr(diag))
    return st, poses, depth, rig, (ll[0], ll[1]), diag


def window_seeded(flows, K, p, T1):
    """One window whose T_1 is given (12 values, R row-major then t); returns
    (status, poses, depth, rigidness, loglik, diag) like window()."""
    flows = _flows(flows)
    T, H, W, _ = flows.shape
    poses = np.zeros((T, 12))
    depth = np.zeros((H, W))
    rig = np.zeros((T, H, W))
    ll = np.zeros(2)
    diag = np.zeros(8)
    st = lib().or_window_seeded(_ptr(flows, C.c_float), T, H, W, _ptr(_d(K)), C.byref(p), _ptr(_d(T1)),
                                _ptr(poses), _ptr(depth), _ptr(rig), _ptr(ll), _ptr(diag))
    return st, poses, depth, rig, ll, diag


def bootstrap_seeded(flows, K, p, T1):
    """The bootstrap with T_1 given: (status, relT [12], theta [H][W], range [2])."""
    flows = _flows(flows)
    T, H, W, _ = flows.shape
    rel = np.zeros(12)
    th = np.zeros((H, W))
    rng = np.zeros(2)
    st = lib().or_bootstrap_seeded(_ptr(flows, C.c_float), T, H, W, _ptr(_d(K)), C.byref(p), _ptr(_d(T1)),
                                   _ptr(rel), _ptr(th), _ptr(rng))
    return st, rel, th, rng


def window_starts(N, T, stride):
    """First frames of the windows over N flows: 0, stride, 2 stride, ... and a
    last window ending at flow N."""
    s, out = 0, [0]
    while s + T < N:
        s = min(s + stride, N - T)
        out.append(s)
    return out


def vo_sequence(flows, K, p, T, stride):
    """Sliding-window visual odometry over N flows X_1..X_N (Sec. 5.3): windows
    of T flows start every `stride` frames; the first is bootstrapped from X_1,
    every later one takes T_1 from the previous window's estimate of the same
    frame pair.  Each window fixes its own scale by |t_1| = 1; the trajectory
    chains them: the scale of window i relative to window i - 1 is the length,
    in window i - 1's units, of the translation that window i normalised.
    Relative pose of frame pair (k, k + 1) comes from the latest window that
    starts at or before frame k.  Returns (status, M [N + 1][12] camera poses
    x_k = M_k x_0 in window 0's scale, per-window poses)."""
    flows = _flows(flows)
    N = flows.shape[0]
    if not (2 <= T <= N and 1 <= stride < T):
        raise ValueError("need 2 <= T <= N and 1 <= stride < T (the next T_1 must lie in the window)")
    starts = window_starts(N, T, stride)
    wposes = []
    for i, s in enumerate(starts):
        fl = flows[s:s + T]
        if i == 0:
            st, poses, *_ = window(fl, K, p)
        else:
            prev = wposes[-1]
            st, poses, *_ = window_seeded(fl, K, p, prev[s - starts[i - 1]])
        if st != 0:
            return st, None, wposes
        wposes.append(poses)
    return 0, vo_chain(wposes, starts, N), wposes


def vo_chain(wposes, starts, N):
    """The trajectory M [N + 1][12] of a sequence from its windows' relative
    poses (each window in its own gauge |t_1| = 1), as in vo_sequence."""
    scale = [1.0]
    for i in range(1, len(starts)):
        scale.append(scale[-1] * np.linalg.norm(np.asarray(wposes[i - 1])[starts[i] - starts[i - 1]][9:]))
    M = [np.concatenate([np.eye(3).ravel(), np.zeros(3)])]
    for k in range(N):
        i = max(j for j, s in enumerate(starts) if s <= k)
        r = np.asarray(wposes[i])[k - starts[i]]
        R, t = r[:9].reshape(3, 3), r[9:] * scale[i]
        Rm, tm = M[-1][:9].reshape(3, 3), M[-1][9:]
        M.append(np.concatenate([(R @ Rm).ravel(), R @ tm + t]))
    return np.array(M)


def window_init(flows, K, p, init_depth, init_rig):
    """window() from a proposed initial state (depth [H,W] > 0, rigidness [T,H,W]),
    used where it explains X_1 better than the bootstrap.  Returns
    (status, poses, depth, rigidness, (L, L1 mass), diag, choice)."""
    flows = _flows(flows)
    T, H, W, _ = flows.shape
    poses = np.zeros((T, 12))
    depth = np.zeros((H, W))
    rig = np.zeros((T, H, W))
    ll = np.zeros(2)
    diag = np.zeros(8)
    choice = C.c_int(-1)
    st = lib().or_window_init(_ptr(flows, C.c_float), T, H, W, _ptr(_d(K)), C.byref(p), _ptr(_d(init_depth)),
                              _ptr(_d(init_rig)), _ptr(poses), _ptr(depth), _ptr(rig), _ptr(ll), _ptr(diag),
                              C.byref(choice))
    return st, poses, depth, rig, (ll[0], ll[1]), diag, choice.value


def window_from_state(flows, K, p, it0, rel, depth, rig, rng):
    """The iterations it0 .. n_iters - 1 from a given start-of-iteration state
    (relative poses [T,12] in the gauge |t_1| = 1, depth [H,W], the previous
    iteration's rigidness [T,H,W], depth range [2]); returns (status, poses,
    depth, rigidness, (L, L1 mass)) like window()."""
    flows = _flows(flows)
    T, H, W, _ = flows.shape
    poses = np.zeros((T, 12))
    dout = np.zeros((H, W))
    rout = np.zeros((T, H, W))
    ll = np.zeros(2)
    st = lib().or_window_from_state(_ptr(flows, C.c_float), T, H, W, _ptr(_d(K)), C.byref(p), int(it0),
                                    _ptr(_d(rel)), _ptr(_d(depth)), _ptr(_d(rig)), _ptr(_d(rng)), _ptr(poses),
                                    _ptr(dout), _ptr(rout), _ptr(ll))
    return st, poses, dout, rout, (ll[0], ll[1])
