"""MI355X (gfx950) window solver of VOLDOR (Min, Yang, Dunn, CVPR 2020).

Thin ctypes binding of ``libvoldor.so`` (C ABI in ``include/voldor.h``).  The
binding only marshals arguments: every step of the solver runs in the HIP
kernels of the library.  PyTorch provides device memory and streams.  If the
library has not been built, importing the native layer raises.
"""
from __future__ import annotations

import ctypes as C
import os
import sys as _sys

import numpy as np

__all__ = ["Params", "WindowDesc", "default_params", "Solver", "Batch", "Net", "philox", "lib", "status_str",
           "VoldorError"]

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libvoldor.so")

OK, EINVAL, ENOMEM, EDEVICE, EDEGENERATE = 0, -1, -2, -3, -4


class VoldorError(RuntimeError):
    def __init__(self, code, what=""):
        super().__init__(f"{what}: {status_str(code)} ({code})")
        self.code = code


class Params(C.Structure):
    """Mirror of voldor_params (include/voldor.h)."""
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


CRITERION_MIE, CRITERION_MLE = 0, 1
RESIDUAL_FISK, RESIDUAL_GAUSS = 0, 1


class WindowDesc(C.Structure):
    """Mirror of voldor_window_desc (include/voldor.h)."""
    _fields_ = [
        ("flows", C.c_void_p), ("T", C.c_int32), ("H", C.c_int32), ("W", C.c_int32),
        ("K", C.c_double * 4), ("poses", C.c_void_p), ("depth", C.c_void_p),
        ("rigidness", C.c_void_p), ("loglik", C.c_void_p),
        ("init_depth", C.c_void_p), ("init_rig", C.c_void_p), ("choice", C.c_void_p),
        ("n_pose_groups", C.c_int32), ("pad", C.c_int32),
    ]


BATCH_GRAPH = 1
BATCH_LOCKSTEP = 2

_lib = None


def lib():
    """Load libvoldor.so; raises if it was not built (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"HIP library not built: {_LIB_PATH} (run __graft_entry__.build())")
    L = C.CDLL(_LIB_PATH)
    vp, i, d, f = C.c_void_p, C.c_int, C.c_double, C.c_float
    P = C.POINTER(Params)
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int)
    sig = {
        "voldor_params_default": (None, [P]),
        "voldor_status_str": (C.c_char_p, [i]),
        "voldor_create": (i, [C.POINTER(vp), i, i, i, i]),
        "voldor_destroy": (None, [vp]),
        "voldor_window": (i, [vp, vp, i, i, i, dp, P, vp, vp, vp, vp, vp]),
        "voldor_window_async": (i, [vp, vp, i, i, i, dp, P, vp, vp, vp, vp, vp, vp]),
        "voldor_window_init": (i, [vp, vp, i, i, i, dp, P, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "voldor_philox": (i, [vp, C.c_uint64, C.c_uint64, vp, i, vp]),
        "voldor_emission": (i, [vp, vp, vp, i, i, i, dp, P, dp, vp, vp, vp, vp, vp]),
        "voldor_sweep": (i, [vp, vp, vp, vp, i, i, i, dp, P, dp, d, d, C.c_int64, i, vp, vp]),
        "voldor_pose_step": (i, [vp, vp, vp, vp, i, i, i, dp, P, dp, i, i, dp, dp, vp, ip, vp]),
        "voldor_pose_scores": (i, [vp, dp, i, ip]),
        "voldor_last_range": (i, [vp, dp]),
        "voldor_window_seeded": (i, [vp, vp, i, i, i, dp, P, vp, vp, vp, vp, vp, vp, vp]),
        "voldor_vo_windows": (i, [i, i, i]),
        "voldor_set_sweep_threads": (i, [vp, i, i]),
        "voldor_get_sweep_threads": (i, [vp, ip, ip]),
        "voldor_set_sweep_lookahead": (i, [vp, i, i]),
        "voldor_get_sweep_lookahead": (i, [vp, ip, ip]),
        "voldor_autotune": (i, [vp, vp, i, i, i, dp, P, ip, ip, vp]),
        "voldor_batch_set_sweep_threads": (i, [vp, i, i]),
        "voldor_batch_set_sweep_lookahead": (i, [vp, i, i]),
        "voldor_batch_autotune": (i, [vp, C.POINTER(WindowDesc), i, P, vp]),
        "voldor_batch_set_timing": (i, [vp, i]),
        "voldor_batch_timing_summary": (i, [vp, dp, ip]),
        "voldor_sweep_tuning": (i, [vp, ip, i]),
        "voldor_residual_fit": (i, [vp, vp, C.c_int64, i, C.c_double, C.c_double, i, dp, dp, vp]),
        "voldor_residual_workspace": (C.c_int64, [C.c_int64, i]),
        "voldor_residual_bins": (i, [vp, vp, C.c_int64, i, C.c_double, C.c_double, vp, vp, vp]),
        "voldor_residual_bins_noalloc": (i, [vp, vp, C.c_int64, i, C.c_double, C.c_double, vp, vp]),
        "voldor_vo_sequence": (i, [vp, vp, i, i, i, dp, P, i, i, vp, vp, vp, vp, vp, vp]),
        "voldor_bootstrap": (i, [vp, vp, i, i, i, dp, P, dp, vp, dp, dp, vp]),
        "voldor_set_timing": (i, [vp, i]),
        "voldor_last_timing": (i, [vp, dp]),
        "voldor_timing_summary": (i, [vp, dp, ip]),
        "voldor_net_create": (i, [C.POINTER(vp), i, i, i, i]),
        "voldor_net_destroy": (None, [vp]),
        "voldor_net_param_count": (i, [vp]),
        "voldor_net_set_params": (i, [vp, C.POINTER(f)]),
        "voldor_net_get_params": (i, [vp, C.POINTER(f)]),
        "voldor_net_forward": (i, [vp, vp, i, i, i, vp, vp, vp, vp]),
        "voldor_net_gradient": (i, [vp, vp, i, i, i, vp, vp, vp, vp, vp]),
        "voldor_net_train_step": (i, [vp, vp, i, i, i, vp, vp, f, vp, vp]),
        "voldor_net_layer": (i, [vp, i, i, vp, vp, vp, i, i, i, vp]),
        "voldor_batch_create": (i, [C.POINTER(vp), i, i, i, i, i, i]),
        "voldor_batch_destroy": (None, [vp]),
        "voldor_window_batch": (i, [vp, C.POINTER(WindowDesc), i, P, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def status_str(code):
    try:
        return lib().voldor_status_str(int(code)).decode()
    except RuntimeError:
        return str(code)


def default_params(**kw):
    p = Params()
    lib().voldor_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _dbl(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _check(code, what):
    if code != OK:
        raise VoldorError(code, what)


def _flows(flows):
    import torch
    if not (isinstance(flows, torch.Tensor) and flows.is_cuda and flows.dtype == torch.float32):
        raise TypeError("flows must be a float32 CUDA tensor [T,H,W,2]")
    if flows.dim() != 4 or flows.shape[3] != 2 or not flows.is_contiguous():
        raise ValueError("flows must be contiguous [T,H,W,2]")
    return flows


def _dev_tensor(t, name, dtype, shape, device, optional=False):
    """t must be a contiguous CUDA tensor of `dtype` and `shape` on `device`
    (None allowed when optional); raises before anything reaches the library."""
    import torch
    if t is None:
        if optional:
            return None
        raise TypeError(f"{name} is required")
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous CUDA {dtype} tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, not {tuple(t.shape)}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} must be on {device}")
    return t


def residual_fit(X, G, nbins=40, v_max=40.0, x_floor=1e-12, min_count=64, stream=None):
    """Fisk laws (a1, a2, b1, b2) of Eq. 6-7 fitted to the residuals |X - G|^2
    binned by |X| (CUDA float32 flows [..., 2]); returns (laws, bins [nbins][4])."""
    import torch
    X = X.to(torch.float32).contiguous()
    G = G.to(torch.float32).contiguous()
    if not (X.is_cuda and G.is_cuda and X.shape == G.shape and X.shape[-1] == 2):
        raise ValueError("X and G must be CUDA tensors of the same shape [..., 2]")
    laws = np.zeros(4)
    bins = np.zeros((nbins, 4))
    _check(lib().voldor_residual_fit(_ptr(X), _ptr(G), X.numel() // 2, nbins, v_max, x_floor, min_count,
                                     laws.ctypes.data_as(C.POINTER(C.c_double)),
                                     bins.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream)),
           "voldor_residual_fit")
    return laws, bins


def _flow_pair(X, G):
    """X and G: contiguous CUDA float32 tensors of one shape [..., 2]; returns n."""
    import torch
    for name, t in (("X", X), ("G", G)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous CUDA float32 tensor [..., 2]")
    if X.shape != G.shape or X.dim() < 1 or X.shape[-1] != 2 or X.numel() == 0:
        raise ValueError("X and G must have one shape [..., 2] with at least one item")
    if X.device != G.device:
        raise ValueError("X and G must be on one device")
    return X.numel() // 2


def _bins_out(out, nbins, device):
    import torch
    if out is None:
        return torch.empty((nbins, 4), dtype=torch.float64, device=device)
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
            and out.numel() >= 4 * nbins and out.device == device):
        raise TypeError("out must be a contiguous CUDA float64 tensor of nbins x 4 elements on the flows' device")
    return out


def residual_bins(X, G, nbins=40, v_max=40.0, x_floor=1e-12, work=None, out=None, stream=None):
    """The binning pass alone, enqueued: returns the CUDA float64 [nbins][4] bins."""
    import torch
    n = _flow_pair(X, G)
    need = int(lib().voldor_residual_workspace(n, nbins))
    _check(need if need < 0 else 0, "voldor_residual_workspace")
    if work is None:
        work = torch.empty(need, dtype=torch.float64, device=X.device)
    elif not (isinstance(work, torch.Tensor) and work.is_cuda and work.dtype == torch.float64
              and work.is_contiguous() and work.numel() >= need and work.device == X.device):
        raise TypeError(f"work must be a contiguous CUDA float64 tensor of at least {need} elements")
    out = _bins_out(out, nbins, X.device)
    _check(lib().voldor_residual_bins(_ptr(X), _ptr(G), n, nbins, v_max, x_floor, _ptr(work), _ptr(out),
                                      _stream(stream)), "voldor_residual_bins")
    return out


def residual_bins_noalloc(X, G, out, nbins=40, v_max=40.0, x_floor=1e-12, stream=None):
    """residual_bins without any device allocation (the library's static
    scratch): out is a preallocated CUDA float64 [nbins][4] tensor."""
    n = _flow_pair(X, G)
    out = _bins_out(out, nbins, X.device)
    _check(lib().voldor_residual_bins_noalloc(_ptr(X), _ptr(G), n, nbins, v_max, x_floor, _ptr(out),
                                              _stream(stream)), "voldor_residual_bins_noalloc")
    return out


class Solver:
    """A context of the HIP library sized for windows up to T_max x H_max x W_max."""

    def __init__(self, T_max, H_max, W_max, S_max=4096):
        import torch
        torch.cuda.init()
        self._ctx = C.c_void_p()
        _check(lib().voldor_create(C.byref(self._ctx), T_max, H_max, W_max, S_max), "voldor_create")
        self.T_max, self.H_max, self.W_max, self.S_max = T_max, H_max, W_max, S_max

    def close(self):
        """Free the context's device workspace (waits for its work)."""
        if self._ctx:
            lib().voldor_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self, _fin=_sys.is_finalizing):
        # at interpreter exit the HIP runtime may already be torn down: leave
        # the memory to the process's end instead of calling into it (the
        # check is bound here: module globals may be gone by then)
        if _fin():
            return
        try:
            self.close()
        except Exception:
            pass

    # -- whole window --------------------------------------------------------
    def window(self, flows, K, params, out=None, stream=None, want_loglik=True):
        """Solve one window.  Returns (poses [T,12] f64, depth [H,W] f32,
        rigidness [T,H,W] f32, loglik [2] f64 or None), all CUDA tensors."""
        import torch
        flows = _flows(flows)
        T, H, W, _ = flows.shape
        dev = flows.device
        if out is None:
            out = (torch.empty((T, 12), dtype=torch.float64, device=dev),
                   torch.empty((H, W), dtype=torch.float32, device=dev),
                   torch.empty((T, H, W), dtype=torch.float32, device=dev),
                   torch.empty(2, dtype=torch.float64, device=dev) if want_loglik else None)
        poses, depth, rig, ll = out
        Kd, Kp = _dbl(K)
        rc = lib().voldor_window(self._ctx, _ptr(flows), T, H, W, Kp, C.byref(params), _ptr(poses),
                                 _ptr(depth), _ptr(rig), _ptr(ll), _stream(stream))
        _check(rc, "voldor_window")
        return poses, depth, rig, ll

    def window_async(self, flows, K, params, out, status, stream=None, want_loglik=True):
        """Enqueue one window without waiting.  out = (poses, depth, rigidness,
        loglik or None) CUDA tensors as returned by window(); status: a CUDA
        int32 tensor element (e.g. statuses[i]) that receives the device status.
        The tensors must stay alive until the stream has run the window."""
        import torch
        flows = _flows(flows)
        T, H, W, _ = flows.shape
        if not (isinstance(status, torch.Tensor) and status.is_cuda and status.dtype == torch.int32):
            raise TypeError("status must be a CUDA int32 tensor element")
        poses, depth, rig, ll = out
        Kd, Kp = _dbl(K)
        rc = lib().voldor_window_async(self._ctx, _ptr(flows), T, H, W, Kp, C.byref(params), _ptr(poses),
                                       _ptr(depth), _ptr(rig), _ptr(ll) if want_loglik else None,
                                       _ptr(status), _stream(stream))
        _check(rc, "voldor_window_async")

    def window_init(self, flows, K, params, init_depth, init_rig, out, status, choice=None, stream=None,
                    want_loglik=True):
        """Enqueue a window that starts from a proposed depth [H,W] and rigidness
        [T,H,W] (CUDA float32) where they explain X_1 better than the bootstrap;
        choice: CUDA int32 element set to 1 when the proposal was used."""
        import torch
        flows = _flows(flows)
        T, H, W, _ = flows.shape
        _dev_tensor(init_depth, "init_depth", torch.float32, (H, W), flows.device)
        _dev_tensor(init_rig, "init_rig", torch.float32, (T, H, W), flows.device)
        _dev_tensor(status, "status", torch.int32, status.shape if isinstance(status, torch.Tensor) else (), flows.device)
        if status.numel() != 1:
            raise ValueError("status must be one CUDA int32 element")
        if choice is not None:
            _dev_tensor(choice, "choice", torch.int32, choice.shape, flows.device)
        poses, depth, rig, ll = out
        Kd, Kp = _dbl(K)
        _check(lib().voldor_window_init(self._ctx, _ptr(flows), T, H, W, Kp, C.byref(params), _ptr(init_depth),
                                        _ptr(init_rig), _ptr(poses), _ptr(depth), _ptr(rig),
                                        _ptr(ll) if want_loglik else None, _ptr(status), _ptr(choice),
                                        _stream(stream)), "voldor_window_init")

    def window_status(self, flows, K, params, stream=None):
        """Like window() but returns the status code instead of raising."""
        import torch
        flows = _flows(flows)
        T, H, W, _ = flows.shape
        dev = flows.device
        poses = torch.zeros((T, 12), dtype=torch.float64, device=dev)
        depth = torch.zeros((H, W), dtype=torch.float32, device=dev)
        rig = torch.zeros((T, H, W), dtype=torch.float32, device=dev)
        Kd, Kp = _dbl(K)
        return lib().voldor_window(self._ctx, _ptr(flows), T, H, W, Kp, C.byref(params), _ptr(poses),
                                   _ptr(depth), _ptr(rig), None, _stream(stream))

    def set_timing(self, enable=True):
        _check(lib().voldor_set_timing(self._ctx, 1 if enable else 0), "voldor_set_timing")

    def last_timing(self):
        """Milliseconds of the last window: bootstrap, pose, sweeps, sweep launches,
        rigidness+gauge, log-likelihood, whole window."""
        out = np.zeros(8)
        _check(lib().voldor_last_timing(self._ctx, out.ctypes.data_as(C.POINTER(C.c_double))),
               "voldor_last_timing")
        keys = ["bootstrap", "pose", "sweeps", "sweep_launches", "rigidness", "loglik", "window"]
        return dict(zip(keys, out[:7].tolist()))

    def timing_summary(self):
        """Wait for the last window's stream; mean phase milliseconds over the
        windows enqueued since the previous summary (the last 32 at most), and
        their number."""
        out = np.zeros(8)
        n = C.c_int(0)
        _check(lib().voldor_timing_summary(self._ctx, out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(n)),
               "voldor_timing_summary")
        keys = ["bootstrap", "pose", "sweeps", "sweep_launches", "rigidness", "loglik", "window"]
        return dict(zip(keys, out[:7].tolist())), n.value

    # -- single steps ---------------------------------------------------------
    def emission(self, theta, flows, K, params, M, stream=None):
        import torch
        flows = _flows(flows)
        T, H, W, _ = flows.shape
        outs = [torch.empty((T, H, W), dtype=torch.float32, device=flows.device) for _ in range(4)]
        Kd, Kp = _dbl(K)
        Md, Mp = _dbl(M)
        th = theta.to(torch.float32).contiguous()
        rc = lib().voldor_emission(self._ctx, _ptr(th), _ptr(flows), T, H, W, Kp, C.byref(params), Mp,
                                   *[_ptr(o) for o in outs], _stream(stream))
        _check(rc, "voldor_emission")
        return outs

    def sweep(self, theta, flows, K, params, M, d_lo, d_hi, global_sweep, direction, want_q=False,
              stream=None):
        import torch
        flows = _flows(flows)
        T, H, W, _ = flows.shape
        th = theta.to(torch.float32).contiguous()
        out = torch.empty_like(th)
        q = torch.empty((T, H, W), dtype=torch.float32, device=flows.device) if want_q else None
        Kd, Kp = _dbl(K)
        Md, Mp = _dbl(M)
        rc = lib().voldor_sweep(self._ctx, _ptr(th), _ptr(out), _ptr(flows), T, H, W, Kp, C.byref(params),
                                Mp, float(d_lo), float(d_hi), int(global_sweep), int(direction), _ptr(q),
                                _stream(stream))
        _check(rc, "voldor_sweep")
        return out, q

    def pose_step(self, theta, rig, flows, K, params, M, t, it, prevT=None, want_samples=False,
                  stream=None):
        import torch
        flows = _flows(flows)
        T, H, W, _ = flows.shape
        th = theta.to(torch.float32).contiguous()
        rg = rig.to(torch.float32).contiguous() if rig is not None else None
        samples = (torch.zeros((4 * params.n_pose_groups, 8), dtype=torch.float64, device=flows.device)
                   if want_samples else None)
        Kd, Kp = _dbl(K)
        Md, Mp = _dbl(M)
        Tout = np.zeros(12)
        diag = (C.c_int * 4)()
        if prevT is not None:
            pv, pp = _dbl(prevT)
        else:
            pv, pp = None, None
        rc = lib().voldor_pose_step(self._ctx, _ptr(th), _ptr(rg), _ptr(flows), T, H, W, Kp, C.byref(params),
                                    Mp, int(t), int(it), pp, Tout.ctypes.data_as(C.POINTER(C.c_double)),
                                    _ptr(samples), diag, _stream(stream))
        _check(rc, "voldor_pose_step")
        return Tout, samples, list(diag)

    def window_seeded(self, flows, K, params, T1, out, status, stream=None, want_loglik=True):
        """Enqueue one window whose T_1 is the CUDA float64 tensor T1 [12] (it may
        be a view of an earlier window's poses); out and status as window_async."""
        import torch
        flows = _flows(flows)
        T, H, W, _ = flows.shape
        if not (isinstance(T1, torch.Tensor) and T1.is_cuda and T1.dtype == torch.float64):
            raise TypeError("T1 must be a CUDA float64 tensor")
        poses, depth, rig, ll = out
        Kd, Kp = _dbl(K)
        _check(lib().voldor_window_seeded(self._ctx, _ptr(flows), T, H, W, Kp, C.byref(params), _ptr(T1),
                                          _ptr(poses), _ptr(depth), _ptr(rig), _ptr(ll) if want_loglik else None,
                                          _ptr(status), _stream(stream)), "voldor_window_seeded")

    def vo_sequence(self, flows, K, params, T, stride, stream=None):
        """Sliding-window VO over flows [N][H][W][2] (CUDA): returns (trajectory
        [N+1][12], per-window poses [windows][T][12], window statuses, last
        window's depth and rigidness) as CUDA tensors, enqueued without waiting."""
        import torch
        flows = _flows(flows)
        N, H, W, _ = flows.shape
        nwin = lib().voldor_vo_windows(N, T, stride)
        _check(nwin if nwin < 0 else 0, "voldor_vo_windows")
        dev = flows.device
        wposes = torch.empty((nwin, T, 12), dtype=torch.float64, device=dev)
        traj = torch.empty((N + 1, 12), dtype=torch.float64, device=dev)
        wstatus = torch.full((nwin,), -99, dtype=torch.int32, device=dev)
        depth = torch.empty((H, W), dtype=torch.float32, device=dev)
        rig = torch.empty((T, H, W), dtype=torch.float32, device=dev)
        Kd, Kp = _dbl(K)
        _check(lib().voldor_vo_sequence(self._ctx, _ptr(flows), N, H, W, Kp, C.byref(params), T, stride,
                                        _ptr(wposes), _ptr(depth), _ptr(rig), _ptr(wstatus), _ptr(traj),
                                        _stream(stream)), "voldor_vo_sequence")
        return traj, wposes, wstatus, depth, rig

    def set_sweep_threads(self, rows, cols):
        """Threads per chain of row and column sweeps (256, 512, 768, 1024; 0 = 512)."""
        _check(lib().voldor_set_sweep_threads(self._ctx, int(rows), int(cols)), "voldor_set_sweep_threads")

    def sweep_threads(self):
        r, c = C.c_int(0), C.c_int(0)
        _check(lib().voldor_get_sweep_threads(self._ctx, C.byref(r), C.byref(c)), "voldor_get_sweep_threads")
        return r.value, c.value

    def set_sweep_lookahead(self, rows, cols):
        """Look-ahead cap of the propagation rounds (0 = none), rows and columns."""
        _check(lib().voldor_set_sweep_lookahead(self._ctx, int(rows), int(cols)), "voldor_set_sweep_lookahead")

    def sweep_lookahead(self):
        r, c = C.c_int(0), C.c_int(0)
        _check(lib().voldor_get_sweep_lookahead(self._ctx, C.byref(r), C.byref(c)), "voldor_get_sweep_lookahead")
        return r.value, c.value

    def autotune(self, flows, K, params, stream=None):
        """Time every sweep width on this window's shape and keep the fastest;
        returns (row threads, column threads)."""
        flows = _flows(flows)
        T, H, W, _ = flows.shape
        Kd, Kp = _dbl(K)
        r, c = C.c_int(0), C.c_int(0)
        _check(lib().voldor_autotune(self._ctx, _ptr(flows), T, H, W, Kp, C.byref(params), C.byref(r), C.byref(c),
                                     _stream(stream)), "voldor_autotune")
        return r.value, c.value

    def sweep_tuning(self):
        """The tuned chain classes: [(chain length, T, threads, look-ahead cap)]."""
        buf = (C.c_int * 64)()
        n = lib().voldor_sweep_tuning(self._ctx, buf, 16)
        _check(n if n < 0 else 0, "voldor_sweep_tuning")
        return [tuple(buf[4 * i:4 * i + 4]) for i in range(n)]

    def last_range(self):
        """[d_lo, d_hi] of the last window on this context, in its output gauge."""
        out = np.zeros(2)
        _check(lib().voldor_last_range(self._ctx, out.ctypes.data_as(C.POINTER(C.c_double))), "voldor_last_range")
        return out

    def pose_scores(self):
        """All-pixel candidate scores of the last pose step run with pose_start=1:
        [0] the previous pose (-inf if none), [1..] the valid samples in (group,
        root) order."""
        buf = np.zeros(1 + 4 * 8192 + 64)
        n = C.c_int(0)
        _check(lib().voldor_pose_scores(self._ctx, buf.ctypes.data_as(C.POINTER(C.c_double)), buf.size,
                                        C.byref(n)), "voldor_pose_scores")
        return buf[:n.value].copy()

    def bootstrap(self, flows, K, params, stream=None):
        """Returns (status, relT [12], theta [H,W] CUDA f32, range [2], info [4])."""
        import torch
        flows = _flows(flows)
        T, H, W, _ = flows.shape
        theta = torch.empty((H, W), dtype=torch.float32, device=flows.device)
        rel, rng, info = np.zeros(12), np.zeros(2), np.zeros(4)
        Kd, Kp = _dbl(K)
        rc = lib().voldor_bootstrap(self._ctx, _ptr(flows), T, H, W, Kp, C.byref(params),
                                    rel.ctypes.data_as(C.POINTER(C.c_double)), _ptr(theta),
                                    rng.ctypes.data_as(C.POINTER(C.c_double)),
                                    info.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream))
        return rc, rel, theta, rng, info


def philox(ctr, key0, key1, stream=None):
    """Philox4x64-10 of a CUDA int64 tensor of counters [n,4] (bit patterns)."""
    import torch
    ctr = ctr.contiguous()
    out = torch.empty_like(ctr)
    _check(lib().voldor_philox(_ptr(ctr), int(key0), int(key1), _ptr(out), ctr.shape[0], _stream(stream)),
           "voldor_philox")
    return out


class Batch:
    """Batch solver over `lanes` concurrent streams (voldor_batch_* in the C ABI);
    each lane owns a workspace for windows up to T_max x H_max x W_max.
    lockstep: the windows of a lane advance together, one launch per kernel
    over all of them (VOLDOR_BATCH_LOCKSTEP)."""

    def __init__(self, lanes, T_max, H_max, W_max, S_max=4096, graph=False, lockstep=False):
        ctx = C.c_void_p()
        flags = (BATCH_GRAPH if graph else 0) | (BATCH_LOCKSTEP if lockstep else 0)
        _check(lib().voldor_batch_create(C.byref(ctx), lanes, T_max, H_max, W_max, S_max, flags),
               "voldor_batch_create")
        self._b = ctx
        self._keep = None

    def close(self):
        """Free the lanes' streams and workspaces (waits for their work)."""
        if getattr(self, "_b", None):
            lib().voldor_batch_destroy(self._b)
            self._b = None
        self._keep = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self, _fin=_sys.is_finalizing):
        if _fin():   # as Solver.__del__
            return
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def outputs(T, H, W, device="cuda"):
        """Output tensors (poses, depth, rigidness, loglik) for one window."""
        import torch
        return (torch.empty((T, 12), dtype=torch.float64, device=device),
                torch.empty((H, W), dtype=torch.float32, device=device),
                torch.empty((T, H, W), dtype=torch.float32, device=device),
                torch.empty(2, dtype=torch.float64, device=device))

    def set_sweep_threads(self, rows, cols):
        """Sweep widths of every lane (as Solver.set_sweep_threads)."""
        _check(lib().voldor_batch_set_sweep_threads(self._b, int(rows), int(cols)), "voldor_batch_set_sweep_threads")

    def set_sweep_lookahead(self, rows, cols):
        """Look-ahead caps of every lane (as Solver.set_sweep_lookahead)."""
        _check(lib().voldor_batch_set_sweep_lookahead(self._b, int(rows), int(cols)),
               "voldor_batch_set_sweep_lookahead")

    @staticmethod
    def _descs(windows):
        n = len(windows)
        descs = (WindowDesc * n)()
        for i, item in enumerate(windows):
            flows, K, out = item[:3]
            init = item[3] if len(item) > 3 else None
            groups = item[4] if len(item) > 4 else 0
            flows = _flows(flows)
            T, H, W, _ = flows.shape
            poses, depth, rig, ll = out
            d = descs[i]
            d.flows = flows.data_ptr()
            d.T, d.H, d.W = T, H, W
            for k in range(4):
                d.K[k] = float(K[k])
            d.poses, d.depth, d.rigidness = poses.data_ptr(), depth.data_ptr(), rig.data_ptr()
            d.loglik = ll.data_ptr() if ll is not None else None
            if init is not None:
                idepth, irig, choice = init
                d.init_depth, d.init_rig = idepth.data_ptr(), irig.data_ptr()
                d.choice = choice.data_ptr() if choice is not None else None
            d.n_pose_groups = int(groups)
        return descs

    def set_timing(self, enable=True):
        _check(lib().voldor_batch_set_timing(self._b, 1 if enable else 0), "voldor_batch_set_timing")

    def timing_summary(self):
        """Phase milliseconds summed over the recorded windows of every lane
        (bootstrap, pose, sweeps, sweep launches, rigidness, loglik, window),
        the milliseconds during which any lane ran sweeps (sweeps_busy), and
        the number of windows."""
        out = np.zeros(8)
        n = C.c_int(0)
        _check(lib().voldor_batch_timing_summary(self._b, out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(n)),
               "voldor_batch_timing_summary")
        keys = ["bootstrap", "pose", "sweeps", "sweep_launches", "rigidness", "loglik", "window", "sweeps_busy"]
        return dict(zip(keys, out.tolist())), n.value

    def autotune(self, windows, params, stream=None):
        """Tune the sweeps on the first window of every distinct shape of
        `windows` (items as in solve); waits for the device."""
        descs = self._descs(windows)
        _check(lib().voldor_batch_autotune(self._b, descs, len(windows), C.byref(params), _stream(stream)),
               "voldor_batch_autotune")

    def solve(self, windows, params, status, stream=None):
        """Enqueue a batch.  windows: list of (flows [T,H,W,2] CUDA float32, K (fx, fy,
        cx, cy), out[, init[, n_pose_groups]]) with out = (poses, depth, rigidness,
        loglik or None) as from outputs(), init = None or (depth, rigidness, choice)
        as window_init, n_pose_groups this window's P3P groups per frame (0: the
        params'); status: CUDA int32 tensor of len(windows) elements.  Returns
        without waiting; the tensors must stay alive until the stream has run it."""
        import torch
        n = len(windows)
        if not (isinstance(status, torch.Tensor) and status.is_cuda and status.dtype == torch.int32
                and status.is_contiguous() and status.numel() >= n):
            raise TypeError("status must be a contiguous CUDA int32 tensor of len(windows) elements")
        descs = self._descs(windows)
        self._keep = (windows, status)
        _check(lib().voldor_window_batch(self._b, descs, n, C.byref(params), _ptr(status), _stream(stream)),
               "voldor_window_batch")


class Net:
    """The learned proposal (voldor_net_* in the C ABI) for windows of T frames."""

    def __init__(self, T, N_max, H_max, W_max):
        ctx = C.c_void_p()
        _check(lib().voldor_net_create(C.byref(ctx), T, N_max, H_max, W_max), "voldor_net_create")
        self._n = ctx
        self.T = T
        self.n_params = lib().voldor_net_param_count(self._n)

    def close(self):
        """Free the network's device buffers (waits for their work)."""
        if getattr(self, "_n", None):
            lib().voldor_net_destroy(self._n)
            self._n = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self, _fin=_sys.is_finalizing):
        if _fin():   # as Solver.__del__
            return
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _loss(loss, device):
        import torch
        if loss is not None and not (isinstance(loss, torch.Tensor) and loss.is_cuda and loss.dtype == torch.float64
                                     and loss.is_contiguous() and loss.numel() >= 1 and loss.device == device):
            raise TypeError("loss must be a contiguous CUDA float64 tensor of at least one element")

    def _batch(self, flows):
        """flows: contiguous CUDA float32 [N, T, H, W, 2] with this net's T."""
        import torch
        if not (isinstance(flows, torch.Tensor) and flows.is_cuda and flows.dtype == torch.float32
                and flows.is_contiguous()):
            raise TypeError("flows must be a contiguous CUDA float32 tensor [N,T,H,W,2]")
        if flows.dim() != 5 or flows.shape[4] != 2 or flows.shape[1] != self.T:
            raise ValueError(f"flows must have shape [N,{self.T},H,W,2], not {tuple(flows.shape)}")
        return flows.shape

    def set_params(self, params):
        a = np.ascontiguousarray(params, dtype=np.float32)
        if a.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        _check(lib().voldor_net_set_params(self._n, a.ctypes.data_as(C.POINTER(C.c_float))), "voldor_net_set_params")

    def get_params(self):
        a = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().voldor_net_get_params(self._n, a.ctypes.data_as(C.POINTER(C.c_float))), "voldor_net_get_params")
        return a

    def forward(self, flows, depth=None, rig=None, z=None, stream=None):
        """flows: CUDA float32 [N,T,H,W,2]; optional outputs as CUDA float32
        tensors: depth [N,H,W], rig [N,T,H,W], z (the network's raw output)
        [N,H,W,16]."""
        import torch
        N, T, H, W, _ = self._batch(flows)
        _dev_tensor(depth, "depth", torch.float32, (N, H, W), flows.device, optional=True)
        _dev_tensor(rig, "rig", torch.float32, (N, T, H, W), flows.device, optional=True)
        _dev_tensor(z, "z", torch.float32, (N, H, W, 16), flows.device, optional=True)
        _check(lib().voldor_net_forward(self._n, _ptr(flows), N, H, W, _ptr(depth), _ptr(rig), _ptr(z),
                                        _stream(stream)), "voldor_net_forward")

    def gradient(self, flows, depth, rig, loss=None, grad=None, stream=None):
        """Loss gradient against labels depth [N,H,W] and rig [N,T,H,W]; loss
        (CUDA float64 [2] or more) and grad (CUDA float32 [n_params]) optional."""
        import torch
        N, T, H, W, _ = self._batch(flows)
        _dev_tensor(depth, "depth", torch.float32, (N, H, W), flows.device)
        _dev_tensor(rig, "rig", torch.float32, (N, T, H, W), flows.device)
        self._loss(loss, flows.device)
        if grad is not None:
            _dev_tensor(grad, "grad", torch.float32, (self.n_params,), flows.device)
        _check(lib().voldor_net_gradient(self._n, _ptr(flows), N, H, W, _ptr(depth), _ptr(rig), _ptr(loss),
                                         _ptr(grad), _stream(stream)), "voldor_net_gradient")

    def train_step(self, flows, depth, rig, lr, loss=None, stream=None):
        import torch
        N, T, H, W, _ = self._batch(flows)
        _dev_tensor(depth, "depth", torch.float32, (N, H, W), flows.device)
        _dev_tensor(rig, "rig", torch.float32, (N, T, H, W), flows.device)
        self._loss(loss, flows.device)
        _check(lib().voldor_net_train_step(self._n, _ptr(flows), N, H, W, _ptr(depth), _ptr(rig), float(lr),
                                           _ptr(loss), _stream(stream)), "voldor_net_train_step")

    def layer(self, k, x, out, mask=None, backward=False, stream=None):
        """Layer k on a BF16 [N,H,W,32] tensor: forward into BF16 [N,H,W,32]
        (float32 [N,H,W,16] for k = 5), or backward (k >= 1) into BF16
        [N,H,W,32] times (mask > 0), mask BF16 [N,H,W,32]."""
        import torch
        if not (isinstance(x, torch.Tensor) and x.dim() == 4 and x.shape[3] == 32):
            raise ValueError("x must be a tensor [N,H,W,32]")
        N, H, W, _ = x.shape
        if not 0 <= int(k) <= 5 or (backward and int(k) < 1):
            raise ValueError("k must be 0..5 (1..5 backward)")
        _dev_tensor(x, "x", torch.bfloat16, (N, H, W, 32), None)
        if not backward and int(k) == 5:
            _dev_tensor(out, "out", torch.float32, (N, H, W, 16), x.device)
        else:
            _dev_tensor(out, "out", torch.bfloat16, (N, H, W, 32), x.device)
        _dev_tensor(mask, "mask", torch.bfloat16, (N, H, W, 32), x.device, optional=not backward)
        _check(lib().voldor_net_layer(self._n, k, 1 if backward else 0, _ptr(x), _ptr(mask), _ptr(out), N, H, W,
                                      _stream(stream)), "voldor_net_layer")
