"""The C-ABI library without a GPU: it loads, exports every function that
include/voldor.h declares, the Python binding knows each of them, and the
host-only calls and argument checks answer before any device work."""
import ctypes as C
import os
import re
import shutil

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "voldor.h")


def declared():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return sorted(set(re.findall(r"\b(voldor_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def vo():
    import paper_2104_06789_amd as m
    if not os.path.exists(m._LIB_PATH):
        if shutil.which(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")) is None:
            pytest.skip("libvoldor.so is not built and hipcc is not available")
        from paper_2104_06789_amd import build
        build.build()
    m.lib()
    return m


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("voldor_window", "voldor_window_async", "voldor_sweep", "voldor_pose_step",
              "voldor_bootstrap", "voldor_emission", "voldor_philox", "voldor_timing_summary"):
        assert n in names


def test_library_exports_every_declared_function(vo):
    raw = C.CDLL(vo._LIB_PATH)
    missing = [n for n in declared() if not hasattr(raw, n)]
    assert not missing


def test_binding_types_every_declared_function(vo):
    lib = vo.lib()
    for n in declared():
        fn = getattr(lib, n)
        assert fn.argtypes is not None, n


def test_params_default_and_status_strings(vo):
    p = vo.default_params()
    assert p.struct_size == C.sizeof(vo.Params)
    assert p.n_iters == 3 and p.sweeps_per_iter == 4 and p.gamma == 0.9
    assert p.sigma2_trans == 0.1 and p.sigma2_rot == 0.004
    assert p.criterion == vo.CRITERION_MIE and p.pose_start == 0 and p.residual_model == vo.RESIDUAL_FISK
    assert vo.status_str(0) == "ok"
    assert vo.status_str(-4) == "degenerate bootstrap"
    assert vo.status_str(12345) == "unknown status"


def test_host_argument_checks(vo):
    lib = vo.lib()
    ctx = C.c_void_p()
    # sizes outside the context limits are refused before any device call
    assert lib.voldor_create(C.byref(ctx), 0, 64, 64, 64) == vo.EINVAL
    assert lib.voldor_create(C.byref(ctx), 17, 64, 64, 64) == vo.EINVAL
    assert lib.voldor_create(C.byref(ctx), 4, 8, 64, 64) == vo.EINVAL
    assert lib.voldor_create(C.byref(ctx), 4, 64, 64, 8193) == vo.EINVAL
    assert lib.voldor_create(None, 4, 64, 64, 64) == vo.EINVAL
    K = (C.c_double * 4)(100.0, 100.0, 32.0, 32.0)
    p = vo.default_params()
    args = (None, None, 2, 64, 64, K, C.byref(p), None, None, None, None)
    assert lib.voldor_window(*args, None) == vo.EINVAL
    assert lib.voldor_window_async(*args, None, None) == vo.EINVAL
    out = (C.c_double * 8)()
    assert lib.voldor_last_timing(None, out) == vo.EINVAL
    assert lib.voldor_timing_summary(None, out, None) == vo.EINVAL
    assert lib.voldor_set_timing(None, 1) == vo.EINVAL


def test_batch_host_argument_checks(vo):
    lib = vo.lib()
    b = C.c_void_p()
    assert lib.voldor_batch_create(C.byref(b), 0, 4, 64, 64, 64, 0) == vo.EINVAL
    assert lib.voldor_batch_create(C.byref(b), 17, 4, 64, 64, 64, 0) == vo.EINVAL
    assert lib.voldor_batch_create(C.byref(b), 2, 4, 64, 64, 64, 4) == vo.EINVAL   # unknown flag
    assert lib.voldor_batch_create(None, 2, 4, 64, 64, 64, 0) == vo.EINVAL
    p = vo.default_params()
    descs = (vo.WindowDesc * 1)()
    assert lib.voldor_window_batch(None, descs, 1, C.byref(p), None, None) == vo.EINVAL
    lib.voldor_batch_destroy(None)


def test_vo_window_count_matches_the_oracle_starts(vo):
    # host-side window schedule of voldor_vo_sequence against the oracle's
    # window_starts; strides that would leave the next T_1 outside a window fail
    import oracle
    lib = vo.lib()
    for N, T, stride in [(12, 5, 1), (12, 5, 3), (5, 5, 2), (9, 4, 3), (30, 6, 1), (31, 6, 4), (16, 16, 15)]:
        assert lib.voldor_vo_windows(N, T, stride) == len(oracle.window_starts(N, T, stride)), (N, T, stride)
    for N, T, stride in [(12, 5, 5), (12, 5, 0), (4, 5, 1), (12, 1, 1), (40, 17, 2)]:
        assert lib.voldor_vo_windows(N, T, stride) == vo.EINVAL, (N, T, stride)


def test_abi_struct_layout_matches_binding(tmp_path):
    # the C compiler's view of the two structs the binding mirrors
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    import paper_2104_06789_amd as vo
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "voldor.h"\n'
        "int main(void) {\n"
        '  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(voldor_window_desc),\n'
        "    offsetof(voldor_window_desc, flows), offsetof(voldor_window_desc, T),\n"
        "    offsetof(voldor_window_desc, K), offsetof(voldor_window_desc, poses),\n"
        "    offsetof(voldor_window_desc, loglik), offsetof(voldor_window_desc, init_depth),\n"
        "    offsetof(voldor_window_desc, choice), sizeof(voldor_params),\n"
        "    offsetof(voldor_params, ms_tol), offsetof(voldor_params, depth_hi),\n"
        "    offsetof(voldor_params, seed), offsetof(voldor_params, criterion),\n"
        "    offsetof(voldor_params, residual_model));\n  return 0;\n}\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run([gcc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    D, P = vo.WindowDesc, vo.Params
    want = [C.sizeof(D), D.flows.offset, D.T.offset, D.K.offset, D.poses.offset, D.loglik.offset,
            D.init_depth.offset, D.choice.offset, C.sizeof(P), P.ms_tol.offset, P.depth_hi.offset, P.seed.offset,
            P.criterion.offset, P.residual_model.offset]
    assert got == want


def test_bench_refuses_more_than_one_gpu():
    # one GPU's share is what bench.py measures; --gpus N > 1 exits with a message
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_binding_rejects_host_tensors_before_any_call(vo):
    # the binding checks device, dtype, contiguity and shape before a pointer
    # reaches the library (a host pointer would fault the GPU)
    import torch
    X = torch.zeros((10, 2))
    with pytest.raises(TypeError):
        vo.residual_bins(X, X)
    with pytest.raises(TypeError):
        vo.residual_bins_noalloc(X, X, torch.zeros((40, 4), dtype=torch.float64))
    with pytest.raises(TypeError):
        vo._dev_tensor(torch.zeros((4, 5)), "depth", torch.float32, (4, 5), None)
    n = vo.Net.__new__(vo.Net)          # no device context: the checks come first
    n.T, n._n, n.n_params = 3, None, 10
    with pytest.raises(TypeError):
        n.forward(torch.zeros((1, 3, 16, 16, 2)))
    with pytest.raises(TypeError):
        n.train_step(torch.zeros((1, 3, 16, 16, 2)), torch.zeros((1, 16, 16)), torch.zeros((1, 3, 16, 16)), 1e-3)
    with pytest.raises(ValueError):
        n.layer(0, torch.zeros((1, 16, 16, 8)), None)
    s = vo.Solver.__new__(vo.Solver)
    s._ctx = C.c_void_p()
    with pytest.raises(TypeError):
        s.window_init(torch.zeros((3, 16, 16, 2)), (10, 10, 8, 8), vo.default_params(), torch.ones((16, 16)),
                      torch.ones((3, 16, 16)), None, None)
