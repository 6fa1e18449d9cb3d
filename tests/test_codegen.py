"""Properties of the library's gfx950 code, read from the built libvoldor.so
with the ROCm tools (no GPU): the batched kernels, which read their argument
pointers from device memory, access memory through global (not flat)
instructions, and the sweep kernels keep every value in registers and LDS
(no private scratch)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LLVM = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


def _tool(name):
    path = os.path.join(LLVM, name)
    if not os.path.exists(path):
        pytest.skip(f"{path} is not available")
    return path


@pytest.fixture(scope="module")
def device_code(tmp_path_factory):
    """{kernel symbol: its disassembly} of every gfx950 code object in the library."""
    import paper_2104_06789_amd as m
    if not os.path.exists(m._LIB_PATH):
        if shutil.which(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")) is None:
            pytest.skip("libvoldor.so is not built and hipcc is not available")
        from paper_2104_06789_amd import build
        build.build()
    if shutil.which("objcopy") is None:
        pytest.skip("objcopy is not available")
    bundler, objdump = _tool("clang-offload-bundler"), _tool("llvm-objdump")
    tmp = tmp_path_factory.mktemp("code")
    fat = tmp / "fatbin"
    subprocess.run(["objcopy", "-O", "binary", "--only-section=.hip_fatbin", m._LIB_PATH, str(fat)], check=True)
    data = fat.read_bytes()
    starts = [i.start() for i in re.finditer(re.escape(MAGIC), data)]
    assert starts, "no offload bundle in the library"
    code = {}
    for n, (a, b) in enumerate(zip(starts, starts[1:] + [len(data)])):
        part, obj = tmp / f"bundle{n}", tmp / f"code{n}.o"
        part.write_bytes(data[a:b])
        subprocess.run([bundler, "--unbundle", "--type=o", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950",
                        f"--input={part}", f"--output={obj}"], check=True)
        dis = subprocess.run([objdump, "-d", str(obj)], check=True, capture_output=True, text=True).stdout
        name = None
        for line in dis.splitlines():
            hdr = re.match(r"^[0-9a-f]+ <(\S+)>:$", line)
            if hdr:
                name = hdr.group(1)
                code[name] = []
            elif name:
                code[name].append(line)
    return code


def test_batched_kernels_use_no_flat_memory_instructions(device_code):
    multi = {k: v for k, v in device_code.items() if "_multi" in k}
    # the lockstep sweep, rigidness, log-likelihood, pose-step and bootstrap kernels
    for part in ("k_sweep_multi", "k_rigidness_multi", "k_pose_groups_multi", "k_pose_ms_multi",
                 "k_boot_score_multi"):
        assert any(part in k for k in multi), part
    flat = {k: sum(1 for l in v if re.search(r"\sflat_(load|store|atomic)", l)) for k, v in multi.items()}
    assert not any(flat.values()), {k: n for k, n in flat.items() if n}
    glob = sum(1 for v in multi.values() for l in v if re.search(r"\sglobal_(load|store)", l))
    assert glob > 0


def test_sweep_kernels_use_no_scratch(device_code):
    sweeps = {k: v for k, v in device_code.items() if "k_sweep" in k}
    assert sweeps
    for k, v in sweeps.items():
        assert not any(re.search(r"\s(scratch|buffer)_(load|store)", l) for l in v), k
