"""Host-only checks of the C ABI: the library loads, exports every symbol that
include/asd.h declares, and validates descriptors before touching a GPU."""
import ctypes as C
import os
import re

import pytest

import workloads as W
from paper_2502_02236_amd import asd as A
from paper_2502_02236_amd import bridge

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "asd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(asd_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = A.lib()
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(A.SYMBOLS)


def _ws(params, systems):
    arr = (A.asd_system_desc * len(systems))(*systems)
    out = C.c_size_t(0)
    return A.lib().asd_workspace_bytes(C.byref(params), arr, len(systems), C.byref(out)), out.value


def test_workspace_size_and_validation():
    w = W.c2_granular_slab()
    p = bridge.params_for(w, A.ASD_FP32)
    si = bridge.SystemInputs(w)
    rc, n = _ws(p, [si.desc])
    assert rc == A.ASD_OK
    # three spin buffers of 3 x 1.32M floats at least
    assert n > 3 * 3 * 200 * 200 * 33 * 4
    p64 = bridge.params_for(w, A.ASD_FP64)
    rc, n64 = _ws(p64, [si.desc])
    assert rc == A.ASD_OK and n64 > n
    bad = bridge.params_for(w, A.ASD_FP32)
    bad.n_shells = 2
    assert _ws(bad, [si.desc])[0] == A.ASD_EINVAL
    bad = bridge.params_for(w, A.ASD_FP32)
    bad.dt = -1.0
    assert _ws(bad, [si.desc])[0] == A.ASD_EINVAL
    bad = bridge.params_for(w, A.ASD_FP32)
    bad.philox_rounds = 3
    assert _ws(bad, [si.desc])[0] == A.ASD_EINVAL
    bad = bridge.params_for(w, A.ASD_FP32, graph_steps=3)
    assert _ws(bad, [si.desc])[0] == A.ASD_EINVAL
    d = bridge.SystemInputs(w.scaled(nx=2)).desc  # periodic axis with 2 cells
    assert _ws(p, [d])[0] == A.ASD_EINVAL
    d = bridge.SystemInputs(w.scaled(bc=(A.ASD_BC_TRACK, 0, 0), track_nx=100)).desc
    assert _ws(p, [d])[0] == A.ASD_EINVAL  # track shorter than the window
    d = bridge.SystemInputs(w.scaled(bc=(0, A.ASD_BC_TRACK, 0))).desc
    assert _ws(p, [d])[0] == A.ASD_EINVAL  # track only along x
    assert b"invalid" in A.lib().asd_strerror(A.ASD_EINVAL)


def test_create_rejects_bad_workspace_without_gpu():
    w = W.c1_plain_sc()
    p = bridge.params_for(w, A.ASD_FP64)
    si = bridge.SystemInputs(w)
    arr = (A.asd_system_desc * 1)(si.desc)
    h = C.c_void_p()
    # NULL workspace and a too-small workspace are refused before any HIP call
    assert A.lib().asd_create(C.byref(p), arr, 1, None, 0, None, C.byref(h)) == A.ASD_EINVAL
    assert A.lib().asd_create(C.byref(p), arr, 1, C.c_void_p(256), 16, None, C.byref(h)) == A.ASD_ENOMEM
    assert A.lib().asd_step(None, 1) == A.ASD_EINVAL
    assert A.lib().asd_philox(1, 3, None, None, -1, None) == A.ASD_EINVAL


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2502_02236_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h", ".inc")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "asd_oracle" not in text, f


def test_fast_division_helper(tmp_path):
    """The kernels' division by a precomputed multiplier equals integer division."""
    import shutil
    import subprocess
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "fastdiv")
    subprocess.run([hipcc, "-O2", "-I", os.path.join(ROOT, "paper_2502_02236_amd", "csrc"),
                    os.path.join(ROOT, "tests", "helpers", "fastdiv_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    checked, bad = map(int, out.stdout.split())
    assert out.returncode == 0 and bad == 0 and checked > 4_000_000


def test_plain_c_client_compiles_and_links(tmp_path):
    """include/asd.h is a C header: a C11 client compiles with gcc and links
    against the library (it is run against the GPU in the parity tests)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("gcc or the HIP headers are not available")
    pkg = os.path.join(ROOT, "paper_2502_02236_amd")
    exe = str(tmp_path / "abi_c_client")
    r = subprocess.run([gcc, "-O1", "-std=c11", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
                        "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "helpers", "abi_c_client.c"), "-o", exe,
                        "-L", pkg, "-lasd", "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath," + pkg],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    u = subprocess.run([exe], capture_output=True, text=True)
    assert u.returncode == 2 and "usage" in u.stderr
