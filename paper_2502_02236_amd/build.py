"""Build libasd.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc.

Usage: python -m paper_2502_02236_amd.build   (or paper_2502_02236_amd.build.build())
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libasd.so")
ARCH = os.environ.get("ASD_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Wall", "-Wno-unused-function",
          # no packed FP32 (v_pk_*_f32) code generation
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

# (source, extra flags)
SOURCES = [
    ("asd_step_f64.hip", ["-ffp-contract=off"]),
    ("asd_step_f32.hip", ["-ffp-contract=fast"]),
    ("asd_misc.hip", ["-ffp-contract=off"]),
    ("asd_demag.hip", ["-ffp-contract=fast"]),
    ("asd_mm.hip", ["-ffp-contract=off"]),
    ("asd_host.cpp", ["-ffp-contract=off"]),
    ("asd_demag_tensor.cpp", ["-ffp-contract=off"]),
]

HEADERS = ["asd_device.h", "asd_internal.h", "asd_step.inc", "asd_fused.inc", "asd_fused_l10.inc",
           "asd_variants.h"]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _compile(src: str, flags: list, srcdir: str = CSRC) -> str:
    obj = os.path.join(BUILD, src + ".o")
    lang = ["-x", "hip"]
    cmd = [hipcc(), *lang, *COMMON, *flags, "-c", os.path.join(srcdir, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def _link(objs: list, lib: str) -> None:
    tmp = lib + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    """Compile every source for gfx950 and link libasd.so next to this file."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda sf: _compile(*sf), SOURCES))
    _link(objs, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def build_probe(src: str, lib: str) -> str:
    """Compile one measurement-only HIP source (not part of libasd) into its own
    shared library `lib` with the library's flags."""
    os.makedirs(BUILD, exist_ok=True)
    obj = _compile(os.path.basename(src), ["-ffp-contract=fast"], os.path.dirname(src))
    _link([obj], lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
