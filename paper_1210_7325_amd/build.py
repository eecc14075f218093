"""Builds the native libraries in-tree.

  libgls.so     the solver (HIP kernels for gfx950 + the C ABI of include/gls.h)
  libglsgen.so  the synthetic-input generator (host C, OpenMP)
  libglsgen_dev.so  its device twin (HIP), for inputs generated in HBM
  tests/c_abi/gls_c_check  a C program using only include/gls.h (test)
  libgls_phase.so  libgls.so with phase timestamps in the paired-block solve
                   (measurement build, read by phase_timing.py)

Run `python -m paper_1210_7325_amd.build` or call build_all().
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # keep MFMA accumulators in VGPRs (no AGPR round trips in the loops)
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
    # never emit packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        sys.stderr.write(out + "\n")
        raise RuntimeError(f"build step failed: {' '.join(cmd)}")
    return out


# translation units of libgls.so, one per step of the path (plus the C ABI)
GLS_UNITS = ("gls_factor.hip", "gls_fixed.hip", "gls_trsm.hip", "gls_trsm_mixed.hip",
             "gls_assemble.hip", "gls_api.cpp", "gls_io.cpp", "gls_noalloc.hip")


def _code_only(text: str) -> str:
    """C++ source without comments and with whitespace runs collapsed (the
    sources hold no string literal containing comment markers)."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def trsm_source_digest() -> str:
    """SHA-256 over everything that decides the FP64 triangular-solve
    kernel's machine code: its source and the shared device headers (code
    only: comments and layout do not count) and the compiler flags.  Counter
    readings taken for one digest are stale for any other."""
    import hashlib
    h = hashlib.sha256()
    for name in ("gls_trsm.hip", "gls_device.h", "gls_internal.h"):
        with open(os.path.join(CSRC, name), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    h.update(" ".join(HIP_FLAGS[:-2]).encode())  # flags without the include paths
    return h.hexdigest()


def build_gls(verbose: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD, exist_ok=True)

    def compile_unit(src):
        obj = os.path.join(BUILD, src + ".o")
        _run([HIPCC, "-x", "hip", *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=min(len(GLS_UNITS), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_unit, GLS_UNITS))
    tmp = os.path.join(PKG, "libgls.so.tmp")
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, os.path.join(PKG, "libgls.so"))
    return os.path.join(PKG, "libgls.so")


def build_phase_timing() -> str:
    """libgls.so's units with gls_trsm.hip replaced by trsm_phase_timing.hip
    (the same kernels plus phase timestamps; a measurement build, not the
    library).  Reuses the other units' objects of build_gls."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in GLS_UNITS:
        if src == "gls_trsm.hip":
            src = "trsm_phase_timing.hip"
            obj = os.path.join(BUILD, src + ".o")
            _run([HIPCC, "-x", "hip", *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        else:
            obj = os.path.join(BUILD, src + ".o")
            if not os.path.exists(obj):
                _run([HIPCC, "-x", "hip", *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    tmp = os.path.join(PKG, "libgls_phase.so.tmp")
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, os.path.join(PKG, "libgls_phase.so"))
    return os.path.join(PKG, "libgls_phase.so")


def build_gen() -> str:
    out = os.path.join(PKG, "libglsgen.so")
    cc = shutil.which("gcc") or "cc"
    tmp = out + ".tmp"
    _run([cc, "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
          os.path.join(CSRC, "datagen.c"), "-o", tmp])
    os.replace(tmp, out)
    return out


def build_gen_dev() -> str:
    """Device twin of the generator (its own library: input generation only)."""
    os.makedirs(BUILD, exist_ok=True)
    obj = os.path.join(BUILD, "datagen_dev.hip.o")
    _run([HIPCC, "-x", "hip", *HIP_FLAGS, "-ffp-contract=off", "-c",
          os.path.join(CSRC, "datagen_dev.hip"), "-o", obj])
    tmp = os.path.join(PKG, "libglsgen_dev.so.tmp")
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", obj, "-o", tmp])
    os.replace(tmp, os.path.join(PKG, "libglsgen_dev.so"))
    return os.path.join(PKG, "libglsgen_dev.so")


def build_c_check() -> str:
    """The C program of tests/c_abi that drives libgls through its C ABI only
    (test infrastructure; found next to its source, libgls.so via rpath)."""
    src = os.path.join(ROOT, "tests", "c_abi", "gls_c_check.c")
    out = os.path.join(ROOT, "tests", "c_abi", "gls_c_check")
    cc = shutil.which("gcc") or "cc"
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    tmp = out + ".tmp"
    _run([cc, "-O2", "-std=c11", "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include", f"-I{INCLUDE}", src,
          "-o", tmp, f"-L{PKG}", "-lgls", f"-L{rocm}/lib", "-lamdhip64", "-lm",
          "-Wl,-rpath,$ORIGIN/../../paper_1210_7325_amd", f"-Wl,-rpath,{rocm}/lib"])
    os.replace(tmp, out)
    return out


def build_mfma_valu_bench() -> str:
    """The issue-rate measurement of MFMAs mixed with VALU instructions (a
    measurement program for the FP32_REFINE solve's ceiling, not part of
    the library)."""
    out = os.path.join(PKG, "mfma_valu_bench")
    tmp = out + ".tmp"
    _run([HIPCC, "-x", "hip", *HIP_FLAGS, os.path.join(CSRC, "mfma_valu_bench.hip"), "-o", tmp])
    os.replace(tmp, out)
    return out


def build_all() -> None:
    build_gen()
    build_gen_dev()
    build_gls()
    build_phase_timing()
    build_c_check()
    build_mfma_valu_bench()


if __name__ == "__main__":
    build_all()
    print("built", os.path.join(PKG, "libgls.so"), os.path.join(PKG, "libglsgen.so"))
