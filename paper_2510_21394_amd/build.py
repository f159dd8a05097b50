"""Compile the HIP sources of the package into libfcgle.so (gfx950), in-tree.

Usage: python -m paper_2510_21394_amd.build  [--jobs N] [--sanitize]
Every HIP translation unit is built with hipcc for gfx950 only; packed FP32 VALU
instructions are disabled for device code (see the design notes).

--sanitize builds _build_san/libfcgle_san.so instead: the same sources with AddressSanitizer and
UndefinedBehaviorSanitizer on the host code only (the device code is unchanged), every
translation unit through clang so that one sanitizer runtime serves them all.  It is for
CPU runs of the host logic (set-up, eigensolver, plan bookkeeping):
    LD_PRELOAD=<clang>/lib/linux/libclang_rt.asan-x86_64.so ASAN_OPTIONS=detect_leaks=0 \
    FCGLE_LIB=paper_2510_21394_amd/_build_san/libfcgle_san.so python -m pytest tests/test_abi_cpu.py
(asan_runtime() returns the preload path).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfcgle.so")

HIP_SOURCES = ["api.hip", "batch.hip", "group_f32.hip", "pointwise.hip", "adjoint.hip", "refine.hip", "krogstad.hip",
               "mp_f64.hip", "mp_f32.hip", "mp_bf16.hip"]
CXX_SOURCES = ["host_math.cpp"]
ARCH = "gfx950"
HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-mcode-object-version=5",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]
CXX_FLAGS = ["-O3", "-std=c++17", "-fPIC"]
LIB_SAN = os.path.join(HERE, "_build_san", "libfcgle_san.so")
# host-only sanitizers: each -fsanitize= applies to the host compilation only
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
SAN_CXX = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


def _hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else (shutil.which("hipcc") or "hipcc")


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"command failed ({p.returncode}): {' '.join(cmd)}\n{out}")
    return out


def _clangxx() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "llvm", "bin", "clang++")


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime to preload for a sanitized build."""
    out = subprocess.run([_clangxx(), "-print-file-name=libclang_rt.asan-x86_64.so"], stdout=subprocess.PIPE,
                         text=True).stdout.strip()
    if not os.path.exists(out):
        rd = subprocess.run([_clangxx(), "-print-resource-dir"], stdout=subprocess.PIPE, text=True).stdout.strip()
        out = os.path.join(rd, "lib", "linux", "libclang_rt.asan-x86_64.so")
    return out


def build(jobs: int = 0, verbose: bool = False, sanitize: bool = False) -> str:
    bdir = BUILD + ("_san" if sanitize else "")
    os.makedirs(bdir, exist_ok=True)
    hipcc = _hipcc()
    cmds, objs = [], []
    for src in HIP_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        cmds.append([hipcc, *HIPCC_FLAGS, *(SAN_HOST if sanitize else []), "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in CXX_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        if sanitize:
            cmds.append([_clangxx(), *CXX_FLAGS, *SAN_CXX, "-c", os.path.join(CSRC, src), "-o", obj])
        else:
            cmds.append(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    jobs = jobs or min(len(cmds), os.cpu_count() or 4, 8)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for out in ex.map(_run, cmds):
            if verbose and out.strip():
                print(out)
    lib = LIB_SAN if sanitize else LIB
    tmp = lib + ".tmp"
    link = [hipcc, f"--offload-arch={ARCH}", "-shared", "-o", tmp, *objs, "-lpthread"]
    if sanitize:
        link += ["-fsanitize=address,undefined", "-shared-libsan"]
    _run(link)
    os.replace(tmp, lib)
    return lib


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=0)
    ap.add_argument("-v", "--verbose", action="store_true")
    ap.add_argument("--sanitize", action="store_true", help="host ASan + UBSan build into libfcgle_san.so")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.verbose, a.sanitize))


if __name__ == "__main__":
    sys.exit(main())
