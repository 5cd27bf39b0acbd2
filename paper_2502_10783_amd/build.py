"""Build libipp.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Every call recompiles: ``python -m paper_2502_10783_amd.build``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libipp.so")
BUILD_DIR = os.path.join(os.path.dirname(HERE), "_build")

ARCH = "gfx950"
COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # binary64/binary32 predicates and bounds must round exactly as written
    "-ffp-contract=off",
    # packed FP32 instructions are not to be generated
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-Wno-unused-but-set-variable",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc",
                 shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libipp)")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    cmd = [hipcc()] + COMMON + ["-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp]
    cmd += objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


# Host code built with AddressSanitizer and UndefinedBehaviorSanitizer (the
# device code is unchanged): the validation, planning and launch code of
# the ABI checked by the CPU tests, e.g.
#   python paper_2502_10783_amd/build.py --sanitize-host
#   LD_PRELOAD=$(hipcc --print-file-name=libclang_rt.asan-x86_64.so) \
#   ASAN_OPTIONS=detect_leaks=0 IPP_LIB=_build/san/libipp_san.so \
#   python -m pytest tests/test_abi.py -m "not gpu"
SAN_DIR = os.path.join(BUILD_DIR, "san")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host",
       "-fsanitize=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile_san(src: str) -> str:
    obj = os.path.join(SAN_DIR, os.path.basename(src) + ".o")
    cmd = ([hipcc()] + [c if c != "-O3" else "-O1" for c in COMMON] +
           ["-g"] + SAN + ["-x", "hip", "-c", src, "-o", obj])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
    return obj


def build_sanitized(verbose: bool = False) -> str:
    os.makedirs(SAN_DIR, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile_san, srcs))
    out = os.path.join(SAN_DIR, "libipp_san.so")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC"] + SAN[:4]
    cmd += ["-shared-libsan", "-o", out] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    if "--sanitize-host" in sys.argv[1:]:
        build_sanitized(verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)
