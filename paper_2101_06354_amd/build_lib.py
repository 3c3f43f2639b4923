"""Build libssimx.so (HIP C++ for gfx950) in-tree with hipcc.

Usage: python paper_2101_06354_amd/build_lib.py [--jobs N]  (by path: importing the package
would first load the library being rebuilt)
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
LIB = os.path.join(HERE, "libssimx.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    # packed FP32 ops stay off: only scalar v_fma/v_add/v_mul_f32 are emitted
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast",
]


def sources() -> list[str]:
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build: every
# -fsanitize applies to the host compilation only (-Xarch_host); the device
# code is the ordinary one.  The library leaves the sanitizer runtime
# unresolved: load it into a process that preloads clang's ASan runtime
# (sanitizer_runtime()) with SSIMX_LIBRARY pointing at it.
SAN_DIR = os.path.join(BUILD, "asan")
SAN_LIB = os.path.join(SAN_DIR, "libssimx.so")
SAN_FLAGS = ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def sanitizer_runtime() -> str:
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("clang's ASan runtime was not found under /opt/rocm/llvm")
    return hits[-1]


def _compile(src: str, out_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    flags = [f for f in HIPCC_FLAGS if f != "-O3"] + list(extra) if extra else HIPCC_FLAGS
    cmd = [hipcc(), *flags, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(jobs: int = 8, verbose: bool = False, sanitize_host: bool = False) -> str:
    out_dir, lib, extra = (SAN_DIR, SAN_LIB, SAN_FLAGS) if sanitize_host else (BUILD, LIB, ())
    os.makedirs(out_dir, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: _compile(s, out_dir, extra), srcs))
    tmp = lib + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib} from {len(srcs)} sources")
    return lib


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--sanitize-host", action="store_true",
                    help="build the host-sanitised library (ASan + UBSan on host code) under _build/asan")
    a = ap.parse_args()
    build(a.jobs, verbose=True, sanitize_host=a.sanitize_host)
    sys.exit(0)
