"""Build libh2vie.so (HIP, gfx950) in-tree.

    python -m paper_1703_01175_amd.build        # or build() from Python

Each source is compiled to an object with hipcc, then linked into
paper_1703_01175_amd/lib/libh2vie.so.  Packed FP32 instructions are disabled
for device code (-packed-fp32-ops).
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libh2vie.so")
SOURCES = ["h2vie_api.cpp", "h2_matvec.hip", "h2_convert.hip", "h2_krylov.hip", "h2_batch.hip", "h2_batch_api.cpp", "h2_learn.hip", "h2_krylov_batch.hip", "h2_matvec_mr.hip", "h2_bicgstab.hip"]
ARCH = os.environ.get("H2VIE_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def compile_flags():
    return ["-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-I", os.path.join(HERE, "..", "include")]


# host code only: AddressSanitizer and UndefinedBehaviorSanitizer (device code is
# built as usual); used by the CPU tests of the host-side validation and planning
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
ASAN_LIB = os.path.join(LIBDIR, "asan", "libh2vie.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    lib = ASAN_LIB if sanitize else LIB
    os.makedirs(os.path.dirname(lib), exist_ok=True)
    objdir = os.path.join(HERE, "_build_asan" if sanitize else "_build")
    os.makedirs(objdir, exist_ok=True)
    cc = hipcc()
    extra = SANITIZE_FLAGS if sanitize else []

    def one(src):
        obj = os.path.join(objdir, src + ".o")
        cmd = [cc, *compile_flags(), *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(len(SOURCES)) as ex:
        objs = list(ex.map(one, SOURCES))
    tmp = lib + ".tmp"
    link_extra = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-shared-libsan"] if sanitize else []
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *link_extra, "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
