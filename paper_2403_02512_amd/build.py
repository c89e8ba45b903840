"""Compile the HIP sources into the in-tree shared library ``libqsv.so``.

Every source is compiled by hipcc for gfx950 only.  Packed-FP32 instruction
selection is switched off for device code (``-packed-fp32-ops``).  Objects go
to ``_build/`` at the repository root; the library lands next to this file so
that tests, the smoke check and the benchmark load exactly this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libqsv.so")
ARCH = "gfx950"

SOURCES = ["tile_f64_two.hip", "tile_f64_one.hip", "tile_f32_two.hip", "tile_f32_one.hip", "kernels.hip",
           "gates.cpp", "plan.cpp", "api.cpp"]
HEADERS = ["qsv_internal.h", "kcommon.h", "k_tile.h"]

DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    is_hip = src.endswith(".hip")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
           f"-I{INCLUDE}", f"-I{CSRC}", "-c", os.path.join(CSRC, src), "-o", obj]
    if is_hip:
        cmd[1:1] = ["-x", "hip"]
        cmd += DEVICE_FLAGS + ["-ffp-contract=fast", "-munsafe-fp-atomics"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    """Compile every source (always) and link libqsv.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


HOST_SOURCES = ["gates.cpp", "plan.cpp", "api.cpp"]
# host-only instrumentation: the kernels (.hip) keep their normal objects
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def build_sanitized(out_dir: str) -> str:
    """A CPU-test build of the library whose host runtime (validation,
    planning, lowering, the C entry points) carries AddressSanitizer and
    UndefinedBehaviorSanitizer, linked with the normal kernel objects.
    Returns the path of its libqsv.so (run it with the ASan runtime
    preloaded)."""
    os.makedirs(out_dir, exist_ok=True)
    kobjs = []
    for src in SOURCES:
        if src.endswith(".hip"):
            obj = os.path.join(BUILD, os.path.basename(src) + ".o")
            kobjs.append(obj if os.path.exists(obj) else _compile(src))
    hobjs = []
    for src in HOST_SOURCES:
        obj = os.path.join(out_dir, src + ".o")
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-O1", "-std=c++17", "-fPIC", "-Wall", *SANITIZE,
               f"-I{INCLUDE}", f"-I{CSRC}", "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        hobjs.append(obj)
    lib = os.path.join(out_dir, "libqsv.so")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-shared-libsan",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", *hobjs, *kobjs, "-o", lib]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return lib


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime the sanitized build links against."""
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    r = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return r.stdout.strip()


if __name__ == "__main__":
    build()
