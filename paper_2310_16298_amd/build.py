"""Build the HIP library ``libstencil.so`` for gfx950 (in-tree).

Every ``csrc/*.hip`` and ``csrc/*.cpp`` file is compiled by hipcc into
``_build/`` in parallel and linked into ``paper_2310_16298_amd/libstencil.so``.

    python -m paper_2310_16298_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libstencil.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wno-unused-result",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON + ["-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "hip"] + COMMON + ["-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources")
    return LIB


# Host-side sanitizer build (CPU tests only): the host sources -- plan and
# line cover, entry points, batches, server, autotuner -- instrumented with
# AddressSanitizer and UndefinedBehaviorSanitizer, linked with the kernel
# objects of the normal build into libstencil_asan.so.  Only the host pass is
# instrumented (each sanitizer flag applies to the host compilation alone).
LIB_ASAN = os.path.join(HERE, "libstencil_asan.so")
SANITIZE_HOST = [
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
    "-Xarch_host", "-fno-omit-frame-pointer",
]


def asan_runtime() -> str:
    """Path of the AddressSanitizer runtime that must be preloaded into a
    process (e.g. python) that loads libstencil_asan.so."""
    res = subprocess.run([os.path.join(os.path.dirname(HIPCC), "..", "llvm", "bin", "clang"),
                          "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return res.stdout.strip()


def build_sanitized(jobs: int | None = None) -> str:
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    kernel_objs = [os.path.join(BUILD, os.path.basename(s) + ".o") for s in srcs if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in kernel_objs):
        build(jobs)
    adir = os.path.join(BUILD, "asan")
    os.makedirs(adir, exist_ok=True)

    def compile_host(src: str) -> str:
        obj = os.path.join(adir, os.path.basename(src) + ".o")
        flags = [f for f in COMMON if f != "-O3"] + ["-O1", "-g"] + SANITIZE_HOST
        cmd = [HIPCC, "-x", "hip"] + flags + ["-c", src, "-o", obj]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stderr}")
        return obj

    host = [s for s in srcs if s.endswith(".cpp")]
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_host, host))
    tmp = LIB_ASAN + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + kernel_objs + [asan_runtime()]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stderr}")
    os.replace(tmp, LIB_ASAN)
    return LIB_ASAN


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "sanitize":
        print(build_sanitized())
    else:
        build(verbose=True)
    sys.exit(0)
