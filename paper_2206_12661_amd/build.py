"""Build ``libgswmtp.so`` (HIP for gfx950) in-tree.

Every ``csrc/*.hip`` file is compiled with hipcc for gfx950 only and linked
into one shared library next to this file.  Objects go to ``_build/``.

``python -m paper_2206_12661_amd.build --sanitize`` builds the library with
its host code instrumented by AddressSanitizer and UndefinedBehaviorSanitizer
(device code as usual, at -O1) into ``_build/san/libgswmtp_san.so``, for
running the CPU tests over the library's host logic (validation, sizing,
layout, failure paths).  The sanitizer runtime is not linked in: the process that
loads this library preloads ``libclang_rt.asan`` (``sanitizer_env``).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgswmtp.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Wno-unused-function", "-Wno-unused-result",
    # no packed-fp32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))
    cmd = [HIPCC, *CFLAGS, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    # the host pass warns that it does not know the device-only feature flag
    noise = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()
             and "warning: unknown target feature" not in l]
    if verbose and noise:
        print("\n".join(noise), file=sys.stderr)
    return obj


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = jobs or min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


SAN_DIR = os.path.join(BUILD, "san")
SAN_LIB = os.path.join(SAN_DIR, "libgswmtp_san.so")
SAN_FLAGS = [
    f"--offload-arch={ARCH}", "-O1", "-std=c++17", "-fPIC", "-Wno-unused-result",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Xarch_host", "-g", "-Xarch_host", "-fno-omit-frame-pointer",
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
]


def build_sanitized(verbose: bool = False) -> str:
    """ASan + UBSan build of the library's host code (see the module docstring)."""
    os.makedirs(SAN_DIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))

    def one(src):
        obj = os.path.join(SAN_DIR, os.path.basename(src).replace(".hip", ".o"))
        cmd = [HIPCC, *SAN_FLAGS, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"sanitized host build failed for {src}:\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(min(len(srcs), 8)) as ex:
        objs = list(ex.map(one, srcs))
    tmp = SAN_LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


def sanitizer_runtime() -> str:
    """Path of the clang AddressSanitizer runtime that hipcc's compiler ships."""
    cands = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not cands:
        cands = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/"
                                 "libclang_rt.asan-x86_64.so"))
    if not cands:
        raise FileNotFoundError("libclang_rt.asan-x86_64.so not found under /opt/rocm")
    return cands[-1]


def sanitizer_env(base=None) -> dict:
    """Environment for a child process that loads the sanitized library: the
    ASan runtime preloaded first (ahead of anything already preloaded), leak
    checks off (the interpreter keeps its allocations), halt on the first
    report, and GSWMTP_LIBRARY naming the sanitized build."""
    env = dict(os.environ if base is None else base)
    pre = env.get("LD_PRELOAD", "")
    env["LD_PRELOAD"] = sanitizer_runtime() + (":" + pre if pre else "")
    env["ASAN_OPTIONS"] = ("detect_leaks=0:halt_on_error=1:alloc_dealloc_mismatch=0:"
                           "protect_shadow_gap=0:detect_odr_violation=0")
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["GSWMTP_LIBRARY"] = SAN_LIB
    return env


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
