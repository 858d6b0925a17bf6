"""The CPU suite over a build of the library whose host code carries
AddressSanitizer and UndefinedBehaviorSanitizer: descriptor validation, the
host-side sizing and layout, the null-argument and fault-injection paths and
the binding's marshalling run instrumented, and any report (out-of-bounds
access, use after free, signed overflow, misaligned load, ...) halts the child
run and fails this test.  Builds the instrumented library when it is missing
or older than a source (about two minutes); no GPU is touched."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _stale(lib: str) -> bool:
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    srcs = glob.glob(os.path.join(ROOT, "paper_2206_12661_amd", "csrc", "*"))
    return any(os.path.getmtime(s) > t for s in srcs)


@pytest.fixture(scope="module")
def san_env():
    from paper_2206_12661_amd import build as b
    try:
        b.sanitizer_runtime()
    except FileNotFoundError as e:
        pytest.skip(str(e))
    if _stale(b.SAN_LIB):
        b.build_sanitized()
    return b.sanitizer_env()


def test_instrumented_library_is_the_one_loaded(san_env):
    code = ("import ctypes, paper_2206_12661_amd as g; lib = g.load_library(); "
            "maps = open('/proc/self/maps').read(); "
            "assert 'libgswmtp_san.so' in maps and 'libclang_rt.asan' in maps, maps[:200]; "
            "assert hasattr(ctypes.CDLL(None), '__asan_init'); "
            "assert not hasattr(ctypes.CDLL(None), 'no_such_symbol_here'); print('ok')")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=san_env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().endswith("ok")


def test_cpu_suite_under_asan_ubsan(san_env):
    here = os.path.basename(__file__)
    r = subprocess.run([sys.executable, "-m", "pytest", "tests", "-q", "-x", "-m", "not gpu",
                        "-p", "no:cacheprovider", f"--deselect=tests/{here}",
                        "--ignore", f"tests/{here}"],
                       cwd=ROOT, env=san_env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in r.stdout
