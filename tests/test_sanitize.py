"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer: a
sanitizer build of the library (paper_1305_3625_amd/build.py --sanitize)
driven through every entry point's GPU-free paths in a child process with
the sanitizer runtime preloaded (tests/sanitize_driver.py).  Slow: the
build takes about a minute; run with RUN_SLOW=1."""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow


def _runtime():
    hits = sorted(glob.glob("/opt/rocm*/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_host_code_under_sanitizers():
    rt = _runtime()
    if rt is None:
        pytest.skip("no clang AddressSanitizer runtime in this image")
    from paper_1305_3625_amd import build
    lib = build.build(sanitize=True)
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    p = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitize_driver.py"), lib], env=env,
                       capture_output=True, text=True, timeout=600)
    assert p.returncode == 0 and "SANITIZE_OK" in p.stdout, p.stdout[-3000:] + p.stderr[-3000:]
