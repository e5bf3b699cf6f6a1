"""The server's scheduler (paper_1305_3625_amd/csrc/server.cpp, unmodified)
on a simulated device, on the CPU: concurrent clients over fused and
multi-pass classes, budgeted admission, queue cap, maxit, load-stepped
sequences, shutdown, chunk graphs (tests/server_fake_scenarios.py); and the
same scenarios under ThreadSanitizer (slow)."""

import os
import subprocess
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import server_fake_scenarios as sfs  # noqa: E402

BUILD = os.path.join(sfs.ROOT, "_build", "fake")


@pytest.fixture(scope="module")
def fake():
    return sfs.Fake(sfs.build(os.path.join(BUILD, "libfftcg_fake.so")))


@pytest.mark.parametrize("scenario", sfs.ALL, ids=lambda s: s.__name__)
def test_scheduler_on_simulated_device(fake, scenario):
    scenario(fake)


@pytest.mark.slow
def test_scheduler_under_thread_sanitizer():
    rt = sfs.tsan_runtime()
    if rt is None:
        pytest.skip("no clang ThreadSanitizer runtime")
    lib = sfs.build(os.path.join(BUILD, "libfftcg_fake_tsan.so"), tsan=True)
    env = dict(os.environ, LD_PRELOAD=rt, TSAN_OPTIONS="halt_on_error=1 report_signal_unsafe=0")
    p = subprocess.run([sys.executable, os.path.join(sfs.ROOT, "tests", "server_fake_scenarios.py"), lib], env=env,
                       capture_output=True, text=True, timeout=900)
    assert p.returncode == 0 and "FAKE_OK" in p.stdout, p.stdout[-3000:] + p.stderr[-5000:]
