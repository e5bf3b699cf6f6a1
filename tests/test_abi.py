"""The C ABI on the CPU: the library loads, exports every symbol the header
declares, and rejects invalid arguments before touching a device."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1305_3625_amd import binding
from workloads import spectrum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fftcg.h")


def header_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fftcg_[a-z_]+)\s*\(", src)))


def test_header_matches_binding_list():
    assert header_symbols() == sorted(binding.EXPORTS)


def test_library_exports_every_symbol(lib):
    for name in header_symbols():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (fftcg_\w+)", out))
    assert set(header_symbols()) <= exported


def test_strerror_and_version(lib):
    assert binding.strerror(0) == "ok"
    assert "invalid" in binding.strerror(-1)
    assert binding.strerror(12345) == "unknown status"
    assert lib.fftcg_version().decode().startswith("fftcg")


def _plan(lib, L, padded, g):
    h = ctypes.c_void_p()
    gp = None if g is None else np.ascontiguousarray(g).ctypes.data_as(ctypes.c_void_p)
    return lib.fftcg_plan(L, padded, gp, ctypes.byref(h))


@pytest.mark.parametrize("L,padded", [(0, 0), (3, 0), (6, 1), (16384, 0), (8192, 1), (1, 0), (8, 2), (8, -1)])
def test_plan_rejects_bad_sizes(lib, L, padded):
    M = max(2, 2 * L if padded == 1 else max(L, 1))
    # sizes are checked before the spectrum is read: past M = 8192 a small
    # buffer stands in
    g = np.ones((M, M)) if M <= 8192 else np.ones((2, 2))
    assert _plan(lib, L, padded, g) == binding.EINVAL


def test_plan_rejects_null(lib):
    assert _plan(lib, 8, 0, None) == binding.EINVAL
    g = spectrum(8, 1e-2)
    assert lib.fftcg_plan(8, 0, g.ctypes.data_as(ctypes.c_void_p), None) == binding.EINVAL


def test_plan_rejects_non_even_and_non_finite(lib):
    g = spectrum(16, 1e-2).copy()
    g[1, 2] *= 1.01          # breaks evenness in m (g[15, 2] unchanged)
    assert _plan(lib, 16, 0, g) == binding.EINVAL
    g = spectrum(16, 1e-2).copy()
    g[3, 3] = np.nan
    assert _plan(lib, 16, 0, g) == binding.EINVAL
    g = spectrum(32, 1e-2).copy()
    g[0, 0] = np.inf
    assert _plan(lib, 16, 1, g) == binding.EINVAL


def test_plan_rejects_non_positive(lib):
    g = spectrum(16, 1e-2) - 1.0     # even, finite, has negative entries
    assert _plan(lib, 16, 0, g) == binding.ENOTSPD
    g = np.zeros((16, 16))
    assert _plan(lib, 16, 0, g) == binding.ENOTSPD


def test_valid_plan_without_gpu_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    assert _plan(lib, 8, 0, spectrum(8, 1e-2)) == binding.EDEVICE


def test_null_plan_calls(lib):
    P = ctypes.c_void_p
    info = binding.Info()
    assert lib.fftcg_apply(None, 0, P(1), P(2), P(3), None) == binding.EINVAL
    assert lib.fftcg_solve(None, 0, P(1), P(2), None, 1e-8, 10, P(3), ctypes.byref(info), None) == binding.EINVAL
    assert lib.fftcg_plan_destroy(None) == binding.EINVAL
    assert lib.fftcg_plan_set_engine(None, 0) == binding.EINVAL
    assert lib.fftcg_plan_info(None, None, None, None, None) == binding.EINVAL
    idx = ctypes.c_int()
    assert lib.fftcg_loadstep(None, P(1), P(2), P(3), ctypes.byref(idx), None) == binding.EINVAL


def test_server_calls_without_server(lib):
    P = ctypes.c_void_p
    tk = ctypes.c_uint64()
    assert lib.fftcg_server_create(None, None) == binding.EINVAL
    assert lib.fftcg_submit(None, None, 0, P(1), P(2), None, 1e-8, 10, ctypes.byref(tk)) == binding.EINVAL
    assert lib.fftcg_poll(None, 1, None, None) == binding.EINVAL
    assert lib.fftcg_server_destroy(None) == binding.EINVAL
    assert lib.fftcg_server_get_stats(None, None) == binding.EINVAL
    o = binding.ServerOpts(0, 0, 0, 0, 0, 0)
    h = ctypes.c_void_p()
    assert lib.fftcg_server_create(ctypes.byref(o), ctypes.byref(h)) == binding.EINVAL   # zero budget


def test_server_create_without_gpu(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    o = binding.ServerOpts(1 << 30, 0, 0, 0, 0, 0)
    h = ctypes.c_void_p()
    assert lib.fftcg_server_create(ctypes.byref(o), ctypes.byref(h)) == binding.EDEVICE


def test_new_calls_reject_null(lib):
    P = ctypes.c_void_p
    idx = ctypes.c_int()
    assert lib.fftcg_loadstep_noalloc(None, P(1), P(2), P(3), ctypes.byref(idx), None) == binding.EINVAL
    assert lib.fftcg_plan_set_error_target(None, 0, 1e-10) == binding.EINVAL
    assert lib.fftcg_plan_set_grid_sync(None, 1) == binding.EINVAL
    assert lib.fftcg_server_reserve(None, P(1), binding.MIXED, 4) == binding.EINVAL
    assert lib.fftcg_server_class_slots(None, P(1), binding.MIXED, ctypes.byref(idx)) == binding.EINVAL
    ms = (ctypes.c_double * 5)()
    assert lib.fftcg_profile_iteration(None, binding.MIXED, P(1), P(2), P(3), 10, ms, None, None) == binding.EINVAL
    st = ctypes.c_int(-1)
    assert lib.fftcg_plan_get_grid_sync(None, binding.MIXED, ctypes.byref(st)) == binding.EINVAL
    assert st.value == -1
    assert lib.fftcg_server_shutdown(None) == binding.EINVAL


CSRC = os.path.join(ROOT, "paper_1305_3625_amd", "csrc")


def test_every_entry_point_catches_exceptions():
    """Nothing throws across the C ABI: every int-returning entry point is a
    function-try-block whose handlers map exceptions to status codes."""
    found = []
    for name in sorted(os.listdir(CSRC)):
        if not name.endswith((".cpp", ".hip")):
            continue
        src = open(os.path.join(CSRC, name)).read()
        for m in re.finditer(r'extern "C" int (fftcg_\w+)\([^{;]*\)\s*(try)?\s*\{', src):
            found.append(m.group(1))
            assert m.group(2) == "try", f"{name}: {m.group(1)} is not guarded"
            # the body's closing brace is followed by the handlers
            depth, i = 0, m.end() - 1
            while True:
                depth += {"{": 1, "}": -1}.get(src[i], 0)
                if depth == 0:
                    break
                i += 1
            assert src[i + 1:i + 40].lstrip().startswith("FFTCG_ABI_CATCH"), m.group(1)
    declared = [s for s in header_symbols() if s not in ("fftcg_strerror", "fftcg_version")]
    assert sorted(found) == sorted(declared)


def test_header_constants_match_binding():
    """Every integer constant the header defines (status codes, precisions,
    engines, preconditioners, grid-sync states) has the binding's constant of
    the same name (without the FFTCG_ prefix) and the same value, and the
    status names cover every status code."""
    with open(os.path.join(ROOT, "include", "fftcg.h")) as f:
        defs = dict(re.findall(r"^#define FFTCG_([A-Z0-9_]+)\s+(-?\d+)\b", f.read(), re.M))
    assert len(defs) == 23  # 11 status codes, 2 precisions, 3 engines, 2 preconditioners, 5 grid states
    for name, val in defs.items():
        assert hasattr(binding, name), name
        assert getattr(binding, name) == int(val), (name, getattr(binding, name), val)
    codes = {int(v) for k, v in defs.items() if k in ("OK", "PENDING") or re.fullmatch(r"E[A-Z]+", k)}
    assert codes == set(binding.STATUS_NAMES)
