"""Drives every C entry point of a host-sanitizer build of the library
through the paths that need no GPU: argument and input validation, the
host-side spectrum construction, status strings.  Run by
tests/test_sanitize.py in a child process with the sanitizer runtime
preloaded; exits non-zero (the sanitizer aborts) on a memory or
undefined-behaviour error."""

import ctypes
import sys

import numpy as np

lib = ctypes.CDLL(sys.argv[1])
P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
EINVAL, ENOTSPD, EDEVICE = -1, -3, -7


def ptr(a):
    return a.ctypes.data_as(P)


def spectrum(M, eps):
    m = np.arange(M)
    c = np.cos(2 * np.pi * np.minimum(m, (M - m) % M) / M)
    return 1.0 / np.sqrt(4.0 - 2.0 * (c[:, None] + c[None, :]) + eps)


h = P()
lib.fftcg_plan.argtypes = [I, I, P, ctypes.POINTER(P)]
for L, pad in [(0, 0), (3, 0), (6, 1), (16384, 0), (8192, 1), (1, 0), (8, 2), (8, -1)]:
    assert lib.fftcg_plan(L, pad, ptr(np.ones(4)), ctypes.byref(h)) == EINVAL, (L, pad)
assert lib.fftcg_plan(8, 0, None, ctypes.byref(h)) == EINVAL
assert lib.fftcg_plan(8, 0, ptr(spectrum(8, 1e-2)), None) == EINVAL
bad = spectrum(16, 1e-2)
bad[1, 2] += 0.5  # not even
assert lib.fftcg_plan(16, 0, ptr(bad), ctypes.byref(h)) == EINVAL
bad = spectrum(16, 1e-2)
bad[3, 3] = np.nan
assert lib.fftcg_plan(16, 0, ptr(bad), ctypes.byref(h)) == EINVAL
assert lib.fftcg_plan(16, 0, ptr(spectrum(16, 1e-2) - 1.0), ctypes.byref(h)) == ENOTSPD
# a valid spectrum is read in full, then the missing GPU is reported
for L, pad in [(16, 0), (2048, 1), (8192, 0)]:
    M = 2 * L if pad else L
    assert lib.fftcg_plan(L, pad, ptr(spectrum(M, 1e-3)), ctypes.byref(h)) == EDEVICE, (L, pad)

# the physical Green's function spectrum: computed on the host in full
lib.fftcg_greens_spectrum.argtypes = [I, I, D, D, D, P]
for L, pad in [(2, 0), (8, 1), (64, 1), (128, 0)]:
    M = 2 * L if pad else L
    out = np.empty((M, M))
    assert lib.fftcg_greens_spectrum(L, pad, 0.25, 1.0, 1.0, ptr(out)) == 0
    assert np.all(np.isfinite(out)) and out.min() > 0
assert lib.fftcg_greens_spectrum(8, 1, 1.0, 1.0, 1.0, ptr(np.empty((16, 16)))) == EINVAL
assert lib.fftcg_greens_spectrum(8, 1, 0.2, -1.0, 1.0, ptr(np.empty((16, 16)))) == EINVAL

# every other entry point: invalid handles and arguments
info = (ctypes.c_byte * 64)()
idx = I()
tk = ctypes.c_uint64()
n = I()
one = ptr(np.ones(4))
for name, args in [
    ("fftcg_plan_destroy", [None]), ("fftcg_plan_set_engine", [None, 0]), ("fftcg_plan_set_precond", [None, 0]),
    ("fftcg_plan_set_error_target", [None, 0, D(1e-10)]), ("fftcg_plan_info", [None, None, None, None, None]),
    ("fftcg_apply", [None, 0, one, one, one, None]),
    ("fftcg_profile_apply", [None, 0, one, one, one, 1, one, None]),
    ("fftcg_solve", [None, 0, one, one, None, D(1e-8), 10, one, info, None]),
    ("fftcg_loadstep", [None, one, one, one, ctypes.byref(idx), None]),
    ("fftcg_loadstep_noalloc", [None, one, one, one, ctypes.byref(idx), None]),
    ("fftcg_fracture", [None, 0, D(1.0), one, 4, D(1e-8), 10, one, one, one, None, None]),
    ("fftcg_server_create", [None, None]),
    ("fftcg_submit", [None, None, 0, one, one, None, D(1e-8), 10, ctypes.byref(tk)]),
    ("fftcg_submit_sequence", [None, None, 1, one, one, one, D(1e-8), 10, 4, ctypes.byref(tk)]),
    ("fftcg_poll", [None, ctypes.c_uint64(1), None, None]),
    ("fftcg_poll_sequence", [None, ctypes.c_uint64(1), None, None, None, None, None]),
    ("fftcg_server_completed", [None, None, 0, ctypes.byref(n)]),
    ("fftcg_server_get_stats", [None, None]),
    ("fftcg_server_shutdown", [None]), ("fftcg_server_destroy", [None]),
    ("fftcg_stream_probe", [3, 0, one, one, S(16), 1, 1, one, None]),
]:
    f = getattr(lib, name)
    f.restype = I
    assert f(*args) == EINVAL, name


class Opts(ctypes.Structure):
    _fields_ = [("memory_budget", S), ("max_slots", I), ("chunk_iters", I), ("refresh_period", I),
                ("queue_cap", I), ("device", I), ("graphs", I)]


srv = P()
assert lib.fftcg_server_create(ctypes.byref(Opts(0, 0, 0, 0, 0, 0, 0)), ctypes.byref(srv)) == EINVAL
assert lib.fftcg_server_create(ctypes.byref(Opts(1 << 30, 0, 0, 0, 0, 0, 2)), ctypes.byref(srv)) == EINVAL
assert lib.fftcg_server_create(ctypes.byref(Opts(1 << 30, 0, 0, 0, 0, 0, 0)), ctypes.byref(srv)) == EDEVICE
lib.fftcg_strerror.restype = ctypes.c_char_p
for code in range(-12, 3):
    assert lib.fftcg_strerror(code)
lib.fftcg_version.restype = ctypes.c_char_p
assert lib.fftcg_version().startswith(b"fftcg")
print("SANITIZE_OK", flush=True)
