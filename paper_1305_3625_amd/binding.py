"""ctypes binding of libfftcg.so (include/fftcg.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  Device arrays are torch tensors on the current HIP device
(float64, contiguous, shape (L, L)); streams are torch streams.  When the
library is not built, ``load()`` raises ``LibraryNotBuilt``; nothing here
falls back to a CPU path.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfftcg.so")

OK, PENDING = 0, 1
EINVAL, ENOMEM, ENOTSPD, ENOCONV, EBREAKDOWN = -1, -2, -3, -4, -5
EAGAIN, EDEVICE, ENOTFOUND, ECANCELED = -6, -7, -8, -9
FP64, MIXED = 0, 1
ENGINE_AUTO, ENGINE_MULTIPASS, ENGINE_FUSED = 0, 1, 2
PRECOND_NONE, PRECOND_CIRCULANT = 0, 1
GRID_UNSUPPORTED, GRID_OFF, GRID_ON, GRID_FELL_BACK, GRID_ON_TURN = 0, 1, 2, 3, 4

STATUS_NAMES = {0: "OK", 1: "PENDING", -1: "EINVAL", -2: "ENOMEM", -3: "ENOTSPD", -4: "ENOCONV",
                -5: "EBREAKDOWN", -6: "EAGAIN", -7: "EDEVICE", -8: "ENOTFOUND", -9: "ECANCELED"}

# every symbol include/fftcg.h declares
EXPORTS = [
    "fftcg_plan", "fftcg_plan_destroy", "fftcg_plan_set_engine", "fftcg_plan_set_precond",
    "fftcg_plan_set_error_target", "fftcg_plan_set_grid_sync", "fftcg_plan_get_grid_sync", "fftcg_plan_info",
    "fftcg_apply", "fftcg_profile_apply", "fftcg_profile_iteration", "fftcg_stream_probe", "fftcg_solve", "fftcg_loadstep", "fftcg_loadstep_noalloc", "fftcg_fracture",
    "fftcg_server_create", "fftcg_submit", "fftcg_submit_sequence", "fftcg_poll",
    "fftcg_poll_sequence", "fftcg_server_completed", "fftcg_server_get_stats", "fftcg_server_reserve", "fftcg_server_class_slots", "fftcg_server_shutdown",
    "fftcg_server_destroy",
    "fftcg_strerror", "fftcg_version", "fftcg_greens_spectrum",
]


class LibraryNotBuilt(RuntimeError):
    pass


class FftcgError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} ({status})")


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_int),
                ("iterations_literal", ctypes.c_int), ("checks", ctypes.c_int),
                ("true_relres", ctypes.c_double), ("error_bound", ctypes.c_double),
                ("lambda_lb", ctypes.c_double), ("device_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerOpts(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_size_t), ("max_slots", ctypes.c_int),
                ("chunk_iters", ctypes.c_int), ("refresh_period", ctypes.c_int),
                ("queue_cap", ctypes.c_int), ("device", ctypes.c_int), ("graphs", ctypes.c_int)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("canceled", ctypes.c_uint64), ("bytes_in_use", ctypes.c_size_t),
                ("queued", ctypes.c_int), ("in_flight", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Loads the library once and declares every signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise LibraryNotBuilt(f"{path} not built; run python -m paper_1305_3625_amd.build")
    # torch ships its own HIP runtime (SONAME libamdhip64.so.7).  Loading it
    # first makes the library bind to that same runtime, so torch's device
    # pointers and streams are valid inside the library; loading the library
    # first would bring a second HIP runtime into the process.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    U64P = ctypes.POINTER(ctypes.c_uint64)
    sig = {
        "fftcg_plan": (I, [I, I, P, ctypes.POINTER(P)]),
        "fftcg_plan_destroy": (I, [P]),
        "fftcg_plan_set_engine": (I, [P, I]),
        "fftcg_plan_set_precond": (I, [P, I]),
        "fftcg_plan_set_error_target": (I, [P, I, D]),
        "fftcg_plan_set_grid_sync": (I, [P, I]),
        "fftcg_plan_get_grid_sync": (I, [P, I, ctypes.POINTER(I)]),
        "fftcg_plan_info": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I),
                                ctypes.POINTER(S)]),
        "fftcg_apply": (I, [P, I, P, P, P, P]),
        "fftcg_profile_apply": (I, [P, I, P, P, P, I, ctypes.POINTER(D), P]),
        "fftcg_profile_iteration": (I, [P, I, P, P, P, I, ctypes.POINTER(D), ctypes.POINTER(I), P]),
        "fftcg_solve": (I, [P, I, P, P, P, D, I, P, ctypes.POINTER(Info), P]),
        "fftcg_loadstep": (I, [P, P, P, P, ctypes.POINTER(I), P]),
        "fftcg_loadstep_noalloc": (I, [P, P, P, P, ctypes.POINTER(I), P]),
        "fftcg_server_create": (I, [ctypes.POINTER(ServerOpts), ctypes.POINTER(P)]),
        "fftcg_submit": (I, [P, P, I, P, P, P, D, I, U64P]),
        "fftcg_submit_sequence": (I, [P, P, I, P, P, P, D, I, I, U64P]),
        "fftcg_poll": (I, [P, ctypes.c_uint64, P, ctypes.POINTER(Info)]),
        "fftcg_poll_sequence": (I, [P, ctypes.c_uint64, P, P, P, P, ctypes.POINTER(Info)]),
        "fftcg_stream_probe": (I, [I, I, P, P, S, I, I, ctypes.POINTER(D), P]),
        "fftcg_server_completed": (I, [P, ctypes.POINTER(ctypes.c_uint64), I, ctypes.POINTER(I)]),
        "fftcg_server_get_stats": (I, [P, ctypes.POINTER(ServerStats)]),
        "fftcg_server_reserve": (I, [P, P, I, I]),
        "fftcg_server_class_slots": (I, [P, P, I, ctypes.POINTER(I)]),
        "fftcg_server_shutdown": (I, [P]),
        "fftcg_server_destroy": (I, [P]),
        "fftcg_fracture": (I, [P, I, ctypes.c_double, P, I, ctypes.c_double, I, P, P, P, P, P]),
        "fftcg_strerror": (ctypes.c_char_p, [I]),
        "fftcg_version": (ctypes.c_char_p, []),
        "fftcg_greens_spectrum": (I, [I, I, ctypes.c_double, ctypes.c_double, ctypes.c_double, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def stream_probe(kind, dst, src, bytes_, blocks, reps=10, nontemporal=False, stream=None):
    """fftcg_stream_probe: mean device ms per launch of a streaming kernel
    (kind 0 read, 1 write, 2 copy) over `bytes_` of device buffers."""
    ms = ctypes.c_double()
    st = load().fftcg_stream_probe(int(kind), int(bool(nontemporal)), _ptr(dst), _ptr(src), int(bytes_),
                                   int(blocks), int(reps), ctypes.byref(ms), _stream(stream))
    if st != OK:
        raise FftcgError(st, "fftcg_stream_probe")
    return ms.value


def greens_spectrum(L, padded, nu, E, a):
    """fftcg_greens_spectrum: spectrum of the Green's function of eq. (1c) on
    the M x M grid (numpy array)."""
    import numpy as np
    M = 2 * L if padded else L
    out = np.empty((M, M))
    st = load().fftcg_greens_spectrum(int(L), int(padded), float(nu), float(E), float(a),
                                      out.ctypes.data_as(ctypes.c_void_p))
    if st != OK:
        raise FftcgError(st, "fftcg_greens_spectrum")
    return out


def strerror(status: int) -> str:
    return load().fftcg_strerror(status).decode()


def _ptr(t):
    """Device pointer of a contiguous float64 torch tensor on a HIP device."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a tensor on the GPU")
    if t.dtype.is_floating_point and t.element_size() != 8:
        raise ValueError("expected float64")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _host(a):
    """Pointer to a C-contiguous float64 numpy array (host)."""
    import numpy as np
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.c_void_p)


class Plan:
    """fftcg_plan: spectral operator of one grid (L, padded, ghat)."""

    def __init__(self, L: int, padded: int, ghat):
        import numpy as np
        lib = load()
        g = np.ascontiguousarray(ghat, dtype=np.float64)
        h = ctypes.c_void_p()
        st = lib.fftcg_plan(int(L), int(padded), g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h))
        if st != OK:
            raise FftcgError(st, "fftcg_plan")
        self.h = h
        self.L, self.padded = int(L), int(padded)
        self.M = 2 * self.L if padded else self.L

    def set_engine(self, engine: int):
        st = load().fftcg_plan_set_engine(self.h, engine)
        if st != OK:
            raise FftcgError(st, "fftcg_plan_set_engine")

    def set_precond(self, kind: int):
        st = load().fftcg_plan_set_precond(self.h, kind)
        if st != OK:
            raise FftcgError(st, "fftcg_plan_set_precond")

    def set_error_target(self, precision: int, tau: float):
        """Fixes the certified error target of `precision` (0: follow tol)."""
        st = load().fftcg_plan_set_error_target(self.h, int(precision), float(tau))
        if st != OK:
            raise FftcgError(st, "fftcg_plan_set_error_target")

    def set_grid_sync(self, mode: int):
        """Update folded into the row-inverse pass behind a grid barrier:
        1 on (default; with the turn pass where it fits), 0 off, 2 as 1 with a
        zero wait limit (fallback tests), 3 on without the turn pass."""
        st = load().fftcg_plan_set_grid_sync(self.h, int(mode))
        if st != OK:
            raise FftcgError(st, "fftcg_plan_set_grid_sync")

    def grid_sync(self, precision: int) -> int:
        """One of GRID_UNSUPPORTED, GRID_OFF, GRID_ON, GRID_FELL_BACK, GRID_ON_TURN."""
        v = ctypes.c_int()
        st = load().fftcg_plan_get_grid_sync(self.h, int(precision), ctypes.byref(v))
        if st != OK:
            raise FftcgError(st, "fftcg_plan_get_grid_sync")
        return v.value

    def info(self):
        L, M, p = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        b = ctypes.c_size_t()
        st = load().fftcg_plan_info(self.h, ctypes.byref(L), ctypes.byref(M), ctypes.byref(p), ctypes.byref(b))
        if st != OK:
            raise FftcgError(st, "fftcg_plan_info")
        return dict(L=L.value, M=M.value, padded=p.value, device_bytes=b.value)

    def fracture(self, k, t, f, steps, tol=1e-8, maxit=10000, precision=MIXED, stream=None):
        """fftcg_fracture: returns (status, broken, dbreak, iters) host arrays."""
        import numpy as np
        broken = np.zeros(steps, dtype=np.int32)
        dbreak = np.zeros(steps)
        iters = np.zeros(steps, dtype=np.int32)
        st = load().fftcg_fracture(self.h, precision, float(k), _ptr(t), int(steps), float(tol), int(maxit), _ptr(f),
                                   broken.ctypes.data_as(ctypes.c_void_p), dbreak.ctypes.data_as(ctypes.c_void_p),
                                   iters.ctypes.data_as(ctypes.c_void_p), _stream(stream))
        return st, broken, dbreak, iters

    def close(self):
        if getattr(self, "h", None) is not None:
            st = load().fftcg_plan_destroy(self.h)
            if st != OK:
                raise FftcgError(st, "fftcg_plan_destroy")
            self.h = None

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None:
                load().fftcg_plan_destroy(self.h)
        except Exception:
            pass

    # -- device calls ------------------------------------------------------
    def apply(self, d, x, y, precision=FP64, stream=None):
        st = load().fftcg_apply(self.h, precision, _ptr(d), _ptr(x), _ptr(y), _stream(stream))
        if st != OK:
            raise FftcgError(st, "fftcg_apply")
        return y

    def profile_apply(self, d, x, y, reps=20, precision=FP64, stream=None):
        """Mean device ms of the three passes of one product (HIP events)."""
        ms = (ctypes.c_double * 3)()
        st = load().fftcg_profile_apply(self.h, precision, _ptr(d), _ptr(x), _ptr(y), int(reps), ms,
                                        _stream(stream))
        if st != OK:
            raise FftcgError(st, "fftcg_profile_apply")
        return [ms[0], ms[1], ms[2]]

    def profile_iteration(self, d, b, x, reps=20, precision=MIXED, stream=None):
        """Mean device ms per launch of the CG iteration's passes (row_fwd,
        col, row_inv, separate update, turn) over `reps` iterations from
        x = 0, and 0 / 1 / 2: separate update / folded / folded with the turn
        pass; x is scratch."""
        ms = (ctypes.c_double * 5)()
        folded = ctypes.c_int()
        st = load().fftcg_profile_iteration(self.h, precision, _ptr(d), _ptr(b), _ptr(x), int(reps), ms,
                                            ctypes.byref(folded), _stream(stream))
        if st != OK:
            raise FftcgError(st, "fftcg_profile_iteration")
        return [ms[0], ms[1], ms[2], ms[3], ms[4]], int(folded.value)

    def solve(self, d, b, x, x0=None, tol=1e-10, maxit=10000, precision=FP64, stream=None,
              raise_on_error=True):
        info = Info()
        st = load().fftcg_solve(self.h, precision, _ptr(d), _ptr(b), _ptr(x0), float(tol), int(maxit),
                                _ptr(x), ctypes.byref(info), _stream(stream))
        if st not in (OK,) and raise_on_error and st != ENOCONV:
            raise FftcgError(st, "fftcg_solve")
        out = info.as_dict()
        out["status"] = st
        return out

    def loadstep(self, x, t, d, stream=None):
        idx = ctypes.c_int(-2)
        st = load().fftcg_loadstep(self.h, _ptr(x), _ptr(t), _ptr(d), ctypes.byref(idx), _stream(stream))
        if st != OK:
            raise FftcgError(st, "fftcg_loadstep")
        return idx.value

    def loadstep_noalloc(self, x, t, d, stream=None):
        """fftcg_loadstep with no allocation (the library's static scratch)."""
        idx = ctypes.c_int(-2)
        st = load().fftcg_loadstep_noalloc(self.h, _ptr(x), _ptr(t), _ptr(d), ctypes.byref(idx),
                                           _stream(stream))
        if st != OK:
            raise FftcgError(st, "fftcg_loadstep_noalloc")
        return idx.value


@dataclass
class Result:
    status: int
    x: object
    info: dict


class Server:
    """fftcg_server_*: continuous-batching solve server (host arrays)."""

    def __init__(self, memory_budget=4 << 30, max_slots=0, chunk_iters=0, refresh_period=0,
                 queue_cap=0, device=0, graphs=True):
        lib = load()
        o = ServerOpts(memory_budget, max_slots, chunk_iters, refresh_period, queue_cap, device,
                       0 if graphs else -1)
        h = ctypes.c_void_p()
        st = lib.fftcg_server_create(ctypes.byref(o), ctypes.byref(h))
        if st != OK:
            raise FftcgError(st, "fftcg_server_create")
        self.h = h

    def submit(self, plan: Plan, d, b, x0=None, tol=1e-8, maxit=10000, precision=MIXED):
        dd, dp = _host(d)
        bb, bp = _host(b)
        xp = None
        if x0 is not None:
            xx, xp = _host(x0)
        t = ctypes.c_uint64()
        st = load().fftcg_submit(self.h, plan.h, precision, dp, bp, xp, float(tol), int(maxit), ctypes.byref(t))
        return st, t.value

    def submit_sequence(self, plan: Plan, d, b, t, steps, tol=1e-8, maxit=10000, precision=MIXED):
        dd, dp = _host(d)
        bb, bp = _host(b)
        tt, tp = _host(t)
        tk = ctypes.c_uint64()
        st = load().fftcg_submit_sequence(self.h, plan.h, precision, dp, bp, tp, float(tol), int(maxit),
                                          int(steps), ctypes.byref(tk))
        return st, tk.value

    def poll(self, ticket, L):
        import numpy as np
        x = np.empty((L, L))
        info = Info()
        st = load().fftcg_poll(self.h, ctypes.c_uint64(ticket), x.ctypes.data_as(ctypes.c_void_p),
                               ctypes.byref(info))
        return Result(st, x if st in (OK, ENOCONV) else None, info.as_dict())

    def poll_sequence(self, ticket, L, steps, bounds=False):
        """x is (x, broken, iters), or (x, broken, iters, step_bounds) with bounds=True."""
        import numpy as np
        x = np.empty((L, L))
        broken = np.empty(steps, dtype=np.int32)
        iters = np.empty(steps, dtype=np.int32)
        eb = np.empty(steps)
        info = Info()
        st = load().fftcg_poll_sequence(self.h, ctypes.c_uint64(ticket), x.ctypes.data_as(ctypes.c_void_p),
                                        broken.ctypes.data_as(ctypes.c_void_p),
                                        iters.ctypes.data_as(ctypes.c_void_p), eb.ctypes.data_as(ctypes.c_void_p),
                                        ctypes.byref(info))
        if st in (OK, ENOCONV):
            return Result(st, (x, broken, iters, eb) if bounds else (x, broken, iters), info.as_dict())
        return Result(st, None, info.as_dict())

    def completed(self, cap=4096):
        """Tickets finished since the last call (each reported once)."""
        out = (ctypes.c_uint64 * cap)()
        n = ctypes.c_int()
        st = load().fftcg_server_completed(self.h, out, int(cap), ctypes.byref(n))
        if st != OK:
            raise FftcgError(st, "fftcg_server_completed")
        return list(out[:n.value])

    def stats(self):
        s = ServerStats()
        st = load().fftcg_server_get_stats(self.h, ctypes.byref(s))
        if st != OK:
            raise FftcgError(st, "fftcg_server_get_stats")
        return s.as_dict()

    def reserve(self, plan, slots, precision=MIXED):
        """Makes the server hold `slots` slots (and pinned buffers) for this
        plan and precision before requests arrive; blocks until done."""
        st = load().fftcg_server_reserve(self.h, plan.h, int(precision), int(slots))
        if st != OK:
            raise FftcgError(st, "fftcg_server_reserve")

    def class_slots(self, plan, precision=MIXED):
        """Slots the server holds for this plan and precision."""
        v = ctypes.c_int()
        st = load().fftcg_server_class_slots(self.h, plan.h, int(precision), ctypes.byref(v))
        if st != OK:
            raise FftcgError(st, "fftcg_server_class_slots")
        return v.value

    def shutdown(self):
        """Stops the server: unfinished requests end ECANCELED, results stay pollable."""
        st = load().fftcg_server_shutdown(self.h)
        if st != OK:
            raise FftcgError(st, "fftcg_server_shutdown")

    def close(self):
        if getattr(self, "h", None) is not None:
            load().fftcg_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
