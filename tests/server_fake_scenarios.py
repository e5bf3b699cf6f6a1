"""Scenarios for the server's scheduler on a simulated device: the unmodified
server.cpp compiled by g++ against tests/fake_hip (a test double of the HIP
runtime) with tests/fake_hip/fake_exec.cpp.  Used by tests/test_server_fake.py
in-process and, under ThreadSanitizer, in a child process:

    python tests/server_fake_scenarios.py LIB

A fake solve finishes after target(b) = 3 + (int)(1000 |b_0|) % 37
iterations with x = b / 2 (at maxit: FFTCG_ENOCONV, x = b / 4); the load
step applies the real rule (argmax of x / t over d != 0)."""

import ctypes
import os
import subprocess
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OK, PENDING, EINVAL, ENOMEM, ENOCONV, EAGAIN, ENOTFOUND, ECANCELED = 0, 1, -1, -2, -4, -6, -8, -9
P, I, D, S, U64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_uint64


CLANG = sorted(__import__("glob").glob("/opt/rocm*/lib/llvm/bin/clang++"))


def tsan_runtime():
    """clang's ThreadSanitizer runtime (it intercepts pthread_cond_clockwait,
    which std::condition_variable::wait_for uses and gcc 11's runtime does
    not, so that one reports false double locks)."""
    hits = sorted(__import__("glob").glob("/opt/rocm*/lib/llvm/lib/clang/*/lib/linux/libclang_rt.tsan-x86_64.so"))
    return hits[-1] if hits and CLANG else None


def build(out, tsan=False):
    """Host build of server.cpp + the simulated device (seconds): g++, or
    clang++ with ThreadSanitizer."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    srcs = [os.path.join(ROOT, "paper_1305_3625_amd", "csrc", "server.cpp"),
            os.path.join(ROOT, "tests", "fake_hip", "fake_exec.cpp")]
    flags = ["-std=c++17", "-O1", "-g", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
             "-I" + os.path.join(ROOT, "tests", "fake_hip"), "-I" + os.path.join(ROOT, "include"),
             "-I" + os.path.join(ROOT, "paper_1305_3625_amd", "csrc")]
    cxx = "g++"
    if tsan:
        flags += ["-fsanitize=thread", "-shared-libsan"]
        cxx = CLANG[-1]
    subprocess.run([cxx, *flags, *srcs, "-o", out, "-lpthread"], check=True)
    return out


class Info(ctypes.Structure):
    _fields_ = [("status", I), ("iterations", I), ("iterations_literal", I), ("checks", I),
                ("true_relres", D), ("error_bound", D), ("lambda_lb", D), ("device_ms", D)]


class Opts(ctypes.Structure):
    _fields_ = [("memory_budget", S), ("max_slots", I), ("chunk_iters", I), ("refresh_period", I),
                ("queue_cap", I), ("device", I), ("graphs", I)]


class Stats(ctypes.Structure):
    _fields_ = [("submitted", U64), ("admitted", U64), ("completed", U64), ("failed", U64),
                ("canceled", U64), ("bytes_in_use", S), ("queued", I), ("in_flight", I)]


class Fake:
    def __init__(self, path):
        self.lib = lib = ctypes.CDLL(path)
        lib.fftcg_fake_plan.argtypes = [I, I, ctypes.POINTER(P)]
        lib.fftcg_fake_plan_refs.argtypes = [P]
        lib.fftcg_fake_plan_free.argtypes = [P]
        lib.fftcg_fake_set_event_delay.argtypes = [I]
        lib.fftcg_fake_launches.restype = ctypes.c_long
        lib.fftcg_server_create.argtypes = [ctypes.POINTER(Opts), ctypes.POINTER(P)]
        lib.fftcg_submit.argtypes = [P, P, I, P, P, P, D, I, ctypes.POINTER(U64)]
        lib.fftcg_submit_sequence.argtypes = [P, P, I, P, P, P, D, I, I, ctypes.POINTER(U64)]
        lib.fftcg_poll.argtypes = [P, U64, P, ctypes.POINTER(Info)]
        lib.fftcg_poll_sequence.argtypes = [P, U64, P, P, P, P, ctypes.POINTER(Info)]
        lib.fftcg_server_completed.argtypes = [P, ctypes.POINTER(U64), I, ctypes.POINTER(I)]
        lib.fftcg_server_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
        lib.fftcg_server_shutdown.argtypes = [P]
        lib.fftcg_server_destroy.argtypes = [P]
        lib.fftcg_server_reserve.argtypes = [P, P, I, I]
        lib.fftcg_server_class_slots.argtypes = [P, P, I, ctypes.POINTER(I)]

    def plan(self, L, fused):
        h = P()
        assert self.lib.fftcg_fake_plan(L, fused, ctypes.byref(h)) == OK
        return h

    def server(self, budget=1 << 30, max_slots=0, chunk=0, queue_cap=0, graphs=0):
        h = P()
        assert self.lib.fftcg_server_create(ctypes.byref(Opts(budget, max_slots, chunk, 0, queue_cap, 0, graphs)),
                                            ctypes.byref(h)) == OK
        return h

    def submit(self, srv, plan, d, b, maxit=10000, precision=1):
        tk = U64()
        st = self.lib.fftcg_submit(srv, plan, precision, d.ctypes.data_as(P), b.ctypes.data_as(P), None, 1e-8,
                                   maxit, ctypes.byref(tk))
        return st, tk.value

    def poll(self, srv, tk, L):
        x = np.empty((L, L))
        info = Info()
        st = self.lib.fftcg_poll(srv, tk, x.ctypes.data_as(P), ctypes.byref(info))
        return st, x, info

    def stats(self, srv):
        s = Stats()
        assert self.lib.fftcg_server_get_stats(srv, ctypes.byref(s)) == OK
        return s

    def completed(self, srv):
        out = (U64 * 4096)()
        n = I()
        assert self.lib.fftcg_server_completed(srv, out, 4096, ctypes.byref(n)) == OK
        return list(out[:n.value])


def target(b):
    return 3 + int(1000.0 * abs(b.flat[0])) % 37


def request(rng, L):
    d = rng.uniform(0.5, 1.5, (L, L))
    b = rng.uniform(0.0, 1.0, (L, L))
    return d, b


def wait_all(f, srv, tickets, timeout=120.0):
    """tickets: {ticket: L}; returns {ticket: (status, x, info)}."""
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for tk, L in tickets.items():
            if tk not in out:
                r = f.poll(srv, tk, L)
                if r[0] != PENDING:
                    out[tk] = r
        assert time.time() - t0 < timeout, f"{len(tickets) - len(out)} pending"
        time.sleep(0.0005)
    return out


def scenario_mix_two_clients(f, n=600, graphs=0, delay=3):
    """Two client threads submit a mix of grid sizes (fused and multi-pass
    classes) while the scheduler runs; every result is exact, reported once
    as completed, and the budget holds throughout."""
    f.lib.fftcg_fake_set_event_delay(delay)
    plans = {8: f.plan(8, 1), 16: f.plan(16, 0), 32: f.plan(32, 0)}
    budget = 40 * (32 * 32 * 40 + 8192)
    srv = f.server(budget=budget, graphs=graphs)
    rng = np.random.default_rng([7, n])
    reqs = [(L,) + request(rng, L) for L in rng.choice([8, 16, 32], size=n)]
    tickets = {}
    lock = threading.Lock()

    def client(part):
        for L, d, b in part:
            st, tk = f.submit(srv, plans[L], d, b)
            assert st == OK
            with lock:
                tickets[tk] = (L, d, b)

    th = [threading.Thread(target=client, args=(reqs[i::2],)) for i in range(2)]
    for t in th:
        t.start()
    peak = 0
    while any(t.is_alive() for t in th):
        s = f.stats(srv)
        assert s.bytes_in_use <= budget
        peak = max(peak, s.in_flight)
        time.sleep(0.0002)
    for t in th:
        t.join()
    res = wait_all(f, srv, {tk: v[0] for tk, v in tickets.items()})
    for tk, (L, d, b) in tickets.items():
        st, x, info = res[tk]
        assert st == OK and info.status == OK, (tk, st)
        assert np.array_equal(x, 0.5 * b)
        assert info.iterations == target(b) and info.checks >= 1
        assert f.poll(srv, tk, L)[0] == ENOTFOUND
    seen = []
    while True:
        c = f.completed(srv)
        if not c:
            break
        seen += c
    assert sorted(seen) == sorted(tickets)
    s = f.stats(srv)
    assert (s.submitted, s.completed, s.failed, s.canceled, s.queued, s.in_flight) == (n, n, 0, 0, 0, 0)
    f.lib.fftcg_server_destroy(srv)
    for p in plans.values():
        assert f.lib.fftcg_fake_plan_refs(p) == 0
        f.lib.fftcg_fake_plan_free(p)
    return peak


def scenario_budget(f):
    """A budget of 2.5 slot footprints: at most two solves are admitted at a
    time, and every request completes."""
    plan = f.plan(16, 0)
    foot = 16 * 16 * 40 + 8192 + 4 * 16 * 16 * 8 + 4 * 1024 + 4096
    srv = f.server(budget=int(2.5 * foot))
    rng = np.random.default_rng([8, 0])
    tks = {}
    for _ in range(40):
        d, b = request(rng, 16)
        st, tk = f.submit(srv, plan, d, b)
        assert st == OK
        tks[tk] = b
    t0 = time.time()
    done = {}
    while len(done) < len(tks):
        s = f.stats(srv)
        assert s.in_flight <= 2 and s.bytes_in_use <= int(2.5 * foot)
        for tk, b in tks.items():
            if tk not in done:
                r = f.poll(srv, tk, 16)
                if r[0] != PENDING:
                    done[tk] = r
        assert time.time() - t0 < 60
    assert all(r[0] == OK and np.array_equal(r[1], 0.5 * tks[tk]) for tk, r in done.items())
    f.lib.fftcg_server_destroy(srv)
    f.lib.fftcg_fake_plan_free(plan)


def scenario_queue_cap_and_maxit(f):
    """A queue of two: a burst meets EAGAIN; requests whose maxit is below
    their iteration count end FFTCG_ENOCONV with the last iterate, the others
    are unaffected."""
    f.lib.fftcg_fake_set_event_delay(2000)  # chunks complete slowly: a burst fills the queue
    plan = f.plan(8, 1)
    srv = f.server(max_slots=1, queue_cap=2)
    rng = np.random.default_rng([9, 0])
    sts, tks = [], {}
    for k in range(30):
        d, b = request(rng, 8)
        maxit = 2 if k % 3 == 0 else 10000
        while True:
            st, tk = f.submit(srv, plan, d, b, maxit=maxit)
            sts.append(st)
            if st == OK:
                tks[tk] = (b, maxit)
                break
            assert st == EAGAIN
            time.sleep(0.0005)
    assert EAGAIN in sts
    res = wait_all(f, srv, {tk: 8 for tk in tks})
    for tk, (b, maxit) in tks.items():
        st, x, info = res[tk]
        if maxit < target(b):
            assert st == ENOCONV and np.array_equal(x, 0.25 * b) and info.iterations == maxit
        else:
            assert st == OK and np.array_equal(x, 0.5 * b)
    f.lib.fftcg_server_destroy(srv)
    f.lib.fftcg_fake_plan_free(plan)
    f.lib.fftcg_fake_set_event_delay(0)


def scenario_invalid_inputs(f):
    """Non-finite or out-of-range inputs are refused at submission (checked
    while they are copied), and nothing is queued for them."""
    plan = f.plan(8, 1)
    srv = f.server()
    rng = np.random.default_rng([12, 0])
    d, b = request(rng, 8)
    for bad_d, bad_b in [(-1.0, None), (np.inf, None), (None, np.nan), (None, -np.inf)]:
        dd, bb = d.copy(), b.copy()
        if bad_d is not None:
            dd[3, 5] = bad_d
        if bad_b is not None:
            bb[7, 7] = bad_b
        assert f.submit(srv, plan, dd, bb)[0] == EINVAL
    t = rng.uniform(0.1, 1.0, (8, 8))
    t[0, 0] = 0.0
    tk = U64()
    assert f.lib.fftcg_submit_sequence(srv, plan, 1, d.ctypes.data_as(P), b.ctypes.data_as(P),
                                       t.ctypes.data_as(P), 1e-8, 100, 4, ctypes.byref(tk)) == EINVAL
    st, tk = f.submit(srv, plan, d, b)  # a valid one still goes through
    assert st == OK
    res = wait_all(f, srv, {tk: 8})
    assert res[tk][0] == OK and np.array_equal(res[tk][1], 0.5 * b)
    s = f.stats(srv)
    assert s.submitted == 1 and s.completed == 1
    f.lib.fftcg_server_destroy(srv)
    f.lib.fftcg_fake_plan_free(plan)


def scenario_sequences(f):
    """Load-stepped sequences: the breaks follow the rule on each step's
    solution, every step's bound and iteration count is reported."""
    plan = f.plan(16, 0)
    srv = f.server()
    rng = np.random.default_rng([10, 0])
    seqs = []
    for k in range(6):
        d, b = request(rng, 16)
        d[rng.random((16, 16)) < 0.2] = 0.0
        t = rng.uniform(0.1, 1.0, (16, 16))
        tk = U64()
        steps = 25
        assert f.lib.fftcg_submit_sequence(srv, plan, 1, d.ctypes.data_as(P), b.ctypes.data_as(P),
                                           t.ctypes.data_as(P), 1e-8, 10000, steps, ctypes.byref(tk)) == OK
        seqs.append((tk.value, d, b, t, steps))
    for tk, d, b, t, steps in seqs:
        x = np.empty((16, 16))
        br = np.empty(steps, dtype=np.int32)
        it = np.empty(steps, dtype=np.int32)
        eb = np.empty(steps)
        info = Info()
        t0 = time.time()
        while True:
            st = f.lib.fftcg_poll_sequence(srv, tk, x.ctypes.data_as(P), br.ctypes.data_as(P),
                                           it.ctypes.data_as(P), eb.ctypes.data_as(P), ctypes.byref(info))
            if st != PENDING:
                break
            assert time.time() - t0 < 60
            time.sleep(0.0005)
        assert st == OK
        live = d.ravel() != 0.0
        ratio = (0.5 * b).ravel() / t.ravel()
        want = []
        for _ in range(steps):
            j = int(np.argmax(np.where(live, ratio, -np.inf)))
            want.append(j)
            live[j] = False
        assert br.tolist() == want
        assert np.all(it == target(b)) and np.all(eb == 1e-9)
        assert np.array_equal(x, 0.5 * b)
    f.lib.fftcg_server_destroy(srv)
    f.lib.fftcg_fake_plan_free(plan)


def scenario_shutdown(f):
    """Shutdown with work queued and running: every request ends OK or
    FFTCG_ECANCELED, the counts agree, later submissions are refused, and
    the plans are free again."""
    f.lib.fftcg_fake_set_event_delay(2000)  # chunks complete slowly
    plan = f.plan(32, 0)
    srv = f.server(max_slots=4)
    rng = np.random.default_rng([11, 0])
    tks = {}
    for _ in range(200):
        d, b = request(rng, 32)
        st, tk = f.submit(srv, plan, d, b)
        assert st == OK
        tks[tk] = b
    assert f.lib.fftcg_server_shutdown(srv) == OK
    d, b = request(rng, 32)
    assert f.submit(srv, plan, d, b)[0] == ECANCELED
    codes = []
    for tk, b in tks.items():
        st, x, info = f.poll(srv, tk, 32)
        assert st in (OK, ECANCELED)
        if st == OK:
            assert np.array_equal(x, 0.5 * b)
        codes.append(st)
    s = f.stats(srv)
    assert s.canceled == codes.count(ECANCELED) >= 1 and s.in_flight == 0 and s.queued == 0
    assert f.lib.fftcg_fake_plan_refs(plan) == 0
    f.lib.fftcg_server_destroy(srv)
    f.lib.fftcg_fake_plan_free(plan)
    f.lib.fftcg_fake_set_event_delay(0)


def scenario_graphs(f):
    """Chunk graphs: with graphs on, a multi-pass class captures each chunk
    shape once and replays it (far fewer launches issued), with the same
    results as direct launches."""
    counts = {}
    for graphs in (-1, 0):
        before = f.lib.fftcg_fake_launches()
        scenario_mix_two_clients(f, n=200, graphs=graphs, delay=1)
        counts[graphs] = f.lib.fftcg_fake_launches() - before
    assert counts[0] < counts[-1] / 2, counts


def scenario_reserve(f):
    """Capacity reservation: the slots exist (and count against the budget)
    before any request, the plan stays referenced until shutdown, limits are
    checked, requests submitted while another thread reserves all complete,
    and a reservation after shutdown is refused."""
    foot = 16 * 16 * 40 + 8192 + 4 * 16 * 16 * 8 + 4 * 1024 + 4096
    plan = f.plan(16, 0)
    srv = f.server(budget=1 << 30, max_slots=8)
    nsl = I(-1)
    assert f.lib.fftcg_server_class_slots(srv, plan, 1, ctypes.byref(nsl)) == OK and nsl.value == 0
    assert f.lib.fftcg_server_reserve(srv, plan, 1, 4) == OK
    assert f.stats(srv).bytes_in_use == 4 * foot
    assert f.lib.fftcg_server_class_slots(srv, plan, 1, ctypes.byref(nsl)) == OK and nsl.value == 4
    assert f.lib.fftcg_server_class_slots(srv, plan, 0, ctypes.byref(nsl)) == OK and nsl.value == 0
    assert f.lib.fftcg_fake_plan_refs(plan) == 1
    assert f.lib.fftcg_server_reserve(srv, plan, 1, 2) == OK  # never shrinks
    assert f.stats(srv).bytes_in_use == 4 * foot
    assert f.lib.fftcg_server_reserve(srv, plan, 1, 9) == EINVAL  # above max_slots
    assert f.lib.fftcg_server_reserve(srv, plan, 3, 2) == EINVAL  # precision
    rng = np.random.default_rng([9, 0])
    tks, res = {}, []
    th = threading.Thread(target=lambda: res.append(f.lib.fftcg_server_reserve(srv, plan, 1, 8)))
    th.start()
    for _ in range(60):
        d, b = request(rng, 16)
        st, tk = f.submit(srv, plan, d, b)
        assert st == OK
        tks[tk] = b
    th.join()
    assert res == [OK]
    out = wait_all(f, srv, {tk: 16 for tk in tks})
    assert all(r[0] == OK and np.array_equal(r[1], 0.5 * tks[tk]) for tk, r in out.items())
    assert f.stats(srv).bytes_in_use == 8 * foot
    # the budget bounds a reservation
    small = f.server(budget=int(2.5 * foot))
    assert f.lib.fftcg_server_reserve(small, plan, 1, 3) == ENOMEM
    assert f.lib.fftcg_server_reserve(small, plan, 1, 2) == OK
    assert f.lib.fftcg_fake_plan_refs(plan) == 2
    f.lib.fftcg_server_destroy(small)
    assert f.lib.fftcg_server_shutdown(srv) == OK
    assert f.lib.fftcg_fake_plan_refs(plan) == 0
    assert f.lib.fftcg_server_reserve(srv, plan, 1, 1) == ECANCELED
    f.lib.fftcg_server_destroy(srv)
    f.lib.fftcg_fake_plan_free(plan)


ALL = [scenario_mix_two_clients, scenario_budget, scenario_queue_cap_and_maxit, scenario_invalid_inputs,
       scenario_sequences,
       scenario_shutdown, scenario_graphs, scenario_reserve]

if __name__ == "__main__":
    fk = Fake(sys.argv[1])
    for sc in ALL:
        sc(fk)
        print("ok", sc.__name__, flush=True)
    print("FAKE_OK", flush=True)
