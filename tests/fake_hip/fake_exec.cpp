// Simulated device for host-only tests of the server's scheduler
// (tests/test_server_fake.py).  Linked with the unmodified server.cpp built
// by g++ against tests/fake_hip/hip/hip_runtime.h.
//
// * "Device" memory is host memory; every stream operation runs when it is
//   issued; an event reports not-ready a random number of times (0 ..
//   the configured delay) before it completes.
// * Stream capture records the captured launches; an instantiated graph
//   replays them.
// * A fake solve of A x = b: each CG iteration counts up; the check at the
//   end of a chunk finishes the solve once its iteration count reaches
//   target(b) = 3 + (int)(1000 |b_0|) % 37 with x = b / 2, or at maxit with
//   FFTCG_ENOCONV and x = b / 4.  The load step applies the real rule
//   (argmax of x / t over d != 0, ties to the smallest index).
// Not part of the product library.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <functional>
#include <mutex>
#include <new>
#include <vector>

#include "common.hpp"
#include "engine.hpp"
#include "fftcg.h"
#include "fftcg_internal.hpp"
#include "fused.hpp"

using namespace fftcg;

// ---- runtime ---------------------------------------------------------------
struct FakeStream {
    int id;
};
struct FakeEvent {
    std::atomic<int> pending{0};
};
struct FakeGraph {
    std::vector<std::function<void()>> ops;
};
struct FakeGraphExec {
    std::vector<std::function<void()>> ops;
};

static std::atomic<int> g_event_delay{0};
static std::atomic<unsigned> g_rng{12345u};
static thread_local FakeStream* t_capture_stream = nullptr;
static thread_local FakeGraph* t_capture = nullptr;

static int rnd(int hi) {  // 0 .. hi
    if (hi <= 0) return 0;
    unsigned x = g_rng.fetch_add(0x9E3779B9u) * 2654435761u;
    return (int)((x >> 8) % (unsigned)(hi + 1));
}

// Runs op now, or records it when the stream is being captured.
static void issue(hipStream_t s, std::function<void()> op) {
    if (t_capture && t_capture_stream == s)
        t_capture->ops.push_back(std::move(op));
    else
        op();
}

hipError_t hipMallocRaw(void** p, size_t n) {
    *p = calloc(1, n ? n : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
    free(p);
    return hipSuccess;
}
hipError_t hipHostMallocRaw(void** p, size_t n, unsigned) { return hipMallocRaw(p, n); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipHostGetDevicePointer(void** d, void* h, unsigned) {
    *d = h;
    return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind) {
    memcpy(dst, src, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
    issue(s, [=] { memcpy(dst, src, n); });
    return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t s) {
    issue(s, [=] { memset(dst, v, n); });
    return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
    static std::atomic<int> next{1};
    *s = new (std::nothrow) FakeStream{next.fetch_add(1)};
    return *s ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) {
    delete s;
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
    *e = new (std::nothrow) FakeEvent();
    return *e ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
    e->pending.store(rnd(g_event_delay.load()));
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
    int p = e->pending.load();
    while (p > 0) {
        if (e->pending.compare_exchange_weak(p, p - 1)) return hipErrorNotReady;
    }
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipGetDeviceCount(int* n) {
    *n = 1;
    return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    if (t_capture) return hipErrorInvalidValue;
    t_capture = new (std::nothrow) FakeGraph();
    t_capture_stream = s;
    return t_capture ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
    if (!t_capture || t_capture_stream != s) return hipErrorInvalidValue;
    *g = t_capture;
    t_capture = nullptr;
    t_capture_stream = nullptr;
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* ex, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
    *ex = new (std::nothrow) FakeGraphExec{g->ops};
    return *ex ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipGraphLaunch(hipGraphExec_t ex, hipStream_t s) {
    for (auto& op : ex->ops) issue(s, op);
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    delete g;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t ex) {
    delete ex;
    return hipSuccess;
}

// ---- the library's host side, simulated -------------------------------------
namespace {
struct FakePlan {
    int L;
    EngineOps ops;
};
std::atomic<long> g_launches{0};

int target_iters(const double* b) { return 3 + (int)(1000.0 * fabs(b[0])) % 37; }

void publish(const SlotDesc& sd, const SolveState* st) {
    if (!sd.host_status) return;
    __atomic_store_n(sd.host_status + 1, st->status, __ATOMIC_RELAXED);
    __atomic_store_n(sd.host_status + 2, st->last_check_iter, __ATOMIC_RELAXED);
    __atomic_store_n(sd.host_status + 3, st->iters, __ATOMIC_RELAXED);
    __atomic_store_n(sd.host_status, 2 * st->gen + (st->done ? 1 : 0), __ATOMIC_RELEASE);
}

void slot_iter(const SlotDesc& sd) {
    SolveState* st = sd.st;
    if (!sd.active || st->done || st->pause) return;
    st->iters += 1;
    if (st->iters >= target_iters(sd.b) || st->iters >= st->maxit) st->pause = 1;
}

void slot_check(const SlotDesc& sd, int L) {
    SolveState* st = sd.st;
    if (!sd.active || st->done) return;
    st->checks += 1;
    const size_t n = (size_t)L * L;
    if (st->iters >= target_iters(sd.b)) {
        st->done = 1;
        st->status = FFTCG_OK;
        st->bound = 1e-9;
        st->true_relres = 1e-10;
        for (size_t i = 0; i < n; ++i) sd.x[i] = 0.5 * sd.b[i];
    } else if (st->iters >= st->maxit) {
        st->done = 1;
        st->status = FFTCG_ENOCONV;
        for (size_t i = 0; i < n; ++i) sd.x[i] = 0.25 * sd.b[i];
    } else {
        st->pause = 0;
        st->last_check_iter = st->iters;
    }
    publish(sd, st);
}

const FakePlan* fp_of(const PlanTabs& t) { return static_cast<const FakePlan*>(t.tw32); }

void fake_iter(int, const PlanTabs& t, const SlotDesc* slots, int nslots, int, hipStream_t s) {
    g_launches.fetch_add(4);
    issue(s, [slots, nslots] {
        for (int i = 0; i < nslots; ++i) slot_iter(slots[i]);
    });
    (void)t;
}
void fake_check(int, const PlanTabs& t, const SlotDesc* slots, int nslots, int, hipStream_t s) {
    g_launches.fetch_add(4);
    const int L = fp_of(t)->L;
    issue(s, [slots, nslots, L] {
        for (int i = 0; i < nslots; ++i) slot_check(slots[i], L);
    });
}
}  // namespace

namespace fftcg {

Workspace::~Workspace() { release(); }
void Workspace::release() {
    void* v[] = {st, slot, e, d32, part, ls_pv, ls_pi, ls_out, r, p, q, z, W};
    for (void* a : v) free(a);
    st = nullptr;
    slot = nullptr;
    e = d32 = nullptr;
    part = nullptr;
    ls_pv = nullptr;
    ls_pi = ls_out = nullptr;
    r = p = q = z = W = nullptr;
}
int Workspace::init(int L_, int M_, int stride_) {
    L = L_;
    M = M_;
    stride = stride_;
    const size_t n = (size_t)L * L;
    if (hipMalloc(&st, sizeof(SolveState)) != hipSuccess || hipMalloc(&slot, sizeof(SlotDesc)) != hipSuccess ||
        hipMalloc(&e, n * 4) != hipSuccess || hipMalloc(&d32, n * 4) != hipSuccess ||
        hipMalloc(&ls_pv, 1024 * 8) != hipSuccess || hipMalloc(&ls_pi, 1024 * 4) != hipSuccess)
        return FFTCG_ENOMEM;
    return FFTCG_OK;
}
size_t workspace_bytes(int L, int, int) { return (size_t)L * L * 40 + 8192; }

void init_state(SolveState* h, const fftcg_plan_s*, int precision, double tol, int maxit, int refresh) {
    memset(h, 0, sizeof(SolveState));
    h->tol = tol;
    h->tau = tol;
    h->maxit = maxit;
    h->refresh = precision == FFTCG_MIXED ? refresh : 0;
    h->pause = 1;
    h->restart = 1;
    h->iters_literal = -1;
    h->mixed = precision == FFTCG_MIXED ? 1 : 0;
}
void fill_slot(SlotDesc* h, const Workspace* w, double* x, const double* b, const double* d) {
    memset(h, 0, sizeof(SlotDesc));
    h->x = x;
    h->b = b;
    h->d = d;
    h->e = w->e;
    h->d32 = w->d32;
    h->st = w->st;
    h->active = 1;
}
int server_engine(const fftcg_plan_s* p) { return p->engine == FFTCG_ENGINE_FUSED ? FFTCG_ENGINE_FUSED : 1; }

void fused_launch(const fftcg_plan_s* p, int, const SlotDesc* slots, int nslots, int max_iters, hipStream_t s) {
    g_launches.fetch_add(1);
    const int L = p->L;
    issue(s, [slots, nslots, max_iters, L] {
        for (int i = 0; i < nslots; ++i) {
            for (int k = 0; k < max_iters && !slots[i].st->done; ++k) {
                if (slots[i].st->pause) slot_check(slots[i], L);
                slot_iter(slots[i]);
            }
            if (slots[i].st->pause) slot_check(slots[i], L);
        }
    });
}
void launch_to_f32(const double* src, float* dst, int n, hipStream_t s) {
    issue(s, [=] {
        for (int i = 0; i < n; ++i) dst[i] = (float)src[i];
    });
}
void launch_loadstep(const double* x, const double* t, double* d, int n, double*, int*, int* out, hipStream_t s,
                     const double* bound_src, double* bound_dst) {
    issue(s, [=] {
        int best = -1;
        double bv = 0.0;
        for (int i = 0; i < n; ++i) {
            if (d[i] == 0.0) continue;
            const double v = x[i] / t[i];
            if (best < 0 || v > bv) {
                best = i;
                bv = v;
            }
        }
        if (best >= 0) d[best] = 0.0;
        *out = best;
        if (bound_dst) *bound_dst = *bound_src;
    });
}

}  // namespace fftcg

fftcg_plan_s::~fftcg_plan_s() { delete static_cast<const FakePlan*>(tabs.tw32); }

// ---- test controls -----------------------------------------------------------
extern "C" int fftcg_fake_plan(int L, int fused, fftcg_plan_t* out) {
    if (L < 2 || !out) return FFTCG_EINVAL;
    fftcg_plan_s* p = new (std::nothrow) fftcg_plan_s();
    FakePlan* f = new (std::nothrow) FakePlan();
    if (!p || !f) return FFTCG_ENOMEM;
    p->L = L;
    p->M = 2 * L;
    p->pad = 1;
    p->stride = 64;
    p->engine = fused ? FFTCG_ENGINE_FUSED : FFTCG_ENGINE_MULTIPASS;
    p->fused_ok = fused ? 1 : 0;
    f->L = L;
    memset(&f->ops, 0, sizeof(EngineOps));
    f->ops.M = 2 * L;
    f->ops.pad = 1;
    f->ops.L = L;
    f->ops.iter = f->ops.iter_pcg = &fake_iter;
    f->ops.check = f->ops.check_pcg = &fake_check;
    p->ops = &f->ops;
    p->tabs.tw32 = f;
    *out = p;
    return FFTCG_OK;
}
extern "C" int fftcg_fake_plan_refs(fftcg_plan_t p) { return p->refs.load(); }
extern "C" void fftcg_fake_plan_free(fftcg_plan_t p) { delete p; }
extern "C" void fftcg_fake_set_event_delay(int d) { g_event_delay.store(d); }
extern "C" long fftcg_fake_launches(void) { return g_launches.load(); }
