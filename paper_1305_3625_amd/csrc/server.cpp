// Continuous-batching solve server.
//
// Requests are grouped into classes by (plan, precision): one grid size and
// one arithmetic each.  Every class has a pool of slots; a slot owns the
// device vectors of one in-flight solve.  The scheduler thread repeatedly,
// for every class:
//   retire  - a slot whose solve finished (status word carrying the slot's
//             current generation) copies x back to the request's pinned
//             buffer; a load-stepped sequence instead runs the load step on
//             the device and restarts the slot from the previous x;
//   admit   - queued requests (FIFO per class) take free slots; new slots are
//             allocated while the device memory held by all slots stays
//             within the budget (idle slots of other classes are released
//             when a class has none);
//   step    - one chunk of CG iterations plus an FP64 check is launched over
//             all slots of the class at once (gridDim.y = slot), on the
//             class's own stream, so classes overlap on the GPU.
// A slot's arithmetic does not depend on the other slots (per-slot
// reductions in a fixed order), so a request gives bitwise the same x alone
// and in any mix.  Host <-> device copies happen only at admission and
// retirement.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "engine.hpp"
#include "fftcg.h"
#include "fftcg_internal.hpp"
#include "fused.hpp"

using namespace fftcg;

namespace {

constexpr int kMaxSteps = 1024;  // capacity of a slot's broken-index buffer
constexpr size_t kMaxCompleted = size_t(1) << 20;  // unreported tickets kept

struct Request {
    uint64_t ticket = 0;
    fftcg_plan_s* plan = nullptr;
    int precision = 0;
    double tol = 0;
    int maxit = 0;
    int steps = 0;  // 0: one solve; > 0: load-stepped sequence
    size_t n = 0;
    double* pin_in = nullptr;  // staging of the inputs: d, b, then x0 and t when given
    bool in_pinned = true;     // false: pageable (over the pinned cap), staged per slot
    double* pin_x = nullptr;   // pinned result (taken when the solve retires)
    bool x_nomem = false;      // no pinned result buffer could be had
    int* pin_broken = nullptr; // pinned sequence result: broken indices
    double* pin_bounds = nullptr; // and each step's certified error bound
    bool has_x0 = false;
    size_t in_bytes = 0;
    int status = FFTCG_PENDING;
    fftcg_info info{};
    std::vector<int> step_iters;
    bool done = false;
};

struct Slot {
    std::unique_ptr<Workspace> ws;
    double* x = nullptr;
    double* b = nullptr;
    double* d = nullptr;
    double* t = nullptr;
    int* broken = nullptr;            // device, one entry per step
    double* bounds = nullptr;         // device, each step's certified error bound
    SolveState* pin_state = nullptr;  // pinned staging of the state
    double* stage = nullptr;          // pinned staging of pageable request inputs (on first use)
    Request* req = nullptr;
    int gen = 0;
    int step = 0;
    bool retiring = false;
    hipEvent_t ev_retire = nullptr;
};

struct Class {
    fftcg_plan_s* plan = nullptr;
    int precision = 0;
    hipStream_t stream = nullptr;
    std::vector<std::unique_ptr<Slot>> slots;
    SlotDesc* d_table = nullptr;  // device slot table (max_slots entries)
    SlotDesc* h_table = nullptr;  // pinned mirror
    int* h_status = nullptr;      // pinned: {done, status, gen, iters} per slot
    int* d_status = nullptr;
    std::deque<Request*> pending;
    hipEvent_t ev[2] = {nullptr, nullptr};
    int inflight = 0;  // chunks launched and not yet seen complete
    int next_ev = 0;
    size_t footprint = 0;  // device bytes per slot
    int refresh = 50;      // MIXED: iterations between FP64 checks
    // multi-pass chunks captured as HIP graphs, by (running slots, preconditioned)
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;
    bool reserved = false;  // fftcg_server_reserve holds a reference to the plan
    std::atomic<int> nslots{0};  // slots.size(), readable by other threads
};

// A capacity reservation waiting for the scheduler thread (which alone adds
// slots to a class); the caller waits on cv_res until done.
struct Reservation {
    Class* c = nullptr;
    int slots = 0;
    int rc = 0;
    bool done = false;
};

}  // namespace

struct fftcg_server_s {
    fftcg_server_opts opts{};
    std::mutex mu;
    std::condition_variable cv;
    std::thread thread;
    std::atomic<bool> stop{false};
    bool shut = false;  // fftcg_server_shutdown has begun (guarded by mu)
    std::map<std::pair<fftcg_plan_s*, int>, std::unique_ptr<Class>> classes;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> requests;
    uint64_t next_ticket = 1;
    std::atomic<size_t> bytes_in_use{0};
    std::atomic<int> in_flight{0};
    int queued = 0;
    fftcg_server_stats stats{};
    std::deque<uint64_t> completed;  // finished, not yet reported tickets
    // pinned host buffers kept for reuse, by size (pinning is slow)
    std::mutex pin_mu;
    std::multimap<size_t, void*> pin_free;
    size_t pin_cached = 0;  // bytes idle in pin_free
    // pageable input buffers kept for reuse (a fresh one page-faults on
    // every first touch while the submission copies into it)
    std::multimap<size_t, void*> page_free;
    size_t page_cached = 0;
    size_t pin_inputs = 0;  // pinned input staging handed out
    size_t pin_input_cap = 0;  // a quarter of the device budget, in [1 MiB, 1 GiB]
    // capacity reservations for the scheduler thread (guarded by mu)
    std::deque<Reservation*> reserves;
    std::condition_variable cv_res;
};

namespace {

void* pin_get(fftcg_server_s* srv, size_t bytes, bool input, bool* pinned);

size_t slot_footprint(const fftcg_plan_s* p) {
    const size_t n = (size_t)p->L * p->L;
    return workspace_bytes(p->L, p->M, p->stride) + 4 * n * 8 + sizeof(int) * kMaxSteps + 4096;
}

void free_slot_memory(Slot* s) {
    double* dv[] = {s->x, s->b, s->d, s->t};
    for (double* v : dv)
        if (v) (void)hipFree(v);
    if (s->broken) (void)hipFree(s->broken);
    if (s->bounds) (void)hipFree(s->bounds);
    if (s->pin_state) (void)hipHostFree(s->pin_state);
    if (s->stage) (void)hipHostFree(s->stage);
    s->stage = nullptr;
    if (s->ev_retire) (void)hipEventDestroy(s->ev_retire);
    s->x = s->b = s->d = s->t = nullptr;
    s->broken = nullptr;
    s->bounds = nullptr;
    s->pin_state = nullptr;
    s->ev_retire = nullptr;
    s->ws.reset();
}

void upload_entry(Class* c, int idx) {
    (void)hipMemcpyAsync(c->d_table + idx, c->h_table + idx, sizeof(SlotDesc), hipMemcpyHostToDevice, c->stream);
}

// Releases idle slots at the end of other classes' pools until `need` more
// bytes fit in the budget (scheduler thread).  hipFree waits for the device.
void reclaim(fftcg_server_s* srv, Class* except, size_t need) {
    std::vector<Class*> cls;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        for (auto& kv : srv->classes)
            if (kv.second.get() != except) cls.push_back(kv.second.get());
    }
    for (Class* c : cls) {
        while (!c->slots.empty() && srv->bytes_in_use.load() + need > srv->opts.memory_budget) {
            Slot* s = c->slots.back().get();
            if (s->req) break;
            (void)hipStreamSynchronize(c->stream);
            free_slot_memory(s);
            c->slots.pop_back();
            c->nslots.store((int)c->slots.size());
            srv->bytes_in_use.fetch_sub(c->footprint);
        }
        if (srv->bytes_in_use.load() + need <= srv->opts.memory_budget) return;
    }
}

// Adds one slot to class c; false when at max_slots, over budget, or the
// allocation fails.
bool add_slot(fftcg_server_s* srv, Class* c) {
    if ((int)c->slots.size() >= srv->opts.max_slots) return false;
    if (srv->bytes_in_use.load() + c->footprint > srv->opts.memory_budget) {
        if (!c->slots.empty()) return false;
        reclaim(srv, c, c->footprint);
        if (srv->bytes_in_use.load() + c->footprint > srv->opts.memory_budget) return false;
    }
    auto s = std::make_unique<Slot>();
    const fftcg_plan_s* p = c->plan;
    const size_t n = (size_t)p->L * p->L;
    s->ws.reset(new Workspace());
    bool ok = s->ws->init(p->L, p->M, p->stride) == FFTCG_OK;
    ok = ok && hipMalloc(&s->x, n * 8) == hipSuccess && hipMalloc(&s->b, n * 8) == hipSuccess &&
         hipMalloc(&s->d, n * 8) == hipSuccess && hipMalloc(&s->t, n * 8) == hipSuccess &&
         hipMalloc(&s->broken, sizeof(int) * kMaxSteps) == hipSuccess &&
         hipMalloc(&s->bounds, sizeof(double) * kMaxSteps) == hipSuccess &&
         hipHostMalloc((void**)&s->pin_state, sizeof(SolveState), hipHostMallocDefault) == hipSuccess &&
         hipEventCreateWithFlags(&s->ev_retire, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        free_slot_memory(s.get());
        return false;
    }
    srv->bytes_in_use.fetch_add(c->footprint);
    const int idx = (int)c->slots.size();
    fill_slot(&c->h_table[idx], s->ws.get(), s->x, s->b, s->d);
    c->h_table[idx].host_status = c->d_status + 4 * idx;
    c->h_table[idx].active = 0;
    memset(c->h_status + 4 * idx, 0, 4 * sizeof(int));
    c->slots.push_back(std::move(s));
    c->nslots.store((int)c->slots.size());
    upload_entry(c, idx);
    return true;
}

int make_class(fftcg_server_s* srv, fftcg_plan_s* plan, int precision, Class** out) {
    auto c = std::make_unique<Class>();
    c->plan = plan;
    c->precision = precision;
    c->footprint = slot_footprint(plan);
    c->refresh = srv->opts.refresh_period;
    const int ms = srv->opts.max_slots;
    bool ok = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) == hipSuccess &&
              hipMalloc((void**)&c->d_table, sizeof(SlotDesc) * ms) == hipSuccess &&
              hipHostMalloc((void**)&c->h_table, sizeof(SlotDesc) * ms, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void**)&c->h_status, sizeof(int) * 4 * ms,
                            hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
              hipHostGetDevicePointer((void**)&c->d_status, c->h_status, 0) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev[0], hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev[1], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        // partial class: released by destroy_class through the map
        srv->classes[{plan, precision}] = std::move(c);
        return FFTCG_EDEVICE;
    }
    memset(c->h_table, 0, sizeof(SlotDesc) * ms);
    memset(c->h_status, 0, sizeof(int) * 4 * ms);
    *out = c.get();
    srv->classes[{plan, precision}] = std::move(c);
    return FFTCG_OK;
}

void destroy_class(Class* c) {
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    for (auto& s : c->slots) free_slot_memory(s.get());
    if (c->d_table) (void)hipFree(c->d_table);
    if (c->h_table) (void)hipHostFree(c->h_table);
    if (c->h_status) (void)hipHostFree(c->h_status);
    for (int i = 0; i < 2; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    if (c->stream) (void)hipStreamDestroy(c->stream);
}

// (Re)starts the solve in slot idx with a fresh state of a new generation;
// the check at the end of the next chunk computes r = b - A x from the slot's
// x (zero, the caller's x0, or the previous step's solution).
void start_solve(Class* c, int idx) {
    Slot* s = c->slots[idx].get();
    Request* q = s->req;
    s->gen += 1;
    init_state(s->pin_state, c->plan, q->precision, q->tol, q->maxit, c->refresh);
    s->pin_state->gen = s->gen;
    (void)hipMemcpyAsync(s->ws->st, s->pin_state, sizeof(SolveState), hipMemcpyHostToDevice, c->stream);
    if (q->precision == FFTCG_MIXED) {
        (void)hipMemsetAsync(s->ws->e, 0, q->n * 4, c->stream);
        launch_to_f32(s->d, s->ws->d32, (int)q->n, c->stream);
    }
}

void admit(Class* c, Request* q, int idx) {
    Slot* s = c->slots[idx].get();
    s->req = q;
    s->step = 0;
    s->retiring = false;
    const size_t n = q->n;
    const double* pin = q->pin_in;
    if (!q->in_pinned) {
        // pageable inputs go through the slot's pinned staging buffer (free:
        // its previous request was admitted, and its copies done, before it
        // retired), allocated the first time a slot needs it: pinning costs
        // milliseconds, and slots fed from the pinned pool never need one.
        // Without it the copies read the pageable buffer, which stays alive
        // until the request is polled.
        if (!s->stage && hipHostMalloc((void**)&s->stage, n * 8 * 4, hipHostMallocDefault) != hipSuccess) {
            s->stage = nullptr;
            (void)hipGetLastError();  // the failure is handled here
        }
        if (s->stage) {
            memcpy(s->stage, q->pin_in, q->in_bytes);
            pin = s->stage;
        }
    }
    hipStream_t st = c->stream;
    (void)hipMemcpyAsync(s->d, pin, n * 8, hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(s->b, pin + n, n * 8, hipMemcpyHostToDevice, st);
    if (q->has_x0)
        (void)hipMemcpyAsync(s->x, pin + 2 * n, n * 8, hipMemcpyHostToDevice, st);
    else
        (void)hipMemsetAsync(s->x, 0, n * 8, st);
    if (q->steps > 0)
        (void)hipMemcpyAsync(s->t, pin + (q->has_x0 ? 3 : 2) * n, n * 8, hipMemcpyHostToDevice, st);
    start_solve(c, idx);
    c->h_table[idx].active = 1;
    upload_entry(c, idx);
}

// Called with srv->mu held.
void finish_request(fftcg_server_s* srv, Request* q, int status, const SolveState& st) {
    q->status = status;
    q->info.status = status;
    q->info.iterations = st.iters;
    q->info.iterations_literal = st.iters_literal;
    q->info.checks = st.checks;
    q->info.true_relres = st.true_relres;
    q->info.error_bound = st.bound;
    q->info.lambda_lb = st.lam_lb;
    q->info.device_ms = 0.0;
    q->done = true;
    srv->completed.push_back(q->ticket);
    if (srv->completed.size() > kMaxCompleted) srv->completed.pop_front();
    if (status == FFTCG_OK || status == FFTCG_ENOCONV)
        srv->stats.completed += 1;
    else if (status == FFTCG_ECANCELED)
        srv->stats.canceled += 1;
    else
        srv->stats.failed += 1;
    q->plan->refs.fetch_sub(1);
}

// One chunk of the multi-pass engine over slots 0..nsl-1: chunk_iters CG
// iterations, then an FP64-check sequence (kernel launches only).
void launch_chunk(fftcg_server_s* srv, Class* c, int nsl, bool pcg) {
    const EngineOps* ops = c->plan->ops;
    const auto iter = pcg ? ops->iter_pcg : ops->iter;
    const auto check = pcg ? ops->check_pcg : ops->check;
    for (int k = 0; k < srv->opts.chunk_iters; ++k)
        iter(c->precision, c->plan->tabs, c->d_table, nsl, c->plan->stride, c->stream);
    check(c->precision, c->plan->tabs, c->d_table, nsl, c->plan->stride, c->stream);
}

// The chunk for nsl running slots as an instantiated HIP graph, captured from
// the class's stream the first time that shape runs (every kernel argument
// is fixed per class and shape: the slot table is device-resident, so a
// replay sees the slots' current contents).  A chunk is some forty kernel
// launches; replayed as one graph it costs the scheduler thread a single
// launch, which keeps the small classes' GPU work from waiting on the host.
// nullptr if capture or instantiation fails (the caller then launches
// directly).
hipGraphExec_t chunk_graph(fftcg_server_s* srv, Class* c, int nsl, bool pcg) {
    const auto key = std::make_pair(nsl, pcg ? 1 : 0);
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) return it->second;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    launch_chunk(srv, c, nsl, pcg);
    if (hipStreamEndCapture(c->stream, &g) != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return nullptr;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess || !ex) return nullptr;
    c->graphs[key] = ex;
    return ex;
}

// Scheduler work for one class; true while it has queued or running work.
bool progress(fftcg_server_s* srv, Class* c) {
    // chunks that completed
    while (c->inflight > 0) {
        const int e = (c->next_ev - c->inflight + 2) & 1;
        if (hipEventQuery(c->ev[e]) != hipSuccess) break;
        c->inflight -= 1;
    }
    const int ns = (int)c->slots.size();
    // retirements whose copies have landed
    for (int i = 0; i < ns; ++i) {
        Slot* s = c->slots[i].get();
        if (!s->req || !s->retiring || hipEventQuery(s->ev_retire) != hipSuccess) continue;
        Request* q = s->req;
        const SolveState st = *s->pin_state;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            if (q->steps > 0) q->step_iters.push_back(st.iters);
            finish_request(srv, q, q->x_nomem ? FFTCG_ENOMEM : st.status, st);
        }
        s->req = nullptr;
        s->retiring = false;
        srv->in_flight.fetch_sub(1);
    }
    // finished solves: status word of the slot's current generation
    for (int i = 0; i < ns; ++i) {
        Slot* s = c->slots[i].get();
        if (!s->req || s->retiring) continue;
        const int* hs = c->h_status + 4 * i;
        // one word: 2 * generation + done (see publish_status)
        if (__atomic_load_n(hs, __ATOMIC_ACQUIRE) != 2 * s->gen + 1) continue;
        Request* q = s->req;
        const int status = __atomic_load_n(hs + 1, __ATOMIC_RELAXED);
        const bool ok = status == FFTCG_OK || status == FFTCG_ENOCONV;
        if (ok && q->steps > 0) {
            // the load step of this solve, on the device
            launch_loadstep(s->x, s->t, s->d, (int)q->n, s->ws->ls_pv, s->ws->ls_pi, s->broken + s->step,
                            c->stream, &s->ws->st->bound, s->bounds + s->step);
            if (s->step + 1 < q->steps) {
                q->step_iters.push_back(__atomic_load_n(hs + 3, __ATOMIC_RELAXED));
                s->step += 1;
                start_solve(c, i);  // warm start: x stays in place
                continue;
            }
        }
        // retire: deactivate, copy results; finished when the copies land
        c->h_table[i].active = 0;
        upload_entry(c, i);
        (void)hipMemcpyAsync(s->pin_state, s->ws->st, sizeof(SolveState), hipMemcpyDeviceToHost, c->stream);
        if (ok) {
            // pinned result buffers are taken only now, so a long queue
            // holds none
            bool pinned = true;
            q->pin_x = (double*)pin_get(srv, q->n * 8, false, &pinned);
            if (q->pin_x)
                (void)hipMemcpyAsync(q->pin_x, s->x, q->n * 8, hipMemcpyDeviceToHost, c->stream);
            else
                q->x_nomem = true;
            if (q->steps > 0)
            {
                (void)hipMemcpyAsync(q->pin_broken, s->broken, sizeof(int) * q->steps, hipMemcpyDeviceToHost,
                                     c->stream);
                (void)hipMemcpyAsync(q->pin_bounds, s->bounds, sizeof(double) * q->steps, hipMemcpyDeviceToHost,
                                     c->stream);
            }
        }
        (void)hipEventRecord(s->ev_retire, c->stream);
        s->retiring = true;
    }
    // admissions (FIFO)
    for (;;) {
        Request* q = nullptr;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            if (c->pending.empty()) break;
            q = c->pending.front();
        }
        int idx = -1;
        for (int i = 0; i < (int)c->slots.size(); ++i)
            if (!c->slots[i]->req) {
                idx = i;
                break;
            }
        if (idx < 0) {
            if (!add_slot(srv, c)) break;
            idx = (int)c->slots.size() - 1;
        }
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            c->pending.pop_front();
            srv->queued -= 1;
            srv->stats.admitted += 1;
        }
        srv->in_flight.fetch_add(1);
        admit(c, q, idx);
    }
    // one chunk over the slots of the class up to the last running one (new
    // requests take the lowest free slot, so a pool grown by a burst costs
    // nothing once the burst is over) when any solve is running
    int last = -1;
    for (int i = 0; i < (int)c->slots.size(); ++i)
        if (c->slots[i]->req && !c->slots[i]->retiring) last = i;
    const bool active = last >= 0;
    if (active && c->inflight < 2) {
        const int nsl = last + 1;
        if (server_engine(c->plan) == FFTCG_ENGINE_FUSED) {
            // one workgroup per slot runs the chunk's iterations and checks
            fused_launch(c->plan, c->precision, c->d_table, nsl, srv->opts.chunk_iters, c->stream);
        } else {
            const bool pcg = c->plan->precond == FFTCG_PRECOND_CIRCULANT;
            hipGraphExec_t ex = srv->opts.graphs >= 0 ? chunk_graph(srv, c, nsl, pcg) : nullptr;
            if (!ex || hipGraphLaunch(ex, c->stream) != hipSuccess) {
                (void)hipGetLastError();  // a failed capture or replay falls back to direct launches
                launch_chunk(srv, c, nsl, pcg);
            }
        }
        (void)hipEventRecord(c->ev[c->next_ev], c->stream);
        c->next_ev ^= 1;
        c->inflight += 1;
    }
    bool busy = active || c->inflight > 0;
    for (auto& s : c->slots)
        if (s->retiring) busy = true;
    std::lock_guard<std::mutex> lk(srv->mu);
    return busy || !c->pending.empty();
}

// Grows class c to `slots` slots, each with its pinned staging buffer, and
// captures the class's chunk graphs for every running-slot count up to
// `slots` (scheduler thread): on the way in, each new chunk shape would
// otherwise be captured and instantiated while requests wait.  FFTCG_ENOMEM
// when the budget or an allocation stops it; the slots made so far stay.
int grow_class(fftcg_server_s* srv, Class* c, int slots) {
    while ((int)c->slots.size() < slots)
        if (!add_slot(srv, c)) return FFTCG_ENOMEM;
    const size_t n = (size_t)c->plan->L * c->plan->L;
    for (int i = 0; i < slots; ++i) {
        Slot* s = c->slots[i].get();
        if (!s->stage && hipHostMalloc((void**)&s->stage, n * 8 * 4, hipHostMallocDefault) != hipSuccess) {
            s->stage = nullptr;
            (void)hipGetLastError();
            return FFTCG_ENOMEM;
        }
    }
    if (srv->opts.graphs >= 0 && server_engine(c->plan) != FFTCG_ENGINE_FUSED) {
        const bool pcg = c->plan->precond == FFTCG_PRECOND_CIRCULANT;
        for (int nsl = 1; nsl <= slots; ++nsl)
            if (!chunk_graph(srv, c, nsl, pcg)) (void)hipGetLastError();  // launched directly later
    }
    return FFTCG_OK;
}

void serve_reservations(fftcg_server_s* srv) {
    std::vector<Reservation*> res;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->reserves.empty()) return;
        res.assign(srv->reserves.begin(), srv->reserves.end());
        srv->reserves.clear();
    }
    for (Reservation* r : res) {
        int rc = FFTCG_OK;
        try {
            rc = grow_class(srv, r->c, r->slots);
        } catch (...) {
            rc = FFTCG_ENOMEM;
        }
        std::lock_guard<std::mutex> lk(srv->mu);
        r->rc = rc;
        r->done = true;
    }
    srv->cv_res.notify_all();
}

void scheduler(fftcg_server_s* srv) {
    (void)hipSetDevice(srv->opts.device);
    while (!srv->stop.load()) {
        serve_reservations(srv);
        std::vector<Class*> cls;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            for (auto& kv : srv->classes) cls.push_back(kv.second.get());
        }
        bool busy = false;
        for (Class* c : cls) {
            // an exception (a failed host allocation) must not end the
            // thread: the class is simply visited again on the next pass
            try {
                busy |= progress(srv, c);
            } catch (...) {
                busy = true;
            }
        }
        if (!busy) {
            std::unique_lock<std::mutex> lk(srv->mu);
            if (srv->queued == 0 && srv->reserves.empty() && !srv->stop.load())
                srv->cv.wait_for(lk, std::chrono::milliseconds(2));
        } else {
            std::this_thread::yield();
        }
    }
}

enum CopyCheck { kFinite, kNonNegative, kPositive };

// dst = src (n doubles), and whether every value is finite (and >= 0, or
// > 0); the test accumulates without branches so the loop streams.
bool copy_checked(double* __restrict__ dst, const double* __restrict__ src, size_t n, CopyCheck kind) {
    bool ok = true;
    for (size_t i = 0; i < n; ++i) {
        const double v = src[i];
        dst[i] = v;
        const bool fin = v - v == 0.0;  // false for inf and nan
        ok &= kind == kFinite ? fin : (kind == kNonNegative ? (fin && v >= 0.0) : (fin && v > 0.0));
    }
    return ok;
}

constexpr size_t kPinCacheBytes = size_t(2) << 30;  // idle pinned buffers kept

// Host buffer of exactly `bytes`: an idle pinned one from the pool, a new
// pinned one, or (inputs only, once pin_input_cap bytes of pinned input
// staging are in use: pinning costs about as much as the copy itself, and a
// long queue need not hold pinned memory) pageable memory.
void* pin_get(fftcg_server_s* srv, size_t bytes, bool input, bool* pinned) {
    *pinned = true;
    {
        std::lock_guard<std::mutex> lk(srv->pin_mu);
        auto it = srv->pin_free.find(bytes);
        if (it != srv->pin_free.end()) {
            void* p = it->second;
            srv->pin_free.erase(it);
            srv->pin_cached -= bytes;
            if (input) srv->pin_inputs += bytes;
            return p;
        }
        if (input && srv->pin_inputs + bytes > srv->pin_input_cap) {
            *pinned = false;
            auto pg = srv->page_free.find(bytes);
            if (pg != srv->page_free.end()) {
                void* p = pg->second;
                srv->page_free.erase(pg);
                srv->page_cached -= bytes;
                return p;
            }
            return malloc(bytes);
        }
        if (input) srv->pin_inputs += bytes;
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
        if (input) {
            std::lock_guard<std::mutex> lk(srv->pin_mu);
            srv->pin_inputs -= bytes;
        }
        return nullptr;
    }
    return p;
}

void pin_put(fftcg_server_s* srv, void* p, size_t bytes, bool input, bool pinned) {
    if (!p) return;
    if (!pinned) {
        {
            std::lock_guard<std::mutex> lk(srv->pin_mu);
            if (srv->page_cached + bytes <= kPinCacheBytes) {
                srv->page_free.emplace(bytes, p);
                srv->page_cached += bytes;
                return;
            }
        }
        free(p);
        return;
    }
    {
        std::lock_guard<std::mutex> lk(srv->pin_mu);
        if (input) srv->pin_inputs -= bytes;
        if (srv->pin_cached + bytes <= kPinCacheBytes) {
            srv->pin_free.emplace(bytes, p);
            srv->pin_cached += bytes;
            return;
        }
    }
    (void)hipHostFree(p);
}

void free_request_buffers(fftcg_server_s* srv, Request* q) {
    pin_put(srv, q->pin_in, q->in_bytes, true, q->in_pinned);
    pin_put(srv, q->pin_x, q->n * 8, false, true);
    pin_put(srv, q->pin_broken, sizeof(int) * (size_t)q->steps, false, true);
    pin_put(srv, q->pin_bounds, sizeof(double) * (size_t)q->steps, false, true);
    q->pin_in = q->pin_x = nullptr;
    q->pin_broken = nullptr;
    q->pin_bounds = nullptr;
}

}  // namespace

extern "C" int fftcg_server_create(const fftcg_server_opts* opts, fftcg_server_t* out) try {
    if (!opts || !out) return FFTCG_EINVAL;
    if (opts->memory_budget == 0 || opts->max_slots < 0 || opts->chunk_iters < 0 || opts->refresh_period < 0 ||
        opts->queue_cap < 0 || (opts->graphs != 0 && opts->graphs != -1))
        return FFTCG_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || opts->device < 0 || opts->device >= ndev) return FFTCG_EDEVICE;
    fftcg_server_s* s = new (std::nothrow) fftcg_server_s();
    if (!s) return FFTCG_ENOMEM;
    s->opts = *opts;
    if (s->opts.max_slots == 0) s->opts.max_slots = 64;
    if (s->opts.chunk_iters == 0) s->opts.chunk_iters = 10;
    if (s->opts.refresh_period == 0) s->opts.refresh_period = 50;
    s->pin_input_cap = std::min(std::max(s->opts.memory_budget / 4, size_t(1) << 20), size_t(1) << 30);
    if (s->opts.queue_cap == 0) s->opts.queue_cap = 1 << 20;
    s->thread = std::thread(scheduler, s);
    *out = s;
    return FFTCG_OK;
} FFTCG_ABI_CATCH

static int submit_common(fftcg_server_t srv, fftcg_plan_t plan, int precision, const double* d, const double* b,
                         const double* x0, const double* t, double tol, int maxit, int steps, uint64_t* ticket) {
    if (!srv || !plan || !d || !b || !ticket) return FFTCG_EINVAL;
    if (precision != FFTCG_FP64 && precision != FFTCG_MIXED) return FFTCG_EINVAL;
    if (!(tol > 0.0) || !(tol < 1.0) || maxit < 1) return FFTCG_EINVAL;
    if (!plan->ops) return FFTCG_EINVAL;
    if (slot_footprint(plan) > srv->opts.memory_budget) return FFTCG_ENOMEM;
    const size_t n = (size_t)plan->L * plan->L;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->shut) return FFTCG_ECANCELED;
        if (srv->queued >= srv->opts.queue_cap) return FFTCG_EAGAIN;
    }
    std::unique_ptr<Request> q(new (std::nothrow) Request());
    if (!q) return FFTCG_ENOMEM;
    q->plan = plan;
    q->precision = precision;
    q->tol = tol;
    q->maxit = maxit;
    q->steps = steps;
    q->n = n;
    q->has_x0 = x0 != nullptr;
    q->in_bytes = n * 8 * (2 + (x0 ? 1 : 0) + (t ? 1 : 0));
    bool pinned = true;
    q->pin_in = (double*)pin_get(srv, q->in_bytes, true, &q->in_pinned);
    if (steps > 0) {
        q->pin_broken = (int*)pin_get(srv, sizeof(int) * steps, false, &pinned);
        q->pin_bounds = (double*)pin_get(srv, sizeof(double) * steps, false, &pinned);
    }
    if (!q->pin_in || (steps > 0 && (!q->pin_broken || !q->pin_bounds))) {
        free_request_buffers(srv, q.get());
        return FFTCG_ENOMEM;
    }
    // inputs are checked while they are copied: one pass over the caller's
    // memory (the copy dominates a large request's submission)
    const bool valid = copy_checked(q->pin_in, d, n, kNonNegative) && copy_checked(q->pin_in + n, b, n, kFinite) &&
                       (!x0 || copy_checked(q->pin_in + 2 * n, x0, n, kFinite)) &&
                       (!t || copy_checked(q->pin_in + (x0 ? 3 : 2) * n, t, n, kPositive));
    if (!valid) {
        free_request_buffers(srv, q.get());
        return FFTCG_EINVAL;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->shut || srv->queued >= srv->opts.queue_cap) {
        free_request_buffers(srv, q.get());
        return srv->shut ? FFTCG_ECANCELED : FFTCG_EAGAIN;
    }
    Class* c = nullptr;
    auto it = srv->classes.find({plan, precision});
    if (it == srv->classes.end()) {
        const int rc = make_class(srv, plan, precision, &c);
        if (rc != FFTCG_OK) {
            free_request_buffers(srv, q.get());
            return rc;
        }
    } else {
        c = it->second.get();
    }
    // the two container insertions may throw (std::bad_alloc): the request
    // is queued only once the ticket map owns it, and leaves the map again
    // if queueing fails, so no container is left pointing at a freed request
    const uint64_t tk = srv->next_ticket;
    Request* raw = q.get();
    raw->ticket = tk;
    srv->requests.emplace(tk, std::move(q));
    try {
        c->pending.push_back(raw);
    } catch (...) {
        free_request_buffers(srv, raw);
        srv->requests.erase(tk);
        throw;
    }
    srv->next_ticket += 1;
    *ticket = tk;
    plan->refs.fetch_add(1);
    srv->queued += 1;
    srv->stats.submitted += 1;
    srv->cv.notify_all();
    return FFTCG_OK;
}

extern "C" int fftcg_submit(fftcg_server_t srv, fftcg_plan_t plan, int precision, const double* d, const double* b,
                            const double* x0, double tol, int maxit, uint64_t* ticket) try {
    return submit_common(srv, plan, precision, d, b, x0, nullptr, tol, maxit, 0, ticket);
} FFTCG_ABI_CATCH

extern "C" int fftcg_submit_sequence(fftcg_server_t srv, fftcg_plan_t plan, int precision, const double* d,
                                     const double* b, const double* t, double tol, int maxit, int steps,
                                     uint64_t* ticket) try {
    if (!t || steps < 1 || steps > kMaxSteps) return FFTCG_EINVAL;
    return submit_common(srv, plan, precision, d, b, nullptr, t, tol, maxit, steps, ticket);
} FFTCG_ABI_CATCH

extern "C" int fftcg_server_reserve(fftcg_server_t srv, fftcg_plan_t plan, int precision, int slots) try {
    if (!srv || !plan || !plan->ops) return FFTCG_EINVAL;
    if (precision != FFTCG_FP64 && precision != FFTCG_MIXED) return FFTCG_EINVAL;
    if (slots < 0 || slots > srv->opts.max_slots) return FFTCG_EINVAL;
    if ((size_t)slots * slot_footprint(plan) > srv->opts.memory_budget) return FFTCG_ENOMEM;
    Reservation r;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->shut) return FFTCG_ECANCELED;
        Class* c = nullptr;
        auto it = srv->classes.find({plan, precision});
        if (it == srv->classes.end()) {
            const int rc = make_class(srv, plan, precision, &c);
            if (rc != FFTCG_OK) return rc;
        } else {
            c = it->second.get();
        }
        if (!c->reserved) {
            // the class now outlives any request: the plan stays referenced
            // (fftcg_plan_destroy refuses it) until the server shuts down
            c->reserved = true;
            plan->refs.fetch_add(1);
        }
        r.c = c;
        r.slots = slots;
        srv->reserves.push_back(&r);
    }
    srv->cv.notify_all();
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        srv->cv_res.wait(lk, [&] { return r.done; });
    }
    if (r.rc != FFTCG_OK) return r.rc;
    // pinned input (d and b) and result buffers for as many requests, so
    // that their submissions and completions find them in the pool
    const size_t n = (size_t)plan->L * plan->L;
    for (int k = 0; k < slots; ++k) {
        void* pi = nullptr;
        void* px = nullptr;
        if (hipHostMalloc(&pi, n * 8 * 2, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&px, n * 8, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            if (pi) (void)hipHostFree(pi);
            return FFTCG_ENOMEM;
        }
        pin_put(srv, pi, n * 8 * 2, false, true);
        pin_put(srv, px, n * 8, false, true);
    }
    return FFTCG_OK;
} FFTCG_ABI_CATCH

extern "C" int fftcg_server_class_slots(fftcg_server_t srv, fftcg_plan_t plan, int precision, int* slots) try {
    if (!srv || !plan || !slots) return FFTCG_EINVAL;
    if (precision != FFTCG_FP64 && precision != FFTCG_MIXED) return FFTCG_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->classes.find({plan, precision});
    *slots = it == srv->classes.end() ? 0 : it->second->nslots.load();
    return FFTCG_OK;
} FFTCG_ABI_CATCH

static int poll_common(fftcg_server_t srv, uint64_t ticket, double* x, int* broken, int* step_iters,
                       double* step_bounds, fftcg_info* info, bool seq) {
    if (!srv) return FFTCG_EINVAL;
    std::unique_ptr<Request> q;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->requests.find(ticket);
        if (it == srv->requests.end()) return FFTCG_ENOTFOUND;
        if (seq != (it->second->steps > 0)) return FFTCG_EINVAL;
        if (!it->second->done) return FFTCG_PENDING;
        q = std::move(it->second);
        srv->requests.erase(it);
    }
    const int st = q->status;
    if (st == FFTCG_OK || st == FFTCG_ENOCONV) {
        if (x) memcpy(x, q->pin_x, q->n * 8);
        if (seq && broken) memcpy(broken, q->pin_broken, sizeof(int) * q->steps);
        if (seq && step_bounds) memcpy(step_bounds, q->pin_bounds, sizeof(double) * q->steps);
        if (seq && step_iters)
            for (int i = 0; i < q->steps; ++i) step_iters[i] = i < (int)q->step_iters.size() ? q->step_iters[i] : -1;
    }
    if (info) *info = q->info;
    free_request_buffers(srv, q.get());
    return st;
}

extern "C" int fftcg_poll(fftcg_server_t srv, uint64_t ticket, double* x, fftcg_info* info) try {
    return poll_common(srv, ticket, x, nullptr, nullptr, nullptr, info, false);
} FFTCG_ABI_CATCH

extern "C" int fftcg_poll_sequence(fftcg_server_t srv, uint64_t ticket, double* x, int* broken, int* step_iters,
                                   double* step_bounds, fftcg_info* info) try {
    return poll_common(srv, ticket, x, broken, step_iters, step_bounds, info, true);
} FFTCG_ABI_CATCH

extern "C" int fftcg_server_completed(fftcg_server_t srv, uint64_t* out, int cap, int* n) try {
    if (!srv || !n || cap < 0 || (cap > 0 && !out)) return FFTCG_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    int k = 0;
    while (k < cap && !srv->completed.empty()) {
        out[k++] = srv->completed.front();
        srv->completed.pop_front();
    }
    *n = k;
    return FFTCG_OK;
} FFTCG_ABI_CATCH

extern "C" int fftcg_server_get_stats(fftcg_server_t srv, fftcg_server_stats* out) try {
    if (!srv || !out) return FFTCG_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->stats;
    out->bytes_in_use = srv->bytes_in_use.load();
    out->queued = srv->queued;
    out->in_flight = srv->in_flight.load();
    return FFTCG_OK;
} FFTCG_ABI_CATCH

// Stops the scheduler, then ends every request still queued or running with
// FFTCG_ECANCELED (a solve whose results were already being copied back
// finishes with its own status) and releases the device memory.  Results stay
// pollable.  Runs once; later calls return at once.
static void shutdown_server(fftcg_server_s* srv) {
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->shut) return;
        srv->shut = true;  // later submissions return FFTCG_ECANCELED
    }
    srv->stop.store(true);
    srv->cv.notify_all();
    if (srv->thread.joinable()) srv->thread.join();
    {
        // reservations the scheduler did not reach
        std::lock_guard<std::mutex> lk(srv->mu);
        for (Reservation* r : srv->reserves) {
            r->rc = FFTCG_ECANCELED;
            r->done = true;
        }
        srv->reserves.clear();
    }
    srv->cv_res.notify_all();
    // the scheduler has stopped and no submission adds a class any more: the
    // classes are this thread's alone
    for (auto& kv : srv->classes) {
        Class* c = kv.second.get();
        if (c->stream) (void)hipStreamSynchronize(c->stream);
        for (auto& sp : c->slots) {
            Slot* s = sp.get();
            Request* q = s->req;
            if (!q) continue;
            if (!s->retiring) {
                // the iterations done so far go into the canceled request's info
                if (hipMemcpy(s->pin_state, s->ws->st, sizeof(SolveState), hipMemcpyDeviceToHost) != hipSuccess)
                    memset(s->pin_state, 0, sizeof(SolveState));
            }
            const SolveState st = *s->pin_state;
            std::lock_guard<std::mutex> lk(srv->mu);
            if (s->retiring) {
                // its result copies have landed (the stream is synchronised)
                if (q->steps > 0) q->step_iters.push_back(st.iters);
                finish_request(srv, q, q->x_nomem ? FFTCG_ENOMEM : st.status, st);
            } else {
                finish_request(srv, q, FFTCG_ECANCELED, st);
            }
            s->req = nullptr;
            s->retiring = false;
            srv->in_flight.fetch_sub(1);
        }
        std::lock_guard<std::mutex> lk(srv->mu);
        const SolveState none{};
        for (Request* q : c->pending) {
            finish_request(srv, q, FFTCG_ECANCELED, none);
            srv->queued -= 1;
        }
        c->pending.clear();
    }
    for (auto& kv : srv->classes) {
        destroy_class(kv.second.get());
        if (kv.second->reserved) kv.second->plan->refs.fetch_sub(1);
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->classes.clear();
    srv->bytes_in_use.store(0);
}

extern "C" int fftcg_server_shutdown(fftcg_server_t srv) try {
    if (!srv) return FFTCG_EINVAL;
    shutdown_server(srv);
    return FFTCG_OK;
} FFTCG_ABI_CATCH

extern "C" int fftcg_server_destroy(fftcg_server_t srv) try {
    if (!srv) return FFTCG_EINVAL;
    shutdown_server(srv);
    for (auto& kv : srv->requests) {
        Request* q = kv.second.get();
        if (!q->done) q->plan->refs.fetch_sub(1);
        free_request_buffers(srv, q);
    }
    for (auto& kv : srv->pin_free) (void)hipHostFree(kv.second);
    for (auto& kv : srv->page_free) free(kv.second);
    delete srv;
    return FFTCG_OK;
} FFTCG_ABI_CATCH
