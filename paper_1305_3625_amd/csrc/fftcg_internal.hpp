// Host-side internals shared by the C ABI, the fused engine and the server.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <new>
#include <vector>

#include "engine.hpp"
#include "fftcg.h"
#include "fftcg_types.hpp"

// Catch clauses of every C entry point, written as a function-try-block
// (`extern "C" int f(...) try { ... } FFTCG_ABI_CATCH`): no C++ exception
// crosses the C ABI.  A failed allocation of host containers becomes
// FFTCG_ENOMEM; anything else the C++ runtime throws (thread or mutex
// errors) FFTCG_EDEVICE.
#define FFTCG_ABI_CATCH                  \
    catch (const std::bad_alloc&) {      \
        return FFTCG_ENOMEM;             \
    }                                    \
    catch (...) {                        \
        return FFTCG_EDEVICE;            \
    }

namespace fftcg {

// Device buffers of one in-flight solve (reused across solves of a plan).
struct Workspace {
    int L = 0, M = 0, stride = 0;
    // interval between FP64 checks seen in the last single solve on this
    // workspace (first guess for the next one's chunk lengths; 0 = none)
    int check_period = 0;
    int check_period_prec = -1;  // precision and preconditioning it was seen with
    void* W = nullptr;  // pruned half spectrum, L x M/2 complex (FP64-sized)
    void* r = nullptr;  // working vectors, L*L doubles each (FP32 uses half)
    void* p = nullptr;
    void* q = nullptr;
    void* z = nullptr;     // preconditioned residual (preconditioned CG)
    float* e = nullptr;    // FP32 correction (mixed mode)
    float* d32 = nullptr;  // FP32 diagonal (mixed mode)
    double* part = nullptr;
    SolveState* st = nullptr;
    SlotDesc* slot = nullptr;
    SlotDesc* h_slot = nullptr;    // pinned staging
    SolveState* h_state = nullptr; // pinned staging
    int* h_status = nullptr;       // pinned, device-visible: {done, status}
    int* d_status = nullptr;       // device view of h_status
    double* ls_pv = nullptr;       // load-step partials
    int* ls_pi = nullptr;
    int* ls_out = nullptr;
    int* h_ls = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // launches of the grid-synchronised update on this workspace's partial
    // sums (each launch's barrier token is the next value)
    unsigned long long grid_token = 0;
    int init(int L, int M, int stride);
    void release();
    ~Workspace();
};

size_t workspace_bytes(int L, int M, int stride);
void cos_sin_2pi(long r, long M, double* c, double* s);
int plan_validate(int L, int padded, const double* g, double* gmin, double* gmax);
void init_state(SolveState* h, const struct ::fftcg_plan_s* p, int precision, double tol, int maxit, int refresh);
void fill_slot(SlotDesc* h, const Workspace* w, double* x, const double* b, const double* d);
int chunk_iters_for(int L);
int solve_validate(fftcg_plan_t plan, int precision, const void* d, const void* b, double tol, int maxit,
                   const void* x);

}  // namespace fftcg

namespace fftcg {
struct FusedOps;
}

struct fftcg_plan_s {
    int L = 0, M = 0, pad = 0, device = 0;
    int engine = FFTCG_ENGINE_AUTO;
    int precond = FFTCG_PRECOND_NONE;
    // certified error target per precision (FFTCG_FP64, FFTCG_MIXED); 0: the
    // solve's residual tolerance
    double tau_fixed[2] = {0.0, 0.0};
    int stride = 64;
    double gmin = 0, gmax = 0;
    const fftcg::EngineOps* ops = nullptr;
    void* tw32 = nullptr;
    void* tw64 = nullptr;
    void* ghq32 = nullptr;
    void* ghq64 = nullptr;
    void* ghN32 = nullptr;
    void* ghN64 = nullptr;
    fftcg::PlanTabs tabs{};
    std::vector<double> quarter;  // ghat(m, k), m, k in [0, M/2], FP64
    size_t device_bytes = 0;
    void* apply_W = nullptr;
    hipEvent_t apply_ev = nullptr;
    // fused (single-workgroup) engine: compiled size and constant tables
    int fused_ok = 0;
    const fftcg::FusedOps* fops = nullptr;
    void* f_tab64 = nullptr;  // per-plan constant tables of the fused engine
    void* f_tab32 = nullptr;
    size_t fused_bytes = 0;
    // update folded into the row-inverse pass behind a grid-wide barrier
    // (single solves, plain CG): mode 0 off, 1 on, 2 on with a zero wait
    // limit (tests of the fallback); capability per precision, found at
    // plan creation; set once a barrier gave up (the plan then keeps the
    // separate update kernel until the mode is set again)
    int grid_mode = 1;
    bool grid_cap[2] = {false, false};
    bool turn_cap[2] = {false, false};  // the turn pass (k_row_turn) resident as a whole, per precision
    std::atomic<int> grid_broken{0};
    std::mutex mu;
    std::vector<fftcg::Workspace*> free_ws;
    std::vector<fftcg::Workspace*> all_ws;
    std::atomic<int> refs{0};
    ~fftcg_plan_s();
};

namespace fftcg {
int plan_engine(const fftcg_plan_s* p);
int server_engine(const fftcg_plan_s* p);
Workspace* plan_acquire(fftcg_plan_s* p);
void plan_release(fftcg_plan_s* p, Workspace* w);
}  // namespace fftcg
