// C ABI: plans, operator products, device-resident CG solves, load steps.
//
// Sec. 3 of the paper: the CG loop of Listing 2 runs with every product
// evaluated by FFT (eq. (3)); Sec. 4: the GPU does almost all the work and
// reports only a few values to the CPU when the solver has finished.  Here a
// solve is a stream of kernel launches: an initial FP64 residual check, then
// chunks of CG iterations each followed by a (usually empty) FP64 check.  The
// CG scalars and the stop decision live in device memory; the host reads one
// pinned status word per chunk, two chunks behind the device so the GPU never
// waits for the host.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "engine.hpp"
#include "fftcg.h"
#include "fftcg_internal.hpp"
#include "fused.hpp"

namespace fftcg {

// ---- engine registry --------------------------------------------------------
#define FFTCG_DECL(M, P) const EngineOps* fftcg_engine_ops_##M##_##P();
#define FFTCG_SIZES(X)                                                                          \
    X(2, 0) X(4, 0) X(8, 0) X(16, 0) X(32, 0) X(64, 0) X(128, 0) X(256, 0) X(512, 0) X(1024, 0) \
        X(2048, 0) X(4096, 0) X(8192, 0) X(4, 1) X(8, 1) X(16, 1) X(32, 1) X(64, 1) X(128, 1)    \
            X(256, 1) X(512, 1) X(1024, 1) X(2048, 1) X(4096, 1) X(8192, 1)
FFTCG_SIZES(FFTCG_DECL)
#undef FFTCG_DECL

const EngineOps* find_engine(int M, int pad) {
#define FFTCG_CASE(MM, PP) \
    if (M == MM && pad == PP) return fftcg_engine_ops_##MM##_##PP();
    FFTCG_SIZES(FFTCG_CASE)
#undef FFTCG_CASE
    return nullptr;
}

// ---- helpers ----------------------------------------------------------------
static bool ispow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// cos and sin of 2 pi r / M with the argument reduced exactly: integer
// quadrant and octant folding, then the library functions on [0, pi/4].
void cos_sin_2pi(long r, long M, double* c, double* s) {
    r %= M;
    if (r < 0) r += M;
    if (M % 8 != 0) {
        // M in {1, 2, 4}: the values are exactly 0 or +-1
        const double k = (double)r / (double)M;
        const double tc[4] = {1.0, 0.0, -1.0, 0.0}, ts[4] = {0.0, 1.0, 0.0, -1.0};
        const int q = (int)(k * 4.0 + 0.5) & 3;
        *c = tc[q];
        *s = ts[q];
        return;
    }
    const long q = (4 * r) / M;
    const long e1 = r - q * (M / 4);
    double cc, ss;
    const double twopi = 6.283185307179586476925286766559;
    if (2 * e1 <= M / 4) {
        cc = cos(twopi * (double)e1 / (double)M);
        ss = sin(twopi * (double)e1 / (double)M);
    } else {
        const long f = M / 4 - e1;
        cc = sin(twopi * (double)f / (double)M);
        ss = cos(twopi * (double)f / (double)M);
    }
    switch (q) {
        case 0: *c = cc; *s = ss; break;
        case 1: *c = -ss; *s = cc; break;
        case 2: *c = -cc; *s = -ss; break;
        default: *c = ss; *s = -cc; break;
    }
}

#define HIPCHK(x)                                  \
    do {                                           \
        hipError_t e_ = (x);                       \
        if (e_ != hipSuccess) return FFTCG_EDEVICE; \
    } while (0)

static int check_device() {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return FFTCG_EDEVICE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FFTCG_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return FFTCG_EDEVICE;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return FFTCG_EDEVICE;
    return FFTCG_OK;
}

// ---- workspaces -------------------------------------------------------------
Workspace::~Workspace() { release(); }

void Workspace::release() {
    void* dev[] = {W, r, p, q, z, e, d32, part, st, slot, ls_pv, ls_pi, ls_out};
    for (void* v : dev)
        if (v) (void)hipFree(v);
    if (h_slot) (void)hipHostFree(h_slot);
    if (h_state) (void)hipHostFree(h_state);
    if (h_status) (void)hipHostFree(h_status);
    if (h_ls) (void)hipHostFree(h_ls);
    for (int i = 0; i < 2; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    W = r = p = q = z = nullptr;
    e = d32 = nullptr;
    part = nullptr;
    st = nullptr;
    slot = nullptr;
    h_slot = nullptr;
    h_state = nullptr;
    h_status = nullptr;
    ls_pv = nullptr;
    ls_pi = ls_out = nullptr;
    h_ls = nullptr;
    ev[0] = ev[1] = ev0 = ev1 = nullptr;
}

size_t workspace_bytes(int L, int M, int stride) {
    const size_t n = (size_t)L * L;
    const size_t N = (size_t)M / 2;
    return N * L * 16 + 4 * n * 8 + 2 * n * 4 + (size_t)NPART_SETS * stride * 8 + sizeof(SolveState) +
           sizeof(SlotDesc) + 4096;
}

int Workspace::init(int L_, int M_, int stride_) {
    L = L_;
    M = M_;
    stride = stride_;
    const size_t n = (size_t)L * L;
    const size_t N = (size_t)M / 2;
    HIPCHK(hipMalloc(&W, std::max<size_t>(N * L * 16, 256)));
    HIPCHK(hipMalloc(&r, n * 8));
    HIPCHK(hipMalloc(&p, n * 8));
    HIPCHK(hipMalloc(&q, n * 8));
    HIPCHK(hipMalloc(&z, n * 8));
    HIPCHK(hipMalloc((void**)&e, n * 4));
    HIPCHK(hipMalloc((void**)&d32, n * 4));
    HIPCHK(hipMalloc((void**)&part, (size_t)NPART_SETS * stride * 8));
    HIPCHK(hipMalloc((void**)&st, sizeof(SolveState)));
    HIPCHK(hipMalloc((void**)&slot, sizeof(SlotDesc)));
    const int nb = loadstep_blocks((int)n);
    HIPCHK(hipMalloc((void**)&ls_pv, nb * 8));
    HIPCHK(hipMalloc((void**)&ls_pi, nb * 4));
    HIPCHK(hipMalloc((void**)&ls_out, 16));
    HIPCHK(hipHostMalloc((void**)&h_slot, sizeof(SlotDesc), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&h_state, sizeof(SolveState), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&h_status, 16, hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer((void**)&d_status, h_status, 0));
    HIPCHK(hipHostMalloc((void**)&h_ls, 16, hipHostMallocDefault));
    HIPCHK(hipMemset(part, 0, (size_t)NPART_SETS * stride * 8));
    for (int i = 0; i < 2; ++i) HIPCHK(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
    HIPCHK(hipEventCreate(&ev0));
    HIPCHK(hipEventCreate(&ev1));
    return FFTCG_OK;
}

}  // namespace fftcg

using namespace fftcg;

// ---- plan -------------------------------------------------------------------
static int plan_stride(const EngineOps* ops, int L) {
    int s = std::max(64, L);
    if (ops) s = std::max({s, ops->rowblk32, ops->rowblk64, ops->g4});
    return (s + 63) & ~63;
}

template <typename T>
static std::vector<T> build_ghq(const double* g, int M, int TT) {
    const int N = M / 2, MH = M / 2 + 1, NT = N / TT;
    const double s = 1.0 / ((double)M * (double)M);
    std::vector<T> out((size_t)NT * MH * TT);
    for (int kt = 0; kt < NT; ++kt)
        for (int m = 0; m < MH; ++m)
            for (int kk = 0; kk < TT; ++kk)
                out[((size_t)kt * MH + m) * TT + kk] = (T)(g[(size_t)m * M + kt * TT + kk] * s);
    return out;
}

template <typename T>
static std::vector<T> build_ghN(const double* g, int M) {
    const int N = M / 2;
    const double s = 1.0 / ((double)M * (double)M);
    std::vector<T> out(N + 1);
    for (int m = 0; m <= N; ++m) out[m] = (T)(g[(size_t)m * M + N] * s);
    return out;
}

template <typename T>
static int upload(void** dst, const std::vector<T>& v, size_t* bytes) {
    const size_t b = std::max<size_t>(v.size() * sizeof(T), 16);
    HIPCHK(hipMalloc(dst, b));
    HIPCHK(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    *bytes += b;
    return FFTCG_OK;
}

fftcg_plan_s::~fftcg_plan_s() {
    for (Workspace* w : all_ws) delete w;
    void* dev[] = {tw32, tw64, ghq32, ghq64, ghN32, ghN64, apply_W};
    for (void* v : dev)
        if (v) (void)hipFree(v);
    if (apply_ev) (void)hipEventDestroy(apply_ev);
    fused_free(this);
}

int fftcg::plan_validate(int L, int padded, const double* g, double* gmin_out, double* gmax_out) {
    if (padded != 0 && padded != 1) return FFTCG_EINVAL;
    if (!ispow2(L) || L < 2 || (padded ? 2 * L : L) > 8192) return FFTCG_EINVAL;
    if (!g) return FFTCG_EINVAL;
    const int M = padded ? 2 * L : L;
    double gmin = INFINITY, gmax = 0.0;
    for (size_t i = 0; i < (size_t)M * M; ++i) {
        if (!isfinite(g[i])) return FFTCG_EINVAL;
        gmin = std::min(gmin, g[i]);
        gmax = std::max(gmax, fabs(g[i]));
    }
    const double tolv = 1e-12 * gmax;
    for (int m = 0; m < M; ++m)
        for (int k = 0; k < M; ++k) {
            const double v = g[(size_t)m * M + k];
            if (fabs(v - g[(size_t)((M - m) % M) * M + k]) > tolv) return FFTCG_EINVAL;
            if (fabs(v - g[(size_t)m * M + (M - k) % M]) > tolv) return FFTCG_EINVAL;
        }
    if (!(gmin > 0.0)) return FFTCG_ENOTSPD;
    *gmin_out = gmin;
    *gmax_out = gmax;
    return FFTCG_OK;
}

extern "C" int fftcg_plan(int L, int padded, const double* kernel_spectrum, fftcg_plan_t* out) try {
    if (!out) return FFTCG_EINVAL;
    double gmin = 0, gmax = 0;
    int rc = plan_validate(L, padded, kernel_spectrum, &gmin, &gmax);
    if (rc != FFTCG_OK) return rc;
    rc = check_device();
    if (rc != FFTCG_OK) return rc;
    const int M = padded ? 2 * L : L;
    // owned here until returned, so an exception below releases it
    std::unique_ptr<fftcg_plan_s> owner(new (std::nothrow) fftcg_plan_s());
    fftcg_plan_s* p = owner.get();
    if (!p) return FFTCG_ENOMEM;
    p->L = L;
    p->M = M;
    p->pad = padded;
    p->gmin = gmin;
    p->gmax = gmax;
    (void)hipGetDevice(&p->device);
    p->ops = find_engine(M, padded);
    p->stride = plan_stride(p->ops, L);
    if (p->ops) {
        p->grid_cap[0] = p->ops->grid_capable(FFTCG_FP64);
        p->grid_cap[1] = p->ops->grid_capable(FFTCG_MIXED);
        p->turn_cap[0] = p->grid_cap[0] && p->ops->turn_capable(FFTCG_FP64);
        p->turn_cap[1] = p->grid_cap[1] && p->ops->turn_capable(FFTCG_MIXED);
    }
    // quarter spectrum (host copy, FP64) for the fused engine
    p->quarter.resize((size_t)(M / 2 + 1) * (M / 2 + 1));
    for (int m = 0; m <= M / 2; ++m)
        for (int k = 0; k <= M / 2; ++k) p->quarter[(size_t)m * (M / 2 + 1) + k] = kernel_spectrum[(size_t)m * M + k];
    // twiddles exp(-2 pi i m / M)
    std::vector<double> tw64(2 * (size_t)M);
    std::vector<float> tw32(2 * (size_t)M);
    for (int m = 0; m < M; ++m) {
        double c, s;
        cos_sin_2pi(m, M, &c, &s);
        tw64[2 * m] = c;
        tw64[2 * m + 1] = -s;
        tw32[2 * m] = (float)c;
        tw32[2 * m + 1] = (float)-s;
    }
    size_t bytes = 0;
    int r2 = FFTCG_OK;
    if (p->ops) {
        r2 = upload(&p->tw32, tw32, &bytes);
        if (r2 == FFTCG_OK) r2 = upload(&p->tw64, tw64, &bytes);
        if (r2 == FFTCG_OK) r2 = upload(&p->ghq32, build_ghq<float>(kernel_spectrum, M, p->ops->tt32), &bytes);
        if (r2 == FFTCG_OK) r2 = upload(&p->ghq64, build_ghq<double>(kernel_spectrum, M, p->ops->tt64), &bytes);
        if (r2 == FFTCG_OK) r2 = upload(&p->ghN32, build_ghN<float>(kernel_spectrum, M), &bytes);
        if (r2 == FFTCG_OK) r2 = upload(&p->ghN64, build_ghN<double>(kernel_spectrum, M), &bytes);
        if (r2 == FFTCG_OK && hipMalloc(&p->apply_W, std::max<size_t>((size_t)(M / 2) * L * 16, 256)) != hipSuccess)
            r2 = FFTCG_ENOMEM;
        bytes += (size_t)(M / 2) * L * 16;
        if (r2 == FFTCG_OK && hipEventCreateWithFlags(&p->apply_ev, hipEventDisableTiming) != hipSuccess)
            r2 = FFTCG_EDEVICE;
    }
    if (r2 == FFTCG_OK) r2 = fused_init(p, kernel_spectrum);
    if (r2 != FFTCG_OK) return r2 == FFTCG_EDEVICE ? FFTCG_EDEVICE : FFTCG_ENOMEM;
    p->tabs = PlanTabs{p->tw32, p->ghq32, p->ghN32, p->tw64, p->ghq64, p->ghN64};
    p->device_bytes = bytes + p->fused_bytes;
    p->engine = FFTCG_ENGINE_AUTO;
    *out = owner.release();
    return FFTCG_OK;
} FFTCG_ABI_CATCH

extern "C" int fftcg_plan_destroy(fftcg_plan_t plan) try {
    if (!plan) return FFTCG_EINVAL;
    if (plan->refs.load() > 0) return FFTCG_EINVAL;
    (void)hipDeviceSynchronize();
    delete plan;
    return FFTCG_OK;
} FFTCG_ABI_CATCH

// AUTO: one workgroup per solve beats four kernel launches per iteration on
// the smallest grids.  A single solve takes the fused engine up to M = 64; a
// server class, whose slots share each launch of the multi-pass engine, up
// to M = 128 (measured crossovers: at M = 128 one fused solve is 15-25%
// slower than a multi-pass one, while 64 batched solves run as fast or
// faster fused; from M = 256 on the fused engine's serial rounds cost more).
int fftcg::plan_engine(const fftcg_plan_s* p) {
    if (p->precond != FFTCG_PRECOND_NONE) return FFTCG_ENGINE_MULTIPASS;  // the fused engine has no preconditioner
    if (p->engine == FFTCG_ENGINE_AUTO)
        return p->fused_ok && p->M <= 64 ? FFTCG_ENGINE_FUSED : FFTCG_ENGINE_MULTIPASS;
    return p->engine;
}

int fftcg::server_engine(const fftcg_plan_s* p) {
    if (p->precond != FFTCG_PRECOND_NONE) return FFTCG_ENGINE_MULTIPASS;
    if (p->engine == FFTCG_ENGINE_AUTO)
        return p->fused_ok && p->M <= 128 ? FFTCG_ENGINE_FUSED : FFTCG_ENGINE_MULTIPASS;
    return p->engine;
}

extern "C" int fftcg_plan_set_engine(fftcg_plan_t plan, int engine) try {
    if (!plan) return FFTCG_EINVAL;
    if (engine == FFTCG_ENGINE_AUTO) {
        plan->engine = engine;
        return FFTCG_OK;
    }
    if (engine == FFTCG_ENGINE_MULTIPASS) {
        if (!plan->ops) return FFTCG_EINVAL;
        plan->engine = engine;
        return FFTCG_OK;
    }
    if (engine == FFTCG_ENGINE_FUSED) {
        if (!plan->fused_ok) return FFTCG_EINVAL;
        plan->engine = engine;
        return FFTCG_OK;
    }
    return FFTCG_EINVAL;
} FFTCG_ABI_CATCH

extern "C" int fftcg_plan_set_precond(fftcg_plan_t plan, int kind) try {
    if (!plan) return FFTCG_EINVAL;
    if (kind != FFTCG_PRECOND_NONE && kind != FFTCG_PRECOND_CIRCULANT) return FFTCG_EINVAL;
    if (kind == FFTCG_PRECOND_CIRCULANT && !plan->ops) return FFTCG_EINVAL;
    if (plan->refs.load() > 0) return FFTCG_EINVAL;  // requests in a server use it
    std::lock_guard<std::mutex> lk(plan->mu);
    plan->precond = kind;
    return FFTCG_OK;
} FFTCG_ABI_CATCH

extern "C" int fftcg_plan_set_error_target(fftcg_plan_t plan, int precision, double tau) try {
    if (!plan) return FFTCG_EINVAL;
    if (precision != FFTCG_FP64 && precision != FFTCG_MIXED) return FFTCG_EINVAL;
    if (!(tau == 0.0 || (tau > 0.0 && tau < 1.0))) return FFTCG_EINVAL;
    if (plan->refs.load() > 0) return FFTCG_EINVAL;  // requests in a server use it
    std::lock_guard<std::mutex> lk(plan->mu);
    plan->tau_fixed[precision == FFTCG_MIXED ? 1 : 0] = tau;
    return FFTCG_OK;
} FFTCG_ABI_CATCH

// whether solves in `precision` on this plan use the turn pass (the folded
// update's mode, and the turn pass's grid resident as a whole)
static bool plan_turn(fftcg_plan_t plan, int precision) {
    return (plan->grid_mode == 1 || plan->grid_mode == 2) && plan->turn_cap[precision == FFTCG_MIXED];
}

extern "C" int fftcg_plan_set_grid_sync(fftcg_plan_t plan, int mode) try {
    if (!plan) return FFTCG_EINVAL;
    if (mode < 0 || mode > 3) return FFTCG_EINVAL;
    std::lock_guard<std::mutex> lk(plan->mu);
    plan->grid_mode = mode;
    plan->grid_broken.store(0);
    return FFTCG_OK;
} FFTCG_ABI_CATCH

extern "C" int fftcg_plan_get_grid_sync(fftcg_plan_t plan, int precision, int* state) try {
    if (!plan || !state) return FFTCG_EINVAL;
    if (precision != FFTCG_FP64 && precision != FFTCG_MIXED) return FFTCG_EINVAL;
    if (!plan->ops || !plan->grid_cap[precision == FFTCG_MIXED ? 1 : 0])
        *state = FFTCG_GRID_UNSUPPORTED;
    else if (plan->grid_mode == 0)
        *state = FFTCG_GRID_OFF;
    else if (plan->grid_broken.load())
        *state = FFTCG_GRID_FELL_BACK;
    else
        *state = plan_turn(plan, precision) ? FFTCG_GRID_ON_TURN : FFTCG_GRID_ON;
    return FFTCG_OK;
} FFTCG_ABI_CATCH

extern "C" int fftcg_plan_info(fftcg_plan_t plan, int* L, int* M, int* padded, size_t* device_bytes) try {
    if (!plan) return FFTCG_EINVAL;
    if (L) *L = plan->L;
    if (M) *M = plan->M;
    if (padded) *padded = plan->pad;
    if (device_bytes) *device_bytes = plan->device_bytes;
    return FFTCG_OK;
} FFTCG_ABI_CATCH

// ---- apply -------------------------------------------------------------------
// Wait limit of the grid-wide barrier (ticks of the 100 MHz constant clock):
// 20 ms, a thousand times the 8-20 us between the first and the last
// arrival in a resident grid; a solve abandoned at a barrier costs this once.
constexpr long long kGridWaitTicks = 2000000;

static bool overlap(const void* a, const void* b, size_t n) {
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + n && y < x + n;
}

extern "C" int fftcg_apply(fftcg_plan_t plan, int precision, const double* d, const double* x, double* y,
                           void* stream) try {
    if (!plan || !d || !x || !y) return FFTCG_EINVAL;
    if (precision != FFTCG_FP64 && precision != FFTCG_MIXED) return FFTCG_EINVAL;
    const size_t nb = (size_t)plan->L * plan->L * 8;
    if (overlap(y, x, nb) || overlap(y, d, nb)) return FFTCG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(plan->mu);
    if (plan_engine(plan) == FFTCG_ENGINE_FUSED) {
        return fused_apply(plan, precision, d, x, y, s);
    }
    if (!plan->ops) return FFTCG_EINVAL;
    HIPCHK(hipStreamWaitEvent(s, plan->apply_ev, 0));
    plan->ops->apply(precision, plan->tabs, d, x, y, plan->apply_W, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(plan->apply_ev, s));
    return FFTCG_OK;
} FFTCG_ABI_CATCH

extern "C" int fftcg_profile_apply(fftcg_plan_t plan, int precision, const double* d, const double* x, double* y,
                                   int reps, double* ms_per_pass, void* stream) try {
    if (!plan || !d || !x || !y || !ms_per_pass || reps < 1) return FFTCG_EINVAL;
    if (precision != FFTCG_FP64 && precision != FFTCG_MIXED) return FFTCG_EINVAL;
    const size_t nb = (size_t)plan->L * plan->L * 8;
    if (overlap(y, x, nb) || overlap(y, d, nb)) return FFTCG_EINVAL;
    if (!plan->ops || plan_engine(plan) == FFTCG_ENGINE_FUSED) return FFTCG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(plan->mu);
    hipEvent_t ev[4];
    for (int i = 0; i < 4; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) return FFTCG_EDEVICE;
    int rc = FFTCG_OK;
    double acc[3] = {0, 0, 0};
    constexpr int RUN = 8;  // back-to-back launches per timed run
    const int blocks = (reps + RUN - 1) / RUN;
    if (hipStreamWaitEvent(s, plan->apply_ev, 0) != hipSuccess) rc = FFTCG_EDEVICE;
    for (int it = 0; it < blocks && rc == FFTCG_OK; ++it) {
        (void)hipEventRecord(ev[0], s);
        for (int pass = 0; pass < 3; ++pass) {
            for (int k = 0; k < RUN; ++k)
                plan->ops->apply_pass(precision, pass, plan->tabs, d, x, y, plan->apply_W, s);
            (void)hipEventRecord(ev[pass + 1], s);
        }
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(ev[3]) != hipSuccess) {
            rc = FFTCG_EDEVICE;
            break;
        }
        for (int pass = 0; pass < 3; ++pass) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev[pass], ev[pass + 1]);
            acc[pass] += ms;
        }
    }
    (void)hipEventRecord(plan->apply_ev, s);
    for (int i = 0; i < 4; ++i) (void)hipEventDestroy(ev[i]);
    if (rc == FFTCG_OK)
        for (int pass = 0; pass < 3; ++pass) ms_per_pass[pass] = acc[pass] / (blocks * RUN);
    return rc;
} FFTCG_ABI_CATCH

extern "C" int fftcg_profile_iteration(fftcg_plan_t plan, int precision, const double* d, const double* b,
                                       double* x, int reps, double* ms_per_pass, int* folded, void* stream) try {
    if (!plan || !d || !b || !x || !ms_per_pass || reps < 1 || reps > 100) return FFTCG_EINVAL;
    if (precision != FFTCG_FP64 && precision != FFTCG_MIXED) return FFTCG_EINVAL;
    if (!plan->ops || plan_engine(plan) == FFTCG_ENGINE_FUSED) return FFTCG_EINVAL;
    const size_t n = (size_t)plan->L * plan->L;
    if (overlap(x, d, n * 8) || overlap(x, b, n * 8)) return FFTCG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const EngineOps* ops = plan->ops;
    const bool grid = plan->grid_mode != 0 && !plan->grid_broken.load() && plan->grid_cap[precision == FFTCG_MIXED];
    const bool turn = grid && plan_turn(plan, precision);
    if (turn && reps < 2) return FFTCG_EINVAL;
    // the launches in the order a solve's chunk makes them: with the turn
    // pass row_fwd, col, (turn, col) x (reps - 1), row_inv; else per
    // iteration row_fwd, col, row_inv and (without the folded update) update
    std::vector<int> seq;
    if (turn) {
        seq = {0, 1};
        for (int k = 1; k < reps; ++k) seq.insert(seq.end(), {4, 1});
        seq.push_back(2);
    } else {
        for (int k = 0; k < reps; ++k)
            for (int pass = 0; pass < (grid ? 3 : 4); ++pass) seq.push_back(pass);
    }
    Workspace* w = plan_acquire(plan);
    if (!w) return FFTCG_ENOMEM;
    int rc = FFTCG_OK;
    // a start and an end event per launch, recorded by the launch itself
    // (the kernel's own execution, as a kernel trace reports it)
    std::vector<hipEvent_t> ev((size_t)2 * seq.size(), nullptr);
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            rc = FFTCG_EDEVICE;
        }
    do {
        if (rc != FFTCG_OK) break;
        // plain CG from x = 0 with nothing that would pause the iterations:
        // no periodic check, no reliable update, an unreachable tolerance
        fill_slot(w->h_slot, w, x, b, d);
        w->h_slot->mask = nullptr;
        init_state(w->h_state, plan, precision, 1e-30, 1 << 30, 0);
        w->h_state->pcg = 0;
        w->h_state->delta2 = 0.0;
        w->h_state->bar_limit = kGridWaitTicks;
        for (int i = 0; i < 4; ++i) w->h_status[i] = 0;
        hipError_t he = hipMemcpyAsync(w->slot, w->h_slot, sizeof(SlotDesc), hipMemcpyHostToDevice, s);
        if (he == hipSuccess) he = hipMemcpyAsync(w->st, w->h_state, sizeof(SolveState), hipMemcpyHostToDevice, s);
        if (he == hipSuccess) he = hipMemsetAsync(x, 0, n * 8, s);
        if (he == hipSuccess && precision == FFTCG_MIXED) {
            he = hipMemsetAsync(w->e, 0, n * 4, s);
            if (he == hipSuccess) launch_to_f32(d, w->d32, (int)n, s);
        }
        if (he != hipSuccess) {
            rc = FFTCG_EDEVICE;
            break;
        }
        ops->check0(precision, plan->tabs, w->slot, 1, plan->stride, s);
        for (size_t i = 0; i < seq.size(); ++i) {
            const int pass = seq[i];
            unsigned long long token = 0;
            if (grid && pass == 2) {
                token = ++w->grid_token;
            } else if (pass == 4) {
                token = w->grid_token + 1;
                w->grid_token += 2;
            }
            ops->iter_pass(precision, pass, grid, plan->tabs, w->slot, plan->stride, token, ev[2 * i], ev[2 * i + 1],
                           s);
        }
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(w->h_state, w->st, sizeof(SolveState), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = FFTCG_EDEVICE;
            break;
        }
        const SolveState st = *w->h_state;
        if (st.status == ST_EGRID) {
            plan->grid_broken.store(1);
            rc = FFTCG_EDEVICE;
            break;
        }
        if (st.done || st.pause || st.iters != reps) {
            rc = (st.done && st.status < 0) ? st.status : FFTCG_EINVAL;
            break;
        }
        double acc[5] = {0, 0, 0, 0, 0};
        int cnt[5] = {0, 0, 0, 0, 0};
        for (size_t i = 0; i < seq.size(); ++i) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
            acc[seq[i]] += ms;
            cnt[seq[i]] += 1;
        }
        // (the separate update launches nothing when the update is folded)
        for (int pass = 0; pass < 5; ++pass)
            ms_per_pass[pass] = (cnt[pass] > 0 && !(grid && pass == 3)) ? acc[pass] / cnt[pass] : 0.0;
        if (folded) *folded = turn ? 2 : (grid ? 1 : 0);
    } while (0);
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    plan_release(plan, w);
    return rc;
} FFTCG_ABI_CATCH

extern "C" int fftcg_stream_probe(int kind, int nontemporal, void* dst, const void* src, size_t bytes, int blocks,
                                  int reps, double* ms_per_launch, void* stream) try {
    if (kind < 0 || kind > 2 || !ms_per_launch || bytes == 0 || bytes % 16 != 0 || blocks < 1 ||
        blocks > (1 << 20) || reps < 1)
        return FFTCG_EINVAL;
    if (!dst || ((uintptr_t)dst & 15)) return FFTCG_EINVAL;  // kind 0: the sink
    if (kind != 1 && (!src || ((uintptr_t)src & 15))) return FFTCG_EINVAL;
    if (kind == 2 && overlap(dst, src, bytes)) return FFTCG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t ev[2] = {nullptr, nullptr};
    int rc = FFTCG_OK;
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) rc = FFTCG_EDEVICE;
    if (rc == FFTCG_OK) {
        launch_stream(kind, nontemporal != 0, blocks, dst, src, bytes, s);  // untimed first launch
        (void)hipEventRecord(ev[0], s);
        for (int r = 0; r < reps; ++r) launch_stream(kind, nontemporal != 0, blocks, dst, src, bytes, s);
        (void)hipEventRecord(ev[1], s);
        float ms = 0.f;
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
            hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess)
            rc = FFTCG_EDEVICE;
        else
            *ms_per_launch = ms / reps;
    }
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    return rc;
} FFTCG_ABI_CATCH

// ---- solve -------------------------------------------------------------------
Workspace* fftcg::plan_acquire(fftcg_plan_s* p) {
    std::lock_guard<std::mutex> lk(p->mu);
    if (!p->free_ws.empty()) {
        Workspace* w = p->free_ws.back();
        p->free_ws.pop_back();
        return w;
    }
    Workspace* w = new (std::nothrow) Workspace();
    if (!w) return nullptr;
    if (w->init(p->L, p->M, p->stride) != FFTCG_OK) {
        delete w;
        return nullptr;
    }
    p->all_ws.push_back(w);
    return w;
}

void fftcg::plan_release(fftcg_plan_s* p, Workspace* w) {
    std::lock_guard<std::mutex> lk(p->mu);
    p->free_ws.push_back(w);
}

void fftcg::init_state(SolveState* h, const fftcg_plan_s* p, int precision, double tol, int maxit, int refresh) {
    memset(h, 0, sizeof(SolveState));
    h->tol = tol;
    // certified relative error target: the plan's fixed one for this
    // precision, else the residual tolerance
    h->tau = p->tau_fixed[precision == FFTCG_MIXED ? 1 : 0] > 0.0 ? p->tau_fixed[precision == FFTCG_MIXED ? 1 : 0]
                                                                   : tol;
    h->gmin = p->gmin;
    h->maxit = maxit;
    h->refresh = precision == FFTCG_MIXED ? refresh : 0;
    h->pause = 1;
    h->restart = 1;
    h->iters_literal = -1;
    h->mixed = precision == FFTCG_MIXED ? 1 : 0;
    h->trigger_rr = 0.0;
    h->best_rt = INFINITY;
    // mixed mode: residual replacement each time the FP32 recursive residual
    // has fallen by 1e-2 since the last one (reliable updates)
    // (preconditioned solves: by 1e-4, as they run only tens of iterations,
    // so the FP32 recursion drifts little between replacements)
#ifndef FFTCG_CG_DELTA2
#define FFTCG_CG_DELTA2 1e-4
#endif
    h->delta2 = precision == FFTCG_MIXED ? (p->precond == FFTCG_PRECOND_CIRCULANT ? 1e-8 : FFTCG_CG_DELTA2) : 0.0;
    h->rho_ref = 0.0;
    h->pcg = p->precond == FFTCG_PRECOND_CIRCULANT ? 1 : 0;
}

void fftcg::fill_slot(SlotDesc* h, const Workspace* w, double* x, const double* b, const double* d) {
    memset(h, 0, sizeof(SlotDesc));
    h->x = x;
    h->b = b;
    h->d = d;
    h->r = w->r;
    h->p = w->p;
    h->q = w->q;
    h->z = w->z;
    h->e = w->e;
    h->d32 = w->d32;
    h->W = w->W;
    h->part = w->part;
    h->st = w->st;
    h->host_status = w->d_status;
    h->active = 1;
}

int fftcg::chunk_iters_for(int L) { return L >= 512 ? 10 : 16; }

int fftcg::solve_validate(fftcg_plan_t plan, int precision, const void* d, const void* b, double tol, int maxit,
                   const void* x) {
    if (!plan || !d || !b || !x) return FFTCG_EINVAL;
    if (precision != FFTCG_FP64 && precision != FFTCG_MIXED) return FFTCG_EINVAL;
    if (!(tol > 0.0) || !(tol < 1.0) || !isfinite(tol)) return FFTCG_EINVAL;
    if (maxit < 1) return FFTCG_EINVAL;
    return FFTCG_OK;
}

static void fill_info(fftcg_info* info, const SolveState& st, float ms) {
    if (!info) return;
    info->status = st.status;
    info->iterations = st.iters;
    info->iterations_literal = st.iters_literal;
    info->checks = st.checks;
    info->true_relres = st.true_relres;
    info->error_bound = st.bound;
    info->lambda_lb = st.lam_lb;
    info->device_ms = ms;
}

// Chunk lengths of a single solve.  Each chunk is K iterations followed by
// an FP64-check sequence; a check that falls due inside a chunk leaves the
// rest of its iterations idle, and a check sequence with no check due does
// nothing, so chunks should end where the next check falls due.  Checks come
// at roughly even intervals (a residual replacement each time r.r has fallen
// by a fixed factor, or every refresh iterations), so the next one is
// expected one interval after the last.  The host sees the iteration count
// and last check of the chunk before the one in flight.  Until a solve has
// seen an interval of its own it takes the one the previous solve on the
// same workspace ended with (solves on one plan tend to be alike).
// Planned chunks run up to this many nominal chunk lengths while the next
// check is expected further off: one chunk then covers a whole check
// interval (about 30 iterations at L = 2048), and each chunk boundary costs
// a check sequence that exits at once, the launch gap, and with the turn
// pass a forward and a row-inverse pass in place of one turn.  4 against 2:
// plain L = 2048 / 1024 / 512 mixed +0.5 / +0.7 / +1.3%, preconditioned
// L = 2048 / 512 +0.4 / +1.2%, the same iterations and checks.
constexpr int kChunkSpan = 4;

struct ChunkPlanner {
    int kmax;
    int known_iters = 0;  // iterations at the end of the last chunk the host has seen
    int last_check = 0;   // iteration of the last check seen (the first is at 0)
    int period = 0;       // last interval between checks, 0 = none seen yet
    int k_prev = 0;       // length of the chunk in flight
    ChunkPlanner(int km, int guess) : kmax(km), period(guess) {}
    int next() {
        int k = kmax;
        if (period > 0) {
            const int start = known_iters + k_prev;  // expected start of this chunk
            const int due = last_check + period;
            // up to kChunkSpan nominal chunks while the next check is far
            // off.  A check due once `due` iterations are done is decided by
            // the forward pass of iteration `due`, so the chunk takes that
            // iteration in: it pauses there and the check sequence after the
            // chunk runs the check (ending before it left the decision to a
            // further chunk: plain +0.2 to +0.5%, preconditioned +1.4 to +4%)
            k = due > start ? std::min(kChunkSpan * kmax, due - start + 1) : 2;
        }
        k_prev = k;
        return k;
    }
    void observe(int iters, int check_iter) {
        known_iters = iters;
        if (check_iter > last_check) {
            period = check_iter - last_check;
            last_check = check_iter;
        }
    }
};

static int solve_multipass_once(fftcg_plan_t plan, Workspace* w, int precision, const double* d, const double* b,
                                const double* x0, double tol, int maxit, double* x, fftcg_info* info,
                                hipStream_t s, const uint8_t* mask, bool grid);

static int solve_multipass(fftcg_plan_t plan, int precision, const double* d, const double* b, const double* x0,
                           double tol, int maxit, double* x, fftcg_info* info, hipStream_t s,
                           const uint8_t* mask = nullptr) {
    Workspace* w = plan_acquire(plan);
    if (!w) return FFTCG_ENOMEM;
    const size_t n = (size_t)plan->L * plan->L;
    bool grid = plan->grid_mode != 0 && !plan->grid_broken.load() && plan->grid_cap[precision == FFTCG_MIXED] &&
                plan->precond == FFTCG_PRECOND_NONE;
    int rc = FFTCG_OK;
    // a warm start in place is kept in q, which the grid-synchronised path
    // never writes, so that a solve abandoned at a barrier can be repeated
    if (grid && x0 && x0 == x &&
        hipMemcpyAsync(w->q, x, n * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
        grid = false;
    rc = solve_multipass_once(plan, w, precision, d, b, x0, tol, maxit, x, info, s, mask, grid);
    if (rc == ST_EGRID) {
        // the grid was not resident as a whole (other work on the device):
        // the plan falls back to the separate update kernel, and the solve
        // is repeated from its start
        plan->grid_broken.store(1);
        rc = FFTCG_OK;
        if (x0 && x0 == x && hipMemcpyAsync(x, w->q, n * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
            rc = FFTCG_EDEVICE;
        if (rc == FFTCG_OK)
            rc = solve_multipass_once(plan, w, precision, d, b, x0, tol, maxit, x, info, s, mask, false);
        if (rc == ST_EGRID) rc = FFTCG_EDEVICE;
    }
    plan_release(plan, w);
    return rc;
}

static int solve_multipass_once(fftcg_plan_t plan, Workspace* w, int precision, const double* d, const double* b,
                                const double* x0, double tol, int maxit, double* x, fftcg_info* info,
                                hipStream_t s, const uint8_t* mask, bool grid) {
    const EngineOps* ops = plan->ops;
    const size_t n = (size_t)plan->L * plan->L;
    int rc = FFTCG_OK;
    do {
        fill_slot(w->h_slot, w, x, b, d);
        w->h_slot->mask = mask;
        init_state(w->h_state, plan, precision, tol, maxit, 50);
        w->h_state->bar_limit = plan->grid_mode == 2 ? 0 : kGridWaitTicks;
        for (int i = 0; i < 4; ++i) w->h_status[i] = 0;
        if (hipMemcpyAsync(w->slot, w->h_slot, sizeof(SlotDesc), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(w->st, w->h_state, sizeof(SolveState), hipMemcpyHostToDevice, s) != hipSuccess) {
            rc = FFTCG_EDEVICE;
            break;
        }
        if (hipEventRecord(w->ev0, s) != hipSuccess) {
            rc = FFTCG_EDEVICE;
            break;
        }
        hipError_t he = hipSuccess;
        if (!x0)
            he = hipMemsetAsync(x, 0, n * 8, s);
        else if (x0 != x)
            he = hipMemcpyAsync(x, x0, n * 8, hipMemcpyDeviceToDevice, s);
        if (he == hipSuccess && precision == FFTCG_MIXED) {
            he = hipMemsetAsync(w->e, 0, n * 4, s);
            if (he == hipSuccess) launch_to_f32(d, w->d32, (int)n, s);
        }
        if (he != hipSuccess) {
            rc = FFTCG_EDEVICE;
            break;
        }
        const bool pcg = plan->precond == FFTCG_PRECOND_CIRCULANT;
        const auto iter = pcg ? ops->iter_pcg : ops->iter;
        const auto check = pcg ? ops->check_pcg : ops->check;
        // from zero the first residual is b itself: no product
        const auto first = x0 ? check : (pcg ? ops->check0_pcg : ops->check0);
        first(precision, plan->tabs, w->slot, 1, plan->stride, s);
        // preconditioned solves check every few iterations (they converge in
        // tens): shorter chunks leave fewer iterations idle behind a check
        const int kmax = pcg ? std::max(2, chunk_iters_for(plan->L) / 2) : chunk_iters_for(plan->L);
        const long max_chunks = 2 * (long)maxit + 64;
        // (mixed precision only: an FP64 solve's one interval is its whole
        // length, a poor guess for the next solve)
        const int pkey = 2 * precision + (pcg ? 1 : 0);
        const bool carry = precision == FFTCG_MIXED && w->check_period_prec == pkey;
        ChunkPlanner planner(kmax, carry ? w->check_period : 0);
        long c = 0;
        bool finished = false;
        while (!finished) {
            const int K = planner.next();
            if (grid)
                ops->iter_grid_chunk(precision, plan->tabs, w->slot, plan->stride, &w->grid_token, K,
                                     plan_turn(plan, precision), s);
            else
                for (int k = 0; k < K; ++k) iter(precision, plan->tabs, w->slot, 1, plan->stride, s);
            check(precision, plan->tabs, w->slot, 1, plan->stride, s);
            if (hipGetLastError() != hipSuccess || hipEventRecord(w->ev[c & 1], s) != hipSuccess) {
                rc = FFTCG_EDEVICE;
                break;
            }
            if (c >= 1) {
                if (hipEventSynchronize(w->ev[(c - 1) & 1]) != hipSuccess) {
                    rc = FFTCG_EDEVICE;
                    break;
                }
                if (__atomic_load_n(&w->h_status[0], __ATOMIC_ACQUIRE)) finished = true;
                planner.observe(__atomic_load_n(&w->h_status[3], __ATOMIC_RELAXED),
                                __atomic_load_n(&w->h_status[2], __ATOMIC_RELAXED));
            }
            ++c;
            if (c > max_chunks) {
                rc = FFTCG_EDEVICE;
                break;
            }
        }
        if (rc != FFTCG_OK) break;
        w->check_period = planner.period;
        w->check_period_prec = pkey;
        if (hipEventRecord(w->ev1, s) != hipSuccess ||
            hipMemcpyAsync(w->h_state, w->st, sizeof(SolveState), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = FFTCG_EDEVICE;
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, w->ev0, w->ev1);
        const SolveState st = *w->h_state;
        if (st.bzero) {
            if (hipMemsetAsync(x, 0, n * 8, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
                rc = FFTCG_EDEVICE;
                break;
            }
        }
        rc = st.status;
        if (rc != ST_EGRID) fill_info(info, st, ms);
    } while (0);
    return rc;
}

extern "C" int fftcg_solve(fftcg_plan_t plan, int precision, const double* d, const double* b, const double* x0,
                           double tol, int maxit, double* x, fftcg_info* info, void* stream) try {
    int rc = solve_validate(plan, precision, d, b, tol, maxit, x);
    if (rc != FFTCG_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (plan_engine(plan) == FFTCG_ENGINE_FUSED) return fused_solve(plan, precision, d, b, x0, tol, maxit, x, info, s);
    if (!plan->ops) return FFTCG_EINVAL;
    return solve_multipass(plan, precision, d, b, x0, tol, maxit, x, info, s);
} FFTCG_ABI_CATCH

// ---- load step ---------------------------------------------------------------
extern "C" int fftcg_loadstep(fftcg_plan_t plan, const double* x, const double* t, double* d, int* index,
                              void* stream) try {
    if (!plan || !x || !t || !d || !index) return FFTCG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Workspace* w = plan_acquire(plan);
    if (!w) return FFTCG_ENOMEM;
    const int n = plan->L * plan->L;
    launch_loadstep(x, t, d, n, w->ls_pv, w->ls_pi, w->ls_out, s);
    int rc = FFTCG_OK;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(w->h_ls, w->ls_out, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        rc = FFTCG_EDEVICE;
    else
        *index = w->h_ls[0];
    plan_release(plan, w);
    return rc;
} FFTCG_ABI_CATCH

extern "C" int fftcg_loadstep_noalloc(fftcg_plan_t plan, const double* x, const double* t, double* d, int* index,
                                      void* stream) try {
    if (!plan || !x || !t || !d || !index) return FFTCG_EINVAL;
    const long n = (long)plan->L * plan->L;
    if (n > 0x7fffffffL) return FFTCG_EINVAL;
    const int rc = loadstep_noalloc(x, t, d, (int)n, index, (hipStream_t)stream);
    return rc == 0 ? FFTCG_OK : (rc == -1 ? FFTCG_EINVAL : FFTCG_EDEVICE);
} FFTCG_ABI_CATCH

// ---- misc -------------------------------------------------------------------
extern "C" const char* fftcg_strerror(int status) {
    switch (status) {
        case FFTCG_OK: return "ok";
        case FFTCG_PENDING: return "pending";
        case FFTCG_EINVAL: return "invalid argument";
        case FFTCG_ENOMEM: return "out of memory or over budget";
        case FFTCG_ENOTSPD: return "spectrum not positive: operator not SPD";
        case FFTCG_ENOCONV: return "not converged within maxit";
        case FFTCG_EBREAKDOWN: return "CG breakdown (p.q <= 0 or non-finite)";
        case FFTCG_EAGAIN: return "queue full, try again";
        case FFTCG_EDEVICE: return "device error or no gfx950 GPU";
        case FFTCG_ENOTFOUND: return "unknown ticket";
        case FFTCG_ECANCELED: return "canceled";
        default: return "unknown status";
    }
}

extern "C" const char* fftcg_version(void) { return "fftcg 0.1.0 (gfx950)"; }

// ---- quasi-static fracture driver -------------------------------------------
// Sec. 2: displacement control with uniform fibre stiffness k.  At unit
// displacement the intact fibres carry f with (I/k + G)_II f_I = 1_I (eq. (2)
// divided by k, restricted to the intact set I; broken fibres carry no force
// and are projected out of the solve).  The fibre with the largest f_i/t_i
// breaks next, at the displacement D = t_i/f_i; then the next step solves
// again, warm-started from the previous forces.
extern "C" int fftcg_fracture(fftcg_plan_t plan, int precision, double k, const double* t, int steps, double tol,
                              int maxit, double* f, int* broken, double* dbreak, int* iters, void* stream) try {
    if (!plan || !t || !f || !broken || !dbreak) return FFTCG_EINVAL;
    if (precision != FFTCG_FP64 && precision != FFTCG_MIXED) return FFTCG_EINVAL;
    if (!(k > 0.0) || !isfinite(k) || !(tol > 0.0 && tol < 1.0) || maxit < 1) return FFTCG_EINVAL;
    const size_t n = (size_t)plan->L * plan->L;
    if (steps < 1 || (size_t)steps > n || !plan->ops) return FFTCG_EINVAL;
    const int rc0 = check_device();
    if (rc0 != FFTCG_OK) return rc0;
    hipStream_t s = (hipStream_t)stream;
    uint8_t* mask = nullptr;
    double *d = nullptr, *b = nullptr, *pv = nullptr, *outv = nullptr, *h_v = nullptr;
    int *pi = nullptr, *out = nullptr, *h_i = nullptr;
    const int nb = loadstep_blocks((int)n);
    int rc = FFTCG_OK;
    if (hipMalloc(&mask, n) != hipSuccess || hipMalloc(&d, n * 8) != hipSuccess || hipMalloc(&b, n * 8) != hipSuccess ||
        hipMalloc(&pv, nb * 8) != hipSuccess || hipMalloc(&pi, nb * 4) != hipSuccess ||
        hipMalloc(&out, 16) != hipSuccess || hipMalloc(&outv, 16) != hipSuccess ||
        hipHostMalloc((void**)&h_v, 16, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h_i, 16, hipHostMallocDefault) != hipSuccess)
        rc = FFTCG_ENOMEM;
    if (rc == FFTCG_OK) {
        launch_fill(d, 1.0 / k, (int)n, s);
        launch_fill(b, 1.0, (int)n, s);
        if (hipMemsetAsync(mask, 1, n, s) != hipSuccess || hipMemsetAsync(f, 0, n * 8, s) != hipSuccess ||
            hipGetLastError() != hipSuccess)
            rc = FFTCG_EDEVICE;
    }
    for (int step = 0; step < steps && rc == FFTCG_OK; ++step) {
        fftcg_info info{};
        const int st = solve_multipass(plan, precision, d, b, f, tol, maxit, f, &info, s, mask);
        if (st != FFTCG_OK) {
            rc = st;
            break;
        }
        launch_breakstep(f, t, mask, (int)n, pv, pi, out, outv, s);
        if (hipGetLastError() != hipSuccess || hipMemcpyAsync(h_i, out, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(h_v, outv, 8, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
            rc = FFTCG_EDEVICE;
            break;
        }
        broken[step] = h_i[0];
        dbreak[step] = h_v[0] > 0.0 ? 1.0 / h_v[0] : INFINITY;
        if (iters) iters[step] = info.iterations;
    }
    (void)hipStreamSynchronize(s);
    void* dv[] = {mask, d, b, pv, pi, out, outv};
    for (void* v : dv)
        if (v) (void)hipFree(v);
    if (h_v) (void)hipHostFree(h_v);
    if (h_i) (void)hipHostFree(h_i);
    return rc;
} FFTCG_ABI_CATCH
