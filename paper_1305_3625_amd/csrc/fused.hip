// Fused single-workgroup engine: host side (tables, dispatch to the kernels
// compiled per grid size in fused_inst.hip).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <vector>

#include "common.hpp"
#include "fftcg_internal.hpp"
#include "fused.hpp"

namespace fftcg {

#define FFTCG_FUSED_DECL(M, P) const FusedOps* fftcg_fused_ops_##M##_##P();
#define FFTCG_FUSED_SIZES(X)                                                                            \
    X(2, 0) X(4, 0) X(8, 0) X(16, 0) X(32, 0) X(64, 0) X(128, 0) X(256, 0) X(4, 1) X(8, 1) X(16, 1) \
        X(32, 1) X(64, 1) X(128, 1) X(256, 1)
FFTCG_FUSED_SIZES(FFTCG_FUSED_DECL)
#undef FFTCG_FUSED_DECL

const FusedOps* find_fused(int M, int pad) {
#define FFTCG_CASE(MM, PP) \
    if (M == MM && pad == PP) return fftcg_fused_ops_##MM##_##PP();
    FFTCG_FUSED_SIZES(FFTCG_CASE)
#undef FFTCG_CASE
    return nullptr;
}

namespace {

FusedTabs tabs_of(const fftcg_plan_s* p) {
    const char* b64 = (const char*)p->f_tab64;
    const char* b32 = (const char*)p->f_tab32;
    const int M = p->M;
    FusedTabs ft;
    ft.tw64 = b64;
    ft.gq64 = b64 + sizeof(double) * 2 * M;
    ft.tw32 = b32;
    ft.gq32 = b32 + sizeof(float) * 2 * M;
    return ft;
}

}  // namespace

int fused_init(fftcg_plan_s* p, const double* g) {
    p->fused_ok = 0;
    p->fused_bytes = 0;
    p->fops = find_fused(p->M, p->pad);
    if (!p->fops) return FFTCG_OK;
    const int M = p->M, MH = M / 2 + 1;
    const double s = 1.0 / ((double)M * (double)M);
    std::vector<double> t64(2 * (size_t)M + (size_t)MH * MH);
    std::vector<float> t32(2 * (size_t)M + (size_t)MH * MH);
    for (int m = 0; m < M; ++m) {
        double c, sn;
        cos_sin_2pi(m, M, &c, &sn);
        t64[2 * m] = c;
        t64[2 * m + 1] = -sn;
        t32[2 * m] = (float)c;
        t32[2 * m + 1] = (float)-sn;
    }
    for (int m = 0; m < MH; ++m)
        for (int k = 0; k < MH; ++k) {
            const double v = g[(size_t)m * M + k] * s;
            t64[2 * M + (size_t)m * MH + k] = v;
            t32[2 * M + (size_t)m * MH + k] = (float)v;
        }
    if (hipMalloc(&p->f_tab64, t64.size() * 8) != hipSuccess) return FFTCG_ENOMEM;
    if (hipMalloc(&p->f_tab32, t32.size() * 4) != hipSuccess) return FFTCG_ENOMEM;
    if (hipMemcpy(p->f_tab64, t64.data(), t64.size() * 8, hipMemcpyHostToDevice) != hipSuccess) return FFTCG_EDEVICE;
    if (hipMemcpy(p->f_tab32, t32.data(), t32.size() * 4, hipMemcpyHostToDevice) != hipSuccess) return FFTCG_EDEVICE;
    p->fused_bytes = t64.size() * 8 + t32.size() * 4;
    p->fused_ok = 1;
    return FFTCG_OK;
}

void fused_free(fftcg_plan_s* p) {
    if (p->f_tab64) (void)hipFree(p->f_tab64);
    if (p->f_tab32) (void)hipFree(p->f_tab32);
    p->f_tab64 = p->f_tab32 = nullptr;
}

// Caller holds the plan lock; W is the plan's apply buffer, ordered by its event.
int fused_apply(fftcg_plan_s* p, int precision, const double* d, const double* x, double* y, hipStream_t s) {
    if (!p->fused_ok || !p->apply_W) return FFTCG_EINVAL;
    if (hipStreamWaitEvent(s, p->apply_ev, 0) != hipSuccess) return FFTCG_EDEVICE;
    p->fops->apply(precision == FFTCG_FP64 ? 0 : 1, tabs_of(p), d, x, y, p->apply_W, s);
    if (hipGetLastError() != hipSuccess || hipEventRecord(p->apply_ev, s) != hipSuccess) return FFTCG_EDEVICE;
    return FFTCG_OK;
}

void fused_launch(const fftcg_plan_s* p, int precision, const SlotDesc* slots, int nslots, int max_iters,
                  hipStream_t s) {
    p->fops->solve(precision == FFTCG_FP64 ? 0 : 1, tabs_of(p), slots, nslots, max_iters, s);
}

int fused_solve(fftcg_plan_s* p, int precision, const double* d, const double* b, const double* x0, double tol,
                int maxit, double* x, fftcg_info* info, hipStream_t s) {
    if (!p->fused_ok) return FFTCG_EINVAL;
    Workspace* w = plan_acquire(p);
    if (!w) return FFTCG_ENOMEM;
    const size_t n = (size_t)p->L * p->L;
    int rc = FFTCG_OK;
    do {
        fill_slot(w->h_slot, w, x, b, d);
        w->h_slot->host_status = nullptr;
        init_state(w->h_state, p, precision, tol, maxit, 50);
        if (hipMemcpyAsync(w->slot, w->h_slot, sizeof(SlotDesc), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(w->st, w->h_state, sizeof(SolveState), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipEventRecord(w->ev0, s) != hipSuccess) {
            rc = FFTCG_EDEVICE;
            break;
        }
        hipError_t he = hipSuccess;
        if (!x0)
            he = hipMemsetAsync(x, 0, n * 8, s);
        else if (x0 != x)
            he = hipMemcpyAsync(x, x0, n * 8, hipMemcpyDeviceToDevice, s);
        if (he == hipSuccess && precision == FFTCG_MIXED) he = hipMemsetAsync(w->e, 0, n * 4, s);
        if (he != hipSuccess) {
            rc = FFTCG_EDEVICE;
            break;
        }
        fused_launch(p, precision, w->slot, 1, 1 << 30, s);
        if (hipGetLastError() != hipSuccess || hipEventRecord(w->ev1, s) != hipSuccess ||
            hipMemcpyAsync(w->h_state, w->st, sizeof(SolveState), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = FFTCG_EDEVICE;
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, w->ev0, w->ev1);
        const SolveState st = *w->h_state;
        if (st.bzero && (hipMemsetAsync(x, 0, n * 8, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)) {
            rc = FFTCG_EDEVICE;
            break;
        }
        rc = st.done ? st.status : FFTCG_EDEVICE;
        if (info) {
            info->status = rc;
            info->iterations = st.iters;
            info->iterations_literal = st.iters_literal;
            info->checks = st.checks;
            info->true_relres = st.true_relres;
            info->error_bound = st.bound;
            info->lambda_lb = st.lam_lb;
            info->device_ms = ms;
        }
    } while (0);
    plan_release(p, w);
    return rc;
}

}  // namespace fftcg
