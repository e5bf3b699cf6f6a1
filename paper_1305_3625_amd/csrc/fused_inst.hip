// Instantiates the fused single-workgroup engine for one grid; compiled once
// per (FFTCG_M, FFTCG_PAD) by the build script.
#include "fused_kernels.hpp"

#ifndef FFTCG_M
#error "FFTCG_M must be defined"
#endif
#ifndef FFTCG_PAD
#error "FFTCG_PAD must be defined"
#endif

#define FFTCG_CAT2(a, b, c) a##b##_##c
#define FFTCG_CAT(a, b, c) FFTCG_CAT2(a, b, c)
#define FFTCG_FUSED_FN FFTCG_CAT(fftcg_fused_ops_, FFTCG_M, FFTCG_PAD)

namespace fftcg {
namespace {

constexpr int M = FFTCG_M;
constexpr int PAD = FFTCG_PAD;

void solve_fn(int prec, const FusedTabs& ft, const SlotDesc* slots, int nslots, int max_iters, hipStream_t s) {
    if (prec == 0)
        hipLaunchKernelGGL((k_fused_solve<double, M, PAD>), dim3(nslots), dim3(FNT), 0, s, ft, slots, max_iters);
    else
        hipLaunchKernelGGL((k_fused_solve<float, M, PAD>), dim3(nslots), dim3(FNT), 0, s, ft, slots, max_iters);
}

void apply_fn(int prec, const FusedTabs& ft, const double* d, const double* x, double* y, void* W,
              hipStream_t s) {
    if (prec == 0)
        hipLaunchKernelGGL((k_fused_apply<double, M, PAD>), dim3(1), dim3(FNT), 0, s, ft, d, x, y, W);
    else
        hipLaunchKernelGGL((k_fused_apply<float, M, PAD>), dim3(1), dim3(FNT), 0, s, ft, d, x, y, W);
}

const FusedOps kOps = {M, PAD, FLds<M, PAD>::BYTES, &solve_fn, &apply_fn};

}  // namespace

const FusedOps* FFTCG_FUSED_FN() { return &kOps; }

}  // namespace fftcg
