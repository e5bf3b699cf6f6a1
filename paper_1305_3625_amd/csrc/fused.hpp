// Fused single-workgroup engine for small grids (M <= 256): one workgroup
// holds a whole solve; the operator product and the CG update run with no
// kernel boundary between iterations.
#pragma once
#include <hip/hip_runtime.h>

#include "fftcg.h"
#include "fftcg_types.hpp"

struct fftcg_plan_s;

namespace fftcg {

// Per-plan constant tables (device pointers).
struct FusedTabs {
    const void* tw64;  // cx<double>[M]: exp(-2 pi i m / M)
    const void* tw32;  // cx<float>[M]
    const void* gq64;  // double[(M/2+1)^2]: ghat(m, k) / M^2, m, k in [0, M/2], row-major
    const void* gq32;  // float[(M/2+1)^2]
};

// Launchers of one compiled size (precision 0 = FP64, 1 = FP32 inner
// iterations / operator).
struct FusedOps {
    int M, pad;
    int lds_bytes;  // exchange buffer of a solve workgroup
    void (*solve)(int prec, const FusedTabs& ft, const SlotDesc* slots, int nslots, int max_iters,
                  hipStream_t s);
    void (*apply)(int prec, const FusedTabs& ft, const double* d, const double* x, double* y, void* W,
                  hipStream_t s);
};

const FusedOps* find_fused(int M, int pad);

int fused_init(fftcg_plan_s* p, const double* spectrum);
void fused_free(fftcg_plan_s* p);
int fused_apply(fftcg_plan_s* p, int precision, const double* d, const double* x, double* y, hipStream_t s);
int fused_solve(fftcg_plan_s* p, int precision, const double* d, const double* b, const double* x0, double tol,
                int maxit, double* x, fftcg_info* info, hipStream_t s);
// Runs up to max_iters CG iterations (plus the checks they need) for every
// slot of the table, one workgroup per slot.
void fused_launch(const fftcg_plan_s* p, int precision, const SlotDesc* slots, int nslots, int max_iters,
                  hipStream_t s);

}  // namespace fftcg
