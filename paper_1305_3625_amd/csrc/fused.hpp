// Fused single-workgroup engine for small grids (M <= 128): one workgroup
// holds a whole solve; the operator product and the CG update run in LDS
// with no kernel boundary between iterations.
#pragma once
#include <hip/hip_runtime.h>

#include "fftcg.h"
#include "fftcg_types.hpp"

struct fftcg_plan_s;

namespace fftcg {

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
