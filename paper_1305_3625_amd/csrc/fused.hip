// Fused single-workgroup engine (placeholder until the LDS engine lands):
// reports itself unavailable so every plan uses the multi-pass engine.
#include "fftcg_internal.hpp"
#include "fused.hpp"

namespace fftcg {

int fused_init(fftcg_plan_s* p, const double*) {
    p->fused_ok = 0;
    p->fused_bytes = 0;
    return FFTCG_OK;
}
void fused_free(fftcg_plan_s*) {}
int fused_apply(fftcg_plan_s*, int, const double*, const double*, double*, hipStream_t) { return FFTCG_EINVAL; }
int fused_solve(fftcg_plan_s*, int, const double*, const double*, const double*, double, int, double*, fftcg_info*,
                hipStream_t) {
    return FFTCG_EINVAL;
}

}  // namespace fftcg
