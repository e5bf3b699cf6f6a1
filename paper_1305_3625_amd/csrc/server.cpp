// Continuous-batching server (scheduler under construction: creation fails).
#include "fftcg.h"

extern "C" int fftcg_server_create(const fftcg_server_opts*, fftcg_server_t*) { return FFTCG_EDEVICE; }
extern "C" int fftcg_submit(fftcg_server_t, fftcg_plan_t, int, const double*, const double*, const double*, double,
                            int, uint64_t*) { return FFTCG_EINVAL; }
extern "C" int fftcg_submit_sequence(fftcg_server_t, fftcg_plan_t, int, const double*, const double*,
                                     const double*, double, int, int, uint64_t*) { return FFTCG_EINVAL; }
extern "C" int fftcg_poll(fftcg_server_t, uint64_t, double*, fftcg_info*) { return FFTCG_EINVAL; }
extern "C" int fftcg_poll_sequence(fftcg_server_t, uint64_t, double*, int*, int*, fftcg_info*) {
    return FFTCG_EINVAL;
}
extern "C" int fftcg_server_get_stats(fftcg_server_t, fftcg_server_stats*) { return FFTCG_EINVAL; }
extern "C" int fftcg_server_destroy(fftcg_server_t) { return FFTCG_EINVAL; }
