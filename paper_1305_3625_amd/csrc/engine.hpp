// Host-side view of one compiled engine (one FFT grid size M and boundary
// condition).  Each engine_inst_<M>_<pad>.o fills one EngineOps with
// launchers for the multi-pass kernels of that size.
#pragma once
#include <hip/hip_runtime.h>
#include "fftcg_types.hpp"

namespace fftcg {

struct PlanTabs {
    const void* tw32;   // cx<float>[M]
    const void* ghq32;  // float, tile layout of the FP32 column pass
    const void* ghN32;  // float[M/2 + 1]
    const void* tw64;   // cx<double>[M]
    const void* ghq64;  // double, tile layout of the FP64 column pass
    const void* ghN64;  // double[M/2 + 1]
};

struct EngineOps {
    int M, pad, L;
    int tt32, tt64;          // columns per tile of the column pass
    int rowblk32, rowblk64;  // blocks of the row passes (= partial counts)
    int g4;                  // blocks of the update kernel (= r.r partial count)
    // y = d x + C x, precision 0 = FP64, 1 = FP32 operator
    void (*apply)(int prec, const PlanTabs& t, const double* d, const double* x, double* y,
                  void* W, hipStream_t s);
    // one pass of an operator product: 0 row_fwd, 1 col, 2 row_inv
    void (*apply_pass)(int prec, int pass, const PlanTabs& t, const double* d, const double* x, double* y,
                       void* W, hipStream_t s);
    // one CG iteration for nslots slots (row_fwd, col, row_inv, update)
    void (*iter)(int prec, const PlanTabs& t, const SlotDesc* slots, int nslots, int stride,
                 hipStream_t s);
    // one FP64 check (row_fwd, col, row_inv on x, then the finaliser)
    void (*check)(int prec, const PlanTabs& t, const SlotDesc* slots, int nslots, int stride,
                  hipStream_t s);
    // the same two for CG with the Fourier-space (circulant) preconditioner
    void (*iter_pcg)(int prec, const PlanTabs& t, const SlotDesc* slots, int nslots, int stride,
                     hipStream_t s);
    void (*check_pcg)(int prec, const PlanTabs& t, const SlotDesc* slots, int nslots, int stride,
                      hipStream_t s);
    // the initial check of a solve started from x = 0 (no product: r = b)
    void (*check0)(int prec, const PlanTabs& t, const SlotDesc* slots, int nslots, int stride, hipStream_t s);
    void (*check0_pcg)(int prec, const PlanTabs& t, const SlotDesc* slots, int nslots, int stride,
                       hipStream_t s);
    // one CG iteration of a single slot with the update folded into the
    // row-inverse pass behind a grid-wide barrier (row_fwd, col, row_inv);
    // token: unique per launch on the slot's partial-sum buffer.  Returns
    // false (and runs the separate kernels) where grid_capable is false.
    bool (*iter_grid)(int prec, const PlanTabs& t, const SlotDesc* slot, int stride, unsigned long long token,
                      hipStream_t s);
    // one pass of a plain-CG iteration of one slot (measurement aid): 0 the
    // forward row pass, 1 the column pass, 2 the row-inverse pass (with the
    // folded update when grid), 3 the separate update (nothing when grid),
    // 4 the turn pass (grid only; tokens token and token + 1); the launch
    // records ev0 as the kernel starts and ev1 as it ends
    void (*iter_pass)(int prec, int pass, bool grid, const PlanTabs& t, const SlotDesc* slot, int stride,
                      unsigned long long token, hipEvent_t ev0, hipEvent_t ev1, hipStream_t s);
    // whether iter_grid applies on the current device: the whole
    // row-inverse grid resident at once, and no more r.r partials per pass
    // than the update kernel writes
    bool (*grid_capable)(int prec);
    // K (>= 1) such iterations of a single slot, as a chunk: with turn, the
    // row-inverse pass of every iteration but the last goes on into the next
    // iteration's forward row pass (k_row_turn), so the chunk launches
    // row_fwd, col, (turn, col) x (K - 1), row_inv; without it, K times
    // iter_grid.  *token is advanced past every token the launches use.
    void (*iter_grid_chunk)(int prec, const PlanTabs& t, const SlotDesc* slot, int stride,
                            unsigned long long* token, int K, bool turn, hipStream_t s);
    // whether the turn pass is resident as a whole as well (implies
    // grid_capable)
    bool (*turn_capable)(int prec);
};

const EngineOps* find_engine(int M, int pad);

}  // namespace fftcg
