// Structures shared by the host driver and the device kernels.
//
// One solve (or one serving slot) owns a SlotDesc: pointers to its vectors,
// its FFT workspace, its reduction partials and its SolveState.  Kernels are
// launched with gridDim.y = number of slots and read their slot's descriptor
// from device memory, so a captured launch sequence stays valid when the
// vectors behind a slot change.
#pragma once
#include <stdint.h>

namespace fftcg {

// CG state of one solve, in device memory.  Each field has exactly one
// writer per kernel launch (block 0 of the named kernel, or the single-block
// check finaliser), and no other block of that launch reads it, so no
// intra-launch synchronisation is needed.  One exception: when the folded
// update's grid-wide barrier gives up, every block that gave up stores the
// same status and done values (atomically) and the solve is abandoned.
struct SolveState {
    double rho_cur;      // r_k . r_k (r_k . z_k preconditioned)  (row-forward kernel, block 0)
    double rho_prev;     // the same for k - 1                    (update kernel, block 0)
    double alpha;        // alpha of the last iteration whose x update is pending
    double tol;          // residual rule ||r||/||b|| <= tol
    double tau;          // certified error target
    double gmin;         // min ghat
    double bnorm;        // ||b||
    double lam_lb;       // min d + min ghat
    double trigger_rr;   // recursive r.r at or below which a check is made
    double last_rt;      // ||b - A x|| at the last check
    double xnorm;        // ||x|| at the last check
    double true_relres;  // last ||r||/||b||
    double bound;        // certified relative error bound at the last check
    double best_rt;      // smallest true residual seen
    double rho_ref;      // r.r right after the last check (residual replacement)
    double delta2;       // reliable-update threshold: check when r.r <= delta2 * rho_ref
    double dbar;         // mean of d (first check), for the preconditioner
    int iters;           // CG iterations done
    int maxit;
    int refresh;         // FP64 check period (0 = only at candidate convergence)
    int last_check_iter; // iteration count at the last check
    int pause;           // 1: iterations stop until the next check
    int done;            // 1: finished (status valid)
    int status;          // FFTCG_* code
    int restart;         // 1: next direction is p = r (no beta)
    int checks;          // number of FP64 checks done
    int worse;           // consecutive checks without residual decrease
    int iters_literal;   // iteration count when the residual rule first held
    int bzero;           // b == 0 detected
    int mixed;           // 1: working vectors are FP32
    int gen;             // generation of this solve (published with the status)
    int pcg;             // 1: Fourier-space (circulant) preconditioned CG
    int need_pre;        // 1: z = P^{-1} r is due after a check (check finaliser)
    long long bar_limit;  // wait limit of the update's grid-wide barrier, ticks of the 100 MHz clock
};

// Internal solve status (never returned to callers): a grid-wide barrier
// gave up waiting, so the host repeats the solve without it.
constexpr int ST_EGRID = -100;

// Per-slot descriptor (device memory).
struct SlotDesc {
    double* x;           // solution (FP64), updated in place
    double* y;           // output of a single operator product (apply)
    const double* b;     // right-hand side (FP64)
    const double* d;     // diagonal (FP64)
    void* r;             // residual           (working precision)
    void* p;             // search direction   (working precision)
    void* q;             // A p                (working precision)
    void* z;             // preconditioned residual (working precision)
    float* e;            // FP32 correction accumulated since the last check
    float* d32;          // FP32 copy of d (mixed mode)
    void* W;             // FFT workspace (pruned half spectrum, in place)
    double* part;        // reduction partials, NPART_SETS x npart_stride
    SolveState* st;      // CG state
    int* host_status;    // device-visible pinned host word pair, or nullptr
    const uint8_t* mask; // nullptr, or 1 = intact / 0 = broken per element:
                         // broken entries are projected out (f_i = 0)
    int active;          // 0: every kernel returns at once for this slot
    int pad_;
};

// Partial-sum sets inside SlotDesc::part.
enum PartSet {
    PS_PQ = 0,        // p . q per block of the row-inverse pass
    PS_RR = 1,        // r . r per block of the update kernel (or the check)
    PS_CHK_R = 2,     // (b - A x)^2 per block of the FP64 check
    PS_CHK_X = 3,     // x^2
    PS_CHK_B = 4,     // b^2
    PS_CHK_RW = 5,    // (working-precision r)^2
    PS_CHK_DMIN = 6,  // min d
    PS_CHK_BAD = 7,   // count of non-finite / negative inputs
    PS_CHK_DIFF = 8,  // |r64 - r_recursive|^2: drift of the recursive residual
    PS_RZ = 9,        // r . z per block of the preconditioner's row-inverse pass
    PS_CHK_DSUM = 10, // sum of d (for its mean)
    PS_BAR = 11,      // grid-wide barrier: arrival token per block (64-bit words)
    PS_BARREL = 12,   // [0] the barrier's release word (64 bits)
    NPART_SETS = 13
};

}  // namespace fftcg
