/*
 * fftcg.h -- C ABI of the MI355X FFT-convolution conjugate-gradient solver.
 *
 * Problem (Gjerden, "Making the case of GPUs in courses on computational
 * physics", Sec. 2 eqs. (1a)-(1c), (2); Sec. 3 eq. (3) and Listing 2):
 *
 *     A x = b,   A = diag(d) + C,
 *     (C v)(i) = sum_{j in [0,L)^2} g_M((i - j) mod M) v(j),
 *     g_M = inverse 2-D DFT of the multiplier ghat (M x M, real, even).
 *
 * Sec. 3 notes the Green's function depends only on the separation of two
 * sites, so C is a convolution and is diagonal in Fourier space (eq. (3)):
 * C v = F^{-1}(ghat . F v).  The periodic grid uses M = L; the zero-padded
 * grid uses M = 2L and crops, which gives the linear convolution.  The paper
 * treats the system as symmetric positive definite and solves it with
 * unpreconditioned CG (Sec. 3 Listing 2, Sec. 4).  With a uniform fibre
 * stiffness k, eq. (2) divided by k is this system with d = 1/k, b = D and
 * x = f.
 *
 * Conventions for every call:
 *   - Return value is a status code below; nothing throws, aborts or prints.
 *   - Arguments are validated before any device work; invalid arguments
 *     return FFTCG_EINVAL and leave every output untouched.
 *   - Out-parameters are written only on FFTCG_OK (and on FFTCG_ENOCONV for
 *     fftcg_solve / fftcg_poll, which return the last iterate).
 *   - The library never frees caller memory.
 *   - Grids are L x L, row-major, element (i1, i2) at index i1 * L + i2.
 *   - "device pointer" means memory of the current HIP device (hipMalloc or a
 *     torch CUDA/HIP tensor); "host pointer" means ordinary host memory.
 *   - Streams are hipStream_t passed as void* (NULL = the default stream).
 */
#ifndef FFTCG_H
#define FFTCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define FFTCG_OK          0
#define FFTCG_PENDING     1   /* fftcg_poll only: request still in flight   */
#define FFTCG_EINVAL     -1   /* invalid argument or invalid input data     */
#define FFTCG_ENOMEM     -2   /* device allocation failed / over budget     */
#define FFTCG_ENOTSPD    -3   /* min ghat <= 0: A not positive definite     */
#define FFTCG_ENOCONV    -4   /* maxit reached; x holds the last iterate    */
#define FFTCG_EBREAKDOWN -5   /* p.q <= 0 or non-finite inside CG           */
#define FFTCG_EAGAIN     -6   /* server queue full; retry later             */
#define FFTCG_EDEVICE    -7   /* HIP runtime error / no usable gfx950 GPU   */
#define FFTCG_ENOTFOUND  -8   /* unknown or already retired ticket          */
#define FFTCG_ECANCELED  -9   /* request cancelled by server shutdown       */

/* ---- precision modes ----------------------------------------------------
 * FFTCG_FP64 : every step in FP64.
 * FFTCG_MIXED: the FFT passes, spectral multiply and the vectors r, p, q in
 *              FP32; dot products accumulate in FP64; alpha/beta in FP64; an
 *              FP64 true residual r = b - A x (FP64 operator) every
 *              refresh period (50 iterations) and at candidate convergence,
 *              with residual replacement.  Convergence is declared only at an
 *              FP64 check.                                                  */
#define FFTCG_FP64  0
#define FFTCG_MIXED 1

/* ---- engines (fftcg_plan_set_engine) -----------------------------------
 * AUTO     : the fused engine for M <= 64 in single solves and for
 *            M <= 128 in server classes, the multi-pass engine above.
 * MULTIPASS: three HBM passes per product (row R2C, column FFT*ghat*IFFT,
 *            row C2R + epilogue); every grid.
 * FUSED    : one workgroup per solve, whole CG loop in one kernel, the
 *            product's half spectrum in the slot's buffer (L1/L2-resident)
 *            and its transforms in registers and LDS; M <= 256.            */
#define FFTCG_ENGINE_AUTO      0
#define FFTCG_ENGINE_MULTIPASS 1
#define FFTCG_ENGINE_FUSED     2

/* ---- preconditioner (fftcg_plan_set_precond) ---------------------------
 * NONE     : plain CG as in Sec. 3, Listing 2 (the paper ran without one,
 *            Sec. 4).  Default.
 * CIRCULANT: CG preconditioned by the inverse of the M-periodic circulant
 *            mean(d) I + C (Fourier-space diagonal, eq. (3)), applied to the
 *            zero-padded residual and cropped: z = crop(F^-1 (F pad(r) /
 *            (mean(d) + ghat))).  Symmetric positive definite; exact for a
 *            periodic grid with uniform d.  Costs one more product-like pass
 *            triple per iteration and cuts iterations 3-5x on the padded
 *            workloads.  Multi-pass engine only (a plan with it never uses
 *            the fused engine).                                            */
#define FFTCG_PRECOND_NONE      0
#define FFTCG_PRECOND_CIRCULANT 1

typedef struct fftcg_plan_s*   fftcg_plan_t;
typedef struct fftcg_server_s* fftcg_server_t;

/* Per-solve report.  Relative quantities are relative to ||b||_2. */
typedef struct {
    int    status;              /* same as the call's return value           */
    int    iterations;          /* CG iterations performed                   */
    int    iterations_literal;  /* iteration count at the first FP64 check
                                   where ||r||/||b|| <= tol held (-1: never)   */
    int    checks;              /* FP64 true-residual checks performed       */
    double true_relres;         /* ||b - A x||/||b|| at the last FP64 check  */
    double error_bound;         /* certified bound on ||x - x*||/||x*||      */
    double lambda_lb;           /* min(d) + min(ghat): lower eigenvalue bound */
    double device_ms;           /* device time of the solve (HIP events)     */
} fftcg_info;

/* fftcg_plan -- build the spectral operator for one grid.
 *   L               grid side, power of two, L >= 2, M <= 8192 (L <= 4096
 *                   padded, L <= 8192 periodic).
 *   padded          0: periodic grid, M = L.  1: zero-padded, M = 2L.
 *   kernel_spectrum HOST pointer to M*M doubles, ghat[m*M + n] (m along the
 *                   row index).  Copied; the caller keeps ownership.
 *                   Must be finite and even in each index
 *                   (ghat[m,n] == ghat[(M-m)%M, n] == ghat[m, (M-n)%M] to a
 *                   relative 1e-12 of max|ghat|), else FFTCG_EINVAL; must have
 *                   min > 0, else FFTCG_ENOTSPD (Sec. 3: CG needs SPD).
 *   out             receives the plan handle.
 * Sec. 3 / eq. (3): the static spectrum is transformed once at set-up; the
 * normalisation 1/M^2 of the inverse transform (Listing 3) is folded into the
 * stored spectrum.  The plan owns its device memory (current device).       */
int fftcg_plan(int L, int padded, const double* kernel_spectrum, fftcg_plan_t* out);

/* fftcg_greens_spectrum -- the spectrum of the physical Green's function of
 * Sec. 2, eq. (1c): G(Delta) = (1 - nu^2)/(pi E a) * P(Delta), P the
 * integral of 1/r over the unit square centred at the lattice separation
 * Delta (the 1/r kernel averaged over the source fibre's plaquette, lengths
 * in units of a), tabulated on the M x M grid (M = padded ? 2L : L) at
 * separations min(i, M - i) per index, and transformed by a DFT.  Writes the
 * real, even, positive spectrum to `spectrum` (HOST pointer, M*M doubles,
 * [m*M + n]), ready for fftcg_plan.  Host computation (plan time); no GPU.
 * FFTCG_EINVAL unless L is a power of two with 2 <= L and M <= 8192, E > 0, a > 0 and
 * |nu| < 1 (all finite).  With uniform fibre stiffness k the system of
 * eq. (2) divided by k is diag(1/k) + C with this spectrum.               */
int fftcg_greens_spectrum(int L, int padded, double nu, double E, double a, double* spectrum);

/* Releases the plan.  FFTCG_EINVAL if a server still holds requests on it.  */
int fftcg_plan_destroy(fftcg_plan_t plan);

/* Selects the engine used by later calls on this plan (testing and tuning).
 * FFTCG_EINVAL if the engine does not support this grid.                   */
int fftcg_plan_set_engine(fftcg_plan_t plan, int engine);

/* fftcg_plan_set_precond -- preconditioner of the solves started with this
 * plan afterwards (fftcg_solve, and server requests admitted afterwards).
 * FFTCG_EINVAL for an unknown kind, or while server requests use the plan.
 * Not to be called concurrently with solves on the same plan.             */
int fftcg_plan_set_precond(fftcg_plan_t plan, int kind);

/* fftcg_plan_set_error_target -- the certified relative-error target tau of
 * later solves in `precision` on this plan (fftcg_solve, fftcg_fracture, and
 * server requests admitted afterwards).  tau = 0 (the default) makes tau
 * equal to each solve's residual tolerance tol; 0 < tau < 1 fixes it, e.g.
 * 1e-10 for FFTCG_FP64 and 1e-8 for FFTCG_MIXED, whatever tol is.  A solve
 * then stops when ||r||/||b|| <= tol AND the residual certifies
 * ||x - x*||/||x*|| <= tau (see fftcg_solve).  FFTCG_EINVAL for another
 * precision or tau, or while server requests use the plan.  Not to be called
 * concurrently with solves on the same plan.                               */
int fftcg_plan_set_error_target(fftcg_plan_t plan, int precision, double tau);

/* fftcg_plan_set_grid_sync -- how the multi-pass engine ends a CG iteration
 * in fftcg_solve and fftcg_fracture (Sec. 3, the r update of Listing 2).
 *   mode 1 (default): where the device allows it, the update r <- r - alpha q
 *          runs inside the row-inverse pass: each workgroup keeps its q in
 *          registers, all workgroups meet at a grid-wide barrier (the
 *          plan checks that the pass's whole grid fits the device at once)
 *          once their p.q partials are stored, and then update their own
 *          rows.  q never reaches memory and one kernel per
 *          iteration is saved.  Both precisions, without a preconditioner,
 *          on grids whose row-inverse pass is resident as a whole
 *          (fftcg_plan_get_grid_sync reports where).
 *          Where the device also holds the whole grid of the turn pass,
 *          the row-inverse pass of every iteration but the last of a chunk
 *          goes on, after a second grid-wide barrier (for r.r and beta),
 *          into the next iteration's forward row pass on the same rows
 *          (p <- r + beta p, the pending x update, the row transform), so
 *          that r and p are not read back from memory.
 *   mode 0: the separate update kernel (as server classes always use).
 *   mode 2: as mode 1 with the barrier's wait limit at zero, so that
 *          workgroups give up at once; for tests of the fallback below.
 *   mode 3: as mode 1 without the turn pass.
 * A barrier that is not met within its wait limit (20 ms; another stream's
 * work can hold part of the device) abandons the solve, which is then
 * repeated from its start with mode 0 semantics; the plan keeps the separate
 * kernel from then on, until this call sets a mode again.  The result is
 * the same either way (up to the rounding of the r.r partial sums).
 * FFTCG_EINVAL for a NULL plan or another mode.  Not to be called
 * concurrently with solves on the same plan.                               */
int fftcg_plan_set_grid_sync(fftcg_plan_t plan, int mode);

#define FFTCG_GRID_UNSUPPORTED 0 /* not on this grid, device or precision   */
#define FFTCG_GRID_OFF         1 /* supported, mode 0                       */
#define FFTCG_GRID_ON          2 /* supported and used by later solves      */
#define FFTCG_GRID_FELL_BACK   3 /* a barrier gave up; separate kernel used */
#define FFTCG_GRID_ON_TURN     4 /* as FFTCG_GRID_ON, with the turn pass    */

/* fftcg_plan_get_grid_sync -- *state = one of FFTCG_GRID_* for solves in
 * `precision` on this plan.  FFTCG_EINVAL for a NULL argument or another
 * precision.                                                               */
int fftcg_plan_get_grid_sync(fftcg_plan_t plan, int precision, int* state);

/* Reports L, M, padded, and the plan's device bytes (any pointer may be NULL). */
int fftcg_plan_info(fftcg_plan_t plan, int* L, int* M, int* padded, size_t* device_bytes);

/* fftcg_apply -- y = (diag(d) + C) x, one operator product (Sec. 3 Listing 4
 * plus the element-wise term that completes the left-hand side).
 *   precision  FFTCG_FP64, or FFTCG_MIXED: x is rounded to FP32 and C is
 *              applied in FP32; d*x is formed in FP64; y is FP64.
 *   d, x, y    DEVICE pointers to L*L doubles.  y must not overlap x or d.
 *   stream     hipStream_t; the call is stream-ordered and asynchronous.   */
int fftcg_apply(fftcg_plan_t plan, int precision, const double* d,
                const double* x, double* y, void* stream);

/* fftcg_profile_apply -- measurement aid: times each of the three passes
 * of fftcg_apply (row forward, column, row inverse) with HIP events on
 * `stream` around runs of 8 back-to-back launches of that pass, repeated
 * ceil(reps / 8) times (every column run starts from a fresh row-forward
 * output), and stores the mean device milliseconds per launch of each pass
 * in ms_per_pass[0..2] (HOST pointer).  y is scratch (overwritten; not
 * the product).  Blocks until done.  FFTCG_EINVAL for the fused engine.   */
int fftcg_profile_apply(fftcg_plan_t plan, int precision, const double* d,
                        const double* x, double* y, int reps,
                        double* ms_per_pass, void* stream);

/* fftcg_profile_iteration -- measurement aid: runs `reps` (1..100)
 * iterations of the CG iteration that fftcg_solve runs on this plan (plain
 * CG, Sec. 3 Listing 2) on (d, b) from x = 0, without FP64 checks, and times
 * every kernel with a start and an end event recorded by its own launch
 * (hipExtLaunchKernel: the kernel's execution, as a kernel trace reports
 * it).  ms_per_pass (HOST array of 5) receives the mean device milliseconds
 * per launch of [0] the forward row pass (with the CG prologue), [1] the
 * column pass, [2] the row-inverse pass (with the folded update when it
 * applies, fftcg_plan_set_grid_sync), [3] the separate update kernel (0 when
 * folded), [4] the turn pass (0 when not used).  The launches follow a
 * solve's chunk: with the turn pass, row_fwd, col, (turn, col) x (reps - 1),
 * row_inv (so [0] and [2] are single launches; reps >= 2), else reps times
 * each pass.  *folded (HOST, may be NULL) = 0 separate update, 1 folded,
 * 2 folded with the turn pass.
 * d, b: DEVICE, L*L doubles; x: DEVICE scratch of L*L doubles (the iterate,
 * overwritten), not overlapping d or b.  Blocks until done.  FFTCG_EINVAL
 * for the fused engine or bad arguments (reps = 1 with the turn pass), and
 * when the iterations stopped
 * early (b = 0); FFTCG_EBREAKDOWN if they broke down; FFTCG_EDEVICE if the
 * folded update's barrier gave up (the plan then keeps the separate
 * kernel).                                                                 */
int fftcg_profile_iteration(fftcg_plan_t plan, int precision, const double* d,
                            const double* b, double* x, int reps,
                            double* ms_per_pass, int* folded, void* stream);

/* fftcg_stream_probe -- measurement aid: the HBM rate of plain streaming
 * kernels, the practical ceiling of the memory-bound passes.  kind 0 reads
 * `bytes` from src (16-byte loads, summed; dst is a sink that receives 4
 * bytes only if the data sums to non-zero), 1 writes zeros to dst, 2 copies
 * src to dst (`bytes` each, no overlap); with
 * nontemporal != 0 the loads and stores carry the non-temporal hint.
 * `blocks` workgroups of 256 threads stride over the buffer.  Times `reps`
 * back-to-back launches with HIP events on `stream` and stores the mean
 * device milliseconds per launch in *ms_per_launch (HOST).  src and dst are
 * DEVICE pointers, 16-byte aligned, `bytes` a positive multiple of 16; src
 * must hold zeros for kind 0.  Blocks until done.                         */
int fftcg_stream_probe(int kind, int nontemporal, void* dst, const void* src, size_t bytes,
                       int blocks, int reps, double* ms_per_launch, void* stream);

/* fftcg_solve -- CG solve of (diag(d) + C) x = b (Sec. 3 Listing 2).
 *   d, b       DEVICE pointers, L*L doubles; d >= 0 and finite, b finite
 *              (checked on the device: FFTCG_EINVAL).
 *   x0         DEVICE pointer to the start vector, or NULL for zero.  x may
 *              equal x0 (warm start in place).
 *   tol        residual rule ||b - A x||/||b|| <= tol, on an FP64 true
 *              residual.  0 < tol < 1.
 *   maxit      iteration cap, >= 1.  Reaching it returns FFTCG_ENOCONV with
 *              x = last iterate and info filled.
 *   x          DEVICE pointer, L*L doubles: the solution.
 *   info       host pointer or NULL.
 *   stream     hipStream_t used for all work; the call blocks until done.
 * Stopping: the residual rule AND the certified rule
 *   ||r|| <= tau * lambda_lb * ||x|| / (1 + tau),  lambda_lb = min d + min ghat,
 * which guarantees ||x - x*||/||x*|| <= tau (both checked on an FP64 true
 * residual).  tau = tol unless the plan fixes it per precision
 * (fftcg_plan_set_error_target).  b = 0 gives x = 0, FFTCG_OK and 0
 * iterations.  A non-finite value met inside CG (for instance from a
 * non-finite x0) ends the solve with FFTCG_EBREAKDOWN.  x is the solve's
 * working iterate: after an error other than FFTCG_EINVAL its contents are
 * unspecified.                                                            */
int fftcg_solve(fftcg_plan_t plan, int precision, const double* d,
                const double* b, const double* x0, double tol, int maxit,
                double* x, fftcg_info* info, void* stream);

/* fftcg_loadstep -- one load step of the load-stepped workload: among the
 * entries with d_i != 0, find i* = argmax x_i / t_i (FP64; ties to the
 * smallest row-major index) and set d_{i*} = 0 (Sec. 2: a bond whose strain
 * exceeds its threshold breaks).
 *   x, t       DEVICE pointers, L*L doubles (t > 0).
 *   d          DEVICE pointer, L*L doubles, updated in place.
 *   index      HOST pointer: receives i*, or -1 if every d_i is 0.
 * Blocks until the index is known.                                         */
int fftcg_loadstep(fftcg_plan_t plan, const double* x, const double* t,
                   double* d, int* index, void* stream);

/* fftcg_loadstep_noalloc -- fftcg_loadstep for callers that cannot allocate
 * device or pinned memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): same arguments, rule and result, bitwise.
 * Its argmax partials live in a 16 KiB array in the library's device memory
 * (one per GPU, held until the process ends) instead of a workspace the plan
 * allocates on first use; it calls no allocating routine.  That array holds
 * the partials of at most 1024 blocks, which covers every plan's grid (the
 * partial count is capped at 1024); FFTCG_EINVAL if a grid ever needed more.
 * Every call on one GPU shares the array: calls that overlap on the same GPU
 * (two host threads, or two streams) race and must be serialised by the
 * caller.  index is a HOST pointer; blocks until the index is known.         */
int fftcg_loadstep_noalloc(fftcg_plan_t plan, const double* x, const double* t,
                           double* d, int* index, void* stream);

/* fftcg_fracture -- the quasi-static fracture driver of Sec. 2: uniform
 * fibre stiffness k (> 0), displacement control, fibres breaking one at a
 * time.  Each step solves, at unit displacement, (I/k + G)_II f_I = 1_I on
 * the intact fibres I (eq. (2) divided by k; broken fibres carry no force and
 * are projected out of the solve), to the relative error tol (certified as
 * for fftcg_solve, `precision` as there), warm-started from the previous
 * step; then the intact fibre with the largest f_i / t_i breaks (ties to the
 * smallest row-major index), at the displacement D = t_i / f_i.
 *   t        DEVICE pointer, L*L thresholds (> 0; a gradient across the grid
 *            directs the front, Sec. 2).
 *   steps    number of fibres to break, 1 <= steps <= L*L.
 *   f        DEVICE pointer, L*L doubles: forces at unit displacement of the
 *            last step's intact set (zero on broken fibres).
 *   broken   HOST, steps ints: the fibre broken at each step.
 *   dbreak   HOST, steps doubles: the displacement at which it breaks
 *            (+inf if no intact fibre carries a positive force).
 *   iters    HOST, steps ints, or NULL: CG iterations of each step's solve.
 * Multi-pass engine (the plan's preconditioner setting applies).  Blocks
 * until done; the first failing solve's status is returned (FFTCG_ENOCONV
 * included) with the steps done so far written.                           */
int fftcg_fracture(fftcg_plan_t plan, int precision, double k, const double* t, int steps, double tol,
                   int maxit, double* f, int* broken, double* dbreak, int* iters, void* stream);

/* ---- continuous-batching server ---------------------------------------- */
typedef struct {
    size_t memory_budget;     /* bytes of device memory for request slots   */
    int    max_slots;         /* slots per grid size (0: default 64)        */
    int    chunk_iters;       /* CG iterations per step launch (0: 10)      */
    int    refresh_period;    /* MIXED FP64 check period (0: 50)            */
    int    queue_cap;         /* pending requests (0: 1<<20)                */
    int    device;            /* HIP device ordinal                         */
    int    graphs;            /* 0: each multi-pass chunk shape (running
                                 slots) is captured once as a HIP graph and
                                 replayed; -1: kernels launched directly    */
} fftcg_server_opts;

typedef struct {
    uint64_t submitted, admitted, completed, failed, canceled;
    size_t   bytes_in_use;
    int      queued;
    int      in_flight;
} fftcg_server_stats;

/* Starts the server's scheduler thread on opts->device.                    */
int fftcg_server_create(const fftcg_server_opts* opts, fftcg_server_t* out);

/* fftcg_submit -- enqueue one solve (same semantics as fftcg_solve).
 *   d, b       HOST pointers, L*L doubles, copied before return.
 *   x0         HOST pointer or NULL (zero start), copied before return.
 *   ticket     receives the request id.
 * FFTCG_EAGAIN when the queue is full; FFTCG_ENOMEM when one request's device
 * footprint exceeds the whole budget; FFTCG_EINVAL for bad arguments or
 * non-finite / negative data.  Never blocks on the GPU.                    */
int fftcg_submit(fftcg_server_t srv, fftcg_plan_t plan, int precision,
                 const double* d, const double* b, const double* x0,
                 double tol, int maxit, uint64_t* ticket);

/* fftcg_submit_sequence -- enqueue a load-stepped sequence: `steps` solves
 * of the same grid; after each solve the load step (fftcg_loadstep rule)
 * breaks one entry and the next solve is warm-started from the previous x.
 *   t          HOST pointer, L*L thresholds, copied.
 * fftcg_poll then returns the final x, and fftcg_poll_sequence the broken
 * indices in order.                                                         */
int fftcg_submit_sequence(fftcg_server_t srv, fftcg_plan_t plan, int precision,
                          const double* d, const double* b, const double* t,
                          double tol, int maxit, int steps, uint64_t* ticket);

/* fftcg_poll -- FFTCG_PENDING, or the request's final status with x (HOST
 * pointer, L*L doubles) and info copied out; the ticket is then retired and
 * later polls return FFTCG_ENOTFOUND.  x or info may be NULL.  FFTCG_ENOMEM
 * if no pinned host buffer for the result could be allocated when the solve
 * finished (x is then not written).                                        */
int fftcg_poll(fftcg_server_t srv, uint64_t ticket, double* x, fftcg_info* info);

/* fftcg_poll_sequence -- like fftcg_poll for a sequence ticket; also copies
 * the broken indices (HOST pointer, `steps` ints), the per-step iteration
 * counts (HOST pointer, `steps` ints) and each step's certified relative
 * error bound (HOST pointer, `steps` doubles); each may be NULL.  A sequence
 * is deterministic: the first s steps of a longer sequence on the same
 * inputs break the same entries and end at bitwise the same x.            */
int fftcg_poll_sequence(fftcg_server_t srv, uint64_t ticket, double* x,
                        int* broken, int* step_iters, double* step_bounds,
                        fftcg_info* info);

/* fftcg_server_completed -- tickets whose requests finished since the last
 * call, in completion order, so a client polls only those.
 *   out   HOST array of cap entries; n receives the number written.
 * Each ticket is reported once; fftcg_poll then returns its result.  The
 * server keeps the 2^20 most recent unreported tickets (older ones are
 * dropped, their results stay pollable).  FFTCG_EINVAL on NULL srv/n, cap<0
 * or NULL out with cap>0.                                                  */
int fftcg_server_completed(fftcg_server_t srv, uint64_t* out, int cap, int* n);

/* Counters of the server (host pointer).                                   */
int fftcg_server_get_stats(fftcg_server_t srv, fftcg_server_stats* out);

/* fftcg_server_reserve -- capacity planning: makes the server hold `slots`
 * request slots (device memory, within the budget) for solves with this
 * plan and precision, each with its pinned staging buffer, captures the
 * class's chunk graphs for up to `slots` running solves, and caches pinned
 * input and result buffers for as many requests (solves without x0), so
 * that a burst of that class neither allocates device memory, pins host
 * memory nor builds graphs on its way in.  Blocks until the slots exist (the scheduler
 * thread makes them).  The plan stays referenced by the server
 * (fftcg_plan_destroy refuses it) until fftcg_server_shutdown or
 * fftcg_server_destroy.  Idle reserved slots can still be released when
 * another class needs the budget.  FFTCG_EINVAL for bad arguments or slots
 * above max_slots; FFTCG_ENOMEM when the budget or an allocation cannot hold
 * them (the slots made so far stay); FFTCG_ECANCELED after shutdown.       */
int fftcg_server_reserve(fftcg_server_t srv, fftcg_plan_t plan, int precision, int slots);

/* fftcg_server_class_slots -- *slots = the slots the server holds for
 * solves with this plan and precision (0 if none), busy or idle; for sizing
 * fftcg_server_reserve from a server that has seen the load.  FFTCG_EINVAL
 * for a NULL argument or another precision.                                */
int fftcg_server_class_slots(fftcg_server_t srv, fftcg_plan_t plan, int precision, int* slots);

/* fftcg_server_shutdown -- stops the scheduler; every request still queued
 * or in flight ends with FFTCG_ECANCELED (info.iterations: the iterations it
 * had run), except one whose results were already being copied back, which
 * keeps its own status.  Device memory of the slots is released.  Results
 * stay pollable until fftcg_server_destroy; later submissions return
 * FFTCG_ECANCELED.  A second call does nothing.  Blocks until the device
 * work of the server's streams has finished.                               */
int fftcg_server_shutdown(fftcg_server_t srv);

/* Shuts the server down (fftcg_server_shutdown) and frees it with every
 * unpolled result; the handle is invalid afterwards.                       */
int fftcg_server_destroy(fftcg_server_t srv);

/* Static description of a status code.                                     */
const char* fftcg_strerror(int status);

/* Library version string.                                                  */
const char* fftcg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FFTCG_H */
