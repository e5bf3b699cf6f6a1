// Multi-pass engine: one operator product A v = d * v + C v in three HBM
// passes over the pruned half spectrum W (L rows x M/2 packed columns).
//
//   row_fwd  (gather + forward R2C along rows)   v rows -> W
//   col      (forward FFT, * ghat/M^2, inverse FFT along columns, in place)
//   row_inv  (C2R along rows + crop + epilogue)   W -> q = d*v + Cv, partials
//
// Eq. (3) of the paper: C is diagonal in Fourier space, so one product is a
// forward 2-D transform, a pointwise multiply by the static spectrum and an
// inverse transform (Listing 4), the scaling of Listing 3 being folded into
// the stored spectrum.  Listing 4 copies the real input into a complex buffer
// and back; here the real input is packed two-per-complex (z[n] = v[2n] +
// i v[2n+1]) so the row transforms have length M/2 and the column pass
// touches only the M/2 non-redundant column frequencies.  The Nyquist column
// k = M/2 is real for every row, as is k = 0, so both ride in packed column 0
// (real part k = 0, imaginary part k = M/2).
//
// On the zero-padded grid (M = 2L) rows >= L and inputs >= L are zero, so the
// row pass transforms only L rows and the first radix-16 stage of every
// forward transform sees only its lower 8 inputs; outputs >= L are cropped,
// so the last inverse stage stores only its lower 8 outputs.
//
// W layout: tiles of TT columns, W[((kt * L) + i) * TT + kk] for column
// k = kt * TT + kk, so a column tile is one contiguous block and each row
// writes runs of RPW * TT complex values.
#pragma once
#include <stddef.h>
#include <type_traits>
#include "fftcg_dev.hpp"
#include "fftcg_types.hpp"

namespace fftcg {
inline namespace FFTCG_RADIX_NS {

#ifndef FFTCG_STATUS_CODES
#define FFTCG_STATUS_CODES
enum { ST_OK = 0, ST_EINVAL = -1, ST_ENOCONV = -4, ST_EBREAKDOWN = -5 };
#endif

__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }
__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <typename T, int M, int PAD>
struct Geo {
    static constexpr int L = PAD ? M / 2 : M;
    static constexpr int N = M / 2;  // complex row length = number of packed columns
    // row passes
    static constexpr int ER = fft_elems(N);
    static constexpr int PR = N / ER;
    static constexpr int ROW_WORDS = LdsLay<T, 1, 4, 1>::words(N);
    // LDS budget per workgroup: 72 KB (two workgroups per CU); on the largest
    // grid (M = 8192) one workgroup of twice the size takes 144 KB, so that
    // rows and column tiles still come in pairs and W moves in 32-byte runs
    static constexpr int LDS_CAP_BYTES = M >= 8192 ? 147456 : 73728;
    static constexpr int ROW_LDS_CAP = LDS_CAP_BYTES / (int)sizeof(cx<T>);
#ifndef FFTCG_ROW_NT
#define FFTCG_ROW_NT 256
#endif
    static constexpr int ROW_NT = M >= 8192 ? 2 * FFTCG_ROW_NT : FFTCG_ROW_NT;
    static constexpr int RPW0 = cmin(L, cmax(1, ROW_NT / PR));
    static constexpr int RPW_fit(int r) { return (r > 1 && r * ROW_WORDS > ROW_LDS_CAP) ? RPW_fit(r / 2) : r; }
    static constexpr int RPW = RPW_fit(RPW0);
    static constexpr int ROW_THREADS = RPW * PR;
    static constexpr int ROW_BLOCKS = L / RPW;
    // column pass
    static constexpr int EC = fft_elems(M);
    static constexpr int PC = M / EC;
    static constexpr int COL_LDS_CAP = LDS_CAP_BYTES / (int)sizeof(cx<T>);
    static constexpr int TT_fit(int t) {
        return (t > 1 && (t * M + (t * M) / 16 + t > COL_LDS_CAP || t * PC > 1024)) ? TT_fit(t / 2) : t;
    }
#ifndef FFTCG_COL_TTMAX
#define FFTCG_COL_TTMAX 4
#endif
    static constexpr int TT = TT_fit(cmin(N, FFTCG_COL_TTMAX));
    static constexpr int COL_SH = ilog2c(16 * TT);
    static constexpr int COL_THREADS = TT * PC;
    static constexpr int NTILE = N / TT;
    static constexpr int MH = M / 2 + 1;
};

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Row blocks that share 128-byte lines of W must run on the same XCD,
// so block b works on logical block (b % 8) * (G / 8) + b / 8: each XCD gets
// a contiguous range of rows, visited in order.
__device__ __forceinline__ int xcd_remap(int b, int G) {
    if (G < 16 || (G & 7)) return b;
    return (b & 7) * (G >> 3) + (b >> 3);
}

// Status words for the host (pinned, device-visible): [1] status, [2] the
// iteration of the last FP64 check, [3] iterations, then [0] = 2 *
// generation + done with release order.  Done and the solve's generation
// travel in one word, so a host polling a reused slot can never pair a stale
// done of the previous occupant with the new generation; a host that sees
// done also sees the status.
__device__ __forceinline__ void publish_status(const SlotDesc& sd, int done, int status, int gen, int iters,
                                               int last_check) {
    if (!sd.host_status) return;
    __hip_atomic_store(sd.host_status + 1, status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(sd.host_status + 2, last_check, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(sd.host_status + 3, iters, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(sd.host_status, 2 * gen + (done ? 1 : 0), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ---- CG control shared by both engines --------------------------------------

// Whether an FP64 check must come before the next iteration, given the
// recursive r.r: at maxit; every `refresh` iterations (mixed mode); when the
// recursive residual meets the stop rule; or, as a reliable update, once it
// has fallen by sqrt(delta2) since the last replacement (past that point the
// working-precision recursion may drift from the true residual).  The last
// two need an iteration since the previous check, so checks alternate with
// progress.
// iters: the iteration count the decision is for (st->iters, unless the
// caller has counted an iteration whose store to st it cannot read back)
__device__ __forceinline__ bool check_due(const SolveState* st, double rr, int iters) {
    const bool progressed = iters > st->last_check_iter;
    const bool periodic = st->refresh > 0 && iters - st->last_check_iter >= st->refresh;
    const bool candidate = progressed && !(rr > st->trigger_rr);
    // a reliable update is skipped when the convergence trigger lies within
    // a factor 100 (10 in the residual norm) below its threshold: the check at
    // candidate convergence comes soon and replaces the residual as well
    const double rel = st->delta2 * st->rho_ref;
    const bool reliable = progressed && rr <= rel && st->trigger_rr < 1e-2 * rel;
    return iters >= st->maxit || candidate || periodic || reliable;
}
__device__ __forceinline__ bool check_due(const SolveState* st, double rr) { return check_due(st, rr, st->iters); }

// Outcome of an FP64 check from its reductions: |b - A x|^2 (R), |x|^2 (X),
// |b|^2 (B), |r_working|^2 (RW), invalid-input count (BAD), drift of the
// recursive residual (DIFF), min d.  Updates the state (one thread); returns
// 1 when CG continues with the replaced residual (r.r = RW), 0 when done.
__device__ inline int check_decide(SolveState* st, double R, double X, double B, double RW, double BAD,
                                   double DIFF, double dmin) {
    const bool first = st->checks == 0;
    st->checks += 1;
    if (first) {
        st->bnorm = sqrt(B);
        st->lam_lb = dmin + st->gmin;
    }
    const double rt = sqrt(R), xn = sqrt(X), bn = st->bnorm;
    if (first && BAD > 0.0) {
        st->status = ST_EINVAL;
        st->done = 1;
        return 0;
    }
    if (first && bn == 0.0) {
        st->status = ST_OK;
        st->done = 1;
        st->bzero = 1;
        st->true_relres = 0.0;
        st->bound = 0.0;
        return 0;
    }
    if (!isfinite(rt) || !isfinite(xn)) {
        st->status = ST_EBREAKDOWN;
        st->done = 1;
        return 0;
    }
    const double tau = st->tau, lam = st->lam_lb;
    const bool lit = rt <= st->tol * bn;
    const double cert_target = tau * lam * xn / (1.0 + tau);
    const bool cert = rt <= cert_target;
    const double e = rt / lam;
    st->true_relres = rt / bn;
    st->bound = xn > e ? e / (xn - e) : 1.0e300;
    if (lit && st->iters_literal < 0) st->iters_literal = st->iters;
    if (lit && cert) {
        st->status = ST_OK;
        st->done = 1;
        return 0;
    }
    if (st->iters >= st->maxit) {
        st->status = ST_ENOCONV;
        st->done = 1;
        return 0;
    }
    double trig = st->tol * bn;
    if (xn > 0.0 && cert_target < trig) trig = cert_target;
    st->trigger_rr = trig * trig;
    if (first) {
        st->worse = 0;
        st->best_rt = rt;
    } else if (rt >= st->best_rt) {
        st->worse += 1;
    } else {
        st->worse = 0;
        st->best_rt = rt;
    }
    if (st->worse >= 2) {
        st->restart = 1;
        st->worse = 0;
    }
    // Keeping p after the replacement is sound only while the recursive
    // residual still tracked the true one; past 10% drift the old direction
    // is no longer conjugate, so restart.
    if (!first && !(DIFF <= 0.01 * R)) st->restart = 1;
    st->rho_ref = RW;
    st->alpha = 0.0;
    st->last_check_iter = st->iters;
    st->last_rt = rt;
    st->xnorm = xn;
    st->pause = 0;
    return 1;
}

// ---- slot access policies -------------------------------------------------
struct ByPtr {
    const SlotDesc* p;
    // a copy, read once: the kernels' stores cannot alias it, so its fields
    // stay in registers instead of being read again after every store
    __device__ __forceinline__ SlotDesc get() const { return p[blockIdx.y]; }
};
struct ByVal {
    SlotDesc s;
    __device__ __forceinline__ const SlotDesc& get() const { return s; }
};

// gates: which slots a kernel works on (inactive slots first, then the
// solve's state; pause and done are adjacent words, read with one load).
__device__ __forceinline__ typename VecT<int, 2>::type pause_done(const SolveState* st) {
    static_assert(offsetof(SolveState, done) == offsetof(SolveState, pause) + sizeof(int) &&
                      offsetof(SolveState, pause) % 8 == 0,
                  "pause and done form one aligned 8-byte word");
    return *gbl(reinterpret_cast<const typename VecT<int, 2>::type*>(&st->pause));
}
struct GateAlways {
    static __device__ __forceinline__ bool ok(const SlotDesc&) { return true; }
};
struct GateIter {  // CG iteration kernels
    static __device__ __forceinline__ bool ok(const SlotDesc& sd) {
        if (!sd.active) return false;
        const auto pd = pause_done(sd.st);
        return (pd.x | pd.y) == 0;
    }
};
struct GateCheck {  // FP64 check kernels
    static __device__ __forceinline__ bool ok(const SlotDesc& sd) {
        if (!sd.active) return false;
        const auto pd = pause_done(sd.st);
        return pd.x != 0 && pd.y == 0;
    }
};
struct GatePre {  // preconditioner after a check that continues the solve
    static __device__ __forceinline__ bool ok(const SlotDesc& sd) {
        if (!sd.active) return false;
        const int done = *gbl(&sd.st->done), need = *gbl(&sd.st->need_pre);
        return (done == 0) & (need != 0);
    }
};

template <typename T>
struct Tab {
    const cx<T>* tw;   // exp(-2 pi i m / M), m in [0, M)
    const T* ghq;      // quarter spectrum / M^2 in tile layout
    const T* ghN;      // ghat(m, M/2) / M^2, m in [0, M/2]
};

template <typename T, int N>
struct PairT;
template <>
struct PairT<float, 2> { using type = float2; };
template <>
struct PairT<double, 2> { using type = double2; };

// a pair of consecutive elements (even index) of a device array
template <typename T>
__device__ __forceinline__ cx<T> ld2(const T* p) {
    return gld(reinterpret_cast<const cx<T>*>(p));
}
template <typename T>
__device__ __forceinline__ void st2(T* p, cx<T> c) {
    gst(reinterpret_cast<cx<T>*>(p), c);
}
__device__ __forceinline__ cx<double> ld2f(const float* p) {
    const cx<float> v = gld(reinterpret_cast<const cx<float>*>(p));
    return mkc((double)v.x, (double)v.y);
}
// Projection onto the intact entries of a masked solve: (m0, m1) in {0, 1}
// for the pair at idx (both 1 without a mask).
struct Mask2 {
    double m0, m1;
};
__device__ __forceinline__ Mask2 mask2(const SlotDesc& sd, size_t idx) {
    if (!sd.mask) return Mask2{1.0, 1.0};
    const auto* m = gbl(sd.mask + idx);
    return Mask2{(double)m[0], (double)m[1]};
}

// ==== prologues of the row-forward pass ====================================

// fftcg_apply: transform x (FP64 in memory), rounded to T.
template <typename T>
struct ProApply {
    static constexpr int NACC = 0;
    static constexpr bool PREF = false;
    struct Sh {};
    using Gate = GateAlways;
    static __device__ __forceinline__ bool begin(const SlotDesc&, Sh&, int, int) { return true; }
    template <int L>
    static __device__ __forceinline__ cx<T> load2(const SlotDesc& sd, const Sh&, int row, int col, double*) {
        cx<double> v = ld2<double>(sd.x + (size_t)row * L + col);
        return mkc((T)v.x, (T)v.y);
    }
};

// CG iteration: x_acc += alpha p_old (pending update of the last iteration),
// p = r + beta p_old (or p = r on restart), then transform p.
// W: working precision of r, p; XA: accumulator (double: x itself; float: e).
template <typename W, typename XA, int NT>
struct ProCG {
    static constexpr int NACC = 0;
    struct Sh {
        double red[(NT + 63) / 64];
        W alpha, beta;
        int restart;
    };
    using Gate = GateIter;
    static __device__ __forceinline__ bool begin(const SlotDesc& sd, Sh& sh, int npart_rr, int stride) {
        if (!GateIter::ok(sd)) return false;
        SolveState* st = sd.st;
        const double rr = sum_partials<NT>(sd.part + PS_RR * stride, npart_rr, sh.red);
        if (check_due(st, rr)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) st->pause = 1;
            return false;
        }
        const int restart = st->restart;
        const double beta = restart ? 0.0 : rr / st->rho_prev;
        sh.alpha = (W)st->alpha;
        sh.beta = (W)beta;
        sh.restart = restart;
        if (blockIdx.x == 0 && threadIdx.x == 0) st->rho_cur = rr;
        return true;
    }
    // FP32: the pair's r and p are requested before the r.r reduction
    // (fetch), so that the reduction's latency overlaps them; the arithmetic
    // (combine) is the same either way.  The pending x update (late) runs
    // after the transform: its reads then overlap the W writes instead of
    // lengthening the pass's first, read-only phase (p stays in registers
    // until then, within the pass's register budget)
    static constexpr bool PREF = sizeof(W) == 4;
#ifndef FFTCG_LATE_X
#define FFTCG_LATE_X 1
#endif
    static constexpr bool LATE_X = PREF && FFTCG_LATE_X;
    struct Raw {
        cx<W> r, p;
        cx<XA> x;
    };
    static __device__ __forceinline__ XA* xacc(const SlotDesc& sd) {
        return reinterpret_cast<XA*>(sizeof(XA) == 8 ? (void*)sd.x : (void*)sd.e);
    }
    template <int L>
    static __device__ __forceinline__ Raw fetch(const SlotDesc& sd, int row, int col) {
        const size_t idx = (size_t)row * L + col;
        Raw w;
        w.r = ld2<W>(reinterpret_cast<const W*>(sd.r) + idx);
        w.p = ld2<W>(reinterpret_cast<const W*>(sd.p) + idx);
        if constexpr (!LATE_X) w.x = ld2<XA>(xacc(sd) + idx);
        return w;
    }
    template <int L>
    static __device__ __forceinline__ cx<W> combine(const SlotDesc& sd, const Sh& sh, const Raw& w, int row,
                                                    int col, double*) {
        const size_t idx = (size_t)row * L + col;
        cx<W> p2;
        if (sh.restart) {
            p2 = w.r;
        } else {
            const cx<W> po = w.p;
            p2 = mkc(w.r.x + sh.beta * po.x, w.r.y + sh.beta * po.y);
            if constexpr (!LATE_X) {
                if (sh.alpha != W(0)) {
                    cx<XA> xv = w.x;
                    xv.x += (XA)sh.alpha * (XA)po.x;
                    xv.y += (XA)sh.alpha * (XA)po.y;
                    st2<XA>(xacc(sd) + idx, xv);
                }
            }
        }
        st2<W>(reinterpret_cast<W*>(sd.p) + idx, p2);
        return p2;
    }
    // the pending x update of the pair, after the transform (LATE_X)
    template <int L>
    static __device__ __forceinline__ void late(const SlotDesc& sd, const Sh& sh, const Raw& w, int row, int col) {
        if (sh.restart || sh.alpha == W(0)) return;
        const size_t idx = (size_t)row * L + col;
        cx<XA> xv = ld2<XA>(xacc(sd) + idx);
        xv.x += (XA)sh.alpha * (XA)w.p.x;
        xv.y += (XA)sh.alpha * (XA)w.p.y;
        st2<XA>(xacc(sd) + idx, xv);
    }
    template <int L>
    static __device__ __forceinline__ cx<W> load2(const SlotDesc& sd, const Sh& sh, int row, int col, double*) {
        const size_t idx = (size_t)row * L + col;
        W* p = reinterpret_cast<W*>(sd.p);
        const W* r = reinterpret_cast<const W*>(sd.r);
        cx<W> r2 = ld2<W>(r + idx);
        cx<W> p2;
        if (sh.restart) {
            p2 = r2;
        } else {
            cx<W> po = ld2<W>(p + idx);
            p2 = mkc(r2.x + sh.beta * po.x, r2.y + sh.beta * po.y);
            if (sh.alpha != W(0)) {
                XA* xa = xacc(sd);
                cx<XA> xv = ld2<XA>(xa + idx);
                xv.x += (XA)sh.alpha * (XA)po.x;
                xv.y += (XA)sh.alpha * (XA)po.y;
                st2<XA>(xa + idx, xv);
            }
        }
        st2<W>(p + idx, p2);
        return p2;
    }
};

// FP64 check: x <- x + e + alpha p (flush of the pending updates), e <- 0,
// transform x in FP64.
template <typename W, int NT>
struct ProCheck {
    static constexpr int NACC = 0;
    static constexpr bool PREF = false;
    struct Sh {
        double alpha;
        int mixed;
    };
    using Gate = GateCheck;
    static __device__ __forceinline__ bool begin(const SlotDesc& sd, Sh& sh, int, int) {
        if (!GateCheck::ok(sd)) return false;
        sh.alpha = sd.st->alpha;
        sh.mixed = sd.st->mixed;
        return true;
    }
    template <int L>
    static __device__ __forceinline__ cx<double> load2(const SlotDesc& sd, const Sh& sh, int row, int col,
                                                       double*) {
        const size_t idx = (size_t)row * L + col;
        cx<double> xv = ld2<double>(sd.x + idx);
        if (sh.mixed) {
            cx<double> ev = ld2f(sd.e + idx);
            xv.x += ev.x;
            xv.y += ev.y;
            st2<float>(sd.e + idx, mkc(0.0f, 0.0f));
        }
        if (sh.alpha != 0.0) {
            const W* p = reinterpret_cast<const W*>(sd.p);
            cx<W> pv = ld2<W>(p + idx);
            xv.x += sh.alpha * (double)pv.x;
            xv.y += sh.alpha * (double)pv.y;
        }
        const Mask2 mk = mask2(sd, idx);  // broken entries carry no force
        xv.x *= mk.m0;
        xv.y *= mk.m1;
        st2<double>(sd.x + idx, xv);
        return xv;
    }
};

// Preconditioned CG (Fourier-space circulant preconditioner), first half of
// an iteration: beta = (r.z) / (r.z)_old from the partials of the
// preconditioner pass, p = z + beta p (p = z on restart), pending x update,
// then transform p.  The stop triggers still use r.r.  NPZ: partial count of
// the r.z sums.
template <typename W, typename XA, int NT, int NPZ>
struct ProPCG {
    static constexpr int NACC = 0;
    // FP32: z, p and the x correction are requested before the reductions
    static constexpr bool PREF = sizeof(W) == 4;
    struct Sh {
        double red[2 * ((NT + 63) / 64)];
        double tot[2];
        W alpha, beta;
        int restart;
    };
    using Gate = GateIter;
    static __device__ __forceinline__ bool begin(const SlotDesc& sd, Sh& sh, int npart_rr, int stride) {
        if (!GateIter::ok(sd)) return false;
        SolveState* st = sd.st;
        double rr, rz;
        if constexpr (NT % 64 == 0) {
            // r.r and r.z reduced together (each in sum_partials' order)
            double a2[2] = {0.0, 0.0};
            const auto* prr = gbl(sd.part + PS_RR * stride);
            const auto* prz = gbl(sd.part + PS_RZ * stride);
            for (int i = threadIdx.x; i < npart_rr; i += NT) a2[0] += prr[i];
            for (int i = threadIdx.x; i < NPZ; i += NT) a2[1] += prz[i];
            const double t = block_reduce_n<NT, 2, 0u>(a2, sh.red);
            if (threadIdx.x < 2) sh.tot[threadIdx.x] = t;
            __syncthreads();
            rr = sh.tot[0];
            rz = sh.tot[1];
        } else {
            rr = sum_partials<NT>(sd.part + PS_RR * stride, npart_rr, sh.red);
            rz = sum_partials<NT>(sd.part + PS_RZ * stride, NPZ, sh.red);
        }
        if (check_due(st, rr)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) st->pause = 1;
            return false;
        }
        const int restart = st->restart;
        const double beta = restart ? 0.0 : rz / st->rho_prev;
        sh.alpha = (W)st->alpha;
        sh.beta = (W)beta;
        sh.restart = restart;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->rho_cur = rz;
            st->need_pre = 0;
        }
        return true;
    }
    struct Raw {
        cx<W> z, p;
        cx<XA> x;
    };
    static __device__ __forceinline__ XA* xacc(const SlotDesc& sd) {
        return reinterpret_cast<XA*>(sizeof(XA) == 8 ? (void*)sd.x : (void*)sd.e);
    }
    template <int L>
    static __device__ __forceinline__ Raw fetch(const SlotDesc& sd, int row, int col) {
        const size_t idx = (size_t)row * L + col;
        Raw w;
        w.z = ld2<W>(reinterpret_cast<const W*>(sd.z) + idx);
        w.p = ld2<W>(reinterpret_cast<const W*>(sd.p) + idx);
        w.x = ld2<XA>(xacc(sd) + idx);
        return w;
    }
    template <int L>
    static __device__ __forceinline__ cx<W> combine(const SlotDesc& sd, const Sh& sh, const Raw& w, int row,
                                                    int col, double*) {
        const size_t idx = (size_t)row * L + col;
        cx<W> p2;
        if (sh.restart) {
            p2 = w.z;
        } else {
            const cx<W> po = w.p;
            p2 = mkc(w.z.x + sh.beta * po.x, w.z.y + sh.beta * po.y);
            if (sh.alpha != W(0)) {
                cx<XA> xv = w.x;
                xv.x += (XA)sh.alpha * (XA)po.x;
                xv.y += (XA)sh.alpha * (XA)po.y;
                st2<XA>(xacc(sd) + idx, xv);
            }
        }
        st2<W>(reinterpret_cast<W*>(sd.p) + idx, p2);
        return p2;
    }
    template <int L>
    static __device__ __forceinline__ cx<W> load2(const SlotDesc& sd, const Sh& sh, int row, int col, double*) {
        const size_t idx = (size_t)row * L + col;
        W* p = reinterpret_cast<W*>(sd.p);
        const W* z = reinterpret_cast<const W*>(sd.z);
        cx<W> z2 = ld2<W>(z + idx);
        cx<W> p2;
        if (sh.restart) {
            p2 = z2;
        } else {
            cx<W> po = ld2<W>(p + idx);
            p2 = mkc(z2.x + sh.beta * po.x, z2.y + sh.beta * po.y);
            if (sh.alpha != W(0)) {
                XA* xa = reinterpret_cast<XA*>(sizeof(XA) == 8 ? (void*)sd.x : (void*)sd.e);
                cx<XA> xv = ld2<XA>(xa + idx);
                xv.x += (XA)sh.alpha * (XA)po.x;
                xv.y += (XA)sh.alpha * (XA)po.y;
                st2<XA>(xa + idx, xv);
            }
        }
        st2<W>(p + idx, p2);
        return p2;
    }
};

// Preconditioned CG, second half: alpha = (r.z) / (p.q) from the partials of
// the operator's row-inverse pass (breakdown if p.q <= 0), r <- r - alpha q
// with partial r.r, then transform r for z = P^{-1} r.  NPQ: partial count of
// the p.q sums.
template <typename W, int NT, int NPQ>
struct ProUpdPre {
    static constexpr int NACC = 1;
    static constexpr bool PREF = sizeof(W) == 4;  // r and q requested before the p.q reduction
    static constexpr int SET = PS_RR;
    struct Sh {
        double red[(NT + 63) / 64];
        W alpha;
    };
    using Gate = GateIter;
    static __device__ __forceinline__ bool begin(const SlotDesc& sd, Sh& sh, int, int stride) {
        if (!GateIter::ok(sd)) return false;
        SolveState* st = sd.st;
        const double pq = sum_partials<NT>(sd.part + PS_PQ * stride, NPQ, sh.red);
        const double rho = st->rho_cur;
        if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rho)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                st->status = ST_EBREAKDOWN;
                st->done = 1;
                publish_status(sd, 1, ST_EBREAKDOWN, st->gen, st->iters, st->last_check_iter);
            }
            return false;
        }
        const double alpha = rho / pq;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->alpha = alpha;
            st->rho_prev = rho;
            st->iters += 1;
            st->restart = 0;
        }
        sh.alpha = (W)alpha;
        return true;
    }
    template <int L>
    static __device__ __forceinline__ cx<W> load2(const SlotDesc& sd, const Sh& sh, int row, int col,
                                                  double* acc) {
        const size_t idx = (size_t)row * L + col;
        W* r = reinterpret_cast<W*>(sd.r);
        const W* q = reinterpret_cast<const W*>(sd.q);
        const cx<W> r2 = ld2<W>(r + idx), q2 = ld2<W>(q + idx);
        const cx<W> rn = mkc(r2.x - sh.alpha * q2.x, r2.y - sh.alpha * q2.y);
        st2<W>(r + idx, rn);
        acc[0] += (double)rn.x * (double)rn.x + (double)rn.y * (double)rn.y;
        return rn;
    }
    struct Raw {
        cx<W> r, q;
    };
    template <int L>
    static __device__ __forceinline__ Raw fetch(const SlotDesc& sd, int row, int col) {
        const size_t idx = (size_t)row * L + col;
        return Raw{ld2<W>(reinterpret_cast<const W*>(sd.r) + idx), ld2<W>(reinterpret_cast<const W*>(sd.q) + idx)};
    }
    template <int L>
    static __device__ __forceinline__ cx<W> combine(const SlotDesc& sd, const Sh& sh, const Raw& w, int row,
                                                    int col, double* acc) {
        const size_t idx = (size_t)row * L + col;
        const cx<W> rn = mkc(w.r.x - sh.alpha * w.q.x, w.r.y - sh.alpha * w.q.y);
        st2<W>(reinterpret_cast<W*>(sd.r) + idx, rn);
        acc[0] += (double)rn.x * (double)rn.x + (double)rn.y * (double)rn.y;
        return rn;
    }
};

// Preconditioner after a check that continues the solve: transform the
// replaced residual r.
template <typename W>
struct ProPre {
    static constexpr int NACC = 0;
    static constexpr bool PREF = false;
    struct Sh {};
    using Gate = GatePre;
    static __device__ __forceinline__ bool begin(const SlotDesc& sd, Sh&, int, int) { return GatePre::ok(sd); }
    template <int L>
    static __device__ __forceinline__ cx<W> load2(const SlotDesc& sd, const Sh&, int row, int col, double*) {
        return ld2<W>(reinterpret_cast<const W*>(sd.r) + (size_t)row * L + col);
    }
};

// ==== epilogues of the row-inverse pass ====================================

// fftcg_apply: y = d * x (FP64) + C x.
template <typename T>
struct EpiApply {
    static constexpr int NACC = 0;
    static constexpr bool PREF = false;
    using Gate = GateAlways;
    static __device__ __forceinline__ bool begin(const SlotDesc&) { return true; }
    template <int L>
    static __device__ __forceinline__ void out2(const SlotDesc& sd, int row, int col, T c0, T c1, double*) {
        const size_t idx = (size_t)row * L + col;
        cx<double> dv = ld2<double>(sd.d + idx);
        cx<double> xv = ld2<double>(sd.x + idx);
        st2<double>(sd.y + idx, mkc(dv.x * xv.x + (double)c0, dv.y * xv.y + (double)c1));
    }
    static __device__ __forceinline__ void finish(const SlotDesc&, const double*, int) {}
};

// CG iteration: q = d p + C p; partial p . q (FP64 accumulation).
template <typename W>
struct EpiCG {
    static constexpr int NACC = 1;
    static constexpr int SET = PS_PQ;
    using Gate = GateIter;
    static __device__ __forceinline__ bool begin(const SlotDesc& sd) { return GateIter::ok(sd); }
    // FP32: p and d of every output are requested before the transform, so
    // their reads neither wait behind the q stores (which may alias them as
    // far as the compiler knows) nor expose their latency after it
    static constexpr bool PREF = sizeof(W) == 4;
    struct Pre {
        cx<W> p, d;
    };
    template <int L>
    static __device__ __forceinline__ Pre pre(const SlotDesc& sd, int row, int col) {
        const size_t idx = (size_t)row * L + col;
        Pre v;
        v.p = ld2<W>(reinterpret_cast<const W*>(sd.p) + idx);
        if constexpr (sizeof(W) == 4) {
            v.d = ld2<float>(sd.d32 + idx);
        } else {
            v.d = ld2<double>(sd.d + idx);
        }
        return v;
    }
    template <int L>
    static __device__ __forceinline__ void out2(const SlotDesc& sd, int row, int col, W c0, W c1, double* acc) {
        out2p<L>(sd, row, col, c0, c1, pre<L>(sd, row, col), acc);
    }
    template <int L>
    static __device__ __forceinline__ void out2p(const SlotDesc& sd, int row, int col, W c0, W c1, const Pre& pr,
                                                 double* acc) {
        const size_t idx = (size_t)row * L + col;
        W* q = reinterpret_cast<W*>(sd.q);
        const cx<W> pv = pr.p, dv = pr.d;
        cx<W> qv = mkc(dv.x * pv.x + c0, dv.y * pv.y + c1);
        if (sd.mask) {
            const Mask2 mk = mask2(sd, idx);
            qv = mkc(qv.x * (W)mk.m0, qv.y * (W)mk.m1);
        }
        st2<W>(q + idx, qv);
        acc[0] += (double)pv.x * (double)qv.x + (double)pv.y * (double)qv.y;
    }
    // q of a pair without storing it (the grid-synchronised update below)
    template <int L>
    static __device__ __forceinline__ cx<W> outq(const SlotDesc& sd, int row, int col, W c0, W c1, const Pre& pr,
                                                 double* acc) {
        const cx<W> pv = pr.p, dv = pr.d;
        cx<W> qv = mkc(dv.x * pv.x + c0, dv.y * pv.y + c1);
        if (sd.mask) {
            const Mask2 mk = mask2(sd, (size_t)row * L + col);
            qv = mkc(qv.x * (W)mk.m0, qv.y * (W)mk.m1);
        }
        acc[0] += (double)pv.x * (double)qv.x + (double)pv.y * (double)qv.y;
        return qv;
    }
};

// The CG epilogue with the residual update folded in: q = A p never leaves
// registers.  After every workgroup has published its p.q
// partial (a grid-wide barrier; the host launches this only where the whole
// grid fits the device at once), each workgroup forms alpha = rho / (p.q)
// from all partials in the same order and updates r <- r - alpha q on its
// own rows, with the r.r partials of the next iteration.  It replaces the
// separate update kernel: one pass over q fewer, and one kernel fewer.
template <typename W>
struct EpiCGU : EpiCG<W> {
    static constexpr bool UPD = true;
};
template <class E, class = void>
struct EpiUpd {
    static constexpr bool value = false;
};
template <class E>
struct EpiUpd<E, decltype((void)E::UPD)> {
    static constexpr bool value = E::UPD;
};

// Grid-wide barrier without read-modify-write traffic on one address (1,024
// atomic additions to one counter serialise where they are performed and
// cost tens of microseconds).  Each launch carries a token that no other
// launch on the same partial-sum buffer uses.  A workgroup arrives by
// storing the token to its own word flags[b]; workgroup 0 waits until every
// flag holds the token, then stores it to the release word *rel, which the
// others wait for.  All of these are agent-scope atomics, performed where
// every XCD sees them, and each step waits for the previous step's value, so
// no cache-wide fence is needed (a release/acquire pair at agent scope
// writes back and invalidates the L2 of every workgroup's XCD, which costs
// more than the whole update).  Waits are bounded: after `limit` ticks of
// the 100 MHz constant clock the workgroup gives up and false is returned (a
// grid that is not resident as a whole cannot complete the barrier).
// Called by every thread of the workgroup; returns the same value in all.
template <int NT>
__device__ inline bool grid_barrier(unsigned long long* flags, unsigned long long* rel, unsigned long long token,
                                    long long limit) {
    __shared__ int s_ok;
    const int tid = threadIdx.x;
    const unsigned int nb = gridDim.x;
    if (tid == 0) __hip_atomic_store(flags + blockIdx.x, token, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    int ok = 1;
    if (blockIdx.x == 0) {
        for (;;) {
            int mine = 1;
            for (unsigned int i = tid; i < nb; i += NT)
                mine &= __hip_atomic_load(flags + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == token;
            const int expired = (long long)(__builtin_amdgcn_s_memrealtime() - t0) > limit;
            // both decisions are taken by the whole workgroup
            if (__syncthreads_and(mine)) break;
            if (__syncthreads_or(expired)) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (ok && tid == 0) __hip_atomic_store(rel, token, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        if (tid == 0) {
            while (__hip_atomic_load(rel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != token) {
                if ((long long)(__builtin_amdgcn_s_memrealtime() - t0) > limit) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            s_ok = ok;
        }
        __syncthreads();
        ok = s_ok;
    }
    return ok != 0;
}

// FP64 check: r64 = b - d x - C x; r (working precision) <- r64; partials of
// |r64|^2, |x|^2, |b|^2, |r|^2, min d, the count of invalid inputs and
// |r64 - r_old|^2 (drift of the recursive residual it replaces).
template <typename W>
struct EpiCheck {
    static constexpr int NACC = 8;
    static constexpr bool PREF = false;
    using Gate = GateCheck;
    static __device__ __forceinline__ bool begin(const SlotDesc& sd) { return GateCheck::ok(sd); }
    template <int L>
    static __device__ __forceinline__ void out2(const SlotDesc& sd, int row, int col, double c0, double c1,
                                                double* acc) {
        const size_t idx = (size_t)row * L + col;
        cx<double> xv = ld2<double>(sd.x + idx);
        cx<double> bv = ld2<double>(sd.b + idx);
        cx<double> dv = ld2<double>(sd.d + idx);
        const Mask2 mk = mask2(sd, idx);
        const double r0 = mk.m0 * (bv.x - (dv.x * xv.x + c0));
        const double r1 = mk.m1 * (bv.y - (dv.y * xv.y + c1));
        bv = mkc(mk.m0 * bv.x, mk.m1 * bv.y);
        const W w0 = (W)r0, w1 = (W)r1;
        W* rp = reinterpret_cast<W*>(sd.r) + idx;
        if (sd.st->checks > 0) {  // the first check has no recursive residual yet
            const cx<W> ro = ld2<W>(rp);
            acc[6] += (r0 - (double)ro.x) * (r0 - (double)ro.x) + (r1 - (double)ro.y) * (r1 - (double)ro.y);
        }
        st2<W>(rp, mkc(w0, w1));
        acc[0] += r0 * r0 + r1 * r1;
        acc[1] += xv.x * xv.x + xv.y * xv.y;
        acc[2] += bv.x * bv.x + bv.y * bv.y;
        acc[3] += (double)w0 * (double)w0 + (double)w1 * (double)w1;
        acc[4] = fmin(acc[4], fmin(mk.m0 > 0.0 ? dv.x : 1.0e300, mk.m1 > 0.0 ? dv.y : 1.0e300));
        const bool ok = isfinite(bv.x) && isfinite(bv.y) && isfinite(dv.x) && isfinite(dv.y) &&
                        dv.x >= 0.0 && dv.y >= 0.0;
        acc[5] += ok ? 0.0 : 1.0;
        acc[7] += dv.x + dv.y;
    }
};

// Preconditioner: z = C' r (C' the convolution with 1/(dbar + ghat); no
// diagonal term); partial r . z (FP64 accumulation).
template <typename W, class G>
struct EpiPre {
    static constexpr int NACC = 1;
    static constexpr int SET = PS_RZ;
    using Gate = G;
    static __device__ __forceinline__ bool begin(const SlotDesc& sd) { return G::ok(sd); }
    static constexpr bool PREF = sizeof(W) == 4;  // r requested before the transform
    struct Pre {
        cx<W> r;
    };
    template <int L>
    static __device__ __forceinline__ Pre pre(const SlotDesc& sd, int row, int col) {
        return Pre{ld2<W>(reinterpret_cast<const W*>(sd.r) + (size_t)row * L + col)};
    }
    template <int L>
    static __device__ __forceinline__ void out2(const SlotDesc& sd, int row, int col, W c0, W c1, double* acc) {
        out2p<L>(sd, row, col, c0, c1, pre<L>(sd, row, col), acc);
    }
    template <int L>
    static __device__ __forceinline__ void out2p(const SlotDesc& sd, int row, int col, W c0, W c1, const Pre& pr,
                                                 double* acc) {
        const size_t idx = (size_t)row * L + col;
        const cx<W> rv = pr.r;
        if (sd.mask) {
            const Mask2 mk = mask2(sd, idx);
            c0 *= (W)mk.m0;
            c1 *= (W)mk.m1;
        }
        st2<W>(reinterpret_cast<W*>(sd.z) + idx, mkc(c0, c1));
        acc[0] += (double)rv.x * (double)c0 + (double)rv.y * (double)c1;
    }
};

// Whether a prologue defers part of its work until after the transform.
template <class P, class = void>
struct ProLate {
    static constexpr bool value = false;
};
template <class P>
struct ProLate<P, decltype((void)P::LATE_X)> {
    static constexpr bool value = P::LATE_X;
};

// A prologue's fetched operands kept for its late part (int otherwise).
template <class P, bool = ProLate<P>::value>
struct LateRaw {
    using type = int;
};
template <class P>
struct LateRaw<P, true> {
    using type = typename P::Raw;
};

// Prefetched epilogue operands of an epilogue with PREF (its Pre type).
template <class Epi, bool = Epi::PREF>
struct EpiPreT {
    using type = int;
};
template <class Epi>
struct EpiPreT<Epi, true> {
    using type = typename Epi::Pre;
};

// ==== kernels ==============================================================

// The forward row transform of the thread's inputs v (the row's packed
// values, as the prologue placed them), the split of the packed transform
// into the half spectrum of the real row, and the W stores of the
// workgroup's rows (block rb).
template <typename T, int M, int PAD, int NT>
__device__ __forceinline__ void row_fwd_out(cx<T>* v, cx<T>* lds, const Tab<T>& tab, const SlotDesc& sd, int rb) {
    using G = Geo<T, M, PAD>;
    constexpr int N = G::N, E = G::ER, P = G::PR, RPW = G::RPW, L = G::L, TT = G::TT;
    constexpr int WORDS = G::ROW_WORDS;
    const int tid = threadIdx.x;
    const int rl = tid / P, j = tid % P;
    LdsLay<T, 1, 4, 1> lay{lds + rl * WORDS, 0};
    constexpr int NSTG = fft_nstages(N);
    fft_run<T, N, M, -1, false, PAD != 0>(v, lay, j, tab.tw);
    constexpr int RL = NSTG > 0 ? fft_radix(N, false, NSTG - 1) : 1;
    if constexpr (NSTG > 1) __syncthreads();  // the transform's last reads before these writes
#pragma unroll
    for (int u = 0; u < E / RL; ++u) lay.template st_run<RL, N / RL>(j + u * P, v + u * RL);
    __syncthreads();
    cx<T>* Wb = reinterpret_cast<cx<T>*>(sd.W);
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int qi = tid + s * NT;
        const int kk = qi % TT;
        const int il = (qi / TT) % RPW;
        const int kt = qi / (TT * RPW);
        const int k = kt * TT + kk;
        LdsLay<T, 1, 4, 1> rl2{lds + il * WORDS, 0};
        const cx<T> Zk = rl2.ld(k);
        cx<T> out;
        if (k == 0) {
            out = mkc(Zk.x + Zk.y, Zk.x - Zk.y);
        } else {
            const cx<T> B = conjc(rl2.ld(N - k));
            const cx<T> s1 = Zk + B, d1 = Zk - B;
            const cx<T> wd = cmul(tab.tw[k], d1);
            out = mkc(T(0.5) * (s1.x + wd.y), T(0.5) * (s1.y - wd.x));
        }
        gst(Wb + ((size_t)kt * L + rb * RPW + il) * TT + kk, out);
    }
}

template <typename T, int M, int PAD, class Pro, class Slot, int NT>
__global__ void __launch_bounds__(NT) k_row_fwd(Tab<T> tab, Slot slot, int npart_rr, int stride) {
    using G = Geo<T, M, PAD>;
    constexpr int N = G::N, E = G::ER, P = G::PR, RPW = G::RPW, L = G::L;
    constexpr int WORDS = G::ROW_WORDS;
    static_assert(NT == G::ROW_THREADS, "row-forward block size");
    __shared__ cx<T> lds[RPW * WORDS];
    __shared__ typename Pro::Sh sh;
    __shared__ double fred[(NT + 63) / 64];
    const SlotDesc& sd = slot.get();
    double acc = 0.0;
    const int tid = threadIdx.x;
    const int rl = tid / P, j = tid % P;
    const int rb = xcd_remap(blockIdx.x, gridDim.x);
    const int row = rb * RPW + rl;
    cx<T> v[E];
    constexpr int NSTG = fft_nstages(N);
    constexpr int R1 = NSTG > 0 ? fft_radix(N, false, 0) : 1;
    constexpr int RK = PAD ? R1 / 2 : R1;  // inputs per run (the rest are known zeros on the padded grid)
    constexpr bool LATE = ProLate<Pro>::value;
    typename LateRaw<Pro>::type late_raw[LATE ? (E / R1) * RK : 1];
    if constexpr (Pro::PREF && (E / R1) * RK <= 8) {
        // the inputs are requested before begin()'s reductions
        if (!Pro::Gate::ok(sd)) return;
        typename Pro::Raw raw[(E / R1) * RK];
#pragma unroll
        for (int u = 0; u < E / R1; ++u)
#pragma unroll
            for (int r = 0; r < RK; ++r)
                raw[u * RK + r] = Pro::template fetch<L>(sd, row, 2 * ((j + u * P) + r * (N / R1)));
        if (!Pro::begin(sd, sh, npart_rr, stride)) return;
#pragma unroll
        for (int u = 0; u < E / R1; ++u)
#pragma unroll
            for (int r = 0; r < RK; ++r)
                v[u * R1 + r] = Pro::template combine<L>(sd, sh, raw[u * RK + r], row,
                                                         2 * ((j + u * P) + r * (N / R1)), &acc);
        if constexpr (LATE) {
#pragma unroll
            for (int i = 0; i < (E / R1) * RK; ++i) late_raw[i] = raw[i];
        }
    } else {
        if (!Pro::begin(sd, sh, npart_rr, stride)) return;
#pragma unroll
        for (int u = 0; u < E / R1; ++u)
#pragma unroll
            for (int r = 0; r < RK; ++r)
                v[u * R1 + r] = Pro::template load2<L>(sd, sh, row, 2 * ((j + u * P) + r * (N / R1)), &acc);
    }
    row_fwd_out<T, M, PAD, NT>(v, lds, tab, sd, rb);
    if constexpr (LATE && Pro::PREF && (E / R1) * RK <= 8) {
#pragma unroll
        for (int u = 0; u < E / R1; ++u)
#pragma unroll
            for (int r = 0; r < RK; ++r)
                Pro::template late<L>(sd, sh, late_raw[u * RK + r], row, 2 * ((j + u * P) + r * (N / R1)));
    }
    if constexpr (Pro::NACC > 0) {
        const double s = block_sum<NT>(acc, fred);
        if (tid == 0) sd.part[Pro::SET * stride + blockIdx.x] = s;
    }
}

// Multiplier of the preconditioner from the stored ghat / M^2:
// 1 / (M^2 (dbar + ghat)) = 1 / (M^2 dbar + M^4 g).  Real, positive and even
// like ghat, so the preconditioner is symmetric positive definite.
__device__ __forceinline__ float pre_mul(float g, float c2, float c4) {
    return __builtin_amdgcn_rcpf(fmaf(c4, g, c2));
}
__device__ __forceinline__ double pre_mul(double g, double c2, double c4) { return 1.0 / fma(c4, g, c2); }

// PRE: multiply by the preconditioner's multiplier instead of ghat / M^2.
template <typename T, int M, int PAD, class Gate, class Slot, int NT, bool PRE = false>
__global__ void __launch_bounds__(NT) k_col(Tab<T> tab, Slot slot) {
    using G = Geo<T, M, PAD>;
    constexpr int E = G::EC, P = G::PC, TT = G::TT, L = G::L, MH = G::MH;
    static_assert(NT == G::COL_THREADS, "column block size");
    using Lay = LdsLay<T, TT, G::COL_SH, TT>;
    __shared__ cx<T> lds[Lay::words(M)];
    const SlotDesc& sd = slot.get();
    if (!Gate::ok(sd)) return;
    const int kt = blockIdx.x;
    const int tid = threadIdx.x, kk = tid % TT, j = tid / TT;
    Lay lay{lds, kk};
    cx<T>* Wt = reinterpret_cast<cx<T>*>(sd.W) + (size_t)kt * L * TT;
    cx<T> v[E];
    constexpr int NSTG = fft_nstages(M);
    constexpr int R1 = fft_radix(M, false, 0);
#pragma unroll
    for (int u = 0; u < E / R1; ++u)
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            if (PAD && r >= R1 / 2) continue;
            const int n = (j + u * P) + r * (M / R1);
            v[u * R1 + r] = gld(Wt + (size_t)n * TT + kk);
        }
    constexpr int RL = fft_radix(M, false, NSTG - 1);
    const T* g = tab.ghq + (size_t)kt * MH * TT;
    // the spectrum values this thread multiplies by, requested together with
    // the column data so their latency is not exposed after the transform
    T gpre[E];
#pragma unroll
    for (int u = 0; u < E / RL; ++u)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int m = (j + u * P) + r * (M / RL);
            const int mp = m <= M - m ? m : M - m;
            gpre[u * RL + r] = g[mp * TT + kk];
        }
    const T c2 = PRE ? (T)((double)M * (double)M * sd.st->dbar) : T(0);
    const T c4 = (T)((double)M * (double)M * (double)M * (double)M);
    if constexpr (PRE) {
#pragma unroll
        for (int i = 0; i < E; ++i) gpre[i] = pre_mul(gpre[i], c2, c4);
    }
    fft_run<T, M, M, -1, false, PAD != 0>(v, lay, j, tab.tw);
    if (kt == 0) {
        // packed column 0 carries k = 0 (real part) and k = M/2 (imaginary
        // part): result(m) = s(m) W(m) + t(m) conj(W(M - m)),
        // s = (g0 + gN)/2, t = (g0 - gN)/2.
        if constexpr (NSTG > 1) __syncthreads();  // the transform's last reads before these writes
#pragma unroll
        for (int u = 0; u < E / RL; ++u) lay.template st_run<RL, M / RL>(j + u * P, v + u * RL);
        // this thread's values of the spectrum's column M/2, read together
        // (inside the per-element branch below each read would wait for the
        // previous element)
        T gN[E];
#pragma unroll
        for (int u = 0; u < E / RL; ++u)
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int m = (j + u * P) + r * (M / RL);
                gN[u * RL + r] = tab.ghN[m <= M - m ? m : M - m];
            }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < E / RL; ++u)
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int m = (j + u * P) + r * (M / RL);
                const cx<T> a = v[u * RL + r];
                if (kk == 0) {
                    const cx<T> bm = conjc(lay.ld((M - m) & (M - 1)));
                    const T g0 = gpre[u * RL + r];
                    const T gNv = PRE ? pre_mul(gN[u * RL + r], c2, c4) : gN[u * RL + r];
                    const T s = T(0.5) * (g0 + gNv), t = T(0.5) * (g0 - gNv);
                    v[u * RL + r] = mkc(s * a.x + t * bm.x, s * a.y + t * bm.y);
                } else {
                    v[u * RL + r] = scalec(a, gpre[u * RL + r]);
                }
            }
        __syncthreads();
    } else {
#pragma unroll
        for (int u = 0; u < E / RL; ++u)
#pragma unroll
            for (int r = 0; r < RL; ++r) v[u * RL + r] = scalec(v[u * RL + r], gpre[u * RL + r]);
    }
    // the forward transform's (or column 0's) reads of the buffer came before
    fft_run<T, M, M, +1, true, false, Lay, true>(v, lay, j, tab.tw);
    constexpr int RZ = fft_radix(M, true, NSTG - 1);
#pragma unroll
    for (int u = 0; u < E / RZ; ++u)
#pragma unroll
        for (int r = 0; r < RZ; ++r) {
            if (PAD && r >= RZ / 2) continue;
            const int n = (j + u * P) + r * (M / RZ);
            gst(Wt + (size_t)n * TT + kk, v[u * RZ + r]);
        }
}

// Body of the row-inverse pass; token: the grid-wide barrier's arrival
// token of this launch (epilogues with the folded update only).
// FWD (with the folded update only): the pass goes on into the next
// iteration's forward row pass on the same rows (k_row_turn).
template <typename T, int M, int PAD, class Epi, class Slot, int NT, bool FWD = false>
__device__ __forceinline__ void row_inv_body(const Tab<T>& tab, const Slot& slot, int stride,
                                             unsigned long long token) {
    using G = Geo<T, M, PAD>;
    constexpr int N = G::N, E = G::ER, P = G::PR, RPW = G::RPW, L = G::L, TT = G::TT;
    constexpr int WORDS = G::ROW_WORDS;
    static_assert(NT == G::ROW_THREADS, "row-inverse block size");
    __shared__ cx<T> lds[RPW * WORDS];
    __shared__ double red[(Epi::NACC > 1 ? Epi::NACC : 1) * ((NT + 63) / 64)];
    const SlotDesc& sd = slot.get();
    if (!Epi::begin(sd)) return;
    const int tid = threadIdx.x;
    const int rl = tid / P, j = tid % P;
    const int row0 = xcd_remap(blockIdx.x, gridDim.x) * RPW;
    // FWD: the iteration count as this launch found it (block 0 advances
    // st->iters after the first barrier; read before this workgroup arrives)
    __shared__ int s_iters;
    if (FWD && tid == 0) s_iters = sd.st->iters;
    const cx<T>* Wb = reinterpret_cast<const cx<T>*>(sd.W);
    // all of this thread's spectrum values are requested before the first
    // is stored to LDS (more reads in flight per wave)
    cx<T> wv[E];
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int qi = tid + s * NT;
        const int kk = qi % TT;
        const int il = (qi / TT) % RPW;
        const int kt = qi / (TT * RPW);
        wv[s] = gld(Wb + ((size_t)kt * L + row0 + il) * TT + kk);
    }
    constexpr int NSTG = fft_nstages(N);
    constexpr int R1 = NSTG > 0 ? fft_radix(N, true, 0) : 1;
    constexpr int S1 = N / R1;
    // the unpack's twiddles, requested with the spectrum (before the barrier)
    cx<T> twk[E];
#pragma unroll
    for (int u = 0; u < E / R1; ++u)
#pragma unroll
        for (int r = 0; r < R1; ++r) twk[u * R1 + r] = gld(tab.tw + (j + u * P) + r * S1);
    constexpr int RL = NSTG > 0 ? fft_radix(N, true, NSTG - 1) : 1;
    constexpr int RK = (PAD && RL > 1) ? RL / 2 : RL;  // outputs kept per run (the rest are cropped)
    const int row = row0 + rl;
    // the epilogue's operands (Epi::PREF), requested with the spectrum; not
    // in the turn pass (FWD) on the largest rows (16 pairs a thread), which
    // keeps p of the pairs to its end and would otherwise exceed 128 VGPRs
    // (four workgroups per CU)
    constexpr bool PF = Epi::PREF && !(FWD && E >= 16);
    using PreT = typename EpiPreT<Epi>::type;
    PreT pre[PF ? (E / RL) * RK : 1];
    if constexpr (PF) {
#pragma unroll
        for (int u = 0; u < E / RL; ++u)
#pragma unroll
            for (int r = 0; r < RK; ++r)
                pre[u * RK + r] = Epi::template pre<L>(sd, row, 2 * ((j + u * P) + r * (N / RL)));
    }
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int qi = tid + s * NT;
        const int kk = qi % TT;
        const int il = (qi / TT) % RPW;
        const int kt = qi / (TT * RPW);
        LdsLay<T, 1, 4, 1> l2{lds + il * WORDS, 0};
        l2.st(kt * TT + kk, wv[s]);
    }
    __syncthreads();
    LdsLay<T, 1, 4, 1> lay{lds + rl * WORDS, 0};
    cx<T> v[E];
#pragma unroll
    for (int u = 0; u < E / R1; ++u) {
        // Y at k = jj + r S1, and the partners N - k = (S1 - jj) + (R1-1-r) S1
        // (jj > 0) or (R1 - r) S1 (jj == 0), read as two runs
        const int jj = j + u * P;
        cx<T> A[R1], Bv[R1];
        lay.template ld_run<R1, S1>(jj, A);
        lay.template ld_run<R1, S1>(jj == 0 ? 0 : S1 - jj, Bv);
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            const int k = jj + r * S1;
            const cx<T> Y = A[r];
            cx<T> Z;
            if (k == 0) {
                Z = mkc(Y.x + Y.y, Y.x - Y.y);
            } else {
                const cx<T> B = conjc(jj == 0 ? Bv[(R1 - r) % R1] : Bv[R1 - 1 - r]);
                const cx<T> s1 = Y + B, d1 = Y - B;
                const cx<T> wd = cmul(conjc(twk[u * R1 + r]), d1);
                Z = mkc(s1.x - wd.y, s1.y + wd.x);
            }
            v[u * R1 + r] = Z;
        }
    }
    __syncthreads();
    fft_run<T, N, M, +1, true, false>(v, lay, j, tab.tw);
    double acc[Epi::NACC > 0 ? Epi::NACC : 1];
#pragma unroll
    for (int a = 0; a < (Epi::NACC > 0 ? Epi::NACC : 1); ++a) acc[a] = 0.0;
    if constexpr (Epi::NACC > 4) acc[4] = 1.0e300;
    constexpr bool UPD = EpiUpd<Epi>::value;
    constexpr int NO = (E / RL) * RK;  // outputs (pairs) of this thread
    cx<T> qk[UPD ? NO : 1], rk[UPD ? NO : 1];
    static_assert(!FWD || UPD, "the fused forward pass follows the folded update");
    cx<T> pk[FWD ? NO : 1];  // FWD: p of the pairs, for the next direction and the x update
#pragma unroll
    for (int u = 0; u < E / RL; ++u)
#pragma unroll
        for (int r = 0; r < RK; ++r) {
            const int n = (j + u * P) + r * (N / RL);
            if constexpr (UPD) {
                // p and d prefetched with the spectrum (PF), or read here
                typename Epi::Pre pr;
                if constexpr (PF)
                    pr = pre[u * RK + r];
                else
                    pr = Epi::template pre<L>(sd, row, 2 * n);
                qk[u * RK + r] = Epi::template outq<L>(sd, row, 2 * n, v[u * RL + r].x, v[u * RL + r].y, pr, acc);
                if constexpr (FWD) pk[u * RK + r] = pr.p;
            } else if constexpr (Epi::PREF) {
                Epi::template out2p<L>(sd, row, 2 * n, v[u * RL + r].x, v[u * RL + r].y, pre[u * RK + r], acc);
            } else {
                Epi::template out2<L>(sd, row, 2 * n, v[u * RL + r].x, v[u * RL + r].y, acc);
            }
        }
    if constexpr (UPD) {
        // r of the same pairs, requested before the reduction and the barrier
        // so that its latency hides behind them
#pragma unroll
        for (int u = 0; u < E / RL; ++u)
#pragma unroll
            for (int r = 0; r < RK; ++r)
                rk[u * RK + r] = ld2<T>(reinterpret_cast<const T*>(sd.r) + (size_t)row * L + 2 * ((j + u * P) + r * (N / RL)));
    }
    if constexpr (Epi::NACC > 0 && !UPD) {
        double* part = sd.part;
        if constexpr (Epi::NACC == 1) {
            const double s = block_sum<NT>(acc[0], red);
            if (tid == 0) part[Epi::SET * stride + blockIdx.x] = s;
        } else {
            const int sets[8] = {PS_CHK_R,    PS_CHK_X,   PS_CHK_B,    PS_CHK_RW,
                                 PS_CHK_DMIN, PS_CHK_BAD, PS_CHK_DIFF, PS_CHK_DSUM};
            if constexpr (NT % 64 == 0) {
                // set 4 (min d) is a minimum, the others sums
                const double s = block_reduce_n<NT, 8, 1u << 4>(acc, red);
                if (tid < 8) part[sets[tid] * stride + blockIdx.x] = s;
            } else {
#pragma unroll
                for (int a = 0; a < 8; ++a) {
                    const double s = (a == 4) ? block_min<NT>(acc[a], red) : block_sum<NT>(acc[a], red);
                    if (tid == 0) part[sets[a] * stride + blockIdx.x] = s;
                }
            }
        }
    }
    if constexpr (UPD) {
        SolveState* st = sd.st;
        auto* pq_bits = reinterpret_cast<unsigned long long*>(sd.part + PS_PQ * stride);
        auto* bar_rel = reinterpret_cast<unsigned long long*>(sd.part + PS_BARREL * stride);
        const double s_pq = block_sum<NT>(acc[0], red);
        if (tid == 0) {
            // the partial is exchanged atomically and its completion awaited
            // (s_waitcnt 0) before the arrival is stored
            (void)__hip_atomic_exchange(pq_bits + blockIdx.x, __builtin_bit_cast(unsigned long long, s_pq),
                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_s_waitcnt(0);
        }
        auto* bar_flags = reinterpret_cast<unsigned long long*>(sd.part + PS_BAR * stride);
        // the grid was not resident as a whole: the solve is abandoned and
        // the host repeats it with the separate update kernel
        auto give_up = [&]() {
            if (tid == 0) {
                __hip_atomic_store(&st->status, ST_EGRID, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&st->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                publish_status(sd, 1, ST_EGRID, st->gen, st->iters, st->last_check_iter);
            }
        };
        if (!grid_barrier<NT>(bar_flags, bar_rel, token, st->bar_limit)) {
            give_up();
            return;
        }
        // every partial: strided per thread, then the block sum (the update
        // kernel's order when both reduce with the same thread count)
        double spq = 0.0;
        for (int i = tid; i < (int)gridDim.x; i += NT)
            spq += __builtin_bit_cast(double, __hip_atomic_load(pq_bits + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        const double pq = block_sum<NT>(spq, red);
        const double rho = st->rho_cur;
        if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rho)) {
            if (blockIdx.x == 0 && tid == 0) {
                st->status = ST_EBREAKDOWN;
                st->done = 1;
                publish_status(sd, 1, ST_EBREAKDOWN, st->gen, st->iters, st->last_check_iter);
            }
            return;
        }
        const double alpha = rho / pq;
        if (blockIdx.x == 0 && tid == 0) {
            st->alpha = alpha;
            st->rho_prev = rho;
            st->iters += 1;
            st->restart = 0;
        }
        const T a = (T)alpha;
        double rr = 0.0;
#pragma unroll
        for (int u = 0; u < E / RL; ++u)
#pragma unroll
            for (int r = 0; r < RK; ++r) {
                cx<T> rv = rk[u * RK + r];
                const cx<T> qv = qk[u * RK + r];
                rv.x -= a * qv.x;
                rv.y -= a * qv.y;
                st2<T>(reinterpret_cast<T*>(sd.r) + (size_t)row * L + 2 * ((j + u * P) + r * (N / RL)), rv);
                rr += (double)rv.x * rv.x + (double)rv.y * rv.y;
                if constexpr (FWD) rk[u * RK + r] = rv;
            }
        const double srr = block_sum<NT>(rr, red);
        if constexpr (!FWD) {
            if (tid == 0) sd.part[PS_RR * stride + blockIdx.x] = srr;
        } else {
            // The next iteration's forward row pass on the same rows, as
            // ProCG in k_row_fwd computes it: beta = r.r / rho from every
            // workgroup's r.r partial (a second barrier, token + 1; the same
            // summation order), the check decision, p <- r + beta p, the
            // transform, and the pending x update x <- x + alpha p_old.  The
            // forward pass's first radix equals this pass's last, so the
            // thread holds the same pairs of r and p in both.
            auto* rr_bits = reinterpret_cast<unsigned long long*>(sd.part + PS_RR * stride);
            if (tid == 0) {
                (void)__hip_atomic_exchange(rr_bits + blockIdx.x, __builtin_bit_cast(unsigned long long, srr),
                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_s_waitcnt(0);
            }
            if (!grid_barrier<NT>(bar_flags, bar_rel, token + 1, st->bar_limit)) {
                give_up();
                return;
            }
            double s2 = 0.0;
            for (int i = tid; i < (int)gridDim.x; i += NT)
                s2 += __builtin_bit_cast(double, __hip_atomic_load(rr_bits + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            const double rrn = block_sum<NT>(s2, red);
            if (check_due(st, rrn, s_iters + 1)) {
                if (blockIdx.x == 0 && tid == 0) st->pause = 1;
                return;
            }
            if (blockIdx.x == 0 && tid == 0) st->rho_cur = rrn;
            const T beta = (T)(rrn / rho);
            constexpr int R1 = NSTG > 0 ? fft_radix(N, false, 0) : 1;
            static_assert(R1 == RL, "forward first radix and inverse last radix");
            cx<T> v2[E];
#pragma unroll
            for (int u = 0; u < E / RL; ++u)
#pragma unroll
                for (int r = 0; r < RK; ++r) {
                    const cx<T> rv = rk[u * RK + r], po = pk[u * RK + r];
                    const cx<T> p2 = mkc(rv.x + beta * po.x, rv.y + beta * po.y);
                    st2<T>(reinterpret_cast<T*>(sd.p) + (size_t)row * L + 2 * ((j + u * P) + r * (N / RL)), p2);
                    v2[u * RL + r] = p2;
                }
            if (a != T(0)) {
                T* xa = reinterpret_cast<T*>(sizeof(T) == 8 ? (void*)sd.x : (void*)sd.e);
#pragma unroll
                for (int u = 0; u < E / RL; ++u)
#pragma unroll
                    for (int r = 0; r < RK; ++r) {
                        T* xp = xa + (size_t)row * L + 2 * ((j + u * P) + r * (N / RL));
                        cx<T> xv = ld2<T>(xp);
                        xv.x += a * pk[u * RK + r].x;
                        xv.y += a * pk[u * RK + r].y;
                        st2<T>(xp, xv);
                    }
            }
            // the forward transform reads its twiddles afresh (the pointer is
            // opaque to the compiler) rather than reusing the inverse half's
            // loads of the same entries across both barriers; the block
            // index is kept uniform
            Tab<T> tab2 = tab;
            asm volatile("" : "+s"(tab2.tw));
            row_fwd_out<T, M, PAD, NT>(v2, lds, tab2, sd, __builtin_amdgcn_readfirstlane(row0 / RPW));
        }
    }
}

template <typename T, int M, int PAD, class Epi, class Slot, int NT>
__global__ void __launch_bounds__(NT) k_row_inv(Tab<T> tab, Slot slot, int stride) {
    row_inv_body<T, M, PAD, Epi, Slot, NT>(tab, slot, stride, 0);
}

// The CG row-inverse pass with the residual update folded in (EpiCGU).
// token: unique per launch (the host counts launches per workspace), so
// arrival words left by an abandoned launch can never match a later one.
template <typename T, int M, int PAD, class Slot, int NT>
__global__ void __launch_bounds__(NT) k_row_inv_upd(Tab<T> tab, Slot slot, int stride, unsigned long long token) {
    row_inv_body<T, M, PAD, EpiCGU<T>, Slot, NT>(tab, slot, stride, token);
}

// One CG iteration's turn in one pass (k_row_inv_upd followed by k_row_fwd):
// q's row inverse, the folded update, and the next direction's forward row
// transform, with two grid-wide barriers (tokens token and token + 1).  Four
// waves per SIMD are asked for: the whole grid must be resident (four
// 256-thread workgroups per CU at M = 4096), which caps it at 128 VGPRs.
template <typename T, int M, int PAD, class Slot, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
k_row_turn(Tab<T> tab, Slot slot, int stride, unsigned long long token) {
    row_inv_body<T, M, PAD, EpiCGU<T>, Slot, NT, true>(tab, slot, stride, token);
}

// r <- r - alpha q, partial r . r.  alpha = rho / (p . q) from the partials
// of the row-inverse pass (all blocks reduce them in the same order).
template <typename W, int NT>
__global__ void __launch_bounds__(NT) k_update(ByPtr slot, int n, int npart_pq, int stride) {
    __shared__ double red[(NT + 63) / 64];
    const SlotDesc& sd = slot.get();
    if (!GateIter::ok(sd)) return;
    SolveState* st = sd.st;
    constexpr int VW = sizeof(W) == 4 ? 4 : 2;
    using V = typename VecT<W, VW>::type;
    const int nv = n / VW;
    const int per = (nv + gridDim.x - 1) / gridDim.x;
    const int lo = blockIdx.x * per;
    const int hi = lo + per < nv ? lo + per : nv;
    auto* r = gbl(reinterpret_cast<V*>(sd.r));
    const auto* q = gbl(reinterpret_cast<const V*>(sd.q));
    // the first PF vectors of r and q are requested before the p.q reduction
    // so its latency overlaps the HBM reads
    constexpr int PF = 4;
    V rp[PF], qp[PF];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        const int i = lo + threadIdx.x + u * NT;
        if (i < hi) {
            rp[u] = r[i];
            qp[u] = q[i];
        }
    }
    const double pq = sum_partials<NT>(sd.part + PS_PQ * stride, npart_pq, red);
    const double rho = st->rho_cur;
    if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rho)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->status = ST_EBREAKDOWN;
            st->done = 1;
            publish_status(sd, 1, ST_EBREAKDOWN, st->gen, st->iters, st->last_check_iter);
        }
        return;
    }
    const double alpha = rho / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->alpha = alpha;
        st->rho_prev = rho;
        st->iters += 1;
        st->restart = 0;
    }
    const W a = (W)alpha;
    double acc = 0.0;
    auto upd = [&](V rv, const V qv) {
        if constexpr (VW == 4) {
            rv.x -= a * qv.x;
            rv.y -= a * qv.y;
            rv.z -= a * qv.z;
            rv.w -= a * qv.w;
            acc += (double)rv.x * rv.x + (double)rv.y * rv.y + (double)rv.z * rv.z + (double)rv.w * rv.w;
        } else {
            rv.x -= a * qv.x;
            rv.y -= a * qv.y;
            acc += rv.x * rv.x + rv.y * rv.y;
        }
        return rv;
    };
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        const int i = lo + threadIdx.x + u * NT;
        if (i < hi) r[i] = upd(rp[u], qp[u]);
    }
    for (int i = lo + threadIdx.x + PF * NT; i < hi; i += NT) r[i] = upd(r[i], q[i]);
    const double s = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) sd.part[PS_RR * stride + blockIdx.x] = s;
}

// The first FP64 check of a solve started from x = 0: r = b - A 0 = b, so
// no product is needed.  One pass over b and d writes r and the check's
// partials (the same values the full check would produce, bitwise: C 0 and
// d 0 are exactly zero); the finaliser then decides as usual.  npart blocks.
template <typename W, int NT>
__global__ void __launch_bounds__(NT) k_check_zero(ByPtr slot, int n, int stride) {
    __shared__ double red[8 * ((NT + 63) / 64)];
    const SlotDesc& sd = slot.get();
    if (!GateCheck::ok(sd)) return;
    const int npairs = n / 2;
    const int per = (npairs + gridDim.x - 1) / gridDim.x;
    const int lo = blockIdx.x * per;
    const int hi = lo + per < npairs ? lo + per : npairs;
    double acc[8] = {0, 0, 0, 0, 1.0e300, 0, 0, 0};
    for (int q = lo + threadIdx.x; q < hi; q += NT) {
        const size_t idx = 2 * (size_t)q;
        const cx<double> b2 = ld2<double>(sd.b + idx), d2 = ld2<double>(sd.d + idx);
        const Mask2 mk = mask2(sd, idx);
        const double r0 = mk.m0 * b2.x, r1 = mk.m1 * b2.y;
        const W w0 = (W)r0, w1 = (W)r1;
        st2<W>(reinterpret_cast<W*>(sd.r) + idx, mkc(w0, w1));
        acc[0] += r0 * r0 + r1 * r1;
        acc[2] += r0 * r0 + r1 * r1;
        acc[3] += (double)w0 * (double)w0 + (double)w1 * (double)w1;
        acc[4] = fmin(acc[4], fmin(mk.m0 > 0.0 ? d2.x : 1.0e300, mk.m1 > 0.0 ? d2.y : 1.0e300));
        const bool ok = isfinite(r0) && isfinite(r1) && isfinite(d2.x) && isfinite(d2.y) && d2.x >= 0.0 &&
                        d2.y >= 0.0;
        acc[5] += ok ? 0.0 : 1.0;
        acc[7] += d2.x + d2.y;
    }
    const int sets[8] = {PS_CHK_R, PS_CHK_X, PS_CHK_B, PS_CHK_RW, PS_CHK_DMIN, PS_CHK_BAD, PS_CHK_DIFF, PS_CHK_DSUM};
    const double v = block_reduce_n<NT, 8, 1u << 4>(acc, red);  // set 4 (min d) a minimum
    if (threadIdx.x < 8) sd.part[sets[threadIdx.x] * stride + blockIdx.x] = v;
}

// Single-block finaliser of an FP64 check: stop decision, residual
// replacement, restart guard, and status for the host.
template <int NT>
__global__ void __launch_bounds__(NT) k_check_final(ByPtr slot, int npart_chk, int npart_rr, int stride, int n) {
    __shared__ double red[8 * ((NT + 63) / 64)];
    __shared__ double s_tot[8];
    __shared__ int s_update;
    const SlotDesc& sd = slot.get();
    if (!sd.active) return;
    SolveState* st = sd.st;
    if (st->done || !st->pause) {
        if (threadIdx.x == 0) publish_status(sd, st->done, st->status, st->gen, st->iters, st->last_check_iter);
        return;
    }
    // the eight partial sets, each summed (min d: minimised) by thread t over
    // t, t + NT, ... and then over the block, all in one exchange; the order
    // is that of sum_partials / block_min
    const int sets[8] = {PS_CHK_R, PS_CHK_X, PS_CHK_B, PS_CHK_RW, PS_CHK_DMIN, PS_CHK_BAD, PS_CHK_DIFF, PS_CHK_DSUM};
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 1.0e300, 0.0, 0.0, 0.0};
    const auto* part = gbl(sd.part);
    for (int i = threadIdx.x; i < npart_chk; i += NT) {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const double v = part[sets[a] * stride + i];
            acc[a] = (a == 4) ? fmin(acc[a], v) : acc[a] + v;
        }
    }
    const double tot = block_reduce_n<NT, 8, 1u << 4>(acc, red);
    if (threadIdx.x < 8) s_tot[threadIdx.x] = tot;
    __syncthreads();
    const double R = s_tot[0], X = s_tot[1], B = s_tot[2], RW = s_tot[3];
    const double dmin = s_tot[4], BAD = s_tot[5], DIFF = s_tot[6], DSUM = s_tot[7];
    if (threadIdx.x == 0) {
        if (st->checks == 0) st->dbar = DSUM / (double)n;
        s_update = check_decide(st, R, X, B, RW, BAD, DIFF, dmin);
        // preconditioned CG: z = P^{-1} r of the replaced residual comes next
        st->need_pre = (s_update && st->pcg) ? 1 : 0;
        publish_status(sd, st->done, st->status, st->gen, st->iters, st->last_check_iter);
    }
    __syncthreads();
    if (s_update) {
        // residual replacement: the next iteration's rho is |r|^2 of the new r
        double* prr = sd.part + PS_RR * stride;
        for (int i = threadIdx.x; i < npart_rr; i += NT) prr[i] = (i == 0) ? RW : 0.0;
    }
}


}  // namespace FFTCG_RADIX_NS
}  // namespace fftcg
