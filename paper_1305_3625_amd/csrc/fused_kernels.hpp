// Fused single-workgroup engine: device code, compiled per grid size.
//
// One workgroup of FNT threads holds a whole solve.  The operator product
// (Sec. 3, eq. (3): forward 2-D transform, multiply by the static spectrum,
// inverse transform, plus the element-wise term) uses the register/LDS
// Stockham transforms of the multi-pass engine, one row or one column per
// group of threads:
//   rows     groups of N/E threads transform one packed row (length N = M/2)
//            each; the real-to-complex unpack reads its partners from LDS;
//   columns  groups of M/E threads transform one packed column (length M),
//            multiply by ghat / M^2 and transform back;
//   rows     the complex-to-real pack reads its partners straight from the
//            half spectrum, then the inverse row transform and the epilogue.
// The half spectrum W (L rows x N packed columns, column-major so a column is
// contiguous) stays in the slot's device buffer: at these sizes it lives in
// the CU's L1/L2, and the LDS holds only the exchange buffers of the rows or
// columns in flight (so several workgroups share a CU).  Phases are separated
// by workgroup barriers; all waves of a workgroup run on one CU, so the
// barrier's workgroup-scope fence orders the global W accesses.
//
// The CG loop of Listing 2 with its reductions runs in the same kernel (no
// launch per iteration); a launch runs up to max_iters iterations and leaves
// the state in device memory, so the server can interleave slots.
#pragma once
#include "fftcg_kernels.hpp"
#include "fused.hpp"

namespace fftcg {
inline namespace FFTCG_RADIX_NS {

constexpr int FNT = 256;  // threads of a fused workgroup

// The same pointer, opaque to the optimiser: table reads through it cannot be
// hoisted out of the round loops (the hoisted twiddles of every transform
// would otherwise stay live in registers across the whole kernel).
template <typename P>
__device__ __forceinline__ P* opaque(P* p) {
    asm volatile("" : "+s"(p));
    return p;
}
// A uniform loop index, likewise opaque: addresses derived from it are
// recomputed in every round instead of being strength-reduced into a set of
// pointers that stay live across the loop.
__device__ __forceinline__ int opaque_i(int v) {
    asm volatile("" : "+s"(v));
    return v;
}

template <typename T, int M, int PAD>
struct FGeo {
    static constexpr int L = PAD ? M / 2 : M;
    static constexpr int N = M / 2;  // packed row length = number of packed columns
    static constexpr int MH = M / 2 + 1;
    // rows: PR threads per row, RR row groups per round
    static constexpr int ER = fft_elems(N);
    static constexpr int PR = N / ER;
    static constexpr int RR = FNT / PR;
    static constexpr int RWORDS = LdsLay<T, 1, 4, 1>::words(N);
    static constexpr int ROUNDS_R = (L + RR - 1) / RR;
    // columns: PC threads per column, CR column groups per round
    static constexpr int EC = fft_elems(M);
    static constexpr int PC = M / EC;
    static constexpr int CR = FNT / PC;
    static constexpr int CWORDS = LdsLay<T, 1, 4, 1>::words(M);
    static constexpr int ROUNDS_C = (N + CR - 1) / CR;
    static constexpr int LDS_WORDS = cmax(RR * RWORDS, CR * CWORDS);
    static_assert(PR <= FNT && PC <= FNT, "one row and one column fit a workgroup");
};

// Forward row pass: row i of the input -> column-major half spectrum
// W[k L + i], k in [0, N); column 0 carries k = 0 and k = N in its real and
// imaginary parts.  The input pairs come in two steps: ldf(i, col) reads
// what a pair needs, ldc(raw, i, col) combines (and stores what the gather
// updates) and returns the pair.  All of a thread's reads come first: a
// store of one pair would otherwise hold up the reads of the next.
template <typename T, int M, int PAD, class LDF, class LDC>
__device__ __forceinline__ void fz_rows_fwd(cx<T>* lds, cx<T>* W, const cx<T>* __restrict__ tw, LDF ldf,
                                            LDC ldc) {
    using G = FGeo<T, M, PAD>;
    constexpr int N = G::N, E = G::ER, P = G::PR, L = G::L;
    constexpr int NSTG = fft_nstages(N);
    constexpr int R1 = NSTG > 0 ? fft_radix(N, false, 0) : 1;
    constexpr int RL = NSTG > 0 ? fft_radix(N, false, NSTG - 1) : 1;
    const int rl = threadIdx.x / P, j = threadIdx.x % P;
    LdsLay<T, 1, 4, 1> lay{lds + rl * G::RWORDS, 0};
#pragma unroll 1
    for (int rd = 0; rd < G::ROUNDS_R; ++rd) {
        const int row = opaque_i(rd) * G::RR + rl;
        const bool act = row < L;
        const cx<T>* twr = opaque(tw);
        cx<T>* Wr = opaque(W);
        cx<T> v[E];
        constexpr int RK = PAD ? R1 / 2 : R1;  // inputs per run (the rest are known zeros on the padded grid)
        if (act) {
            decltype(ldf(0, 0)) raw[(E / R1) * RK];
#pragma unroll
            for (int u = 0; u < E / R1; ++u)
#pragma unroll
                for (int r = 0; r < RK; ++r) raw[u * RK + r] = ldf(row, 2 * ((j + u * P) + r * (N / R1)));
#pragma unroll
            for (int u = 0; u < E / R1; ++u)
#pragma unroll
                for (int r = 0; r < RK; ++r)
                    v[u * R1 + r] = ldc(raw[u * RK + r], row, 2 * ((j + u * P) + r * (N / R1)));
        } else {
#pragma unroll
            for (int i = 0; i < E; ++i) v[i] = mkc(T(0), T(0));
        }
        fft_run<T, N, M, -1, false, PAD != 0>(v, lay, j, twr);
        if constexpr (NSTG > 1) __syncthreads();  // the transform's last reads before these writes
#pragma unroll
        for (int u = 0; u < E / RL; ++u) lay.template st_run<RL, N / RL>(j + u * P, v + u * RL);
        __syncthreads();
        if (act) {
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const int k = j + s * P;
                const cx<T> Zk = lay.ld(k);
                cx<T> out;
                if (k == 0) {
                    out = mkc(Zk.x + Zk.y, Zk.x - Zk.y);
                } else {
                    const cx<T> B = conjc(lay.ld(N - k));
                    const cx<T> s1 = Zk + B, d1 = Zk - B;
                    const cx<T> wd = cmul(gld(twr + k), d1);
                    out = mkc(T(0.5) * (s1.x + wd.y), T(0.5) * (s1.y - wd.x));
                }
                gst(Wr + k * L + row, out);
            }
        }
        __syncthreads();
    }
}

// Column pass in place on W: forward transform of length M (rows >= L are
// zero on the padded grid), multiply by ghat / M^2 (gq[m MH + k], m, k in
// [0, M/2]; ghat is even so m and M - m share a value), inverse transform,
// keep rows < L.  Packed column 0: result(m) = s(m) Y(m) + t(m) conj(Y(M-m)),
// s = (g(m,0) + g(m,N)) / 2, t = (g(m,0) - g(m,N)) / 2.
template <typename T, int M, int PAD>
__device__ __forceinline__ void fz_cols(cx<T>* lds, cx<T>* W, const cx<T>* __restrict__ tw,
                                        const T* __restrict__ gq) {
    using G = FGeo<T, M, PAD>;
    constexpr int E = G::EC, P = G::PC, L = G::L, N = G::N, MH = G::MH;
    constexpr int NSTG = fft_nstages(M);
    constexpr int R1 = fft_radix(M, false, 0);
    constexpr int RL = fft_radix(M, false, NSTG - 1);
    constexpr int RZ = fft_radix(M, true, NSTG - 1);
    const int cl = threadIdx.x / P, j = threadIdx.x % P;
    LdsLay<T, 1, 4, 1> lay{lds + cl * G::CWORDS, 0};
#pragma unroll 1
    for (int rd = 0; rd < G::ROUNDS_C; ++rd) {
        const int c = opaque_i(rd) * G::CR + cl;
        const bool act = c < N;
        cx<T>* Wc = opaque(W) + (act ? c : 0) * L;
        const cx<T>* twr = opaque(tw);
        const T* gqr = opaque(gq);
        cx<T> v[E];
#pragma unroll
        for (int u = 0; u < E / R1; ++u)
#pragma unroll
            for (int r = 0; r < R1; ++r) {
                if (PAD && r >= R1 / 2) continue;
                const int n = (j + u * P) + r * (M / R1);
                v[u * R1 + r] = act ? gld(Wc + n) : mkc(T(0), T(0));
            }
        fft_run<T, M, M, -1, false, PAD != 0>(v, lay, j, twr);
        const bool col0 = rd == 0 && cl == 0;
        if (rd == 0) {
            // column 0 needs Y(M - m) from other threads of its group
            if constexpr (NSTG > 1) __syncthreads();  // the transform's last reads before these writes
#pragma unroll
            for (int u = 0; u < E / RL; ++u) lay.template st_run<RL, M / RL>(j + u * P, v + u * RL);
            __syncthreads();
            if (col0) {
#pragma unroll
                for (int u = 0; u < E / RL; ++u)
#pragma unroll
                    for (int r = 0; r < RL; ++r) {
                        const int m = (j + u * P) + r * (M / RL);
                        const int mp = m <= M - m ? m : M - m;
                        const cx<T> a = v[u * RL + r];
                        const cx<T> bm = conjc(lay.ld((M - m) & (M - 1)));
                        const T g0 = *gbl(gqr + mp * MH), gN = *gbl(gqr + mp * MH + N);
                        const T s = T(0.5) * (g0 + gN), t = T(0.5) * (g0 - gN);
                        v[u * RL + r] = mkc(s * a.x + t * bm.x, s * a.y + t * bm.y);
                    }
            }
            __syncthreads();
        }
        if (act && !col0) {
#pragma unroll
            for (int u = 0; u < E / RL; ++u)
#pragma unroll
                for (int r = 0; r < RL; ++r) {
                    const int m = (j + u * P) + r * (M / RL);
                    const int mp = m <= M - m ? m : M - m;
                    v[u * RL + r] = scalec(v[u * RL + r], *gbl(gqr + mp * MH + c));
                }
        }
        // the forward transform's (or column 0's) reads of the buffer came before
        fft_run<T, M, M, +1, true, false, LdsLay<T, 1, 4, 1>, true>(v, lay, j, opaque(twr));
        if (act) {
#pragma unroll
            for (int u = 0; u < E / RZ; ++u)
#pragma unroll
                for (int r = 0; r < RZ; ++r) {
                    if (PAD && r >= RZ / 2) continue;
                    const int n = (j + u * P) + r * (M / RZ);
                    gst(Wc + n, v[u * RZ + r]);
                }
        }
        __syncthreads();
    }
}

// Inverse row pass: complex-to-real pack of row i of W (partners N - k read
// from W directly), inverse transform, and the epilogue with the
// convolution values c0, c1 at columns col, col + 1 (< L), again in two
// steps: stf(i, col) reads the operands, stc(raw, i, col, c0, c1) finishes.
template <typename T, int M, int PAD, class STF, class STC>
__device__ __forceinline__ void fz_rows_inv(cx<T>* lds, const cx<T>* W, const cx<T>* __restrict__ tw, STF stf,
                                            STC stc) {
    using G = FGeo<T, M, PAD>;
    constexpr int N = G::N, E = G::ER, P = G::PR, L = G::L;
    constexpr int NSTG = fft_nstages(N);
    constexpr int R1 = NSTG > 0 ? fft_radix(N, true, 0) : 1;
    constexpr int S1 = N / R1;
    constexpr int RL = NSTG > 0 ? fft_radix(N, true, NSTG - 1) : 1;
    const int rl = threadIdx.x / P, j = threadIdx.x % P;
    LdsLay<T, 1, 4, 1> lay{lds + rl * G::RWORDS, 0};
#pragma unroll 1
    for (int rd = 0; rd < G::ROUNDS_R; ++rd) {
        const int row = opaque_i(rd) * G::RR + rl;
        const bool act = row < L;
        const int ri = act ? row : 0;
        const cx<T>* twr = opaque(tw);
        const cx<T>* Wr = opaque(W);
        cx<T> v[E];
        // with up to 8 values per thread, the pairs, partners and twiddles
        // are all read before the first unpack (one wait instead of one per
        // value behind its branch); larger counts keep the registers
        constexpr bool HOIST = E <= 8;
        cx<T> Yh[HOIST ? E : 1], Bh[HOIST ? E : 1], Th[HOIST ? E : 1];
        if constexpr (HOIST) {
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int k = (j + (i / R1) * P) + (i % R1) * S1;
                Yh[i] = gld(Wr + k * L + ri);
                Bh[i] = gld(Wr + ((N - k) & (N - 1)) * L + ri);  // k = 0: unused
                Th[i] = gld(twr + k);
            }
        }
#pragma unroll
        for (int u = 0; u < E / R1; ++u)
#pragma unroll
            for (int r = 0; r < R1; ++r) {
                const int k = (j + u * P) + r * S1;
                const int i = u * R1 + r;
                const cx<T> Y = [&] {
                    if constexpr (HOIST) return Yh[i]; else return gld(Wr + k * L + ri);
                }();
                cx<T> Z;
                if (k == 0) {
                    Z = mkc(Y.x + Y.y, Y.x - Y.y);
                } else {
                    const cx<T> B = conjc([&] {
                        if constexpr (HOIST) return Bh[i]; else return gld(Wr + (N - k) * L + ri);
                    }());
                    const cx<T> Tk = [&] {
                        if constexpr (HOIST) return Th[i]; else return gld(twr + k);
                    }();
                    const cx<T> s1 = Y + B, d1 = Y - B;
                    const cx<T> wd = cmul(conjc(Tk), d1);
                    Z = mkc(s1.x - wd.y, s1.y + wd.x);
                }
                v[i] = Z;
            }
        fft_run<T, N, M, +1, true, false>(v, lay, j, opaque(twr));
        if (act) {
            constexpr int RK = (PAD && RL > 1) ? RL / 2 : RL;  // columns >= L are cropped
            decltype(stf(0, 0)) raw[(E / RL) * RK];
#pragma unroll
            for (int u = 0; u < E / RL; ++u)
#pragma unroll
                for (int r = 0; r < RK; ++r) raw[u * RK + r] = stf(row, 2 * ((j + u * P) + r * (N / RL)));
#pragma unroll
            for (int u = 0; u < E / RL; ++u)
#pragma unroll
                for (int r = 0; r < RK; ++r)
                    stc(raw[u * RK + r], row, 2 * ((j + u * P) + r * (N / RL)), v[u * RL + r].x,
                        v[u * RL + r].y);
        }
        __syncthreads();
    }
}

// C v (with the caller's gather and element-wise epilogue, each in two
// steps) for one slot.
template <typename T, int M, int PAD, class LDF, class LDC, class STF, class STC>
__device__ __forceinline__ void fz_product(cx<T>* lds, cx<T>* W, const cx<T>* tw, const T* gq, LDF ldf, LDC ldc,
                                           STF stf, STC stc) {
    fz_rows_fwd<T, M, PAD>(lds, W, tw, ldf, ldc);
    fz_cols<T, M, PAD>(lds, W, tw, gq);
    fz_rows_inv<T, M, PAD>(lds, W, tw, stf, stc);
}

// Operands read in the first step of the two-step gathers and epilogues.
template <typename Wp>
struct ChkIn {  // FP64 check gather: x, e, p
    cx<double> x, e;
    cx<Wp> p;
};
template <typename Wp>
struct ChkOut {  // FP64 check epilogue: x, b, d, the recursive r
    cx<double> x, b, d;
    cx<Wp> r;
};
template <typename Wp>
struct IterIn {  // iteration gather: r, p, and e (FP32) or x (FP64)
    cx<Wp> r, p;
    cx<Wp> xa;
};
template <typename Wp>
struct IterOut {  // iteration epilogue: p, d
    cx<Wp> p;
    cx<double> d;
};

template <int M, int PAD>
struct FLds {
    // the FP64 product (checks) needs the most exchange space
    static constexpr int BYTES = FGeo<double, M, PAD>::LDS_WORDS * (int)sizeof(cx<double>);
};

// One slot per workgroup; runs until done or `max_iters` iterations in this
// launch.  Wp = working precision of the inner iterations.
template <typename Wp, int M, int PAD>
__global__ void __launch_bounds__(FNT) k_fused_solve(FusedTabs ft, const SlotDesc* __restrict__ slots,
                                                     int max_iters) {
    constexpr int L = FGeo<double, M, PAD>::L;
    constexpr int n = L * L;
    __shared__ double lds_raw[FLds<M, PAD>::BYTES / 8];
    __shared__ double red[FNT / 64];
    __shared__ SolveState st;
    __shared__ double s_rr;
    __shared__ int s_flag;
    const SlotDesc& sd = slots[blockIdx.x];
    if (!sd.active) return;
    if (threadIdx.x == 0) st = *sd.st;
    __syncthreads();
    if (st.done) {
        if (threadIdx.x == 0) publish_status(sd, st.done, st.status, st.gen, st.iters, st.last_check_iter);
        return;
    }
    double* x = sd.x;
    const double* b = sd.b;
    const double* d = sd.d;
    Wp* r = reinterpret_cast<Wp*>(sd.r);
    Wp* p = reinterpret_cast<Wp*>(sd.p);
    Wp* q = reinterpret_cast<Wp*>(sd.q);
    float* e = sd.e;
    const bool mixed = st.mixed != 0;
    const cx<double>* tw64 = reinterpret_cast<const cx<double>*>(ft.tw64);
    const double* gq64 = reinterpret_cast<const double*>(ft.gq64);
    const cx<Wp>* tww = reinterpret_cast<const cx<Wp>*>(sizeof(Wp) == 8 ? ft.tw64 : ft.tw32);
    const Wp* gqw = reinterpret_cast<const Wp*>(sizeof(Wp) == 8 ? ft.gq64 : ft.gq32);
    // r.r of the current residual: after a check it is the replaced one;
    // otherwise the last update produced it (kept in the state between launches)
    double rr = st.rho_cur;
    int done_here = 0;
    for (;;) {
        if (st.pause) {
            // ---- FP64 check: flush pending updates (in the product's input
            // gather), r64 = b - A x ----
            const double alpha = st.alpha;
            double acc[7] = {0, 0, 0, 0, 1.0e300, 0, 0};
            const int first = st.checks == 0;
            fz_product<double, M, PAD>(
                reinterpret_cast<cx<double>*>(lds_raw), reinterpret_cast<cx<double>*>(sd.W), tw64, gq64,
                [&](int i, int c) {
                    // x, the correction e and p (every buffer of a slot exists)
                    const int idx = i * L + c;
                    return ChkIn<Wp>{ld2(x + idx), ld2f(e + idx), ld2(p + idx)};
                },
                [&](const ChkIn<Wp>& w, int i, int c) {
                    // x <- x + e + alpha p, e <- 0 (each pair is gathered once)
                    const int idx = i * L + c;
                    cx<double> xv = w.x;
                    if (mixed) {
                        xv = xv + w.e;
                        st2(e + idx, mkc(0.0f, 0.0f));
                    }
                    if (alpha != 0.0) {
                        xv.x += alpha * (double)w.p.x;
                        xv.y += alpha * (double)w.p.y;
                    }
                    st2(x + idx, xv);
                    return xv;
                },
                [&](int i, int c) {
                    const int idx = i * L + c;
                    return ChkOut<Wp>{ld2(x + idx), ld2(b + idx), ld2(d + idx), ld2(r + idx)};
                },
                [&](const ChkOut<Wp>& o, int i, int c, double c0, double c1) {
                    const int idx = i * L + c;
                    const cx<double> x2 = o.x, b2 = o.b, d2 = o.d;
                    const cx<Wp> ro = o.r;
                    const double xv[2] = {x2.x, x2.y}, bv[2] = {b2.x, b2.y}, dv[2] = {d2.x, d2.y};
                    const double cv[2] = {c0, c1}, rold[2] = {(double)ro.x, (double)ro.y};
                    Wp w[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const double rv = bv[h] - (dv[h] * xv[h] + cv[h]);
                        w[h] = (Wp)rv;
                        if (!first) {
                            const double df = rv - rold[h];
                            acc[6] += df * df;
                        }
                        acc[0] += rv * rv;
                        acc[1] += xv[h] * xv[h];
                        acc[2] += bv[h] * bv[h];
                        acc[3] += (double)w[h] * (double)w[h];
                        acc[4] = fmin(acc[4], dv[h]);
                        acc[5] += (isfinite(bv[h]) && isfinite(dv[h]) && dv[h] >= 0.0) ? 0.0 : 1.0;
                    }
                    st2(r + idx, mkc(w[0], w[1]));
                });
            const double R = block_sum<FNT>(acc[0], red), X = block_sum<FNT>(acc[1], red);
            const double B = block_sum<FNT>(acc[2], red), RW = block_sum<FNT>(acc[3], red);
            const double BAD = block_sum<FNT>(acc[5], red), DIFF = block_sum<FNT>(acc[6], red);
            const double dmin = block_min<FNT>(acc[4], red);
            if (threadIdx.x == 0) s_flag = check_decide(&st, R, X, B, RW, BAD, DIFF, dmin);
            __syncthreads();
            if (!s_flag) break;
            rr = RW;
        }
        if (done_here >= max_iters) break;
        // ---- one CG iteration ----
        if (check_due(&st, rr)) {
            __syncthreads();
            if (threadIdx.x == 0) st.pause = 1;
            __syncthreads();
            continue;
        }
        const int restart = st.restart;
        const double beta = restart ? 0.0 : rr / st.rho_prev;
        const double alpha_old = st.alpha;
        const Wp beta_w = (Wp)beta, alpha_w = (Wp)alpha_old;
        __syncthreads();
        if (threadIdx.x == 0) st.rho_cur = rr;
        double pqa = 0.0;
        fz_product<Wp, M, PAD>(
            reinterpret_cast<cx<Wp>*>(lds_raw), reinterpret_cast<cx<Wp>*>(sd.W), tww, gqw,
            [&](int i, int c) {
                // r, p and the pending x update's target: the FP32 correction
                // e when the iterations run in FP32, else x itself
                const int idx = i * L + c;
                IterIn<Wp> w;
                w.r = ld2(r + idx);
                w.p = ld2(p + idx);
                if constexpr (sizeof(Wp) == 4) {
                    w.xa = ld2(e + idx);
                } else {
                    w.xa = ld2(x + idx);
                }
                return w;
            },
            [&](const IterIn<Wp>& w, int i, int c) {
                // p <- r + beta p (p <- r on restart), with the pending
                // x += alpha p_old (FP64 x, or the FP32 correction e)
                const int idx = i * L + c;
                const cx<Wp> r2 = w.r;
                cx<Wp> p2 = r2;
                if (!restart) {
                    const cx<Wp> po = w.p;
                    p2 = mkc(r2.x + beta_w * po.x, r2.y + beta_w * po.y);
                    if (alpha_old != 0.0) {
                        if constexpr (sizeof(Wp) == 4) {
                            cx<float> ev = w.xa;
                            ev.x += (float)alpha_w * (float)po.x;
                            ev.y += (float)alpha_w * (float)po.y;
                            st2(e + idx, ev);
                        } else {
                            cx<double> xv = w.xa;
                            xv.x += alpha_old * (double)po.x;
                            xv.y += alpha_old * (double)po.y;
                            st2(x + idx, xv);
                        }
                    }
                }
                st2(p + idx, p2);
                return p2;
            },
            [&](int i, int c) {
                const int idx = i * L + c;
                return IterOut<Wp>{ld2(p + idx), ld2(d + idx)};
            },
            [&](const IterOut<Wp>& w, int i, int c, Wp c0, Wp c1) {
                const int idx = i * L + c;
                const cx<Wp> pv = w.p;
                const cx<double> dv = w.d;
                const cx<Wp> qv = mkc((Wp)dv.x * pv.x + c0, (Wp)dv.y * pv.y + c1);
                st2(q + idx, qv);
                pqa += (double)pv.x * (double)qv.x + (double)pv.y * (double)qv.y;
            });
        const double pq = block_sum<FNT>(pqa, red);
        if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rr)) {
            if (threadIdx.x == 0) {
                st.status = ST_EBREAKDOWN;
                st.done = 1;
            }
            __syncthreads();
            break;
        }
        const double alpha = rr / pq;
        const Wp aw = (Wp)alpha;
        double acc = 0.0;
        // the pairs of r and q this thread updates are read in one go (up to 8)
        constexpr int UNR = cmax(1, cmin(8, n / (2 * FNT)));
#pragma unroll 1
        for (int i0 = 2 * threadIdx.x; i0 < n; i0 += 2 * FNT * UNR) {
            cx<Wp> rv[UNR], qv[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int i = i0 + 2 * FNT * u;
                if (i < n) {
                    rv[u] = ld2(r + i);
                    qv[u] = ld2(q + i);
                }
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int i = i0 + 2 * FNT * u;
                if (i < n) {
                    const cx<Wp> w = mkc(rv[u].x - aw * qv[u].x, rv[u].y - aw * qv[u].y);
                    st2(r + i, w);
                    acc += (double)w.x * (double)w.x + (double)w.y * (double)w.y;
                }
            }
        }
        const double rr_new = block_sum<FNT>(acc, red);
        if (threadIdx.x == 0) {
            st.alpha = alpha;
            st.rho_prev = rr;
            st.iters += 1;
            st.restart = 0;
            s_rr = rr_new;
        }
        __syncthreads();
        rr = s_rr;
        done_here += 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st.rho_cur = rr;  // carried to the next launch
        *sd.st = st;
        publish_status(sd, st.done, st.status, st.gen, st.iters, st.last_check_iter);
    }
}

// y = d x + C x for one grid (one workgroup), C in precision T.
template <typename T, int M, int PAD>
__global__ void __launch_bounds__(FNT) k_fused_apply(FusedTabs ft, const double* __restrict__ d,
                                                     const double* __restrict__ x, double* __restrict__ y,
                                                     void* Wbuf) {
    constexpr int L = FGeo<T, M, PAD>::L;
    __shared__ cx<T> lds[FGeo<T, M, PAD>::LDS_WORDS];
    const cx<T>* tw = reinterpret_cast<const cx<T>*>(sizeof(T) == 8 ? ft.tw64 : ft.tw32);
    const T* gq = reinterpret_cast<const T*>(sizeof(T) == 8 ? ft.gq64 : ft.gq32);
    fz_product<T, M, PAD>(
        lds, reinterpret_cast<cx<T>*>(Wbuf), tw, gq, [&](int i, int c) { return ld2(x + i * L + c); },
        [&](const cx<double>& v, int, int) { return mkc((T)v.x, (T)v.y); },
        [&](int i, int c) {
            const int idx = i * L + c;
            return ChkIn<double>{ld2(d + idx), ld2(x + idx), mkc(0.0, 0.0)};  // d, x
        },
        [&](const ChkIn<double>& w, int i, int c, T c0, T c1) {
            const cx<double> dv = w.x, xv = w.e;
            st2(y + i * L + c, mkc(dv.x * xv.x + (double)c0, dv.y * xv.y + (double)c1));
        });
}

}  // namespace FFTCG_RADIX_NS
}  // namespace fftcg
