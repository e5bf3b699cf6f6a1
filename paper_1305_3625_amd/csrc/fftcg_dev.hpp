// Device building blocks of the FFT engine for gfx950 (wave64).
//
// * cx<T>        complex value in registers (T = float or double).
// * dft<R,DIR>   radix-R DFT (R = 1, 2, 4, 8, 16) on R registers: radix 16
//                as 4 x 4 with the inner twiddles' scales folded into FMAs,
//                smaller radices as radix-2 decimation-in-frequency layers
//                with compile-time twiddles; HALF_IN skips the upper half of
//                the inputs (known zeros).
// * stages<...>  Stockham self-sorting FFT of length N held by N/E threads of
//                E = min(N, 16) values each.  Butterfly b of a radix-R stage
//                reads positions b + r N/R and writes
//                (b / Ns) Ns R + b % Ns + r Ns, so the output is in natural
//                order and no bit-reversal pass exists.  Between stages the
//                values go through LDS with a padded layout.
// * block reductions with a fixed summation order (wave shuffle tree, then
//   wave partials summed in index order), so every run gives bitwise the
//   same scalars.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Largest radix of a stage (16, 8 or 4).  It is a per-translation-unit
// choice (the fused engine takes 4 or 8 on the smallest grids), so every
// definition that depends on it lives in an inline namespace named after it
// and units built with different radices never share a symbol.
#ifndef FFTCG_MAXR
#define FFTCG_MAXR 16
#endif
#define FFTCG_RNS_CAT2(a, b) a##b
#define FFTCG_RNS_CAT(a, b) FFTCG_RNS_CAT2(a, b)
#define FFTCG_RADIX_NS FFTCG_RNS_CAT(radix, FFTCG_MAXR)

namespace fftcg {
inline namespace FFTCG_RADIX_NS {

template <typename T>
struct cx {
    T x, y;
};

// Pointers into device memory (HBM) reached through the slot table are
// generic pointers to the compiler; in the global address space its loads
// and stores are global_* instructions, which count only in vmcnt and so do
// not hold up LDS traffic the way flat_* instructions do.
template <typename T>
struct GlobalT {
    typedef __attribute__((address_space(1))) T type;
};
template <typename T>
__device__ __forceinline__ typename GlobalT<T>::type* gbl(T* p) {
    return (typename GlobalT<T>::type*)p;
}
// Plain vector types (no constructors), loadable through such pointers.
template <typename T, int K>
struct VecT {
    typedef T type __attribute__((ext_vector_type(K)));
};
template <typename T>
__device__ __forceinline__ cx<T> gld(const cx<T>* p) {
    const auto v = *gbl(reinterpret_cast<const typename VecT<T, 2>::type*>(p));
    cx<T> c;
    c.x = v.x;
    c.y = v.y;
    return c;
}
template <typename T>
__device__ __forceinline__ void gst(cx<T>* p, cx<T> c) {
    typename VecT<T, 2>::type v;
    v.x = c.x;
    v.y = c.y;
    *gbl(reinterpret_cast<typename VecT<T, 2>::type*>(p)) = v;
}

template <typename T>
__device__ __forceinline__ cx<T> mkc(T a, T b) {
    cx<T> r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mkc(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mkc(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return mkc(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cx<T> conjc(cx<T> a) { return mkc(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ cx<T> scalec(cx<T> a, T s) { return mkc(a.x * s, a.y * s); }

// a * exp(DIR * 2 pi i * k / 16); folds to a few adds for constant k.
template <typename T, int DIR>
__device__ __forceinline__ cx<T> rot16(cx<T> a, int k) {
    const T c1 = T(0.92387953251128675613);  // cos(pi/8)
    const T c2 = T(0.70710678118654752440);  // cos(pi/4)
    const T c3 = T(0.38268343236508977173);  // cos(3pi/8)
    const T d = T(DIR);
    switch (k & 15) {
        case 0: return a;
        case 4: return DIR > 0 ? mkc(-a.y, a.x) : mkc(a.y, -a.x);
        case 8: return mkc(-a.x, -a.y);
        case 12: return DIR > 0 ? mkc(a.y, -a.x) : mkc(-a.y, a.x);
        case 2: return mkc(c2 * (a.x - d * a.y), c2 * (d * a.x + a.y));
        case 6: return mkc(c2 * (-a.x - d * a.y), c2 * (d * a.x - a.y));
        case 10: return mkc(c2 * (-a.x + d * a.y), c2 * (-d * a.x - a.y));
        case 14: return mkc(c2 * (a.x + d * a.y), c2 * (-d * a.x + a.y));
        default: break;
    }
    T c, s;
    switch (k & 15) {
        case 1: c = c1; s = c3; break;
        case 3: c = c3; s = c1; break;
        case 5: c = -c3; s = c1; break;
        case 7: c = -c1; s = c3; break;
        case 9: c = -c1; s = -c3; break;
        case 11: c = -c3; s = -c1; break;
        case 13: c = c3; s = -c1; break;
        default: c = c1; s = -c3; break;  // 15
    }
    s = d * s;
    return mkc(a.x * c - a.y * s, a.x * s + a.y * c);
}

__host__ __device__ constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n >> 1); }
__host__ __device__ constexpr int brev(int i, int bits) {
    return bits == 0 ? 0 : (((i & 1) << (bits - 1)) | brev(i >> 1, bits - 1));
}

// Fused multiply-add in the precision of its operands (one rounding).
__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

// a * (DIR i)
template <typename T, int DIR>
__device__ __forceinline__ cx<T> muli(cx<T> a) {
    return DIR > 0 ? mkc(-a.y, a.x) : mkc(a.y, -a.x);
}

// Radix-4 DFT of x0 + s1 u1, x2, s1 u3 (HALF: x2 = u3 = 0; NEG3: the third
// input is -s1 u3), Y[k] = sum_n x_n (DIR i)^(n k), written to y[0..3].
// s1 scales the odd inputs and is folded into the output FMAs; p0 = x0 + x2
// and q0 = x0 - x2 come from the caller (who may fold a scale of x2 there).
template <typename T, int DIR, bool NEG3>
__device__ __forceinline__ void r4_tail(cx<T> p0, cx<T> q0, cx<T> u1, cx<T> u3, T s1, cx<T>* y0, cx<T>* y1,
                                        cx<T>* y2, cx<T>* y3) {
    // r = s1 (u1 +- u3), q = s1 (u1 -+ u3)
    const cx<T> r = NEG3 ? u1 - u3 : u1 + u3;
    const cx<T> q = NEG3 ? u1 + u3 : u1 - u3;
    const T d = T(DIR);
    *y0 = mkc(fmat(s1, r.x, p0.x), fmat(s1, r.y, p0.y));
    *y2 = mkc(fmat(-s1, r.x, p0.x), fmat(-s1, r.y, p0.y));
    // y1 = q0 + (DIR i) s1 q, y3 = q0 - (DIR i) s1 q
    *y1 = mkc(fmat(-d * s1, q.y, q0.x), fmat(d * s1, q.x, q0.y));
    *y3 = mkc(fmat(d * s1, q.y, q0.x), fmat(-d * s1, q.x, q0.y));
}

// Radix-16 DFT as 4 x 4 (index r = n1 + 4 n2, k = k1 + 4 k2):
//   A[n1][k1] = radix-4 over n2 of v[n1 + 4 n2],
//   B[n1][k1] = A[n1][k1] w^(n1 k1),  w = exp(DIR 2 pi i / 16),
//   X[k1 + 4 k2] = radix-4 over n1 of B[n1][k1].
// Every nontrivial w^e is a real scale times a two-operation rotation:
//   w^1 = c8 (1 + t8 Di), w^3 = c8 (t8 + Di), w^9 = -w^1,
//   w^2 = c2 (1 + Di), w^6 = c2 (-1 + Di), w^4 = Di  (Di = DIR i),
// c8 = cos(pi/8), t8 = tan(pi/8), c2 = cos(pi/4); the scales of one column
// k1 are folded into the FMAs of its second radix-4, so a butterfly costs 144
// real operations (112 with the upper half of the inputs zero).
template <typename T, int DIR, bool HALF_IN>
__device__ __forceinline__ void dft16(cx<T>* v) {
    const T c8 = T(0.92387953251128675613);  // cos(pi/8)
    const T t8 = T(0.41421356237309504880);  // tan(pi/8)
    const T c2 = T(0.70710678118654752440);  // cos(pi/4)
    const T d = T(DIR);
    cx<T> A[4][4];
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) {
        const cx<T> x0 = v[n1], x1 = v[n1 + 4];
        if constexpr (HALF_IN) {
            const cx<T> ix1 = muli<T, DIR>(x1);
            A[n1][0] = x0 + x1;
            A[n1][2] = x0 - x1;
            A[n1][1] = x0 + ix1;
            A[n1][3] = x0 - ix1;
        } else {
            const cx<T> x2 = v[n1 + 8], x3 = v[n1 + 12];
            const cx<T> p = x0 + x2, q = x0 - x2, r = x1 + x3, s = muli<T, DIR>(x1 - x3);
            A[n1][0] = p + r;
            A[n1][2] = p - r;
            A[n1][1] = q + s;
            A[n1][3] = q - s;
        }
    }
    // unscaled rotations: U = B / scale
    auto rot1 = [&](cx<T> a) { return mkc(fmat(-d * t8, a.y, a.x), fmat(d * t8, a.x, a.y)); };  // w^1 / c8
    auto rot3 = [&](cx<T> a) { return mkc(fmat(t8, a.x, -d * a.y), fmat(t8, a.y, d * a.x)); };  // w^3 / c8
    auto rot2 = [&](cx<T> a) { return mkc(a.x - d * a.y, a.y + d * a.x); };                   // w^2 / c2
    auto rot6 = [&](cx<T> a) { return mkc(-a.x - d * a.y, -a.y + d * a.x); };                 // w^6 / c2
    // k1 = 0: no twiddles
    {
        const cx<T> p0 = A[0][0] + A[2][0], q0 = A[0][0] - A[2][0];
        r4_tail<T, DIR, false>(p0, q0, A[1][0], A[3][0], T(1), &v[0], &v[4], &v[8], &v[12]);
    }
    // k1 = 1: w^0, c8 rot1, c2 rot2, c8 rot3
    {
        const cx<T> u2 = rot2(A[2][1]);
        const cx<T> p0 = mkc(fmat(c2, u2.x, A[0][1].x), fmat(c2, u2.y, A[0][1].y));
        const cx<T> q0 = mkc(fmat(-c2, u2.x, A[0][1].x), fmat(-c2, u2.y, A[0][1].y));
        r4_tail<T, DIR, false>(p0, q0, rot1(A[1][1]), rot3(A[3][1]), c8, &v[1], &v[5], &v[9], &v[13]);
    }
    // k1 = 2: w^0, c2 rot2, w^4 = Di, c2 rot6
    {
        const cx<T> u2 = muli<T, DIR>(A[2][2]);
        const cx<T> p0 = A[0][2] + u2, q0 = A[0][2] - u2;
        r4_tail<T, DIR, false>(p0, q0, rot2(A[1][2]), rot6(A[3][2]), c2, &v[2], &v[6], &v[10], &v[14]);
    }
    // k1 = 3: w^0, c8 rot3, c2 rot6, -c8 rot1 (w^9 = -w^1)
    {
        const cx<T> u2 = rot6(A[2][3]);
        const cx<T> p0 = mkc(fmat(c2, u2.x, A[0][3].x), fmat(c2, u2.y, A[0][3].y));
        const cx<T> q0 = mkc(fmat(-c2, u2.x, A[0][3].x), fmat(-c2, u2.y, A[0][3].y));
        r4_tail<T, DIR, true>(p0, q0, rot3(A[1][3]), rot1(A[3][3]), c8, &v[3], &v[7], &v[11], &v[15]);
    }
}

// In-register radix-R DFT, X[k] = sum_r v[r] exp(DIR 2 pi i r k / R).
template <typename T, int R, int DIR, bool HALF_IN>
__device__ __forceinline__ void dft(cx<T>* v) {
    if constexpr (R == 1) {
        return;
    } else if constexpr (R == 16) {
        dft16<T, DIR, HALF_IN>(v);
    } else {
        cx<T> t[R];
#pragma unroll
        for (int i = 0; i < R; ++i) t[i] = v[i];
#pragma unroll
        for (int lh = ilog2c(R) - 1; lh >= 0; --lh) {
            const int h = 1 << lh;
#pragma unroll
            for (int g = 0; g < R; g += 2 * h) {
#pragma unroll
                for (int i = 0; i < h; ++i) {
                    const int k16 = i * (16 / (2 * h));
                    cx<T> a = t[g + i];
                    if (HALF_IN && h == R / 2) {
                        t[g + i] = a;
                        t[g + i + h] = rot16<T, DIR>(a, k16);
                    } else {
                        cx<T> b = t[g + i + h];
                        t[g + i] = a + b;
                        t[g + i + h] = rot16<T, DIR>(a - b, k16);
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < R; ++i) v[brev(i, ilog2c(R))] = t[i];
    }
}

// ---- radix plans ----------------------------------------------------------
// Forward order: MAXR, MAXR, ..., then the remainder radix.  Reversed order:
// remainder first.  Lengths below MAXR use one stage.  MAXR = 16 by default.
constexpr int MAXR = FFTCG_MAXR;
constexpr int LGMAXR = MAXR == 16 ? 4 : (MAXR == 8 ? 3 : 2);
__host__ __device__ constexpr int fft_elems(int N) { return N >= MAXR ? MAXR : N; }
__host__ __device__ constexpr int fft_nstages(int N) {
    return N <= 1 ? 0 : (N < MAXR ? 1 : ilog2c(N) / LGMAXR + (ilog2c(N) % LGMAXR ? 1 : 0));
}
__host__ __device__ constexpr int fft_radix(int N, bool rev, int s) {
    // stage s of the plan
    return N < MAXR ? N
                    : (ilog2c(N) % LGMAXR == 0
                           ? MAXR
                           : (rev ? (s == 0 ? (1 << (ilog2c(N) % LGMAXR)) : MAXR)
                                  : (s == fft_nstages(N) - 1 ? (1 << (ilog2c(N) % LGMAXR)) : MAXR)));
}
__host__ __device__ constexpr int fft_ns(int N, bool rev, int s) {
    return s == 0 ? 1 : fft_ns(N, rev, s - 1) * fft_radix(N, rev, s - 1);
}

// LDS layout: complex word w = pos * TT + col, stored at w + (w >> SH) * PADW,
// SH = log2(16 TT): PADW words of padding after every 16 positions, so the
// stride-R writes of the first stage do not all hit one bank.
//
// A run of R positions pos0 + r S has compile-time offsets from the first
// element whenever S is a multiple of 16 (the padding grows by S/16 spans
// per step) or the whole run stays inside one 16-position span (no padding
// in between): the accesses then use immediate LDS offsets.
template <typename T, int TT, int SH, int PADW>
struct LdsLay {
    static_assert((1 << SH) == 16 * TT, "padding span is 16 positions");
    cx<T>* base;
    int col;
    __device__ __forceinline__ int phys(int pos) const {
        int w = pos * TT + col;
        return w + (w >> SH) * PADW;
    }
    __device__ __forceinline__ void st(int pos, cx<T> v) const { base[phys(pos)] = v; }
    __device__ __forceinline__ cx<T> ld(int pos) const { return base[phys(pos)]; }
    static constexpr int words(int n) { return n * TT + ((n * TT) >> SH) * PADW + PADW; }
    // offset in words between run elements r and 0, when it is a constant
    template <int S, int R>
    static constexpr int run_step() {
        return S % 16 == 0 ? S * TT + (S / 16) * PADW : (S * R <= 16 ? S * TT : -1);
    }
    // v[r] -> position pos0 + r S, r < R (runs with S R <= 16 must start so
    // that they stay inside one span, as every caller's runs do)
    template <int R, int S>
    __device__ __forceinline__ void st_run(int pos0, const cx<T>* v) const {
        constexpr int D = run_step<S, R>();
        if constexpr (D >= 0) {
            cx<T>* p = base + phys(pos0);
#pragma unroll
            for (int r = 0; r < R; ++r) p[r * D] = v[r];
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) st(pos0 + r * S, v[r]);
        }
    }
    template <int R, int S>
    __device__ __forceinline__ void ld_run(int pos0, cx<T>* v) const {
        constexpr int D = run_step<S, R>();
        if constexpr (D >= 0) {
            const cx<T>* p = base + phys(pos0);
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = p[r * D];
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = ld(pos0 + r * S);
        }
    }
};

// Twiddles of one radix-R butterfly: v[r] *= w^(r m), r = 1..R-1, with
// w^m = tw[m] = exp(-2 pi i m / MTAB) (DIR = -1) or its conjugate (DIR = +1).
// Four table reads (w^m, w^2m, w^4m, w^8m: the bases); the other powers are
// products of at most three of them.  The bases of a stage are read before
// the LDS exchange that precedes it, so their latency hides behind it.
template <int R>
__host__ __device__ constexpr int tw_nb() {
    return R > 8 ? 4 : (R > 4 ? 3 : (R > 2 ? 2 : 1));
}
template <typename T, int R>
__device__ __forceinline__ void tw_load(cx<T>* pb, const cx<T>* __restrict__ tw, int m) {
    pb[0] = gld(tw + m);
    if constexpr (R > 2) pb[1] = gld(tw + 2 * m);
    if constexpr (R > 4) pb[2] = gld(tw + 4 * m);
    if constexpr (R > 8) pb[3] = gld(tw + 8 * m);
}
template <typename T, int R, int DIR>
__device__ __forceinline__ void tw_apply(cx<T>* v, const cx<T>* pb) {
    cx<T> p[16];
    p[1] = pb[0];
    if constexpr (R > 2) p[2] = pb[1];
    if constexpr (R > 4) p[4] = pb[2];
    if constexpr (R > 8) p[8] = pb[3];
    if constexpr (R > 3) p[3] = cmul(p[1], p[2]);
    if constexpr (R > 5) {
        p[5] = cmul(p[1], p[4]);
        p[6] = cmul(p[2], p[4]);
        p[7] = cmul(p[3], p[4]);
    }
    if constexpr (R > 9) {
#pragma unroll
        for (int r = 1; r < 8; ++r) p[8 + r] = cmul(p[r], p[8]);
    }
#pragma unroll
    for (int r = 1; r < R; ++r) {
        cx<T> w = p[r];
        if (DIR > 0) w.y = -w.y;
        v[r] = cmul(v[r], w);
    }
}

// Runs stages S.. of the length-N transform held by this thread (index j of
// N/E threads).  On entry v[u R + r] holds position (j + u P) + r N / R_S,
// and pre holds the twiddle bases of stage S (if it has twiddles).  On exit
// v[u R_last + r] holds position (j + u P) + r N / R_last.
// tw[m] = exp(-2 pi i m / MTAB); DIR = -1 forward, +1 inverse.
//
// Each exchange is a barrier, the writes, a barrier, the reads.  The first
// barrier keeps the writes from overtaking the reads of the previous
// exchange (or, with LEAD, of whatever the caller read from the buffer
// before); it sits after the stage's arithmetic, so that waves which finished
// their reads compute while the others still read.  The last exchange's reads
// are therefore not fenced: a caller that writes the buffer after the
// transform places a barrier first.
template <typename T, int N, int MTAB, int DIR, bool REV, bool HALF_IN, int S, class Lay, bool LEAD>
__device__ __forceinline__ void stages(cx<T>* v, const Lay& lay, int j, const cx<T>* __restrict__ tw,
                                       const cx<T>* pre) {
    constexpr int E = fft_elems(N);
    constexpr int P = N / E;
    constexpr int R = fft_radix(N, REV, S);
    constexpr int NS = fft_ns(N, REV, S);
    constexpr int NB = E / R;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        if constexpr (NS > 1) tw_apply<T, R, DIR>(v + u * R, pre + u * tw_nb<R>());
        dft<T, R, DIR, HALF_IN && S == 0>(v + u * R);
    }
    if constexpr (S + 1 < fft_nstages(N)) {
        constexpr int R2 = fft_radix(N, REV, S + 1);
        constexpr int NS2 = fft_ns(N, REV, S + 1);
        constexpr int NB2 = E / R2;
        cx<T> nxt[NB2 * tw_nb<R2>()];
        if constexpr (NS2 > 1) {
            constexpr int STEP2 = MTAB / (NS2 * R2);
#pragma unroll
            for (int u = 0; u < NB2; ++u)
                tw_load<T, R2>(nxt + u * tw_nb<R2>(), tw, ((j + u * P) & (NS2 - 1)) * STEP2);
        }
        if constexpr (S > 0 || LEAD) __syncthreads();
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int b = j + u * P;
            const int base = (b / NS) * NS * R + (b & (NS - 1));
            lay.template st_run<R, NS>(base, v + u * R);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NB2; ++u) lay.template ld_run<R2, N / R2>(j + u * P, v + u * R2);
        stages<T, N, MTAB, DIR, REV, HALF_IN, S + 1, Lay, LEAD>(v, lay, j, tw, nxt);
    }
}

// Full transform (all stages).  Length 1 is the identity.  LEAD: the caller
// read the LDS buffer before (its reads are fenced before the first write).
// Returns with the last exchange's reads unfenced (see stages).
template <typename T, int N, int MTAB, int DIR, bool REV, bool HALF_IN, class Lay, bool LEAD = false>
__device__ __forceinline__ void fft_run(cx<T>* v, const Lay& lay, int j,
                                        const cx<T>* __restrict__ tw) {
    // stage 0 has no twiddles (NS = 1)
    if constexpr (fft_nstages(N) > 0)
        stages<T, N, MTAB, DIR, REV, HALF_IN, 0, Lay, LEAD>(v, lay, j, tw, nullptr);
}

// ---- reductions -----------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Sum over the block of NT threads; result valid in every thread.  sh must
// hold NT/64 doubles.  Fixed order: shuffle tree, then waves in index order.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    if constexpr (NT < 64) {
#pragma unroll
        for (int o = NT / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, NT);
        return v;
    }
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < (NT + 63) / 64; ++w) s += sh[w];
    return s;
}
template <int NT>
__device__ __forceinline__ double block_min(double v, double* sh) {
    if constexpr (NT < 64) {
#pragma unroll
        for (int o = NT / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, NT));
        return v;
    }
    v = wave_min(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = sh[0];
#pragma unroll
    for (int w = 1; w < (NT + 63) / 64; ++w) s = fmin(s, sh[w]);
    return s;
}

// N block reductions in one exchange: every wave reduces its N values with
// the shuffle tree, the wave results go to sh[a * NW + wave], and thread
// a < N combines set a over the waves in index order (a sum, or a min where
// bit a of MINMASK is set).  The order is that of block_sum / block_min, so
// the results are bitwise the same; two barriers instead of 2 N.  The
// result is valid in threads 0..N-1 (thread a holds set a).  sh must hold
// N * NW doubles, NW = NT / 64 (NT a multiple of 64).
template <int NT, int N, unsigned MINMASK>
__device__ __forceinline__ double block_reduce_n(const double* acc, double* sh) {
    static_assert(NT % 64 == 0, "whole waves");
    constexpr int NW = NT / 64;
    double w[N];
#pragma unroll
    for (int a = 0; a < N; ++a) w[a] = ((MINMASK >> a) & 1u) ? wave_min(acc[a]) : wave_sum(acc[a]);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int a = 0; a < N; ++a) sh[a * NW + (threadIdx.x >> 6)] = w[a];
    }
    __syncthreads();
    const int a = threadIdx.x;
    double r = 0.0;
    if (a < N) {
        if ((MINMASK >> a) & 1u) {
            r = sh[a * NW];
            for (int v = 1; v < NW; ++v) r = fmin(r, sh[a * NW + v]);
        } else {
            for (int v = 0; v < NW; ++v) r += sh[a * NW + v];
        }
    }
    return r;
}

// Sum of n partials in a fixed order (thread t takes t, t+NT, ...).
template <int NT>
__device__ __forceinline__ double sum_partials(const double* __restrict__ p, int n, double* sh) {
    double s = 0.0;
    const auto* g = gbl(p);
    for (int i = threadIdx.x; i < n; i += NT) s += g[i];
    return block_sum<NT>(s, sh);
}

}  // namespace FFTCG_RADIX_NS
}  // namespace fftcg
