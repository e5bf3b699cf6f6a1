// Fused single-workgroup engine for small grids (M <= 64).
//
// One workgroup holds a whole solve: the operator product (Sec. 3, eq. (3):
// forward 2-D transform, multiply by the static spectrum, inverse transform,
// plus the element-wise term) runs on an M x M/2 complex buffer in LDS, and
// the CG loop of Listing 2 with its reductions runs in the same kernel, so an
// iteration costs no kernel launch.  Grids this small are latency bound; the
// engine trades arithmetic efficiency (radix-2 stages, one barrier each) for
// zero launches.  A launch runs up to a given number of iterations and
// leaves the state in device memory, so the server can interleave slots.
//
// Transforms are in place: forward ones are decimation in frequency (natural
// order in, bit-reversed out) and inverse ones decimation in time
// (bit-reversed in, natural out), so no bit-reversal pass exists; the
// multiply and the real-to-complex (un)packing index through bit reversal.
// The packing is that of the multi-pass engine: row v[2n] + i v[2n+1], column
// 0 carrying the k = 0 and k = M/2 columns in its real and imaginary parts.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <vector>

#include "common.hpp"
#include "fftcg_internal.hpp"
#include "fftcg_kernels.hpp"
#include "fused.hpp"

namespace fftcg {
namespace {

constexpr int FNT = 256;   // threads of a fused workgroup
constexpr int FUSED_MAX_M = 64;

struct FusedTabs {
    const cx<double>* tw64;  // exp(-2 pi i m / M), m < M
    const cx<float>* tw32;
    const double* gq64;      // ghat(m, k) / M^2, m, k in [0, M/2], row-major
    const float* gq32;
    int L, M, pad;
};

__device__ __forceinline__ int brevn(int k, int bits) {
    return bits == 0 ? 0 : (int)(__brev((unsigned)k) >> (32 - bits));
}

// count transforms of length n; element e of transform t at buf[t*ts + e*es]
template <typename T, int DIR>
__device__ void fft_dif(cx<T>* buf, int count, int n, int lg, int ts, int es, const cx<T>* tw, int M) {
    const int half = n >> 1;
    for (int lh = lg - 1; lh >= 0; --lh) {
        const int h = 1 << lh;
        const int tws = M >> (lh + 1);  // M / (2h)
        for (int t = threadIdx.x; t < count * half; t += FNT) {
            const int tr = t >> (lg - 1), bi = t & (half - 1);
            const int k = bi & (h - 1);
            const int i0 = ((bi >> lh) << (lh + 1)) + k;
            cx<T>* base = buf + tr * ts;
            const cx<T> a = base[i0 * es], c = base[(i0 + h) * es];
            cx<T> w = tw[k * tws];
            if (DIR > 0) w.y = -w.y;
            base[i0 * es] = a + c;
            base[(i0 + h) * es] = cmul(a - c, w);
        }
        __syncthreads();
    }
}

template <typename T, int DIR>
__device__ void fft_dit(cx<T>* buf, int count, int n, int lg, int ts, int es, const cx<T>* tw, int M) {
    const int half = n >> 1;
    for (int lh = 0; lh < lg; ++lh) {
        const int h = 1 << lh;
        const int tws = M >> (lh + 1);
        for (int t = threadIdx.x; t < count * half; t += FNT) {
            const int tr = t >> (lg - 1), bi = t & (half - 1);
            const int k = bi & (h - 1);
            const int i0 = ((bi >> lh) << (lh + 1)) + k;
            cx<T>* base = buf + tr * ts;
            cx<T> w = tw[k * tws];
            if (DIR > 0) w.y = -w.y;
            const cx<T> a = base[i0 * es], c = cmul(base[(i0 + h) * es], w);
            base[i0 * es] = a + c;
            base[(i0 + h) * es] = a - c;
        }
        __syncthreads();
    }
}

// out = d * v + C v for one slot.  ld(i, col) returns (v[i][col], v[i][col+1])
// as T; st(i, col, c0, c1) receives (C v)[i][col], (C v)[i][col+1].
template <typename T, class LD, class ST>
__device__ void fused_product(cx<T>* buf, const FusedTabs& ft, const cx<T>* tw, const T* gq, LD ld, ST st) {
    const int L = ft.L, M = ft.M, N = M / 2;
    const int lgN = 31 - __clz(N), lgM = 31 - __clz(M);
    const int ncols = ft.pad ? L / 2 : N;  // packed inputs per row that are nonzero
    // gather rows (rows >= L zero)
    for (int t = threadIdx.x; t < M * N; t += FNT) {
        const int i = t / N, n = t - i * N;
        buf[t] = (i < L && n < ncols) ? ld(i, 2 * n) : mkc(T(0), T(0));
    }
    __syncthreads();
    if (N > 1) fft_dif<T, -1>(buf, L, N, lgN, N, 1, tw, M);
    // real-to-complex unpack, in place on bit-reversed rows
    const int np = N / 2 + 1;
    for (int t = threadIdx.x; t < L * np; t += FNT) {
        const int i = t / np, k = t - i * np;
        cx<T>* row = buf + i * N;
        if (k == 0) {
            const cx<T> z = row[0];
            row[0] = mkc(z.x + z.y, z.x - z.y);
            continue;
        }
        const int pk = brevn(k, lgN), pn = brevn(N - k, lgN);
        const cx<T> A = row[pk], B = row[pn];
        {
            const cx<T> s1 = A + conjc(B), d1 = A - conjc(B);
            const cx<T> wd = cmul(tw[k], d1);
            row[pk] = mkc(T(0.5) * (s1.x + wd.y), T(0.5) * (s1.y - wd.x));
        }
        if (N - k != k) {
            const cx<T> s1 = B + conjc(A), d1 = B - conjc(A);
            const cx<T> wd = cmul(tw[N - k], d1);
            row[pn] = mkc(T(0.5) * (s1.x + wd.y), T(0.5) * (s1.y - wd.x));
        }
    }
    __syncthreads();
    // column transforms (length M; rows >= L are zero on the padded grid)
    fft_dif<T, -1>(buf, N, M, lgM, 1, N, tw, M);
    // multiply by ghat / M^2; packed column 0 pairs m with M - m
    const int MH = M / 2 + 1;
    for (int t = threadIdx.x; t < M * N; t += FNT) {
        const int p = t / N, c = t - p * N;
        if (c == 0) continue;
        const int m = brevn(p, lgM), k = brevn(c, lgN);
        const int mp = m <= M - m ? m : M - m;
        buf[t] = scalec(buf[t], gq[mp * MH + k]);
    }
    for (int m = threadIdx.x; m <= M / 2; m += FNT) {
        const int m2 = (M - m) & (M - 1);
        const int pa = brevn(m, lgM), pb = brevn(m2, lgM);
        const T ga = gq[m * MH], gNa = gq[m * MH + N];
        const cx<T> a = buf[pa * N], b = buf[pb * N];
        const T s = T(0.5) * (ga + gNa), tt = T(0.5) * (ga - gNa);  // ghat even: same for m and M - m
        buf[pa * N] = mkc(s * a.x + tt * b.x, s * a.y - tt * b.y);
        if (pb != pa) buf[pb * N] = mkc(s * b.x + tt * a.x, s * b.y - tt * a.y);
    }
    __syncthreads();
    fft_dit<T, +1>(buf, N, M, lgM, 1, N, tw, M);
    // complex-to-real pack on rows < L, in place: columns are still at
    // bit-reversed positions (Y[k] at brev(k)), which is the input order of
    // the inverse row transform; pairs (k, N - k) go to one thread
    for (int t = threadIdx.x; t < L * np; t += FNT) {
        const int i = t / np, k = t - i * np;
        cx<T>* row = buf + i * N;
        if (k == 0) {
            const cx<T> y = row[0];
            row[0] = mkc(y.x + y.y, y.x - y.y);
            continue;
        }
        const int pk = brevn(k, lgN), pn = brevn(N - k, lgN);
        const cx<T> A = row[pk], B = row[pn];
        {
            const cx<T> s1 = A + conjc(B), d1 = A - conjc(B);
            const cx<T> wd = cmul(conjc(tw[k]), d1);
            row[pk] = mkc(s1.x - wd.y, s1.y + wd.x);
        }
        if (N - k != k) {
            const cx<T> s1 = B + conjc(A), d1 = B - conjc(A);
            const cx<T> wd = cmul(conjc(tw[N - k]), d1);
            row[pn] = mkc(s1.x - wd.y, s1.y + wd.x);
        }
    }
    __syncthreads();
    if (N > 1) fft_dit<T, +1>(buf, L, N, lgN, N, 1, tw, M);
    for (int t = threadIdx.x; t < L * ncols; t += FNT) {
        const int i = t / ncols, n = t - i * ncols;
        const cx<T> z = buf[i * N + n];
        st(i, 2 * n, z.x, z.y);
    }
    __syncthreads();
}

template <int NT>
__device__ __forceinline__ double bsum(double v, double* red) { return block_sum<NT>(v, red); }

// One slot per workgroup; runs until done or `max_iters` iterations in this
// launch.  W = working precision of the inner iterations.
template <typename W>
__global__ void __launch_bounds__(FNT) k_fused_solve(FusedTabs ft, const SlotDesc* __restrict__ slots, int max_iters) {
    extern __shared__ double dyn[];
    __shared__ double red[FNT / 64];
    __shared__ SolveState st;
    __shared__ double s_rr;
    __shared__ int s_flag;
    const SlotDesc& sd = slots[blockIdx.x];
    if (!sd.active) return;
    if (threadIdx.x == 0) st = *sd.st;
    __syncthreads();
    if (st.done) {
        if (threadIdx.x == 0) publish_status(sd, st.done, st.status, st.gen, st.iters);
        return;
    }
    const int L = ft.L, n = L * L;
    double* x = sd.x;
    const double* b = sd.b;
    const double* d = sd.d;
    W* r = reinterpret_cast<W*>(sd.r);
    W* p = reinterpret_cast<W*>(sd.p);
    W* q = reinterpret_cast<W*>(sd.q);
    float* e = sd.e;
    const bool mixed = st.mixed != 0;
    // r.r of the current residual: after a check it is the replaced one;
    // otherwise the last update produced it (kept in the state between launches)
    double rr = st.rho_cur;
    int done_here = 0;
    for (;;) {
        if (st.pause) {
            // ---- FP64 check: flush pending updates, r64 = b - A x ----
            const double alpha = st.alpha;
            for (int i = threadIdx.x; i < n; i += FNT) {
                double xv = x[i];
                if (mixed) {
                    xv += (double)e[i];
                    e[i] = 0.0f;
                }
                if (alpha != 0.0) xv += alpha * (double)p[i];
                x[i] = xv;
            }
            __syncthreads();
            double acc[7] = {0, 0, 0, 0, 1.0e300, 0, 0};
            const int first = st.checks == 0;
            cx<double>* buf = reinterpret_cast<cx<double>*>(dyn);
            fused_product<double>(
                buf, ft, ft.tw64, ft.gq64,
                [&](int i, int c) { return mkc(x[i * L + c], x[i * L + c + 1]); },
                [&](int i, int c, double c0, double c1) {
                    const int idx = i * L + c;
                    const double cv[2] = {c0, c1};
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const double xv = x[idx + h], bv = b[idx + h], dv = d[idx + h];
                        const double rv = bv - (dv * xv + cv[h]);
                        const W w = (W)rv;
                        if (!first) {
                            const double df = rv - (double)r[idx + h];
                            acc[6] += df * df;
                        }
                        r[idx + h] = w;
                        acc[0] += rv * rv;
                        acc[1] += xv * xv;
                        acc[2] += bv * bv;
                        acc[3] += (double)w * (double)w;
                        acc[4] = fmin(acc[4], dv);
                        acc[5] += (isfinite(bv) && isfinite(dv) && dv >= 0.0) ? 0.0 : 1.0;
                    }
                });
            double R = bsum<FNT>(acc[0], red), X = bsum<FNT>(acc[1], red), B = bsum<FNT>(acc[2], red);
            double RW = bsum<FNT>(acc[3], red), BAD = bsum<FNT>(acc[5], red), DIFF = bsum<FNT>(acc[6], red);
            double dmin = block_min<FNT>(acc[4], red);
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
        __syncthreads();
        if (threadIdx.x == 0) st.rho_cur = rr;
        for (int i = threadIdx.x; i < n; i += FNT) {
            const W rv = r[i];
            if (restart) {
                p[i] = rv;
            } else {
                const W po = p[i];
                if (alpha_old != 0.0) {
                    if (mixed)
                        e[i] += (float)alpha_old * (float)po;
                    else
                        x[i] += alpha_old * (double)po;
                }
                p[i] = rv + (W)beta * po;
            }
        }
        __syncthreads();
        double pqa = 0.0;
        cx<W>* bufw = reinterpret_cast<cx<W>*>(dyn);
        const cx<W>* tww = reinterpret_cast<const cx<W>*>(sizeof(W) == 8 ? (const void*)ft.tw64 : (const void*)ft.tw32);
        const W* gqw = reinterpret_cast<const W*>(sizeof(W) == 8 ? (const void*)ft.gq64 : (const void*)ft.gq32);
        fused_product<W>(
            bufw, ft, tww, gqw, [&](int i, int c) { return mkc(p[i * L + c], p[i * L + c + 1]); },
            [&](int i, int c, W c0, W c1) {
                const int idx = i * L + c;
                const W cv[2] = {c0, c1};
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const W pv = p[idx + h];
                    const W qv = (W)d[idx + h] * pv + cv[h];
                    q[idx + h] = qv;
                    pqa += (double)pv * (double)qv;
                }
            });
        const double pq = bsum<FNT>(pqa, red);
        if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rr)) {
            if (threadIdx.x == 0) {
                st.status = ST_EBREAKDOWN;
                st.done = 1;
            }
            __syncthreads();
            break;
        }
        const double alpha = rr / pq;
        double acc = 0.0;
        for (int i = threadIdx.x; i < n; i += FNT) {
            const W rv = r[i] - (W)alpha * q[i];
            r[i] = rv;
            acc += (double)rv * (double)rv;
        }
        const double rr_new = bsum<FNT>(acc, red);
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
        publish_status(sd, st.done, st.status, st.gen, st.iters);
    }
}

template <typename T>
__global__ void __launch_bounds__(FNT) k_fused_apply(FusedTabs ft, const double* d, const double* x, double* y) {
    extern __shared__ double dyn[];
    const int L = ft.L;
    cx<T>* buf = reinterpret_cast<cx<T>*>(dyn);
    const cx<T>* tw = reinterpret_cast<const cx<T>*>(sizeof(T) == 8 ? (const void*)ft.tw64 : (const void*)ft.tw32);
    const T* gq = reinterpret_cast<const T*>(sizeof(T) == 8 ? (const void*)ft.gq64 : (const void*)ft.gq32);
    fused_product<T>(
        buf, ft, tw, gq, [&](int i, int c) { return mkc((T)x[i * L + c], (T)x[i * L + c + 1]); },
        [&](int i, int c, T c0, T c1) {
            const int idx = i * L + c;
            y[idx] = d[idx] * x[idx] + (double)c0;
            y[idx + 1] = d[idx + 1] * x[idx + 1] + (double)c1;
        });
}

FusedTabs tabs_of(const fftcg_plan_s* p) {
    const void* const* t = reinterpret_cast<const void* const*>(p->f_tab64);
    (void)t;
    FusedTabs ft;
    const char* b64 = (const char*)p->f_tab64;
    const char* b32 = (const char*)p->f_tab32;
    const int M = p->M, MH = M / 2 + 1;
    ft.tw64 = (const cx<double>*)b64;
    ft.gq64 = (const double*)(b64 + sizeof(double) * 2 * M);
    ft.tw32 = (const cx<float>*)b32;
    ft.gq32 = (const float*)(b32 + sizeof(float) * 2 * M);
    (void)MH;
    ft.L = p->L;
    ft.M = p->M;
    ft.pad = p->pad;
    return ft;
}

size_t fused_lds_bytes(const fftcg_plan_s* p) { return (size_t)p->M * (p->M / 2) * sizeof(cx<double>); }

}  // namespace

int fused_init(fftcg_plan_s* p, const double* g) {
    p->fused_ok = 0;
    p->fused_bytes = 0;
    if (p->M > FUSED_MAX_M) return FFTCG_OK;
    const int M = p->M, MH = M / 2 + 1;
    const double s = 1.0 / ((double)M * (double)M);
    std::vector<double> t64(2 * (size_t)M + (size_t)MH * MH);
    std::vector<float> t32(2 * (size_t)M + (size_t)MH * MH);
    for (int m = 0; m < M; ++m) {
        double c, sn;
        cos_sin_2pi(m, M, &c, &sn);
        t64[2 * m] = c;
        t64[2 * m + 1] = -sn;
        t32[2 * m] = (float)c;
        t32[2 * m + 1] = (float)-sn;
    }
    for (int m = 0; m < MH; ++m)
        for (int k = 0; k < MH; ++k) {
            const double v = g[(size_t)m * M + k] * s;
            t64[2 * M + (size_t)m * MH + k] = v;
            t32[2 * M + (size_t)m * MH + k] = (float)v;
        }
    if (hipMalloc(&p->f_tab64, t64.size() * 8) != hipSuccess) return FFTCG_ENOMEM;
    if (hipMalloc(&p->f_tab32, t32.size() * 4) != hipSuccess) return FFTCG_ENOMEM;
    if (hipMemcpy(p->f_tab64, t64.data(), t64.size() * 8, hipMemcpyHostToDevice) != hipSuccess) return FFTCG_EDEVICE;
    if (hipMemcpy(p->f_tab32, t32.data(), t32.size() * 4, hipMemcpyHostToDevice) != hipSuccess) return FFTCG_EDEVICE;
    p->fused_bytes = t64.size() * 8 + t32.size() * 4;
    p->fused_ok = 1;
    return FFTCG_OK;
}

void fused_free(fftcg_plan_s* p) {
    if (p->f_tab64) (void)hipFree(p->f_tab64);
    if (p->f_tab32) (void)hipFree(p->f_tab32);
    p->f_tab64 = p->f_tab32 = nullptr;
}

int fused_apply(fftcg_plan_s* p, int precision, const double* d, const double* x, double* y, hipStream_t s) {
    if (!p->fused_ok) return FFTCG_EINVAL;
    const FusedTabs ft = tabs_of(p);
    const size_t lds = fused_lds_bytes(p);
    if (precision == FFTCG_FP64)
        hipLaunchKernelGGL(k_fused_apply<double>, dim3(1), dim3(FNT), lds, s, ft, d, x, y);
    else
        hipLaunchKernelGGL(k_fused_apply<float>, dim3(1), dim3(FNT), lds, s, ft, d, x, y);
    return hipGetLastError() == hipSuccess ? FFTCG_OK : FFTCG_EDEVICE;
}

void fused_launch(const fftcg_plan_s* p, int precision, const SlotDesc* slots, int nslots, int max_iters,
                  hipStream_t s) {
    const FusedTabs ft = tabs_of(p);
    const size_t lds = fused_lds_bytes(p);
    if (precision == FFTCG_FP64)
        hipLaunchKernelGGL(k_fused_solve<double>, dim3(nslots), dim3(FNT), lds, s, ft, slots, max_iters);
    else
        hipLaunchKernelGGL(k_fused_solve<float>, dim3(nslots), dim3(FNT), lds, s, ft, slots, max_iters);
}

int fused_solve(fftcg_plan_s* p, int precision, const double* d, const double* b, const double* x0, double tol,
                int maxit, double* x, fftcg_info* info, hipStream_t s) {
    if (!p->fused_ok) return FFTCG_EINVAL;
    Workspace* w = plan_acquire(p);
    if (!w) return FFTCG_ENOMEM;
    const size_t n = (size_t)p->L * p->L;
    int rc = FFTCG_OK;
    do {
        fill_slot(w->h_slot, w, x, b, d);
        w->h_slot->host_status = nullptr;
        init_state(w->h_state, p, precision, tol, maxit, 50);
        if (hipMemcpyAsync(w->slot, w->h_slot, sizeof(SlotDesc), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(w->st, w->h_state, sizeof(SolveState), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipEventRecord(w->ev0, s) != hipSuccess) {
            rc = FFTCG_EDEVICE;
            break;
        }
        hipError_t he = hipSuccess;
        if (!x0)
            he = hipMemsetAsync(x, 0, n * 8, s);
        else if (x0 != x)
            he = hipMemcpyAsync(x, x0, n * 8, hipMemcpyDeviceToDevice, s);
        if (he == hipSuccess && precision == FFTCG_MIXED) he = hipMemsetAsync(w->e, 0, n * 4, s);
        if (he != hipSuccess) {
            rc = FFTCG_EDEVICE;
            break;
        }
        fused_launch(p, precision, w->slot, 1, 1 << 30, s);
        if (hipGetLastError() != hipSuccess || hipEventRecord(w->ev1, s) != hipSuccess ||
            hipMemcpyAsync(w->h_state, w->st, sizeof(SolveState), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = FFTCG_EDEVICE;
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, w->ev0, w->ev1);
        const SolveState st = *w->h_state;
        if (st.bzero && (hipMemsetAsync(x, 0, n * 8, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)) {
            rc = FFTCG_EDEVICE;
            break;
        }
        rc = st.done ? st.status : FFTCG_EDEVICE;
        if (info) {
            info->status = rc;
            info->iterations = st.iters;
            info->iterations_literal = st.iters_literal;
            info->checks = st.checks;
            info->true_relres = st.true_relres;
            info->error_bound = st.bound;
            info->lambda_lb = st.lam_lb;
            info->device_ms = ms;
        }
    } while (0);
    plan_release(p, w);
    return rc;
}

}  // namespace fftcg
