// Instantiates the multi-pass engine for one grid; compiled once per
// (FFTCG_M, FFTCG_PAD) by the build script.
#include <string.h>

#include <hip/hip_ext.h>

#include "engine.hpp"
#include "fftcg_kernels.hpp"

#ifndef FFTCG_M
#error "FFTCG_M must be defined"
#endif
#ifndef FFTCG_PAD
#error "FFTCG_PAD must be defined"
#endif

#define FFTCG_CAT2(a, b, c) a##b##_##c
#define FFTCG_CAT(a, b, c) FFTCG_CAT2(a, b, c)
#define FFTCG_OPS_FN FFTCG_CAT(fftcg_engine_ops_, FFTCG_M, FFTCG_PAD)

namespace fftcg {
namespace {

constexpr int M = FFTCG_M;
constexpr int PAD = FFTCG_PAD;
template <typename T>
using G = Geo<T, M, PAD>;
constexpr int LL = G<float>::L;
constexpr int UPD_NT = 256;
constexpr int g4_blocks() {
    return cmax(1, cmin(1024, LL * LL / 1024));
}

template <typename T>
Tab<T> tab_of(const PlanTabs& t);
template <>
Tab<float> tab_of<float>(const PlanTabs& t) {
    return Tab<float>{(const cx<float>*)t.tw32, (const float*)t.ghq32, (const float*)t.ghN32};
}
template <>
Tab<double> tab_of<double>(const PlanTabs& t) {
    return Tab<double>{(const cx<double>*)t.tw64, (const double*)t.ghq64, (const double*)t.ghN64};
}

template <typename T>
void apply_pass_t(int pass, const PlanTabs& pt, const double* d, const double* x, double* y, void* W,
                  hipStream_t s) {
    constexpr int RT = G<T>::ROW_THREADS, CT = G<T>::COL_THREADS;
    ByVal sv;
    memset(&sv.s, 0, sizeof(SlotDesc));
    sv.s.d = d;
    sv.s.x = const_cast<double*>(x);
    sv.s.y = y;
    sv.s.W = W;
    sv.s.active = 1;
    const Tab<T> tab = tab_of<T>(pt);
    if (pass == 0)
        hipLaunchKernelGGL((k_row_fwd<T, M, PAD, ProApply<T>, ByVal, RT>), dim3(G<T>::ROW_BLOCKS), dim3(RT), 0,
                           s, tab, sv, 0, 0);
    else if (pass == 1)
        hipLaunchKernelGGL((k_col<T, M, PAD, GateAlways, ByVal, CT>), dim3(G<T>::NTILE), dim3(CT), 0, s, tab, sv);
    else
        hipLaunchKernelGGL((k_row_inv<T, M, PAD, EpiApply<T>, ByVal, RT>), dim3(G<T>::ROW_BLOCKS), dim3(RT), 0,
                           s, tab, sv, 0);
}

template <typename T>
void apply_t(const PlanTabs& pt, const double* d, const double* x, double* y, void* W, hipStream_t s) {
    for (int pass = 0; pass < 3; ++pass) apply_pass_t<T>(pass, pt, d, x, y, W, s);
}

void apply_pass_fn(int prec, int pass, const PlanTabs& pt, const double* d, const double* x, double* y, void* W,
                   hipStream_t s) {
    if (prec == 0)
        apply_pass_t<double>(pass, pt, d, x, y, W, s);
    else
        apply_pass_t<float>(pass, pt, d, x, y, W, s);
}

void apply_fn(int prec, const PlanTabs& pt, const double* d, const double* x, double* y, void* W,
              hipStream_t s) {
    if (prec == 0)
        apply_t<double>(pt, d, x, y, W, s);
    else
        apply_t<float>(pt, d, x, y, W, s);
}

template <typename W, typename XA>
void iter_t(const PlanTabs& pt, const SlotDesc* slots, int nslots, int stride, hipStream_t s) {
    constexpr int RT = G<W>::ROW_THREADS, CT = G<W>::COL_THREADS;
    const ByPtr sp{slots};
    const Tab<W> tab = tab_of<W>(pt);
    hipLaunchKernelGGL((k_row_fwd<W, M, PAD, ProCG<W, XA, RT>, ByPtr, RT>), dim3(G<W>::ROW_BLOCKS, nslots),
                       dim3(RT), 0, s, tab, sp, g4_blocks(), stride);
    hipLaunchKernelGGL((k_col<W, M, PAD, GateIter, ByPtr, CT>), dim3(G<W>::NTILE, nslots), dim3(CT), 0, s, tab,
                       sp);
    hipLaunchKernelGGL((k_row_inv<W, M, PAD, EpiCG<W>, ByPtr, RT>), dim3(G<W>::ROW_BLOCKS, nslots), dim3(RT), 0,
                       s, tab, sp, stride);
    hipLaunchKernelGGL((k_update<W, UPD_NT>), dim3(g4_blocks(), nslots), dim3(UPD_NT), 0, s, sp, LL * LL,
                       G<W>::ROW_BLOCKS, stride);
}

void iter_fn(int prec, const PlanTabs& pt, const SlotDesc* slots, int nslots, int stride, hipStream_t s);

// The same iteration for one slot with the update inside the row-inverse
// pass (EpiCGU): the row-forward pass then reduces that pass's RB r.r
// partials.  RB <= g4_blocks() (grid_capable_fn), so after an FP64 check,
// which writes g4_blocks() of them (|r|^2 first, zeros after), the first RB
// still hold the whole sum.
template <typename W>
void iter_grid_t(const PlanTabs& pt, const SlotDesc* slot, int stride, unsigned long long token, hipStream_t s) {
    constexpr int RT = G<W>::ROW_THREADS, CT = G<W>::COL_THREADS, RB = G<W>::ROW_BLOCKS;
    const ByPtr sp{slot};
    const Tab<W> tab = tab_of<W>(pt);
    hipLaunchKernelGGL((k_row_fwd<W, M, PAD, ProCG<W, W, RT>, ByPtr, RT>), dim3(RB), dim3(RT), 0, s, tab, sp, RB,
                       stride);
    hipLaunchKernelGGL((k_col<W, M, PAD, GateIter, ByPtr, CT>), dim3(G<W>::NTILE), dim3(CT), 0, s, tab, sp);
    hipLaunchKernelGGL((k_row_inv_upd<W, M, PAD, ByPtr, RT>), dim3(RB), dim3(RT), 0, s, tab, sp, stride, token);
}

bool iter_grid_fn(int prec, const PlanTabs& pt, const SlotDesc* slot, int stride, unsigned long long token,
                  hipStream_t s) {
    const bool fits = prec == 0 ? G<double>::ROW_BLOCKS <= g4_blocks() : G<float>::ROW_BLOCKS <= g4_blocks();
    if (!fits) {
        iter_fn(prec, pt, slot, 1, stride, s);
        return false;
    }
    if (prec == 0)
        iter_grid_t<double>(pt, slot, stride, token, s);
    else
        iter_grid_t<float>(pt, slot, stride, token, s);
    return true;
}

// The turn pass saves the reads of r and p and one launch per iteration but
// adds a second barrier.  Measured against the folded update alone (whole
// mixed solves, alternating in one process): padded L = 2048 +4.2%, L = 256
// +2.2%, L = 512 +0.5%, padded L = 512 FP64 +1.9%, periodic M = 256 / 512 /
// 2048 +1.2 / +2.4 / +5.2%; but padded L = 1024 (M = 2048) -1.2% and
// periodic M = 1024 -0.7%, so it is not offered on those two grids.
constexpr bool kTurnPays = PAD ? M != 2048 : M != 1024;
// Built where its grid can be resident at once: not in FP64 on rows of 16
// pairs a thread and more (over 200 VGPRs, two workgroups per CU).
template <typename W>
constexpr bool kTurnBuilt = !(sizeof(W) == 8 && G<W>::ER >= 16);

template <typename W>
void iter_pass_t(int pass, bool grid, const PlanTabs& pt, const SlotDesc* slot, int stride, unsigned long long token,
                 hipEvent_t e0, hipEvent_t e1, hipStream_t s) {
    constexpr int RT = G<W>::ROW_THREADS, CT = G<W>::COL_THREADS, RB = G<W>::ROW_BLOCKS;
    const ByPtr sp{slot};
    const Tab<W> tab = tab_of<W>(pt);
    if (pass == 0) {
        hipExtLaunchKernelGGL((k_row_fwd<W, M, PAD, ProCG<W, W, RT>, ByPtr, RT>), dim3(RB), dim3(RT), 0, s, e0, e1, 0,
                              tab, sp, grid ? RB : g4_blocks(), stride);
    } else if (pass == 1) {
        hipExtLaunchKernelGGL((k_col<W, M, PAD, GateIter, ByPtr, CT>), dim3(G<W>::NTILE), dim3(CT), 0, s, e0, e1, 0,
                              tab, sp);
    } else if (pass == 2) {
        if (grid) {
            hipExtLaunchKernelGGL((k_row_inv_upd<W, M, PAD, ByPtr, RT>), dim3(RB), dim3(RT), 0, s, e0, e1, 0, tab, sp,
                                  stride, token);
            return;
        }
        hipExtLaunchKernelGGL((k_row_inv<W, M, PAD, EpiCG<W>, ByPtr, RT>), dim3(RB), dim3(RT), 0, s, e0, e1, 0, tab,
                              sp, stride);
    } else if (pass == 3) {
        if (!grid)
            hipExtLaunchKernelGGL((k_update<W, UPD_NT>), dim3(g4_blocks()), dim3(UPD_NT), 0, s, e0, e1, 0, sp,
                                  LL * LL, RB, stride);
    } else if constexpr (kTurnBuilt<W>) {
        if (grid)
            hipExtLaunchKernelGGL((k_row_turn<W, M, PAD, ByPtr, RT>), dim3(RB), dim3(RT), 0, s, e0, e1, 0, tab, sp,
                                  stride, token);
    }
}

void iter_pass_fn(int prec, int pass, bool grid, const PlanTabs& pt, const SlotDesc* slot, int stride,
                  unsigned long long token, hipEvent_t e0, hipEvent_t e1, hipStream_t s) {
    if (prec == 0)
        iter_pass_t<double>(pass, grid && G<double>::ROW_BLOCKS <= g4_blocks(), pt, slot, stride, token, e0, e1, s);
    else
        iter_pass_t<float>(pass, grid && G<float>::ROW_BLOCKS <= g4_blocks(), pt, slot, stride, token, e0, e1, s);
}

// whether every workgroup of kernel `kern` (RB of RT threads) can be
// resident at once on the current device
template <int RT, int RB>
bool whole_grid_resident(const void* kern) {
    if (RB > g4_blocks()) return false;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, RT, 0) != hipSuccess) return false;
    return (long)per_cu * cus >= RB;
}

template <typename W>
bool grid_capable_t() {
    constexpr int RT = G<W>::ROW_THREADS, RB = G<W>::ROW_BLOCKS;
    return whole_grid_resident<RT, RB>(reinterpret_cast<const void*>(k_row_inv_upd<W, M, PAD, ByPtr, RT>));
}

bool grid_capable_fn(int prec) {
    return prec == 0 ? grid_capable_t<double>() : grid_capable_t<float>();
}

template <typename W>
bool turn_capable_t() {
    constexpr int RT = G<W>::ROW_THREADS, RB = G<W>::ROW_BLOCKS;
    if constexpr (!kTurnBuilt<W>)
        return false;
    else
        return kTurnPays && grid_capable_t<W>() &&
               whole_grid_resident<RT, RB>(reinterpret_cast<const void*>(k_row_turn<W, M, PAD, ByPtr, RT>));
}

bool turn_capable_fn(int prec) {
    return prec == 0 ? turn_capable_t<double>() : turn_capable_t<float>();
}

template <typename W>
void iter_grid_chunk_t(const PlanTabs& pt, const SlotDesc* slot, int stride, unsigned long long* token, int K,
                       bool turn, hipStream_t s) {
    if constexpr (kTurnBuilt<W>) {
        if (turn) {
            constexpr int RT = G<W>::ROW_THREADS, CT = G<W>::COL_THREADS, RB = G<W>::ROW_BLOCKS;
            const ByPtr sp{slot};
            const Tab<W> tab = tab_of<W>(pt);
            hipLaunchKernelGGL((k_row_fwd<W, M, PAD, ProCG<W, W, RT>, ByPtr, RT>), dim3(RB), dim3(RT), 0, s, tab,
                               sp, RB, stride);
            hipLaunchKernelGGL((k_col<W, M, PAD, GateIter, ByPtr, CT>), dim3(G<W>::NTILE), dim3(CT), 0, s, tab, sp);
            for (int k = 1; k < K; ++k) {
                const unsigned long long t = *token + 1;
                *token += 2;
                hipLaunchKernelGGL((k_row_turn<W, M, PAD, ByPtr, RT>), dim3(RB), dim3(RT), 0, s, tab, sp, stride, t);
                hipLaunchKernelGGL((k_col<W, M, PAD, GateIter, ByPtr, CT>), dim3(G<W>::NTILE), dim3(CT), 0, s, tab,
                                   sp);
            }
            hipLaunchKernelGGL((k_row_inv_upd<W, M, PAD, ByPtr, RT>), dim3(RB), dim3(RT), 0, s, tab, sp, stride,
                               ++*token);
            return;
        }
    }
    for (int k = 0; k < K; ++k) iter_grid_t<W>(pt, slot, stride, ++*token, s);
}

void iter_grid_chunk_fn(int prec, const PlanTabs& pt, const SlotDesc* slot, int stride, unsigned long long* token,
                        int K, bool turn, hipStream_t s) {
    if (prec == 0)
        iter_grid_chunk_t<double>(pt, slot, stride, token, K, turn, s);
    else
        iter_grid_chunk_t<float>(pt, slot, stride, token, K, turn, s);
}

void iter_fn(int prec, const PlanTabs& pt, const SlotDesc* slots, int nslots, int stride, hipStream_t s) {
    if (prec == 0)
        iter_t<double, double>(pt, slots, nslots, stride, s);
    else
        iter_t<float, float>(pt, slots, nslots, stride, s);
}

template <typename W>
void check_t(const PlanTabs& pt, const SlotDesc* slots, int nslots, int stride, hipStream_t s) {
    constexpr int RT = G<double>::ROW_THREADS, CT = G<double>::COL_THREADS;
    const ByPtr sp{slots};
    const Tab<double> tab = tab_of<double>(pt);
    hipLaunchKernelGGL((k_row_fwd<double, M, PAD, ProCheck<W, RT>, ByPtr, RT>),
                       dim3(G<double>::ROW_BLOCKS, nslots), dim3(RT), 0, s, tab, sp, 0, stride);
    hipLaunchKernelGGL((k_col<double, M, PAD, GateCheck, ByPtr, CT>), dim3(G<double>::NTILE, nslots), dim3(CT), 0,
                       s, tab, sp);
    hipLaunchKernelGGL((k_row_inv<double, M, PAD, EpiCheck<W>, ByPtr, RT>), dim3(G<double>::ROW_BLOCKS, nslots),
                       dim3(RT), 0, s, tab, sp, stride);
    hipLaunchKernelGGL((k_check_final<256>), dim3(1, nslots), dim3(256), 0, s, sp, G<double>::ROW_BLOCKS,
                       g4_blocks(), stride, LL * LL);
}

void check_fn(int prec, const PlanTabs& pt, const SlotDesc* slots, int nslots, int stride, hipStream_t s) {
    if (prec == 0)
        check_t<double>(pt, slots, nslots, stride, s);
    else
        check_t<float>(pt, slots, nslots, stride, s);
}

// Preconditioned CG (Fourier-space circulant preconditioner): the operator
// product with the direction (row_fwd with p = z + beta p, col, row_inv with
// q and p.q), then r <- r - alpha q fused into the row-forward pass of the
// preconditioner product (with r.r), its column pass with 1/(dbar + ghat),
// and its row-inverse pass writing z and r.z.
template <typename W, typename XA>
void iter_pcg_t(const PlanTabs& pt, const SlotDesc* slots, int nslots, int stride, hipStream_t s) {
    constexpr int RT = G<W>::ROW_THREADS, CT = G<W>::COL_THREADS, RB = G<W>::ROW_BLOCKS;
    const ByPtr sp{slots};
    const Tab<W> tab = tab_of<W>(pt);
    hipLaunchKernelGGL((k_row_fwd<W, M, PAD, ProPCG<W, XA, RT, RB>, ByPtr, RT>), dim3(RB, nslots), dim3(RT), 0, s,
                       tab, sp, RB, stride);
    hipLaunchKernelGGL((k_col<W, M, PAD, GateIter, ByPtr, CT>), dim3(G<W>::NTILE, nslots), dim3(CT), 0, s, tab,
                       sp);
    hipLaunchKernelGGL((k_row_inv<W, M, PAD, EpiCG<W>, ByPtr, RT>), dim3(RB, nslots), dim3(RT), 0, s, tab, sp,
                       stride);
    hipLaunchKernelGGL((k_row_fwd<W, M, PAD, ProUpdPre<W, RT, RB>, ByPtr, RT>), dim3(RB, nslots), dim3(RT), 0, s,
                       tab, sp, 0, stride);
    hipLaunchKernelGGL((k_col<W, M, PAD, GateIter, ByPtr, CT, true>), dim3(G<W>::NTILE, nslots), dim3(CT), 0, s,
                       tab, sp);
    hipLaunchKernelGGL((k_row_inv<W, M, PAD, EpiPre<W, GateIter>, ByPtr, RT>), dim3(RB, nslots), dim3(RT), 0, s,
                       tab, sp, stride);
}

void iter_pcg_fn(int prec, const PlanTabs& pt, const SlotDesc* slots, int nslots, int stride, hipStream_t s) {
    if (prec == 0)
        iter_pcg_t<double, double>(pt, slots, nslots, stride, s);
    else
        iter_pcg_t<float, float>(pt, slots, nslots, stride, s);
}

// FP64 check of the preconditioned solve (r.r partial count = the working
// precision's row blocks), then z = P^{-1} r and r.z of the replaced
// residual when the solve continues.
template <typename W>
void check_pcg_t(const PlanTabs& pt, const SlotDesc* slots, int nslots, int stride, hipStream_t s) {
    constexpr int RT = G<double>::ROW_THREADS, CT = G<double>::COL_THREADS;
    constexpr int RTW = G<W>::ROW_THREADS, CTW = G<W>::COL_THREADS, RBW = G<W>::ROW_BLOCKS;
    const ByPtr sp{slots};
    const Tab<double> tab = tab_of<double>(pt);
    const Tab<W> tabw = tab_of<W>(pt);
    hipLaunchKernelGGL((k_row_fwd<double, M, PAD, ProCheck<W, RT>, ByPtr, RT>),
                       dim3(G<double>::ROW_BLOCKS, nslots), dim3(RT), 0, s, tab, sp, 0, stride);
    hipLaunchKernelGGL((k_col<double, M, PAD, GateCheck, ByPtr, CT>), dim3(G<double>::NTILE, nslots), dim3(CT), 0,
                       s, tab, sp);
    hipLaunchKernelGGL((k_row_inv<double, M, PAD, EpiCheck<W>, ByPtr, RT>), dim3(G<double>::ROW_BLOCKS, nslots),
                       dim3(RT), 0, s, tab, sp, stride);
    hipLaunchKernelGGL((k_check_final<256>), dim3(1, nslots), dim3(256), 0, s, sp, G<double>::ROW_BLOCKS, RBW,
                       stride, LL * LL);
    hipLaunchKernelGGL((k_row_fwd<W, M, PAD, ProPre<W>, ByPtr, RTW>), dim3(RBW, nslots), dim3(RTW), 0, s, tabw, sp,
                       0, stride);
    hipLaunchKernelGGL((k_col<W, M, PAD, GatePre, ByPtr, CTW, true>), dim3(G<W>::NTILE, nslots), dim3(CTW), 0, s,
                       tabw, sp);
    hipLaunchKernelGGL((k_row_inv<W, M, PAD, EpiPre<W, GatePre>, ByPtr, RTW>), dim3(RBW, nslots), dim3(RTW), 0, s,
                       tabw, sp, stride);
}

void check_pcg_fn(int prec, const PlanTabs& pt, const SlotDesc* slots, int nslots, int stride, hipStream_t s) {
    if (prec == 0)
        check_pcg_t<double>(pt, slots, nslots, stride, s);
    else
        check_pcg_t<float>(pt, slots, nslots, stride, s);
}

// The initial check of a solve started from zero (x = 0, e = 0 already
// written by the host): r = b in one pass, then the finaliser (and, for the
// preconditioned solve, z = P^{-1} r).
template <typename W>
void check0_t(bool pcg, const PlanTabs& pt, const SlotDesc* slots, int nslots, int stride, hipStream_t s) {
    constexpr int RTW = G<W>::ROW_THREADS, CTW = G<W>::COL_THREADS, RBW = G<W>::ROW_BLOCKS;
    const ByPtr sp{slots};
    hipLaunchKernelGGL((k_check_zero<W, 256>), dim3(G<double>::ROW_BLOCKS, nslots), dim3(256), 0, s, sp, LL * LL,
                       stride);
    hipLaunchKernelGGL((k_check_final<256>), dim3(1, nslots), dim3(256), 0, s, sp, G<double>::ROW_BLOCKS,
                       pcg ? RBW : g4_blocks(), stride, LL * LL);
    if (pcg) {
        const Tab<W> tabw = tab_of<W>(pt);
        hipLaunchKernelGGL((k_row_fwd<W, M, PAD, ProPre<W>, ByPtr, RTW>), dim3(RBW, nslots), dim3(RTW), 0, s, tabw,
                           sp, 0, stride);
        hipLaunchKernelGGL((k_col<W, M, PAD, GatePre, ByPtr, CTW, true>), dim3(G<W>::NTILE, nslots), dim3(CTW), 0,
                           s, tabw, sp);
        hipLaunchKernelGGL((k_row_inv<W, M, PAD, EpiPre<W, GatePre>, ByPtr, RTW>), dim3(RBW, nslots), dim3(RTW), 0,
                           s, tabw, sp, stride);
    }
}

void check0_fn(int prec, const PlanTabs& pt, const SlotDesc* slots, int nslots, int stride, hipStream_t s) {
    if (prec == 0)
        check0_t<double>(false, pt, slots, nslots, stride, s);
    else
        check0_t<float>(false, pt, slots, nslots, stride, s);
}

void check0_pcg_fn(int prec, const PlanTabs& pt, const SlotDesc* slots, int nslots, int stride, hipStream_t s) {
    if (prec == 0)
        check0_t<double>(true, pt, slots, nslots, stride, s);
    else
        check0_t<float>(true, pt, slots, nslots, stride, s);
}

const EngineOps kOps = {M,
                        PAD,
                        LL,
                        G<float>::TT,
                        G<double>::TT,
                        G<float>::ROW_BLOCKS,
                        G<double>::ROW_BLOCKS,
                        g4_blocks(),
                        &apply_fn,
                        &apply_pass_fn,
                        &iter_fn,
                        &check_fn,
                        &iter_pcg_fn,
                        &check_pcg_fn,
                        &check0_fn,
                        &check0_pcg_fn,
                        &iter_grid_fn,
                        &iter_pass_fn,
                        &grid_capable_fn,
                        &iter_grid_chunk_fn,
                        &turn_capable_fn};

}  // namespace

const EngineOps* FFTCG_OPS_FN() { return &kOps; }

}  // namespace fftcg
