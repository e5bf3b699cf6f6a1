// Size-independent kernels: FP32 copy of the diagonal, and the load-step
// argmax (Sec. 2: after each solve the bond with the largest strain relative
// to its threshold breaks).
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.hpp"
#include "fftcg_dev.hpp"

namespace fftcg {

__global__ void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

// (value, index) argmax with ties to the smaller index; entries with d == 0
// are excluded (value -inf, index n).
struct VI {
    double v;
    int i;
};
__device__ __forceinline__ VI better(VI a, VI b) {
    if (a.v > b.v) return a;
    if (b.v > a.v) return b;
    return a.i <= b.i ? a : b;
}
__device__ __forceinline__ VI wave_best(VI a) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        VI b;
        b.v = __shfl_xor(a.v, o, 64);
        b.i = __shfl_xor(a.i, o, 64);
        a = better(a, b);
    }
    return a;
}
constexpr int LS_NT = 256;

__device__ VI block_best(VI a) {
    __shared__ double sv[LS_NT / 64];
    __shared__ int si[LS_NT / 64];
    a = wave_best(a);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        sv[threadIdx.x >> 6] = a.v;
        si[threadIdx.x >> 6] = a.i;
    }
    __syncthreads();
    VI r{sv[0], si[0]};
    for (int w = 1; w < LS_NT / 64; ++w) r = better(r, VI{sv[w], si[w]});
    return r;
}

// Entries whose marker is 0 are excluded: d == 0 (load-stepped sequences:
// the broken bond has no diagonal term left) or mask == 0 (fracture driver:
// the broken fibre is projected out).
template <typename MK>
__global__ void __launch_bounds__(LS_NT)
    k_loadstep_partial(const double* __restrict__ x, const double* __restrict__ t, const MK* __restrict__ mk,
                       int n, double* __restrict__ pv, int* __restrict__ pi) {
    VI best{-INFINITY, n};
    for (int i = blockIdx.x * LS_NT + threadIdx.x; i < n; i += gridDim.x * LS_NT) {
        if (mk[i] != MK(0)) best = better(best, VI{x[i] / t[i], i});
    }
    best = block_best(best);
    if (threadIdx.x == 0) {
        pv[blockIdx.x] = best.v;
        pi[blockIdx.x] = best.i;
    }
}

template <typename MK>
__global__ void __launch_bounds__(LS_NT)
    k_loadstep_final(const double* __restrict__ pv, const int* __restrict__ pi, int nb, int n,
                     MK* __restrict__ mk, int* __restrict__ out, double* __restrict__ out_v) {
    VI best{-INFINITY, n};
    for (int b = threadIdx.x; b < nb; b += LS_NT) best = better(best, VI{pv[b], pi[b]});
    best = block_best(best);
    if (threadIdx.x == 0) {
        const int idx = best.i < n ? best.i : -1;
        if (idx >= 0) mk[idx] = MK(0);
        out[0] = idx;
        if (out_v) out_v[0] = idx >= 0 ? best.v : 0.0;
    }
}

void launch_to_f32(const double* src, float* dst, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_f32, dim3((n + 255) / 256), dim3(256), 0, s, src, dst, n);
}

int loadstep_blocks(int n) {
    int b = (n + LS_NT * 16 - 1) / (LS_NT * 16);
    return b < 1 ? 1 : (b > 1024 ? 1024 : b);
}

void launch_loadstep(const double* x, const double* t, double* d, int n, double* pv, int* pi, int* out,
                     hipStream_t s) {
    const int nb = loadstep_blocks(n);
    hipLaunchKernelGGL(k_loadstep_partial<double>, dim3(nb), dim3(LS_NT), 0, s, x, t, d, n, pv, pi);
    hipLaunchKernelGGL(k_loadstep_final<double>, dim3(1), dim3(LS_NT), 0, s, pv, pi, nb, n, d, out,
                       (double*)nullptr);
}

void launch_breakstep(const double* x, const double* t, uint8_t* mask, int n, double* pv, int* pi, int* out,
                      double* out_v, hipStream_t s) {
    const int nb = loadstep_blocks(n);
    hipLaunchKernelGGL(k_loadstep_partial<uint8_t>, dim3(nb), dim3(LS_NT), 0, s, x, t, mask, n, pv, pi);
    hipLaunchKernelGGL(k_loadstep_final<uint8_t>, dim3(1), dim3(LS_NT), 0, s, pv, pi, nb, n, mask, out, out_v);
}

// ---- load step without allocation ------------------------------------------
// The argmax partials of one load step (at most LS_MAX_BLOCKS blocks: values,
// then indices) and the result word, in a file-scope device array: every call
// on a device shares that device's copy.  Nothing needs clearing: each call's
// partial kernel writes every partial its final kernel reads, and the final
// kernel writes the result word.  Calls that overlap on one device race on it.
constexpr int LS_MAX_BLOCKS = 1024;
constexpr size_t LS_SCRATCH_BYTES = 16384;
static_assert(LS_MAX_BLOCKS * (sizeof(double) + sizeof(int)) + 4 * sizeof(int) <= LS_SCRATCH_BYTES,
              "load-step scratch too small");
static __device__ __align__(256) unsigned char scratch[LS_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// Device address of this device's copy of `scratch` (looked up once per
// device, with that device current); nullptr on a HIP error.
static void* scratch_on(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

int loadstep_noalloc(const double* x, const double* t, double* d, int n, int* index, hipStream_t s) {
    const int nb = loadstep_blocks(n);
    if (n < 1 || nb > LS_MAX_BLOCKS) return -1;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return -2;
    unsigned char* base = (unsigned char*)scratch_on(dev);
    if (!base) return -2;
    double* pv = (double*)base;
    int* pi = (int*)(base + LS_MAX_BLOCKS * sizeof(double));
    int* out = pi + LS_MAX_BLOCKS;
    launch_loadstep(x, t, d, n, pv, pi, out, s);
    if (hipGetLastError() != hipSuccess) return -2;
    int h = -1;
    if (hipMemcpyAsync(&h, out, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return -2;
    *index = h;
    return 0;
}

__global__ void k_fill(double* __restrict__ a, double v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

void launch_fill(double* a, double v, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, s, a, v, n);
}

}  // namespace fftcg
