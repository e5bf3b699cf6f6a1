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

// (bound_src, bound_dst: when given, the value at bound_src -- the finished
// solve's certified error bound -- is recorded at bound_dst.)
template <typename MK>
__global__ void __launch_bounds__(LS_NT)
    k_loadstep_final(const double* __restrict__ pv, const int* __restrict__ pi, int nb, int n,
                     MK* __restrict__ mk, int* __restrict__ out, double* __restrict__ out_v,
                     const double* __restrict__ bound_src, double* __restrict__ bound_dst) {
    VI best{-INFINITY, n};
    for (int b = threadIdx.x; b < nb; b += LS_NT) best = better(best, VI{pv[b], pi[b]});
    best = block_best(best);
    if (threadIdx.x == 0) {
        const int idx = best.i < n ? best.i : -1;
        if (idx >= 0) mk[idx] = MK(0);
        out[0] = idx;
        if (out_v) out_v[0] = idx >= 0 ? best.v : 0.0;
        if (bound_dst) bound_dst[0] = bound_src[0];
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
                     hipStream_t s, const double* bound_src, double* bound_dst) {
    const int nb = loadstep_blocks(n);
    hipLaunchKernelGGL(k_loadstep_partial<double>, dim3(nb), dim3(LS_NT), 0, s, x, t, d, n, pv, pi);
    hipLaunchKernelGGL(k_loadstep_final<double>, dim3(1), dim3(LS_NT), 0, s, pv, pi, nb, n, d, out,
                       (double*)nullptr, bound_src, bound_dst);
}

void launch_breakstep(const double* x, const double* t, uint8_t* mask, int n, double* pv, int* pi, int* out,
                      double* out_v, hipStream_t s) {
    const int nb = loadstep_blocks(n);
    hipLaunchKernelGGL(k_loadstep_partial<uint8_t>, dim3(nb), dim3(LS_NT), 0, s, x, t, mask, n, pv, pi);
    hipLaunchKernelGGL(k_loadstep_final<uint8_t>, dim3(1), dim3(LS_NT), 0, s, pv, pi, nb, n, mask, out, out_v,
                       (const double*)nullptr, (double*)nullptr);
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

// ---- HBM streaming probes -----------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int SP_NT = 256;

template <bool NT>
__device__ __forceinline__ v4f sp_load(const v4f* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    return *p;
}
template <bool NT>
__device__ __forceinline__ void sp_store(v4f* p, v4f v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// kind 0 read, 1 write, 2 copy; four independent 16-byte accesses in flight
// per thread and iteration.
template <int KIND, bool NT>
__global__ void __launch_bounds__(SP_NT)
    k_stream(v4f* __restrict__ dst, const v4f* __restrict__ src, size_t n, float* __restrict__ sink) {
    const size_t stride = (size_t)gridDim.x * SP_NT;
    size_t i = (size_t)blockIdx.x * SP_NT + threadIdx.x;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (; i + 3 * stride < n; i += 4 * stride) {
        if constexpr (KIND == 1) {
            const v4f z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int u = 0; u < 4; ++u) sp_store<NT>(dst + i + u * stride, z);
        } else {
            v4f v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = sp_load<NT>(src + i + u * stride);
            if constexpr (KIND == 2) {
#pragma unroll
                for (int u = 0; u < 4; ++u) sp_store<NT>(dst + i + u * stride, v[u]);
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) acc += v[u];
            }
        }
    }
    for (; i < n; i += stride) {
        if constexpr (KIND == 1) {
            const v4f z = {0.f, 0.f, 0.f, 0.f};
            sp_store<NT>(dst + i, z);
        } else {
            const v4f v = sp_load<NT>(src + i);
            if constexpr (KIND == 2)
                sp_store<NT>(dst + i, v);
            else
                acc += v;
        }
    }
    if constexpr (KIND == 0) {
        const float t = acc.x + acc.y + acc.z + acc.w;
        if (t != 0.f) sink[0] = t;  // zero data: never stored, but the loads stay
    }
}

template <int KIND, bool NT>
static void launch_stream_k(int blocks, void* dst, const void* src, size_t n, hipStream_t s) {
    hipLaunchKernelGGL((k_stream<KIND, NT>), dim3(blocks), dim3(SP_NT), 0, s, (v4f*)dst, (const v4f*)src, n,
                       (float*)dst);
}

void launch_stream(int kind, bool nt, int blocks, void* dst, const void* src, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 16;
    switch (kind * 2 + (nt ? 1 : 0)) {
        case 0: launch_stream_k<0, false>(blocks, dst, src, n, s); break;
        case 1: launch_stream_k<0, true>(blocks, dst, src, n, s); break;
        case 2: launch_stream_k<1, false>(blocks, dst, src, n, s); break;
        case 3: launch_stream_k<1, true>(blocks, dst, src, n, s); break;
        case 4: launch_stream_k<2, false>(blocks, dst, src, n, s); break;
        default: launch_stream_k<2, true>(blocks, dst, src, n, s); break;
    }
}

__global__ void k_fill(double* __restrict__ a, double v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

void launch_fill(double* a, double v, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, s, a, v, n);
}

}  // namespace fftcg
