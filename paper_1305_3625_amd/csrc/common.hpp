// Launchers of the size-independent kernels (common.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fftcg {

void launch_to_f32(const double* src, float* dst, int n, hipStream_t s);
int loadstep_blocks(int n);
// argmax over d != 0 of x / t (ties to the smaller index), d[i*] = 0,
// *out = i* or -1.  pv / pi hold loadstep_blocks(n) partials.  When
// bound_dst is given, *bound_dst = *bound_src as well (device pointers).
void launch_loadstep(const double* x, const double* t, double* d, int n, double* pv, int* pi, int* out,
                     hipStream_t s, const double* bound_src = nullptr, double* bound_dst = nullptr);
// the same over mask != 0, mask[i*] = 0, and *out_v = x[i*] / t[i*].
void launch_breakstep(const double* x, const double* t, uint8_t* mask, int n, double* pv, int* pi, int* out,
                      double* out_v, hipStream_t s);
// launch_loadstep with its partials in the library's static device array
// (no allocation), then *index (host) = i*.  Blocks.  0 on success, -1 if n
// is outside [1, 2^31) or needs more partials than the array holds, -2 on a
// HIP error.
int loadstep_noalloc(const double* x, const double* t, double* d, int n, int* index, hipStream_t s);
// HBM streaming probe: kind 0 read src (sink: dst, written only for
// non-zero data), 1 zero-fill dst, 2 copy src -> dst; bytes / 16 vectors.
void launch_stream(int kind, bool nontemporal, int blocks, void* dst, const void* src, size_t bytes,
                   hipStream_t s);
// a[i] = v, i < n.
void launch_fill(double* a, double v, int n, hipStream_t s);

}  // namespace fftcg
