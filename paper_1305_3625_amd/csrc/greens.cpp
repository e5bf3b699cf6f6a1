// Spectrum of the physical Green's function of Sec. 2, eq. (1c), on the FFT
// grid (plan-time, host).
//
// Eq. (1c): the 1/r response of an elastic half-space averaged over the
// square plaquette (side a) of the source fibre, times (1 - nu^2)/(pi E a^2).
// With lengths in units of a the plaquette integral is a * P(Delta), P the
// integral of 1/r over the unit square centred at the lattice separation
// Delta; P is the four-corner sum of the primitive x ln(y + r) + y ln(x + r)
// of 1/r.  The sum cancels O(r log r) terms down to O(1/r), so it runs in
// extended precision.  On the M x M grid index a maps to the separation
// magnitude min(a, M - a), which makes the table exactly even; its DFT is
// then real and even and is computed by a radix-2 FFT along rows, then
// columns (rows in parallel).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <thread>
#include <vector>

#include "fftcg.h"
#include "fftcg_internal.hpp"

namespace {

using ld = long double;

ld xlog(ld x, ld u) { return x != 0.0L ? x * logl(u) : 0.0L; }  // u > 0 whenever x != 0

ld primitive(ld x, ld y) {
    const ld r = sqrtl(x * x + y * y);
    return xlog(x, y + r) + xlog(y, x + r);
}

double plaquette(double dx, double dy) {
    const ld x0 = (ld)dx - 0.5L, x1 = (ld)dx + 0.5L, y0 = (ld)dy - 0.5L, y1 = (ld)dy + 0.5L;
    return (double)(primitive(x1, y1) - primitive(x0, y1) - primitive(x1, y0) + primitive(x0, y0));
}

// In-place radix-2 DFT (forward sign) of length n = 2^lg on v, with
// tw[k] = exp(-2 pi i k / n), k < n/2.
void fft_inplace(std::complex<double>* v, int n, int lg, const std::complex<double>* tw) {
    for (int i = 0, j = 0; i < n; ++i) {
        if (i < j) std::swap(v[i], v[j]);
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j |= bit;
    }
    for (int s = 1; s <= lg; ++s) {
        const int h = 1 << (s - 1), step = n >> s;
        for (int b = 0; b < n; b += 2 * h)
            for (int k = 0; k < h; ++k) {
                const std::complex<double> t = tw[k * step] * v[b + k + h];
                v[b + k + h] = v[b + k] - t;
                v[b + k] += t;
            }
    }
}

// DFT of every line of the M x M real array a (lines of length M with
// stride `ls` between elements and `os` between lines), real part kept.
void dft_lines(double* a, int M, size_t ls, size_t os, const std::vector<std::complex<double>>& tw) {
    int lg = 0;
    while ((1 << lg) < M) ++lg;
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const int nth = (int)std::min<unsigned>(hw, (unsigned)M);
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t)
        th.emplace_back([=, &tw]() {
            std::vector<std::complex<double>> buf(M);
            for (int line = t; line < M; line += nth) {
                double* base = a + (size_t)line * os;
                for (int i = 0; i < M; ++i) buf[i] = std::complex<double>(base[(size_t)i * ls], 0.0);
                fft_inplace(buf.data(), M, lg, tw.data());
                for (int i = 0; i < M; ++i) base[(size_t)i * ls] = buf[i].real();
            }
        });
    for (auto& x : th) x.join();
}

}  // namespace

extern "C" int fftcg_greens_spectrum(int L, int padded, double nu, double E, double a, double* spectrum) try {
    if (!spectrum || (padded != 0 && padded != 1)) return FFTCG_EINVAL;
    if (L < 2 || (L & (L - 1)) || (padded ? 2 * L : L) > 8192) return FFTCG_EINVAL;
    if (!(E > 0.0) || !(a > 0.0) || !isfinite(E) || !isfinite(a) || !isfinite(nu) || !(fabs(nu) < 1.0))
        return FFTCG_EINVAL;
    const int M = padded ? 2 * L : L;
    const double pref = (1.0 - nu * nu) / (M_PI * E * a);
    std::vector<double> sepv(M);
    for (int i = 0; i < M; ++i) sepv[i] = (double)std::min(i, M - i);
    // the table is even and symmetric: evaluate P on one octant of separations
    const int H = M / 2 + 1;
    std::vector<double> oct((size_t)H * H);
    for (int i = 0; i < H; ++i)
        for (int j = 0; j <= i; ++j) oct[(size_t)i * H + j] = oct[(size_t)j * H + i] = pref * plaquette(i, j);
    for (int m = 0; m < M; ++m)
        for (int n = 0; n < M; ++n)
            spectrum[(size_t)m * M + n] = oct[(size_t)sepv[m] * H + (size_t)sepv[n]];
    std::vector<std::complex<double>> tw(std::max(1, M / 2));
    for (int k = 0; k < M / 2; ++k) {
        double c, s;
        fftcg::cos_sin_2pi(k, M, &c, &s);
        tw[k] = std::complex<double>(c, -s);
    }
    dft_lines(spectrum, M, 1, (size_t)M, tw);  // rows
    dft_lines(spectrum, M, (size_t)M, 1, tw);  // columns
    // exact evenness of the result (the DFT of an even table is even; the
    // FFT's rounding is not): average each value with its mirror images
    for (int m = 0; m <= M / 2; ++m)
        for (int n = 0; n <= M / 2; ++n) {
            const int m2 = (M - m) % M, n2 = (M - n) % M;
            const double v = 0.25 * (spectrum[(size_t)m * M + n] + spectrum[(size_t)m2 * M + n] +
                                     spectrum[(size_t)m * M + n2] + spectrum[(size_t)m2 * M + n2]);
            spectrum[(size_t)m * M + n] = spectrum[(size_t)m2 * M + n] = spectrum[(size_t)m * M + n2] =
                spectrum[(size_t)m2 * M + n2] = v;
        }
    return FFTCG_OK;
} FFTCG_ABI_CATCH
