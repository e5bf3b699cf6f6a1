"""Input recipes for the five benchmark workloads.

Every array is generated on the host in float64 from numpy's PCG64
(``np.random.default_rng(seed_list)``) so the GPU path and the oracle see
identical bits.  The draw order inside one instance is fixed:
d (uniform), zero mask, b, t.

Workloads (sizes are the physical grid side ``L``; ``M`` is the FFT grid):

* C1  periodic L=64 (M=64), eps=1e-2, d~U(0.5,1.5), b~U(0,1), FP64, tol 1e-10.
* C2  padded L=512 (M=1024), eps=1e-3, d~U(0.5,1.5) with Bernoulli(0.3)
      zeros, b~U(0,1), FP64, tol 1e-10.
* C3  padded L=2048 (M=4096), eps=1e-4, d as C2, b~N(0,1), mixed precision,
      error target 1e-8.
* C4  serving: 20,000 requests, exponential inter-arrival times with mean
      0.5 ms, M drawn from {128,256,512,1024} with p={.4,.3,.2,.1} (L=M/2),
      eps=1e-3, d as C2, b~U(0,1), mixed precision, tol 1e-8.
* C5  load-stepped sequences: M=1024 (L=512), eps=1e-3, t~U(0,1), d=1,
      b=1, 1,000 steps each, 64 sequences, mixed precision, tol 1e-8.
"""

from __future__ import annotations

import numpy as np


def _cos_table(M: int) -> np.ndarray:
    """cos(2*pi*m/M) for m in [0, M), exactly even: c[m] == c[M-m] bitwise.

    The argument is folded to min(m, M-m) before the library cosine, so the
    spectrum built from it is exactly even in each index.
    """
    m = np.arange(M)
    folded = np.minimum(m, (M - m) % M)
    return np.cos(2.0 * np.pi * folded / M)


def spectrum(M: int, eps: float) -> np.ndarray:
    """Synthetic long-range kernel spectrum on the M x M FFT grid.

    ghat[m, n] = 1 / sqrt(4 - 2 cos(2 pi m / M) - 2 cos(2 pi n / M) + eps),
    indexed ``[m, n]`` with m along the slow (row) axis.  It is the lattice
    analogue of the Fourier transform of a 1/r kernel: real, positive, even in
    each index, symmetric under m <-> n, with maximum 1/sqrt(eps) at (0, 0).
    """
    c = _cos_table(M)
    # c[m] + c[n] is commutative, so the result is exactly symmetric in m, n
    den = 4.0 - 2.0 * (c[:, None] + c[None, :]) + eps
    return 1.0 / np.sqrt(den)


def _uniform_d(rng, L):
    return rng.uniform(0.5, 1.5, size=(L, L))


def _zero_mask(rng, L, p=0.3):
    return rng.random((L, L)) < p


def periodic_instance(L: int, seed, eps: float = 1e-2):
    """Periodic grid instance (M = L): d ~ U(0.5, 1.5), b ~ U(0, 1)."""
    rng = np.random.default_rng(seed)
    d = _uniform_d(rng, L)
    b = rng.uniform(0.0, 1.0, size=(L, L))
    return dict(L=L, M=L, padded=0, eps=eps, ghat=spectrum(L, eps), d=d, b=b)


def padded_instance(L: int, seed, eps: float = 1e-3, zero_frac: float = 0.3,
                    normal_b: bool = False):
    """Zero-padded grid instance (M = 2L): d ~ U(0.5,1.5) with zeros, b."""
    rng = np.random.default_rng(seed)
    d = _uniform_d(rng, L)
    if zero_frac > 0:
        d[_zero_mask(rng, L, zero_frac)] = 0.0
    if normal_b:
        b = rng.standard_normal((L, L))
    else:
        b = rng.uniform(0.0, 1.0, size=(L, L))
    M = 2 * L
    return dict(L=L, M=M, padded=1, eps=eps, ghat=spectrum(M, eps), d=d, b=b)


def c1_instance(s: int):
    return dict(periodic_instance(64, [1, s], eps=1e-2), mode="fp64", tol=1e-10)


def c2_instance(s: int):
    return dict(padded_instance(512, [2, s], eps=1e-3), mode="fp64", tol=1e-10)


def c3_instance(s: int, L: int = 2048):
    inst = padded_instance(L, [3, s], eps=1e-4, normal_b=True)
    return dict(inst, mode="mixed", tol=1e-8)


C4_SIZES = (128, 256, 512, 1024)
C4_PROBS = (0.4, 0.3, 0.2, 0.1)


def c4_schedule(n_requests: int = 20000, mean_gap_s: float = 0.5e-3):
    """Open-loop arrival schedule: (arrival times in s, FFT grid size M)."""
    rng = np.random.default_rng([4, 0])
    gaps = rng.exponential(mean_gap_s, size=n_requests)
    t = np.cumsum(gaps)
    sizes = rng.choice(np.array(C4_SIZES), size=n_requests, p=np.array(C4_PROBS))
    return t, sizes


def c4_request(k: int, M: int, eps: float = 1e-3):
    """Request k of the serving workload on the padded M x M grid (L = M/2)."""
    L = M // 2
    rng = np.random.default_rng([4, 1, k])
    d = _uniform_d(rng, L)
    d[_zero_mask(rng, L)] = 0.0
    b = rng.uniform(0.0, 1.0, size=(L, L))
    return dict(L=L, M=M, padded=1, eps=eps, d=d, b=b, tol=1e-8, mode="mixed")


def c5_sequence(s: int, L: int = 512, eps: float = 1e-3):
    """Load-stepped sequence s: thresholds t ~ U(0,1), d = 1, b = 1."""
    rng = np.random.default_rng([5, s])
    t = rng.uniform(0.0, 1.0, size=(L, L))
    d = np.ones((L, L))
    b = np.ones((L, L))
    return dict(L=L, M=2 * L, padded=1, eps=eps, t=t, d=d, b=b, tol=1e-8,
                mode="mixed")


CONFIGS = {
    "C1": dict(L=64, padded=0, eps=1e-2, mode="fp64", tol=1e-10, seeds=100),
    "C2": dict(L=512, padded=1, eps=1e-3, mode="fp64", tol=1e-10, seeds=10),
    "C3": dict(L=2048, padded=1, eps=1e-4, mode="mixed", tol=1e-8, seeds=3),
    "C4": dict(sizes=C4_SIZES, probs=C4_PROBS, eps=1e-3, mode="mixed",
               tol=1e-8, requests=20000),
    "C5": dict(L=512, padded=1, eps=1e-3, mode="mixed", tol=1e-8,
               sequences=64, steps=1000),
}


def fracture_instance(s: int, L: int = 64, padded: int = 1, gradient: float = 1.0):
    """Thresholds for the fracture driver: t = 1e-3 + U(0,1) + gradient * i1/L
    (a gradient along the row index directs the front); uniform stiffness."""
    rng = np.random.default_rng([6, s])
    i1 = np.arange(L, dtype=np.float64)[:, None] / L
    t = 1e-3 + rng.uniform(0.0, 1.0, (L, L)) + gradient * i1
    return dict(L=L, padded=padded, t=t, k=1.0)
