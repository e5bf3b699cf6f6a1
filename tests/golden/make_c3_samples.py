"""Writes sampled entries of the oracle's solutions of the three zero-padded
L = 2048 mixed-precision instances (eps 1e-4, d ~ U(0.5, 1.5) with 30%
zeros, b ~ N(0, 1); seeds [3, 0..2]).

Each solution is the oracle's FP64 CG with the eq. (3) product (scipy's FFT
as a library step, pinned against the direct real-space sum), run to
stagnation and certified from its own residual.  The full vector (32 MB) is
too large to keep, so the file stores its 2-norm, its certified bound and
1,024 entries at seeded positions: a GPU solution x with relative error e
has |x_i - x*_i| <= e ||x*|| at every entry.  Takes a few minutes on eight
host cores.  Run from the repository root:

    python tests/golden/make_c3_samples.py
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from workloads import c3_instance  # noqa: E402
from oracle import reference_solve  # noqa: E402

SAMPLES = 1024


def sample_positions(seed, n, k=SAMPLES):
    """Seeded sample of k distinct row-major positions in [0, n), with the
    first and last entries always included."""
    rng = np.random.default_rng([80, seed])
    idx = rng.choice(n, size=k - 2, replace=False)
    return np.unique(np.concatenate([[0, n - 1], idx]))


def main(seeds=(0, 1, 2)):
    for s in seeds:
        t0 = time.time()
        inst = c3_instance(s)
        x, info = reference_solve(inst["ghat"], inst["d"], inst["b"], 1, route="fft")
        pos = sample_positions(s, x.size)
        out = dict(
            source="oracle.reference_solve (FP64 CG, eq. (3) product by scipy FFT, run to "
                   "stagnation; Sec. 3)",
            seed=[3, s], L=inst["L"], eps=inst["eps"],
            iterations=info["iterations"], bound=info["bound"],
            xnorm=float(np.linalg.norm(x)),
            pos=pos.tolist(), x=x.ravel()[pos].tolist(),
        )
        with open(os.path.join(HERE, f"padded_L2048_seed{s}_samples.json"), "w") as f:
            json.dump(out, f)
        print(f"seed {s}: {info['iterations']} iterations, bound {info['bound']:.2e}, "
              f"{time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
