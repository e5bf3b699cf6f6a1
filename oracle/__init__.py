"""Plain FP64 CPU oracle for the FFT-convolution conjugate-gradient solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use it.  It shares no code with the HIP path; the only common
code is the seeded input recipes in ``workloads/``.

What it computes (Gjerden, "Making the case of GPUs in courses on
computational physics"):

* Sec. 2, eqs. (1a)-(1c) and (2): each fibre force couples to every other
  through a Green's function that depends only on the separation; the linear
  system for the forces is symmetric positive definite (Sec. 3).  The solver
  works on the SPD form ``A = diag(d) + C`` where ``C`` is the 2-D convolution
  with a real kernel ``g_M`` whose DFT multiplier is ``ghat``.
* Sec. 3, eq. (3): ``C`` is diagonal in Fourier space, so
  ``C v = F^{-1}(ghat * F v)``.  On a zero-padded grid (M = 2L) the circular
  convolution restricted to the L x L grid is the linear convolution.
* Sec. 3: unpreconditioned conjugate gradient (Sec. 4 states no
  preconditioner was used).

Modules:

* ``kernel_table`` -- g_M by a cosine-matrix product (no FFT).
* ``operator``     -- A x by the direct real-space sum, by an assembled
  dense matrix, and (for large grids) by scipy's FFT as a library step.
* ``cg``           -- textbook Hestenes-Stiefel CG.
* ``pcg``          -- CG with the Fourier-space (circulant) preconditioner
  (an extension beyond the paper, which ran without one).
* ``dense``        -- Cholesky solve of the assembled dense system.
* ``greens``       -- the physical Green's function of eq. (1c) and its
  spectrum (plaquette-averaged 1/r kernel, closed form).
* ``bounds``       -- closed-form spectrum bounds and the certified stop rule.
* ``loadstep``     -- the load-step rule of the load-stepped workload.
* ``fracture``     -- the quasi-static fracture driver of Sec. 2 (restricted
  solves with broken fibres projected out).
* ``reference``    -- reference solves run to stagnation and certified.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, brute-force sums, plane-wave eigenpairs, a dense
Cholesky solve or an independent library route.  The paper itself prints no
worked example, solution value, tolerance or iteration count, so parity with
numbers printed in the paper is unpinned (there are none to pin to).
"""

from .kernel_table import kernel_table, kernel_table_bruteforce  # noqa: F401
from .operator import (  # noqa: F401
    conv_direct,
    apply_direct,
    apply_direct_at,
    assemble_dense,
    apply_fft,
)
from .cg import cg  # noqa: F401
from .pcg import pcg, circulant_precond  # noqa: F401
from .dense import solve_dense  # noqa: F401
from .greens import plaquette_integral, green_table, green_spectrum  # noqa: F401
from .bounds import lambda_lb, lambda_ub, kappa_ub, certified_ok, error_bound  # noqa: F401
from .loadstep import loadstep_argmax, loadstep_valid  # noqa: F401
from .fracture import restricted_solve, fracture_sequence  # noqa: F401
from .reference import reference_solve  # noqa: F401
