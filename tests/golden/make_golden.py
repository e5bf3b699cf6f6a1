"""Writes the small golden fixtures in this folder.

Every stored value comes from the CPU oracle (``oracle/``) and the seeded
input recipes (``workloads/``): dense Cholesky solutions of small systems,
periodic and zero-padded.  Run from the repository root:

    python tests/golden/make_golden.py
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from workloads import periodic_instance, padded_instance  # noqa: E402
from oracle import kernel_table, solve_dense, lambda_lb  # noqa: E402

CASES = [
    ("periodic_L8", lambda: periodic_instance(8, [70, 0], eps=1e-2), 0),
    ("padded_L8", lambda: padded_instance(8, [71, 0], eps=1e-3), 1),
    ("periodic_L4", lambda: periodic_instance(4, [72, 0], eps=1e-2), 0),
    ("padded_L2", lambda: padded_instance(2, [73, 0], eps=1e-3), 1),
]


def main():
    for name, make, padded in CASES:
        inst = make()
        g = kernel_table(inst["ghat"])
        x = solve_dense(g, inst["d"], inst["b"], padded)
        out = dict(
            source="oracle.solve_dense (Cholesky of the assembled operator, "
                   "Sec. 2 eq. (2) in SPD form; Sec. 3 eq. (3) multiplier)",
            L=inst["L"], M=inst["M"], padded=padded, eps=inst["eps"],
            d=inst["d"].ravel().tolist(), b=inst["b"].ravel().tolist(),
            x=x.ravel().tolist(),
            lambda_lb=lambda_lb(inst["ghat"], inst["d"]),
        )
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
