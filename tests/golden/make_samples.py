"""Writes seeded sample entries of exact discrete solutions, from the
oracle's sparse direct FP64 solve, with ||u*||^2 and <f, u*> (twice the
negated minimum energy):

* level10_traction_samples.json: the level-10 traction workload (clamped
  unit square, 2^10 x 2^10 nodes, 2,097,152 dofs, seeded eight-mode sine
  traction on the east edge, plane strain E = 1, nu = 0.3);
* lshape9_samples.json: the L-shaped plate of three 2^9 x 2^9 squares
  (1,572,864 dofs, symmetric exact coupling, clamped bottom, seeded traction
  on the top edge).

Calls only the oracle and the shared workload generator; takes a few
minutes per workload and a few GB of memory.  Run from the repository root:

    python tests/golden/make_samples.py [traction|lshape]
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import fem  # noqa: E402

LEVEL = 10
NSAMPLES = 2048
SEED = 20250107


def main(which: str):
    if which == "lshape":
        prob, name, label = W.l_shape(9), "lshape9_samples.json", "l_shape(level=9)"
    else:
        prob, name = W.cantilever_traction(LEVEL), "level10_traction_samples.json"
        label = "cantilever_traction(level=10)"
    u, f = fem.solve_problem(prob)          # both in QTT order (first core fastest)
    rng = np.random.default_rng(SEED)
    idx = np.sort(rng.choice(u.size, size=NSAMPLES, replace=False))
    out = {
        "workload": label,
        "source": "oracle.fem.solve_problem (sparse direct, FP64)",
        "ndofs": int(u.size),
        "seed": SEED,
        "index": [int(i) for i in idx],
        "value": [float(repr_v) for repr_v in u[idx]],
        "norm2": float(u @ u),
        "f_dot_u": float(f @ u),
        "max_abs": float(np.abs(u).max()),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), name)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "traction")
