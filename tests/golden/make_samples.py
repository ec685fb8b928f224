"""Writes seeded sample entries of exact discrete solutions, from the
oracle's sparse direct FP64 solve, with ||u*||^2 and <f, u*> (twice the
negated minimum energy):

* level10_traction_samples.json: the level-10 traction workload (clamped
  unit square, 2^10 x 2^10 nodes, 2,097,152 dofs, seeded eight-mode sine
  traction on the east edge, plane strain E = 1, nu = 0.3);
* lshape9_samples.json: the L-shaped plate of three 2^9 x 2^9 squares
  (1,572,864 dofs, symmetric exact coupling, clamped bottom, seeded traction
  on the top edge).

The samples are 2048 uniformly drawn dofs plus stratified ones where the
solution is hardest to approximate: nodes on and next to the clamped edge,
on and next to the loaded edge, around the square's corners, and for the L
around the re-entrant corner (1, 1) and along the interfaces; "stratum"
names each sample's group.

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


def _dofs(prob, sub, i, j):
    """Z-ordered indices of both components of nodes (i, j) of subdomain
    `sub` (index c + 2 (m + q Z(i, j)))."""
    q = prob.q
    z = fem.zorder(np.asarray(i), np.asarray(j), prob.level)
    g = 2 * (sub + q * z)
    return np.concatenate([g, g + 1])


def _samples(prob, which, ndofs, rng):
    n = 2 ** prob.level
    groups = [("uniform", rng.choice(ndofs, size=NSAMPLES, replace=False))]

    def edge(sub, side, count):
        t = rng.integers(0, n, count)
        off = rng.integers(0, 2, count)          # on the edge or one node in
        i, j = {0: (off, t), 1: (n - 1 - off, t), 2: (t, off), 3: (t, n - 1 - off)}[side]
        return _dofs(prob, sub, i, j)

    def corner(sub, ci, cj, width):
        a = np.arange(width)
        i = a if ci == 0 else n - 1 - a
        j = a if cj == 0 else n - 1 - a
        I, J = np.meshgrid(i, j, indexing="ij")
        return _dofs(prob, sub, I.ravel(), J.ravel())

    if which == "lshape":
        # clamped bottoms of the lower squares, the loaded top of the upper one
        groups.append(("clamped_edge", np.concatenate([edge(0, 2, 128), edge(1, 2, 128)])))
        groups.append(("loaded_edge", edge(2, 3, 256)))
        # the re-entrant corner (1, 1): corner (n-1, n-1) of the first
        # square, (0, n-1) of the second, (n-1, 0) of the third
        groups.append(("reentrant_corner", np.concatenate(
            [corner(0, 1, 1, 6), corner(1, 0, 1, 6), corner(2, 1, 0, 6)])))
        # the interfaces: east side of the first square (shared with the
        # second) and its north side (shared with the third)
        groups.append(("interfaces", np.concatenate([edge(0, 1, 64), edge(0, 3, 64)])))
    else:
        groups.append(("clamped_edge", edge(0, 0, 256)))
        groups.append(("loaded_edge", edge(0, 1, 256)))
        groups.append(("corners", np.concatenate(
            [corner(0, ci, cj, 4) for ci in (0, 1) for cj in (0, 1)])))
    seen = set()
    idx, stratum = [], []
    for name, g in groups:
        for v in np.asarray(g, dtype=np.int64):
            if int(v) not in seen:
                seen.add(int(v))
                idx.append(int(v))
                stratum.append(name)
    order = np.argsort(idx, kind="stable")
    return np.asarray(idx, dtype=np.int64)[order], [stratum[k] for k in order]


def main(which: str):
    if which == "lshape":
        prob, name, label = W.l_shape(9), "lshape9_samples.json", "l_shape(level=9)"
    else:
        prob, name = W.cantilever_traction(LEVEL), "level10_traction_samples.json"
        label = "cantilever_traction(level=10)"
    u, f = fem.solve_problem(prob)          # both in QTT order (first core fastest)
    rng = np.random.default_rng(SEED)
    idx, stratum = _samples(prob, which, u.size, rng)
    out = {
        "workload": label,
        "source": "oracle.fem.solve_problem (sparse direct, FP64)",
        "ndofs": int(u.size),
        "seed": SEED,
        "index": [int(i) for i in idx],
        "stratum": stratum,
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
