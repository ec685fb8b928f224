"""Writes the oracle's exact rounding of the benchmarked step at its full
shape (headline_step_level10.json): the level-10 traction operator of the
oracle's QTT assembly (21 cores), x = random_tt_cores(5, [2]*21,
capped_ranks(.., 64)), the product K x (ranks up to 1600) and its exact TT
rounding to (eps 1e-8, rank 64).  Stored: ||K x||, the relative error
||round(K x) - K x|| / ||K x|| and the ranks of the rounded train.

Calls only the oracle and the shared workload generator; about a minute
of LAPACK work on the host.  Run from the repository root:

    python tests/golden/make_step_reference.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import assembly as A  # noqa: E402
from oracle import qtt as T  # noqa: E402


def diff_norm(a, b):
    """||a - b|| through the orthogonalised difference train."""
    return float(np.linalg.norm(T.orthogonalize_left(T.add(a, b, coeffs=[1.0, -1.0]))[-1]))


def main():
    Kq, _ = A.assemble_qtt(W.cantilever_traction(10))
    modes = [2] * 21
    x = W.random_tt_cores(5, modes, W.capped_ranks(modes, 64))
    Kx = T.matvec(Kq, x)
    nrm = float(np.linalg.norm(T.orthogonalize_left(Kx)[-1]))
    y, info = T.tt_round(Kx, 1e-8, 64, return_info=True)
    out = {
        "workload": "cantilever_traction(level=10) operator, x = random_tt_cores(5, [2]*21, "
                    "capped_ranks([2]*21, 64)), y = tt_round(K x, 1e-8, 64)",
        "source": "oracle.assembly.assemble_qtt, oracle.qtt.matvec, oracle.qtt.tt_round",
        "norm_Kx": nrm,
        "exact_round_err_rel": diff_norm(y, Kx) / nrm,
        "discarded_sigma_rel": info["err"] / nrm,
        "exact_round_ranks": T.ranks(y),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "headline_step_level10.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
