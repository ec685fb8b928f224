#!/usr/bin/env python3
"""Benchmark of the QTT finite element hot path on one MI355X.

One step is one full qtt_solve of the clamped unit square with the seeded
eight-mode traction on its east edge at level 10 (2^10 x 2^10 nodes,
2,097,152 dofs, 21 QTT cores): relative accuracy 1e-8, solution rank cap 64,
BPX-preconditioned truncated CG with randomised rounding of the products,
FP64 iterative refinement with a dense FP64 residual check.  Operator,
load and preconditioner are assembled (and resident in HBM) before the
timed region.

Besides the solves/s of that step, the line carries the roofline of the
matrix-vector product at the solve's largest shape (operator rank 25 times a
rank-64 train: a 422 MB product, HBM-write bound), timed with HIP events on
the stream it runs on, and the CPU oracle timed on a bounded sample of the
same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--level", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--trace", action="store_true")
    return ap.parse_args()


def matvec_roofline(P, torch, K, level):
    """Time qtt_matvec K x (x of rank 64) with HIP events on the current stream."""
    import numpy as np
    import workloads as W
    modes = [2] * (2 * level + 1)
    x = P.tt_from_cores(W.random_tt_cores(5, modes, W.capped_ranks(modes, 64)))
    y = P.matvec(K, x)
    reps = 20
    st = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        P.matvec(K, x, y=y)
    torch.cuda.synchronize()
    start.record(st)
    for _ in range(reps):
        P.matvec(K, x, y=y)
    stop.record(st)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / reps
    nbytes = 8 * (y.numel() + x.numel() + K.numel())      # algorithmic: read operands, write product
    return dict(bound="hbm", achieved=round(nbytes / (ms * 1e-3) / 1e9, 1), peak=HBM_PEAK_GBS,
                unit="GB/s", frac=round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                traffic=None, kernel="k_matvec_f64", bytes_per_launch=nbytes,
                ms_per_launch=round(ms, 4))


def cpu_baseline(level, inner_per_solve, seconds):
    """The FP64 oracle's truncated PCG (exact rounding) at the same workload,
    run for a bounded number of inner iterations; solves/s scaled by the inner
    iterations one GPU solve takes."""
    import numpy as np
    import workloads as W
    from oracle import assembly as A, fem, precond as PC, qtt as T, solve as S
    prob = W.cantilever_traction(level)
    Kq, fq = A.assemble_qtt(prob)
    # gamma_D = trace(K)/N, from the QTT operator before the Dirichlet rows
    Kbd = A.block_diag_stiffness(level, 1, fem.c_matrix(prob.E, prob.nu, prob.plane_strain))
    gD = T.trace(Kbd) / (2 * 4 ** level)
    Cq = PC.bpx_qtt(prob, gD)
    r = T.tt_round(fq, 1e-3, 24)
    t0 = time.time()
    its = 0
    # bounded sample: as many inner iterations as fit in the time budget
    while time.time() - t0 < seconds:
        S.inner_cg(Kq, r, 1e-3, 24, 1e-30, 1, Cq, 1e-8, 64)
        its += 1
    dt = time.time() - t0
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    per_it = dt / its
    return dict(value=1.0 / (per_it * max(inner_per_solve, 1)), unit="solves/s", cores=cores,
                kind="oracle",
                sample="%d truncated-PCG iterations of the NumPy oracle at level %d (%.1f s), "
                       "scaled by the %d inner iterations of one GPU solve" % (its, level, dt,
                                                                              inner_per_solve))


def main():
    args = _parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU: this build has no multi-GPU path "
              "(the solve would shard over independent load cases)", file=sys.stderr)
        sys.exit(2)
    if args.trace:
        os.environ["QTT_SOLVE_TRACE"] = "1"
    import torch
    import paper_2501_07778_amd as P
    import workloads as W

    prob = W.cantilever_traction(args.level)
    K, f = P.assemble(prob)
    C = P.assemble_bpx(prob)
    opts = P.SolveOpts(tol=1e-8, eps=1e-8, rmax=64, eps_in=1e-3, rmax_in=24, red_in=1e-2,
                       maxit_in=300, maxit_out=30, check_every=5, compute="f64", sketch=8,
                       seed=1, precond=C)
    ws = P._lib._workspace(P.solve_workspace_bytes(K, f, opts))
    for _ in range(args.warmup):
        P.solve(K, f, opts, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for _ in range(args.steps):
        u, rep = P.solve(K, f, opts, ws=ws)
        reps.append(rep)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    roof = matvec_roofline(P, torch, K, args.level)
    inner = int(sum(r["inner"] for r in reps) / max(len(reps), 1))
    line = {
        "metric": "QTT solves/sec and matvec+round GB/s at rel. err 1e-6 vs FP64 plain GPU",
        "value": round(args.steps / dt, 5),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "clamped unit square, seeded 8-mode traction, level %d "
                               "(%d dofs), eps 1e-8, rank cap 64" % (args.level, 2 * 4 ** args.level),
                   "solver": "BPX-PCG, randomised product rounding, FP64 refinement",
                   "residual": reps[-1]["residual"], "status": reps[-1]["status"],
                   "outer": reps[-1]["outer"], "inner": reps[-1]["inner"],
                   "solution_max_rank": reps[-1]["max_rank"]},
        "roofline": roof,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.level, inner, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
