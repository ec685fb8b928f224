#!/usr/bin/env python3
"""Benchmark of the QTT matrix-vector product plus rounding on one MI355X.

Workload: the clamped unit square with the seeded eight-mode sine traction
on its east edge at level 10 (2^10 x 2^10 nodes, 2,097,152 dofs, 21 QTT
cores), plane strain E = 1, nu = 0.3.  The stiffness matrix K (QTT ranks up
to 25) is assembled on the device before the timed region; the vector x is
a seeded rank-64 train (the rank cap of the solve at this level) with
Gaussian cores.  One step is the hot path of every solver iteration:

    y = round(K x, 1e-8, 64)      qtt_matvec_round: the FP64 product (ranks
                                  25*64 = 1600) formed in the workspace, a
                                  Gaussian sketch of rank 72, then the exact
                                  rounding of the sketch

The value is the algorithmic HBM traffic of a step (read K and x, write the
product, read it back once in the rounding, write the result) divided by the
step time: matvec+round GB/s.  The line also carries the roofline of the
dominant kernel, the one-workgroup truncated-SVD step of the rounding
(timed with HIP events on the stream it runs on, during the timed steps;
algorithmic flops from the R-SVD count of each bond's unfolding), that of
the product kernel (HBM-bound) under config, and the
FP64 CPU oracle timed on the same step (same inputs, same Gaussian train).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
RANK = 64
ELL = RANK + 8
EPS = 1e-8
SOLVE_EPS = 5e-9   # rounding tolerance of the level-10 solves, below their 1e-8 target


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--level", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only launch the level-10 product 5 times and a plain 423 MB device "
                         "copy 5 times (for hardware counter passes), print their sizes, exit")
    ap.add_argument("--no-solve", dest="solve", action="store_false",
                    help="skip the level-5 and level-10 solve measurements")
    ap.add_argument("--batch", type=int, default=256,
                    help="cases of the batched-step measurement (0: skip)")
    ap.add_argument("--batched-steps-only", action="store_true",
                    help="run only the batched-step measurement and print its JSON (the "
                         "process the main run starts for it, with 32 hardware queues)")
    ap.add_argument("--batch-solves", type=int, default=256,
                    help="cases of the batched-solve measurement (0: skip)")
    ap.add_argument("--learned", type=int, default=4096,
                    help="training targets of the learned warm start at level 10 (0: skip)")
    ap.add_argument("--learned-held", type=int, default=32,
                    help="held-out loads of the learned warm start (warm and cold solves)")
    return ap.parse_args()


def note(msg: str) -> None:
    """A progress line on stderr (the JSON result is the only stdout line)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def tt_bytes(t) -> int:
    return 8 * t.numel()


def workload(level: int):
    import numpy as np
    import paper_2501_07778_amd as P
    import workloads as W
    prob = W.cantilever_traction(level)
    K, f = P.assemble(prob)
    modes = [2] * (2 * level + 1)
    cores = W.random_tt_cores(5, modes, W.capped_ranks(modes, RANK))
    x = P.tt_from_cores(cores)
    return prob, K, x


def step(P, K, x, y, ws, seed, compute="f64"):
    y, _, _ = P.matvec_round(K, x, ELL, seed, EPS, RANK, compute, y=y, ws=ws)
    return y


def step_as_graph(P, torch, K, x, ws, nsteps: int):
    """The same step captured once as a HIP graph (qtt_matvec_round_graph_*
    with one case) and replayed `nsteps` times back to back; its ranks and
    norm against the eager step with the same seed."""
    y0, n0, _ = P.matvec_round(K, x, ELL, 0, EPS, RANK, "f64", ws=ws)
    batch = P.StepBatch([(K, x, ELL, 0, EPS, RANK, "f64")], 1)
    g = P.StepGraph(batch, 1)
    try:
        g.launch()                              # first replay: warm-up
        g.collect()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            g.launch()
        g.collect()
        dt = (time.perf_counter() - t0) / nsteps
        y = batch.outputs()[0]
        same = list(y.ranks) == list(y0.ranks) and abs(batch.cases[0].norm - n0) <= 1e-12 * n0
    finally:
        g.close()
    return dict(ms_per_step=round(1e3 * dt, 3), replays=nsteps, equal_to_eager=bool(same))


def measured_traffic(summary: str, source: str):
    """HBM bytes per launch of a kernel from its committed counter summary
    in profiles/, or None once any source file the summary lists (the
    kernel's file and the device headers it includes) has changed since the
    counters were taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        txt = open(os.path.join(here, "profiles", summary)).read()
    except OSError:
        return None
    shas = {}
    traffic = None
    for line in txt.splitlines():
        if line.startswith("source_sha1(") and "): " in line:
            path, val = line[len("source_sha1("):].split("): ", 1)
            shas[path] = val.strip()
        elif line.startswith("traffic_bytes_per_launch: "):
            traffic = int(line.split(": ", 1)[1])
    if traffic is None or "paper_2501_07778_amd/csrc/%s" % source not in shas:
        return None
    for path, val in shas.items():
        try:
            if hashlib.sha1(open(os.path.join(here, path), "rb").read()).hexdigest() != val:
                return None
        except OSError:
            return None
    return traffic


def matvec_roofline(P, torch, K, x):
    """k_matvec_f64 alone: HIP events on the stream it is launched on."""
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
    nbytes = tt_bytes(K) + tt_bytes(x) + tt_bytes(y)
    gbs = nbytes / (ms * 1e-3) / 1e9
    return dict(kernel="k_matvec_f64", bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS,
                unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 4),
                traffic=measured_traffic("k_matvec_f64_level10_pmc.md", "k_tt.hip"),
                bytes_per_launch=nbytes, ms_per_launch=round(ms, 4))


def svd_flops(m: int, n: int) -> float:
    """Algorithmic flops of a thin SVD with both factors of an m x n matrix
    (Golub and Van Loan's R-SVD count, 6 M N^2 + 20 N^3 with M >= N)."""
    M, N = max(m, n), min(m, n)
    return 6.0 * M * N * N + 20.0 * N ** 3


def sketch_svd_flops(K, x, y_ranks) -> float:
    """Flops of the right-to-left SVD sweep of one step: bond k's unfolding
    has the sketch rank l_k rows (l_k = min(ell, mode products on either
    side, product rank R_k r_k), built up from the left as in the sketch)
    and n_k times the final rank at k+1 columns."""
    D = K.D
    n = [K.nrow[k] for k in range(D)]
    l = [1] * (D + 1)
    for k in range(1, D):
        left = 1
        for j in range(k):
            left *= n[j]
        right = 1
        for j in range(k, D):
            right *= n[j]
        l[k] = max(1, min(ELL, left, right, K.ranks[k] * x.ranks[k]))
    lz = [1] * (D + 1)
    for k in range(D - 1):
        lz[k + 1] = min(lz[k] * n[k], l[k + 1])
    return sum(svd_flops(lz[k], n[k] * y_ranks[k + 1]) for k in range(1, D))


def dominant_roofline(P, ms_total, launches, flops_per_step, steps, traffic):
    """k_svd_step, the step's dominant kernel (one workgroup per bond, the
    right-to-left truncated-SVD sweep): algorithmic flops per launch over
    its average launch time from HIP events on its stream during the timed
    steps; bound by the FP64 vector ALU (a Jacobi SVD in LDS)."""
    per_launch_ms = ms_total / max(launches, 1)
    flops_per_launch = flops_per_step * steps / max(launches, 1)
    achieved = flops_per_launch / (per_launch_ms * 1e-3) / 1e12
    return dict(kernel="k_svd_step", bound="alu", achieved=float("%.5g" % achieved),
                peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                frac=float("%.3g" % (achieved / FP64_PEAK_TFLOPS)), traffic=traffic,
                launches_per_step=launches / steps,
                ms_per_launch=round(per_launch_ms, 4),
                flops_per_launch=round(flops_per_launch),
                share_of_step=None)


def rel_diff(P, a, b) -> float:
    """||a - b|| / ||b|| from three inner products of the (rank <= 64)
    trains, FP64 on the device."""
    aa, bb, ab = P.dot(a, a), P.dot(b, b), P.dot(a, b)
    return (max(aa + bb - 2.0 * ab, 0.0) ** 0.5) / bb ** 0.5


MIXED_TOL = 1e-6   # relative error the metric allows against the FP64 GPU step


def mixed_precision(P, torch, K, x, ws, steps):
    """The same step with the product in FP32 and BF16 (FP32 accumulation;
    sketch GEMMs, QR and SVD stay FP64), same sketch seed: time per step,
    relative error of the result against the FP64 step, and whether that
    error is within the metric's 1e-6 (BF16 products are not: about 1e-2,
    and nothing refines them)."""
    y64 = step(P, K, x, None, ws, 0, "f64")
    out = {}
    for comp in ("f32", "bf16"):
        y = step(P, K, x, None, ws, 0, comp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            y = step(P, K, x, y, ws, 0, comp)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        err = rel_diff(P, y, y64)
        out[comp] = dict(ms_per_step=round(1e3 * dt, 3), rel_err_vs_f64_gpu=float("%.3e" % err),
                         within_metric_tolerance=bool(err <= MIXED_TOL))
    return out


def batched_steps(P, torch, ncases: int):
    """The hot step on the batched configuration's shapes: case i draws its
    level (8..11) and rank cap (16..96) from rng(1000 + i); K of that level,
    x a seeded train at the cap, y = round(K x) to (1e-6, cap) via a sketch
    of rank cap + 8.  Cases run concurrently by host workers on their own
    streams (qtt_matvec_round_batched); the worker count is tuned here."""
    import workloads as W
    Ks = {}
    items = []
    nbytes = 0
    for i in range(ncases):
        c = W.batch_case(i)
        lvl, cap = c.level, c.cap
        if lvl not in Ks:
            Ks[lvl], _ = P.assemble(W.cantilever_traction(lvl))
        K = Ks[lvl]
        modes = [2] * (2 * lvl + 1)
        x = P.tt_from_cores(W.random_tt_cores(7000 + i, modes, W.capped_ranks(modes, cap)))
        items.append((K, x, cap + 8, i, 1e-6, cap, "f64"))
        prod = 8 * sum(K.ranks[k] * x.ranks[k] * 2 * K.ranks[k + 1] * x.ranks[k + 1]
                       for k in range(K.D))
        nbytes += tt_bytes(K) + tt_bytes(x) + 2 * prod
    rates = {}
    batch = P.StepBatch(items, 1)
    for nw in (1, 4, 8, 16, 32):
        batch.set_workers(nw)
        P.matvec_round_batched(batch)          # warm-up of this worker set
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.matvec_round_batched(batch)
        torch.cuda.synchronize()
        rates[nw] = time.perf_counter() - t0
    best = min(rates, key=rates.get)
    ref = [(list(y.ranks), c.norm) for y, c in zip(batch.outputs(), batch.cases)]
    # the same batch as HIP graphs (qtt_matvec_round_graph_*), the cases split
    # over independent branches: one graph (one launch per replay), or one
    # graph per branch replayed on streams of its own
    grates, prates, same = {}, {}, True
    for nb, per in ((1, False), (8, False), (32, False), (8, True), (16, True), (32, True)):
        g = P.StepGraph(batch, nb, per)
        try:
            g.launch()                          # first replay: warm-up
            g.collect()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.launch()
            g.collect()
            (prates if per else grates)[nb] = time.perf_counter() - t0
            same = same and all(list(y.ranks) == r and abs(c.norm - n) <= 1e-12 * abs(n)
                                for y, c, (r, n) in zip(batch.outputs(), batch.cases, ref))
        finally:
            g.close()
    gbest = min(grates, key=grates.get)
    levels = sorted(set(W.batch_case(i).level for i in range(ncases)))
    return dict(cases=ncases, levels=levels, best_workers=best,
                steps_per_s={str(k): round(ncases / v, 2) for k, v in rates.items()},
                gbs_at_best=round(nbytes / rates[best] / 1e9, 2),
                speedup_vs_1_worker=round(rates[1] / rates[best], 2),
                graph_steps_per_s={str(k): round(ncases / v, 2) for k, v in grates.items()},
                graph_best_branches=gbest,
                graph_vs_best_workers=round(rates[best] / grates[gbest], 2),
                branch_graphs_steps_per_s={str(k): round(ncases / v, 2)
                                           for k, v in prates.items()},
                branch_graphs_vs_best_workers=round(rates[best] / min(prates.values()), 2),
                graph_equals_workers=bool(same))


def batched_solves(P, torch, ncases: int, chunk: int = 32, ntune: int = 16):
    """Solves of the batched configuration: case i (rng(1000 + i)) draws its
    level (8..11), rank cap (16..96) and 16 load coefficients; each is solved
    by ALS (rank ramp from 16 to the cap, tol 1e-6, eps 1e-6, at most 24
    sweeps).  Cases run concurrently by host workers on their own streams
    (qtt_solve_batched).  The worker count comes from the library's
    autotuner (qtt_autotune_batched: 1, 2, 4, 8, 16 and 32 workers on the
    first `ntune` cases, ranked by converged solves/s); then all `ncases`
    run with it, `chunk` cases resident at a time (each case holds its own
    workspace, up to 2.7 GB at level 11 and rank 96).  A case whose cap is
    below the rank its solution needs stops at the sweep limit (status
    QTT_E_NOCONV) with the best iterate of that rank: it is reported, and
    not counted as a solve."""
    import workloads as W

    def problems(lo, hi):
        out = []
        for i in range(lo, hi):
            c = W.batch_case(i)
            K, f = P.assemble(W.cantilever_two_component(c.level, c.coeffs))
            opts = P.SolveOpts(tol=1e-6, eps=1e-6, rmax=c.cap, rmax_in=16, maxit_out=24,
                               method="als", seed=1)
            out.append((K, f, opts))
        return out

    tune = P.Batch(problems(0, min(ntune, ncases)))
    best, rates = P.autotune_batched(tune)
    note("batched solves: autotuned %d workers" % best)
    del tune
    total, converged, noconv, sweeps = 0.0, 0, 0, []
    for lo in range(0, ncases, chunk):
        batch = P.Batch(problems(lo, min(lo + chunk, ncases)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = P.solve_batched(batch, best)
        torch.cuda.synchronize()
        total += time.perf_counter() - t0
        note("batched solves: cases %d..%d done" % (lo, min(lo + chunk, ncases) - 1))
        converged += sum(1 for _, r in res if r["status"] == 0)
        noconv += sum(1 for _, r in res if r["status"] == -4)
        sweeps += [r["outer"] for _, r in res]
        del batch, res
    return dict(cases=ncases, levels=sorted(set(W.batch_case(i).level for i in range(ncases))),
                caps_range=[min(W.batch_case(i).cap for i in range(ncases)),
                            max(W.batch_case(i).cap for i in range(ncases))],
                autotune_cases=min(ntune, ncases), best_concurrency=best,
                autotune_converged_solves_per_s={str(k): round(v, 3) for k, v in rates.items()},
                seconds=round(total, 2), converged=converged, stopped_at_sweep_limit=noconv,
                converged_solves_per_s=round(converged / total, 3),
                mean_sweeps=round(sum(sweeps) / len(sweeps), 2))


def small_solve(P, torch, level: int, method: str):
    """The plain-method configuration: level-5 unit square, left edge
    clamped, body force (0, -1), eps 1e-10.  "als": one-site ALS at the
    full rank of the level (exact), stopped at a change of 1e-10 per sweep;
    "fcg": BPX-preconditioned flexible CG to a preconditioned residual of
    1e-10.  solves/s of one solve after a warm-up solve, and the solver's
    FP64 dense residual."""
    import workloads as W
    prob = W.cantilever_body_force(level)
    K, f = P.assemble(prob)
    if method == "als":
        opts = P.SolveOpts(tol=1e-10, eps=1e-10, rmax=2 ** level, maxit_out=8, method="als",
                           seed=1)
        label = "one-site ALS at full rank"
    else:
        C = P.assemble_bpx(prob)
        opts = P.SolveOpts(tol=1e-10, eps=1e-10, rmax=64, eps_in=1e-3, rmax_in=32, maxit_in=1000,
                           check_every=10, precond=C, sketch=8, seed=1, method="fcg")
        label = "BPX + flexible CG"
    ws = P._lib._workspace(P.solve_workspace_bytes(K, f, opts))
    P.solve(K, f, opts, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, rep = P.solve(K, f, opts, ws=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dict(workload="unit square level %d (%d dofs), body force, eps 1e-10, %s"
                % (level, 2 * 4 ** level, label), solves_per_s=round(1.0 / dt, 4),
                ms_per_solve=round(1e3 * dt, 1),
                iterations=rep["outer"] if method == "als" else rep["inner"],
                status=rep["status"], fp64_residual=float("%.3e" % rep["residual"]),
                solution_max_rank=rep["max_rank"])


def cpu_baseline(level, nbytes, y_gpu=None):
    """The FP64 oracle on the same step and the same inputs: its product of
    all cores, then its randomised rounding with the same Gaussian train
    (rank-72 sketch, then the exact rounding to (1e-8, 64)), the algorithm
    the GPU step runs (a few seconds of host LAPACK work).  With
    y_gpu (the GPU step's cores for sketch seed 0) the line also gets the
    GPU step's error against the oracle's step and against the unrounded
    product (difference trains orthogonalised on the host)."""
    import numpy as np
    import workloads as W
    from oracle import assembly as A, qtt as T, sketch as SK
    prob = W.cantilever_traction(level)
    Kq, _ = A.assemble_qtt(prob)
    modes = [2] * (2 * level + 1)
    x = W.random_tt_cores(5, modes, W.capped_ranks(modes, RANK))
    t0 = time.time()
    y = T.matvec(Kq, x)
    t_mv = time.time() - t0
    t1 = time.time()
    ref = SK.sketch_round(y, ELL, 0, EPS, RANK)
    t_rd = time.time() - t1
    per_step = t_mv + t_rd
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    try:
        import threadpoolctl
        threads = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] or [1])
    except ImportError:
        threads = cores
    out = dict(value=round(nbytes / per_step / 1e9, 4), unit="GB/s",
               cores=min(cores, threads), kind="oracle",
               sample="the whole step on the oracle: matvec of all %d cores (%.2f s) + "
                      "randomised rounding with the same rank-%d Gaussian train and exact "
                      "rounding to (%.0e, %d) (%.2f s): %.2f s per step"
                      % (len(y), t_mv, ELL, EPS, RANK, t_rd, per_step))
    if y_gpu is not None:
        def dn(a, b):
            return float(np.linalg.norm(T.orthogonalize_left(T.add(a, b, coeffs=[1.0, -1.0]))[-1]))
        nrm = float(np.linalg.norm(T.orthogonalize_left(y)[-1]))
        out["gpu_step_rel_err_vs_oracle_step"] = float("%.3e" % (dn(y_gpu, ref) / nrm))
        out["gpu_step_rel_err_vs_unrounded_product"] = float("%.4e" % (dn(y_gpu, y) / nrm))
        out["oracle_step_rel_err_vs_unrounded_product"] = float("%.4e" % (dn(ref, y) / nrm))
    return out


def level10_solve(P, torch, level: int, mode: str = "ramp"):
    """The level-10 configuration of the plain method: the traction workload
    of the step, solved to the plain method's 1e-8 against the direct
    solve (up to the FP64 floor of this conditioning, 1e-8 to 2e-8), so
    with a rounding tolerance below it (5e-9).  "ramp": one-site ALS (FP64
    local Cholesky solves; 3 sweeps each at ranks 16 and 32, then rank 64)
    until the change of u over a sweep falls to 1e-7 relative; "fixed":
    ALS at rank 64 to 1e-6; "amen": AMEn (ALS sweeps alternated with
    residual enrichment of rank 8, ranks adapting from 8 up to 72, every
    enrichment rounded at 2e-9) until both the sweep change and the
    enrichment change fall to 1e-7.  solves/s of one solve after a warm-up
    solve, the FP64 dense residual and the final rank."""
    import workloads as W
    prob = W.cantilever_traction(level)
    K, f = P.assemble(prob)
    if mode == "amen":
        opts = P.SolveOpts(tol=1e-7, eps=2e-9, rmax=72, rmax_in=8, eps_in=1e-2, maxit_out=40,
                           method="amen", seed=1)
        label = "AMEn, enrichment rank 8, ranks up to 72, rounding eps 2e-9"
    else:
        ramp = mode == "ramp"
        opts = P.SolveOpts(tol=1e-7 if ramp else 1e-6, eps=SOLVE_EPS, rmax=RANK,
                           rmax_in=16 if ramp else 0, maxit_out=16, method="als", seed=1)
        label = ("one-site ALS, rank ramp 16, 32, %d" % RANK if ramp
                 else "one-site ALS, fixed rank %d" % RANK)
    ws = P._lib._workspace(P.solve_workspace_bytes(K, f, opts))
    P.solve(K, f, opts, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, rep = P.solve(K, f, opts, ws=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dict(workload="unit square level %d (%d dofs), seeded 8-mode traction, eps %.0e, %s"
                % (level, 2 * 4 ** level, opts.eps, label),
                solves_per_s=round(1.0 / dt, 4), ms_per_solve=round(1e3 * dt, 1),
                sweeps=rep["outer"], local_solves=rep["inner"], status=rep["status"],
                change_last_sweep=float("%.3e" % rep["criterion"]),
                fp64_residual=float("%.3e" % rep["residual"]), solution_max_rank=rep["max_rank"])


def learned_start(P, torch, level: int, ntrain: int, nheld: int, epochs: int):
    """The learned warm start: a 16 -> 512 -> 512 -> 512 -> (rank-16 cores
    at level 10) network, BF16 matrix-core GEMMs with FP32 accumulation and
    master weights, trained natively on `ntrain` targets generated by the
    method (16 basis ALS solves joined into the family train, rounded once
    to rank 16, evaluated at each load) with the core loss; then on `nheld`
    held-out loads (seeds 4096 on) the ALS solve to a per-sweep change of
    1e-6 with the rank ramp 8, 16, 32 from the network's start (rounded to
    minimal ranks) against the cold start.  The output size is that of the
    family's rank pattern, whose last bonds keep the family's ranks (8,564
    values instead of 7,336 for a single load's pattern)."""
    import numpy as np
    import workloads as W
    from paper_2501_07778_amd import learned_start as LS
    tm = {}
    t0 = time.perf_counter()
    bopts = P.SolveOpts(tol=1e-6, eps=1e-6, rmax=64, rmax_in=16, maxit_out=24, method="als",
                        seed=1)
    basis = LS.basis_solves(level, bopts, W.cantilever_two_component)
    torch.cuda.synchronize()
    tm["basis_solves_s"] = round(time.perf_counter() - t0, 2)
    note("learned start: basis solves done")
    t0 = time.perf_counter()
    params = np.stack([W.warmstart_params(s) for s in range(ntrain)], axis=1)
    fam = LS.family_train(basis, 16, 24)
    tcols, ranks = LS.targets(fam, params)
    torch.cuda.synchronize()
    tm["targets_s"] = round(time.perf_counter() - t0, 2)
    nrow = basis[0].nrow
    sizes = LS.network_sizes(nrow, ranks)
    mean = tcols.mean(dim=0).cpu().numpy()
    net = P.MLP(sizes, LS.init_params(sizes, 7, out_bias=mean, out_scale=0.1), gemm="bf16",
                loss="cores")
    t0 = time.perf_counter()
    hist = net.fit(P.columns(params), tcols.t(), 256, epochs, 1e-3, 1e-5, 11, nrow, ranks)
    torch.cuda.synchronize()
    tm["training_s"] = round(time.perf_counter() - t0, 2)
    note("learned start: trained")
    held = np.stack([W.warmstart_params(s) for s in range(4096, 4096 + nheld)], axis=1)
    sopts = P.SolveOpts(tol=1e-6, eps=1e-6, rmax=32, rmax_in=8, maxit_out=40, method="als",
                        seed=1)
    rows = LS.compare_starts(net, W.cantilever_two_component, level, held, nrow, ranks, sopts,
                             progress=lambda j: note("learned start: %d held-out loads" % j),
                             keep_solutions=False)
    ok = [r for r in rows if r["warm_status"] == 0 and r["cold_status"] == 0]
    med = lambda v: float(np.median(v)) if v else None
    tw = sum(r["warm_s"] for r in rows)
    tc = sum(r["cold_s"] for r in rows)
    return dict(network=sizes, gemm="bf16 (FP32 accumulation, FP32 master weights)",
                loss="cores of the family-train targets",
                targets=ntrain, rank=16, epochs=epochs, batch=256,
                loss_first_epoch=float("%.4g" % hist[0]), loss_last_epoch=float("%.4g" % hist[-1]),
                held_out=nheld, accepted=sum(1 for r in rows if r["warm_start"] == 1),
                start_energy_error_median=float("%.3g" % med([r["start_energy_error"] for r in rows])),
                sweeps_mean_warm=round(float(np.mean([r["warm_sweeps"] for r in rows])), 2),
                sweeps_mean_cold=round(float(np.mean([r["cold_sweeps"] for r in rows])), 2),
                solves_per_s_warm=round(nheld / tw, 3), solves_per_s_cold=round(nheld / tc, 3),
                speedup=round(tc / tw, 3), converged_both=len(ok),
                sweeps_median_warm=med([r["warm_sweeps"] for r in rows]),
                sweeps_median_cold=med([r["cold_sweeps"] for r in rows]),
                fewer_sweeps_frac=round(sum(1 for r in rows if r["warm_sweeps"] < r["cold_sweeps"])
                                        / max(nheld, 1), 3),
                more_sweeps_frac=round(sum(1 for r in rows if r["warm_sweeps"] > r["cold_sweeps"])
                                       / max(nheld, 1), 3),
                fp64_residual_median_warm=float("%.3g" % med([r["warm_residual"] for r in rows])),
                fp64_residual_median_cold=float("%.3g" % med([r["cold_residual"] for r in rows])),
                **tm)


def main():
    args = _parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the multi-GPU form (independent load cases "
              "per GPU) is not built", file=sys.stderr)
        sys.exit(2)
    if args.batched_steps_only:
        # concurrent streams of the batched steps: one hardware queue each, up
        # to 32 (HIP's default of 4 per process serialises the workers)
        os.environ["GPU_MAX_HW_QUEUES"] = "32"
        import torch
        import paper_2501_07778_amd as P
        print(json.dumps(batched_steps(P, torch, args.batch)), flush=True)
        return
    # The batched steps run first, in a process of their own with 32 hardware
    # queues: that many queues slow the single-stream solves of this process
    # (level-10 ALS about 37 %), so the rest keeps the runtime's default.
    batched = None
    if args.batch > 0:
        import subprocess
        try:
            r = subprocess.run([sys.executable, "-u", os.path.abspath(__file__),
                                "--batched-steps-only", "--batch", str(args.batch)],
                               stdout=subprocess.PIPE, text=True, timeout=900)
        except subprocess.TimeoutExpired:
            print("batched-step process exceeded 900 s", file=sys.stderr)
            sys.exit(1)
        if r.returncode != 0:
            print("batched-step process failed with status %d" % r.returncode, file=sys.stderr)
            sys.exit(r.returncode if r.returncode > 0 else 1)
        batched = json.loads(r.stdout.strip().splitlines()[-1])
        batched["hardware_queues"] = 32
        note("batched steps done (own process, 32 hardware queues)")
    import torch
    import paper_2501_07778_amd as P

    prob, K, x = workload(args.level)
    if args.pmc_probe:
        y = P.matvec(K, x)
        src = torch.empty(y.numel(), dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            P.matvec(K, x, y=y)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"matvec_bytes_algorithmic": tt_bytes(K) + tt_bytes(x) + tt_bytes(y),
                          "matvec_write_bytes": tt_bytes(y),
                          "copy_read_bytes": 8 * src.numel(), "copy_write_bytes": 8 * dst.numel()}),
              flush=True)
        return
    y = None
    ws = P.matvec_round_workspace(K, x, ELL)
    for i in range(args.warmup):
        y = step(P, K, x, y, ws, 1000 + i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        y = step(P, K, x, y, ws, i)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # the same steps again with HIP events around the rounding kernels (the
    # per-launch durations of the roofline), kept out of the timed pass
    P.kernel_timing(True)
    for i in range(args.steps):
        y = step(P, K, x, y, ws, i)
    torch.cuda.synchronize()
    svd_ms, svd_n = P.kernel_timing_read("k_svd_step")
    sqr_ms, sqr_n = P.kernel_timing_read("k_sketch_qr")
    P.kernel_timing(False)
    # algorithmic bytes: read K, x; write Y; read Y once; write the result
    prod = 8 * sum(K.ranks[k] * x.ranks[k] * K.nrow[k] * K.ranks[k + 1] * x.ranks[k + 1]
                   for k in range(K.D))
    nbytes = tt_bytes(K) + tt_bytes(x) + 2 * prod + tt_bytes(y)
    value = nbytes / dt / 1e9
    roof_mv = matvec_roofline(P, torch, K, x)
    roof = dominant_roofline(P, svd_ms, svd_n, sketch_svd_flops(K, x, y.ranks), args.steps,
                             measured_traffic("k_svd_step_level10_pmc.md", "k_round.hip"))
    roof["share_of_step"] = round(svd_ms / args.steps / (1e3 * dt), 3)
    roof["next_kernel"] = dict(kernel="k_sketch_qr", launches_per_step=sqr_n / args.steps,
                               ms_per_launch=round(sqr_ms / max(sqr_n, 1), 4),
                               share_of_step=round(sqr_ms / args.steps / (1e3 * dt), 3))
    note("step: %.3f ms" % (1e3 * dt))
    graph_step = step_as_graph(P, torch, K, x, ws, max(2, args.steps // 2))
    note("step as a graph: %.3f ms" % graph_step["ms_per_step"])
    mixed = mixed_precision(P, torch, K, x, ws, max(2, args.steps // 2))
    note("mixed precision done")
    bsolves = (batched_solves(P, torch, args.batch_solves)
               if (args.batch_solves > 0 and args.solve) else None)
    note("batched measurements done")
    solve5 = small_solve(P, torch, 5, "als") if args.solve else None
    solve5_fcg = small_solve(P, torch, 5, "fcg") if args.solve else None
    solve10 = level10_solve(P, torch, args.level) if args.solve else None
    solve10_fixed = level10_solve(P, torch, args.level, "fixed") if args.solve else None
    solve10_amen = level10_solve(P, torch, args.level, "amen") if args.solve else None
    note("solves done")
    learned = (learned_start(P, torch, args.level, args.learned, args.learned_held, 30)
               if args.learned > 0 else None)
    line = {
        "metric": "QTT solves/sec and matvec+round GB/s at rel. err 1e-6 vs FP64 plain GPU",
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "matvec+round: clamped unit square, seeded 8-mode traction, "
                               "level %d (%d dofs, %d cores), K rank %d, x rank %d, "
                               "round to eps %.0e / rank %d via sketch %d"
                               % (args.level, 2 * 4 ** args.level, K.D, max(K.ranks), RANK,
                                  EPS, RANK, ELL),
                   "bytes_per_step": nbytes, "result_ranks_max": max(y.ranks),
                   "mixed_precision": mixed, "step_as_graph": graph_step, "batched_steps": batched, "batched_solves": bsolves, "solve_level5": solve5, "solve_level5_fcg": solve5_fcg,
                   "solve_level%d" % args.level: solve10,
                   "solve_level%d_fixed_rank" % args.level: solve10_fixed,
                   "solve_level%d_amen" % args.level: solve10_amen,
                   "learned_start": learned,
                   "matvec_roofline": roof_mv},
        "roofline": roof,
    }
    note("learned start done")
    if not args.no_cpu:
        y0 = step(P, K, x, None, ws, 0)
        line["cpu_baseline"] = cpu_baseline(args.level, nbytes, P.tt_to_cores(y0))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
