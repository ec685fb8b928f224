"""The learned warm start end to end, from library calls only: basis solves
of the linear load family, superposed training targets, native training
of the network and warm-versus-cold solves.

The load of the family is linear in its 16 parameters a (the Fourier
coefficients of the east-edge traction, 8 per displacement component), so
the displacement is u(a) = sum_k a_k u_k with u_k the solution for the k-th
unit coefficient.  The method generates its own training data: 16 solves
give every target.  The solutions are joined into one train with the load
index as an extra last core and rounded once to the rank cap (the family
train); evaluated at a load it gives the rank-capped superposition, and all
targets share one gauge, with only the last core depending on a.  (The
alternative, each superposition rounded on its own and its gauge aligned to
a reference by qtt_tt_align, gives targets whose cores vary with a far less
smoothly: a network fits them to about 10 % per core, which compounds over
the cores into starts no better than none in the energy norm.)  Training
runs natively (qtt_warmstart_fit) on the plain core loss of these targets;
a trained network's output for new parameters, rounded to minimal ranks,
is the start vector of qtt_solve, which scales it to its energy minimiser
and falls back to its cold start when it is unusable.
"""
from __future__ import annotations

import time
from typing import List, Optional, Sequence

import numpy as np

from . import _lib as L

NPARAM = 16


def network_sizes(nrow: Sequence[int], ranks: Sequence[int], hidden=(512, 512, 512)):
    nout = sum(ranks[k] * nrow[k] * ranks[k + 1] for k in range(len(nrow)))
    return [NPARAM] + list(hidden) + [nout]


def basis_solves(level: int, opts: L.SolveOpts, problem_of) -> List["L.TT"]:
    """u_k for the 16 unit coefficient vectors; problem_of(level, coeffs)
    builds the load case (the workloads module's generator)."""
    out = []
    for k in range(NPARAM):
        e = np.zeros(NPARAM)
        e[k] = 1.0
        K, f = L.assemble(problem_of(level, e))
        u, rep = L.solve(K, f, opts)
        if rep["status"] not in (0, -4):
            raise L.QttError(rep["status"], "basis solve %d failed" % k)
        out.append(u)
    return out


def family_train(basis, rank: int, ell: int, seed: int = 0) -> "L.TT":
    """The 16 unit-load solutions as one train with the load index as an
    extra last core (mode 16): sum_k u_k (x) e_k by qtt_tt_combine (ranks
    add), rounded once by a rank-ell sketch to the rank cap.  Evaluating it
    at a load vector a (qtt_tt_contract_last) gives the rank-capped
    superposition sum_k a_k u_k, every one in the same gauge: the cores are
    shared and only the last depends on a, linearly."""
    torch = L._torch()
    nrow = basis[0].nrow
    ext = []
    for k, u in enumerate(basis):
        n = u.numel()
        e = torch.zeros(NPARAM, dtype=torch.float64, device="cuda")
        e[k] = 1.0
        ext.append(L.TT(nrow + [NPARAM], None, u.ranks + [1], n + NPARAM,
                        data=torch.cat([u.data[:n], e])))
    fam = L.tt_combine(np.ones(NPARAM), ext)
    L.round_sketch(fam, ell, seed, 0.0, rank)
    return fam


def targets(fam, params: np.ndarray):
    """Columns (nout x n, FP32 device tensor, column-major storage) of the
    family train evaluated at the columns of params (16 x n), and their
    common rank pattern."""
    torch = L._torch()
    n = params.shape[1]
    cols = None
    ranks = None
    for j in range(n):
        y = L.tt_contract_last(fam, params[:, j])
        if cols is None:
            ranks = y.ranks
            cols = torch.empty((n, y.numel()), dtype=torch.float32, device="cuda")
        cols[j].copy_(y.data[:cols.shape[1]])
    return cols, ranks


def aligned_targets(basis, params: np.ndarray, rank: int, ell: int, seed: int = 0, ref=None):
    """The alternative targets: each superposition rounded on its own (the
    best rank-capped train of every load) and brought to the gauge of a
    reference train by qtt_tt_align (the first target when ref is None).
    Returns the columns, the rank pattern and the reference."""
    torch = L._torch()
    nrow = basis[0].nrow
    n = params.shape[1]
    ranks = capped(nrow, rank)
    nout = sum(ranks[k] * nrow[k] * ranks[k + 1] for k in range(len(nrow)))
    cols = torch.empty((n, nout), dtype=torch.float32, device="cuda")
    for j in range(n):
        z = L.tt_combine(params[:, j], basis)
        L.round_sketch(z, ell, seed, 0.0, rank)
        if z.ranks != ranks:
            raise RuntimeError("rounded target ranks %s differ from the pattern %s"
                               % (z.ranks, ranks))
        if ref is None:
            ref = z
        else:
            L.tt_align(z, ref)
        cols[j].copy_(z.data[:nout])
    return cols, ranks, ref


def capped(nrow: Sequence[int], r: int) -> List[int]:
    D = len(nrow)
    out = [1]
    for k in range(1, D):
        left = int(np.prod(nrow[:k], dtype=np.float64))
        right = int(np.prod(nrow[k:], dtype=np.float64))
        out.append(int(min(r, left, right)))
    return out + [1]


def init_params(sizes: Sequence[int], seed: int, out_bias: Optional[np.ndarray] = None,
                out_scale: float = 1.0) -> np.ndarray:
    """He-scaled Gaussian weights, zero biases, flattened in the layout of
    qtt_mlp (W_l column-major, then b_l); the output layer's weights times
    out_scale and its bias out_bias (e.g. the mean target, so that training
    starts from the centre of the targets)."""
    g = np.random.default_rng(seed)
    parts = []
    nl = len(sizes) - 1
    for l in range(nl):
        fan_in, fan_out = sizes[l], sizes[l + 1]
        Wl = g.standard_normal((fan_out, fan_in)) * np.sqrt(2.0 / fan_in)
        b = np.zeros(fan_out)
        if l == nl - 1:
            Wl *= out_scale
            if out_bias is not None:
                b = np.asarray(out_bias, dtype=np.float64).reshape(fan_out)
        parts.append(Wl.reshape(-1, order="F"))
        parts.append(b)
    return np.concatenate(parts).astype(np.float32)


def compare_starts(net, problem_of, level: int, params: np.ndarray, nrow, ranks,
                   opts: L.SolveOpts, progress=None, keep_solutions: bool = True):
    """Per held-out parameter vector: the solve from the network's start and
    the cold solve, with sweeps, seconds, FP64 residual and the difference
    of the two solutions.  The network's train is rounded exactly (eps 0,
    cap opts.rmax) to minimal ranks before the solve; that is part of the
    warm time.  progress(j) is called after every 32nd load; with
    keep_solutions False the rows hold no solution trains."""
    torch = L._torch()
    rows = []
    for j in range(params.shape[1]):
        K, f = L.assemble(problem_of(level, params[:, j]))
        ws = L._workspace(L.solve_workspace_bytes(K, f, opts))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        uc, rc = L.solve(K, f, opts, ws=ws)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t0
        t0 = time.perf_counter()
        x0 = net.infer_tt(params[:, j], nrow, ranks)
        L.round_(x0, 0.0, opts.rmax)
        uw, rw = L.solve(K, f, opts, x0=x0, ws=ws)
        torch.cuda.synchronize()
        tw = time.perf_counter() - t0
        # energy-norm distance of the scaled start from the solution:
        # ||a x0 - u||_K^2 = 2 (J(a x0) - J(u)), J(u) = -<f, u> / 2
        Ju = -0.5 * L.dot(f, uc)
        gap = np.sqrt(max(rw["warm_energy"] - Ju, 0.0) / abs(Ju)) if Ju != 0 else float("nan")
        rows.append(dict(cold_sweeps=rc["outer"], warm_sweeps=rw["outer"], cold_s=tc, warm_s=tw,
                         start_energy_error=gap,
                         cold_residual=rc["residual"], warm_residual=rw["residual"],
                         warm_start=rw["warm_start"], warm_energy=rw["warm_energy"],
                         cold_status=rc["status"], warm_status=rw["status"],
                         u_cold=uc if keep_solutions else None,
                         u_warm=uw if keep_solutions else None))
        if progress is not None and (j + 1) % 32 == 0:
            progress(j + 1)
    return rows
