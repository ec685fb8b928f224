"""TT conjugate gradients with FP64 iterative refinement (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper solves K u = f with AMEn (Sec. 3.5 and Sec. 4), which it cites but
does not describe.  The solve here is driven by the same two operations the
paper's format provides, the QTT matrix-vector product and TT rounding:

  outer loop (FP64 residual):  r = round(f - K u, eps_in, rmax_in); stop when
      ||f - K u|| <= tol ||f|| (the norm is that of the unrounded residual,
      obtained during the rounding's orthogonalisation sweep);
      e = inner_cg(K, r); u = round(u + e, eps, rmax)
  inner loop: plain conjugate gradients on K e = r in which every new
      iterate, residual, search direction and product K p is rounded to
      (eps_in, rmax_in); it stops after reducing its residual by red_in.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import qtt as T


@dataclass
class SolveOpts:
    tol: float = 1e-10
    eps: float = 1e-10
    rmax: int = 1 << 30
    eps_in: float = 1e-4
    rmax_in: int = 1 << 30
    red_in: float = 1e-2
    maxit_in: int = 2000
    maxit_out: int = 40


@dataclass
class SolveReport:
    converged: bool = False
    outer: int = 0
    inner: int = 0
    residuals: List[float] = field(default_factory=list)


def _zero_like(f):
    return [np.zeros((1, c.shape[1], 1)) for c in f]


def inner_cg(K, b, eps, rmax, red, maxit):
    """CG on K x = b with rounding after every update; returns (x, its)."""
    x = None
    r = [c.copy() for c in b]
    p = [c.copy() for c in b]
    rho = T.dot(r, r)
    bn = math.sqrt(rho)
    its = 0
    for its in range(1, maxit + 1):
        q = T.tt_round(T.matvec(K, p), eps, rmax)
        pq = T.dot(p, q)
        alpha = rho / pq
        x = T.scale(p, alpha) if x is None else T.tt_round(T.add(x, p, coeffs=[1.0, alpha]), eps, rmax)
        r = T.tt_round(T.add(r, q, coeffs=[1.0, -alpha]), eps, rmax)
        rho_new = T.dot(r, r)
        if math.sqrt(max(rho_new, 0.0)) <= red * bn:
            break
        beta = rho_new / rho
        p = T.tt_round(T.add(r, p, coeffs=[1.0, beta]), eps, rmax)
        rho = rho_new
    return x, its


def solve(K, f, opts: SolveOpts, x0=None):
    """TT-CG with iterative refinement; returns (u, report)."""
    rep = SolveReport()
    fn = T.norm(f)
    u = x0
    for out in range(opts.maxit_out + 1):
        if u is None:
            r, info = T.tt_round(f, opts.eps_in, opts.rmax_in, return_info=True)
        else:
            Ku = T.matvec(K, u)
            r, info = T.tt_round(T.add(f, Ku, coeffs=[1.0, -1.0]), opts.eps_in,
                                 opts.rmax_in, return_info=True)
        rel = info["norm"] / fn
        rep.residuals.append(rel)
        if rel <= opts.tol:
            rep.converged = True
            break
        if out == opts.maxit_out:
            break
        e, its = inner_cg(K, r, opts.eps_in, opts.rmax_in, opts.red_in, opts.maxit_in)
        rep.inner += its
        u = e if u is None else T.tt_round(T.add(u, e), opts.eps, opts.rmax)
        rep.outer += 1
    if u is None:
        u = _zero_like(f)
    return u, rep
