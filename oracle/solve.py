"""TT conjugate gradients with FP64 iterative refinement (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper solves K u = f with AMEn (Sec. 3, Sec. 3.7 and Sec. 4), which it cites but
does not describe.  The solve here is driven by the same two operations the
paper's format provides, the QTT matrix-vector product and TT rounding:

  outer loop (FP64 residual):  r = round(f - K u, eps_in, rmax_in); stop when
      ||f - K u|| <= tol ||f|| (the norm is that of the unrounded residual,
      obtained during the rounding's orthogonalisation sweep);
      e = inner_cg(K, r); u = round(u + e, eps, rmax)
  inner loop: conjugate gradients on K e = r in truncated form: products
      are formed exactly, the new residual r - alpha K p and direction
      z + beta p are rounded as sums to (eps_in, rmax_in), the iterate to
      (eps, rmax); it stops after reducing its residual by red_in.  With a
      preconditioner C (a QTT matrix approximating K^-1), z = C r.
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


def inner_cg(K, b, eps, rmax, red, maxit, C=None, eps_x=None, rmax_x=None):
    """(P)CG on K x = b in the truncated form: the products K p and C r are
    formed exactly, <p, K p> and <r, C r> use them unrounded, and the new
    residual r - alpha K p and direction C r + beta p are rounded as sums to
    (eps, rmax), so each truncation error is relative to the vector CG
    continues with.  The iterate is rounded to (eps_x, rmax_x): its
    truncation error enters the true residual multiplied by ||K||.
    Returns (x, its)."""
    eps_x = eps if eps_x is None else eps_x
    rmax_x = rmax if rmax_x is None else rmax_x
    x = None
    r = [c.copy() for c in b]
    bn = T.norm(r)
    z = r if C is None else T.matvec(C, r)
    rho = T.dot(r, z)
    p = [c.copy() for c in r] if C is None else T.tt_round(z, eps, rmax)
    its = 0
    for its in range(1, maxit + 1):
        Kp = T.matvec(K, p)
        pKp = T.dot(p, Kp)
        alpha = rho / pKp if pKp > 0 else 0.0
        x = T.scale(p, alpha) if x is None else T.tt_round(T.add(x, p, coeffs=[1.0, alpha]),
                                                           eps_x, rmax_x)
        r = T.tt_round(T.add(r, Kp, coeffs=[1.0, -alpha]), eps, rmax)
        if T.norm(r) <= red * bn:
            break
        z = r if C is None else T.matvec(C, r)
        rho_new = T.dot(r, z)
        beta = rho_new / rho
        p = T.tt_round(T.add(z, p, coeffs=[1.0, beta]), eps, rmax)
        rho = rho_new
    return x, its


def solve(K, f, opts: SolveOpts, x0=None, C=None):
    """TT-(P)CG with iterative refinement; returns (u, report)."""
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
        e, its = inner_cg(K, r, opts.eps_in, opts.rmax_in, opts.red_in, opts.maxit_in, C,
                          opts.eps, opts.rmax)
        rep.inner += its
        u = e if u is None else T.tt_round(T.add(u, e), opts.eps, opts.rmax)
        rep.outer += 1
    if u is None:
        u = _zero_like(f)
    return u, rep


@dataclass
class ChebOpts:
    """Options of the preconditioned Chebyshev solve.

    tol: stop when sqrt(<r, C r>) <= tol sqrt(<f, C f>) (r = f - K u, the
         preconditioned residual; equivalent to the relative energy-norm
         error up to sqrt(lmax/lmin));
    eps, rmax: rounding of the iterate; eps_r, rmax_r: rounding of the
         residual, relative to its own norm; eps_d, rmax_d: rounding of the
         preconditioned residual and of the update direction;
    lmin, lmax: bounds of the spectrum of C K."""
    tol: float = 1e-8
    eps: float = 1e-10
    rmax: int = 1 << 30
    eps_r: float = 1e-3
    rmax_r: int = 1 << 30
    eps_d: float = 1e-3
    rmax_d: int = 1 << 30
    lmin: float = 0.09
    lmax: float = 20.0
    maxit: int = 2000


def chebyshev(K, f, C, opts: ChebOpts, x0=None):
    """Chebyshev semi-iteration for C K u = C f with the true residual
    recomputed every step (Golub and Varga's two-term recurrence, in the
    form of Saad, Iterative Methods for Sparse Linear Systems, Alg. 12.1).
    Every vector is rounded, each relative to its own norm; because the
    residual is never updated recursively, truncation errors do not
    accumulate.  Returns (u, report) with report.residuals the
    preconditioned residual ratios."""
    rep = SolveReport()
    theta = 0.5 * (opts.lmax + opts.lmin)
    delta = 0.5 * (opts.lmax - opts.lmin)
    sigma = theta / delta
    Cf = T.matvec(C, f)
    fCf = T.dot(f, Cf)
    x = x0
    d = None
    rho = 1.0 / sigma
    for it in range(opts.maxit + 1):
        if x is None:
            r = T.tt_round(f, opts.eps_r, opts.rmax_r)
        else:
            r = T.tt_round(T.add(f, T.matvec(K, x), coeffs=[1.0, -1.0]), opts.eps_r, opts.rmax_r)
        Cr = T.matvec(C, r)
        rel = math.sqrt(max(T.dot(r, Cr), 0.0) / fCf)
        rep.residuals.append(rel)
        if rel <= opts.tol:
            rep.converged = True
            break
        if it == opts.maxit:
            break
        z = T.tt_round(Cr, opts.eps_d, opts.rmax_d)
        if d is None:
            d = T.scale(z, 1.0 / theta)
        else:
            rho_new = 1.0 / (2.0 * sigma - rho)
            d = T.tt_round(T.add(d, z, coeffs=[rho_new * rho, 2.0 * rho_new / delta]),
                           opts.eps_d, opts.rmax_d)
            rho = rho_new
        x = d if x is None else T.tt_round(T.add(x, d), opts.eps, opts.rmax)
        rep.inner += 1
    if x is None:
        x = _zero_like(f)
    return x, rep


def fcg(K, f, C, opts: ChebOpts, x0=None):
    """Flexible preconditioned CG with one stored direction and the true
    residual every step (Notay, SIAM J. Sci. Comput. 2000, with m = 1):
        alpha = <f - K x, p> / <p, K p>,  x = round(x + alpha p),
        r = round(f - K x),  z = round(C r),
        beta = <z, K p> / <p, K p>,  p = round(z - beta p).
    alpha is the exact energy minimiser along the direction actually used
    (computed from x and p, not from the rounded r), so the energy error
    decreases at every step whatever the truncation of z and p.  Stop as in
    chebyshev().  lmin and lmax are not used."""
    rep = SolveReport()
    Cf = T.matvec(C, f)
    fCf = T.dot(f, Cf)
    x = x0
    p = None
    for it in range(opts.maxit + 1):
        if x is None:
            r = T.tt_round(f, opts.eps_r, opts.rmax_r)
        else:
            r = T.tt_round(T.add(f, T.matvec(K, x), coeffs=[1.0, -1.0]), opts.eps_r, opts.rmax_r)
        Cr = T.matvec(C, r)
        rel = math.sqrt(max(T.dot(r, Cr), 0.0) / fCf)
        rep.residuals.append(rel)
        if rel <= opts.tol:
            rep.converged = True
            break
        if it == opts.maxit:
            break
        z = T.tt_round(Cr, opts.eps_d, opts.rmax_d)
        if p is None:
            p = z
        else:
            beta = T.dot(z, T.matvec(K, p)) / pKp
            p = T.tt_round(T.add(z, p, coeffs=[1.0, -beta]), opts.eps_d, opts.rmax_d)
        Kp = T.matvec(K, p)
        pKp = T.dot(p, Kp)
        fp = T.dot(f, p) - (0.0 if x is None else T.dot(x, Kp))
        alpha = fp / pKp
        x = T.scale(p, alpha) if x is None else T.tt_round(T.add(x, p, coeffs=[1.0, alpha]),
                                                           opts.eps, opts.rmax)
        rep.inner += 1
    if x is None:
        x = _zero_like(f)
    return x, rep
