"""BPX multilevel preconditioner in QTT form (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper points to tensor-structured BPX preconditioning as what makes
QTT-FEM practical on very fine grids (Sec. 1, its discussion of BPX for
elliptic problems), without giving a construction.  This module writes the
additive multilevel (BPX) preconditioner out plainly:

    C = sum_{l=0}^{d} P_l P_l^T

where P_l interpolates level-l coarse nodal values onto the fine grid of
2^d nodes per direction.  Level-l coarse nodes sit at the fine indices
i = 2^l j, j = 0 .. 2^(d-l) - 1; P_l is linear between consecutive coarse
nodes and constant past the last one, so the coarse spaces are nested Q1
subspaces of the fine space.  A clamped end removes the coarse node on it
(for a clamp at the far end the construction is mirrored), so every coarse
function vanishes there.  In 2-D the prolongation is the tensor product of
the 1-D ones (z-kron in QTT); in 2-D stiffness matrices are scale-free, so
all levels carry unit weight.  Each displacement component uses its own
clamps.  Dirichlet dofs get 1/gamma_D (the inverse of their row of K_bc).
"""
from __future__ import annotations

import numpy as np

from . import qtt as T
from .assembly import EPS_ASSEMBLY

WEST, EAST, SOUTH, NORTH = 0, 1, 2, 3


def prolongation_1d(d: int, l: int, clamp_lo: bool, clamp_hi: bool) -> np.ndarray:
    """Dense 2^d x (number of coarse nodes) interpolation matrix of level l."""
    if clamp_lo and clamp_hi:
        raise ValueError("BPX coarse grids with clamps at both ends are not built")
    n = 2 ** d
    H = 2 ** l
    J = n // H
    P = np.zeros((n, J))
    for i in range(n):
        j, s = divmod(i, H)
        if j < J - 1:
            P[i, j] += 1.0 - s / H
            P[i, j + 1] += s / H
        else:
            P[i, j] += 1.0
    if clamp_lo or clamp_hi:
        P = P[:, 1:]
    if clamp_hi:
        P = P[::-1, :]          # mirrored: coarse nodes counted from the far end
    return P


def _matrix_to_qtt(M: np.ndarray, d: int, eps: float):
    """A 2^d x 2^d matrix as a QTT matrix (digits paired row/column)."""
    A = M.reshape([2] * d + [2] * d, order="F")
    perm = []
    for k in range(d):
        perm += [k, d + k]
    A = np.transpose(A, perm)
    cores = T.tt_svd(np.reshape(A, -1, order="F"), [4] * d, eps)
    return [c.reshape(c.shape[0], 2, 2, c.shape[2], order="F") for c in cores]


def bpx_levels_1d(d: int, clamp_lo: bool, clamp_hi: bool):
    """B_l = P_l P_l^T for l = 0..d (dense), skipping empty coarse spaces."""
    out = []
    for l in range(d + 1):
        P = prolongation_1d(d, l, clamp_lo, clamp_hi)
        if P.shape[1] == 0:
            continue
        out.append((l, P @ P.T))
    return out


def bpx_nodes(d: int, fixed_c) -> list:
    """Node part of C for one component with clamps fixed_c[side] (QTT)."""
    bx = dict(bpx_levels_1d(d, fixed_c[WEST], fixed_c[EAST]))
    by = dict(bpx_levels_1d(d, fixed_c[SOUTH], fixed_c[NORTH]))
    terms = []
    for l in sorted(set(bx) & set(by)):
        terms.append(T.zkron(_matrix_to_qtt(by[l], d, EPS_ASSEMBLY),
                             _matrix_to_qtt(bx[l], d, EPS_ASSEMBLY)))
    return T.round_matrix(T.add(*terms), EPS_ASSEMBLY)


def bpx_qtt(prob, gamma_D: float):
    """C_bc = P C P + (1/gamma_D)(I - P) in QTT for a single square
    subdomain, cores [component | i1 j1 ... id jd]."""
    if prob.q != 1:
        raise ValueError("BPX is built for one square subdomain")
    d = prob.level
    sq = prob.subs[0]
    terms = []
    for c in range(2):
        fixed_c = [sq.fixed[s][c] for s in range(4)]
        node = bpx_nodes(d, fixed_c)
        E = np.zeros((1, 2, 2, 1))
        E[0, c, c, 0] = 1.0
        terms.append([E] + node)
    C = T.round_matrix(T.add(*terms), EPS_ASSEMBLY)
    from .assembly import dirichlet_mask
    mask = dirichlet_mask(prob)
    P = T.diag(mask)
    one = T.ones([c.shape[1] for c in mask])
    Pc = T.diag(T.tt_round(T.add(one, mask, coeffs=[1.0, -1.0]), EPS_ASSEMBLY))
    PCP = T.round_matrix(T.matmat(T.matmat(P, C), P), EPS_ASSEMBLY)
    return T.round_matrix(T.add(PCP, Pc, coeffs=[1.0, 1.0 / gamma_D]), EPS_ASSEMBLY)


def bpx_dense(prob, gamma_D: float) -> np.ndarray:
    """The same operator as a dense matrix in canonical order, built with
    plain Kronecker products (for the pins)."""
    from .fem import dirichlet_mask
    d = prob.level
    n = 2 ** d
    sq = prob.subs[0]
    N = 2 * n * n
    C = np.zeros((N, N))
    for c in range(2):
        fx = [sq.fixed[s][c] for s in range(4)]
        bx = dict(bpx_levels_1d(d, fx[WEST], fx[EAST]))
        by = dict(bpx_levels_1d(d, fx[SOUTH], fx[NORTH]))
        Cc = sum(np.kron(by[l], bx[l]) for l in sorted(set(bx) & set(by)))
        idx = c + 2 * np.arange(n * n)
        C[np.ix_(idx, idx)] = Cc
    m = dirichlet_mask(d, sq)
    return m[:, None] * C * m[None, :] + np.diag((1.0 - m) / gamma_D)
