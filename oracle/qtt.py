"""Plain tensor-train algebra on NumPy arrays (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

A TT is a list of cores.  Vector cores have shape (r_{k-1}, n_k, r_k);
matrix cores (r_{k-1}, n_k, m_k, r_k) (Sec. 4: the entries of a TT vector
are products of the matrices T_k(:, i_k, :); a TT matrix multiplies the
blocks A_k(:, i_k, j_k, :)).  The first core carries the least significant
index digit: the dense index of (i_1, ..., i_D) is i_1 + n_1 (i_2 + n_2 (...))
(the binary quantisation i = sum_k 2^(k-1) i_k of Sec. 4).
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

Cores = List[np.ndarray]


# ------------------------------------------------------------------ basics

def ranks(cores: Cores) -> List[int]:
    return [cores[0].shape[0]] + [c.shape[-1] for c in cores]


def modes(cores: Cores) -> List[int]:
    return [c.shape[1] for c in cores]


def is_matrix(cores: Cores) -> bool:
    return cores[0].ndim == 4


def full_vector(cores: Cores) -> np.ndarray:
    """Dense vector of a TT vector, first core least significant."""
    T = cores[0][0]                              # (n1, r1)
    shape = [cores[0].shape[1]]
    for c in cores[1:]:
        T = np.tensordot(T, c, axes=([T.ndim - 1], [0]))
        shape.append(c.shape[1])
    T = T[..., 0]
    return np.reshape(T, -1, order="F")


def full_matrix(cores: Cores) -> np.ndarray:
    """Dense matrix of a TT matrix: A[(i_1..i_D), (j_1..j_D)]."""
    D = len(cores)
    T = cores[0][0]                              # (n1, m1, r1)
    for c in cores[1:]:
        T = np.tensordot(T, c, axes=([T.ndim - 1], [0]))
    T = T[..., 0]                                # (n1, m1, n2, m2, ...)
    perm = list(range(0, 2 * D, 2)) + list(range(1, 2 * D, 2))
    T = np.transpose(T, perm)
    N = int(np.prod([c.shape[1] for c in cores]))
    M = int(np.prod([c.shape[2] for c in cores]))
    # Fortran flattening of the row digits then of the column digits
    T = np.reshape(T, (N, M), order="F")
    return T


def matrix_as_vector(cores: Cores) -> Cores:
    """View the cores of a TT matrix as vector cores with mode n*m (the
    'long index' remark of Sec. 4)."""
    return [c.reshape(c.shape[0], c.shape[1] * c.shape[2], c.shape[3]) for c in cores]


def vector_as_matrix(cores: Cores, nrow: Sequence[int], ncol: Sequence[int]) -> Cores:
    return [c.reshape(c.shape[0], n, m, c.shape[2]) for c, n, m in zip(cores, nrow, ncol)]


# ------------------------------------------------------------------ TT-SVD

def _truncation_rank(s: np.ndarray, delta: float, rmax: int) -> int:
    """Smallest rank r with sqrt(sum_{i>=r} s_i^2) <= delta, at least 1,
    at most rmax."""
    tail = np.sqrt(np.cumsum((s[::-1] ** 2)))[::-1]   # tail[r] = ||s[r:]||
    r = len(s)
    for k in range(len(s)):
        if tail[k] <= delta:
            r = k
            break
    r = max(1, r)
    return min(r, rmax)


def tt_svd(a: np.ndarray, mode_sizes: Sequence[int], eps: float,
           rmax: int = 1 << 30) -> Cores:
    """TT-SVD (the cited Oseledets algorithm 1): successive truncated SVDs
    of unfoldings with the per-step threshold eps ||a||_F / sqrt(D-1)."""
    D = len(mode_sizes)
    a = np.asarray(a, dtype=np.float64)
    nrm = np.linalg.norm(a)
    delta = eps * nrm / math.sqrt(max(D - 1, 1))
    C = np.reshape(a, (-1,), order="F")
    cores = []
    r = 1
    for k in range(D - 1):
        n = mode_sizes[k]
        C = np.reshape(C, (r * n, -1), order="F")
        U, s, Vt = np.linalg.svd(C, full_matrices=False)
        rk = _truncation_rank(s, delta, rmax)
        cores.append(np.reshape(U[:, :rk], (r, n, rk), order="F"))
        C = s[:rk, None] * Vt[:rk]
        r = rk
    cores.append(np.reshape(C, (r, mode_sizes[-1], 1), order="F"))
    return cores


# ------------------------------------------------------------------ rounding

def orthogonalize_left(cores: Cores) -> Cores:
    """Left-to-right QR sweep: cores 1..D-1 become left-orthogonal, the norm
    moves into the last core."""
    out = [c.copy() for c in cores]
    for k in range(len(out) - 1):
        r0, n, r1 = out[k].shape
        Q, R = np.linalg.qr(out[k].reshape(r0 * n, r1), mode="reduced")
        out[k] = Q.reshape(r0, n, Q.shape[1])
        out[k + 1] = np.tensordot(R, out[k + 1], axes=([1], [0]))
    return out


def tt_round(cores: Cores, eps: float, rmax: int = 1 << 30,
             return_info: bool = False):
    """TT rounding (the cited Oseledets algorithm 2, mirrored): a
    left-to-right QR orthogonalisation sweep, then a right-to-left sweep of
    truncated SVDs with threshold delta = eps ||y||_F / sqrt(D-1) per bond,
    capped at rmax.  Vector cores only; round a matrix through
    ``matrix_as_vector``.  Returns the new cores (and, with
    ``return_info``, a dict with the norm, the discarded-sigma bound
    sqrt(sum of discarded sigma^2 over all bonds) and the per-bond singular
    values)."""
    D = len(cores)
    y = orthogonalize_left(cores)
    nrm = float(np.linalg.norm(y[-1]))
    delta = eps * nrm / math.sqrt(max(D - 1, 1))
    disc2 = 0.0
    sig = [None] * D
    for k in range(D - 1, 0, -1):
        r0, n, r1 = y[k].shape
        M = y[k].reshape(r0, n * r1)
        U, s, Vt = np.linalg.svd(M, full_matrices=False)
        rk = _truncation_rank(s, delta, rmax)
        disc2 += float(np.sum(s[rk:] ** 2))
        sig[k] = s
        y[k] = Vt[:rk].reshape(rk, n, r1)
        y[k - 1] = np.tensordot(y[k - 1], U[:, :rk] * s[:rk], axes=([2], [0]))
    if return_info:
        return y, dict(norm=nrm, err=math.sqrt(disc2), sigma=sig)
    return y


def round_matrix(cores: Cores, eps: float, rmax: int = 1 << 30) -> Cores:
    nr = [c.shape[1] for c in cores]
    nc = [c.shape[2] for c in cores]
    return vector_as_matrix(tt_round(matrix_as_vector(cores), eps, rmax), nr, nc)


# ------------------------------------------------------------------ algebra

def matvec(A: Cores, x: Cores) -> Cores:
    """y = A x core by core (strong Kronecker product of Sec. 4):
    y_k[(a,b), i, (c,d)] = sum_j A_k[a, i, j, c] x_k[b, j, d]."""
    out = []
    for Ak, xk in zip(A, x):
        ra0, n, m, ra1 = Ak.shape
        rb0, m2, rb1 = xk.shape
        assert m == m2
        y = np.einsum("aijc,bjd->abicd", Ak, xk)
        out.append(y.reshape(ra0 * rb0, n, ra1 * rb1))
    return out


def matmat(A: Cores, B: Cores) -> Cores:
    """C = A B core by core: C_k[(a,b), i, j, (c,d)] =
    sum_l A_k[a, i, l, c] B_k[b, l, j, d]."""
    out = []
    for Ak, Bk in zip(A, B):
        ra0, n, l, ra1 = Ak.shape
        rb0, l2, m, rb1 = Bk.shape
        assert l == l2
        c = np.einsum("ailc,bljd->abijcd", Ak, Bk)
        out.append(c.reshape(ra0 * rb0, n, m, ra1 * rb1))
    return out


def hadamard(x: Cores, y: Cores) -> Cores:
    """Entrywise product of two TT vectors (ranks multiply)."""
    out = []
    for a, b in zip(x, y):
        c = np.einsum("aib,cid->acibd", a, b)
        out.append(c.reshape(a.shape[0] * b.shape[0], a.shape[1], a.shape[2] * b.shape[2]))
    return out


def diag(x: Cores) -> Cores:
    """TT matrix diag(x) from a TT vector x."""
    out = []
    for c in x:
        r0, n, r1 = c.shape
        d = np.zeros((r0, n, n, r1))
        for i in range(n):
            d[:, i, i, :] = c[:, i, :]
        out.append(d)
    return out


def add(*terms: Cores, coeffs: Sequence[float] = None) -> Cores:
    """Sum of TTs of equal modes by core concatenation (first core side by
    side, middle cores block-diagonal, last core stacked)."""
    if coeffs is None:
        coeffs = [1.0] * len(terms)
    D = len(terms[0])
    if D == 1:
        return [sum(c * t[0] for c, t in zip(coeffs, terms))]
    out = []
    for k in range(D):
        blocks = [t[k] for t in terms]
        if k == 0:
            blocks = [c * b for c, b in zip(coeffs, blocks)]
            out.append(np.concatenate(blocks, axis=-1))
        elif k == D - 1:
            out.append(np.concatenate(blocks, axis=0))
        else:
            r0 = sum(b.shape[0] for b in blocks)
            r1 = sum(b.shape[-1] for b in blocks)
            shp = (r0,) + blocks[0].shape[1:-1] + (r1,)
            c = np.zeros(shp)
            o0 = o1 = 0
            for b in blocks:
                c[o0:o0 + b.shape[0], ..., o1:o1 + b.shape[-1]] = b
                o0 += b.shape[0]
                o1 += b.shape[-1]
            out.append(c)
    return out


def scale(x: Cores, a: float) -> Cores:
    out = [c.copy() for c in x]
    out[0] = out[0] * a
    return out


def dot(x: Cores, y: Cores) -> float:
    """<x, y> by a left-to-right environment sweep."""
    phi = np.ones((1, 1))
    for a, b in zip(x, y):
        t = np.tensordot(phi, a, axes=([0], [0]))          # (r', n, ra)
        phi = np.tensordot(t, b, axes=([0, 1], [0, 1]))    # (ra, rb)
    return float(phi[0, 0])


def norm(x: Cores) -> float:
    return math.sqrt(max(dot(x, x), 0.0))


def trace(A: Cores) -> float:
    v = np.ones((1,))
    for c in A:
        s = np.einsum("aiib->ab", c)
        v = v @ s
    return float(v[0])


def kron(first: Cores, second: Cores) -> Cores:
    """Kronecker product where ``first`` supplies the less significant
    digits: the cores of ``first`` followed by the cores of ``second``."""
    return [c.copy() for c in first] + [c.copy() for c in second]


def zkron(Y: Cores, X: Cores) -> Cores:
    """Z-ordered Kronecker product Y (x) X: X acts on the digits i_k, Y on
    j_k, and the digits are interleaved i_1, j_1, i_2, j_2, ... (z-kron).
    Core 2k-1 is X_k with Y's open bond carried by an identity, core 2k is
    Y_k with X's bond carried by an identity, so bond ranks are a_k b_k."""
    assert len(X) == len(Y)
    out = []
    mat = X[0].ndim == 4
    for Xk, Yk in zip(X, Y):
        a0, a1 = Xk.shape[0], Xk.shape[-1]
        b0, b1 = Yk.shape[0], Yk.shape[-1]
        Ib = np.eye(b0)
        Ia = np.eye(a1)
        if mat:
            cx = np.einsum("aijc,bd->abijcd", Xk, Ib)
            out.append(cx.reshape(a0 * b0, Xk.shape[1], Xk.shape[2], a1 * b0))
            cy = np.einsum("ac,bijd->abijcd", Ia, Yk)
            out.append(cy.reshape(a1 * b0, Yk.shape[1], Yk.shape[2], a1 * b1))
        else:
            cx = np.einsum("aic,bd->abicd", Xk, Ib)
            out.append(cx.reshape(a0 * b0, Xk.shape[1], a1 * b0))
            cy = np.einsum("ac,bid->abicd", Ia, Yk)
            out.append(cy.reshape(a1 * b0, Yk.shape[1], a1 * b1))
    return out


def ones(mode_sizes: Sequence[int]) -> Cores:
    return [np.ones((1, n, 1)) for n in mode_sizes]


def effective_rank(cores: Cores) -> float:
    """r_e solving r n_1 + sum_{k=2}^{D-1} r^2 n_k + r n_D = storage (Sec. 4);
    matrix cores use n_k m_k."""
    ns = [int(np.prod(c.shape[1:-1])) for c in cores]
    storage = sum(c.size for c in cores)
    if len(cores) == 1:
        return 1.0
    a = sum(ns[1:-1])
    b = ns[0] + ns[-1]
    if a == 0:
        return storage / b
    return (-b + math.sqrt(b * b + 4.0 * a * storage)) / (2.0 * a)
