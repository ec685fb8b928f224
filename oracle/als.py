"""One-site alternating least squares (ALS) for K u = f on the QTT format
(FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper solves its QTT systems with AMEn (named in Sec. 4; Dolgov and
Savostyanov 2014), which optimises one core at a time with the others fixed
and orthogonal.  This is that core step without AMEn's residual enrichment,
at fixed ranks (Holtz, Rohwedder and Schneider 2012), written plainly:

* the frame U_k of core k (cores left of k left-orthogonal, cores right of
  k right-orthogonal) is formed as a dense matrix, so u = U_k vec(X_k);
* the local system (U_k^T K U_k) y = U_k^T f is solved densely and y
  becomes core k; the energy J(u) = u^T K u / 2 - f^T u is then -y^T g / 2;
* the orthogonality centre moves by a QR (forward) or LQ (backward) step of
  the solved core, passing the triangular factor into the next core.

Dense frames limit it to small levels: it is an independent statement of
what the library's sweeps compute through environments.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from . import qtt as T


def _left_part(cores, k) -> np.ndarray:
    """Dense (n_0 ... n_{k-1}) x r_k matrix of cores 0..k-1 (first index fastest)."""
    M = np.ones((1, 1))
    for c in cores[:k]:
        r0, n, r1 = c.shape
        # rows: previous rows fastest, then the new mode index
        M = np.einsum("la,aib->lib", M, c).reshape(M.shape[0] * n, r1, order="F")
    return M


def _right_part(cores, k) -> np.ndarray:
    """Dense r_{k+1} x (n_{k+1} ... n_{D-1}) matrix of cores k+1..D-1."""
    M = np.ones((1, 1))
    for c in reversed(cores[k + 1:]):
        r0, n, r1 = c.shape
        M = np.einsum("aib,br->air", c, M).reshape(r0, n * M.shape[1], order="F")
    return M


def frame(cores, k) -> np.ndarray:
    """U_k with u = U_k vec(X_k) (X_k column-major, (a, i, b) with a fastest)."""
    Lp, Rp = _left_part(cores, k), _right_part(cores, k)
    r0, n, r1 = cores[k].shape
    U = np.einsum("la,ij,br->lirajb", Lp, np.eye(n), Rp)
    return U.reshape(Lp.shape[0] * n * Rp.shape[1], r0 * n * r1, order="F")


def _qr_step(X, k):
    r0, n, r1 = X[k].shape
    Q, R = np.linalg.qr(X[k].reshape(r0 * n, r1, order="F"))
    X[k] = Q.reshape(r0, n, Q.shape[1], order="F")
    X[k + 1] = np.einsum("ab,bic->aic", R, X[k + 1])


def _lq_step(X, k):
    r0, n, r1 = X[k].shape
    Q, R = np.linalg.qr(X[k].reshape(r0, n * r1, order="F").T)
    X[k] = Q.T.reshape(Q.shape[1], n, r1, order="F")
    X[k - 1] = np.einsum("aib,cb->aic", X[k - 1], R)


def als(Kcores, fcores, caps: Sequence[int], sweeps: int, x0=None, seed: int = 0):
    """ALS sweeps at the ranks `caps` (r_0 .. r_D).  Returns the cores and a
    log: per local solve (k, energy, ||y - x_k||, u before, u after)."""
    D = len(fcores)
    n = [c.shape[1] for c in fcores]
    Kd = T.full_matrix(Kcores)
    fd = T.full_vector(fcores)
    rng = np.random.default_rng(seed)
    if x0 is None:
        X = [rng.standard_normal((caps[k], n[k], caps[k + 1])) for k in range(D)]
    else:
        X = [np.zeros((caps[k], n[k], caps[k + 1])) for k in range(D)]
        for k, c in enumerate(x0):
            X[k][:c.shape[0], :, :c.shape[2]] = c
    for k in range(D - 1, 0, -1):
        _lq_step(X, k)
    log: List[Tuple[int, float, float, np.ndarray, np.ndarray]] = []

    def solve(k):
        U = frame(X, k)
        B = U.T @ Kd @ U
        g = U.T @ fd
        before = T.full_vector(X)
        xk = X[k].reshape(-1, order="F")
        y = np.linalg.solve(B, g)
        X[k] = y.reshape(X[k].shape, order="F")
        log.append((k, -0.5 * float(y @ g), float(np.linalg.norm(y - xk)), before,
                    T.full_vector(X)))

    solve(0)
    for s in range(sweeps):
        if s % 2 == 0:
            for k in range(D - 1):
                _qr_step(X, k)
                solve(k + 1)
        else:
            for k in range(D - 1, 0, -1):
                _lq_step(X, k)
                solve(k - 1)
    return X, log
