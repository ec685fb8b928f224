"""Randomised TT rounding (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

TT rounding is the step the paper's solver repeats (Sec. 4, the cited
rounding algorithm).  For a train whose ranks are far above the result's
(a matrix-vector product K x) the rounding can first be randomised:
randomize-then-orthogonalize of Al Daas, Ballard, Cazeaux, Hallman,
Miedlar, Pasha, Reid and Saibaba ("Randomized algorithms for rounding in
the tensor-train format", SIAM J. Sci. Comput. 45, 2023), restated here:

  1. draw a Gaussian train Omega of ranks l_k (target rank plus
     oversampling, bounded by the mode products and the ranks of y);
  2. right-to-left partial contractions W_D = 1,
     W_k[a, l] = sum_{i, b, l'} y_k[a, i, b] Omega_k[l, i, l'] W_{k+1}[b, l'];
  3. left-to-right with Z_0 = y_0: the sketch S = Z_k W_{k+1} (rows (a, i)),
     S = Q R (thin QR), core k = Q, Z_{k+1} = (Q^T Z_k) y_{k+1}; the last
     core is Z_{D-1}.

The result is left-orthogonal with ranks <= l and is then rounded exactly
(``qtt.tt_round``) to the requested accuracy.

The Gaussian numbers are those the library draws: Philox4x32-10 (Salmon,
Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC 2011) on the counter (element, core, call low word, call high word) with
the key (seed low word, seed high word), then the Box-Muller transform of
the first two output words u1 = (w0 + 1/2) 2^-32, u2 = (w1 + 1/2) 2^-32:
g = sqrt(-2 ln u1) cos(2 pi u2).  Element e of core k is its column-major
position e = a + l_k (i + n_k b) for the entry (a, i, b).
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from . import qtt as T

Cores = List[np.ndarray]

_M0, _M1 = 0xD2511F53, 0xCD9E8D57          # Philox4x32 multipliers
_W0, _W1 = 0x9E3779B9, 0xBB67AE85          # Weyl key increments
_MASK = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds on arrays of 32-bit counter words (any integer
    arrays of one shape) and a scalar 64-bit key split into two words.
    Each round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 as 64-bit
    products, new counter (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0), then the
    key advances by the Weyl constants."""
    c = [np.asarray(v, dtype=np.uint64) & _MASK for v in (c0, c1, c2, c3)]
    k0, k1 = np.uint64(k0 & _MASK), np.uint64(k1 & _MASK)
    for _ in range(10):
        p0 = np.uint64(_M0) * c[0]
        p1 = np.uint64(_M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(_MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(_MASK)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = (k0 + np.uint64(_W0)) & np.uint64(_MASK)
        k1 = (k1 + np.uint64(_W1)) & np.uint64(_MASK)
    return c


def gaussian(e, core: int, call: int, seed: int) -> np.ndarray:
    """Standard normal numbers for element indices e of core `core`."""
    e = np.asarray(e, dtype=np.uint64)
    w = philox4x32_10(e, np.full_like(e, core), np.full_like(e, call & _MASK),
                      np.full_like(e, (call >> 32) & _MASK), seed & _MASK, (seed >> 32) & _MASK)
    u1 = (w[0].astype(np.float64) + 0.5) * (1.0 / 4294967296.0)
    u2 = (w[1].astype(np.float64) + 0.5) * (1.0 / 4294967296.0)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(6.283185307179586 * u2)


def sketch_ranks(y: Cores, ell: int) -> List[int]:
    """l_k = min(ell, product of the modes left of bond k, product of the
    modes right of it, rank of y at bond k), l_0 = l_D = 1."""
    D = len(y)
    n = [c.shape[1] for c in y]
    r = T.ranks(y)
    out = [1] * (D + 1)
    for k in range(1, D):
        left = float(np.prod(n[:k], dtype=np.float64))
        right = float(np.prod(n[k:], dtype=np.float64))
        out[k] = int(max(1, min(ell, left, right, r[k])))
    return out


def gaussian_tt(modes: Sequence[int], l: Sequence[int], seed: int, call: int = 0) -> Cores:
    cores = []
    for k, nk in enumerate(modes):
        a, b = l[k], l[k + 1]
        A, I, B = np.meshgrid(np.arange(a), np.arange(nk), np.arange(b), indexing="ij")
        e = A + a * (I + nk * B)
        cores.append(gaussian(e, k, call, seed))
    return cores


def randomized_orthogonalize(y: Cores, ell: int, seed: int, call: int = 0) -> Cores:
    """Steps 1-3 above: the left-orthogonal rank-<=l approximation of y."""
    D = len(y)
    if D < 2:
        return [c.copy() for c in y]
    l = sketch_ranks(y, ell)
    om = gaussian_tt([c.shape[1] for c in y], l, seed, call)
    W = [None] * (D + 1)
    W[D] = np.ones((1, 1))
    for k in range(D - 1, 0, -1):
        # W_k[a, l] = sum_{i,b,l'} y_k[a,i,b] Omega_k[l,i,l'] W_{k+1}[b,l'],
        # contracted as Omega_k W_{k+1}^T first (indices l, i, b), then y_k
        t = np.tensordot(om[k], W[k + 1], axes=([2], [1]))
        W[k] = np.tensordot(y[k], t, axes=([1, 2], [1, 2]))
    out = []
    Z = y[0]
    for k in range(D - 1):
        lz, n, a1 = Z.shape
        S = Z.reshape(lz * n, a1) @ W[k + 1]
        Q, _ = np.linalg.qr(S, mode="reduced")
        out.append(Q.reshape(lz, n, Q.shape[1]))
        M = Q.T @ Z.reshape(lz * n, a1)
        Z = np.tensordot(M, y[k + 1], axes=([1], [0]))
    out.append(Z)
    return out


def sketch_round(y: Cores, ell: int, seed: int, eps: float, rmax: int = 1 << 30,
                 call: int = 0, return_info: bool = False):
    """Randomised rounding: randomized_orthogonalize, then the exact
    rounding to (eps, rmax)."""
    z = randomized_orthogonalize(y, ell, seed, call)
    return T.tt_round(z, eps, rmax, return_info=return_info)
