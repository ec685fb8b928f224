"""Learned warm start: an MLP from load parameters to the QTT cores of the
displacement, trained on the method's own solves (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no learned component; this is the warm-start extension of the
solve.  The network maps the 16 load parameters a (the traction
coefficients) to a flattened train x = TT(o(a)) with a fixed rank pattern
(ranks capped at r, bounded by the mode products), packed core after core,
each core (r_k, n_k, r_{k+1}) in column-major order.  The loss is
gauge-invariant: it compares tensors, not cores,

    L(o, u) = ||TT(o) - u||_F^2 / ||u||_F^2
            = (<x, x> - 2 <x, u> + <u, u>) / <u, u>,

with u the target train (same rank pattern, zero-padded).  Its gradient with
respect to core k of x is, with left environments L_k = sum_i X_<k^T Y_<k
and right environments R_k of the inner product <x, y>,

    d<x, y>/dX_k[a, i, b] = sum_{a', b'} L_k[a, a'] Y_k[a', i, b'] R_{k+1}[b, b'],

twice that for <x, x>.  Training is plain Adam (Kingma and Ba, ICLR 2015)
on the mean loss of a minibatch.  Targets come from superposition: the
problem is linear in a, so u(a) = round(sum_k a_k u_k) with u_k the solves
of the 16 unit loads.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np


def core_shapes(nrow: Sequence[int], ranks: Sequence[int]):
    return [(ranks[k], nrow[k], ranks[k + 1]) for k in range(len(nrow))]


def n_out(nrow, ranks) -> int:
    return int(sum(a * n * b for a, n, b in core_shapes(nrow, ranks)))


def unflatten(o: np.ndarray, nrow, ranks) -> List[np.ndarray]:
    cores, off = [], 0
    for shp in core_shapes(nrow, ranks):
        sz = int(np.prod(shp))
        cores.append(np.reshape(o[off:off + sz], shp, order="F"))
        off += sz
    return cores


def flatten(cores) -> np.ndarray:
    return np.concatenate([np.reshape(c, -1, order="F") for c in cores])


def pad_cores(cores, ranks) -> List[np.ndarray]:
    """Zero-pad a train to the given ranks (same tensor)."""
    out = []
    for k, c in enumerate(cores):
        p = np.zeros((ranks[k], c.shape[1], ranks[k + 1]))
        p[:c.shape[0], :, :c.shape[2]] = c
        out.append(p)
    return out


# ------------------------------------------------------------------ MLP
def init_params(sizes: Sequence[int], seed: int):
    """He-normal weights, zero biases; W_l is (out, in)."""
    rng = np.random.default_rng(seed)
    params = []
    for l in range(len(sizes) - 1):
        fan_in = sizes[l]
        W = rng.standard_normal((sizes[l + 1], sizes[l])) * np.sqrt(2.0 / fan_in)
        if l == len(sizes) - 2:
            W *= 0.1                       # small initial output
        params.append((W, np.zeros(sizes[l + 1])))
    return params


def forward(params, a: np.ndarray):
    """a: (nin, B) -> output (nout, B); returns the output and the cache of
    pre-activations and activations."""
    h = a
    cache = [(None, h)]
    for l, (W, b) in enumerate(params):
        z = W @ h + b[:, None]
        h = np.maximum(z, 0.0) if l < len(params) - 1 else z
        cache.append((z, h))
    return h, cache


def backward(params, cache, dout: np.ndarray):
    """Gradients of a scalar whose gradient w.r.t. the output is dout."""
    grads = [None] * len(params)
    d = dout
    for l in range(len(params) - 1, -1, -1):
        W, b = params[l]
        z, _ = cache[l + 1]
        if l < len(params) - 1:
            d = d * (z > 0.0)
        h_prev = cache[l][1]
        grads[l] = (d @ h_prev.T, d.sum(axis=1))
        d = W.T @ d
    return grads


# ------------------------------------------------------------------ TT loss
def _left_envs(X, Y):
    L = [np.ones((1, 1))]
    for Xk, Yk in zip(X, Y):
        L.append(sum(Xk[:, i, :].T @ L[-1] @ Yk[:, i, :] for i in range(Xk.shape[1])))
    return L


def _right_envs(X, Y):
    D = len(X)
    R = [None] * (D + 1)
    R[D] = np.ones((1, 1))
    for k in range(D - 1, -1, -1):
        R[k] = sum(X[k][:, i, :] @ R[k + 1] @ Y[k][:, i, :].T for i in range(X[k].shape[1]))
    return R


def _env_grad(L, R, Y):
    """d<x, y>/dX_k for every k."""
    return [np.einsum("ab,bic,dc->aid", L[k], Y[k], R[k + 1]) for k in range(len(Y))]


def tt_loss_grad(o: np.ndarray, u_cores, nrow, ranks):
    """Loss L(o, u) and dL/do for one sample."""
    X = unflatten(o, nrow, ranks)
    Lxx, Rxx = _left_envs(X, X), _right_envs(X, X)
    Lxu, Rxu = _left_envs(X, u_cores), _right_envs(X, u_cores)
    xx = float(Lxx[-1][0, 0])
    xu = float(Lxu[-1][0, 0])
    uu = float(_left_envs(u_cores, u_cores)[-1][0, 0])
    loss = (xx - 2.0 * xu + uu) / uu
    gxx = _env_grad(Lxx, Rxx, X)
    gxu = _env_grad(Lxu, Rxu, u_cores)
    g = [(2.0 * a - 2.0 * b) / uu for a, b in zip(gxx, gxu)]
    return loss, flatten(g)


def batch_loss_grad(out: np.ndarray, targets, nrow, ranks):
    """Mean loss over the columns of out (nout, B) and its gradient."""
    B = out.shape[1]
    g = np.zeros_like(out)
    tot = 0.0
    for j in range(B):
        l, gj = tt_loss_grad(out[:, j], targets[j], nrow, ranks)
        tot += l
        g[:, j] = gj / B
    return tot / B, g


def adam_update(params, grads, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place; m, v lists like params."""
    t = step + 1
    for l in range(len(params)):
        for p in range(2):
            g = grads[l][p]
            m[l][p][...] = b1 * m[l][p] + (1 - b1) * g
            v[l][p][...] = b2 * v[l][p] + (1 - b2) * g * g
            mh = m[l][p] / (1 - b1 ** t)
            vh = v[l][p] / (1 - b2 ** t)
            params[l][p][...] -= lr * mh / (np.sqrt(vh) + eps)


def tt_energy_loss_grad(o: np.ndarray, u_cores, A, nrow, ranks):
    """Energy-norm loss ||x - u||_A^2 / ||u||_A^2 for a symmetric positive
    definite QTT matrix A, and dL/do: with z = A x and w = A u formed exactly,
    d<x, A x>/dX_k = 2 d<x, z>/dX_k (z held fixed; A symmetric) and
    d<x, A u>/dX_k = d<x, w>/dX_k."""
    from . import qtt as T
    X = unflatten(o, nrow, ranks)
    z = T.matvec(A, X)
    w = T.matvec(A, u_cores)
    xx, xu, uu = T.dot(X, z), T.dot(X, w), T.dot(u_cores, w)
    loss = (xx - 2.0 * xu + uu) / uu
    gz = _env_grad(_left_envs(X, z), _right_envs(X, z), z)
    gw = _env_grad(_left_envs(X, w), _right_envs(X, w), w)
    g = [(2.0 * a - 2.0 * b) / uu for a, b in zip(gz, gw)]
    return loss, flatten(g)


def batch_energy_loss_grad(out: np.ndarray, targets, A, nrow, ranks):
    B = out.shape[1]
    g = np.zeros_like(out)
    tot = 0.0
    for j in range(B):
        l, gj = tt_energy_loss_grad(out[:, j], targets[j], A, nrow, ranks)
        tot += l
        g[:, j] = gj / B
    return tot / B, g


def batch_core_loss_grad(out: np.ndarray, targets):
    """The plain loss on the packed cores, for targets brought to one gauge:
    mean over the columns of ||o_j - u_j||^2 / ||u_j||^2 and its gradient
    2 (o_j - u_j) / (B ||u_j||^2)."""
    B = out.shape[1]
    g = np.zeros_like(out)
    tot = 0.0
    for j in range(B):
        u = flatten(targets[j])
        uu = float(u @ u)
        d = out[:, j] - u
        tot += float(d @ d) / uu
        g[:, j] = 2.0 * d / (uu * B)
    return tot / B, g


def align_gauge(x, ref):
    """x with the gauge of ref (same modes and ranks): from the last bond to
    the first, the orthogonal Q that minimises ||Q^T X_k - R_k||_F (over the
    left rank index of core k, the rest of the core flattened) is the polar
    factor U V^T of M = X_k R_k^T = U S V^T (orthogonal Procrustes,
    Schoenemann 1966); core k becomes Q^T X_k and core k-1 becomes X_{k-1} Q,
    which leaves the tensor unchanged.  A bond whose M has a singular value
    below 1e-13 of its largest keeps Q = I."""
    X = [c.copy() for c in x]
    for k in range(len(X) - 1, 0, -1):
        r = X[k].shape[0]
        M = X[k].reshape(r, -1) @ ref[k].reshape(r, -1).T
        U, s, Vt = np.linalg.svd(M)
        if not s[0] > 0.0 or s[-1] <= 1e-13 * s[0]:
            continue
        Q = U @ Vt
        X[k] = np.tensordot(Q.T, X[k], axes=(1, 0))
        X[k - 1] = np.tensordot(X[k - 1], Q, axes=(2, 0))
    return X


def tt_angle_loss_grad(o: np.ndarray, u_cores, nrow, ranks, A=None):
    """Scale-invariant loss L = 1 - <x, u>^2 / (<x, x> <u, u>) of x = TT(o)
    in the Frobenius inner product, or in <v, w>_A = <v, A w> for a
    symmetric positive definite QTT matrix A: the squared relative error of
    the best multiple alpha x, alpha = <x, u> / <x, x>.  With the
    environment gradients Gxx = d<x, x>/dX / 2 and Gxu = d<x, u>/dX,
    dL/dX = 2 <x,u> / (<x,x> <u,u>) (<x,u> / <x,x> Gxx - Gxu)."""
    from . import qtt as T
    X = unflatten(o, nrow, ranks)
    z = T.matvec(A, X) if A is not None else X
    w = T.matvec(A, u_cores) if A is not None else u_cores
    xx, xu, uu = T.dot(X, z), T.dot(X, w), T.dot(u_cores, w)
    loss = 1.0 - xu * xu / (xx * uu)
    gxx = _env_grad(_left_envs(X, z), _right_envs(X, z), z)
    gxu = _env_grad(_left_envs(X, w), _right_envs(X, w), w)
    c = 2.0 * xu / (xx * uu)
    g = [c * (xu / xx * a - b) for a, b in zip(gxx, gxu)]
    return loss, flatten(g)


def batch_angle_loss_grad(out: np.ndarray, targets, nrow, ranks, A=None):
    B = out.shape[1]
    g = np.zeros_like(out)
    tot = 0.0
    for j in range(B):
        l, gj = tt_angle_loss_grad(out[:, j], targets[j], nrow, ranks, A)
        tot += l
        g[:, j] = gj / B
    return tot / B, g
