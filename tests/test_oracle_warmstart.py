"""Pins of the warm-start oracle: the TT loss equals the dense relative
error, its gradient and the MLP backward pass match finite differences, and
Adam reduces the loss on a tiny problem."""
import numpy as np
import pytest

import workloads as W
from oracle import qtt as T
from oracle import warmstart as WS


def _setup(seed=0, D=5, r=3):
    nrow = [2] * D
    ranks = W.capped_ranks(nrow, r)
    u = W.random_tt_cores(seed, nrow, ranks)
    return nrow, ranks, u


def test_loss_is_dense_relative_error_and_gauge_invariant():
    nrow, ranks, u = _setup()
    o = np.random.default_rng(1).standard_normal(WS.n_out(nrow, ranks))
    loss, _ = WS.tt_loss_grad(o, u, nrow, ranks)
    xd = T.full_vector(WS.unflatten(o, nrow, ranks))
    ud = T.full_vector(u)
    assert loss == pytest.approx(np.linalg.norm(xd - ud) ** 2 / np.linalg.norm(ud) ** 2, rel=1e-12)
    # a gauge change (G_k S, S^-1 G_{k+1}) leaves the loss unchanged
    X = WS.unflatten(o, nrow, ranks)
    S = np.random.default_rng(2).standard_normal((ranks[2], ranks[2])) + 3 * np.eye(ranks[2])
    X[1] = np.einsum("aib,bc->aic", X[1], S)
    X[2] = np.einsum("cb,bid->cid", np.linalg.inv(S), X[2])
    l2, _ = WS.tt_loss_grad(WS.flatten(X), u, nrow, ranks)
    assert l2 == pytest.approx(loss, rel=1e-10)
    # the target itself gives zero loss
    l0, g0 = WS.tt_loss_grad(WS.flatten(u), u, nrow, ranks)
    assert abs(l0) < 1e-12 and np.abs(g0).max() < 1e-10


def test_loss_gradient_matches_finite_differences():
    nrow, ranks, u = _setup(3)
    rng = np.random.default_rng(4)
    o = rng.standard_normal(WS.n_out(nrow, ranks))
    _, g = WS.tt_loss_grad(o, u, nrow, ranks)
    h = 1e-6
    for idx in rng.choice(o.size, 12, replace=False):
        e = np.zeros_like(o)
        e[idx] = h
        fd = (WS.tt_loss_grad(o + e, u, nrow, ranks)[0] - WS.tt_loss_grad(o - e, u, nrow, ranks)[0]) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-6, abs=1e-9)


def test_mlp_backward_matches_finite_differences():
    nrow, ranks, u = _setup(5)
    P = WS.n_out(nrow, ranks)
    params = WS.init_params([4, 7, 6, P], 6)
    a = np.random.default_rng(7).standard_normal((4, 3))
    targets = [u, [c * 0.5 for c in u], u]

    def total(params):
        out, _ = WS.forward(params, a)
        return WS.batch_loss_grad(out, targets, nrow, ranks)[0]

    out, cache = WS.forward(params, a)
    _, dout = WS.batch_loss_grad(out, targets, nrow, ranks)
    grads = WS.backward(params, cache, dout)
    h = 1e-6
    rng = np.random.default_rng(8)
    for l in range(3):
        for p in range(2):
            arr = params[l][p]
            for flat in rng.choice(arr.size, 4, replace=False):
                idx = np.unravel_index(flat, arr.shape)
                old = arr[idx]
                arr[idx] = old + h
                fp = total(params)
                arr[idx] = old - h
                fm = total(params)
                arr[idx] = old
                assert (fp - fm) / (2 * h) == pytest.approx(grads[l][p][idx], rel=1e-5, abs=1e-9)


def test_adam_fits_a_linear_family():
    """u(a) = sum_k a_k u_k: the MLP learns it well below the zero guess."""
    nrow = [2] * 4
    ranks = W.capped_ranks(nrow, 4)
    basis = [W.random_tt_cores(10 + k, nrow, W.capped_ranks(nrow, 1)) for k in range(3)]
    rng = np.random.default_rng(0)
    A = rng.standard_normal((3, 64))

    def target(a):
        t = T.add(*basis, coeffs=list(a))
        return WS.pad_cores(T.tt_round(t, 1e-12, 4), ranks)

    targets = [target(A[:, j]) for j in range(A.shape[1])]
    params = WS.init_params([3, 32, 32, WS.n_out(nrow, ranks)], 1)
    m = [[np.zeros_like(p) for p in layer] for layer in params]
    v = [[np.zeros_like(p) for p in layer] for layer in params]
    losses = []
    for step in range(300):
        out, cache = WS.forward(params, A)
        loss, dout = WS.batch_loss_grad(out, targets, nrow, ranks)
        losses.append(loss)
        WS.adam_update(params, WS.backward(params, cache, dout), m, v, step, 3e-3)
    assert losses[0] > 0.5 and losses[-1] < 0.05


def test_energy_loss_matches_dense_and_finite_differences():
    from oracle import assembly as A_
    d = 2
    prob = W.cantilever_traction(d)
    Kq, _ = A_.assemble_qtt(prob)
    nrow = [c.shape[1] for c in Kq]
    ranks = W.capped_ranks(nrow, 4)
    u = W.random_tt_cores(11, nrow, ranks)
    o = np.random.default_rng(12).standard_normal(WS.n_out(nrow, ranks))
    loss, g = WS.tt_energy_loss_grad(o, u, Kq, nrow, ranks)
    Kd = T.full_matrix(Kq)
    e = T.full_vector(WS.unflatten(o, nrow, ranks)) - T.full_vector(u)
    ud = T.full_vector(u)
    assert loss == pytest.approx((e @ Kd @ e) / (ud @ Kd @ ud), rel=1e-11)
    h = 1e-6
    rng = np.random.default_rng(13)
    for idx in rng.choice(o.size, 10, replace=False):
        de = np.zeros_like(o)
        de[idx] = h
        fd = (WS.tt_energy_loss_grad(o + de, u, Kq, nrow, ranks)[0]
              - WS.tt_energy_loss_grad(o - de, u, Kq, nrow, ranks)[0]) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-5, abs=1e-8)
