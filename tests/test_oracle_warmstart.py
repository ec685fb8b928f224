"""Pins of the warm-start oracle: the TT loss equals the dense relative
error, its gradient and the MLP backward pass match finite differences, and
Adam reduces the loss on a tiny problem and takes hand-computed steps."""
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


def test_adam_two_steps_match_hand_computation():
    """Adam (Kingma and Ba 2015, bias-corrected moments, b1 = 0.9,
    b2 = 0.999, eps 1e-8, lr 0.01) on one weight and one bias, gradients
    (2, -1/2) then (-1, 4).  Step 1: the corrected moments are g and g^2, so
    each parameter moves by -lr g / (|g| + eps).  Step 2, weight (exact
    fractions): m = 0.9 (0.2) + 0.1 (-1) = 2/25, m / (1 - 0.81) = 8/19;
    v = 0.999 (0.004) + 0.001 (1) = 1249/250000, v / (1 - 0.998001) =
    4996/1999; bias: m = 71/200 -> 71/38, v = 64999/4000000 -> 64999/7996.
    The printed deltas are -lr (corrected m) / (sqrt(corrected v) + eps).
    A missing bias correction or swapped b1 and b2 changes step 2."""
    params = [[np.array([[1.0]]), np.array([0.5])]]
    m = [[np.zeros((1, 1)), np.zeros(1)]]
    v = [[np.zeros((1, 1)), np.zeros(1)]]
    g1 = [[np.array([[2.0]]), np.array([-0.5])]]
    g2 = [[np.array([[-1.0]]), np.array([4.0])]]
    WS.adam_update(params, g1, m, v, 0, 0.01)
    assert params[0][0][0, 0] == pytest.approx(1.0 - 0.009999999950000001, abs=1e-15)
    assert params[0][1][0] == pytest.approx(0.5 + 0.009999999800000003, abs=1e-15)
    WS.adam_update(params, g2, m, v, 1, 0.01)
    assert params[0][0][0, 0] == pytest.approx(1.0 - 0.009999999950000001
                                               - 0.002663370379756864, abs=1e-14)
    assert params[0][1][0] == pytest.approx(0.5 + 0.009999999800000003
                                            - 0.006553266139001128, abs=1e-14)


def _orthogonal(rng, r):
    q, rr = np.linalg.qr(rng.standard_normal((r, r)))
    return q * np.sign(np.diag(rr))


def test_align_gauge_undoes_a_known_gauge_change():
    """Insert random orthogonal G_k G_k^T at every bond of a train (same
    tensor, other cores): aligning the result to the original recovers the
    original cores exactly (the Procrustes optimum is the inverse rotation,
    with zero residual), and the tensor never changes."""
    rng = np.random.default_rng(5)
    nrow = [2, 3, 2, 2, 4, 2]
    ranks = W.capped_ranks(nrow, 5)
    x = W.random_tt_cores(11, nrow, ranks)
    y = [c.copy() for c in x]
    for k in range(1, len(nrow)):
        G = _orthogonal(rng, ranks[k])
        y[k - 1] = np.tensordot(y[k - 1], G, axes=(2, 0))
        y[k] = np.tensordot(G.T, y[k], axes=(1, 0))
    assert max(np.abs(a - b).max() for a, b in zip(x, y)) > 0.1
    z = WS.align_gauge(y, x)
    assert max(np.abs(a - b).max() for a, b in zip(x, z)) <= 1e-12
    assert np.abs(T.full_vector(z) - T.full_vector(y)).max() <= 1e-12 * np.abs(T.full_vector(y)).max()


def test_align_gauge_minimises_the_core_distance():
    """For two unrelated trains the aligned last core is closer to the
    reference's than under any of 200 random orthogonal rotations (the
    Procrustes optimality of each step), and the tensor is unchanged."""
    rng = np.random.default_rng(6)
    nrow = [2] * 6
    ranks = W.capped_ranks(nrow, 4)
    x = W.random_tt_cores(21, nrow, ranks)
    ref = W.random_tt_cores(22, nrow, ranks)
    z = WS.align_gauge(x, ref)
    D = len(nrow)
    best = np.linalg.norm(z[D - 1] - ref[D - 1])
    r = ranks[D - 1]
    for _ in range(200):
        Q = _orthogonal(rng, r)
        assert best <= np.linalg.norm(np.tensordot(Q.T, x[D - 1], axes=(1, 0)) - ref[D - 1]) + 1e-12
    assert np.abs(T.full_vector(z) - T.full_vector(x)).max() <= 1e-12 * np.abs(T.full_vector(x)).max()


def test_core_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    nrow, ranks, u = _setup(seed=3)
    B = 3
    targets = [u] + [W.random_tt_cores(40 + j, nrow, ranks) for j in range(B - 1)]
    out = rng.standard_normal((WS.n_out(nrow, ranks), B))
    loss, g = WS.batch_core_loss_grad(out, targets)
    flat = [WS.flatten(t) for t in targets]
    dense = np.mean([np.sum((out[:, j] - flat[j]) ** 2) / np.sum(flat[j] ** 2) for j in range(B)])
    assert loss == pytest.approx(dense, rel=1e-13)
    h = 1e-6
    for (i, j) in [(0, 0), (5, 1), (WS.n_out(nrow, ranks) - 1, 2)]:
        op, om = out.copy(), out.copy()
        op[i, j] += h
        om[i, j] -= h
        fd = (WS.batch_core_loss_grad(op, targets)[0] - WS.batch_core_loss_grad(om, targets)[0]) / (2 * h)
        assert g[i, j] == pytest.approx(fd, rel=1e-6, abs=1e-10)


@pytest.mark.parametrize("metric", [False, True])
def test_angle_loss_is_the_error_of_the_best_multiple(metric):
    """The angle loss equals ||alpha x - u||^2 / ||u||^2 (dense, alpha the
    least-squares multiple, in the Frobenius or the K norm), is unchanged by
    scaling x, and its gradient matches finite differences."""
    from oracle import assembly as A_
    nrow, ranks, _ = _setup(seed=8, D=7, r=3)
    A = None
    if metric:
        Kq, _ = A_.assemble_qtt(W.cantilever_traction(3))
        A = Kq
        nrow = [c.shape[1] for c in Kq]
        ranks = W.capped_ranks(nrow, 3)
    u = W.random_tt_cores(9, nrow, ranks)
    o = np.random.default_rng(10).standard_normal(WS.n_out(nrow, ranks))
    loss, g = WS.tt_angle_loss_grad(o, u, nrow, ranks, A)
    xd = T.full_vector(WS.unflatten(o, nrow, ranks))
    ud = T.full_vector(u)
    M = T.full_matrix(A) if metric else np.eye(xd.size)
    alpha = (xd @ M @ ud) / (xd @ M @ xd)
    e = alpha * xd - ud
    assert loss == pytest.approx((e @ M @ e) / (ud @ M @ ud), rel=1e-10)
    o2 = o.copy()
    o2[:nrow[0] * ranks[1]] *= -3.0          # scales the first core
    assert WS.tt_angle_loss_grad(o2, u, nrow, ranks, A)[0] == pytest.approx(loss, rel=1e-10)
    h = 1e-6
    for i in [0, 7, WS.n_out(nrow, ranks) - 2]:
        op, om = o.copy(), o.copy()
        op[i] += h
        om[i] -= h
        fd = (WS.tt_angle_loss_grad(op, u, nrow, ranks, A)[0]
              - WS.tt_angle_loss_grad(om, u, nrow, ranks, A)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9)
