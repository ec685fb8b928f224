"""Learned warm start on the GPU: forward pass and gradients of the
gauge-invariant TT loss against the FP64 oracle, and the gain of a network
trained on the method's own solves over the cold start."""
import numpy as np
import pytest

import workloads as W
from oracle import qtt as T
from oracle import warmstart as WS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2501_07778_amd as P
    return P


def _flat_params(params):
    return np.concatenate([np.concatenate([W.reshape(-1, order="F"), b]) for W, b in params])


def test_forward_and_gradient_match_oracle(P):
    nrow = [2] * 7
    ranks = W.capped_ranks(nrow, 6)
    nout = WS.n_out(nrow, ranks)
    sizes = [16, 48, 40, nout]
    params = WS.init_params(sizes, 3)
    B = 9
    a = np.random.default_rng(4).standard_normal((16, B))
    targets = [WS.pad_cores(W.random_tt_cores(30 + j, nrow, W.capped_ranks(nrow, 3)), ranks)
               for j in range(B)]
    net = P.MLP(sizes, _flat_params(params).astype(np.float32))
    out = net.infer(a).cpu().numpy().astype(np.float64)
    ref, cache = WS.forward([(W.astype(np.float32).astype(np.float64), b) for W, b in params], a)
    assert np.abs(out - ref).max() <= 2e-5 * np.abs(ref).max()
    # one train step: Adam's first moment after one step is 0.1 * gradient
    tcols = P.columns(np.stack([WS.flatten(t) for t in targets], axis=1))
    loss = net.train_step(P.columns(a), tcols, nrow, ranks, 1e-4)
    rloss, dout = WS.batch_loss_grad(ref, targets, nrow, ranks)
    assert loss == pytest.approx(rloss, rel=1e-4)
    grads = WS.backward(params, cache, dout)
    g_gpu = net.m.cpu().numpy().astype(np.float64) / 0.1
    g_ref = _flat_params(grads)
    assert np.linalg.norm(g_gpu - g_ref) <= 1e-4 * np.linalg.norm(g_ref)
    assert net.c.step == 1


def test_energy_loss_gradient_matches_oracle(P):
    """The energy-norm loss ||x - u||_K^2 / ||u||_K^2 with the device K: loss
    and gradient (through the network) against the oracle."""
    from oracle import assembly as A_
    d = 3
    Kq, _ = A_.assemble_qtt(W.cantilever_traction(d))
    nrow = [c.shape[1] for c in Kq]
    ranks = W.capped_ranks(nrow, 8)
    nout = WS.n_out(nrow, ranks)
    sizes = [16, 32, nout]
    params = WS.init_params(sizes, 5)
    params[-1] = (params[-1][0], WS.flatten(W.random_tt_cores(7, nrow, ranks)))
    B = 5
    a = np.random.default_rng(6).standard_normal((16, B))
    targets = [WS.pad_cores(W.random_tt_cores(40 + j, nrow, W.capped_ranks(nrow, 4)), ranks)
               for j in range(B)]
    net = P.MLP(sizes, _flat_params(params).astype(np.float32))
    K = P.tt_from_cores(Kq)
    tcols = P.columns(np.stack([WS.flatten(t) for t in targets], axis=1))
    loss = net.train_step(P.columns(a), tcols, nrow, ranks, 1e-4, metric=K)
    p32 = [(W_.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64))
           for W_, b in params]
    ref, cache = WS.forward(p32, a)
    rloss, dout = WS.batch_energy_loss_grad(ref, targets, Kq, nrow, ranks)
    assert loss == pytest.approx(rloss, rel=1e-4)
    g_ref = _flat_params(WS.backward(p32, cache, dout))
    g_gpu = net.m.cpu().numpy().astype(np.float64) / 0.1
    assert np.linalg.norm(g_gpu - g_ref) <= 1e-4 * np.linalg.norm(g_ref)


def test_warm_start_reduces_solve_iterations(P):
    """Level 3: 16 unit-load solves by the method give targets by
    superposition; the network is trained in the energy norm of K (a guess
    that is close in the Frobenius norm but rough can have a larger residual
    than zero); its output starts the solve of held-out loads below the cold
    start's preconditioned residual, and the solve needs fewer iterations."""
    d = 3
    nrow = [2] * (2 * d + 1)
    ranks = W.capped_ranks(nrow, 16)
    opts = dict(tol=1e-9, eps=1e-11, rmax=16, eps_in=1e-3, rmax_in=16, maxit_in=400,
                check_every=1, method="fcg")
    # held-out solves stop at the preconditioned residual 1e-6
    opts6 = dict(opts, tol=1e-6)
    basis, C = [], None
    K = None
    for k in range(16):
        prob = W.cantilever_two_component(d, np.eye(16)[k])
        K, f = P.assemble(prob)
        if C is None:
            C = P.assemble_bpx(prob)
        u, rep = P.solve(K, f, P.SolveOpts(precond=C, **opts))
        assert rep["status"] == 0
        basis.append(T.tt_round(P.tt_to_cores(u), 1e-12))

    def target(a):
        return WS.pad_cores(T.tt_round(T.add(*basis, coeffs=list(a)), 1e-12, 16), ranks)

    ntr, nte = 4096, 6
    A = np.stack([W.warmstart_params(s) for s in range(ntr + nte)], axis=1)
    tr = np.stack([WS.flatten(target(A[:, j])) for j in range(ntr)], axis=1)
    nout = WS.n_out(nrow, ranks)
    sizes = [16, 256, 256, 256, nout]
    prm = WS.init_params(sizes, 0)
    # output bias: a random train of unit scale, so that the multilinear map
    # from cores to tensor does not start at its degenerate point 0
    prm[-1] = (prm[-1][0], WS.flatten(W.random_tt_cores(99, nrow, ranks)))
    net = P.MLP(sizes, _flat_params(prm).astype(np.float32))
    a_dev, t_dev = P.columns(A[:, :ntr]), P.columns(tr)
    bs, steps = 256, 3000
    losses = []
    for step in range(steps):
        j0 = (step * bs) % ntr
        lr = 1e-3 if step < steps // 2 else 2e-4
        losses.append(net.train_step(a_dev[:, j0:j0 + bs], t_dev[:, j0:j0 + bs], nrow, ranks, lr,
                                     metric=K))
    assert np.mean(losses[-16:]) < 0.1 * np.mean(losses[:16])
    out = net.infer(A[:, ntr:])
    gains, start = [], []
    for j in range(nte):
        prob = W.cantilever_two_component(d, A[:, ntr + j])
        _, f = P.assemble(prob)
        cold, rc = P.solve(K, f, P.SolveOpts(precond=C, **opts6))
        x0 = P.tt_from_packed(out[:, j], nrow, ranks)
        warm, rw = P.solve(K, f, P.SolveOpts(precond=C, **opts6), x0=x0)
        assert rc["status"] == 0 and rw["status"] == 0
        gains.append(rc["inner"] - rw["inner"])
        start.append(rw["residual_hist"][0])
        u0 = T.full_vector(P.tt_to_cores(x0))
        uc = T.full_vector(P.tt_to_cores(cold))
        assert np.linalg.norm(u0 - uc) < 0.5 * np.linalg.norm(uc)
    print("warm start: initial preconditioned residual", ["%.3f" % v for v in start],
          "iteration savings", gains)
    # the network's guess starts the iteration below the cold start's 1.0
    assert np.mean(start) < 1.0 and np.mean(gains) > 0
