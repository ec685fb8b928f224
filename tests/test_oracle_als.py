"""Pins of the oracle's one-site ALS (oracle/als.py) against what the
mathematics fixes: the frames are isometries, the local energy identity,
the change of one local solve equals the change of the whole tensor (the
ALS stop rule rests on it), exactness at full rank against the sparse
direct solve, monotone energy, and energy-norm optimality at reduced rank
against the TT-SVD truncation of the exact solution."""
import numpy as np

import workloads as W
from oracle import als as ALS
from oracle import assembly as A
from oracle import fem
from oracle import qtt as T


def _system(d, which="traction"):
    prob = (W.cantilever_traction if which == "traction" else W.cantilever_body_force)(d)
    Kq, fq = A.assemble_qtt(prob)
    return prob, Kq, fq


def test_frames_are_isometries():
    """After the orthogonalisation sweep every frame has orthonormal columns."""
    modes = [2] * 7
    X = W.random_tt_cores(3, modes, W.capped_ranks(modes, 4))
    for k in range(6, 0, -1):
        ALS._lq_step(X, k)
    U = ALS.frame(X, 0)
    np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-13)
    for k in range(6):
        ALS._qr_step(X, k)
        U = ALS.frame(X, k + 1)
        np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-13)
        # the frame reproduces the tensor from its core
        np.testing.assert_allclose(U @ X[k + 1].reshape(-1, order="F"), T.full_vector(X),
                                   atol=1e-12 * np.linalg.norm(T.full_vector(X)))


def test_local_energy_and_change_identities():
    """For every local solve: J(u) = u^T K u / 2 - f^T u equals -y^T g / 2,
    and ||y - x_k|| equals ||u_after - u_before|| (orthonormal frames)."""
    prob, Kq, fq = _system(3)
    Kd, fd = T.full_matrix(Kq), T.full_vector(fq)
    caps = W.capped_ranks([2] * 7, 3)
    _, log = ALS.als(Kq, fq, caps, sweeps=3, seed=1)
    for k, J, dy, before, after in log:
        Jd = 0.5 * after @ Kd @ after - fd @ after
        assert abs(J - Jd) <= 1e-12 * abs(Jd), (k, J, Jd)
        assert abs(dy - np.linalg.norm(after - before)) <= 1e-10 * max(np.linalg.norm(after), 1.0)


def test_energy_never_increases():
    prob, Kq, fq = _system(3, "body")
    caps = W.capped_ranks([2] * 7, 2)
    _, log = ALS.als(Kq, fq, caps, sweeps=4, seed=2)
    J = np.array([e for _, e, _, _, _ in log])
    assert np.all(np.diff(J) <= 1e-13 * np.abs(J[:-1]))


def test_full_rank_equals_direct_solve():
    """With ranks at the mode-product bound the frame of the middle core
    spans the whole space (r_k n r_{k+1} = 2^D), so the first forward sweep
    reaches the sparse direct solution and later solves change nothing."""
    for d in (2, 3):
        prob, Kq, fq = _system(d)
        uref, _ = fem.solve_problem(prob)
        D = 2 * d + 1
        caps = W.capped_ranks([2] * D, 2 ** d)
        X, log = ALS.als(Kq, fq, caps, sweeps=2, seed=d)
        u = T.full_vector(X)
        assert np.linalg.norm(u - uref) <= 1e-11 * np.linalg.norm(uref)
        # the initial solve plus the D - 1 solves of the forward sweep
        assert max(dy for _, _, dy, _, _ in log[D:]) <= 1e-10 * np.linalg.norm(uref)


def test_reduced_rank_is_energy_optimal():
    """ALS minimises the energy, i.e. the K-norm error, over the trains of
    its ranks: at ranks 4 and 6 on level 3 its K-norm error is below that of
    the TT-SVD truncation of the exact solution (a train of the same ranks,
    optimal in the l2 norm instead), while in l2 the truncation is closer."""
    prob, Kq, fq = _system(3)
    uref, _ = fem.solve_problem(prob)
    Kd = T.full_matrix(Kq)

    def energy(v):
        return np.sqrt(v @ Kd @ v)

    for r in (4, 6):
        caps = W.capped_ranks([2] * 7, r)
        X, _ = ALS.als(Kq, fq, caps, sweeps=12, seed=4)
        e_als = T.full_vector(X) - uref
        e_svd = T.full_vector(T.tt_svd(uref, [2] * 7, 0.0, r)) - uref
        assert energy(e_als) <= energy(e_svd) * (1 + 1e-9), (r, energy(e_als), energy(e_svd))
        assert np.linalg.norm(e_svd) <= np.linalg.norm(e_als)
