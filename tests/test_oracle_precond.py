"""Pins of the oracle's BPX preconditioner: nested coarse spaces, exact QTT
form of the dense definition, symmetry and definiteness, and a condition
number of C K that stays bounded while that of K grows 4x per level."""
import numpy as np
import pytest

import workloads as W
from oracle import assembly as A
from oracle import fem
from oracle import precond as PC
from oracle import qtt as T
from oracle import solve as S


@pytest.mark.parametrize("d", [2, 3, 5])
def test_prolongations_are_nested_q1_interpolants(d):
    n = 2 ** d
    for lo, hi in ((False, False), (True, False), (False, True)):
        for l in range(d):
            P = PC.prolongation_1d(d, l, lo, hi)
            Pc = PC.prolongation_1d(d, l + 1, lo, hi)
            if Pc.shape[1] == 0:
                continue
            # every coarser function is a combination of finer ones
            coef, *_ = np.linalg.lstsq(P, Pc, rcond=None)
            assert np.abs(P @ coef - Pc).max() < 1e-12
            if lo:
                assert np.all(P[0] == 0)
            if hi:
                assert np.all(P[-1] == 0)
            if not lo and not hi:
                np.testing.assert_allclose(P.sum(axis=1), 1.0)   # constants reproduced
            # piecewise linear: second differences vanish away from coarse nodes
            H = 2 ** l
            for col in P.T:
                dd = np.diff(col, 2)
                kinks = np.nonzero(np.abs(dd) > 1e-12)[0] + 1
                assert all((k % H == 0) or (hi and (n - 1 - k) % H == 0) for k in kinks)
    assert np.array_equal(PC.prolongation_1d(d, 0, False, False), np.eye(n))


@pytest.mark.parametrize("d", [2, 3, 4])
def test_bpx_qtt_equals_dense(d):
    prob = W.cantilever_traction(d)
    K, f, mask, info = fem.assemble_system(prob)
    Cq = PC.bpx_qtt(prob, info["gamma_D"])
    Cd = PC.bpx_dense(prob, info["gamma_D"])
    perm = fem.qtt_permutation(d)
    Cz = np.zeros_like(Cd)
    Cz[np.ix_(perm, perm)] = Cd
    np.testing.assert_allclose(T.full_matrix(Cq), Cz, atol=1e-12 * np.abs(Cd).max())


def test_bpx_condition_numbers():
    kc, kk = [], []
    for d in (3, 4, 5):
        prob = W.cantilever_traction(d)
        K, f, mask, info = fem.assemble_system(prob)
        Kd = K.toarray()
        Cd = PC.bpx_dense(prob, info["gamma_D"])
        np.testing.assert_allclose(Cd, Cd.T, atol=1e-14)
        assert np.linalg.eigvalsh(Cd).min() > 0
        L = np.linalg.cholesky(Cd)
        ev = np.linalg.eigvalsh(L.T @ Kd @ L)
        # the default lower spectral bound of the Chebyshev solve
        assert ev.min() > 0.09
        kc.append(ev.max() / ev.min())
        kk.append(np.linalg.cond(Kd))
    assert kk[2] / kk[1] > 3.5 and kk[1] / kk[0] > 3.5      # K: x4 per level
    assert max(kc) < 200 and kc[2] / kc[1] < 1.5             # C K: bounded


@pytest.mark.parametrize("d", [3, 4])
def test_oracle_pcg_solve_matches_direct(d):
    prob = W.cantilever_traction(d)
    K, f, mask, info = fem.assemble_system(prob)
    Kq, fq = A.assemble_qtt(prob)
    Cq = PC.bpx_qtt(prob, info["gamma_D"])
    uref, _ = fem.solve_problem(prob)
    u, rep = S.solve(Kq, fq, S.SolveOpts(tol=1e-10, eps=1e-11, eps_in=1e-3, red_in=1e-3,
                                         rmax_in=32), C=Cq)
    assert rep.converged
    assert np.linalg.norm(T.full_vector(u) - uref) <= 1e-9 * np.linalg.norm(uref)
    u0, rep0 = S.solve(Kq, fq, S.SolveOpts(tol=1e-10, eps=1e-11, eps_in=1e-3, red_in=1e-3,
                                           rmax_in=32))
    assert rep.inner < rep0.inner


@pytest.mark.parametrize("d", [3, 4])
def test_oracle_chebyshev_matches_direct(d):
    """Chebyshev iteration on C K u = C f with the true residual every step:
    the energy-type stop at tol gives the direct solution to about tol."""
    prob = W.cantilever_traction(d)
    K, f, mask, info = fem.assemble_system(prob)
    Kq, fq = A.assemble_qtt(prob)
    Cq = PC.bpx_qtt(prob, info["gamma_D"])
    uref, _ = fem.solve_problem(prob)
    Cd = PC.bpx_dense(prob, info["gamma_D"])
    Lc = np.linalg.cholesky(Cd)
    ev = np.linalg.eigvalsh(Lc.T @ K.toarray() @ Lc)
    o = S.ChebOpts(tol=1e-9, eps=1e-12, eps_r=1e-3, eps_d=1e-3, lmin=0.09, lmax=1.05 * ev.max())
    u, rep = S.chebyshev(Kq, fq, Cq, o)
    assert rep.converged
    err = np.linalg.norm(T.full_vector(u) - uref) / np.linalg.norm(uref)
    assert err <= 1e-8
    # an upper bound below the spectrum makes the same iteration diverge
    o.lmax = 0.5 * ev.max()
    o.maxit = 60
    _, rep_bad = S.chebyshev(Kq, fq, Cq, o)
    assert not rep_bad.converged and rep_bad.residuals[-1] > 1.0


@pytest.mark.parametrize("d", [2, 3])
def test_oracle_fcg_untruncated_is_preconditioned_cg(d):
    """Without truncation (every eps 0) flexible CG with one stored direction
    is preconditioned CG: its k-th iterate equals the k-th iterate of
    SciPy's PCG (x0 = 0, preconditioner C applied as z = C r) on the dense
    Z-ordered system.  A wrong sign or operand in alpha or beta breaks the
    K-conjugacy and fails this."""
    import scipy.sparse.linalg as spla
    prob = W.cantilever_traction(d)
    K, f, mask, info = fem.assemble_system(prob)
    Kq, fq = A.assemble_qtt(prob)
    Cq = PC.bpx_qtt(prob, info["gamma_D"])
    Kz = fem.permute_matrix_to_qtt(K, d).toarray()
    fz = fem.to_qtt_order(f, d)
    Cz = T.full_matrix(Cq)
    iterates = []
    spla.cg(Kz, fz, rtol=1e-300, atol=0.0, maxiter=8,
            M=spla.LinearOperator(Kz.shape, matvec=lambda r: Cz @ r),
            callback=lambda xk: iterates.append(xk.copy()))
    assert len(iterates) == 8
    o = S.ChebOpts(tol=0.0, eps=0.0, eps_r=0.0, eps_d=0.0)
    for k in (1, 2, 4, 8):
        o.maxit = k
        u, rep = S.fcg(Kq, fq, Cq, o)
        assert rep.inner == k
        ref = iterates[k - 1]
        err = np.linalg.norm(T.full_vector(u) - ref) / np.linalg.norm(ref)
        assert err <= 1e-9, (k, err)


@pytest.mark.parametrize("d", [3, 4])
def test_oracle_fcg_matches_direct(d):
    """Truncated flexible CG (rounded residual, preconditioned residual and
    direction) reaches the direct solution to about its tolerance."""
    prob = W.cantilever_traction(d)
    K, f, mask, info = fem.assemble_system(prob)
    Kq, fq = A.assemble_qtt(prob)
    Cq = PC.bpx_qtt(prob, info["gamma_D"])
    uref, _ = fem.solve_problem(prob)
    o = S.ChebOpts(tol=1e-9, eps=1e-12, eps_r=1e-3, eps_d=1e-3, maxit=400)
    u, rep = S.fcg(Kq, fq, Cq, o)
    assert rep.converged
    err = np.linalg.norm(T.full_vector(u) - uref) / np.linalg.norm(uref)
    assert err <= 1e-8, err
