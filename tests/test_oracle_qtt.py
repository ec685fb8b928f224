"""Pins of the CPU QTT oracle: brute force against dense linear algebra on
small tensors, the TT-SVD/rounding guarantees, and the exact reconstruction
of the sparse FEM stiffness and load from their QTT forms."""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import workloads as W
from oracle import assembly as A
from oracle import fem
from oracle import qtt as T
from oracle import solve as S


def _rand_tt(seed, modes, r, ncol=None):
    ranks = W.capped_ranks(modes, r) if ncol is None else W.capped_ranks(
        [a * b for a, b in zip(modes, ncol)], r)
    return W.random_tt_cores(seed, modes, ranks, ncol=ncol)


def test_full_vector_digit_order():
    """Unit tensor e_(i1) x ... x e_(iD) sits at index sum_k i_k 2^(k-1)
    (binary quantisation, first digit least significant)."""
    digits = [1, 0, 1, 1, 0]
    cores = []
    for b in digits:
        c = np.zeros((1, 2, 1))
        c[0, b, 0] = 1
        cores.append(c)
    v = T.full_vector(cores)
    idx = sum(b << k for k, b in enumerate(digits))
    assert v[idx] == 1 and v.sum() == 1


def test_full_matrix_digit_order():
    rb, cb = [1, 0, 1], [0, 1, 1]
    cores = []
    for a, b in zip(rb, cb):
        c = np.zeros((1, 2, 2, 1))
        c[0, a, b, 0] = 1
        cores.append(c)
    M = T.full_matrix(cores)
    i = sum(a << k for k, a in enumerate(rb))
    j = sum(b << k for k, b in enumerate(cb))
    assert M[i, j] == 1 and M.sum() == 1


@settings(max_examples=25, deadline=None)
@given(st.integers(0, 10 ** 6), st.integers(2, 6), st.integers(1, 5), st.integers(2, 3))
def test_matvec_matches_dense(seed, D, r, n):
    modes = [n] * D
    A_ = _rand_tt(seed, modes, r + 1, ncol=modes)
    x = _rand_tt(seed + 1, modes, r)
    y = T.matvec(A_, x)
    np.testing.assert_allclose(T.full_vector(y), T.full_matrix(A_) @ T.full_vector(x),
                               rtol=1e-12, atol=1e-12 * np.abs(T.full_vector(y)).max())
    assert T.ranks(y) == [a * b for a, b in zip(T.ranks(A_), T.ranks(x))]


@settings(max_examples=25, deadline=None)
@given(st.integers(0, 10 ** 6), st.integers(2, 7), st.integers(1, 6))
def test_dot_add_hadamard_match_dense(seed, D, r):
    modes = [2] * D
    x = _rand_tt(seed, modes, r)
    y = _rand_tt(seed + 7, modes, r + 1)
    xd, yd = T.full_vector(x), T.full_vector(y)
    assert T.dot(x, y) == pytest.approx(xd @ yd, rel=1e-11, abs=1e-12)
    assert T.norm(x) == pytest.approx(np.linalg.norm(xd), rel=1e-12)
    np.testing.assert_allclose(T.full_vector(T.add(x, y, coeffs=[0.5, -2.0])), 0.5 * xd - 2 * yd,
                               atol=1e-12)
    np.testing.assert_allclose(T.full_vector(T.hadamard(x, y)), xd * yd, atol=1e-12)


@settings(max_examples=20, deadline=None)
@given(st.integers(0, 10 ** 6), st.integers(2, 7), st.integers(1, 12),
       st.sampled_from([0.0, 1e-12, 1e-6, 1e-3, 0.1]))
def test_round_guarantee(seed, D, r, eps):
    """||y - round(y)|| <= eps ||y|| and ranks bounded by the unfolding sizes."""
    modes = [2] * D
    y = _rand_tt(seed, modes, r)
    z, info = T.tt_round(y, eps, return_info=True)
    yd, zd = T.full_vector(y), T.full_vector(z)
    err = np.linalg.norm(yd - zd)
    assert err <= eps * np.linalg.norm(yd) * (1 + 1e-10) + 1e-13 * np.linalg.norm(yd)
    assert info["norm"] == pytest.approx(np.linalg.norm(yd), rel=1e-12)
    assert info["err"] == pytest.approx(err, rel=1e-6, abs=1e-13 * np.linalg.norm(yd))
    rk = T.ranks(z)
    for k in range(1, D):
        assert rk[k] <= min(2 ** k, 2 ** (D - k))


def test_round_singular_values_equal_dense_unfoldings():
    """Without truncation the per-bond singular values of the rounding are
    those of the dense unfoldings (left digits x right digits)."""
    modes = [2, 3, 2, 2, 2, 3]
    y = _rand_tt(11, modes, 5)
    _, info = T.tt_round(y, 0.0, return_info=True)
    yd = T.full_vector(y)
    for k in range(1, len(modes)):
        left = int(np.prod(modes[:k]))
        s = np.linalg.svd(np.reshape(yd, (left, -1), order="F"), compute_uv=False)
        sk = info["sigma"][k]
        m = min(len(s), len(sk))
        np.testing.assert_allclose(sk[:m], s[:m], rtol=1e-10, atol=1e-13 * s[0])
        assert np.all(s[m:] < 1e-12 * s[0])


def test_round_idempotent_and_rank_cap():
    y = _rand_tt(5, [2] * 8, 8)
    z = T.tt_round(y, 1e-3)
    z2 = T.tt_round(z, 1e-3)
    assert T.ranks(z2) == T.ranks(z)
    np.testing.assert_allclose(T.full_vector(z2), T.full_vector(z), atol=1e-12)
    c = T.tt_round(y, 0.0, rmax=3)
    assert max(T.ranks(c)) <= 3
    # the capped result is the right-to-left truncated SVD sweep: its error
    # equals the reported bound up to rounding
    _, info = T.tt_round(y, 0.0, rmax=3, return_info=True)
    err = np.linalg.norm(T.full_vector(c) - T.full_vector(y))
    assert err == pytest.approx(info["err"], rel=1e-8)


def test_round_zero_tensor():
    y = [np.zeros((1, 2, 3)), np.zeros((3, 2, 2)), np.zeros((2, 2, 1))]
    z = T.tt_round(y, 1e-8)
    assert T.ranks(z) == [1, 1, 1, 1]
    assert np.all(T.full_vector(z) == 0)


def test_tt_svd_matches_brute_force():
    rng = np.random.default_rng(3)
    a = rng.standard_normal(2 ** 8)
    c = T.tt_svd(a, [2] * 8, 0.0)
    np.testing.assert_allclose(T.full_vector(c), a, atol=1e-12)
    # a sampled function with exact QTT rank 2: sin(omega j)
    j = np.arange(2 ** 10)
    c = T.tt_svd(np.sin(0.37 * j), [2] * 10, 1e-12)
    assert max(T.ranks(c)) == 2


@pytest.mark.parametrize("d", [1, 2, 4, 6])
def test_one_d_factors(d):
    n = 2 ** d
    np.testing.assert_array_equal(T.full_matrix(A.qtt_shift(d)), np.eye(n, k=1))
    assert max(T.ranks(A.qtt_shift(d))) <= 2
    h = 0.37
    K1, M1, G1 = A.one_d_matrices(d, h)
    K1d = (2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)) / h
    K1d[0, 0] = K1d[-1, -1] = 1 / h
    M1d = (4 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)) * h / 6
    M1d[0, 0] = M1d[-1, -1] = 2 * h / 6
    if n == 2:
        K1d = np.array([[1, -1], [-1, 1]]) / h
        M1d = np.array([[2, 1], [1, 2]]) * h / 6
    # G1[a, b] = int phi_a' phi_b by the trapezoid-exact element rule
    G1d = np.zeros((n, n))
    for e in range(n - 1):
        G1d[e, e] += -0.5
        G1d[e, e + 1] += -0.5
        G1d[e + 1, e] += 0.5
        G1d[e + 1, e + 1] += 0.5
    np.testing.assert_allclose(T.full_matrix(K1), K1d, atol=1e-13 / h)
    np.testing.assert_allclose(T.full_matrix(M1), M1d, atol=1e-14)
    np.testing.assert_allclose(T.full_matrix(G1), G1d, atol=1e-14)
    j = np.arange(n)
    np.testing.assert_allclose(T.full_vector(A.qtt_sine(d, 0.71)), np.sin(0.71 * j), atol=1e-13)


def test_zkron_is_zordered_kronecker():
    d = 3
    n = 2 ** d
    X = _rand_tt(1, [2] * d, 2, ncol=[2] * d)
    Y = _rand_tt(2, [2] * d, 3, ncol=[2] * d)
    Zc = T.zkron(Y, X)
    dense = np.kron(T.full_matrix(Y), T.full_matrix(X))      # canonical i + n j
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    zi = fem.zorder(i, j, d).ravel(order="F")               # canonical -> Z
    Pd = np.zeros((n * n, n * n))
    Pd[zi, np.arange(n * n)] = 1
    np.testing.assert_allclose(T.full_matrix(Zc), Pd @ dense @ Pd.T, atol=1e-13)


@pytest.mark.parametrize("d", [2, 3, 4])
@pytest.mark.parametrize("which", ["body", "traction", "lshape", "lshape-paper"])
def test_qtt_assembly_equals_sparse_fem(d, which):
    """dense(QTT K) and dense(QTT f) equal the element-loop sparse system,
    permuted to Z-order (Alg. 1 realised with z-kron)."""
    coupling = "paper" if which == "lshape-paper" else "symmetric"
    prob = {"body": W.cantilever_body_force, "traction": W.cantilever_traction,
            "lshape": W.l_shape, "lshape-paper": W.l_shape}[which](d)
    K, f, _, _ = fem.assemble_system(prob, coupling)
    Kz = fem.permute_matrix_to_qtt(K, d, prob.q).toarray()
    fz = fem.to_qtt_order(f, d, prob.q)
    Kq, fq = A.assemble_qtt(prob, coupling)
    np.testing.assert_allclose(T.full_matrix(Kq), Kz, atol=1e-13 * np.abs(Kz).max())
    np.testing.assert_allclose(T.full_vector(fq), fz, atol=1e-13 * np.abs(fz).max())


def test_stiffness_rank_profile():
    """Operator ranks with the component core first plateau at 25
    (clamped unit square) for every level."""
    for d in (5, 6):
        Kq, _ = A.assemble_qtt(W.cantilever_traction(d))
        r = T.ranks(Kq)
        assert r[:4] == [1, 4, 14, 23] and max(r) == 25 and r[-3:] == [16, 4, 1]


@pytest.mark.parametrize("d", [3, 4])
def test_oracle_solve_matches_direct(d):
    prob = W.cantilever_body_force(d)
    uref, _ = fem.solve_problem(prob)
    Kq, fq = A.assemble_qtt(prob)
    u, rep = S.solve(Kq, fq, S.SolveOpts(tol=1e-10, eps=1e-10, eps_in=1e-3, red_in=1e-2, rmax_in=32))
    assert rep.converged
    err = np.linalg.norm(T.full_vector(u) - uref) / np.linalg.norm(uref)
    assert err < 1e-9


def test_effective_rank():
    """r_e of a TT whose ranks are all r equals r (storage equation of Sec. 4)."""
    D, r = 6, 4
    cores = W.random_tt_cores(0, [2] * D, [1] + [r] * (D - 1) + [1])
    assert T.effective_rank(cores) == pytest.approx(r)
