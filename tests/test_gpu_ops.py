"""Parity of the HIP tensor-train operations with the FP64 CPU oracle, through
the C ABI, on seeded random tensor trains (several tiles, ragged ranks, odd
modes) and at the bond shapes of the level-10 workload."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import qtt as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2501_07778_amd as P
    return P


def _vec(seed, modes, r):
    return W.random_tt_cores(seed, modes, W.capped_ranks(modes, r))


def _mat(seed, modes, r):
    ranks = W.capped_ranks([m * m for m in modes], r)
    return W.random_tt_cores(seed, modes, ranks, ncol=modes)


CASES = [
    ([2, 2, 2, 2, 2], 3, 4),
    ([2, 3, 2, 2, 2, 2], 5, 7),
    ([2, 2, 2, 2, 2, 2, 2, 2, 2], 9, 33),    # ragged: 33 spans several 64-lanes
    ([2] * 11, 25, 70),                     # ranks beyond one wave along b
    ([2], 1, 1),
]


@pytest.mark.parametrize("modes,ra,rx", CASES)
@pytest.mark.parametrize("compute", ["f64"])
def test_matvec_cores_bit_close(P, modes, ra, rx, compute):
    A = _mat(1, modes, ra)
    x = _vec(2, modes, rx)
    y_ref = T.matvec(A, x)
    y = P.matvec(P.tt_from_cores(A), P.tt_from_cores(x), compute)
    assert y.ranks == T.ranks(y_ref)
    got = P.tt_to_cores(y)
    for g, r in zip(got, y_ref):
        # each output is a sum of m products: equal up to the order of rounding
        scale = np.abs(r).max() + 1e-300
        assert np.abs(g - r).max() <= 4e-16 * scale * 4


@pytest.mark.parametrize("compute,tol", [("f32", 2e-6), ("bf16", 2e-2)])
def test_matvec_low_precision(P, compute, tol):
    modes = [2] * 9
    A = _mat(3, modes, 7)
    x = _vec(4, modes, 12)
    y_ref = T.full_vector(T.matvec(A, x))
    y = P.matvec(P.tt_from_cores(A), P.tt_from_cores(x), compute)
    yd = T.full_vector(P.tt_to_cores(y))
    assert np.linalg.norm(yd - y_ref) <= tol * np.linalg.norm(y_ref)


@pytest.mark.parametrize("modes,r,eps,rmax", [
    ([2] * 6, 5, 1e-10, 0),
    ([2, 3, 2, 2, 2, 2, 2], 9, 1e-6, 0),
    ([2] * 10, 20, 1e-3, 0),
    ([2] * 10, 20, 0.0, 6),
    ([4] * 5, 12, 1e-8, 0),
    ([2] * 8, 70, 1e-12, 0),                 # unfoldings larger than a tile
    ([2] * 16, 128, 1e-10, 0),               # Jacobi with logged rotations replayed
    ([2] * 16, 128, 1e-3, 40),
    ([2] * 12, 200, 1e-9, 0),                # global-memory Jacobi, > 64 pairs per round
])
def test_round_matches_oracle(P, modes, r, eps, rmax):
    y = _vec(7, modes, r)
    ref, info = T.tt_round(y, eps, rmax if rmax > 0 else 1 << 30, return_info=True)
    t = P.tt_from_cores(y)
    nrm, err = P.round_(t, eps, rmax)
    got = P.tt_to_cores(t)
    yd = T.full_vector(y)
    gd = T.full_vector(got)
    rd = T.full_vector(ref)
    assert nrm == pytest.approx(info["norm"], rel=1e-12)
    # rounding guarantee against the exact tensor
    if rmax == 0:
        assert np.linalg.norm(gd - yd) <= eps * np.linalg.norm(yd) * (1 + 1e-8) + 1e-13 * np.linalg.norm(yd)
    # same tensor as the oracle up to FP64 noise (gauge-free comparison)
    assert np.linalg.norm(gd - rd) <= 1e-11 * np.linalg.norm(yd) + 2 * max(err, info["err"])
    # ranks: equal, or off by one at a near-tie of singular values
    for a, b in zip(t.ranks, T.ranks(ref)):
        assert abs(a - b) <= 1
    assert err == pytest.approx(info["err"], rel=1e-6, abs=1e-13 * np.linalg.norm(yd))
    # result is right-orthogonal except the first core
    for c in got[1:]:
        M = c.reshape(c.shape[0], -1, order="F")
        np.testing.assert_allclose(M @ M.T, np.eye(c.shape[0]), atol=1e-12)


@pytest.mark.parametrize("modes,r", [([2] * 10, 12), ([2] * 8, 37), ([2, 3, 2, 2, 2, 2], 9)])
def test_round_degenerate_unfoldings(P, modes, r):
    """Degenerate inputs of the SVD steps, against the oracle's rounding:
    x + x (core concatenation) doubles every rank with exactly dependent
    columns, and zeroing one rank component of a middle core leaves zero
    columns in its unfoldings.  The rounded tensors match the oracle's, the
    ranks come back to the oracle's, and the kept cores stay orthonormal."""
    x = _vec(31, modes, r)
    z = [c.copy() for c in x]
    mid = len(z) // 2
    z[mid][:, :, 0] = 0.0
    for y in (T.add(x, x), z):
        ref, info = T.tt_round(y, 1e-12, return_info=True)
        t = P.tt_from_cores(y)
        nrm, err = P.round_(t, 1e-12, 0)
        got = P.tt_to_cores(t)
        yd = T.full_vector(y)
        gd = T.full_vector(got)
        assert nrm == pytest.approx(info["norm"], rel=1e-12)
        assert np.linalg.norm(gd - yd) <= 1e-11 * np.linalg.norm(yd)
        assert np.linalg.norm(gd - T.full_vector(ref)) <= 1e-11 * np.linalg.norm(yd)
        assert t.ranks == T.ranks(ref), (t.ranks, T.ranks(ref))
        for c in got[1:]:
            M = c.reshape(c.shape[0], -1, order="F")
            np.testing.assert_allclose(M @ M.T, np.eye(c.shape[0]), atol=1e-12)


def test_round_of_matvec_product(P):
    """The hot-path combination: round(K x) against the oracle."""
    from oracle import assembly as A
    prob = W.cantilever_traction(4)
    Kq, fq = A.assemble_qtt(prob)
    x = T.tt_round(fq, 1e-12)
    ref, info = T.tt_round(T.matvec(Kq, x), 1e-8, return_info=True)
    y = P.matvec(P.tt_from_cores(Kq), P.tt_from_cores(x))
    nrm, err = P.round_(y, 1e-8)
    gd = T.full_vector(P.tt_to_cores(y))
    rd = T.full_vector(ref)
    assert nrm == pytest.approx(info["norm"], rel=1e-12)
    assert np.linalg.norm(gd - rd) <= 2e-8 * np.linalg.norm(rd)


def test_round_zero_and_single_core(P):
    y = [np.zeros((1, 2, 3)), np.zeros((3, 2, 2)), np.zeros((2, 2, 1))]
    t = P.tt_from_cores(y)
    nrm, err = P.round_(t, 1e-8)
    assert nrm == 0.0 and t.ranks == [1, 1, 1, 1]
    assert np.all(T.full_vector(P.tt_to_cores(t)) == 0)
    one = [np.arange(6, dtype=float).reshape(1, 6, 1)]
    t = P.tt_from_cores(one)
    nrm, _ = P.round_(t, 1e-8)
    assert nrm == pytest.approx(np.linalg.norm(np.arange(6)))


@pytest.mark.parametrize("modes,r1,r2", [([2] * 7, 5, 9), ([2, 3, 2, 2], 2, 3), ([2] * 12, 40, 17)])
def test_dot_and_axpby(P, modes, r1, r2):
    x = _vec(11, modes, r1)
    y = _vec(12, modes, r2)
    tx, ty = P.tt_from_cores(x), P.tt_from_cores(y)
    assert P.dot(tx, ty) == pytest.approx(T.dot(x, y), rel=1e-12, abs=1e-14)
    z = P.axpby(0.5, tx, -2.0, ty)
    ref = T.add(x, y, coeffs=[0.5, -2.0])
    assert z.ranks == T.ranks(ref)
    for g, r in zip(P.tt_to_cores(z), ref):
        np.testing.assert_array_equal(g, r)


def test_matvec_level10_shapes_sampled(P):
    """Full-size bond shapes of the level-10 traction workload (operator rank
    25, vector rank 64, 21 cores): cores of the product checked on sampled
    cores against the oracle's formula, computed one core at a time."""
    from oracle import assembly as A
    Kq, _ = A.assemble_qtt(W.cantilever_traction(10))
    modes = [2] * 21
    x = W.random_tt_cores(5, modes, W.capped_ranks(modes, 64))
    y = P.matvec(P.tt_from_cores(Kq), P.tt_from_cores(x))
    got = P.tt_to_cores(y)
    for k in (0, 1, 7, 10, 15, 20):
        ref = T.matvec([Kq[k]], [x[k]])[0]
        assert np.abs(got[k] - ref).max() <= 2e-15 * np.abs(ref).max()


@pytest.mark.parametrize("ell,eps", [(12, 1e-6), (30, 1e-10)])
def test_sketch_rounding_against_exact(P, ell, eps):
    """Randomised rounding (Gaussian sketch of rank ell, then the exact
    rounding) of a matvec product: its error against the exact tensor is close
    to the oracle's best error at the same final ranks."""
    from oracle import assembly as A
    prob = W.cantilever_traction(5)
    Kq, fq = A.assemble_qtt(prob)
    x = T.tt_round(_vec(3, [2] * 11, 6), 0.0)
    y = T.matvec(Kq, x)
    yd = T.full_vector(y)
    ref, info = T.tt_round(y, eps, return_info=True)
    t = P.matvec(P.tt_from_cores(Kq), P.tt_from_cores(x))
    nrm, err = P.round_sketch(t, ell, 11, eps, 0)
    gd = T.full_vector(P.tt_to_cores(t))
    assert max(t.ranks) <= ell
    # the sketch captures the dominant subspace: the error is at most a
    # small multiple of the rank-ell optimum plus the requested accuracy
    opt, _ = T.tt_round(y, 0.0, ell, return_info=True)
    best = np.linalg.norm(T.full_vector(opt) - yd)
    assert np.linalg.norm(gd - yd) <= 10 * best + 2 * eps * np.linalg.norm(yd)


@pytest.mark.parametrize("ell", [0, 40])
def test_matvec_round_fused(P, ell):
    """qtt_matvec_round equals round(A x) of the oracle (exact path) and the
    separate product + sketch rounding (same seed, same sketch)."""
    from oracle import assembly as A
    Kq, fq = A.assemble_qtt(W.cantilever_traction(5))
    x = T.tt_round(_vec(3, [2] * 11, 6), 0.0)
    yref = T.full_vector(T.matvec(Kq, x))
    K, tx = P.tt_from_cores(Kq), P.tt_from_cores(x)
    y, nrm, err = P.matvec_round(K, tx, ell, 9, 1e-10, 0)
    yd = T.full_vector(P.tt_to_cores(y))
    assert nrm == pytest.approx(np.linalg.norm(yref), rel=1e-10)
    if ell == 0:
        ref = T.full_vector(T.tt_round(T.matvec(Kq, x), 1e-10))
        assert np.linalg.norm(yd - ref) <= 1e-12 * np.linalg.norm(yref) + 2e-10 * np.linalg.norm(yref)
        assert np.linalg.norm(yd - yref) <= 1e-10 * np.linalg.norm(yref) * (1 + 1e-6)
    else:
        t = P.matvec(K, tx)
        P.round_sketch(t, ell, 9, 1e-10, 0)
        td = T.full_vector(P.tt_to_cores(t))
        assert y.ranks == t.ranks
        assert np.linalg.norm(yd - td) <= 1e-12 * np.linalg.norm(yref)


def test_matvec_round_batched_equals_single(P):
    """Hot steps of different levels and ranks run by 3 workers on their own
    streams equal the same steps run one at a time (same sketch seeds)."""
    from oracle import assembly as A
    items = []
    for i, (d, r) in enumerate([(4, 8), (5, 12), (3, 5), (6, 16), (5, 7)]):
        Kq, _ = A.assemble_qtt(W.cantilever_traction(d))
        modes = [2] * (2 * d + 1)
        x = W.random_tt_cores(20 + i, modes, W.capped_ranks(modes, r))
        items.append((P.tt_from_cores(Kq), P.tt_from_cores(x), 24 if i % 2 else 0, 7 + i,
                      1e-8, 20, "f64"))
    batch = P.StepBatch(items, 3)
    outs = P.matvec_round_batched(batch)
    for (K, x, ell, seed, eps, rmax, comp), y in zip(items, outs):
        y1, _, _ = P.matvec_round(K, x, ell, seed, eps, rmax, comp)
        assert y.ranks == y1.ranks
        a, b = T.full_vector(P.tt_to_cores(y)), T.full_vector(P.tt_to_cores(y1))
        assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)


@pytest.mark.parametrize("nbranch,per_branch", [(1, False), (4, False), (4, True), (8, True)])
def test_matvec_round_graph_equals_single(P, nbranch, per_branch):
    """The batch of hot steps captured into one HIP graph (cases on `nbranch`
    branches, or one graph per branch; 8 branches for 6 cases leave two
    empty) gives, on every replay, the ranks, trains, norms and errors of
    the same steps run one at a time (one case with FP32 products).  Between replays the outputs are
    overwritten with NaN and other eager work runs on the same stream, so
    each replay is checked on what it wrote itself."""
    import torch
    from oracle import assembly as A
    items = []
    for i, (d, r) in enumerate([(4, 8), (5, 12), (3, 5), (6, 16), (5, 7), (4, 3)]):
        Kq, _ = A.assemble_qtt(W.cantilever_traction(d))
        modes = [2] * (2 * d + 1)
        x = W.random_tt_cores(20 + i, modes, W.capped_ranks(modes, r))
        items.append((P.tt_from_cores(Kq), P.tt_from_cores(x), 24 if i % 2 else 0, 7 + i,
                      1e-8, 20, "f32" if i == 4 else "f64"))
    ref = [P.matvec_round(K, x, ell, seed, eps, rmax, comp)
           for (K, x, ell, seed, eps, rmax, comp) in items]
    batch = P.StepBatch(items, nbranch)
    g = P.StepGraph(batch, nbranch, per_branch)
    try:
        for rep in range(3):
            for y in batch.outputs():
                y.data.fill_(float("nan"))
            g.launch()
            K, x, ell, seed, eps, rmax, comp = items[rep]
            P.matvec_round(K, x, ell, seed + 100, eps, rmax, comp)  # eager work between
            outs = g.collect()
            for i, ((y1, n1, e1), y) in enumerate(zip(ref, outs)):
                assert y.ranks == y1.ranks, (rep, i)
                a = T.full_vector(P.tt_to_cores(y))
                b = T.full_vector(P.tt_to_cores(y1))
                assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b), (rep, i)
                assert batch.cases[i].norm == pytest.approx(n1, rel=1e-13)
                assert batch.cases[i].err == pytest.approx(e1, rel=1e-9, abs=1e-13 * n1)
                assert batch.cases[i].status == 0
    finally:
        g.close()
    torch.cuda.synchronize()


def test_matvec_round_graph_refuses_small_output(P):
    """A y whose capacity is below the ranks the rounding may leave is refused
    when the graph is built (the replay cannot check it)."""
    from oracle import assembly as A
    Kq, _ = A.assemble_qtt(W.cantilever_traction(4))
    modes = [2] * 9
    x = W.random_tt_cores(3, modes, W.capped_ranks(modes, 6))
    batch = P.StepBatch([(P.tt_from_cores(Kq), P.tt_from_cores(x), 0, 1, 1e-8, 20, "f64")], 1)
    y = batch.outputs()[0]
    y.c.capacity = 10
    with pytest.raises(P.QttError):
        P.StepGraph(batch, 1)


def _diff_norm(a, b):
    """||a - b|| of two TT vectors from the oracle: the difference train
    (core concatenation) orthogonalised left to right, whose last core
    carries the norm (no cancellation, unlike <a,a> - 2<a,b> + <b,b>)."""
    return float(np.linalg.norm(T.orthogonalize_left(T.add(a, b, coeffs=[1.0, -1.0]))[-1]))


@pytest.mark.parametrize("d,r,ell,eps", [(4, 6, 12, 1e-6), (5, 8, 20, 1e-10)])
def test_sketch_rounding_matches_oracle_sketch(P, d, r, ell, eps):
    """qtt_round_sketch draws the same Gaussian train as the oracle
    (Philox4x32-10 on the same counters) and takes the same
    randomize-then-orthogonalize steps, so the rounded tensors agree to
    round-off."""
    from oracle import assembly as A
    from oracle import sketch as SK
    Kq, _ = A.assemble_qtt(W.cantilever_traction(d))
    modes = [2] * (2 * d + 1)
    x = W.random_tt_cores(40 + d, modes, W.capped_ranks(modes, r))
    y = T.matvec(Kq, x)
    ref = T.full_vector(SK.sketch_round(y, ell, 77, eps))
    t = P.tt_from_cores(y)
    P.round_sketch(t, ell, 77, eps, 0)
    got = T.full_vector(P.tt_to_cores(t))
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_headline_step_at_full_shape(P):
    """The benchmarked step at its full shape: level-10 traction operator
    (21 cores, rank 25), seeded rank-64 x, y = round(K x) by a rank-72
    sketch then the exact rounding to (1e-8, 64).  Against the oracle on the
    same inputs: equal to the oracle's randomised rounding (same Gaussian
    train) to round-off, and its error against the unrounded product K x
    within a small factor of the error of the oracle's exact rounding
    (stored by tests/golden/make_step_reference.py).  x has a flat
    spectrum, so the rank cap decides: the exact rounding's error is
    0.115, the rank-72 sketch's about 1.8 times that (the randomised range
    finder with oversampling p loses up to sqrt(1 + r/(p-1)) on a flat
    tail)."""
    import json
    import os
    from oracle import assembly as A
    from oracle import sketch as SK
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "headline_step_level10.json")))
    prob = W.cantilever_traction(10)
    Kq, _ = A.assemble_qtt(prob)
    modes = [2] * 21
    xc = W.random_tt_cores(5, modes, W.capped_ranks(modes, 64))
    K, _ = P.assemble(prob)
    print("headline step: level 10, x rank 64, sketch 72", flush=True)
    y, nrm, err = P.matvec_round(K, P.tt_from_cores(xc), 72, 0, 1e-8, 64)
    got = P.tt_to_cores(y)
    Kx = T.matvec(Kq, xc)
    ref_sk, info = SK.sketch_round(Kx, 72, 0, 1e-8, 64, return_info=True)
    nKx = gold["norm_Kx"]
    e_vs_sketch = _diff_norm(got, ref_sk) / nKx
    e_gpu = _diff_norm(got, Kx) / nKx
    e_exact = gold["exact_round_err_rel"]
    print("headline step: ||y - oracle sketch|| %.2e, ||y - Kx|| %.3e, exact rounding %.3e, "
          "ranks %d" % (e_vs_sketch, e_gpu, e_exact, max(y.ranks)), flush=True)
    # the norm is the sketched train's (the rounding's input), as the oracle's
    assert nrm == pytest.approx(info["norm"], rel=1e-10)
    assert max(y.ranks) <= 64
    # with the flat spectrum the cap keeps 64 of 72 nearly equal singular
    # directions, an ill-conditioned choice: round-off differences (Gaussian
    # numbers from two libm's, summation orders) move the result by up to
    # ~1e-9 (measured 5e-10); the step's own accuracy is eps = 1e-8
    assert e_vs_sketch <= 1e-8
    assert e_gpu <= 2.5 * e_exact


def test_dot_wide_operands_against_oracle(P):
    """<x, y> of a rank-40 train with a rank-1000 matrix-vector product
    (level 8: the intermediates exceed what one workgroup handles, so the
    per-core chip-wide GEMM path runs) against the oracle's dot."""
    from oracle import assembly as A
    Kq, _ = A.assemble_qtt(W.cantilever_traction(8))
    modes = [2] * 17
    x = W.random_tt_cores(61, modes, W.capped_ranks(modes, 40))
    z = W.random_tt_cores(62, modes, W.capped_ranks(modes, 40))
    y = T.matvec(Kq, z)
    assert max(T.ranks(y)) * max(T.ranks(x)) * 2 > 64 * 1024
    ref = T.dot(x, y)
    got = P.dot(P.tt_from_cores(x), P.tt_from_cores(y))
    assert got == pytest.approx(ref, rel=1e-11, abs=1e-12 * T.norm(x) * T.norm(y))


def test_device_rank_mirror_and_explicit_gamma(P):
    """A producer writes its ranks to the caller's device mirror (d_ranks)
    too; an explicit coupling penalty equal to the paper's default gives the
    same operator, another one a different operator."""
    import torch
    K, f = P.assemble(W.cantilever_traction(4))
    x = P.tt_from_cores(W.random_tt_cores(3, K.nrow, W.capped_ranks(K.nrow, 5)))
    dr = torch.full((K.D + 1,), -1, dtype=torch.int32, device="cuda")
    y = P.matvec(K, x)
    y.c.d_ranks = dr.data_ptr()
    P.round_(y, 1e-6, 4)
    torch.cuda.synchronize()
    assert dr.cpu().tolist() == y.ranks
    prob = W.l_shape(3)
    K1, _ = P.assemble(prob)
    from oracle import fem
    Kd, _, _, info = fem.assemble_system(prob)
    for gamma, same in ((info["gamma"], True), (3.0 * info["gamma"], False)):
        K2, _ = P.assemble(prob, gamma=gamma)
        d = np.abs(T.full_matrix(P.tt_to_cores(K1)) - T.full_matrix(P.tt_to_cores(K2))).max()
        assert (d <= 1e-12) == same, (gamma, d)
