"""Pins of the oracle's randomised rounding: the counter-based generator
against its published known-answer vectors, the Gaussian transform by its
distribution, and the randomize-then-orthogonalize sweep by exactness when
the sketch rank reaches the train's ranks, left-orthogonality, and an error
close to the best one at the sketch rank."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import assembly as A
from oracle import qtt as T
from oracle import sketch as S

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answer_vectors():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        out = S.philox4x32_10(*v[:6])
        assert [int(o) for o in out] == v[6:]


def test_gaussian_numbers_are_standard_normal():
    from scipy import stats
    g = S.gaussian(np.arange(200000), 3, 7, 12345)
    assert abs(g.mean()) < 5.0 / np.sqrt(g.size)
    assert abs(g.var() - 1.0) < 5.0 * np.sqrt(2.0 / g.size)
    assert stats.kstest(g, "norm").pvalue > 1e-3
    # different cores, calls and seeds give different streams
    assert not np.array_equal(g[:100], S.gaussian(np.arange(100), 4, 7, 12345))
    assert not np.array_equal(g[:100], S.gaussian(np.arange(100), 3, 8, 12345))
    assert not np.array_equal(g[:100], S.gaussian(np.arange(100), 3, 7, 12346))


def _product(d, r, seed):
    Kq, _ = A.assemble_qtt(W.cantilever_traction(d))
    modes = [2] * (2 * d + 1)
    x = W.random_tt_cores(seed, modes, W.capped_ranks(modes, r))
    return T.matvec(Kq, x)


def test_full_rank_sketch_reproduces_the_train():
    """With l_k equal to the ranks the sketch spans the whole range of every
    unfolding, so the sweep reproduces y exactly and its cores 0..D-2 have
    orthonormal columns."""
    y = _product(3, 3, 1)
    z = S.randomized_orthogonalize(y, 10 ** 6, seed=5)
    assert S.sketch_ranks(y, 10 ** 6)[1:-1] == [min(a, b) for a, b in
                                               zip(T.ranks(y)[1:-1], S.sketch_ranks(y, 10 ** 9)[1:-1])]
    yd = T.full_vector(y)
    assert np.linalg.norm(T.full_vector(z) - yd) <= 1e-12 * np.linalg.norm(yd)
    for c in z[:-1]:
        M = c.reshape(-1, c.shape[2])
        assert np.abs(M.T @ M - np.eye(M.shape[1])).max() <= 1e-12


@pytest.mark.parametrize("r", [4, 6])
def test_sketch_error_is_near_the_best_at_its_rank(r):
    """Below the ranks of y (level 4, ranks up to 16) a sketch of rank
    r + 4 is at least as accurate as the TT-SVD truncation to rank r, and a
    sketch of rank r alone is within a small factor of it (the randomised
    range finder's bound, oversampling p: error ~ (1 + r/(p-1))^(1/2) times
    the tail), for three seeds."""
    y = _product(4, 4, 2)
    yd = T.full_vector(y)
    best = np.linalg.norm(T.full_vector(T.tt_round(y, 0.0, r)) - yd)
    assert best > 1e-2 * np.linalg.norm(yd)          # the rank limit is active
    for seed in (9, 10, 11):
        z = S.randomized_orthogonalize(y, r + 4, seed=seed)
        assert max(T.ranks(z)) <= r + 4
        assert np.linalg.norm(T.full_vector(z) - yd) <= 1.5 * best
        z0 = S.randomized_orthogonalize(y, r, seed=seed)
        assert np.linalg.norm(T.full_vector(z0) - yd) <= 3.0 * best
    # the final exact rounding keeps the tensor when eps = 0 and no cap
    zr = S.sketch_round(y, r + 4, 9, 0.0)
    z = S.randomized_orthogonalize(y, r + 4, seed=9)
    assert np.linalg.norm(T.full_vector(zr) - T.full_vector(z)) <= 1e-12 * np.linalg.norm(yd)
