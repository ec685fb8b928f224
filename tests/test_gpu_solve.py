"""Parity of qtt_assemble_stiffness and qtt_solve (through the C ABI) with
the FP64 oracle: the assembled QTT operator and load against the oracle's
QTT assembly and the sparse FEM, and the solution against a sparse direct
solve."""
import numpy as np
import pytest

import workloads as W
from oracle import assembly as A
from oracle import fem
from oracle import precond as PC
from oracle import qtt as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2501_07778_amd as P
    return P


@pytest.mark.parametrize("d", [2, 3, 5])
@pytest.mark.parametrize("which", ["body", "traction", "lshape", "lshape-paper"])
def test_assembly_matches_sparse_fem(P, d, which):
    if which.startswith("lshape") and d == 5:
        d = 4
    coupling = "paper" if which == "lshape-paper" else "symmetric"
    prob = {"body": W.cantilever_body_force, "traction": W.cantilever_traction,
            "lshape": W.l_shape, "lshape-paper": W.l_shape}[which](d)
    Kt, ft = P.assemble(prob, coupling)
    Kc, fc = P.tt_to_cores(Kt), P.tt_to_cores(ft)
    K, f, _, _ = fem.assemble_system(prob, coupling)
    Kz = fem.permute_matrix_to_qtt(K, d, prob.q).toarray()
    fz = fem.to_qtt_order(f, d, prob.q)
    np.testing.assert_allclose(T.full_matrix(Kc), Kz, atol=1e-12 * np.abs(Kz).max())
    np.testing.assert_allclose(T.full_vector(fc), fz, atol=1e-12 * np.abs(fz).max())
    # ranks agree with the oracle's QTT assembly (both rounded at 1e-14)
    Ko, fo = A.assemble_qtt(prob, coupling)
    assert max(Kt.ranks) <= max(T.ranks(Ko)) + 2


def _tt_matrix_entries(cores, rows, cols):
    """Entries A[rows, cols] of a TT matrix (first core least significant):
    for each pair a product of the core slices G_k[:, i_k, j_k, :]."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    M = np.ones((rows.size, 1))
    stride = 1
    for G in cores:
        n = G.shape[1]
        ik, jk = (rows // stride) % n, (cols // stride) % n
        M = np.einsum("sa,sab->sb", M, np.transpose(G[:, ik, jk, :], (1, 0, 2)))
        stride *= n
    return M[:, 0]


def _tt_vector_entries(cores, index):
    index = np.asarray(index, dtype=np.int64)
    M = np.ones((index.size, 1))
    stride = 1
    for G in cores:
        n = G.shape[1]
        M = np.einsum("sa,sab->sb", M, np.transpose(G[:, (index // stride) % n, :], (1, 0, 2)))
        stride *= n
    return M[:, 0]


def _edge_rows(d, q, sub, side, comp, count, rng):
    """Z-ordered dof indices of nodes on (or one node inside) one side of
    subdomain `sub`."""
    n = 2 ** d
    t = rng.integers(0, n, count)
    inner = rng.integers(0, 2, count)
    i, j = {0: (inner, t), 1: (n - 1 - inner, t), 2: (t, inner), 3: (t, n - 1 - inner)}[side]
    return comp + 2 * (sub + q * fem.zorder(i, j, d))


@pytest.mark.parametrize("which", ["traction10", "lshape9"])
def test_assembly_full_size_matches_sparse_fem_entries(P, which):
    """Full sizes of the level-10 traction workload (2,097,152 dofs) and the
    level-9 L-shape (1,572,864 dofs): sampled entries of the library's QTT
    stiffness and load against the element-loop sparse FEM of the oracle
    (Q1 elements, 2x2 Gauss, coupling and Dirichlet rows), permuted to
    Z-order.  The samples are every stored entry of seeded random rows, rows
    on the clamped and loaded edges (and the re-entrant corner of the L),
    and as many seeded random (row, column) pairs, nearly all structural
    zeros.  The assembly is exact algebra rounded at 1e-14 (relative
    Frobenius), which bounds each entry's error by 1e-14 times the
    Frobenius norm."""
    if which == "traction10":
        prob, d, clamp, load = W.cantilever_traction(10), 10, [(0, 0)], [(0, 1)]
    else:
        prob, d, clamp, load = W.l_shape(9), 9, [(0, 2), (1, 2)], [(2, 3)]
    q = prob.q
    Kt, ft = P.assemble(prob)
    Kc, fc = P.tt_to_cores(Kt), P.tt_to_cores(ft)
    K, f, _, _ = fem.assemble_system(prob)
    Kz = fem.permute_matrix_to_qtt(K, d, q).tocsr()
    fz = fem.to_qtt_order(f, d, q)
    N = Kz.shape[0]
    rng = np.random.default_rng(20250107)
    rows = [rng.integers(0, N, 256)]
    for sub, side in clamp + load:
        for comp in (0, 1):
            rows.append(_edge_rows(d, q, sub, side, comp, 32, rng))
    if q > 1:      # nodes at the re-entrant corner (1, 1) of each square
        n = 2 ** d
        for sub, (i, j) in enumerate([(n - 1, n - 1), (0, n - 1), (n - 1, 0)]):
            for di in (-1, 0, 1):
                for dj in (-1, 0, 1):
                    ii, jj = min(max(i + di, 0), n - 1), min(max(j + dj, 0), n - 1)
                    for comp in (0, 1):
                        rows.append(np.array([comp + 2 * (sub + q * int(fem.zorder(ii, jj, d)))]))
    rows = np.unique(np.concatenate(rows))
    sub = Kz[rows].tocoo()
    r_nz, c_nz, v_nz = rows[sub.row], sub.col, sub.data
    r_rand, c_rand = rng.integers(0, N, 4096), rng.integers(0, N, 4096)
    v_rand = np.asarray(Kz[r_rand, c_rand]).ravel()
    rr = np.concatenate([r_nz, r_rand])
    cc = np.concatenate([c_nz, c_rand])
    ref = np.concatenate([v_nz, v_rand])
    got = _tt_matrix_entries(Kc, rr, cc)
    # the rounding at eps = 1e-14 (relative Frobenius) bounds every entry's
    # error by 1e-14 ||K||_F; FP64 products of 21 cores add a few ulps
    err = np.abs(got - ref).max() / np.sqrt(np.sum(Kz.data ** 2))
    print("%s: %d matrix entries, max error / ||K||_F = %.2e, max error / max|K| = %.2e"
          % (which, ref.size, err, np.abs(got - ref).max() / np.abs(Kz.data).max()), flush=True)
    assert err <= 1.5e-14, err
    fi = np.unique(np.concatenate([rows, rng.integers(0, N, 4096)]))
    gotf = _tt_vector_entries(fc, fi)
    errf = np.abs(gotf - fz[fi]).max() / np.linalg.norm(fz)
    print("%s: %d load entries, max error / ||f|| = %.2e" % (which, fi.size, errf), flush=True)
    assert errf <= 1.5e-14, errf
    if q == 1:
        assert max(Kt.ranks) == 25


@pytest.mark.parametrize("d", [3, 5])
def test_solve_body_force_matches_direct(P, d):
    """Plain FP64 solve of the clamped unit square under body force (level 5
    is the small workload: eps 1e-10, tolerance 1e-10)."""
    prob = W.cantilever_body_force(d)
    uref, _ = fem.solve_problem(prob)
    K, f = P.assemble(prob)
    opts = P.SolveOpts(tol=1e-10, eps=1e-10, rmax=64, eps_in=1e-3, rmax_in=32,
                       red_in=1e-2, maxit_in=3000, maxit_out=30, check_every=5)
    u, rep = P.solve(K, f, opts)
    assert rep["status"] == 0, rep
    ud = T.full_vector(P.tt_to_cores(u))
    err = np.linalg.norm(ud - uref) / np.linalg.norm(uref)
    assert err <= 1e-8, (err, rep)
    # FP64 residual of the returned iterate, recomputed by the oracle
    Ks, fs, _, _ = fem.assemble_system(prob)
    r = fem.permute_matrix_to_qtt(Ks, d) @ ud - fem.to_qtt_order(fs, d)
    assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(fs)


def test_solve_traction_and_lshape(P):
    for prob, tol in ((W.cantilever_traction(4), 1e-9), (W.l_shape(3), 1e-9)):
        uref, _ = fem.solve_problem(prob)
        K, f = P.assemble(prob)
        opts = P.SolveOpts(tol=1e-11, eps=1e-11, rmax=96, eps_in=1e-3, rmax_in=48,
                           red_in=1e-2, maxit_in=3000, maxit_out=30, check_every=5)
        u, rep = P.solve(K, f, opts)
        ud = T.full_vector(P.tt_to_cores(u))
        err = np.linalg.norm(ud - uref) / np.linalg.norm(uref)
        assert rep["status"] == 0 and err <= tol, (err, rep)


def test_solve_warm_start_and_zero_load(P):
    prob = W.cantilever_body_force(3)
    K, f = P.assemble(prob)
    opts = P.SolveOpts(tol=1e-10, eps=1e-12, rmax=64, eps_in=1e-3, rmax_in=32,
                       maxit_in=2000, check_every=5)
    u, rep = P.solve(K, f, opts)
    # restarting from the converged solution costs no refinement step
    u2, rep2 = P.solve(K, f, opts, x0=u)
    assert rep2["outer"] == 0 and rep2["status"] == 0
    # zero load gives the zero solution
    z = P.tt_from_cores([np.zeros((1, c, 1)) for c in f.nrow])
    u3, rep3 = P.solve(K, z, opts)
    assert np.all(T.full_vector(P.tt_to_cores(u3)) == 0)


def test_solve_reports_noconv(P):
    prob = W.cantilever_body_force(4)
    K, f = P.assemble(prob)
    opts = P.SolveOpts(tol=1e-12, eps=1e-12, rmax=64, eps_in=1e-3, rmax_in=32,
                       maxit_in=3, maxit_out=1, check_every=1)
    u, rep = P.solve(K, f, opts)
    assert rep["status"] == -4 and rep["outer"] == 1


@pytest.mark.parametrize("d", [2, 3, 4])
def test_bpx_assembly_matches_oracle(P, d):
    from oracle import precond as PC
    prob = W.cantilever_traction(d)
    K, f, mask, info = fem.assemble_system(prob)
    Ct = P.assemble_bpx(prob)
    Cd = PC.bpx_dense(prob, info["gamma_D"])
    perm = fem.qtt_permutation(d)
    Cz = np.zeros_like(Cd)
    Cz[np.ix_(perm, perm)] = Cd
    np.testing.assert_allclose(T.full_matrix(P.tt_to_cores(Ct)), Cz, atol=1e-12 * np.abs(Cd).max())


@pytest.mark.parametrize("d", [4, 5])
def test_pcg_solve_matches_direct(P, d):
    prob = W.cantilever_traction(d)
    uref, _ = fem.solve_problem(prob)
    K, f = P.assemble(prob)
    C = P.assemble_bpx(prob)
    opts = P.SolveOpts(tol=1e-10, eps=1e-11, rmax=64, eps_in=1e-3, rmax_in=32,
                       red_in=1e-3, maxit_in=500, maxit_out=20, check_every=5, precond=C)
    u, rep = P.solve(K, f, opts)
    ud = T.full_vector(P.tt_to_cores(u))
    err = np.linalg.norm(ud - uref) / np.linalg.norm(uref)
    assert rep["status"] == 0 and err <= 1e-8, (err, rep)
    # the same first correction solve without the preconditioner needs more
    # iterations (capped run: one refinement step)
    opts.precond = None
    opts.maxit_out = 1
    u0, rep0 = P.solve(K, f, opts)
    assert rep0["inner"] > rep["inner"] / max(rep["outer"], 1)


@pytest.mark.parametrize("d", [4])
def test_pcg_sketched_solve_matches_direct(P, d):
    """Randomised rounding of the products K p and C r (sketch oversampling
    8) inside preconditioned CG: same solution to the tolerance, and the
    FP64 residual the solver reports agrees with the oracle's."""
    prob = W.cantilever_traction(d)
    uref, _ = fem.solve_problem(prob)
    K, f = P.assemble(prob)
    C = P.assemble_bpx(prob)
    opts = P.SolveOpts(tol=1e-9, eps=1e-11, rmax=64, eps_in=1e-3, rmax_in=24, red_in=1e-3,
                       maxit_in=400, maxit_out=20, check_every=5, precond=C, sketch=8, seed=7)
    u, rep = P.solve(K, f, opts)
    ud = T.full_vector(P.tt_to_cores(u))
    err = np.linalg.norm(ud - uref) / np.linalg.norm(uref)
    assert rep["status"] == 0 and err <= 1e-7, (err, rep)
    Ks, fs, _, _ = fem.assemble_system(prob)
    r = fem.permute_matrix_to_qtt(Ks, d) @ ud - fem.to_qtt_order(fs, d)
    assert np.linalg.norm(r) / np.linalg.norm(fs) == pytest.approx(rep["residual"], rel=1e-3)


@pytest.mark.parametrize("method", ["chebyshev", "fcg"])
@pytest.mark.parametrize("d,rin,sketch", [(3, 16, 0), (4, 16, 0), (5, 32, 8)])
def test_bpx_solves_match_direct(P, d, rin, sketch, method):
    """BPX-preconditioned Chebyshev solve (true residual every step): the
    solution matches the sparse direct solve; the spectral bound estimated
    on the device lies above the dense spectrum of C K; the reported FP64
    residual equals the oracle's residual of the returned iterate."""
    prob = W.cantilever_traction(d)
    uref, _ = fem.solve_problem(prob)
    K, f = P.assemble(prob)
    C = P.assemble_bpx(prob)
    opts = P.SolveOpts(tol=1e-9, eps=1e-11, rmax=64, eps_in=1e-3, rmax_in=rin, maxit_in=400,
                       check_every=5, precond=C, sketch=sketch, seed=5, method=method)
    u, rep = P.solve(K, f, opts)
    ud = T.full_vector(P.tt_to_cores(u))
    err = np.linalg.norm(ud - uref) / np.linalg.norm(uref)
    assert rep["status"] == 0 and err <= 1e-8, (err, rep)
    assert rep["criterion"] <= 1e-9
    Ks, fs, mask, info = fem.assemble_system(prob)
    if d <= 4 and method == "chebyshev":
        Cd = PC.bpx_dense(prob, info["gamma_D"])
        Lc = np.linalg.cholesky(Cd)
        lmax = np.linalg.eigvalsh(Lc.T @ Ks.toarray() @ Lc).max()
        assert lmax < rep["lmax"] < 1.3 * lmax
    r = fem.permute_matrix_to_qtt(Ks, d) @ ud - fem.to_qtt_order(fs, d)
    assert np.linalg.norm(r) / np.linalg.norm(fs) == pytest.approx(rep["residual"], rel=1e-6)


def test_bpx_solves_reject_bad_options(P):
    prob = W.cantilever_traction(2)
    K, f = P.assemble(prob)
    with pytest.raises(P.QttError):
        P.solve(K, f, P.SolveOpts(method="chebyshev"))           # no preconditioner
    C = P.assemble_bpx(prob)
    with pytest.raises(P.QttError):
        P.solve(K, f, P.SolveOpts(method="chebyshev", precond=C, rmax=16, rmax_in=32))
    with pytest.raises(P.QttError):
        P.solve(K, f, P.SolveOpts(method="fcg"))                 # no preconditioner


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_mixed_precision_fcg(P, compute):
    """Products of the correction (C r) in FP32 or BF16 with FP32
    accumulation, residual and rounding in FP64: the solve still reaches the
    FP64 solution; error reported against the oracle's direct solve and
    against the FP64 GPU solve."""
    d = 5
    prob = W.cantilever_traction(d)
    uref, _ = fem.solve_problem(prob)
    K, f = P.assemble(prob)
    C = P.assemble_bpx(prob)
    base = dict(tol=1e-9, eps=1e-11, rmax=64, eps_in=1e-3, rmax_in=32, maxit_in=600,
                check_every=5, precond=C, method="fcg")
    u64, rep64 = P.solve(K, f, P.SolveOpts(**base))
    ulp, replp = P.solve(K, f, P.SolveOpts(compute=compute, **base))
    d64 = T.full_vector(P.tt_to_cores(u64))
    dlp = T.full_vector(P.tt_to_cores(ulp))
    assert rep64["status"] == 0 and replp["status"] == 0
    err_oracle = np.linalg.norm(dlp - uref) / np.linalg.norm(uref)
    err_gpu64 = np.linalg.norm(dlp - d64) / np.linalg.norm(d64)
    print("mixed %s: iterations %d (FP64 %d), error vs oracle %.2e, vs FP64 GPU %.2e"
          % (compute, replp["inner"], rep64["inner"], err_oracle, err_gpu64))
    assert err_oracle <= 1e-8 and err_gpu64 <= 1e-8


def test_batched_solves_equal_single_solves(P):
    """Load cases of different levels, seeds and inner rank caps solved
    concurrently (qtt_solve_batched, 4 workers on their own streams) give the
    same iterates as one solve at a time; the autotuner returns one of its
    candidates and a rate for each."""
    cases = []
    for i, d in enumerate([3, 4, 3, 5, 4, 3]):
        prob = W.cantilever_traction(d, seed=i)
        K, f = P.assemble(prob)
        C = P.assemble_bpx(prob)
        opts = P.SolveOpts(tol=1e-9, eps=1e-11, rmax=64, eps_in=1e-3, rmax_in=16 + 8 * (i % 3),
                           maxit_in=400, check_every=5, precond=C, method="fcg")
        cases.append((K, f, opts))
    batch = P.Batch(cases)
    res = P.solve_batched(batch, 4)
    for (K, f, opts), (u, rep) in zip(cases, res):
        u1, rep1 = P.solve(K, f, opts)
        assert rep["status"] == 0 and rep["inner"] == rep1["inner"]
        assert u.ranks == u1.ranks
        a, b = T.full_vector(P.tt_to_cores(u)), T.full_vector(P.tt_to_cores(u1))
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)
    # the autotuner runs on a batch with a case that stops at its iteration
    # limit (QTT_E_NOCONV): that case is timed but not counted as a solve
    K, f, opts = cases[0]
    stuck = P.SolveOpts(tol=1e-9, eps=1e-11, rmax=64, eps_in=1e-3, rmax_in=16, maxit_in=2,
                        check_every=1, precond=opts.precond, method="fcg")
    small = P.Batch([cases[0], (K, f, stuck), cases[2]])
    best, rates = P.autotune_batched(small)
    assert best in rates and all(r > 0 for r in rates.values())
    st = [r["status"] for _, r in small.results()]
    assert st == [0, -4, 0], st


@pytest.mark.parametrize("d", [2, 3, 5])
@pytest.mark.parametrize("which", ["skewed", "strip"])
def test_assembly_of_parallelogram_and_strip_matches_sparse_fem(P, d, which):
    """Non-square subdomains (a parallelogram, stiffness from the constant
    Jacobian of its affine map) and the paper's cantilever strip of 20
    square subdomains (uniform tip traction, plane stress, E = 64, nu = 0):
    the QTT operator and load equal the element-loop sparse FEM in Z-order."""
    if which == "strip" and d == 5:
        d = 4
    prob = W.skewed_cantilever(d) if which == "skewed" else W.cantilever_strip(d)
    Kt, ft = P.assemble(prob)
    K, f, _, _ = fem.assemble_system(prob)
    Kz = fem.permute_matrix_to_qtt(K, d, prob.q).toarray()
    fz = fem.to_qtt_order(f, d, prob.q)
    np.testing.assert_allclose(T.full_matrix(P.tt_to_cores(Kt)), Kz, atol=1e-12 * np.abs(Kz).max())
    np.testing.assert_allclose(T.full_vector(P.tt_to_cores(ft)), fz, atol=1e-12 * np.abs(fz).max())


@pytest.mark.parametrize("which,d,rmax,bound", [("skewed", 5, 64, 1e-9), ("strip", 3, 128, 3e-7),
                                                 ("strip", 5, 64, 2e-5)])
def test_solve_parallelogram_and_strip_against_direct(P, which, d, rmax, bound):
    """The parallelogram subdomain by ALS at full rank (the mode-product
    bounds): the oracle's sparse direct solve to 1e-9.  The cantilever
    strip (20 squares in a row, aspect ratio 20) by AMEn: its conditioning
    puts a floor under the per-sweep change (between 5e-8 and 1.5e-7 at
    level 3, depending on the rounding's last bits, and near 2e-6 at level
    5, 40,960 dofs, where one-site ALS at rank 48 stalls too), so the stop
    tolerances are 3e-7 and 3e-6 and the errors against the direct solve
    3e-7 and 2e-5 (measured 2e-8 to 3e-8 in 8 sweeps and 3.4e-6 to 3.9e-6
    in 12 to 14)."""
    prob = W.skewed_cantilever(d) if which == "skewed" else W.cantilever_strip(d)
    uref, _ = fem.solve_problem(prob)
    K, f = P.assemble(prob)
    if which == "skewed":
        opts = P.SolveOpts(tol=1e-10, eps=0.0, rmax=rmax, maxit_out=30, rmax_in=0, method="als",
                           seed=1)
    else:
        opts = P.SolveOpts(tol=3e-7 if d == 3 else 3e-6, eps=1e-10, rmax=rmax, rmax_in=8,
                           eps_in=1e-2, maxit_out=80, method="amen", seed=1)
    print("solve %s d=%d rank %d" % (which, d, rmax), flush=True)
    u, rep = P.solve(K, f, opts)
    assert rep["status"] == 0, rep
    err = np.linalg.norm(T.full_vector(P.tt_to_cores(u)) - uref) / np.linalg.norm(uref)
    print("%s d=%d: error %.2e, sweeps %d, rank %d" % (which, d, err, rep["outer"],
                                                      rep["max_rank"]), flush=True)
    assert err <= bound, err
