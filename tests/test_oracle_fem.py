"""Pins of the sparse FEM oracle against facts the paper and the mathematics
fix: closed forms, invariants, special cases and independent constructions."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import fem
from conftest import golden_path


def _golden_material():
    vals = {}
    for line in open(golden_path("material.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, a, b = line.split()
        vals[name] = int(a) / int(b)
    return vals


def test_material_constants():
    g = _golden_material()
    lam, mu = fem.lame(1.0, 0.3)
    assert lam == pytest.approx(g["lambda"], rel=1e-15)
    assert mu == pytest.approx(g["mu"], rel=1e-15)
    C = fem.c_matrix(1.0, 0.3, plane_strain=True)
    assert C[0, 0] == pytest.approx(g["C11"], rel=1e-15)
    assert C[1, 1] == pytest.approx(g["C11"], rel=1e-15)
    assert C[0, 1] == pytest.approx(g["C12"], rel=1e-15)
    assert C[2, 2] == pytest.approx(g["C33"], rel=1e-15)
    # with nu = 0 plane stress and plane strain coincide (the paper's own
    # material, E = 64, nu = 0)
    np.testing.assert_allclose(fem.c_matrix(64.0, 0.0, True), fem.c_matrix(64.0, 0.0, False))


def test_zorder_golden_d2():
    rows = [list(map(int, l.split())) for l in open(golden_path("zorder_d2.txt"))
            if l.strip() and not l.startswith("#")]
    Z = np.array(rows)
    i, j = np.meshgrid(np.arange(4), np.arange(4), indexing="ij")
    np.testing.assert_array_equal(fem.zorder(i, j, 2), Z)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_zorder_bijection_and_string_interleave(d):
    n = 2 ** d
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    z = fem.zorder(i, j, d)
    assert sorted(z.ravel().tolist()) == list(range(n * n))
    # independent construction: interleave the binary strings (MSB first)
    for a in range(n):
        for b in range(n):
            sa = format(a, "0%db" % d)
            sb = format(b, "0%db" % d)
            s = "".join(y + x for x, y in zip(sa, sb))   # ... j_k i_k ...
            assert int(s, 2) == z[a, b]


def test_qtt_permutation_dofs():
    d, q = 2, 3
    perm = fem.qtt_permutation(d, q)
    n = 4
    # canonical dof c + 2(i + n j + n^2 m) -> c + 2(m + q Z)
    for m in range(q):
        for j in range(n):
            for i in range(n):
                for c in range(2):
                    g = c + 2 * (i + n * j + n * n * m)
                    assert perm[g] == c + 2 * (m + q * int(fem.zorder(i, j, d)))


def test_element_stiffness_invariants():
    C = fem.c_matrix(1.0, 0.3)
    for h in [1.0, 0.1, 1.0 / 31]:
        xy = np.array([[0, 0], [h, 0], [h, h], [0, h]], dtype=float)
        ke, me = fem.element_matrices(xy, C)
        np.testing.assert_allclose(ke, ke.T, atol=1e-15)
        # square element diagonal (C11 + C33)/3 is independent of h in 2-D
        np.testing.assert_allclose(np.diag(ke), (C[0, 0] + C[2, 2]) / 3.0, rtol=1e-14)
        # rigid-body modes: two translations and the infinitesimal rotation
        tx = np.tile([1.0, 0.0], 4)
        ty = np.tile([0.0, 1.0], 4)
        rot = np.ravel([[-y, x] for x, y in xy])
        for v in (tx, ty, rot):
            assert np.abs(ke @ v).max() < 1e-14 * np.abs(ke).max()
        ev = np.linalg.eigvalsh(ke)
        assert (ev[:3] < 1e-13).all() and (ev[3:] > 1e-3).all()
        # mass matrix sums to the element area
        assert me.sum() == pytest.approx(h * h, rel=1e-14)


def test_distorted_element_rigid_modes():
    """Isoparametric map on a general quadrilateral keeps the rigid-body
    null space (the element integrals of Sec. 3.4 with the full Jacobian)."""
    C = fem.c_matrix(1.0, 0.3)
    xy = np.array([[0.0, 0.0], [1.2, 0.1], [1.0, 0.9], [-0.1, 1.1]])
    ke, _ = fem.element_matrices(xy, C)
    rot = np.ravel([[-y, x] for x, y in xy])
    for v in (np.tile([1.0, 0.0], 4), np.tile([0.0, 1.0], 4), rot):
        assert np.abs(ke @ v).max() < 1e-13
    np.testing.assert_allclose(ke, ke.T, atol=1e-14)


@pytest.mark.parametrize("d", [2, 3, 4])
def test_global_stiffness_null_modes_and_patch(d):
    C = fem.c_matrix(1.0, 0.3)
    K, M = fem.assemble_square(d, 0.0, 0.0, 1.0, C)
    n = 2 ** d
    h = 1.0 / (n - 1)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    x = (h * i).ravel(order="F")       # canonical L = i + n j
    y = (h * j).ravel(order="F")
    assert abs(K - K.T).max() < 1e-15 * abs(K).max()
    u = np.zeros(2 * n * n)
    for mode in range(3):
        u[:] = 0
        if mode == 0:
            u[0::2] = 1
        elif mode == 1:
            u[1::2] = 1
        else:
            u[0::2] = -y
            u[1::2] = x
        assert np.abs(K @ u).max() < 1e-13
    # patch test: a linear field has zero residual at interior nodes
    u[0::2] = 0.3 + 0.7 * x - 0.2 * y
    u[1::2] = -0.1 + 0.4 * x + 0.9 * y
    r = K @ u
    interior = ((i > 0) & (i < n - 1) & (j > 0) & (j < n - 1)).ravel(order="F")
    assert np.abs(r[0::2][interior]).max() < 1e-13
    assert np.abs(r[1::2][interior]).max() < 1e-13
    # interior diagonal 4 (C11 + C33) / 3
    L = 1 + n * 1
    assert K[2 * L, 2 * L] == pytest.approx(4 * (C[0, 0] + C[2, 2]) / 3, rel=1e-14)


@pytest.mark.parametrize("d", [2, 3])
def test_spd_after_dirichlet(d):
    for prob in (W.cantilever_body_force(d), W.l_shape(d)):
        K, f, mask, _ = fem.assemble_system(prob)
        Kd = K.toarray()
        np.testing.assert_allclose(Kd, Kd.T, atol=1e-14)
        assert np.linalg.eigvalsh(Kd).min() > 0
        # constrained dofs: unit rows scaled by gamma_D and zero load
        assert (f[mask == 0] == 0).all()


def test_body_force_total():
    """Consistent load of a constant body force sums to area x force."""
    for d in (2, 3, 5):
        prob = W.cantilever_body_force(d)
        _, f, _, _ = fem.assemble_replicated(prob)
        assert f[1::2].sum() == pytest.approx(-1.0, rel=1e-13)
        assert abs(f[0::2].sum()) < 1e-15


def test_traction_total_is_trapezoid_integral():
    """The consistent edge load of the nodal interpolant sums to the
    trapezoid rule of t, which converges to the exact integral
    sum_k a_k (1 - (-1)^k) / (k pi) at second order."""
    a = W.traction_amplitudes(0)
    exact = sum(ak * (1 - (-1) ** k) / (k * np.pi) for k, ak in enumerate(a, start=1))
    errs = []
    for d in (3, 4, 5, 6):
        prob = W.cantilever_traction(d)
        _, f, _, _ = fem.assemble_replicated(prob)
        n = 2 ** d
        s = np.linspace(0.0, 1.0, n)
        t = sum(ak * np.sin(k * np.pi * s) for k, ak in enumerate(a, start=1))
        trap = (s[1] - s[0]) * (t.sum() - 0.5 * (t[0] + t[-1]))
        assert f[1::2].sum() == pytest.approx(trap, rel=1e-12, abs=1e-14)
        errs.append(abs(f[1::2].sum() - exact))
    rates = [np.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    assert min(rates[1:]) > 1.7


def test_direct_solve_residual():
    prob = W.cantilever_traction(5)
    K, f, _, _ = fem.assemble_system(prob)
    u = fem.direct_solve(K, f)
    assert np.linalg.norm(K @ u - f) <= 1e-12 * np.linalg.norm(f)


@pytest.mark.parametrize("d", [2, 3, 4])
def test_lshape_coupling_equals_unique_mesh(d):
    """Both couplings (paper's and symmetric) reproduce the solution of an
    independently built conforming L-mesh with unique nodes."""
    prob = W.l_shape(d)
    ref = fem.lshape_unique_solution(prob)
    for coupling in ("symmetric", "paper"):
        K, f, _, _ = fem.assemble_system(prob, coupling)
        u = fem.direct_solve(K, f)
        assert np.abs(u - ref).max() <= 1e-11 * np.abs(ref).max()
    Ks, _, _, _ = fem.assemble_system(prob, "symmetric")
    Kp, _, _, _ = fem.assemble_system(prob, "paper")
    assert abs(Ks - Ks.T).max() < 1e-14
    assert abs(Kp - Kp.T).max() > 1e-3        # the paper's form is not symmetric


def test_mesh_convergence_tip_displacement():
    """Displacement converges under refinement (h = 1/(2^d - 1)): successive
    differences of the mean tip deflection shrink by about 4x (Q1, smooth
    load)."""
    vals = []
    for d in (3, 4, 5, 6):
        prob = W.cantilever_body_force(d)
        u, _ = fem.solve_problem(prob, order="canonical")
        n = 2 ** d
        tip = fem.side_nodes(n, 1)
        vals.append(u[2 * tip + 1].mean())
    diffs = np.abs(np.diff(vals))
    assert diffs[1] < diffs[0] / 2.5 and diffs[2] < diffs[1] / 2.5


@pytest.mark.parametrize("d", [2, 3, 4])
def test_parallelogram_subdomain_null_modes_patch_and_area(d):
    """A parallelogram subdomain (edge vectors (1.3, 0) and (0.4, 1)): rigid
    modes in the null space, the patch test (a linear field leaves zero
    residual at interior nodes), total mass = area |det A|."""
    sq = W.skewed_cantilever(d).subs[0]
    C = fem.c_matrix(1.0, 0.3)
    K, M = fem.assemble_square(d, sq.x0, sq.y0, sq.side, C, sq.edges)
    n = 2 ** d
    x, y = fem.node_coords(d, sq)
    assert abs(K - K.T).max() < 1e-15 * abs(K).max()
    u = np.zeros(2 * n * n)
    for mode in range(3):
        u[:] = 0
        if mode == 0:
            u[0::2] = 1
        elif mode == 1:
            u[1::2] = 1
        else:
            u[0::2] = -y
            u[1::2] = x
        assert np.abs(K @ u).max() < 1e-13 * abs(K).max()
    u[0::2] = 0.3 + 0.7 * x - 0.2 * y
    u[1::2] = -0.1 + 0.4 * x + 0.9 * y
    r = K @ u
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    interior = ((i > 0) & (i < n - 1) & (j > 0) & (j < n - 1)).ravel(order="F")
    assert np.abs(r[0::2][interior]).max() < 1e-12 * abs(K).max()
    assert np.abs(r[1::2][interior]).max() < 1e-12 * abs(K).max()
    assert M.sum() == pytest.approx(1.3 * 1.0 - 0.0 * 0.4, rel=1e-13)


def test_rotated_square_equals_rotated_stiffness():
    """A unit square rotated by 30 degrees (edges (c, s), (-s, c)) has the
    stiffness of the axis-aligned square with every nodal displacement
    rotated: K_rot = Q K Q^T, Q = diag of the 2x2 rotation per node
    (isotropic material)."""
    d = 3
    n = 2 ** d
    c, s = np.cos(np.pi / 6), np.sin(np.pi / 6)
    C = fem.c_matrix(1.0, 0.3)
    K0, M0 = fem.assemble_square(d, 0.0, 0.0, 1.0, C)
    Kr, Mr = fem.assemble_square(d, 0.0, 0.0, 1.0, C, (c, s, -s, c))
    R = np.array([[c, -s], [s, c]])
    Q = np.kron(np.eye(n * n), R)
    np.testing.assert_allclose(Kr.toarray(), Q @ K0.toarray() @ Q.T, atol=1e-13)
    np.testing.assert_allclose(Mr.toarray(), M0.toarray(), atol=1e-15)


def test_constant_traction_resultant():
    """A uniform traction t on a side of length L has nodal loads summing to
    t L (the cantilever strip's tip load: 3 on the unit-height end)."""
    prob = W.cantilever_strip(3, q=2, traction=-3.0)
    K, f, mask, info = fem.assemble_system(prob)
    assert f[1::2].sum() == pytest.approx(-3.0, rel=1e-13)
    assert abs(f[0::2].sum()) < 1e-14


def test_cantilever_strip_tip_deflection_converges_to_beam_theory():
    """The paper's cantilever beam (20 unit squares in a row, clamped end,
    uniform end traction 3 on unit height, plane stress E = 64, nu = 0):
    the mean tip deflection of the FEM solution approaches Timoshenko's
    P L^3 / (3 E I) + P L / (k G A) = 1500 + 2.25 (P = 3, L = 20, I = 1/12,
    G = 32, shear factor 5/6) as the level grows (Q1 bending converges
    from below)."""
    ref = 3.0 * 20.0 ** 3 / (3.0 * 64.0 / 12.0) + 3.0 * 20.0 / (5.0 / 6.0 * 32.0)
    errs = []
    for d in (2, 3, 4, 5):
        prob = W.cantilever_strip(d)
        u, _ = fem.solve_problem(prob, order="canonical")
        n = 2 ** d
        L = (n - 1) + n * np.arange(n)
        tip = -u[1 + 2 * (L + n * n * (prob.q - 1))].mean()
        errs.append(abs(tip - ref) / ref)
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    assert errs[2] < 3e-3 and errs[3] < 1e-3, errs
