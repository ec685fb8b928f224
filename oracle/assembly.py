"""QTT assembly of the stiffness matrix and load vector (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Builds K and f directly in Z-ordered QTT form (Alg. 1), cores ordered
[component | subdomain (q > 1) | i1 j1 i2 j2 ... id jd].  The subdomain
stiffness is the sum over the 16 vertex pairs of shifted element integrals
(the nodal and subdomain stiffness equations of Sec. 3.5); on a uniform
square mesh with exact 2x2 Gauss quadrature that sum equals a short sum of
Kronecker products of three 1-D matrices on n = 2^d nodes (h = side/(n-1)):

  K1 = (1/h)  tridiag(-1, 2, -1), end diagonals 1   (int phi_a' phi_b')
  M1 = (h/6)  tridiag( 1, 4,  1), end diagonals 2   (int phi_a  phi_b )
  G1 = 1/2 (J^T - J) - 1/2 e0 e0^T + 1/2 e_{n-1} e_{n-1}^T  (int phi_a' phi_b)

with J the upper shift.  In canonical order (y (x) x):
  K_xx = C11 M1(x)K1 + C33 K1(x)M1,   K_yy = C22 K1(x)M1 + C33 M1(x)K1,
  K_xy = C12 G1^T(x)G1 + C33 G1(x)G1^T,   K_yx = K_xy^T,
and z-kron replaces (x) to put the result in Z-order.  The 1-D factors are
written down as exact QTT matrices: I and the corner projectors have rank 1,
the shift J has rank 2 (a binary carry).
"""
from __future__ import annotations

import math
from typing import List

import numpy as np

from . import qtt as T
from .fem import c_matrix

Cores = List[np.ndarray]

EPS_ASSEMBLY = 1e-14


# ------------------------------------------------------------------ 1-D QTT

def qtt_identity(d: int) -> Cores:
    return [np.eye(2).reshape(1, 2, 2, 1) for _ in range(d)]


def qtt_shift(d: int) -> Cores:
    """J with J[a, a+1] = 1.  Reading the digits from the least significant
    one, b = a + 1 holds iff each digit b_k = (a_k + c_k) mod 2 with the
    carry c_{k+1} = (a_k + c_k) div 2, c_1 = 1 and no final carry; the bond
    index is the carry."""
    core = np.zeros((2, 2, 2, 2))            # [c_in, a, b, c_out]
    for cin in range(2):
        for a in range(2):
            s = a + cin
            core[cin, a, s % 2, s // 2] = 1.0
    cores = []
    for k in range(d):
        c = core
        if k == 0:
            c = c[1:2]
        if k == d - 1:
            c = c[..., 0:1]
        cores.append(c.copy())
    return cores


def qtt_transpose(A: Cores) -> Cores:
    return [np.transpose(c, (0, 2, 1, 3)).copy() for c in A]


def qtt_corner(d: int, bit: int) -> Cores:
    """e_k e_k^T with k = 0 (bit = 0) or k = 2^d - 1 (bit = 1)."""
    c = np.zeros((1, 2, 2, 1))
    c[0, bit, bit, 0] = 1.0
    return [c.copy() for _ in range(d)]


def qtt_outer_unit(d: int, row_bit: int, col_bit: int) -> Cores:
    """e_a e_b^T with a, b in {0, 2^d - 1} selected by the bits."""
    c = np.zeros((1, 2, 2, 1))
    c[0, row_bit, col_bit, 0] = 1.0
    return [c.copy() for _ in range(d)]


def qtt_unit_vector(d: int, bit: int) -> Cores:
    c = np.zeros((1, 2, 1))
    c[0, bit, 0] = 1.0
    return [c.copy() for _ in range(d)]


def one_d_matrices(d: int, h: float):
    I = qtt_identity(d)
    J = qtt_shift(d)
    Jt = qtt_transpose(J)
    E0 = qtt_corner(d, 0)
    En = qtt_corner(d, 1)
    K1 = T.add(I, J, Jt, E0, En, coeffs=[2.0 / h, -1.0 / h, -1.0 / h, -1.0 / h, -1.0 / h])
    M1 = T.add(I, J, Jt, E0, En, coeffs=[4.0 * h / 6, h / 6, h / 6, -2.0 * h / 6, -2.0 * h / 6])
    G1 = T.add(J, Jt, E0, En, coeffs=[-0.5, 0.5, -0.5, 0.5])
    rm = lambda A: T.round_matrix(A, EPS_ASSEMBLY)
    return rm(K1), rm(M1), rm(G1)


def qtt_sine(d: int, omega: float) -> Cores:
    """sin(omega * j) for j = 0..2^d-1 as an exact rank-2 QTT vector: the
    state (cos phi, sin phi) of the partial angle phi is rotated by
    omega 2^(k-1) j_k at digit k."""
    cores = []
    for k in range(d):
        th = omega * (2 ** k)
        c = np.zeros((2, 2, 2))
        for b in range(2):
            a = th * b
            ca, sa = math.cos(a), math.sin(a)
            c[:, b, :] = np.array([[ca, sa], [-sa, ca]])
        if k == 0:
            c = c[0:1]                     # start from (cos 0, sin 0) = (1, 0)
        if k == d - 1:
            c = c[..., 1:2]                # read the sine component
        cores.append(c.copy())
    return cores


# ------------------------------------------------------------------ blocks

def _selector(n: int, a: int, b: int) -> np.ndarray:
    e = np.zeros((1, n, n, 1))
    e[0, a, b, 0] = 1.0
    return e


def _unit(n: int, a: int) -> np.ndarray:
    e = np.zeros((1, n, 1))
    e[0, a, 0] = 1.0
    return e


def square_stiffness_blocks(d: int, C: np.ndarray):
    """K_xx, K_xy, K_yx, K_yy of one square subdomain in Z-ordered QTT.
    Scale-free in 2-D: K1 ~ 1/h and M1 ~ h, so h = 1 is used."""
    K1, M1, G1 = one_d_matrices(d, 1.0)
    G1t = qtt_transpose(G1)
    c11, c12, c22, c33 = C[0, 0], C[0, 1], C[1, 1], C[2, 2]
    z = T.zkron
    Kxx = T.add(z(M1, K1), z(K1, M1), coeffs=[c11, c33])
    Kyy = T.add(z(K1, M1), z(M1, K1), coeffs=[c22, c33])
    Kxy = T.add(z(G1t, G1), z(G1, G1t), coeffs=[c12, c33])
    Kyx = T.add(z(G1, G1t), z(G1t, G1), coeffs=[c12, c33])
    return Kxx, Kxy, Kyx, Kyy


def _prefix(q: int, comp_core: np.ndarray, sub_core: np.ndarray, nodes: Cores) -> Cores:
    pre = [comp_core]
    if q > 1:
        pre.append(sub_core)
    return pre + [c.copy() for c in nodes]


def block_diag_stiffness(d: int, q: int, C: np.ndarray) -> Cores:
    """K_bd = sum_{c,c'} E_{cc'} (x) I_q (x) K_{cc'} (same K^(m) on every
    square subdomain)."""
    Kxx, Kxy, Kyx, Kyy = square_stiffness_blocks(d, C)
    Iq = np.eye(q).reshape(1, q, q, 1)
    terms = []
    for (a, b), Kab in zip([(0, 0), (0, 1), (1, 0), (1, 1)], [Kxx, Kxy, Kyx, Kyy]):
        terms.append(_prefix(q, _selector(2, a, b), Iq, Kab))
    return T.round_matrix(T.add(*terms), EPS_ASSEMBLY)


def square_stiffness_dense_factor(d: int, C: np.ndarray) -> Cores:
    return block_diag_stiffness(d, 1, C)


# ------------------------------------------------------------------ masks

def side_delta(d: int, side: int) -> Cores:
    """Indicator of the nodes of one side as a Z-ordered QTT vector."""
    one = [np.ones((1, 2, 1)) for _ in range(d)]
    if side == 0:
        return T.zkron(one, qtt_unit_vector(d, 0))
    if side == 1:
        return T.zkron(one, qtt_unit_vector(d, 1))
    if side == 2:
        return T.zkron(qtt_unit_vector(d, 0), one)
    if side == 3:
        return T.zkron(qtt_unit_vector(d, 1), one)
    raise ValueError(side)


def dirichlet_mask(prob) -> Cores:
    d, q = prob.level, prob.q
    one = [np.ones((1, 2, 1)) for _ in range(2 * d)]
    terms = []
    for m, sq in enumerate(prob.subs):
        for c in range(2):
            node = one
            for s in range(4):
                if sq.fixed[s][c]:
                    node = T.hadamard(node, T.add(one, side_delta(d, s), coeffs=[1.0, -1.0]))
                    node = T.tt_round(node, EPS_ASSEMBLY)
            terms.append(_prefix(q, _unit(2, c), _unit(q, m), node))
    return T.tt_round(T.add(*terms), EPS_ASSEMBLY)


# ------------------------------------------------------------------ loads

def _mass_times(d: int, h: float, v: Cores) -> Cores:
    _, M1, _ = one_d_matrices(d, h)
    return T.tt_round(T.matvec(M1, v), EPS_ASSEMBLY)


def load_vector(prob) -> Cores:
    """f = M fbar for the body force plus edge mass times nodal traction
    values (the load-vector equation of Sec. 3.5), per subdomain and component."""
    d, q = prob.level, prob.q
    n = 2 ** d
    terms = []
    for m, sq in enumerate(prob.subs):
        h = sq.side / (n - 1)
        for c in range(2):
            if prob.body[c] != 0.0:
                one1 = [np.ones((1, 2, 1)) for _ in range(d)]
                m1 = _mass_times(d, h, one1)
                node = T.scale(T.zkron(m1, m1), prob.body[c])
                terms.append(_prefix(q, _unit(2, c), _unit(q, m), node))
        for tr in prob.tractions:
            if tr.sub != m:
                continue
            sines = [T.scale(qtt_sine(d, k * math.pi / (n - 1)), a)
                     for k, a in enumerate(tr.amp, start=1) if a != 0.0]
            if not sines:
                continue
            tbar = T.tt_round(T.add(*sines), EPS_ASSEMBLY)
            edge = _mass_times(d, h, tbar)
            if tr.side in (0, 1):
                node = T.zkron(edge, qtt_unit_vector(d, tr.side))
            else:
                node = T.zkron(qtt_unit_vector(d, tr.side - 2), edge)
            terms.append(_prefix(q, _unit(2, tr.comp), _unit(q, m), node))
    if not terms:
        return [np.zeros((1, c, 1)) for c in ([2] + ([q] if q > 1 else []) + [2] * (2 * d))]
    return T.tt_round(T.add(*terms), EPS_ASSEMBLY)


# ------------------------------------------------------------------ coupling

def _touch(sm, sp):
    """Node correspondences between two squares of equal side: returns
    (X row bit, X col bit or None, Y row bit, Y col bit or None); None
    means the digit runs over the whole side (identity)."""
    s = sm.side
    dx = round((sp.x0 - sm.x0) / s)
    dy = round((sp.y0 - sm.y0) / s)
    if (dx, dy) == (1, 0):
        return (1, 0), None          # m east side ~ p west side, j free
    if (dx, dy) == (-1, 0):
        return (0, 1), None
    if (dx, dy) == (0, 1):
        return None, (1, 0)          # m north ~ p south, i free
    if (dx, dy) == (0, -1):
        return None, (0, 1)
    if abs(dx) == 1 and abs(dy) == 1:
        xb = (1, 0) if dx == 1 else (0, 1)
        yb = (1, 0) if dy == 1 else (0, 1)
        return xb, yb
    return "none"


def connectivity(prob, m: int, p: int) -> Cores:
    """Pi^(mp): rows on subdomain m, columns on p, 1 where nodes coincide
    (Sec. 3.6.1), identity on the component digit."""
    d, q = prob.level, prob.q
    t = _touch(prob.subs[m], prob.subs[p])
    if t == "none":
        return None
    xb, yb = t
    X = qtt_identity(d) if xb is None else qtt_outer_unit(d, *xb)
    Y = qtt_identity(d) if yb is None else qtt_outer_unit(d, *yb)
    return _prefix(q, np.eye(2).reshape(1, 2, 2, 1), _selector(q, m, p), T.zkron(Y, X))


def coupled_operator(prob, Kbd: Cores, fbd: Cores, coupling: str):
    d, q = prob.level, prob.q
    Pis = {}
    for m in range(q):
        for p in range(q):
            if m != p:
                P = connectivity(prob, m, p)
                if P is not None:
                    Pis[(m, p)] = P
    lap_terms = []
    for (m, p), P in Pis.items():
        if m < p:
            Q = Pis[(p, m)]
            lap_terms += [T.matmat(P, Q), T.matmat(Q, P), P, Q]
    coeffs = [1.0, 1.0, -1.0, -1.0] * (len(lap_terms) // 4)
    L = T.round_matrix(T.add(*lap_terms, coeffs=coeffs), EPS_ASSEMBLY)
    Ksq = square_stiffness_dense_factor(d, c_matrix(prob.E, prob.nu, prob.plane_strain))
    gamma = T.trace(Ksq) / (2 * 4 ** d)
    N = 2 * q * 4 ** d
    I = [np.eye(c.shape[1]).reshape(1, c.shape[1], c.shape[1], 1) for c in Kbd]
    if coupling == "paper":
        Pi = T.round_matrix(T.add(*Pis.values()), EPS_ASSEMBLY)
        IP = T.round_matrix(T.add(I, Pi), EPS_ASSEMBLY)
        K = T.round_matrix(T.add(T.matmat(IP, Kbd), L, coeffs=[1.0, gamma]), EPS_ASSEMBLY)
        f = T.tt_round(T.matvec(IP, fbd), EPS_ASSEMBLY)
        return K, f, gamma
    # symmetric: T = I - W L with W = diag(1/(deg+1)), deg = partner count
    deg = [np.einsum("aiib->aib", c) for c in
           T.round_matrix(T.add(*[T.matmat(P, Pis[(p, m)]) for (m, p), P in Pis.items()]),
                          EPS_ASSEMBLY)]
    # 1/(deg+1) on deg in {0,1,2,3} by its cubic interpolant
    xs = np.array([0.0, 1.0, 2.0, 3.0])
    coef = np.linalg.solve(np.vander(xs, 4, increasing=True), 1.0 / (xs + 1.0))
    one = T.ones([c.shape[1] for c in deg])
    d2 = T.tt_round(T.hadamard(deg, deg), EPS_ASSEMBLY)
    d3 = T.tt_round(T.hadamard(d2, deg), EPS_ASSEMBLY)
    w = T.tt_round(T.add(one, deg, d2, d3, coeffs=list(coef)), EPS_ASSEMBLY)
    Tm = T.round_matrix(T.add(I, T.matmat(T.diag(w), L), coeffs=[1.0, -1.0]), EPS_ASSEMBLY)
    TK = T.round_matrix(T.matmat(Tm, Kbd), EPS_ASSEMBLY)
    TKT = T.round_matrix(T.matmat(TK, Tm), EPS_ASSEMBLY)
    K = T.round_matrix(T.add(TKT, L, coeffs=[1.0, gamma]), EPS_ASSEMBLY)
    f = T.tt_round(T.matvec(Tm, fbd), EPS_ASSEMBLY)
    return K, f, gamma


# ------------------------------------------------------------------ Alg. 1

def assemble_qtt(prob, coupling: str = "symmetric"):
    """Global QTT stiffness and load after coupling and Dirichlet conditions
    (Alg. 1): K_bc = P K P + gamma_D (I - P), f_bc = P f with P = diag(mask)
    and gamma_D = trace(K)/N."""
    d, q = prob.level, prob.q
    if any(getattr(sq, "edges", None) is not None for sq in prob.subs) or \
            any(getattr(t, "constant", 0.0) != 0.0 for t in prob.tractions):
        raise NotImplementedError("the QTT assembly oracle covers square subdomains and sine "
                                  "tractions; use fem.assemble_system for the others")
    C = c_matrix(prob.E, prob.nu, prob.plane_strain)
    Kbd = block_diag_stiffness(d, q, C)
    fbd = load_vector(prob)
    if q > 1:
        K, f, _ = coupled_operator(prob, Kbd, fbd, coupling)
    else:
        K, f = Kbd, fbd
    N = 2 * q * 4 ** d
    gD = T.trace(K) / N
    mask = dirichlet_mask(prob)
    P = T.diag(mask)
    one = T.ones([c.shape[1] for c in mask])
    Pc = T.diag(T.tt_round(T.add(one, mask, coeffs=[1.0, -1.0]), EPS_ASSEMBLY))
    PKP = T.round_matrix(T.matmat(T.matmat(P, K), P), EPS_ASSEMBLY)
    Kbc = T.round_matrix(T.add(PKP, Pc, coeffs=[1.0, gD]), EPS_ASSEMBLY)
    fbc = T.tt_round(T.hadamard(mask, f), EPS_ASSEMBLY)
    return Kbc, fbc
