"""Plain sparse Q1 finite elements for 2-D linear elasticity (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions
-----------
* Each square subdomain carries n = 2^d nodes per side (Sec. 3.2: "2^d nodes
  per side partition"), so the mesh spacing is h = side / (n - 1).
* Canonical node index L = i + n*j (Sec. 3.2); vector dofs interleave the
  components, dof(L, c) = 2*L + c with c = 0 for x and c = 1 for y (the
  0-based form of N_ij = 2L+1, 2L+2).
* With q subdomains the replicated ("canonical") dof index is
  g = c + 2*(L + n*n*m), subdomain-major.  ``qtt_permutation`` maps it to the
  QTT order g_Z = c + 2*(m + q*Z(i, j)) whose TT cores are, least significant
  first, [c | m | i1 j1 i2 j2 ... id jd] (Z-order, Sec. 3.2).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# ------------------------------------------------------------------ material

def lame(E: float, nu: float):
    """Lame constants (Sec. 2): lambda = E nu / ((1+nu)(1-2nu)),
    mu = E / (2(1+nu))."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def c_matrix(E: float, nu: float, plane_strain: bool = True) -> np.ndarray:
    """Voigt constitutive matrix C of eq. (Cmat).  Plane strain takes
    C11 = C22 = lambda + 2 mu, C12 = lambda, C33 = mu; plane stress takes
    C11 = E/(1-nu^2), C12 = nu C11, C33 = E/(2(1+nu))."""
    if plane_strain:
        lam, mu = lame(E, nu)
        c11, c12, c33 = lam + 2.0 * mu, lam, mu
    else:
        c11 = E / (1.0 - nu * nu)
        c12 = nu * c11
        c33 = E / (2.0 * (1.0 + nu))
    return np.array([[c11, c12, 0.0], [c12, c11, 0.0], [0.0, 0.0, c33]])


# ------------------------------------------------------------------ ordering

def zorder(i, j, d: int):
    """Z-order index of node (i, j) (Sec. 3.2): the bits of i and j are
    interleaved, i_1 (least significant bit of i) first, then j_1, i_2, ..."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    z = np.zeros(np.broadcast(i, j).shape, dtype=np.int64)
    for k in range(d):
        z |= ((i >> k) & 1) << (2 * k)
        z |= ((j >> k) & 1) << (2 * k + 1)
    return z


def qtt_permutation(d: int, q: int = 1) -> np.ndarray:
    """perm[g_canonical] = g_qtt for the replicated dof vector."""
    n = 2 ** d
    m, j, i, c = np.meshgrid(np.arange(q), np.arange(n), np.arange(n),
                             np.arange(2), indexing="ij")
    g_can = c + 2 * (i + n * j + n * n * m)
    g_z = c + 2 * (m + q * zorder(i, j, d))
    perm = np.empty(g_can.size, dtype=np.int64)
    perm[g_can.ravel()] = g_z.ravel()
    return perm


def to_qtt_order(v: np.ndarray, d: int, q: int = 1) -> np.ndarray:
    perm = qtt_permutation(d, q)
    out = np.empty_like(v)
    out[perm] = v
    return out


def from_qtt_order(v: np.ndarray, d: int, q: int = 1) -> np.ndarray:
    return v[qtt_permutation(d, q)]


def permute_matrix_to_qtt(K: sp.spmatrix, d: int, q: int = 1) -> sp.csr_matrix:
    perm = qtt_permutation(d, q)
    K = K.tocoo()
    return sp.csr_matrix((K.data, (perm[K.row], perm[K.col])), shape=K.shape)


# ------------------------------------------------------------------ element

_GAUSS_X = np.array([-1.0, 1.0]) / np.sqrt(3.0)
_GAUSS_W = np.array([1.0, 1.0])
# reference corners in the order the paper maps the element vertices:
# (-1,-1), (1,-1), (1,1), (-1,1)
_REF = np.array([[-1.0, -1.0], [1.0, -1.0], [1.0, 1.0], [-1.0, 1.0]])


def _shape(xi: float, eta: float):
    """Bilinear shape functions Phi_c and their (xi, eta) gradients."""
    N = 0.25 * (1.0 + _REF[:, 0] * xi) * (1.0 + _REF[:, 1] * eta)
    dN = np.empty((4, 2))
    dN[:, 0] = 0.25 * _REF[:, 0] * (1.0 + _REF[:, 1] * eta)
    dN[:, 1] = 0.25 * _REF[:, 1] * (1.0 + _REF[:, 0] * xi)
    return N, dN


def element_matrices(xy: np.ndarray, C: np.ndarray):
    """Element stiffness (8x8) and scalar mass (4x4) of one quadrilateral.

    ``xy`` holds the four vertices mapped to (-1,-1), (1,-1), (1,1), (-1,1).
    Stiffness: sum over the 2x2 tensor Gauss rule of B^T C B |J|
    (the element-integral definition of Sec. 3.4 and the quadrature
    formula after it), with
    B = [[Nx, 0], [0, Ny], [Ny, Nx]] per vertex (the strain-displacement matrix of Sec. 3.3.2).  Mass:
    sum of Phi_a Phi_b |J| (the load matrix G_{c1,c2}).  Dof order within
    the element: 2*vertex + component.
    """
    ke = np.zeros((8, 8))
    me = np.zeros((4, 4))
    for gx, wx in zip(_GAUSS_X, _GAUSS_W):
        for gy, wy in zip(_GAUSS_X, _GAUSS_W):
            N, dN = _shape(gx, gy)
            J = dN.T @ xy              # J[a, b] = d x_b / d xi_a
            detJ = np.linalg.det(J)
            dNxy = dN @ np.linalg.inv(J).T   # rows: vertices, cols: d/dx, d/dy
            B = np.zeros((3, 8))
            B[0, 0::2] = dNxy[:, 0]
            B[1, 1::2] = dNxy[:, 1]
            B[2, 0::2] = dNxy[:, 1]
            B[2, 1::2] = dNxy[:, 0]
            ke += wx * wy * (B.T @ C @ B) * detJ
            me += wx * wy * np.outer(N, N) * detJ
    return ke, me


def edge_mass(p0: np.ndarray, p1: np.ndarray) -> np.ndarray:
    """2x2 mass matrix of the linear trace on a straight edge, by 2-point
    Gauss on the edge."""
    L = np.linalg.norm(p1 - p0)
    m = np.zeros((2, 2))
    for g, w in zip(_GAUSS_X, _GAUSS_W):
        N = np.array([0.5 * (1.0 - g), 0.5 * (1.0 + g)])
        m += w * np.outer(N, N) * 0.5 * L
    return m


# ------------------------------------------------------------------ subdomain

def square_nodes(d: int, x0: float, y0: float, side: float):
    n = 2 ** d
    h = side / (n - 1)
    return n, h


def edge_vectors(sq):
    """Images (a, b) of the parameter square's unit vectors: (side, 0) and
    (0, side) for a square, the given edges for a parallelogram."""
    if getattr(sq, "edges", None) is None:
        return np.array([sq.side, 0.0]), np.array([0.0, sq.side])
    ax, ay, bx, by = sq.edges
    return np.array([ax, ay]), np.array([bx, by])


def node_coords(d: int, sq):
    """Coordinates of the 2^d x 2^d nodes in canonical order (index
    i + n j): (x0, y0) + s a + t b with s = i / (n - 1), t = j / (n - 1)."""
    n = 2 ** d
    a, b = edge_vectors(sq)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    s, t = i.ravel(order="F") / (n - 1), j.ravel(order="F") / (n - 1)
    return sq.x0 + s * a[0] + t * b[0], sq.y0 + s * a[1] + t * b[1]


def assemble_square(d: int, x0: float, y0: float, side: float,
                    C: np.ndarray, edges=None):
    """Element-loop assembly of the stiffness K^(m) and scalar mass M^(m) of
    one subdomain with 2^d nodes per side, canonical order: the square
    [x0, x0+side] x [y0, y0+side], or with edges = (ax, ay, bx, by) the
    parallelogram spanned by them (every element the same parallelogram,
    its integrals by the 2x2 Gauss rule with the element's Jacobian)."""
    n = 2 ** d
    nel = n - 1
    ie, je = np.meshgrid(np.arange(nel), np.arange(nel), indexing="ij")
    ie = ie.ravel()
    je = je.ravel()
    # all elements are congruent: integrate once
    if edges is None:
        a, b = np.array([side, 0.0]), np.array([0.0, side])
    else:
        a, b = np.array(edges[:2], dtype=float), np.array(edges[2:], dtype=float)
    ea, eb = a / nel, b / nel
    xy = np.array([[0.0, 0.0], ea, ea + eb, eb])
    ke, me = element_matrices(xy, C)
    vi = np.stack([ie, ie + 1, ie + 1, ie], axis=1)
    vj = np.stack([je, je, je + 1, je + 1], axis=1)
    nodes = vi + n * vj                              # (nel^2, 4)
    dofs = np.empty((nodes.shape[0], 8), dtype=np.int64)
    dofs[:, 0::2] = 2 * nodes
    dofs[:, 1::2] = 2 * nodes + 1
    rows = np.repeat(dofs, 8, axis=1).ravel()
    cols = np.tile(dofs, (1, 8)).ravel()
    vals = np.tile(ke.ravel(), nodes.shape[0])
    K = sp.csr_matrix((vals, (rows, cols)), shape=(2 * n * n, 2 * n * n))
    rows = np.repeat(nodes, 4, axis=1).ravel()
    cols = np.tile(nodes, (1, 4)).ravel()
    vals = np.tile(me.ravel(), nodes.shape[0])
    M = sp.csr_matrix((vals, (rows, cols)), shape=(n * n, n * n))
    return K, M


def side_nodes(n: int, side: int) -> np.ndarray:
    """Canonical node indices along a side, ordered by increasing arclength
    (side 0 = west i=0, 1 = east i=n-1, 2 = south j=0, 3 = north j=n-1)."""
    t = np.arange(n)
    if side == 0:
        return 0 + n * t
    if side == 1:
        return (n - 1) + n * t
    if side == 2:
        return t + n * 0
    if side == 3:
        return t + n * (n - 1)
    raise ValueError(side)


def traction_load(d: int, sq, tr) -> np.ndarray:
    """Consistent nodal load of a traction t_c(s) = t0 + sum_k a_k
    sin(k pi s) on one side: edge mass matrix times the nodal values of t
    (the edge analogue of the load-vector equation of Sec. 3.5)."""
    n = 2 ** d
    a, b = edge_vectors(sq)
    h = np.linalg.norm(b if tr.side <= 1 else a) / (n - 1)   # element edge length
    f = np.zeros(2 * n * n)
    nodes = side_nodes(n, tr.side)
    s = np.arange(n) / (n - 1)
    tbar = np.full(n, float(getattr(tr, "constant", 0.0)))
    for k, amp in enumerate(tr.amp, start=1):
        tbar += amp * np.sin(k * np.pi * s)
    me = edge_mass(np.array([0.0, 0.0]), np.array([h, 0.0]))
    for e in range(n - 1):
        loc = me @ tbar[e:e + 2]
        f[2 * nodes[e] + tr.comp] += loc[0]
        f[2 * nodes[e + 1] + tr.comp] += loc[1]
    return f


def body_load(d: int, M: sp.spmatrix, body) -> np.ndarray:
    """f = M fbar for a constant body force (the load-vector equation of Sec. 3.5)."""
    n = 2 ** d
    f = np.zeros(2 * n * n)
    ones = np.ones(n * n)
    for c in range(2):
        if body[c] != 0.0:
            f[c::2] += body[c] * (M @ ones)
    return f


def dirichlet_mask(d: int, sq) -> np.ndarray:
    """1 for free dofs, 0 for dofs clamped by ``sq.fixed`` (Sec. 3.8)."""
    n = 2 ** d
    m = np.ones(2 * n * n)
    for s in range(4):
        for c in range(2):
            if sq.fixed[s][c]:
                m[2 * side_nodes(n, s) + c] = 0.0
    return m


# ------------------------------------------------------------------ coupling

def interface_pairs(prob):
    """Matched replicated dofs of coinciding nodes of different subdomains.

    Returns a list of (g_a, g_b) canonical replicated dof pairs with a from
    the lower-numbered subdomain; two nodes match when their coordinates
    coincide (the connectivity matrices Pi^(mp) of Sec. 3.6.1)."""
    d = prob.level
    n = 2 ** d
    coords = []
    for m, sq in enumerate(prob.subs):
        x, y = node_coords(d, sq)
        coords.append((np.arange(n * n), x, y))
    pairs = []
    tol = 1e-9
    for m in range(prob.q):
        Lm, xm, ym = coords[m]
        for p in range(m + 1, prob.q):
            Lp, xp, yp = coords[p]
            # boundary nodes only need checking, but a dense search is fine
            bm = (np.isclose(xm, xm.min()) | np.isclose(xm, xm.max()) |
                  np.isclose(ym, ym.min()) | np.isclose(ym, ym.max()))
            bp = (np.isclose(xp, xp.min()) | np.isclose(xp, xp.max()) |
                  np.isclose(yp, yp.min()) | np.isclose(yp, yp.max()))
            im = np.nonzero(bm)[0]
            ip = np.nonzero(bp)[0]
            dx = np.abs(xm[im][:, None] - xp[ip][None, :])
            dy = np.abs(ym[im][:, None] - yp[ip][None, :])
            a, b = np.nonzero((dx < tol) & (dy < tol))
            for ia, ib in zip(im[a], ip[b]):
                for c in range(2):
                    ga = c + 2 * (Lm[ia] + n * n * m)
                    gb = c + 2 * (Lp[ib] + n * n * p)
                    pairs.append((ga, gb))
    return pairs


def assemble_replicated(prob):
    """Block-diagonal stiffness, load and Dirichlet mask of all subdomains
    (replicated interface nodes), canonical replicated order."""
    d = prob.level
    C = c_matrix(prob.E, prob.nu, prob.plane_strain)
    Ks, fs, ms = [], [], []
    for m, sq in enumerate(prob.subs):
        K, M = assemble_square(d, sq.x0, sq.y0, sq.side, C, getattr(sq, "edges", None))
        f = body_load(d, M, prob.body)
        for tr in prob.tractions:
            if tr.sub == m:
                f = f + traction_load(d, sq, tr)
        Ks.append(K)
        fs.append(f)
        ms.append(dirichlet_mask(d, sq))
    Kbd = sp.block_diag(Ks, format="csr")
    return Kbd, np.concatenate(fs), np.concatenate(ms), Ks[0]


def coupling_matrices(prob, N: int):
    """Pi (sum over ordered pairs of the connectivity matrices), the copy
    graph Laplacian L_Gamma and the copy-averaging projector T.

    For a group G of coinciding copies, L_G is the complete-graph Laplacian
    and the averaging projector on G is I - L_G / |G|."""
    pairs = interface_pairs(prob)
    if not pairs:
        Z = sp.csr_matrix((N, N))
        return Z, Z, sp.identity(N, format="csr"), pairs
    a = np.array([p[0] for p in pairs])
    b = np.array([p[1] for p in pairs])
    ones = np.ones(len(pairs))
    Pi = sp.csr_matrix((np.concatenate([ones, ones]),
                        (np.concatenate([a, b]), np.concatenate([b, a]))),
                       shape=(N, N))
    deg = np.asarray(Pi.sum(axis=1)).ravel()
    Lg = sp.diags(deg) - Pi
    # group sizes: connected components of the copy graph
    ncomp, lab = sp.csgraph.connected_components(Pi, directed=False)
    size = np.bincount(lab)
    gsize = size[lab].astype(np.float64)
    # T = I - sum_G L_G/|G|; each group is a complete graph here
    W = sp.diags(1.0 / gsize)
    T = sp.identity(N, format="csr") - W @ Lg
    return Pi.tocsr(), Lg.tocsr(), T.tocsr(), pairs


def assemble_system(prob, coupling: str = "symmetric"):
    """Global stiffness and load after coupling and Dirichlet conditions,
    canonical replicated order.

    coupling = "symmetric": K = T Kbd T + gamma L_Gamma, f = T fbd.
    coupling = "paper": row block m holds K^(m) U^(m) + sum_p Pi^(mp) K^(p)
    U^(p) + gamma (D_m U^(m) - sum_p Pi^(mp) U^(p)) and the load
    f^(m) + sum_p Pi^(mp) f^(p) (Sec. 3.6.1 with the multiplier sign of the
    solution-concatenation subsection).
    gamma is the mean diagonal of the subdomain stiffness K^(1).
    Dirichlet: K_bc = P K P + gamma_D (I - P), f_bc = P f, P = diag(mask),
    gamma_D the mean diagonal of the coupled K (Sec. 3.8).
    """
    Kbd, fbd, mask, K1 = assemble_replicated(prob)
    N = Kbd.shape[0]
    info = {}
    if prob.q == 1:
        K, f = Kbd, fbd
    else:
        Pi, Lg, T, _ = coupling_matrices(prob, N)
        gamma = K1.diagonal().mean()
        info["gamma"] = gamma
        if coupling == "symmetric":
            K = (T @ Kbd @ T + gamma * Lg).tocsr()
            f = T @ fbd
        elif coupling == "paper":
            I = sp.identity(N, format="csr")
            K = ((I + Pi) @ Kbd + gamma * Lg).tocsr()
            f = (I + Pi) @ fbd
        else:
            raise ValueError(coupling)
    gD = K.diagonal().mean()
    info["gamma_D"] = gD
    P = sp.diags(mask)
    K_bc = (P @ K @ P + gD * sp.diags(1.0 - mask)).tocsr()
    f_bc = mask * f
    return K_bc, f_bc, mask, info


def direct_solve(K: sp.spmatrix, f: np.ndarray) -> np.ndarray:
    """Sparse LU (SuperLU) solve in FP64."""
    lu = spla.splu(K.tocsc(), permc_spec="MMD_AT_PLUS_A",
                   options=dict(SymmetricMode=True))
    return lu.solve(f)


def solve_problem(prob, coupling: str = "symmetric", order: str = "qtt"):
    """Direct FP64 solution of the discrete problem; returned in QTT order
    (``order="qtt"``) or canonical replicated order."""
    K, f, mask, info = assemble_system(prob, coupling)
    u = direct_solve(K, f)
    if order == "qtt":
        return (to_qtt_order(u, prob.level, prob.q), to_qtt_order(f, prob.level, prob.q))
    return u, f


# ------------------------------------------------------------------ L-mesh

def lshape_unique_solution(prob):
    """Independent construction for the L-shaped plate of three unit squares:
    one conforming mesh with unique nodes on the (2n-1)^2 grid minus the
    upper-right quadrant, same element routine, same loads and clamps.
    Returns the solution mapped onto the replicated canonical dofs."""
    d = prob.level
    n = 2 ** d
    h = 1.0 / (n - 1)
    G = 2 * n - 1
    C = c_matrix(prob.E, prob.nu, prob.plane_strain)
    xy = np.array([[0.0, 0.0], [h, 0.0], [h, h], [0.0, h]])
    ke, me = element_matrices(xy, C)
    inside = np.zeros((G, G), dtype=bool)
    I, J = np.meshgrid(np.arange(G), np.arange(G), indexing="ij")
    inside[(I <= n - 1) | (J <= n - 1)] = True
    gid = -np.ones((G, G), dtype=np.int64)
    gid[inside] = np.arange(inside.sum())
    Nn = int(inside.sum())
    rows, cols, vals = [], [], []
    for ie in range(G - 1):
        for je in range(G - 1):
            if ie >= n - 1 and je >= n - 1:
                continue
            v = [gid[ie, je], gid[ie + 1, je], gid[ie + 1, je + 1], gid[ie, je + 1]]
            dofs = np.array([[2 * a, 2 * a + 1] for a in v]).ravel()
            rows.append(np.repeat(dofs, 8))
            cols.append(np.tile(dofs, 8))
            vals.append(ke.ravel())
    K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(2 * Nn, 2 * Nn))
    f = np.zeros(2 * Nn)
    mask = np.ones(2 * Nn)
    # clamps: bottom y = 0 (J = 0), as in the workload
    for Ig in range(G):
        if inside[Ig, 0]:
            mask[2 * gid[Ig, 0]] = 0.0
            mask[2 * gid[Ig, 0] + 1] = 0.0
    # traction on top edge y = 2 (J = G-1), x in [0, 1] (I <= n-1)
    tr = prob.tractions[0]
    s = np.arange(n) / (n - 1)
    tbar = np.zeros(n)
    for k, a in enumerate(tr.amp, start=1):
        tbar += a * np.sin(k * np.pi * s)
    me_e = edge_mass(np.array([0.0, 0.0]), np.array([h, 0.0]))
    for e in range(n - 1):
        loc = me_e @ tbar[e:e + 2]
        f[2 * gid[e, G - 1] + tr.comp] += loc[0]
        f[2 * gid[e + 1, G - 1] + tr.comp] += loc[1]
    gD = K.diagonal().mean()
    P = sp.diags(mask)
    Kb = (P @ K @ P + gD * sp.diags(1.0 - mask)).tocsr()
    u = direct_solve(Kb, mask * f)
    # map onto replicated canonical dofs
    out = np.zeros(2 * 3 * n * n)
    offs = [(0, 0), (n - 1, 0), (0, n - 1)]
    for m, (oi, oj) in enumerate(offs):
        i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        L = (i + n * j).ravel()
        g = gid[(i + oi).ravel(), (j + oj).ravel()]
        for c in range(2):
            out[c + 2 * (L + n * n * m)] = u[2 * g + c]
    return out
