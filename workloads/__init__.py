"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module holds no arithmetic of the method: it only names the workloads
(geometry, material, boundary and load *parameters*) and draws the random
numbers that either side consumes.  Both sides turn these parameters into a
stiffness matrix, a load vector or a solution with their own code.

Workloads follow the paper's 2-D linear elasticity setting (Sec. 2-3): square
Q1 subdomains with 2^d nodes per side, plane strain material (E, nu), a clamp
on some sides, and either a body force or a traction given as a short sine
series along one side.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# side numbering used by every workload: 0 = west (x = x0), 1 = east,
# 2 = south (y = y0), 3 = north
WEST, EAST, SOUTH, NORTH = 0, 1, 2, 3


@dataclass(frozen=True)
class Square:
    """One square subdomain [x0, x0+side] x [y0, y0+side], or, with
    ``edges = (ax, ay, bx, by)``, the parallelogram
    {(x0, y0) + s (ax, ay) + t (bx, by) : s, t in [0, 1]} (``side`` is then
    unused).  Nodes sit at s, t = i / (2^d - 1); the sides are numbered as
    for the square (west s = 0, east s = 1, south t = 0, north t = 1).

    ``fixed[s][c]`` is True when component c (0 = x, 1 = y) is clamped on
    side s of this subdomain.
    """
    x0: float
    y0: float
    side: float
    fixed: Tuple[Tuple[bool, bool], ...] = ((False, False),) * 4
    edges: Optional[Tuple[float, float, float, float]] = None

    def edge_vectors(self):
        """(a, b): the images of the unit vectors of the parameter square."""
        if self.edges is None:
            return (self.side, 0.0), (0.0, self.side)
        ax, ay, bx, by = self.edges
        return (ax, ay), (bx, by)


@dataclass(frozen=True)
class Traction:
    """Traction t_comp(s) = constant + sum_k amp[k-1] * sin(k*pi*s) on side
    ``side`` of subdomain ``sub``; s in [0, 1] is the normalised arclength
    along the side (x for south/north sides, y for west/east sides)."""
    sub: int
    side: int
    comp: int
    amp: Tuple[float, ...]
    constant: float = 0.0


@dataclass(frozen=True)
class Problem:
    level: int
    subs: Tuple[Square, ...]
    E: float = 1.0
    nu: float = 0.3
    plane_strain: bool = True
    body: Tuple[float, float] = (0.0, 0.0)
    tractions: Tuple[Traction, ...] = ()

    @property
    def q(self) -> int:
        return len(self.subs)

    @property
    def n(self) -> int:
        return 2 ** self.level

    @property
    def ndof(self) -> int:
        return 2 * self.q * 4 ** self.level


def traction_amplitudes(seed: int, nmodes: int = 8) -> np.ndarray:
    """N(0,1) amplitudes of the sine modes, drawn from PCG64(seed)."""
    return np.random.default_rng(seed).standard_normal(nmodes)


def unit_square_clamped_west() -> Square:
    clamp = ((True, True), (False, False), (False, False), (False, False))
    return Square(0.0, 0.0, 1.0, clamp)


def cantilever_body_force(level: int) -> Problem:
    """Unit square, west edge clamped, uniform body force (0, -1)."""
    return Problem(level=level, subs=(unit_square_clamped_west(),),
                   body=(0.0, -1.0))


def cantilever_traction(level: int, seed: int = 0, nmodes: int = 8) -> Problem:
    """Unit square, west edge clamped, vertical traction on the east edge
    with ``nmodes`` seeded N(0,1) sine amplitudes."""
    a = tuple(float(v) for v in traction_amplitudes(seed, nmodes))
    return Problem(level=level, subs=(unit_square_clamped_west(),),
                   tractions=(Traction(0, EAST, 1, a),))


def cantilever_two_component(level: int, coeffs: Sequence[float]) -> Problem:
    """Unit square, west edge clamped, east-edge traction with 16 Fourier
    coefficients: the first 8 drive t_x, the last 8 drive t_y."""
    c = [float(v) for v in coeffs]
    return Problem(level=level, subs=(unit_square_clamped_west(),),
                   tractions=(Traction(0, EAST, 0, tuple(c[:8])),
                              Traction(0, EAST, 1, tuple(c[8:16]))))


def l_shape(level: int, seed: int = 0, nmodes: int = 8) -> Problem:
    """L-shaped plate from three unit squares: Omega1 = [0,1]^2,
    Omega2 = [1,2]x[0,1], Omega3 = [0,1]x[1,2]; bottom (y = 0) clamped on
    Omega1 and Omega2; vertical traction with seeded amplitudes on the top
    edge (y = 2) of Omega3."""
    free = (False, False)
    clamp = (True, True)
    s1 = Square(0.0, 0.0, 1.0, (free, free, clamp, free))
    s2 = Square(1.0, 0.0, 1.0, (free, free, clamp, free))
    s3 = Square(0.0, 1.0, 1.0, (free, free, free, free))
    a = tuple(float(v) for v in traction_amplitudes(seed, nmodes))
    return Problem(level=level, subs=(s1, s2, s3),
                   tractions=(Traction(2, NORTH, 1, a),))


def cantilever_strip(level: int, q: int = 20, traction: float = -3.0) -> Problem:
    """The paper's cantilever beam (Sec. 5): q unit squares in a row
    (length-to-height ratio q, 2^level nodes per subdomain side), the west
    edge of the first clamped, a uniform vertical traction on the east edge
    of the last (the free end); plane stress with E = 64 and nu = 0."""
    clamp = ((True, True), (False, False), (False, False), (False, False))
    free = ((False, False),) * 4
    subs = tuple(Square(float(m), 0.0, 1.0, clamp if m == 0 else free) for m in range(q))
    return Problem(level=level, subs=subs, E=64.0, nu=0.0, plane_strain=False,
                   tractions=(Traction(q - 1, EAST, 1, (), float(traction)),))


def skewed_cantilever(level: int, shear: float = 0.4, stretch: float = 1.3, seed: int = 0,
                      nmodes: int = 8) -> Problem:
    """A non-square subdomain: the parallelogram with edge vectors
    a = (stretch, 0) and b = (shear, 1), its west side (s = 0) clamped and
    the seeded sine traction of the cantilever workloads on its east side,
    plane strain E = 1, nu = 0.3."""
    clamp = ((True, True), (False, False), (False, False), (False, False))
    sub = Square(0.0, 0.0, 1.0, clamp, edges=(float(stretch), 0.0, float(shear), 1.0))
    a = tuple(float(v) for v in traction_amplitudes(seed, nmodes))
    return Problem(level=level, subs=(sub,), tractions=(Traction(0, EAST, 1, a),))


# ---------------------------------------------------------------- batched
@dataclass(frozen=True)
class BatchCase:
    level: int
    cap: int
    coeffs: Tuple[float, ...]


def batch_case(i: int) -> BatchCase:
    """Load case i of the batched workload: level uniform in 8..11, rank cap
    uniform in 16..96, 16 N(0,1) Fourier coefficients (PCG64(1000+i))."""
    g = np.random.default_rng(1000 + i)
    level = int(g.integers(8, 12))
    cap = int(g.integers(16, 97))
    c = tuple(float(v) for v in g.standard_normal(16))
    return BatchCase(level, cap, c)


def warmstart_params(s: int) -> np.ndarray:
    """Load parameters of sample s of the learned-warm-start workload."""
    return np.random.default_rng(100000 + s).standard_normal(16)


# ---------------------------------------------------------------- random TT
def random_tt_cores(seed: int, nrow: Sequence[int], ranks: Sequence[int],
                    ncol: Optional[Sequence[int]] = None,
                    scale: str = "unit") -> List[np.ndarray]:
    """Random FP64 TT cores with the given modes and ranks (ranks has
    len(nrow)+1 entries, ranks[0] = ranks[-1] = 1).  Vector cores have shape
    (r0, n, r1); matrix cores (r0, n, m, r1).  Entries are N(0,1) scaled by
    1/sqrt(r0*n) so that products of many cores stay O(1)."""
    g = np.random.default_rng(seed)
    cores = []
    for k, n in enumerate(nrow):
        r0, r1 = ranks[k], ranks[k + 1]
        if ncol is None:
            shape = (r0, n, r1)
            fan = r0 * n
        else:
            shape = (r0, n, ncol[k], r1)
            fan = r0 * n
        c = g.standard_normal(shape)
        if scale == "unit":
            c /= np.sqrt(fan)
        cores.append(c)
    return cores


def capped_ranks(modes: Sequence[int], r: int) -> List[int]:
    """Bond ranks min(r, prod of left modes, prod of right modes)."""
    D = len(modes)
    out = [1]
    for k in range(1, D):
        left = int(np.prod(modes[:k], dtype=np.float64)) if k else 1
        right = int(np.prod(modes[k:], dtype=np.float64))
        out.append(int(min(r, left, right)))
    out.append(1)
    return out


def qtt_modes(level: int, q: int = 1) -> List[int]:
    """Mode sizes of the vector cores [component | subdomain | i1 j1 ... id jd]."""
    m = [2]
    if q > 1:
        m.append(q)
    m += [2] * (2 * level)
    return m
