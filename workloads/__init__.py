"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds the *input recipe* only: random numbers, macro-tetrahedron
geometries, coefficient descriptors, right-hand sides and the named workload
configurations.  It contains none of the smoother's arithmetic (no assembly,
no factorisation, no sweeps, no coefficient evaluation), so the oracle and the
HIP library can both consume its outputs without sharing method code.

Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014).  A uniform double in [0,1) is the top 53 bits
of the output times 2^-53; U[a,b] = a + (b-a) u.

Geometry recipe for a jittered macro-tetrahedron: start from the reference
vertices (0,0,0),(1,0,0),(0,1,0),(0,0,1); add 12 draws of U[-j,j] in the order
v1.x, v1.y, v1.z, v2.x, ... ; accept if det J > 0 and the aspect ratio
R_circ / (3 r_in) < 4, else redraw all 12 (continuing the same stream).
The right-hand side is U[-1,1] on the interior lattice in lexicographic order
(z slowest, then y, then x) drawn after the geometry from the same stream.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

MASK64 = (1 << 64) - 1

# coefficient kinds (the same integer codes are used at the C-ABI)
COEFF_CONST = 0      # kappa = p0
COEFF_SINPROD = 1    # kappa = p0 + p1 sin(2 pi p2 X) sin(2 pi p2 Y) sin(2 pi p2 Z)
COEFF_EXPSINCOS = 2  # kappa = exp(p0 sin(2 pi p2 X) cos(2 pi p2 Y))
COEFF_POLY = 3       # kappa = p0 + p1 (X^i + Y^i + Z^i), i = int(p2)

REFERENCE_TET = ((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))


class SplitMix64:
    """Counter-based SplitMix64 stream (published constants)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def uniform_ab(self, a: float, b: float) -> float:
        return a + (b - a) * self.uniform()

    def uniform_array(self, count: int, a: float, b: float) -> np.ndarray:
        """`count` draws of U[a,b]; vectorised SplitMix64 with identical output."""
        if count == 0:
            return np.zeros(0)
        golden = np.uint64(0x9E3779B97F4A7C15)
        k = np.arange(1, count + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            z = np.uint64(self.state) + k * golden
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            z = z ^ (z >> np.uint64(31))
        self.state = (self.state + count * 0x9E3779B97F4A7C15) & MASK64
        u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
        return a + (b - a) * u


def num_interior(level: int) -> int:
    """#{(x,y,z): x,y,z >= 1, x+y+z <= 2^L - 1} = C(2^L - 1, 3)."""
    n = 1 << level
    return (n - 1) * (n - 2) * (n - 3) // 6


def aspect_ratio(verts: Sequence[Sequence[float]]) -> float:
    """R_circ / (3 r_in): 1 for the regular tetrahedron."""
    v = np.asarray(verts, dtype=np.float64)
    e = v[1:] - v[0]
    vol6 = abs(np.linalg.det(e))
    if vol6 == 0.0:
        return math.inf
    faces = [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]
    area = sum(0.5 * np.linalg.norm(np.cross(v[b] - v[a], v[c] - v[a])) for a, b, c in faces)
    r_in = 3.0 * (vol6 / 6.0) / area
    # circumcentre c solves 2 (v_i - v_0) . c = |v_i|^2 - |v_0|^2
    rhs = np.array([v[i] @ v[i] - v[0] @ v[0] for i in (1, 2, 3)])
    c = np.linalg.solve(2.0 * e, rhs)
    r_circ = np.linalg.norm(c - v[0])
    return r_circ / (3.0 * r_in)


def det_j(verts) -> float:
    v = np.asarray(verts, dtype=np.float64)
    return float(np.linalg.det((v[1:] - v[0]).T))


def jittered_tet(rng: SplitMix64, jitter: float, max_aspect: float = 4.0):
    while True:
        v = [[REFERENCE_TET[i][k] + rng.uniform_ab(-jitter, jitter) for k in range(3)] for i in range(4)]
        if det_j(v) > 0.0 and aspect_ratio(v) < max_aspect:
            return tuple(tuple(row) for row in v)


@dataclasses.dataclass(frozen=True)
class Tet:
    """One macro-tetrahedron problem: geometry, level, coefficient and seeded RHS."""
    verts: tuple
    level: int
    coeff_kind: int
    coeff_params: tuple  # 4 doubles
    rhs_state: int       # SplitMix64 state right before the RHS draws

    @property
    def n_interior(self) -> int:
        return num_interior(self.level)

    def rhs(self) -> np.ndarray:
        r = SplitMix64(0)
        r.state = self.rhs_state
        return r.uniform_array(self.n_interior, -1.0, 1.0)


def make_tet(seed: int, level: int, coeff_kind: int, coeff_params, jitter: float = 0.0) -> Tet:
    rng = SplitMix64(seed)
    verts = jittered_tet(rng, jitter) if jitter > 0.0 else REFERENCE_TET
    p = tuple(float(c) for c in coeff_params) + (0.0,) * (4 - len(coeff_params))
    return Tet(verts, level, coeff_kind, p, rng.state)


KAPPA_SIN = (COEFF_SINPROD, (1.0, 0.5, 1.0, 0.0))     # 1 + 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z)
KAPPA_EXP = (COEFF_EXPSINCOS, (0.5, 0.0, 2.0, 0.0))   # exp(0.5 sin(4 pi x) cos(4 pi y))


def batch_tets(seed: int, count: int, levels: Sequence[int], coeff=KAPPA_SIN, jitter=0.15) -> List[Tet]:
    """Tet i uses SplitMix64(seed ^ i): one draw picks the level, then geometry, then RHS."""
    out = []
    for i in range(count):
        rng = SplitMix64(seed ^ i)
        level = levels[min(int(rng.uniform() * len(levels)), len(levels) - 1)]
        verts = jittered_tet(rng, jitter)
        out.append(Tet(verts, level, coeff[0], coeff[1], rng.state))
    return out


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    tets: tuple
    variant: str          # "stored_f64" | "surr_f64" | "surr_f32"
    degree: int
    stride: int
    sweeps: int
    rel_tol: float = 0.0


def workload(name: str) -> Workload:
    """The five named workloads (sizes from the method's test problems)."""
    if name == "ref_L4":
        t = make_tet(1, 4, COEFF_CONST, (1.0,))
        return Workload(name, (t,), "stored_f64", 0, 0, 10)
    if name == "jit_L7_sin":
        t = make_tet(2, 7, *KAPPA_SIN, jitter=0.15)
        return Workload(name, (t,), "surr_f64", 4, 4, 20)
    if name == "jit_L8_sin":
        t = make_tet(3, 8, *KAPPA_SIN, jitter=0.15)
        return Workload(name, (t,), "surr_f32", 4, 4, 20, 1e-10)
    if name == "batch256_L567":
        return Workload(name, tuple(batch_tets(4, 256, (5, 6, 7))), "surr_f32", 4, 4, 20)
    if name == "jit_L9_exp":
        t = make_tet(5, 9, *KAPPA_EXP, jitter=0.15)
        return Workload(name, (t,), "surr_f32", 6, 4, 20)
    if name == "flat_L8_const":
        # trirectangular tetrahedron of height 0.1, unit coefficient: the
        # distorted tetrahedron of the anisotropic-degree study
        t = Tet(FLAT_TET, 8, COEFF_CONST, (1.0, 0.0, 0.0, 0.0), SplitMix64(6).state)
        return Workload(name, (t,), "surr_f32", 6, 4, 20)
    raise KeyError(name)


FLAT_TET = ((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 0.1))
WORKLOADS = ("ref_L4", "jit_L7_sin", "jit_L8_sin", "batch256_L567", "jit_L9_exp", "flat_L8_const")
