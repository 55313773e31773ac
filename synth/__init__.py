"""Seeded synthetic workloads shared by the oracle and the HIP path.

This module holds no part of the discontinuous Galerkin method: it builds
meshes (vertex coordinates and tetrahedra), draws per-element material
values and mode amplitudes, and provides the closed-form cavity fields as
plain Python callables.  Each side projects those fields onto its own basis.

Mesh recipe (cube cavity, Section 2.2 uses a sphere instead; the sphere mesh
is not available, so PEC cube cavities stand in):
  * the unit cube [0,1]^3 split into an n x n x n grid of cells, h = 1/n;
  * vertex id  ix + (n+1)*(iy + (n+1)*iz);
  * each cell split into the 6 Kuhn (Freudenthal) tetrahedra
    (c, c+e_s1, c+e_s1+e_s2, c+(1,1,1)h) for the 6 permutations s of the axes;
    vertex ids then increase along every tetrahedron, so the local vertex order
    is already the sorted global order;
  * optional jitter: interior vertices move by U(-j*h, j*h) in every
    coordinate, boundary vertices only in their tangential coordinates, and
    cube corners stay fixed, so the domain remains the unit cube.
Random draws use numpy's PCG64 ``default_rng(seed)`` in the fixed order
jitter -> eps -> amplitudes -> arrivals.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

# The six axis permutations, in a fixed order.
_PERMS = list(itertools.permutations(range(3)))


def kuhn_mesh(n: int, jitter: float = 0.0, rng: np.random.Generator | None = None):
    """Return (verts float64[nv,3], tets int64[nt,4]) of the Kuhn split of n^3 cells."""
    if n < 1:
        raise ValueError("n must be >= 1")
    m = n + 1
    h = 1.0 / n
    g = np.arange(m)
    iz, iy, ix = np.meshgrid(g, g, g, indexing="ij")
    ijk = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)  # vertex id order
    verts = ijk.astype(np.float64) * h
    if jitter > 0.0:
        if rng is None:
            raise ValueError("jitter needs an rng")
        d = rng.uniform(-jitter * h, jitter * h, size=verts.shape)
        on_bnd = (ijk == 0) | (ijk == n)
        d[on_bnd] = 0.0  # boundary coordinates stay on their faces
        verts = verts + d
    tets = []
    for cz in range(n):
        for cy in range(n):
            for cx in range(n):
                for perm in _PERMS:
                    c = np.array([cx, cy, cz])
                    path = [c.copy()]
                    for ax in perm:
                        c = c.copy()
                        c[ax] += 1
                        path.append(c)
                    tets.append([p[0] + m * (p[1] + m * p[2]) for p in path])
    return verts, np.asarray(tets, dtype=np.int64)


def single_tet(vertices=None):
    """One tetrahedron (by default the reference one)."""
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float) if vertices is None else np.asarray(vertices, float)
    return v, np.array([[0, 1, 2, 3]], dtype=np.int64)


def two_tets(rng: np.random.Generator | None = None):
    """Two tetrahedra sharing one face, vertex ids deliberately unsorted in one tet."""
    v = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 1.0, 0.1], [0.1, 0.2, 1.0], [0.9, 0.9, 0.8]])
    if rng is not None:
        v = v + rng.uniform(-0.05, 0.05, size=v.shape)
    return v, np.array([[0, 1, 2, 3], [4, 3, 2, 1]], dtype=np.int64)


# ---------------------------------------------------------------------------
# Closed-form PEC cube cavity fields (eps = mu = 1 unless scaled by the caller)
# E = (Ax cos kx x sin ky y sin kz z, Ay sin cos sin, Az sin sin cos), k = pi (l,m,n),
# k . A = 0, omega = |k| / sqrt(eps mu);  H follows from mu dH/dt = -curl E.
# ---------------------------------------------------------------------------

@dataclass
class CavityMode:
    lmn: tuple
    amp: tuple  # (Ax, Ay, Az), must satisfy k.A = 0
    eps: float = 1.0
    mu: float = 1.0

    @property
    def k(self):
        return np.pi * np.asarray(self.lmn, float)

    @property
    def omega(self):
        return float(np.linalg.norm(self.k) / math.sqrt(self.eps * self.mu))

    def _spatial_e(self, x):
        kx, ky, kz = self.k
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        ax, ay, az = self.amp
        return np.stack([
            ax * np.cos(kx * X) * np.sin(ky * Y) * np.sin(kz * Z),
            ay * np.sin(kx * X) * np.cos(ky * Y) * np.sin(kz * Z),
            az * np.sin(kx * X) * np.sin(ky * Y) * np.cos(kz * Z),
        ], axis=-1)

    def _spatial_curl_e(self, x):
        kx, ky, kz = self.k
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        ax, ay, az = self.amp
        cx, sx = np.cos(kx * X), np.sin(kx * X)
        cy, sy = np.cos(ky * Y), np.sin(ky * Y)
        cz, sz = np.cos(kz * Z), np.sin(kz * Z)
        # d/dy Ez - d/dz Ey, d/dz Ex - d/dx Ez, d/dx Ey - d/dy Ex
        return np.stack([
            az * sx * ky * cy * cz - ay * sx * cy * kz * cz,
            ax * cx * sy * kz * cz - az * kx * cx * sy * cz,
            ay * kx * cx * cy * sz - ax * cx * ky * cy * sz,
        ], axis=-1)

    def E(self, x, t=0.0):
        """Electric field at points x[...,3] and time t (standing wave, E ~ cos wt)."""
        return self._spatial_e(x) * math.cos(self.omega * t)

    def H(self, x, t=0.0):
        """Magnetic field: mu dH/dt = -curl E  =>  H = -curl E0 sin(wt) / (mu w)."""
        w = self.omega
        return -self._spatial_curl_e(x) * (math.sin(w * t) / (self.mu * w))


def te101(eps: float = 1.0, mu: float = 1.0, scale: float = 1.0) -> CavityMode:
    """TE101 of the unit cube: E = (0, sin pi x sin pi z, 0) cos wt, w = pi sqrt(2/(eps mu))."""
    return CavityMode((1, 0, 1), (0.0, scale, 0.0), eps, mu)


class ModeSum:
    """Superposition of cavity modes sharing eps and mu."""

    def __init__(self, modes):
        self.modes = list(modes)

    def E(self, x, t=0.0):
        return sum(m.E(x, t) for m in self.modes)

    def H(self, x, t=0.0):
        return sum(m.H(x, t) for m in self.modes)


def three_mode_sum(rng: np.random.Generator, eps: float = 1.0, mu: float = 1.0) -> ModeSum:
    """TE101 + TE011 + TE110 with N(0,1) amplitudes drawn in that order.

    TE011 is E = (sin pi y sin pi z, 0, 0), TE101 is (0, sin pi x sin pi z, 0),
    TE110 is (0, 0, sin pi x sin pi y); all three have w = pi sqrt(2/(eps mu)).
    """
    a = rng.standard_normal(3)
    return ModeSum([
        CavityMode((1, 0, 1), (0.0, a[0], 0.0), eps, mu),
        CavityMode((0, 1, 1), (a[1], 0.0, 0.0), eps, mu),
        CavityMode((1, 1, 0), (0.0, 0.0, a[2]), eps, mu),
    ])


# ---------------------------------------------------------------------------
# The five workloads.  Sizes follow the benchmark table; the shapes of the
# paper's own experiments (a 2078-tet mesh, a 30-element sphere) are not
# available, so cube cavities of the stated sizes stand in for them.
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    n: int
    p: int
    dtype: str  # "f64" or "f32"
    steps: int
    seed: int
    jitter: float = 0.0
    eps_choices: tuple = (1.0,)
    init: str = "te101"  # "te101", "three_mode", "random"
    extra: dict = field(default_factory=dict)

    @property
    def K(self):
        return 6 * self.n ** 3


WORKLOADS = {
    "cube2_p2_f64": Workload("cube2_p2_f64", 2, 2, "f64", 100, 1),
    "cube16_p4_f32": Workload("cube16_p4_f32", 16, 4, "f32", 1000, 2, init="three_mode"),
    "cube32_p6_f32": Workload("cube32_p6_f32", 32, 6, "f32", 500, 3, jitter=0.1, eps_choices=(1.0, 4.0), init="three_mode"),
    "cube24_p8_dense": Workload("cube24_p8_dense", 24, 8, "f32", 200, 4, init="random"),
}


def build_workload(w: Workload):
    """Draw everything a workload needs, in the fixed order jitter -> eps -> amplitudes.

    Returns dict(verts, tets, eps[K], mu[K], field) where ``field`` is a ModeSum /
    CavityMode (closed-form initial E, H) or, for init == "random", an rng to draw
    modal coefficients from.
    """
    rng = np.random.default_rng(w.seed)
    verts, tets = kuhn_mesh(w.n, w.jitter, rng if w.jitter > 0 else None)
    K = tets.shape[0]
    if len(w.eps_choices) > 1:
        eps = rng.choice(np.asarray(w.eps_choices, float), size=K)
    else:
        eps = np.full(K, w.eps_choices[0])
    mu = np.ones(K)
    if w.init == "te101":
        fld = te101()
    elif w.init == "three_mode":
        fld = three_mode_sum(rng)
    else:
        fld = rng
    return dict(verts=verts, tets=tets, eps=eps, mu=mu, field=fld)


def splitmix64(seed: int, count: int) -> np.ndarray:
    """SplitMix64 (Steele, Lea, Flood 2014) as uniform doubles in [-1, 1).

    Used wherever a start vector must be identical on both sides without
    passing it in (the power iteration of the time-step estimate).
    """
    out = np.empty(count, dtype=np.float64)
    mask = (1 << 64) - 1
    s = seed & mask
    for i in range(count):
        s = (s + 0x9E3779B97F4A7C15) & mask
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        z = z ^ (z >> 31)
        out[i] = (z >> 11) * (1.0 / (1 << 53)) * 2.0 - 1.0
    return out
