"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module only *prepares inputs*: closed surface meshes shaped like the
paper's scatterers (a sphere, Sec. 3.1; the paper's optimised shapes are
replaced by a cube), random densities, incidence directions, admittances and
observation points.  It contains none of the boundary-element arithmetic
(no kernels, quadrature, tree or solver) so that the oracle and the HIP
library stay independent of each other.

Conventions
-----------
* Meshes are ``(V, T)``: ``V`` float64 ``(n_vert, 3)``, ``T`` int32
  ``(n_tri, 3)``, triangles ordered counter-clockwise when seen from the
  fluid, i.e. the right-hand normal points out of the scatterer, matching the
  paper's normal that is exterior with respect to the scatterer (Sec. 2.1).
* Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64) and are
  drawn in a fixed order: densities (real block, then imaginary block), then
  directions, then admittances, then observation points, then element picks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "icosphere", "cube_surface", "complex_normal", "unit_directions",
    "Workload", "workload", "WORKLOADS",
]


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
def _orient_outward(V: np.ndarray, T: np.ndarray, inside: np.ndarray) -> np.ndarray:
    """Flip triangles whose right-hand normal points towards ``inside``."""
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    nrm = np.cross(b - a, c - a)
    cen = (a + b + c) / 3.0
    flip = np.einsum("ij,ij->i", nrm, cen - inside) < 0
    T = T.copy()
    T[flip, 1], T[flip, 2] = T[flip, 2].copy(), T[flip, 1].copy()
    return T


def _icosahedron():
    g = (1.0 + math.sqrt(5.0)) / 2.0
    pts = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            pts.append((s1, s2 * g, 0.0))
            pts.append((0.0, s1, s2 * g))
            pts.append((s2 * g, 0.0, s1))
    V = np.array(pts, dtype=np.float64)
    # faces = triples of mutually adjacent vertices (edge length 2 before scaling)
    d2 = ((V[:, None, :] - V[None, :, :]) ** 2).sum(-1)
    adj = np.abs(d2 - 4.0) < 1e-9
    faces = []
    n = len(V)
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if adj[i, k] and adj[j, k]:
                    faces.append((i, j, k))
    assert len(faces) == 20
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    T = np.array(faces, dtype=np.int64)
    return V, T


def icosphere(level: int, radius: float = 1.0):
    """Unit icosahedron refined ``level`` times by 4-way midpoint splits,
    new vertices pushed to the sphere.  ``n_tri = 20 * 4**level``."""
    V, T = _icosahedron()
    T = _orient_outward(V, T, np.zeros(3))
    verts = [tuple(v) for v in V]
    for _ in range(level):
        cache: dict = {}

        def mid(i, j):
            key = (i, j) if i < j else (j, i)
            if key not in cache:
                m = np.add(verts[i], verts[j]) * 0.5
                m = m / np.linalg.norm(m)
                cache[key] = len(verts)
                verts.append(tuple(m))
            return cache[key]

        newT = []
        for a, b, c in T:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            newT += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        T = np.array(newT, dtype=np.int64)
    V = np.array(verts, dtype=np.float64) * radius
    return V, T.astype(np.int32)


def ball_mesh(level: int, n_shell: int = 3):
    """Tetrahedral mesh of the unit ball whose boundary faces are the
    triangles of ``icosphere(level)``: concentric scaled copies of the surface
    vertices at radii s / n_shell (s = n_shell .. 1), the prism between two
    shells over each surface triangle split into three tetrahedra (with the
    triangle's vertices sorted a < b < c, inner shell 0 and outer shell 1:
    (a0 b0 c0 c1), (a0 b0 b1 c1), (a0 a1 b1 c1), so every quadrilateral face
    is cut along the same diagonal from both sides), the innermost layer
    joined to the centre.  Returns (nodes, tets, V, T): the first len(V)
    nodes are the surface vertices V, T the surface triangles (the
    icosphere's, outward normals)."""
    V, T = icosphere(level)
    nv = len(V)
    shells = [V * (s / n_shell) for s in range(n_shell, 0, -1)]   # shell index 0 = surface
    nodes = np.vstack(shells + [np.zeros((1, 3))])
    centre = n_shell * nv

    def idx(shell, v):  # shell 0 = surface (radius 1), n_shell - 1 = innermost
        return shell * nv + v

    tets = []
    for tri in T:
        a, b, c = sorted(int(v) for v in tri)
        for sh in range(n_shell - 1):       # outer shell sh, inner shell sh + 1
            a1, b1, c1 = idx(sh, a), idx(sh, b), idx(sh, c)
            a0, b0, c0 = idx(sh + 1, a), idx(sh + 1, b), idx(sh + 1, c)
            tets += [(a0, b0, c0, c1), (a0, b0, b1, c1), (a0, a1, b1, c1)]
        inner = n_shell - 1
        tets.append((centre, idx(inner, a), idx(inner, b), idx(inner, c)))
    return nodes, np.array(tets, dtype=np.int32), V, T


def cube_surface(n: int = 64, half: float = 1.0):
    """Surface of the cube ``[-half, half]^3``; each face is an ``n x n`` grid
    of squares, each split along its (i,j)->(i+1,j+1) diagonal.
    ``n_tri = 12 n^2``, ``n_vert = 6 n^2 + 2``."""
    index: dict = {}
    verts = []

    def vid(ijk):
        if ijk not in index:
            index[ijk] = len(verts)
            verts.append(ijk)
        return index[ijk]

    tris = []
    for axis in range(3):
        for side in (0, n):
            u_ax, v_ax = [a for a in range(3) if a != axis]
            for i in range(n):
                for j in range(n):
                    def P(ii, jj):
                        c = [0, 0, 0]
                        c[axis] = side
                        c[u_ax] = ii
                        c[v_ax] = jj
                        return vid(tuple(c))
                    p00, p10, p11, p01 = P(i, j), P(i + 1, j), P(i + 1, j + 1), P(i, j + 1)
                    tris.append((p00, p10, p11))
                    tris.append((p00, p11, p01))
    V = (np.array(verts, dtype=np.float64) * (2.0 * half / n)) - half
    T = np.array(tris, dtype=np.int64)
    T = _orient_outward(V, T, np.zeros(3))
    return V, T.astype(np.int32)


# --------------------------------------------------------------------------
# random inputs
# --------------------------------------------------------------------------
def complex_normal(rng: np.random.Generator, n: int) -> np.ndarray:
    """Complex vector with Re and Im ~ N(0,1); real block drawn first."""
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    return re + 1j * im


def unit_directions(rng: np.random.Generator, m: int) -> np.ndarray:
    """``m`` directions uniform on the unit sphere (normalised Gaussians)."""
    g = rng.standard_normal((m, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def admittance(rng: np.random.Generator, n: int, hi: float = 0.5) -> np.ndarray:
    """Per-element complex admittance, Re and Im independently U[0, hi]."""
    re = rng.uniform(0.0, hi, n)
    im = rng.uniform(0.0, hi, n)
    return re + 1j * im


# --------------------------------------------------------------------------
# the five workloads (sizes, wavenumbers and seeds)
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    mesh: str              # "ico<level>" or "cube<n>"
    k: float
    seed: int
    order: int | None = None     # fixed expansion order, None = chosen from tolerance
    leaf_cap: int = 32
    tol: float = 1e-6
    extra: dict = field(default_factory=dict)

    def mesh_arrays(self):
        if self.mesh.startswith("ico"):
            return icosphere(int(self.mesh[3:]))
        if self.mesh.startswith("cube"):
            return cube_surface(int(self.mesh[4:]))
        raise ValueError(self.mesh)

    @property
    def alpha(self) -> complex:
        """Burton-Miller coupling i/k."""
        return 1j / self.k


WORKLOADS = {
    "sphere1280_k1": Workload("sphere1280_k1", "ico3", 1.0, 1, order=8, leaf_cap=32),
    "sphere20480_k4": Workload("sphere20480_k4", "ico5", 4.0, 2),
    "sphere81920_k8": Workload("sphere81920_k8", "ico6", 8.0, 3),
    "cube49152_k6": Workload("cube49152_k6", "cube64", 6.0, 4),
    # twice the wavenumber on the same mesh (~21 elements per wavelength):
    # higher expansion orders, where the rotation-based translations pay
    "sphere81920_k16": Workload("sphere81920_k16", "ico6", 16.0, 6),
}


# mixed-mesh batch: 16 state solves and the 16 matching adjoint solves
BATCH_LEVELS = (4, 5, 6)
BATCH_KS = (2.0, 4.0, 8.0)


def batch32(seed: int = 5):
    """State solve s = 0..15 runs on icosphere level ``[4,5,6][s mod 3]`` at
    ``k = [2,4,8][(s div 3) mod 3]`` with a seeded incidence direction; the
    adjoint solve s reuses its mesh and k.  Returns ``(cases, obs)`` with
    cases = [(level, k, direction)] and 8 observation points on the
    radius-3 sphere."""
    rng = np.random.default_rng(seed)
    dirs = unit_directions(rng, 16)
    obs = 3.0 * unit_directions(rng, 8)
    cases = [(BATCH_LEVELS[s % 3], BATCH_KS[(s // 3) % 3], dirs[s]) for s in range(16)]
    return cases, obs


def workload(name: str) -> Workload:
    return WORKLOADS[name]


# --------------------------------------------------------------------------
# the elastic-sphere benchmark of the BEM-FEM coupling (Sec. 3.1): a tungsten
# sphere of radius 0.25 in water, plane wave along x_3 at omega = 1; material
# constants normalised by water's density and bulk modulus (so c_f = 1 and
# k = omega).  The paper meshes the surface with 2456 triangles and the body
# with 3007 nodes; the stand-in is the ball mesh over the 1280-triangle
# icosphere with 5 shells (3211 nodes, 9633 unknowns).
# --------------------------------------------------------------------------
@dataclass
class ElasticSphere:
    radius: float = 0.25
    level: int = 3
    n_shell: int = 5
    rho_s: float = 64.85
    young: float = 174.57
    poisson: float = 0.3
    rho_f: float = 1.0
    omega: float = 1.0
    direction: tuple = (0.0, 0.0, 1.0)

    @property
    def lam(self) -> float:
        """Lame's first parameter E nu / ((1 + nu)(1 - 2 nu))."""
        nu = self.poisson
        return self.young * nu / ((1 + nu) * (1 - 2 * nu))

    @property
    def mu(self) -> float:
        """Shear modulus E / (2 (1 + nu))."""
        return self.young / (2 * (1 + self.poisson))

    def mesh(self):
        """(nodes, tets, V, T) scaled to the sphere's radius."""
        nodes, tets, V, T = ball_mesh(self.level, self.n_shell)
        return nodes * self.radius, tets, V * self.radius, T


ELASTIC_SPHERE = ElasticSphere()
