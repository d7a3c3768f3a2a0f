"""Pins of the oracle's finite elements and coupled operator (oracle/fem.py,
Sec. 2.3: Eq. fem_2 with linear tetrahedra, Eqs. renritupu, kousokuu,
GMRES), CPU only:

* the ball mesh is conforming and its boundary faces are the surface
  triangles (outward normals);
* linear shape functions: gradients sum to zero and reproduce the identity;
* the stiffness annihilates the six rigid motions; an affine displacement
  has exactly the strain energy V (lam tr(e)^2 + 2 mu e:e) (patch test);
* the mass matrix integrates rho over the volume;
* the coupling integrates the normal (its total over a closed surface
  vanishes) and C diag(1 / area) is symmetric;
* rigid limit: a body ever stiffer and heavier leaves the sound-hard
  operator (C -> 0).
"""
from collections import Counter

import numpy as np

from oracle import fem
from workloads import ball_mesh


def _mesh(level=1, n_shell=2):
    return ball_mesh(level, n_shell)


def test_ball_mesh_is_conforming_with_the_surface_as_boundary():
    nodes, tets, V, T = _mesh(2, 3)
    assert np.allclose(nodes[:len(V)], V)
    cnt = Counter()
    for t in tets:
        for f in ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)):
            cnt[tuple(sorted(t[list(f)]))] += 1
    assert max(cnt.values()) == 2
    bnd = {f for f, c in cnt.items() if c == 1}
    assert bnd == {tuple(sorted(t)) for t in T}
    vols = [abs(fem.tet_geometry(nodes[t])[0]) for t in tets]
    assert min(vols) > 0
    # the polyhedral ball's volume equals the volume enclosed by its surface
    X = V[T]
    enclosed = np.einsum("ij,ij->i", X[:, 0], np.cross(X[:, 1], X[:, 2])).sum() / 6
    assert abs(sum(vols) - enclosed) < 1e-12 * enclosed and enclosed > 0


def test_shape_function_gradients():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(4, 3))
    vol, g = fem.tet_geometry(X)
    assert abs(vol) > 1e-3
    assert np.max(np.abs(g.sum(axis=0))) < 1e-12
    assert np.max(np.abs(X.T @ g - np.eye(3))) < 1e-12     # sum_a x_a (x) grad phi_a = I


def test_stiffness_rigid_modes_and_patch_test():
    nodes, tets, _, _ = _mesh(1, 2)
    lam, mu = 2.3, 0.7
    K, M = fem.elasticity_matrices(nodes, tets, lam, mu, 1.0)
    scale = np.max(np.abs(K))
    n = len(nodes)
    for i in range(3):                     # translations
        u = np.zeros((n, 3))
        u[:, i] = 1.0
        assert np.max(np.abs(K @ u.ravel())) < 1e-12 * scale
    for w in np.eye(3):                    # infinitesimal rotations w x x
        u = np.cross(w[None, :], nodes)
        assert np.max(np.abs(K @ u.ravel())) < 1e-12 * scale
    rng = np.random.default_rng(4)
    G = rng.normal(size=(3, 3))
    u = (nodes @ G.T).ravel()              # u(x) = G x
    e = 0.5 * (G + G.T)
    vol = sum(abs(fem.tet_geometry(nodes[t])[0]) for t in tets)
    energy = vol * (lam * np.trace(e) ** 2 + 2 * mu * np.sum(e * e))
    assert abs(u @ K @ u - energy) < 1e-12 * energy
    # interior nodes carry no force under a constant stress
    f = (K @ u).reshape(n, 3)
    surf = np.zeros(n, dtype=bool)
    surf[:len(_mesh(1, 2)[2])] = True
    assert np.max(np.abs(f[~surf])) < 1e-12 * np.max(np.abs(f))


def test_mass_matrix_integrates_density():
    nodes, tets, _, _ = _mesh(1, 2)
    rho = 1.7
    _, M = fem.elasticity_matrices(nodes, tets, 1.0, 1.0, rho)
    vol = sum(abs(fem.tet_geometry(nodes[t])[0]) for t in tets)
    n = len(nodes)
    for i in range(3):
        c = np.zeros((n, 3))
        c[:, i] = 1.0
        assert abs(c.ravel() @ M @ c.ravel() - rho * vol) < 1e-12 * rho * vol
    # consistent mass: the quadratic x_i^2 integrates exactly (degree 2)
    xq = np.zeros((n, 3))
    xq[:, 0] = nodes[:, 0]
    exact = 0.0
    for t in tets:
        X = nodes[t]
        V = abs(fem.tet_geometry(X)[0])
        s = X[:, 0]
        exact += V * (s.sum() ** 2 + (s * s).sum()) / 20
    assert abs(xq.ravel() @ M @ xq.ravel() - rho * exact) < 1e-12 * rho * exact


def test_coupling_integrates_the_normal():
    nodes, tets, V, T = _mesh(2, 2)
    Tc, N, area, nrm = fem.surface_coupling(nodes, T)
    n = len(nodes)
    # sum over the three vertices: A_j n_j; over the closed surface: 0
    tot = N.reshape(n, 3, len(T)).sum(axis=0)
    assert np.max(np.abs(tot - (area[:, None] * nrm).T)) < 1e-14
    assert np.max(np.abs(tot.sum(axis=1))) < 1e-12
    # outward normals on the sphere
    cen = nodes[T].mean(axis=1)
    assert np.all(np.einsum("ij,ij->i", nrm, cen) > 0)
    C = fem.coupling_matrix(nodes, tets, T, 2.0, 1.0, 1.5, 1.0, 1.3)
    S = C / area[None, :]
    assert np.max(np.abs(S - S.T)) < 1e-10 * np.max(np.abs(S))


def test_rigid_limit():
    nodes, tets, V, T = _mesh(1, 2)
    base = np.max(np.abs(fem.coupling_matrix(nodes, tets, T, 2.0, 1.0, 1.5, 1.0, 1.3)))
    for s in (1e4, 1e8):
        C = fem.coupling_matrix(nodes, tets, T, 2.0 * s, 1.0 * s, 1.5 * s, 1.0, 1.3)
        assert np.max(np.abs(C)) < 3.0 / s * base
