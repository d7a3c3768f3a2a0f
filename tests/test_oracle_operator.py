"""Pins for the oracle's assembled operator, solver, sphere series and gradient.

* sphere eigenvalues: on the unit sphere the four boundary operators act on
  the degree-1 harmonic by closed-form factors built from j_1, h_1 (addition
  theorem); a wrong sign or a swapped operand fails by O(1);
* the Mie series is checked against exp(i k r cos t) (partial-wave sum), the
  rigid condition dp/dr = 0 at r = a (finite differences) and the Wronskian
  collapse of the surface field;
* the boundary-element solution converges to the Mie series on refined
  icospheres;
* GMRES agrees with LU; the discrete-adjoint gradient of J agrees with central
  finite differences of J.
"""
import math

import numpy as np
import pytest
from scipy.special import spherical_jn, spherical_yn

from oracle import bem, mie, solve
from workloads import admittance, icosphere, unit_directions


def _h1(n, x, d=False):
    return spherical_jn(n, x, d) + 1j * spherical_yn(n, x, d)


@pytest.fixture(scope="module")
def sphere320():
    V, T = icosphere(2)
    g = bem.Geometry(V, T)
    k = 1.0
    return g, k, bem.assemble_block(g, k)


def test_sphere_eigenvalues_degree_one(sphere320):
    g, k, (S, K, Kp, H) = sphere320
    z = g.cen[:, 2] / np.linalg.norm(g.cen, axis=1)
    j, jp, h, hp = spherical_jn(1, k), spherical_jn(1, k, True), _h1(1, k), _h1(1, k, True)
    lam = {"S": 1j * k * j * h,
           "K": 0.5j * k * k * (jp * h + j * hp),
           "Kp": 0.5j * k * k * (jp * h + j * hp),
           "H": 1j * k ** 3 * jp * hp}
    # discretisation error only (flat facets, constant elements, centroids)
    bound = {"S": 0.03, "K": 0.06, "Kp": 0.3, "H": 0.06}
    for name, M in (("S", S), ("K", K), ("Kp", Kp), ("H", H)):
        err = np.linalg.norm(M @ z - lam[name] * z) / np.linalg.norm(lam[name] * z)
        assert err < bound[name], (name, err)
        # and the opposite sign is far off
        err_neg = np.linalg.norm(M @ z + lam[name] * z) / np.linalg.norm(lam[name] * z)
        assert err_neg > 1.5


def test_mie_series_properties():
    k, a = 2.5, 1.0
    t = np.linspace(-1, 1, 7)
    r = 1.7
    assert np.allclose(mie.incident_series(k, r, t), np.exp(1j * k * r * t), atol=1e-13)
    h = 1e-6
    dr = (mie.total_field(k, a, a + h, t) - mie.total_field(k, a, a - h, t)) / (2 * h)
    assert np.abs(dr).max() < 1e-7
    assert np.allclose(mie.total_field(k, a, a, t), mie.surface_pressure(k * a, t), atol=1e-12)


@pytest.mark.slow
def test_bem_solution_converges_to_mie(sphere320):
    errs = []
    for lev in (1, 2):
        V, T = icosphere(lev)
        g = bem.Geometry(V, T)
        k, alpha = 1.0, 1j
        if lev == 2:
            _, _, (S, K, Kp, H) = sphere320
        else:
            S, K, Kp, H = bem.assemble_block(g, k)
        A = 0.5 * np.eye(g.n_elem) - K - alpha * H
        b = bem.plane_wave_rhs(g, k, alpha, [0, 0, 1.0])
        p = solve.dense_solve(A, b)
        ref = mie.surface_pressure(k, g.cen[:, 2] / np.linalg.norm(g.cen, axis=1))
        errs.append(np.linalg.norm(p - ref) / np.linalg.norm(ref))
    assert errs[1] < 0.012
    assert errs[1] < 0.5 * errs[0]


def test_gmres_matches_lu(sphere320):
    g, k, (S, K, Kp, H) = sphere320
    alpha = 1j / k
    A = 0.5 * np.eye(g.n_elem) - K - alpha * H
    b = bem.plane_wave_rhs(g, k, alpha, unit_directions(np.random.default_rng(5), 1)[0])
    x_lu = solve.dense_solve(A, b)
    x, info = solve.gmres(lambda v: A @ v, b, tol=1e-10, restart=20)
    assert info["converged"]
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-10
    assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) < 1e-8


def test_gmres_reports_non_convergence(sphere320):
    g, k, (S, K, Kp, H) = sphere320
    A = 0.5 * np.eye(g.n_elem) - K - 1j * H
    b = bem.plane_wave_rhs(g, k, 1j, [1.0, 0, 0])
    x, info = solve.gmres(lambda v: A @ v, b, tol=1e-12, restart=5, max_iter=5)
    assert not info["converged"] and info["iters"] == 5


def test_adjoint_blocks_are_conjugate_transposes(sphere320):
    g, k, _ = sphere320
    alpha = 1j / k
    rng = np.random.default_rng(3)
    rows = rng.choice(g.n_elem, 7, replace=False)
    Mp, Mq = bem.bm_blocks(g, k, alpha, rows, None)
    y = rng.standard_normal(7) + 1j * rng.standard_normal(7)
    yfull = np.zeros(g.n_elem, dtype=complex)
    yfull[rows] = y
    cols = rng.choice(g.n_elem, 9, replace=False)
    u, w = bem.matvec_adjoint(g, k, alpha, yfull, cols=cols)
    assert np.allclose(u, (Mp.conj().T @ y)[cols], atol=1e-13)
    assert np.allclose(w, (Mq.conj().T @ y)[cols], atol=1e-13)


@pytest.mark.slow
def test_objective_gradient_matches_central_differences():
    V, T = icosphere(1)
    g = bem.Geometry(V, T)
    k, alpha = 1.5, 1j / 1.5
    rng = np.random.default_rng(4)
    beta = admittance(rng, g.n_elem)
    pts = 3.0 * unit_directions(rng, 8)
    d = np.array([0.0, 0.6, 0.8])
    Mp, Mq = bem.bm_blocks(g, k, alpha)
    J, grad, _ = solve.objective_and_gradient(g, k, alpha, beta, d, pts, Mp, Mq)
    h = 1e-5
    for e in rng.choice(g.n_elem, 6, replace=False):
        for unit, comp in ((1.0, grad[e].real), (1j, grad[e].imag)):
            bp, bm_ = beta.copy(), beta.copy()
            bp[e] += unit * h
            bm_[e] -= unit * h
            Jp = solve.objective_and_gradient(g, k, alpha, bp, d, pts, Mp, Mq)[0]
            Jm = solve.objective_and_gradient(g, k, alpha, bm_, d, pts, Mp, Mq)[0]
            fd = (Jp - Jm) / (2 * h)
            assert abs(fd - comp) < 1e-6 * max(1.0, abs(comp)), (e, unit, fd, comp)


def test_representation_far_field_matches_mie(sphere320):
    g, k, (S, K, Kp, H) = sphere320
    alpha = 1j / k
    A = 0.5 * np.eye(g.n_elem) - K - alpha * H
    d = np.array([0.0, 0.0, 1.0])
    p = solve.dense_solve(A, bem.plane_wave_rhs(g, k, alpha, d))
    pts = 3.0 * unit_directions(np.random.default_rng(9), 8)
    got = solve.represent(g, k, pts, p, np.zeros_like(p), d)
    ref = mie.total_field(k, 1.0, 3.0, pts[:, 2] / 3.0)
    assert np.abs(got - ref).max() < 0.01 * np.abs(ref).max()
