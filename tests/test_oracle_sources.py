"""Pins for the point-source right-hand side and for the conventional
(alpha = 0) equation's fictitious frequencies.

* A point source receding along -d with amplitude 4 pi R e^{-ikR} tends to
  the plane wave exp(i k d.x): point_source_rhs approaches plane_wave_rhs
  (already pinned through the Mie series) at the rate 1/R.
* The alpha part of the right-hand side is the normal derivative of the
  incident field: central differences of p_inc along n at the centroids.
* Reciprocity of rigid scattering: the total field at x_o of a source at x_s
  equals the total field at x_s of a source at x_o; the discrete fields
  (dense solve + representation) agree to discretisation accuracy, and
  better on the finer mesh.
* Fictitious frequency (the non-uniqueness the paper names in Sec. 2.1 and
  leaves open in Sec. 4): the unit sphere's interior Dirichlet eigenvalue
  k = pi (j_0(k) = 0) makes I/2 - K singular; its discrete copy has a
  smallest singular value orders of magnitude below the Burton-Miller
  matrix's, and its solution misses the Mie series by orders of magnitude
  more.
"""
import numpy as np
import pytest

from oracle import bem, mie, solve
from workloads import icosphere, unit_directions


@pytest.fixture(scope="module")
def sphere320():
    V, T = icosphere(2)
    return bem.Geometry(V, T)


def test_far_point_source_tends_to_plane_wave(sphere320):
    g = sphere320
    k, alpha = 2.0, 0.5j
    d = np.array([0.36, -0.48, 0.8])
    ref = bem.plane_wave_rhs(g, k, alpha, d)
    errs = []
    for R in (1e2, 1e3, 1e4):
        amp = 4.0 * np.pi * R * np.exp(-1j * k * R)
        b = bem.point_source_rhs(g, k, alpha, -R * d, [amp])
        errs.append(np.linalg.norm(b - ref) / np.linalg.norm(ref))
    assert errs[2] < 2e-4
    for a, b_ in zip(errs, errs[1:]):
        assert 7.0 < a / b_ < 13.0     # first order in 1/R


def test_alpha_part_is_the_normal_derivative(sphere320):
    g = sphere320
    k = 3.0
    rng = np.random.default_rng(4)
    src = 2.5 * unit_directions(rng, 3)
    amp = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    b0 = bem.point_source_rhs(g, k, 0.0, src, amp)
    b1 = bem.point_source_rhs(g, k, 1.0, src, amp)
    assert np.allclose(b0, solve.point_source_field(k, g.cen, src, amp), rtol=1e-14, atol=0)
    h = 1e-5
    dn = (solve.point_source_field(k, g.cen + h * g.normal, src, amp)
          - solve.point_source_field(k, g.cen - h * g.normal, src, amp)) / (2 * h)
    assert np.linalg.norm((b1 - b0) - dn) < 1e-8 * np.linalg.norm(dn)


def _total_field(g, k, src, obs):
    """Total field at obs of a unit point source at src, rigid scatterer."""
    alpha = 1j / k
    Mp, _ = bem.bm_blocks(g, k, alpha)
    p = np.linalg.solve(Mp, bem.point_source_rhs(g, k, alpha, src, [1.0]))
    Kh, _ = solve.represent_blocks(g, k, obs[None, :])
    return solve.point_source_field(k, obs, src, [1.0])[0] + (Kh @ p)[0]


def test_reciprocity_of_the_discrete_rigid_problem():
    k = 1.5
    xs = np.array([0.4, 1.9, -0.7])
    xo = np.array([-2.2, 0.3, 1.1])
    gaps = []
    for lvl in (2, 3):
        V, T = icosphere(lvl)
        g = bem.Geometry(V, T)
        a, b = _total_field(g, k, xs, xo), _total_field(g, k, xo, xs)
        gaps.append(abs(a - b) / abs(a))
    assert gaps[1] < 5e-3
    assert gaps[1] < gaps[0]


def _smallest_singular(M):
    return np.linalg.svd(M, compute_uv=False)[-1]


# Discrete copy of k = pi on the 320-element sphere: the minimum of the
# smallest singular value of I/2 - K near pi, located by a golden-section
# search over the oracle's matrices (sigma_min ~7e-4 there).
KSTAR_ICO2 = 3.1904


def test_conventional_equation_fails_at_the_fictitious_frequency():
    V, T = icosphere(2)
    g = bem.Geometry(V, T)
    kstar = KSTAR_ICO2
    assert abs(kstar - np.pi) < 0.1
    s_star = _smallest_singular(bem.bm_blocks(g, kstar, 0.0)[0])
    s_side = min(_smallest_singular(bem.bm_blocks(g, kstar + dk, 0.0)[0]) for dk in (-0.06, 0.06))
    s_bm = _smallest_singular(bem.bm_blocks(g, kstar, 1j / kstar)[0])
    # a deep, local dip of the conventional matrix only
    assert s_star < 0.05 * s_side and s_star < 0.01 * s_bm
    # solutions against the Mie series at k*
    d = np.array([0.0, 0.0, 1.0])
    ref = mie.surface_pressure(kstar, g.cen[:, 2] / np.linalg.norm(g.cen, axis=1))
    e = {}
    for name, alpha in (("cbie", 0.0), ("bm", 1j / kstar)):
        Mp, _ = bem.bm_blocks(g, kstar, alpha)
        p = np.linalg.solve(Mp, bem.plane_wave_rhs(g, kstar, alpha, d))
        e[name] = np.linalg.norm(p - ref) / np.linalg.norm(ref)
    assert e["bm"] < 0.05
    assert e["cbie"] > 5.0 * e["bm"]
