"""Pins of the elastic-sphere series (oracle/elastic_sphere.py; the analytic
solution Sec. 3.1 checks the BEM-FEM solver against), CPU only:

* a sphere ever stiffer and heavier tends to the rigid sphere (the Mie
  series of oracle/mie.py), with a difference falling as 1 / scale;
* lossless scattering: every partial wave keeps its amplitude,
  |1 + 2 A_n| = 1;
* the discrete BEM-FEM oracle (linear tetrahedra, collocation BEM, dense
  solves of the coupled operator) converges to the series under mesh
  refinement for a soft body whose elastic response changes the surface
  pressure by 23% against the rigid sphere; a sign error in the solid's
  normal traction (planted in a copy of the series) misses the discrete
  solution by 6.8%, five times the coarse mesh's 1.3%.
"""
import numpy as np

from oracle import bem as obem
from oracle import elastic_sphere as es
from oracle import fem, mie
from workloads import ball_mesh

SOFT = dict(lam=2.0, mu=1.0, rho_s=1.5, rho_f=1.0)


def test_rigid_limit_is_the_mie_series():
    ct = np.linspace(-1, 1, 13)
    pr = mie.surface_pressure(2.0, ct)
    errs = []
    for s in (1e4, 1e6, 1e8):
        p = es.surface_pressure(2.0, 1.0, 2.0 * s, 1.0 * s, 1.5 * s, 1.0, 2.0, ct)
        errs.append(np.max(np.abs(p - pr)) / np.max(np.abs(pr)))
    assert errs[0] > 1e-5 and errs[1] < errs[0] / 50 and errs[2] < errs[1] / 50
    assert errs[2] < 1e-6


def test_partial_waves_are_unitary():
    for k, a in ((1.0, 1.0), (3.0, 0.7), (0.3, 2.0)):
        A, _, _ = es.coefficients(k, a, SOFT["lam"], SOFT["mu"], SOFT["rho_s"], SOFT["rho_f"], k)
        assert np.max(np.abs(np.abs(1 + 2 * A) - 1)) < 1e-12


def _discrete_error(level, n_shell, omega=1.0):
    nodes, tets, V, T = ball_mesh(level, n_shell)
    g = obem.Geometry(V, T)
    Mp, Mq = obem.bm_blocks(g, omega, 0.0)
    C = fem.coupling_matrix(nodes, tets, T, SOFT["lam"], SOFT["mu"], SOFT["rho_s"],
                            SOFT["rho_f"], omega)
    b = obem.plane_wave_rhs(g, omega, 0.0, np.array([0.0, 0.0, 1.0]))
    p = np.linalg.solve(fem.coupled_operator(Mp, Mq, C), b)
    ct = g.cen[:, 2] / np.linalg.norm(g.cen, axis=1)
    pa = es.surface_pressure(omega, 1.0, SOFT["lam"], SOFT["mu"], SOFT["rho_s"], SOFT["rho_f"],
                             omega, ct)
    pr = mie.surface_pressure(omega, ct)
    return (float(np.linalg.norm(p - pa) / np.linalg.norm(pa)),
            float(np.linalg.norm(pr - pa) / np.linalg.norm(pa)))


def test_discrete_coupled_oracle_converges_to_the_series():
    e2, rigid = _discrete_error(2, 2)     # 320 boundary triangles, 975 unknowns
    e3, _ = _discrete_error(3, 3)         # 1280 boundary triangles, 5781 unknowns
    assert rigid > 0.2                    # the elastic response matters
    assert e2 < 0.02 and e3 < 0.01 and e3 < 0.7 * e2
