"""GPU tests of the paper's own source term and of the conventional
equation's fictitious frequencies.

* Point-source right-hand side (Eq. hel) against the oracle, alpha = i/k and
  alpha = 0.
* Rigid scattering of a point source: the GPU solve plus field evaluation
  against the oracle's dense solve at an exterior point, and reciprocity
  (source and receiver swapped) to discretisation accuracy.
* Conventional (alpha = 0) against Burton-Miller near the unit sphere's
  interior Dirichlet eigenvalue k = pi (the non-uniqueness of Sec. 2.1,
  left open in Sec. 4): over a scan of k, the conventional equation's GMRES
  step count peaks sharply at its discrete resonance while Burton-Miller's
  stays flat, and there its solution misses the Mie series by far more.
"""
import numpy as np
import pytest

from oracle import bem as obem
from oracle import mie, solve
from workloads import icosphere

pytestmark = pytest.mark.gpu


def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1606_02383_amd as bem
    bem.load_library()
    return bem


def _log(msg):
    print(msg, flush=True)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


SRC = np.array([[0.4, 1.9, -0.7], [-1.5, -1.2, 2.0]])
AMP = np.array([1.0 + 0.5j, -0.3 + 0.8j])


@pytest.mark.parametrize("alpha", [None, 0j])
def test_point_source_rhs_against_oracle(alpha):
    bem = _lib()
    V, T = icosphere(3)
    k = 1.5
    a = 1j / k if alpha is None else alpha
    plan = bem.Plan(bem.Problem(V, T, k, alpha=alpha))
    g = obem.Geometry(V, T)
    b = plan.point_source_rhs(SRC, AMP).cpu().numpy()
    ref = obem.point_source_rhs(g, k, a, SRC, AMP)
    e = _rel(b, ref)
    _log(f"case: point-source rhs alpha={a}: rel err {e:.2e}")
    assert e < 1e-13


def test_point_source_scattering_parity_and_reciprocity():
    import torch
    bem = _lib()
    V, T = icosphere(3)
    k = 1.5
    g = obem.Geometry(V, T)
    plan = bem.Plan(bem.Problem(V, T, k))
    Mp, _ = obem.bm_blocks(g, k, 1j / k)
    xs, xo = np.array([0.4, 1.9, -0.7]), np.array([-2.2, 0.3, 1.1])
    fields = {}
    for name, src, obs in (("s->o", xs, xo), ("o->s", xo, xs)):
        b = plan.point_source_rhs(src[None, :], [1.0])
        for mode in (0, 1):
            p, info = plan.solve(b, opts=bem.GmresOptions(tol=1e-10, mode=mode, inner_tol=1e-4))
            assert info["converged"]
            scat = plan.eval_field(p, None, obs[None, :]).cpu().numpy()[0]
            fields[(name, mode)] = solve.point_source_field(k, obs, src, [1.0])[0] + scat
        pr = np.linalg.solve(Mp, obem.point_source_rhs(g, k, 1j / k, src, [1.0]))
        Kh, _ = solve.represent_blocks(g, k, obs[None, :])
        ref = solve.point_source_field(k, obs, src, [1.0])[0] + (Kh @ pr)[0]
        for mode in (0, 1):
            e = abs(fields[(name, mode)] - ref) / abs(ref)
            _log(f"case: point source {name} mode {mode}: field {fields[(name, mode)]:.6f} "
                 f"vs dense oracle {ref:.6f} (rel {e:.1e})")
            assert e < 1e-6
    gap = abs(fields[("s->o", 0)] - fields[("o->s", 0)]) / abs(fields[("s->o", 0)])
    _log(f"  reciprocity gap {gap:.2e}")
    assert gap < 5e-3


def test_conventional_equation_resonance_against_burton_miller():
    """GMRES converges on both equations at every k (the plane-wave
    right-hand side stays consistent with the range), but near its discrete
    resonance the conventional equation's solution is polluted by the
    near-null mode, in a peak as narrow as the smallest singular value is
    small.  A golden-section search over k near pi for the largest error
    against the Mie series finds it; Burton-Miller's error there is the one
    it has away from the resonance."""
    bem = _lib()
    V, T = icosphere(3)
    g = obem.Geometry(V, T)
    d = np.array([0.0, 0.0, 1.0])
    cos_t = g.cen[:, 2] / np.linalg.norm(g.cen, axis=1)
    opts = bem.GmresOptions(tol=1e-10, restart=50, max_iter=800)

    def mie_error(k, alpha):
        plan = bem.Plan(bem.Problem(V, T, float(k), alpha=alpha, fmm_tol=1e-8))
        x, info = plan.solve(plan.plane_wave_rhs(d), opts=opts)
        assert info["converged"]
        return _rel(x.cpu().numpy(), mie.surface_pressure(float(k), cos_t))

    # bracket from a coarse scan, then golden section on the largest error
    ks = np.linspace(3.10, 3.22, 13)
    e = [mie_error(k, 0j) for k in ks]
    i = int(np.argmax(e))
    a, b = ks[max(i - 1, 0)], ks[min(i + 1, len(ks) - 1)]
    gr = (np.sqrt(5.0) - 1.0) / 2.0
    c, dd = b - gr * (b - a), a + gr * (b - a)
    fc, fd = mie_error(c, 0j), mie_error(dd, 0j)
    for _ in range(16):
        if fc > fd:
            b, dd, fd = dd, c, fc
            c = b - gr * (b - a)
            fc = mie_error(c, 0j)
        else:
            a, c, fc = c, dd, fd
            dd = a + gr * (b - a)
            fd = mie_error(dd, 0j)
    kpk = 0.5 * (a + b)
    e_cbie, e_bm = mie_error(kpk, 0j), mie_error(kpk, None)
    e_cbie_far, e_bm_far = mie_error(2.8, 0j), mie_error(2.8, None)
    _log(f"case: conventional equation resonance at k = {kpk:.6f} (pi = {np.pi:.6f}): "
         f"error vs Mie alpha=0 {e_cbie:.3e} (at k = 2.8: {e_cbie_far:.3e}), "
         f"Burton-Miller {e_bm:.3e} (at k = 2.8: {e_bm_far:.3e})")
    assert abs(kpk - np.pi) < 0.12
    assert e_cbie >= 5 * e_bm and e_cbie >= 5 * e_cbie_far
    assert e_bm <= 1.5 * e_bm_far
