"""GPU parity of the off-surface field, its gradient and the topological
derivative T_Omega (Eq. danseitpoderi) on a design-domain lattice.

* bem_eval_field_grad against the oracle's representation and its gradient
  (white-noise p and q, plane-wave and point-source incident fields).
* The whole evaluation of the paper's solver step 8 on a 21^3 lattice around
  the 1280-element sphere: state solve (plane wave), J over 8 observation
  points, adjoint solve with point sources of intensity 2 conj(p) there,
  both fields and their gradients at the lattice points outside the
  scatterer, T_Omega for the sound-hard limit and for an ABS-like solid in
  water (the paper's material pair of Sec. 3.2), against the oracle's dense
  solves and fields on 600 sampled lattice points.
"""
import numpy as np
import pytest

from oracle import bem as obem
from oracle import solve
from workloads import complex_normal, icosphere, unit_directions

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


def _oracle_field(g, k, pts, p, q, d=None, src=None, amp=None, chunk=300):
    """Total field and gradient by the oracle, in chunks of points."""
    f = np.zeros(len(pts), dtype=np.complex128)
    gr = np.zeros((len(pts), 3), dtype=np.complex128)
    for a in range(0, len(pts), chunk):
        x = pts[a:a + chunk]
        Kh, Sh = solve.represent_blocks(g, k, x)
        f[a:a + chunk] = Kh @ p - (Sh @ q if q is not None else 0)
        gr[a:a + chunk] = solve.represent_grad(g, k, x, p, q)
        if d is not None:
            inc = np.exp(1j * k * (x @ d))
            f[a:a + chunk] += inc
            gr[a:a + chunk] += (1j * k * inc)[:, None] * d[None, :]
        if src is not None:
            f[a:a + chunk] += solve.point_source_field(k, x, src, amp)
            gr[a:a + chunk] += solve.point_source_grad(k, x, src, amp)
    return f, gr


def _lattice(n, half, rmin):
    t = np.linspace(-half, half, n)
    X = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)
    return X[np.linalg.norm(X, axis=1) > rmin]


def test_field_gradient_against_oracle():
    import torch
    bem = _lib()
    V, T = icosphere(3)
    k = 2.0
    g = obem.Geometry(V, T)
    plan = bem.Plan(bem.Problem(V, T, k))
    rng = np.random.default_rng(61)
    p, q = complex_normal(rng, len(T)), complex_normal(rng, len(T))
    pts = _lattice(9, 2.0, 1.3)
    d = np.array([0.6, 0.0, -0.8])
    src = np.array([[2.5, 0.2, 0.1], [-0.3, -2.8, 0.4]])
    amp = np.array([0.7 + 0.1j, -0.2 + 0.9j])
    f, gr = plan.eval_field_grad(torch.from_numpy(p), torch.from_numpy(q), pts, direction=d,
                                 src=src, amp=amp)
    fr, grr = _oracle_field(g, k, pts, p, q, d, src, amp)
    ef, eg = _rel(f.cpu().numpy(), fr), _rel(gr.cpu().numpy(), grr)
    _log(f"case: field and gradient at {len(pts)} points: rel err {ef:.2e} / {eg:.2e}")
    assert ef < 1e-12 and eg < 1e-12
    # without incident fields and without q: the same pieces
    f0, g0 = plan.eval_field_grad(torch.from_numpy(p), None, pts)
    fr0, gr0 = _oracle_field(g, k, pts, p, None)
    assert _rel(f0.cpu().numpy(), fr0) < 1e-12 and _rel(g0.cpu().numpy(), gr0) < 1e-12


def test_topological_derivative_on_a_lattice():
    import torch
    bem = _lib()
    V, T = icosphere(3)
    k = 2.0
    g = obem.Geometry(V, T)
    d = np.array([0.0, 0.0, 1.0])
    rng = np.random.default_rng(62)
    obs = 3.0 * unit_directions(rng, 8)
    plan = bem.Plan(bem.Problem(V, T, k, fmm_tol=1e-9))
    opts = bem.GmresOptions(tol=1e-11)
    # state
    p, info = plan.solve(plan.plane_wave_rhs(d), opts=opts)
    assert info["converged"]
    pobs = plan.eval_field(p, None, obs, direction=d).cpu().numpy()
    J = float(np.sum(np.abs(pobs) ** 2))
    amp = 2.0 * np.conj(pobs)
    # adjoint: the field radiated by sources of intensity dJ/dp at the points
    pt, info_t = plan.solve(plan.point_source_rhs(obs, amp), opts=opts)
    assert info_t["converged"]
    lat = _lattice(21, 2.5, 1.25)
    fs, gs = plan.eval_field_grad(p, None, lat, direction=d)
    fa, ga = plan.eval_field_grad(pt, None, lat, src=obs, amp=amp)
    mats = {"rigid": dict(), "abs_in_water": dict(rho_s=1.1, lam_s=1.17 / (3 * (1 - 2 * 0.369)))}
    Tg = {name: bem.topological_derivative(fs, gs, fa, ga, omega=k, **m).cpu().numpy()
          for name, m in mats.items()}
    # oracle: dense solves, fields on sampled lattice points
    Mp, _ = obem.bm_blocks(g, k, 1j / k)
    pr = np.linalg.solve(Mp, obem.plane_wave_rhs(g, k, 1j / k, d))
    pobs_r = solve.represent(g, k, obs, pr, np.zeros_like(pr), d)
    Jr = float(np.sum(np.abs(pobs_r) ** 2))
    amp_r = 2.0 * np.conj(pobs_r)
    ptr = np.linalg.solve(Mp, obem.point_source_rhs(g, k, 1j / k, obs, amp_r))
    pick = np.sort(rng.choice(len(lat), 600, replace=False))
    x = lat[pick]
    fsr, gsr = _oracle_field(g, k, x, pr, None, d=d)
    far, gar = _oracle_field(g, k, x, ptr, None, src=obs, amp=amp_r)
    _log(f"case: T_Omega on {len(lat)} lattice points (21^3 outside r = 1.25): J {J:.8e} "
         f"(oracle {Jr:.8e})")
    assert abs(J - Jr) < 1e-8 * Jr
    for name, m in mats.items():
        rho_s, lam_s = m.get("rho_s", np.inf), m.get("lam_s", np.inf)
        Tr = solve.topological_derivative(fsr, gsr, far, gar, 1.0, rho_s, 1.0, lam_s, k)
        e = _rel(Tg[name][pick], Tr)
        _log(f"  {name}: T in [{Tg[name].min():.4e}, {Tg[name].max():.4e}], rel err on 600 "
             f"sampled points {e:.2e}")
        assert e < 1e-7
        assert Tg[name].min() < 0 < Tg[name].max()
