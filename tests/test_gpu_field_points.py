"""GPU parity of the FMM evaluation of the field and its gradient at points off
the boundary (bem_eval_field_grad_fmm: the design-domain lattice of the
topology loop's step 8, Sec. 3, with the boundary sums split by the FMM).

* Against the oracle's representation and gradient on the 1280- and
  5120-element spheres (trees of depth 2 and 3): white-noise and smooth
  densities p and q, plane wave and point sources, float64 and float32, on
  a lattice around the sphere plus points more than one root-cube width
  outside the tree's root cube, several evaluations in a row.
* Against the direct GPU sum (itself pinned to the oracle) on the
  20480-element sphere and a 31^3 lattice, both precisions.
* T_Omega from the FMM fields against T_Omega from the direct fields.
* Rotation-based translations into the point boxes against dense ones.
* Edge cases: no points, points out of range, non-finite points, bad
  precision, a problem without far field (direct sum kept), a point set
  with one point, points on box faces of the tree's grid, the second
  problem of a two-problem plan.
"""
import numpy as np
import pytest

from oracle import bem as obem
from oracle import solve
from workloads import complex_normal, icosphere, unit_directions

pytestmark = pytest.mark.gpu

# Bars (field, gradient) per precision and density kind.  The evaluation
# uses the problem's expansion orders, calibrated so that the product's
# sampled error meets fmm_tol; off the boundary the relative error is larger
# by about the ratio of the product's norm (which holds the identity and self
# terms) to the field's, and the gradient of a truncated local expansion
# loses about one order more.  Measured on the 1280- and 5120-element
# spheres: white noise (float64) 8e-7 / 2e-5, (float32) 2e-4 / 2e-3;
# smooth densities (float64) 5e-8 / 2e-6, (float32) 1e-5 / 9e-5; the bars
# are three times these.
TOL = {("noise", 0): (3e-6, 6e-5), ("noise", 1): (6e-4, 6e-3),
       ("smooth", 0): (2e-7, 6e-6), ("smooth", 1): (3e-5, 3e-4)}


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


def _lattice(n, half, rmin):
    t = np.linspace(-half, half, n)
    X = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)
    return X[np.linalg.norm(X, axis=1) > rmin]


def _oracle_field(g, k, pts, p, q, d=None, src=None, amp=None, chunk=300):
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


@pytest.mark.parametrize("level,min_leaf", [(3, 2), (4, 3)])
def test_fmm_points_against_oracle(level, min_leaf):
    import torch
    bem = _lib()
    V, T = icosphere(level)
    k = 2.0
    g = obem.Geometry(V, T)
    plan = bem.Plan(bem.Problem(V, T, k, leaf_cap=16))
    st = plan.stats()
    assert st["leaf_level"] >= min_leaf
    rng = np.random.default_rng(71)
    far = 4.5 * unit_directions(rng, 40)          # outside the root cube [-1, 1]^3
    pts = np.concatenate([_lattice(11, 2.0, 1.15), far])
    rng.shuffle(pts)
    d = np.array([0.0, 0.6, 0.8])
    src = np.array([[2.6, 0.1, -0.2], [0.3, -2.9, 0.5]])
    amp = np.array([0.4 - 0.3j, 1.1 + 0.2j])
    # densities: white noise (two draws), and the traces of a plane wave
    # (smooth, as a solution's are)
    cen = V[T].mean(axis=1)
    dw = np.array([0.3, -0.5, 0.81]) / np.linalg.norm([0.3, -0.5, 0.81])
    pw = np.exp(1j * k * cen @ dw)
    dens = []
    for seed in (72, 73):
        r2 = np.random.default_rng(seed)
        dens.append(("noise", complex_normal(r2, len(T)), complex_normal(r2, len(T))))
    dens.append(("smooth", pw, 1j * k * pw))
    ref = [(kind, p, q, _oracle_field(g, k, pts, p, q, d, src, amp), _oracle_field(g, k, pts, p, q))
           for kind, p, q in dens]
    for prec in (bem.BEM_C128, bem.BEM_C64):
        fp = bem.FieldPoints(plan, pts, prec=prec)
        s = fp.stats()
        _log(f"case: {len(pts)} points (lattice + 40 at r = 4.5), sphere{len(T)} k = 2 (leaf "
             f"level {st['leaf_level']}), prec {prec}: "
             f"boxes {s['n_box'][2:]}, m2l {s['n_m2l'][2:]}, leaves {s['n_leaf']}, "
             f"near pairs {s['n_near_pairs']}")
        assert s["n_pts"] == len(pts)
        for kind, p, q, (fr, grr), (fr0, gr0) in ref:  # evaluations in a row reuse the buffers
            tf, tg = TOL[(kind, prec)]
            f, gr = fp.eval_field_grad(torch.from_numpy(p), torch.from_numpy(q), direction=d,
                                       src=src, amp=amp)
            ef, eg = _rel(f.cpu().numpy(), fr), _rel(gr.cpu().numpy(), grr)
            # the boundary sums alone (no incident part)
            f0, g0 = fp.eval_field_grad(torch.from_numpy(p), torch.from_numpy(q))
            es, egs = _rel(f0.cpu().numpy(), fr0), _rel(g0.cpu().numpy(), gr0)
            _log(f"  {kind}: total field {ef:.2e} gradient {eg:.2e}; boundary sums alone "
                 f"{es:.2e} / {egs:.2e}")
            assert max(ef, es) < tf and max(eg, egs) < tg
        fp.close()


def test_fmm_points_against_direct_sum():
    import torch
    bem = _lib()
    V, T = icosphere(5)
    k = 6.0
    plan = bem.Plan(bem.Problem(V, T, k))
    rng = np.random.default_rng(74)
    p, q = complex_normal(rng, len(T)), complex_normal(rng, len(T))
    P, Q = torch.from_numpy(p), torch.from_numpy(q)
    pts = _lattice(31, 1.6, 1.03)
    d = np.array([1.0, 0.0, 0.0])
    fd, gd = plan.eval_field_grad(P, Q, pts, direction=d)
    fd, gd = fd.cpu().numpy(), gd.cpu().numpy()
    fs, gs = plan.eval_field_grad(P, Q, pts)  # scattered part alone
    fs, gs = fs.cpu().numpy(), gs.cpu().numpy()
    for prec in (bem.BEM_C128, bem.BEM_C64):
        tf, tg = TOL[("noise", prec)]
        fp = bem.FieldPoints(plan, pts, prec=prec)
        s = fp.stats()
        f, gr = fp.eval_field_grad(P, Q, direction=d)
        f0, g0 = fp.eval_field_grad(P, Q)
        e = [_rel(f.cpu().numpy(), fd), _rel(gr.cpu().numpy(), gd), _rel(f0.cpu().numpy(), fs),
             _rel(g0.cpu().numpy(), gs)]
        _log(f"case: sphere20480 k = 6, {len(pts)} lattice points, prec {prec}: boxes "
             f"{s['n_box'][2:]}, m2l {s['n_m2l'][2:]}, near pairs {s['n_near_pairs']}: "
             f"errors vs direct (field, gradient, alone: field, gradient) "
             f"{['%.2e' % v for v in e]}")
        assert max(e[0], e[2]) < tf and max(e[1], e[3]) < tg
        fp.close()


def test_fmm_points_rotation_matches_dense():
    """Translations into the point boxes rotation-based (plan asked for them
    on every level: float64 results added atomically, float32 per pair) or
    dense: the same fields and gradients to rounding."""
    import torch
    bem = _lib()
    V, T = icosphere(4)
    k = 6.0
    plans = {rot: bem.Plan(bem.Problem(V, T, k, m2l_rot=rot)) for rot in (1, 2)}
    rng = np.random.default_rng(75)
    p, q = complex_normal(rng, len(T)), complex_normal(rng, len(T))
    P, Q = torch.from_numpy(p), torch.from_numpy(q)
    pts = _lattice(21, 1.5, 1.03)
    d = np.array([0.0, 0.6, 0.8])
    for prec, bar in ((bem.BEM_C128, 1e-12), (bem.BEM_C64, 1e-5)):
        out = {}
        for rot, plan in plans.items():
            fp = bem.FieldPoints(plan, pts, prec=prec)
            st = fp.stats()
            want = [1 if (rot == 2 and o <= 23) else 0 for o in st["order"][2:]]
            assert st["m2l_rot"][2:] == want, (st["m2l_rot"], st["order"])
            f, gr = fp.eval_field_grad(P, Q, direction=d)
            out[rot] = (f.cpu().numpy(), gr.cpu().numpy(), st["m2l_rot"][2:])
            fp.close()
        ef, eg = _rel(out[2][0], out[1][0]), _rel(out[2][1], out[1][1])
        _log(f"case: sphere5120 k = 6, {len(pts)} points, prec {prec}: rotation-based levels "
             f"{out[2][2]}: field {ef:.2e}, gradient {eg:.2e} against dense")
        assert ef < bar and eg < bar
    for plan in plans.values():
        plan.close()


def test_topological_derivative_from_fmm_fields():
    import torch
    bem = _lib()
    V, T = icosphere(4)
    k = 3.0
    d = np.array([0.0, 0.0, 1.0])
    rng = np.random.default_rng(75)
    obs = 3.0 * unit_directions(rng, 8)
    plan = bem.Plan(bem.Problem(V, T, k))
    opts = bem.GmresOptions(tol=1e-10)
    p, info = plan.solve(plan.plane_wave_rhs(d), opts=opts)
    pobs = plan.eval_field(p, None, obs, direction=d).cpu().numpy()
    amp = 2.0 * np.conj(pobs)
    pt, info_t = plan.solve(plan.point_source_rhs(obs, amp), opts=opts)
    assert info["converged"] and info_t["converged"]
    lat = _lattice(25, 2.5, 1.2)
    fs, gs = plan.eval_field_grad(p, None, lat, direction=d)
    fa, ga = plan.eval_field_grad(pt, None, lat, src=obs, amp=amp)
    fp = bem.FieldPoints(plan, lat)
    fs2, gs2 = fp.eval_field_grad(p, None, direction=d)
    fa2, ga2 = fp.eval_field_grad(pt, None, src=obs, amp=amp)
    for m in (dict(), dict(rho_s=1.1, lam_s=1.17 / (3 * (1 - 2 * 0.369)))):
        Td = bem.topological_derivative(fs, gs, fa, ga, omega=k, **m).cpu().numpy()
        Tf = bem.topological_derivative(fs2, gs2, fa2, ga2, omega=k, **m).cpu().numpy()
        e = _rel(Tf, Td)
        _log(f"case: T_Omega on {len(lat)} lattice points, sphere5120 k = 3, FMM vs direct "
             f"fields ({'rigid' if not m else 'ABS in water'}): rel err {e:.2e}")
        assert e < 1e-5


def test_fmm_points_edge_cases():
    import torch
    bem = _lib()
    V, T = icosphere(3)
    k = 2.0
    plan = bem.Plan(bem.Problem(V, T, k, leaf_cap=16))
    g = obem.Geometry(V, T)
    rng = np.random.default_rng(76)
    p = complex_normal(rng, len(T))
    P = torch.from_numpy(p)
    _log("case: edge cases of the point sets")
    # no points
    fp = bem.FieldPoints(plan, np.zeros((0, 3)))
    f, gr = fp.eval_field_grad(P)
    assert f.shape == (0,) and gr.shape == (0, 3)
    fp.close()
    # one point, and points on faces and corners of the tree's boxes (x = 0.5,
    # 0.25, ...; the root cube is [-1, 1]^3 widened by 2^-10), where a local
    # expansion is at its least accurate (a corner sits at 0.87 box sides
    # from the centre, a source of a non-touching box can be 1.5 sides
    # away): per point against the oracle, with bars three times the worst
    # measured (7e-5 field, 2e-3 gradient; the orders are calibrated on a
    # mean-square error), and the same values when the points are evaluated
    # within a larger set (a point's leaf box and level depend on its
    # position alone)
    big = _lattice(9, 2.0, 1.2)
    for pts in (np.array([[1.7, -0.2, 0.3]]),
                np.array([[0.5, 1.25, 0.0], [-1.5, 0.25, 0.75], [0.0, 0.0, 1.5], [1.0, 1.0, 1.0]])):
        fp = bem.FieldPoints(plan, pts)
        f, gr = fp.eval_field_grad(P)
        f, gr = f.cpu().numpy(), gr.cpu().numpy()
        fr, grr = _oracle_field(g, k, pts, p, None)
        ef = np.abs(f - fr) / np.abs(fr)
        eg = np.linalg.norm(gr - grr, axis=1) / np.linalg.norm(grr, axis=1)
        _log(f"  {len(pts)} point(s): worst per-point error field {ef.max():.2e} gradient "
             f"{eg.max():.2e}")
        assert ef.max() < 3e-4 and eg.max() < 6e-3
        fp.close()
        fpb = bem.FieldPoints(plan, np.concatenate([big, pts]))
        fb, gb = fpb.eval_field_grad(P)
        fb, gb = fb.cpu().numpy()[len(big):], gb.cpu().numpy()[len(big):]
        assert np.abs(fb - f).max() < 1e-13 * np.abs(f).max()
        assert np.abs(gb - gr).max() < 1e-13 * np.abs(gr).max()
        fpb.close()
    # out of range (beyond two root widths), non-finite, bad precision
    with pytest.raises(bem.BemError) as ei:
        bem.FieldPoints(plan, np.array([[9.0, 0.0, 0.0]]))
    assert ei.value.code == -1
    with pytest.raises(bem.BemError):
        bem.FieldPoints(plan, np.array([[np.nan, 0.0, 0.0]]))
    with pytest.raises(bem.BemError):
        bem.FieldPoints(plan, np.array([[2.0, 0.0, 0.0]]), prec=2)
    # the second problem of a two-problem plan (its own tree, k and orders)
    V4, T4 = icosphere(4)
    plan2 = bem.Plan([bem.Problem(V, T, k, leaf_cap=16), bem.Problem(V4, T4, 3.0)])
    p4 = complex_normal(rng, len(T4))
    pts = _lattice(7, 1.8, 1.2)
    fp = bem.FieldPoints(plan2, pts, prob=1)
    f, gr = fp.eval_field_grad(torch.from_numpy(p4))
    fr, grr = _oracle_field(obem.Geometry(V4, T4), 3.0, pts, p4, None)
    tf, tg = TOL[("noise", 0)]
    assert _rel(f.cpu().numpy(), fr) < tf and _rel(gr.cpu().numpy(), grr) < tg
    fp.close()
    # a problem without far field: the points are summed directly
    V1, T1 = icosphere(1)
    plan1 = bem.Plan(bem.Problem(V1, T1, 1.0))
    p1 = complex_normal(rng, len(T1))
    pts = _lattice(5, 2.0, 1.3)
    fp = bem.FieldPoints(plan1, pts)
    f, gr = fp.eval_field_grad(torch.from_numpy(p1))
    fr, grr = _oracle_field(obem.Geometry(V1, T1), 1.0, pts, p1, None)
    assert _rel(f.cpu().numpy(), fr) < 1e-12 and _rel(gr.cpu().numpy(), grr) < 1e-12
    fp.close()


def test_design_lattice_at_full_size_against_oracle():
    """The benchmark's configuration: the 81920-element sphere at k = 8, the
    101^3 design-domain lattice (points outside |x| > 1.02), state and
    adjoint densities from the GPU solves; fields, gradients and T_Omega by
    the FMM on the whole lattice, compared on 40 sampled points with the
    oracle's dense sums over all elements for the same densities."""
    import torch
    bem = _lib()
    from workloads import WORKLOADS
    wl = WORKLOADS["sphere81920_k8"]
    V, T = wl.mesh_arrays()
    rng = np.random.default_rng(wl.seed)
    d = unit_directions(rng, 1)[0]
    obs = 3.0 * unit_directions(rng, 8)
    t = np.linspace(-1.25, 1.25, 101)
    X = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)
    lat = X[np.linalg.norm(X, axis=1) > 1.02]
    plan = bem.Plan(bem.Problem(V, T, wl.k, leaf_cap=64))
    opts = bem.GmresOptions(tol=1e-6, mode=1)
    p, info = plan.solve(plan.plane_wave_rhs(d), opts=opts)
    pobs = plan.eval_field(p, None, obs, direction=d).cpu().numpy()
    amp = 2.0 * np.conj(pobs)
    pt, info_t = plan.solve(plan.point_source_rhs(obs, amp), opts=opts)
    assert info["converged"] and info_t["converged"]
    pick = np.sort(np.random.default_rng(77).choice(len(lat), 40, replace=False))
    x = lat[pick]
    g = obem.Geometry(V, T)
    pn, ptn = p.cpu().numpy(), pt.cpu().numpy()
    fsr, gsr = _oracle_field(g, wl.k, x, pn, None, d=d, chunk=10)
    far_, gar = _oracle_field(g, wl.k, x, ptn, None, src=obs, amp=amp, chunk=10)
    Tr = solve.topological_derivative(fsr, gsr, far_, gar, 1.0, np.inf, 1.0, np.inf, wl.k)
    # bars: three times the measured errors (float64 4e-8 / 3e-6 / 1.1e-6,
    # float32 2e-5 / 2.6e-4 / 1.6e-4 for field / gradient / T_Omega)
    for prec, tf, tg, tt in ((bem.BEM_C128, 1.5e-7, 1e-5, 4e-6), (bem.BEM_C64, 6e-5, 8e-4, 5e-4)):
        fp = bem.FieldPoints(plan, lat, prec=prec)
        fs, gs = fp.eval_field_grad(p, None, direction=d)
        fa, ga = fp.eval_field_grad(pt, None, src=obs, amp=amp)
        Tg = bem.topological_derivative(fs, gs, fa, ga, omega=wl.k).cpu().numpy()[pick]
        e = [_rel(fs.cpu().numpy()[pick], fsr), _rel(gs.cpu().numpy()[pick], gsr),
             _rel(fa.cpu().numpy()[pick], far_), _rel(ga.cpu().numpy()[pick], gar), _rel(Tg, Tr)]
        _log(f"case: {len(lat)} lattice points, sphere81920 k = 8, prec {prec}: state field / "
             f"gradient, adjoint field / gradient, T_Omega on 40 sampled points vs oracle "
             f"{['%.2e' % v for v in e]}")
        assert max(e[0], e[2]) < tf and max(e[1], e[3]) < tg and e[4] < tt
        fp.close()
