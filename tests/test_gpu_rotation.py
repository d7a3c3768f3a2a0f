"""GPU tests of the rotation-based multipole-to-local translations
(point-and-shoot: rotate the multipole onto the translation axis, translate
along it, rotate back; bem_problem.m2l_rot).

* One mesh planned twice, with dense translations only (m2l_rot = 1) and
  with rotation-based ones on every level whose order allows (m2l_rot = 2):
  forward and adjoint products, float64 and float32, agree to rounding.
  Cases: calibrated orders with the input cut of the translations across
  three boxes, fixed orders without a cut, low orders, orders above 15 (the
  larger LDS tile) and at the kernel's maximum 23, and an order above it
  (levels stay dense).
* The rotation-based products against the oracle's exact rows on the
  20480-element sphere at k = 4, and the adjoint dot test.
* A batch of solves on a plan of two problems whose levels all use the
  rotation-based kernel (launches merging levels and problems) against the
  same systems solved one by one on a dense plan.
* The tuner (m2l_rot = 0) reports per level what it kept; its product
  matches the dense plan's, on the 20480-element sphere at k = 4 and on the
  81920-element sphere at k = 16 (higher orders; there also against the
  oracle's rows and columns).
"""
import numpy as np
import pytest

from oracle import bem as obem
from workloads import WORKLOADS, complex_normal, icosphere, unit_directions

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


# (name, icosphere level, k, order64, order32): order 0 = calibrated / rule
CASES = [
    ("ico4_k4_calibrated", 4, 4.0, 0, 0),
    ("ico4_k8_fixed_20_12", 4, 8.0, 20, 12),
    ("ico3_k2_fixed_5_3", 3, 2.0, 5, 3),
    ("ico3_k6_fixed_23_16", 3, 6.0, 23, 16),
    ("ico3_k6_fixed_26_8", 3, 6.0, 26, 8),
]


def _pair_of_plans(bem, lvl, k, o64, o32):
    V, T = icosphere(lvl)
    mk = lambda rot: bem.Plan(bem.Problem(V, T, k, order64=o64, order32=o32, m2l_rot=rot))
    return V, T, mk(1), mk(2)


@pytest.mark.parametrize("name,lvl,k,o64,o32", CASES)
def test_rotation_matches_dense(name, lvl, k, o64, o32):
    import torch
    bem = _lib()
    _log(f"case: {name}")
    V, T, dense, rot = _pair_of_plans(bem, lvl, k, o64, o32)
    sd, sr = dense.stats(), rot.stats()
    L = sr["leaf_level"]
    assert sd["order64"] == sr["order64"] and sd["order32"] == sr["order32"]
    assert sd["far_cut"] == sr["far_cut"]
    _log(f"  L={L} orders f64 {sr['order64'][2:]} f32 {sr['order32'][2:]} far_cut "
         f"{sr['far_cut']} rot f64 {sr['m2l_rot64'][2:]} f32 {sr['m2l_rot32'][2:]}")
    for l in range(2, L + 1):
        assert sd["m2l_rot64"][l] == 0 and sd["m2l_rot32"][l] == 0
        assert sr["m2l_rot64"][l] == (1 if sr["order64"][l] <= 23 else 0)
        assert sr["m2l_rot32"][l] == (1 if sr["order32"][l] <= 23 else 0)
    rng = np.random.default_rng(11 + lvl)
    n = len(T)
    p, q, yv = complex_normal(rng, n), complex_normal(rng, n), complex_normal(rng, n)
    for prec, bar in ((0, 1e-13), (1, 1e-6)):
        a = dense.matvec(torch.from_numpy(p), torch.from_numpy(q), prec=prec).cpu().numpy()
        b = rot.matvec(torch.from_numpy(p), torch.from_numpy(q), prec=prec).cpu().numpy()
        ua, wa = (t.cpu().numpy() for t in dense.matvec_adjoint(torch.from_numpy(yv), prec=prec))
        ub, wb = (t.cpu().numpy() for t in rot.matvec_adjoint(torch.from_numpy(yv), prec=prec))
        e, eu, ew = _rel(b, a), _rel(ub, ua), _rel(wb, wa)
        _log(f"  prec {prec}: forward {e:.2e}, adjoint u {eu:.2e} w {ew:.2e}")
        assert e < bar and eu < bar and ew < bar
        # the rotation-based adjoint is the adjoint of the rotation-based product
        lhs = np.vdot(yv, b)
        rhs = np.vdot(ub, p) + np.vdot(wb, q)
        dot = abs(lhs - rhs) / abs(lhs)
        _log(f"  prec {prec}: dot test {dot:.1e}")
        assert dot < (1e-12 if prec == 0 else 1e-5)
    dense.close()
    rot.close()


def test_rotation_against_oracle_rows_sphere20480():
    import torch
    bem = _lib()
    wl = WORKLOADS["sphere20480_k4"]
    V, T = wl.mesh_arrays()
    _log("case: sphere20480_k4 rotation-based M2L against oracle rows")
    plan = bem.Plan(bem.Problem(V, T, wl.k, leaf_cap=64, m2l_rot=2))
    st = plan.stats()
    L = st["leaf_level"]
    assert all(st["m2l_rot64"][l] == 1 and st["m2l_rot32"][l] == 1 for l in range(2, L + 1))
    g = obem.Geometry(V, T)
    rng = np.random.default_rng(wl.seed)
    p, q = complex_normal(rng, len(T)), complex_normal(rng, len(T))
    rows = np.sort(rng.choice(len(T), 64, replace=False))
    ref = obem.matvec(g, wl.k, wl.alpha, p, q, rows=rows, block=16)
    for prec, bar in ((0, 1e-6), (1, 1e-4)):
        y = plan.matvec(torch.from_numpy(p), torch.from_numpy(q), prec=prec).cpu().numpy()
        e = _rel(y[rows], ref)
        _log(f"  prec {prec}: sampled rel-L2 err {e:.3e}")
        assert e < bar
    yv = complex_normal(rng, len(T))
    cols = np.sort(rng.choice(len(T), 24, replace=False))
    u, w = plan.matvec_adjoint(torch.from_numpy(yv))
    uref, wref = obem.matvec_adjoint(g, wl.k, wl.alpha, yv, cols=cols, block=8)
    eu, ew = _rel(u.cpu().numpy()[cols], uref), _rel(w.cpu().numpy()[cols], wref)
    _log(f"  adjoint columns: u {eu:.3e} w {ew:.3e}")
    assert eu < 1e-6 and ew < 1e-6
    plan.close()


def test_rotation_batch_of_solves():
    bem = _lib()
    meshes = [(icosphere(3), 3.0), (icosphere(4), 5.0)]
    probs = lambda rot: [bem.Problem(V, T, k, m2l_rot=rot) for (V, T), k in meshes]
    _log("case: batch of 6 solves over two problems, rotation-based M2L")
    rot = bem.Plan(probs(2))
    dense = bem.Plan(probs(1))
    rng = np.random.default_rng(5)
    systems = []
    for i in range(6):
        pr = i % 2
        d = unit_directions(rng, 1)[0]
        systems.append(dict(prob=pr, b=rot.plane_wave_rhs(d, prob=pr), adjoint=(i >= 4)))
    opts = bem.GmresOptions(tol=1e-9, restart=60, mode=0)
    xs, infos = rot.solve_batch(systems, opts)
    for i, (s, x, inf) in enumerate(zip(systems, xs, infos)):
        assert inf["converged"], inf
        ref, _ = dense.solve(s["b"], adjoint=s["adjoint"], opts=opts, prob=s["prob"])
        e = _rel(x.cpu().numpy(), ref.cpu().numpy())
        _log(f"  system {i} (problem {s['prob']}, adjoint {s['adjoint']}): "
             f"{inf['iterations']} its, vs dense plan {e:.2e}")
        assert e < 1e-7
    rot.close()
    dense.close()


def test_tuner_choice_matches_dense():
    import torch
    bem = _lib()
    wl = WORKLOADS["sphere20480_k4"]
    V, T = wl.mesh_arrays()
    _log("case: sphere20480_k4 tuned M2L variant per level")
    tuned = bem.Plan(bem.Problem(V, T, wl.k, leaf_cap=64))
    dense = bem.Plan(bem.Problem(V, T, wl.k, leaf_cap=64, m2l_rot=1))
    st = tuned.stats()
    _log(f"  kept rotation-based levels: f64 {st['m2l_rot64'][2:]} f32 {st['m2l_rot32'][2:]}")
    assert all(v in (0, 1) for v in st["m2l_rot64"] + st["m2l_rot32"])
    rng = np.random.default_rng(3)
    p, q = complex_normal(rng, len(T)), complex_normal(rng, len(T))
    for prec, bar in ((0, 1e-11), (1, 2e-5)):
        a = dense.matvec(torch.from_numpy(p), torch.from_numpy(q), prec=prec).cpu().numpy()
        b = tuned.matvec(torch.from_numpy(p), torch.from_numpy(q), prec=prec).cpu().numpy()
        assert _rel(b, a) < bar
    tuned.close()
    dense.close()


def test_bad_rotation_request_is_rejected():
    bem = _lib()
    V, T = icosphere(2)
    with pytest.raises(bem.BemError):
        bem.Plan(bem.Problem(V, T, 2.0, m2l_rot=3))


def test_larger_kd_sphere81920_k16():
    """The 81920-element sphere at k = 16 (twice the benchmark's k h): the
    orders rise, the tuner keeps the rotation-based translations where they
    are faster; the product matches the oracle's rows and the dense-only
    plan's product, the adjoint the oracle's columns."""
    import torch
    bem = _lib()
    wl = WORKLOADS["sphere81920_k16"]
    V, T = wl.mesh_arrays()
    _log("case: sphere81920_k16 tuned plan against the oracle and a dense-only plan")
    tuned = bem.Plan(bem.Problem(V, T, wl.k, leaf_cap=64))
    st = tuned.stats()
    _log(f"  orders f64 {st['order64'][2:]} f32 {st['order32'][2:]}, far cut {st['far_cut']}, "
         f"rotation-based f64 {st['m2l_rot64'][2:]} f32 {st['m2l_rot32'][2:]}")
    g = obem.Geometry(V, T)
    rng = np.random.default_rng(wl.seed)
    p, q = complex_normal(rng, len(T)), complex_normal(rng, len(T))
    rows = np.sort(rng.choice(len(T), 32, replace=False))
    ref = obem.matvec(g, wl.k, wl.alpha, p, q, rows=rows, block=16)
    ys = {}
    for prec, bar in ((0, 1e-6), (1, 1e-4)):
        y = tuned.matvec(torch.from_numpy(p), torch.from_numpy(q), prec=prec).cpu().numpy()
        ys[prec] = y
        e = _rel(y[rows], ref)
        _log(f"  prec {prec}: sampled rel-L2 err {e:.3e}")
        assert e < bar
    yv = complex_normal(rng, len(T))
    cols = np.sort(rng.choice(len(T), 16, replace=False))
    u, w = tuned.matvec_adjoint(torch.from_numpy(yv))
    uref, wref = obem.matvec_adjoint(g, wl.k, wl.alpha, yv, cols=cols, block=8)
    eu, ew = _rel(u.cpu().numpy()[cols], uref), _rel(w.cpu().numpy()[cols], wref)
    _log(f"  adjoint columns: u {eu:.3e} w {ew:.3e}")
    assert eu < 1e-6 and ew < 1e-6
    tuned.close()
    dense = bem.Plan(bem.Problem(V, T, wl.k, leaf_cap=64, m2l_rot=1))
    for prec, bar in ((0, 1e-13), (1, 1e-6)):
        y = dense.matvec(torch.from_numpy(p), torch.from_numpy(q), prec=prec).cpu().numpy()
        e = _rel(ys[prec], y)
        _log(f"  prec {prec}: tuned vs dense-only plan {e:.2e}")
        assert e < bar
    dense.close()
