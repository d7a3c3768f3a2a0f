"""GPU parity of operator variants and product paths the default workloads
do not reach, each against the CPU oracle with the same coupling.

* alpha = 0 (the paper's own conventional equation, I/2 - D with S on q)
  and alpha = 0.3 + 0.5i (a coupling with a real part: the near-field
  kernels' general-alpha instantiations): forward products with and
  without q, adjoint products with and without w, and the adjoint dot
  test, in float64 and float32, on the 1280-element sphere.
* Products with q = 0 and adjoint products without w (the rigid paths,
  with their own near-field, P2M and finish variants) under every stream
  schedule and direct-translation depth the tuner can pick, both
  precisions.
* A batch of 12 rigid systems (state and adjoint) on three problems against
  dense LU solves.
"""
import numpy as np
import pytest

from oracle import bem as obem
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


_DENSE = {}


def _dense(alpha):
    if alpha not in _DENSE:
        V, T = icosphere(3)
        g = obem.Geometry(V, T)
        _DENSE[alpha] = (V, T, g, obem.bm_blocks(g, 1.0, alpha))
    return _DENSE[alpha]


@pytest.mark.parametrize("alpha", [0j, 0.3 + 0.5j])
def test_alpha_variants_against_oracle(alpha):
    import torch
    bem = _lib()
    V, T, g, (Mp, Mq) = _dense(alpha)
    n = len(T)
    _log(f"case: alpha = {alpha} sphere1280, forward/adjoint/dot, float64 and float32")
    plan = bem.Plan(bem.Problem(V, T, 1.0, alpha=alpha, leaf_cap=32))
    rng = np.random.default_rng(31)
    p, q, yv = complex_normal(rng, n), complex_normal(rng, n), complex_normal(rng, n)
    P, Q, Y = (torch.from_numpy(v) for v in (p, q, yv))
    ref_y, ref_y0 = Mp @ p + Mq @ q, Mp @ p
    ref_u, ref_w = Mp.conj().T @ yv, Mq.conj().T @ yv
    for prec, tol in ((bem.BEM_C128, 1e-6), (bem.BEM_C64, 1e-4)):
        y = plan.matvec(P, Q, prec=prec).cpu().numpy()
        y0 = plan.matvec(P, None, prec=prec).cpu().numpy()
        u, w = plan.matvec_adjoint(Y, prec=prec)
        u, w = u.cpu().numpy(), w.cpu().numpy()
        u0, w0 = plan.matvec_adjoint(Y, prec=prec, want_w=False)
        assert w0 is None
        u0 = u0.cpu().numpy()
        errs = dict(y=_rel(y, ref_y), y_q0=_rel(y0, ref_y0), u=_rel(u, ref_u), w=_rel(w, ref_w),
                    u_w0=_rel(u0, ref_u))
        dot = abs(np.vdot(yv, y) - (np.vdot(u, p) + np.vdot(w, q))) / abs(np.vdot(yv, y))
        _log(f"  prec {prec}: " + " ".join(f"{k} {v:.2e}" for k, v in errs.items())
             + f" dot {dot:.2e}")
        for k_, v in errs.items():
            assert v < tol, (k_, v)
        assert dot < (1e-12 if prec == bem.BEM_C128 else 1e-5)
    if alpha == 0j:
        # the conventional operator: the identity part is exactly I/2 on p and
        # nothing on q (alpha/2 = 0): the q-only product is S q alone
        S = obem.assemble_block(g, 1.0)[0]
        yq = plan.matvec(torch.zeros(n, dtype=torch.complex128), Q).cpu().numpy()
        assert _rel(yq, S @ q) < 1e-6


def test_rigid_paths_under_every_schedule():
    """q = NULL forward and w = NULL adjoint products, both precisions, every
    stream schedule (and the direct translations where built), against the
    oracle's Mp p and Mp^H y."""
    import torch
    bem = _lib()
    V, T, g, (Mp, Mq) = _dense(1j)
    n = len(T)
    plan = bem.Plan(bem.Problem(V, T, 1.0, leaf_cap=16))
    st = plan.stats()
    _log(f"case: rigid paths, leaf level {st['leaf_level']}, schedules 0..5")
    assert st["n_m2l"][st["leaf_level"]] > 0
    rng = np.random.default_rng(37)
    p, yv = complex_normal(rng, n), complex_normal(rng, n)
    P, Y = torch.from_numpy(p), torch.from_numpy(yv)
    ref_y, ref_u = Mp @ p, Mp.conj().T @ yv
    for prec, tol in ((bem.BEM_C128, 1e-6), (bem.BEM_C64, 1e-4)):
        for sched in range(6):
            for depth in (0, 1):
                try:
                    plan.set_tuning(prec, schedule=sched, direct_depth=depth)
                except RuntimeError:
                    continue  # no direct translations built at this depth
                y = plan.matvec(P, None, prec=prec).cpu().numpy()
                u, w = plan.matvec_adjoint(Y, prec=prec, want_w=False)
                ey, eu = _rel(y, ref_y), _rel(u.cpu().numpy(), ref_u)
                _log(f"  prec {prec} schedule {sched} depth {depth}: y {ey:.2e} u {eu:.2e}")
                assert ey < tol and eu < tol
        plan.set_tuning(prec, schedule=0, direct_depth=0)


def test_rigid_batch_against_dense_lu():
    import torch
    bem = _lib()
    meshes = [(icosphere(1), 2.0, 64), (icosphere(2), 3.0, 8), (icosphere(3), 1.0, 32)]
    plan = bem.Plan([bem.Problem(V, T, k, leaf_cap=cap) for (V, T), k, cap in meshes])
    rng = np.random.default_rng(41)
    systems, answers = [], []
    for prob, ((V, T), k, _) in enumerate(meshes):
        g = obem.Geometry(V, T)
        Mp, _ = obem.bm_blocks(g, k, 1j / k)
        for d in unit_directions(rng, 2):
            b = obem.plane_wave_rhs(g, k, 1j / k, d)
            systems.append(dict(prob=prob, b=torch.from_numpy(b)))
            answers.append(np.linalg.solve(Mp, b))
        for _ in range(2):
            c = complex_normal(rng, len(T))
            systems.append(dict(prob=prob, b=torch.from_numpy(c), adjoint=True))
            answers.append(np.linalg.solve(Mp.conj().T, c))
    _log(f"case: rigid batch of {len(systems)} systems (state and adjoint, 3 problems)")
    for mode in (0, 1):
        xs, infos = plan.solve_batch(systems, bem.GmresOptions(tol=1e-9, restart=40, mode=mode,
                                                               inner_tol=1e-4))
        for i, (x, info, ans) in enumerate(zip(xs, infos, answers)):
            e = _rel(x.cpu().numpy(), ans)
            assert info["converged"] and info["resid"] <= 1e-9, (mode, i, info["resid"])
            assert e < 1e-5, (mode, i, e)
        _log(f"  mode {mode}: worst error vs LU "
             f"{max(_rel(x.cpu().numpy(), a) for x, a in zip(xs, answers)):.2e}")
