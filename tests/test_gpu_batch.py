"""GPU tests of the batched solver and of the leaf-level tuner.

* A plan holding three problems (80-element coarse sphere on the direct
  path, a 320-element ellipsoid with ragged leaves, the 1280-element
  sphere) solved in one batch: state systems with an admittance boundary
  and adjoint systems, float64 GMRES and mixed-precision refinement.  Each
  solution is checked against the oracle's dense matrices (LU solve) and
  against the same system solved on its own.
* A batch on the 5120-element sphere with several right-hand sides of one
  problem (systems sharing a problem run one after another on its stream).
* The C ABI rejects malformed batches on the host.
* leaf_level < 0: the tuner keeps one of the candidate levels and the
  product it keeps matches the oracle's rows.
"""
import ctypes

import numpy as np
import pytest

from oracle import bem as obem
from workloads import admittance, complex_normal, icosphere, unit_directions

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


def _meshes():
    V1, T1 = icosphere(1)
    V2, T2 = icosphere(2)
    V2 = V2 * np.array([1.0, 0.6, 1.3])
    V3, T3 = icosphere(3)
    return [(V1, T1, 2.0, 64), (V2, T2, 3.0, 5), (V3, T3, 1.0, 32)]


@pytest.fixture(scope="module")
def three():
    bem = _lib()
    meshes = _meshes()
    _log("plan: three problems (80, 320, 1280 elements)")
    plan = bem.Plan([bem.Problem(V, T, k, leaf_cap=cap) for V, T, k, cap in meshes])
    dense = []
    for V, T, k, _ in meshes:
        g = obem.Geometry(V, T)
        Mp, Mq = obem.bm_blocks(g, k, 1j / k)
        dense.append((g, Mp, Mq))
    return bem, plan, meshes, dense


def _systems(plan, meshes, dense, seed):
    """One state system (plane wave, admittance) and one adjoint system
    (random right-hand side, admittance) per problem, with dense LU answers."""
    import torch
    rng = np.random.default_rng(seed)
    systems, answers = [], []
    for prob, ((V, T, k, _), (g, Mp, Mq)) in enumerate(zip(meshes, dense)):
        n = len(T)
        sigma = admittance(rng, n)
        d = unit_directions(rng, 1)[0]
        b = obem.plane_wave_rhs(g, k, 1j / k, d)
        A = Mp + Mq * sigma[None, :]
        systems.append(dict(prob=prob, b=torch.from_numpy(b), sigma=torch.from_numpy(sigma)))
        answers.append(np.linalg.solve(A, b))
        c = complex_normal(rng, n)
        systems.append(dict(prob=prob, b=torch.from_numpy(c), sigma=torch.from_numpy(sigma),
                            adjoint=True))
        answers.append(np.linalg.solve(A.conj().T, c))
    return systems, answers


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_against_dense_lu_and_single_solves(three, mode):
    bem, plan, meshes, dense = three
    systems, answers = _systems(plan, meshes, dense, seed=21 + mode)
    tol = 1e-8
    opts = bem.GmresOptions(tol=tol, restart=30, mode=mode, inner_tol=1e-4)
    _log(f"case: batch of {len(systems)} systems, mode {mode}")
    xs, infos = plan.solve_batch(systems, opts)
    for i, (s, x, info, ans) in enumerate(zip(systems, xs, infos, answers)):
        xb = x.cpu().numpy()
        e_lu = _rel(xb, ans)
        xi, ii = plan.solve(s["b"], sigma=s["sigma"], adjoint=s.get("adjoint", False),
                            opts=opts, prob=s["prob"])
        e_single = _rel(xb, xi.cpu().numpy())
        _log(f"  sys {i} prob {s['prob']} adj {int(s.get('adjoint', False))}: "
             f"its {info['iterations']} (single {ii['iterations']}) mv64 {info['matvec64']} "
             f"mv32 {info['matvec32']} resid {info['resid']:.2e} vs LU {e_lu:.2e} "
             f"vs single {e_single:.2e}")
        assert info["converged"] and info["resid"] <= tol
        assert (info["matvec32"] > 0) == (mode == 1)
        # the FMM operator differs from the dense one by its own accuracy
        assert e_lu < 1e-5
        # same algorithm on the same operator: same answer to the tolerance
        assert e_single < 1e-6
        assert abs(info["iterations"] - ii["iterations"]) <= 2


def test_batch_of_many_right_hand_sides_one_problem():
    import torch
    bem = _lib()
    V, T = icosphere(4)
    k = 2.0
    plan = bem.Plan(bem.Problem(V, T, k))
    g = obem.Geometry(V, T)
    rng = np.random.default_rng(5)
    dirs = unit_directions(rng, 6)
    sigma = torch.from_numpy(admittance(rng, len(T)))
    systems = []
    for i, d in enumerate(dirs):
        b = plan.plane_wave_rhs(d)
        systems.append(dict(prob=0, b=b, sigma=sigma if i % 2 else None, adjoint=(i % 3 == 2)))
    opts = bem.GmresOptions(tol=1e-6, restart=50, mode=1)
    _log("case: batch of 6 systems on the 5120-element sphere")
    xs, infos = plan.solve_batch(systems, opts)
    rows = np.sort(rng.choice(len(T), 24, replace=False))
    for i, (s, x, info) in enumerate(zip(systems, xs, infos)):
        assert info["converged"] and info["resid"] <= 1e-6
        xi, ii = plan.solve(s["b"], sigma=s["sigma"], adjoint=s["adjoint"], opts=opts)
        e = _rel(x.cpu().numpy(), xi.cpu().numpy())
        _log(f"  sys {i}: mv32 {info['matvec32']} mv64 {info['matvec64']} "
             f"resid {info['resid']:.2e} vs single {e:.2e}")
        assert e < 1e-5
        if not s["adjoint"]:
            # residual of the batch solution on exact oracle rows
            xb = x.cpu().numpy()
            sg = None if s["sigma"] is None else s["sigma"].numpy()
            q = None if sg is None else sg * xb
            r = s["b"].cpu().numpy()[rows] - obem.matvec(g, k, 1j / k, xb, q, rows=rows, block=8)
            rr = np.linalg.norm(r) / np.linalg.norm(s["b"].cpu().numpy()[rows])
            _log(f"    oracle residual on sampled rows {rr:.2e}")
            assert rr < 1e-5


def test_batch_rejects_malformed_calls(three):
    import torch
    bem, plan, meshes, dense = three
    lib = bem.load_library()
    n = plan.n[0]
    b = torch.ones(n, dtype=torch.complex128, device="cuda")
    x = torch.zeros_like(b)
    _log("case: malformed batches")

    def call(probs, bs, xs, ns=None):
        ns = len(probs) if ns is None else ns
        P = (ctypes.c_int32 * max(len(probs), 1))(*probs)
        B = (ctypes.c_void_p * max(len(bs), 1))(*bs)
        X = (ctypes.c_void_p * max(len(xs), 1))(*xs)
        o = bem.GmresOptions(tol=1e-6).c()
        infos = (bem._Info * max(ns, 1))()
        return lib.bem_gmres_solve_batch(plan._h, ns, P, None, None, B, X, ctypes.byref(o),
                                         infos, None)

    inv = -1  # BEM_E_INVALID
    assert call([0], [b.data_ptr()], [x.data_ptr()], ns=0) == inv
    assert call([7], [b.data_ptr()], [x.data_ptr()]) == inv
    assert call([0, 0], [b.data_ptr(), b.data_ptr()], [x.data_ptr(), x.data_ptr()]) == inv
    assert call([0], [x.data_ptr()], [x.data_ptr()]) == inv
    with pytest.raises(RuntimeError, match="INVALID"):
        plan.solve_batch([dict(prob=0, b=b)], bem.GmresOptions(tol=0.0))


def test_leaf_level_tuner():
    import torch
    bem = _lib()
    V, T = icosphere(4)
    k = 4.0
    auto = bem.Plan(bem.Problem(V, T, k))
    L0 = auto.stats()["leaf_level"]
    _log(f"case: leaf-level tuner (occupancy rule picks {L0})")
    tuned = bem.Plan(bem.Problem(V, T, k, leaf_level=-1))
    st = tuned.stats()
    _log(f"  tuned level {st['leaf_level']}, {st['tuned_ms']:.3f} ms per float32 product")
    assert st["leaf_level"] in (L0 - 1, L0, L0 + 1)
    assert st["tuned_ms"] > 0.0
    assert auto.stats()["tuned_ms"] == 0.0
    g = obem.Geometry(V, T)
    rng = np.random.default_rng(13)
    p, q = complex_normal(rng, len(T)), complex_normal(rng, len(T))
    rows = np.sort(rng.choice(len(T), 48, replace=False))
    ref = obem.matvec(g, k, 1j / k, p, q, rows=rows, block=16)
    y = tuned.matvec(torch.from_numpy(p), torch.from_numpy(q)).cpu().numpy()
    e = _rel(y[rows], ref)
    _log(f"  tuned plan float64 product vs oracle rows {e:.2e}")
    assert e < 1e-6
