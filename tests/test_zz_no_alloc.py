"""The allocation-free product (bem_fmm_matvec_noalloc) against
bem_fmm_matvec through the C ABI: two calls in a row on one device, the
second on a smaller problem (the static buffer keeps the first call's
contents), float64 and float32, with and without q, with the plan's tuned
translations and with rotation-based multipole-to-local translations on
every level; a problem whose buffers exceed the static buffer is rejected
before any launch."""
import ctypes

import numpy as np
import pytest

from workloads import complex_normal, icosphere

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


def _call(bem, fn, plan, prob, prec, p, q, y):
    import torch
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return getattr(bem._LIB, fn)(plan._h, prob, prec, bem._ptr(p), bem._ptr(q), bem._ptr(y), 1, s)


@pytest.mark.parametrize("rot", [0, 2])
def test_noalloc_product_matches_the_allocating_one(rot):
    import torch
    bem = _lib()
    meshes = [(icosphere(3), 1.0), (icosphere(2), 2.0)]
    plan = bem.Plan([bem.Problem(V, T, k, leaf_cap=16, m2l_rot=rot) for (V, T), k in meshes])
    _log(f"case: m2l_rot={rot}, rotation-based levels f64 {plan.stats(0)['m2l_rot64'][2:]}")
    rng = np.random.default_rng(71)
    for prec, tol in ((bem.BEM_C128, 1e-12), (bem.BEM_C64, 1e-6)):
        for prob in (0, 1):          # the second call on the smaller problem
            n = plan.n[prob]
            p = torch.from_numpy(complex_normal(rng, n)).cuda()
            q = torch.from_numpy(complex_normal(rng, n)).cuda()
            for qq in (q, None):
                y_ref = torch.empty_like(p)
                y_na = torch.full_like(p, float("nan"))
                assert _call(bem, "bem_fmm_matvec", plan, prob, prec, p, qq, y_ref) == 0
                rc = _call(bem, "bem_fmm_matvec_noalloc", plan, prob, prec, p, qq, y_na)
                assert rc == 0, bem._LIB.bem_last_error().decode()
                torch.cuda.synchronize()
                a, b = y_na.cpu().numpy(), y_ref.cpu().numpy()
                err = float(np.linalg.norm(a - b) / np.linalg.norm(b))
                _log(f"  prec {prec} prob {prob} (n={n}) q={'yes' if qq is not None else 'no'}: "
                     f"rel diff {err:.2e}")
                assert np.all(np.isfinite(a)) and err <= tol


def test_noalloc_rejects_problems_beyond_the_static_buffer():
    import torch
    bem = _lib()
    V, T = icosphere(5)
    plan = bem.Plan(bem.Problem(V, T, 4.0))
    n = plan.n[0]
    p = torch.ones(n, dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(p)
    rc = _call(bem, "bem_fmm_matvec_noalloc", plan, 0, bem.BEM_C128, p, None, y)
    msg = bem._LIB.bem_last_error().decode()
    _log(f"  n={n} float64: status {rc}, '{msg}'")
    assert rc == -1 and "too large" in msg
    torch.cuda.synchronize()
    assert float(y.abs().max()) == 0.0      # nothing was launched
