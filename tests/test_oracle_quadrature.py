"""Pins for the oracle's kernel, quadrature, near-singular and self integrals.

Each check compares the oracle with something other than itself: finite
differences, closed forms (triangle monomial moments, the solid angle of a
triangle), an independent singularity-removing rule (Duffy), or an exact
invariant of the discrete Laplace operators on a closed polyhedron.
"""
import math

import numpy as np
import pytest

from oracle import bem
from workloads import icosphere

RNG = np.random.default_rng(1234)


def _tri():
    a = np.array([0.1, -0.2, 0.05])
    b = np.array([1.0, 0.1, -0.1])
    c = np.array([0.3, 0.9, 0.2])
    return a, b, c


def test_rules_integrate_monomials_exactly():
    # unit right triangle (0,0),(1,0),(0,1): int x^i y^j = i! j! / (i+j+2)!
    A, B, C = np.array([0.0, 0, 0]), np.array([1.0, 0, 0]), np.array([0.0, 1, 0])
    bary, w = bem._collapsed_rule(8)
    pts = bary[:, 0:1] * A + bary[:, 1:2] * B + bary[:, 2:3] * C
    for i in range(8):
        for j in range(8 - i):
            exact = math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)
            got = 0.5 * np.sum(w * pts[:, 0] ** i * pts[:, 1] ** j)
            assert abs(got - exact) < 1e-15, (i, j)
    pts = bem.Q3_BARY[:, 0:1] * A + bem.Q3_BARY[:, 1:2] * B + bem.Q3_BARY[:, 2:3] * C
    for i in range(3):
        for j in range(3 - i):
            exact = math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)
            got = 0.5 * np.sum(bem.Q3_W * pts[:, 0] ** i * pts[:, 1] ** j)
            assert abs(got - exact) < 1e-15, (i, j)
    # ...and the 3-point rule is not exact at degree 3 (it is a degree-2 rule)
    got = 0.5 * np.sum(bem.Q3_W * pts[:, 0] ** 3)
    assert abs(got - 6 / math.factorial(5)) > 1e-4


@pytest.mark.parametrize("k", [0.0, 1.0, 7.5])
def test_kernel_normal_derivatives_match_finite_differences(k):
    for _ in range(5):
        x = RNG.standard_normal(3)
        y = RNG.standard_normal(3)
        nx = RNG.standard_normal(3); nx /= np.linalg.norm(nx)
        ny = RNG.standard_normal(3); ny /= np.linalg.norm(ny)
        h = 1e-5

        def G(xx, yy):
            return bem.kernels(xx, nx, yy, ny, k)[0]

        def Gy(xx, yy):
            return bem.kernels(xx, nx, yy, ny, k)[1]

        G0, Gy0, Gx0, Gxy0 = bem.kernels(x, nx, y, ny, k)
        fd_y = (G(x, y + h * ny) - G(x, y - h * ny)) / (2 * h)
        fd_x = (G(x + h * nx, y) - G(x - h * nx, y)) / (2 * h)
        fd_xy = (Gy(x + h * nx, y) - Gy(x - h * nx, y)) / (2 * h)
        assert abs(fd_y - Gy0) < 1e-8 * max(1.0, abs(Gy0))
        assert abs(fd_x - Gx0) < 1e-8 * max(1.0, abs(Gx0))
        assert abs(fd_xy - Gxy0) < 1e-7 * max(1.0, abs(Gxy0))
        r = np.linalg.norm(x - y)
        assert abs(G0 - np.exp(1j * k * r) / (4 * math.pi * r)) < 1e-15


def _solid_angle(x, a, b, c):
    """Signed solid angle of triangle (a,b,c) at x, van Oosterom & Strackee
    (1983); positive when x lies on the side opposite to (b-a)x(c-a)."""
    R1, R2, R3 = a - x, b - x, c - x
    l1, l2, l3 = (np.linalg.norm(v) for v in (R1, R2, R3))
    num = np.dot(R1, np.cross(R2, R3))
    den = l1 * l2 * l3 + np.dot(R1, R2) * l3 + np.dot(R1, R3) * l2 + np.dot(R2, R3) * l1
    return 2.0 * math.atan2(num, den)


def test_near_integrals_laplace_double_layer_is_solid_angle():
    a, b, c = _tri()
    n = np.cross(b - a, c - a); n /= np.linalg.norm(n)
    cen = (a + b + c) / 3
    xs = [cen + 0.05 * n, cen - 0.3 * n + 0.2 * (b - a), a + 0.01 * n + 0.3 * (a - cen),
          0.5 * (a + b) + 0.02 * (a + b - 2 * c) + 0.0 * n, cen + 1.5 * (b - c)]
    for x in xs:
        nx = RNG.standard_normal(3); nx /= np.linalg.norm(nx)
        val = bem.near_integrals(x[None], nx[None], a[None], b[None], c[None], n[None], 0.0)[0]
        omega = _solid_angle(x, a, b, c)
        assert abs(val[1] - (-omega / (4 * math.pi))) < 1e-12
        # hypersingular = n_x . grad_x of the double layer: finite differences
        h = 1e-5
        fd = (-_solid_angle(x + h * nx, a, b, c) + _solid_angle(x - h * nx, a, b, c)) / (8 * math.pi * h)
        assert abs(val[3] - fd) < 1e-6 * max(1.0, abs(fd))


@pytest.mark.parametrize("k", [1.0, 8.0])
def test_near_integrals_gradient_consistency(k):
    """int G_x = n_x . grad_x int G and int G_xy = n_x . grad_x int G_y."""
    a, b, c = _tri()
    n = np.cross(b - a, c - a); n /= np.linalg.norm(n)
    for x in [0.5 * (a + b) + 0.08 * (a + b - 2 * c), (a + b + c) / 3 + 0.07 * n]:
        nx = RNG.standard_normal(3); nx /= np.linalg.norm(nx)
        h = 1e-5

        def I(xx):
            return bem.near_integrals(xx[None], nx[None], a[None], b[None], c[None], n[None], k)[0]

        v = I(x)
        fd = (I(x + h * nx) - I(x - h * nx)) / (2 * h)
        assert abs(v[2] - fd[0]) < 1e-7 * max(1.0, abs(v[2]))
        assert abs(v[3] - fd[1]) < 1e-6 * max(1.0, abs(v[3]))


def test_near_integrals_match_uniform_refinement():
    """Against 4^7 uniform sub-triangles with the 3-point rule, Richardson-
    extrapolated (an independent, low-order method)."""
    a, b, c = _tri()
    n = np.cross(b - a, c - a); n /= np.linalg.norm(n)
    x = 0.5 * (a + b) + 0.15 * (a + b - 2 * c) + 0.05 * n
    k = 3.0

    def uniform(depth):
        tris = [(a, b, c)]
        for _ in range(depth):
            nt = []
            for A, B, C in tris:
                ab, bc, ca = (A + B) / 2, (B + C) / 2, (C + A) / 2
                nt += [(A, ab, ca), (B, bc, ab), (C, ca, bc), (ab, bc, ca)]
            tris = nt
        A = np.array([t[0] for t in tris]); B = np.array([t[1] for t in tris]); C = np.array([t[2] for t in tris])
        pts = (bem.Q3_BARY[None, :, 0, None] * A[:, None] + bem.Q3_BARY[None, :, 1, None] * B[:, None]
               + bem.Q3_BARY[None, :, 2, None] * C[:, None])
        ar = 0.5 * np.linalg.norm(np.cross(B - A, C - A), axis=1)
        vals = bem.kernels(x, n * 0 + np.array([0.0, 0.6, 0.8]), pts, n, k)
        return np.array([(v * ar[:, None] / 3).sum() for v in vals])

    u6, u7 = uniform(6), uniform(7)
    rich = u7 + (u7 - u6) / 7.0          # error ~ h^3 for the degree-2 rule
    nx = np.array([0.0, 0.6, 0.8])
    val = bem.near_integrals(x[None], nx[None], a[None], b[None], c[None], n[None], k)[0]
    for t in range(4):
        assert abs(val[t] - rich[t]) < 1e-6 * abs(rich).max()


def _duffy_self(geom, i, f, n=48):
    """int over element i of f(r) with the weak singularity at the centroid
    removed by the Duffy map on the three sub-triangles apex = centroid."""
    t, w = np.polynomial.legendre.leggauss(n)
    u = 0.5 * (t + 1); wu = 0.5 * w
    x = geom.cen[i]
    V = [geom.a[i], geom.b[i], geom.c[i]]
    tot = 0.0 + 0.0j
    for e in range(3):
        P0, P1 = V[e], V[(e + 1) % 3]
        jac = np.linalg.norm(np.cross(P0 - x, P1 - P0))
        U, W = np.meshgrid(u, u, indexing="ij")
        pts = x + U[..., None] * (P0 - x) + (U * W)[..., None] * (P1 - P0)
        r = np.linalg.norm(pts - x, axis=-1)
        tot += np.sum(np.outer(wu, wu) * U * jac * f(r))
    return tot


@pytest.mark.parametrize("k", [0.0, 1.0, 8.0])
def test_self_single_layer_against_duffy(k):
    V, T = icosphere(1)
    V = V * 0.7
    geom = bem.Geometry(V, T)
    S, H = bem.self_terms(geom, k, [0, 5, 17])
    for j, i in enumerate([0, 5, 17]):
        ref = _duffy_self(geom, i, lambda r: np.exp(1j * k * r) / (4 * math.pi * r))
        assert abs(S[j] - ref) < 1e-12 * abs(ref)


def test_self_hypersingular_static_is_double_layer_limit():
    """H0_ii equals the limit of d/dn of the triangle's Laplace double layer
    (solid angle) as the point approaches the centroid along the normal."""
    V, T = icosphere(1)
    geom = bem.Geometry(V, T)
    for i in [0, 9, 33]:
        _, H = bem.self_terms(geom, 0.0, [i])
        a, b, c, n, x = geom.a[i], geom.b[i], geom.c[i], geom.normal[i], geom.cen[i]
        L = geom.ell[i]

        def W(z):
            return -_solid_angle(x + z * n, a, b, c) / (4 * math.pi)

        def dW(z0):
            h = 1e-3 * z0
            return (W(z0 + h) - W(z0 - h)) / (2 * h)

        z1, z2 = 1e-3 * L, 2e-3 * L
        lim = (4 * dW(z1) - dW(z2)) / 3    # dW(z) = dW(0) + O(z^2): extrapolate
        assert abs(H[0] - lim) < 1e-8 * abs(lim)


@pytest.mark.parametrize("k", [1.0, 8.0])
def test_self_hypersingular_dynamic_part_against_duffy(k):
    """H_ii - H0_ii is the proper integral of G_xy - G0_xy (in-plane form)."""
    V, T = icosphere(1)
    geom = bem.Geometry(V, T)
    idx = [2, 40]
    _, Hk = bem.self_terms(geom, k, idx)
    _, H0 = bem.self_terms(geom, 0.0, idx)

    def diff(r):
        G = np.exp(1j * k * r) / (4 * math.pi * r)
        g1 = G * (1j * k - 1 / r)
        return -g1 / r - 1.0 / (4 * math.pi * r ** 3)

    for j, i in enumerate(idx):
        ref = _duffy_self(geom, i, diff, n=64)
        assert abs((Hk[j] - H0[j]) - ref) < 1e-10 * max(1.0, abs(ref))


def test_laplace_discrete_invariants_on_closed_polyhedron():
    """k = 0, every pair integrated exactly: sum_j K0_ij = -1/2 (solid angle
    at a face centroid) and sum_j H0_ij = 0 (the double layer of a constant
    density has zero gradient), to roundoff."""
    V, T = icosphere(1)
    geom = bem.Geometry(V * 1.3, T)
    S, K, Kp, H = bem.assemble_block(geom, 0.0, eta=1e9)
    assert np.abs(K.sum(1) + 0.5).max() < 1e-11
    assert np.abs(H.sum(1)).max() < 1e-9 * np.abs(H).max()
