"""Plane-wave scattering by a homogeneous isotropic elastic sphere in a fluid
(oracle, closed-form reference).

TEST INFRASTRUCTURE ONLY (see the package header).

Sec. 3.1 checks the BEM-FEM solver against the analytic solution for an
elastic sphere, which the paper only cites; this module derives it from the
governing equations of Sec. 2.1 (Helmholtz equation in the fluid, Navier's
equation in the solid, continuity of the normal displacement and of the
normal traction, no shear traction on the interface) with the time factor
exp(-i omega t):

* fluid, incident wave exp(i k z) and outgoing scattered wave:
  p = sum_n (2n+1) i^n [j_n(kr) + A_n h_n(kr)] P_n(cos t),
  h_n = j_n + i y_n, and dp/dr = rho_f omega^2 u_r at r = a;
* solid, u = grad phi + curl curl (r psi) (r the position vector) with
  phi = sum (2n+1) i^n B_n j_n(k_L r) P_n, psi = sum (2n+1) i^n C_n j_n(k_T r) P_n,
  k_L = omega / c_L, c_L^2 = (lam + 2 mu) / rho_s, k_T = omega / c_T,
  c_T^2 = mu / rho_s; per degree n (common factor (2n+1) i^n):
  u_r = B k_L j_n'(x_L) + C n(n+1) j_n(x_T) / r,
  sigma_rr = B [-rho_s omega^2 j_n(x_L) + 2 mu k_L^2 (j_n + j_n'')(x_L)]
             + 2 mu C n(n+1) [x_T j_n'(x_T) - j_n(x_T)] / r^2,
  sigma_rt = (mu / r^2) {2 B [x_L j_n'(x_L) - j_n(x_L)]
             + C [(2 n(n+1) - 2 - x_T^2) j_n(x_T) - 2 x_T j_n'(x_T)]} dP_n/dt,
  x_L = k_L r, x_T = k_T r (the shear potential's radial parts follow from the
  spherical Bessel equation);
* at r = a: u_r continuous, sigma_rr = -p, sigma_rt = 0: three equations per
  n >= 1 for (A_n, B_n, C_n); for n = 0 the shear potential does not enter
  and the shear condition is void.
"""
from __future__ import annotations

import numpy as np
from scipy.special import eval_legendre, spherical_jn, spherical_yn


def _h(n, x, derivative=False):
    return spherical_jn(n, x, derivative) + 1j * spherical_yn(n, x, derivative)


def _j2(n, x):
    """Second derivative of j_n from the spherical Bessel equation."""
    j, jp = spherical_jn(n, x), spherical_jn(n, x, True)
    return -2.0 / x * jp - (1.0 - n * (n + 1) / x ** 2) * j


def n_terms(k, a, lam, mu, rho_s, omega):
    """Degrees kept: beyond the largest of k a, k_L a, k_T a by a margin at
    which the omitted terms fall below rounding."""
    kT = omega / np.sqrt(mu / rho_s)
    x = max(k * a, kT * a)
    return int(x + 4.0 * np.cbrt(x) + 25)


def coefficients(k, a, lam, mu, rho_s, rho_f, omega, nmax=None):
    """A_n, B_n, C_n for n = 0..nmax (scattered-wave, compressional and
    shear coefficients of the expansions above)."""
    if nmax is None:
        nmax = n_terms(k, a, lam, mu, rho_s, omega)
    kL = omega / np.sqrt((lam + 2 * mu) / rho_s)
    kT = omega / np.sqrt(mu / rho_s)
    xL, xT, x = kL * a, kT * a, k * a
    A = np.zeros(nmax + 1, complex)
    B = np.zeros(nmax + 1, complex)
    C = np.zeros(nmax + 1, complex)
    w2f = rho_f * omega ** 2
    for n in range(nmax + 1):
        jL, jLp, jLpp = spherical_jn(n, xL), spherical_jn(n, xL, True), _j2(n, xL)
        jT, jTp = spherical_jn(n, xT), spherical_jn(n, xT, True)
        jf, jfp = spherical_jn(n, x), spherical_jn(n, x, True)
        hf, hfp = _h(n, x), _h(n, x, True)
        nn = n * (n + 1)
        # rows: normal displacement, normal traction, shear traction
        # unknowns: A, B, C
        M = np.array([
            [-k / w2f * hfp, kL * jLp, nn * jT / a],
            [hf, -rho_s * omega ** 2 * jL + 2 * mu * kL ** 2 * (jL + jLpp),
             2 * mu * nn * (xT * jTp - jT) / a ** 2],
            [0.0, 2 * (xL * jLp - jL), (2 * nn - 2 - xT ** 2) * jT - 2 * xT * jTp],
        ], dtype=complex)
        rhs = np.array([k / w2f * jfp, -jf, 0.0], dtype=complex)
        if n == 0:
            s = np.linalg.solve(M[:2, :2], rhs[:2])
            A[n], B[n] = s
        else:
            A[n], B[n], C[n] = np.linalg.solve(M, rhs)
    return A, B, C


def surface_pressure(k, a, lam, mu, rho_s, rho_f, omega, cos_t, nmax=None):
    """Total pressure p(a, t) on the sphere for the unit plane wave exp(i k z)."""
    A, _, _ = coefficients(k, a, lam, mu, rho_s, rho_f, omega, nmax)
    cos_t = np.asarray(cos_t, dtype=float)
    p = np.zeros(cos_t.shape, complex)
    for n in range(len(A)):
        p += (2 * n + 1) * 1j ** n * (spherical_jn(n, k * a) + A[n] * _h(n, k * a)) \
            * eval_legendre(n, cos_t)
    return p
