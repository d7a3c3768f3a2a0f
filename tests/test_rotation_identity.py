"""CPU check of the identities the rotation-based multipole-to-local
translations rest on (the factorisation is this implementation's way of
applying the FMM translations of Sec. 2.3; checked here from scipy's
spherical harmonics and Bessel functions, independently of the HIP code):

* rotating a function rotates its spherical-harmonic coefficients degree by
  degree with D(Q)[m][m'] = int conj(Y_n^m(x)) Y_n^m'(Q^T x) dOmega; for
  Q = R_z(phi) R_y(theta), D(Q) = diag(e^{-i m phi}) d with d = D(R_y(theta))
  real and orthogonal;
* the singular-to-regular translation T(t) (column (n, m): the coefficients
  of S_n^m(t + r) in the regular wave functions R_n'^m'(r)) satisfies
  T(Q t) = D(Q) T(t) D(Q)^H, and T(|t| e_z) couples equal orders m only.

The rotation blocks come from the same product rule the library uses
(Gauss-Legendre in cos(theta) times equispaced azimuths, exact for the
degree-2n integrand); T by projecting S_n^m(t + r) on a small sphere
|r| = rho onto the spherical harmonics (its content beyond degree ~30 is
below rounding for rho / |t| = 1/4).
"""
import numpy as np
from scipy import special as sp

P = 4        # degrees 0 .. P
K = 2.0      # wavenumber


def _Y(n, m, th, ph):
    return sp.sph_harm_y(n, m, th, ph)


def _grid(nu, nph):
    u, w = np.polynomial.legendre.leggauss(nu)
    th, ph = np.arccos(u), 2 * np.pi * np.arange(nph) / nph
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    return TH.ravel(), PH.ravel(), np.outer(w, np.full(nph, 2 * np.pi / nph)).ravel()


def _xyz(th, ph):
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1)


def _sph(x):
    r = np.linalg.norm(x, axis=-1)
    return r, np.arccos(np.clip(x[..., 2] / r, -1, 1)), np.arctan2(x[..., 1], x[..., 0])


def _Ry(t):
    c, s = np.cos(t), np.sin(t)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


def _Rz(f):
    c, s = np.cos(f), np.sin(f)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def _rot_block(n, Q):
    """D(Q) of degree n: [m][m'] = sum_q w_q conj(Y_n^m(x_q)) Y_n^m'(Q^T x_q)."""
    th, ph, w = _grid(n + 1, 2 * n + 2)
    _, thr, phr = _sph(_xyz(th, ph) @ Q)            # rows Q^T x
    A = np.array([_Y(n, m, th, ph) for m in range(-n, n + 1)])
    B = np.array([_Y(n, m, thr, phr) for m in range(-n, n + 1)])
    return (np.conj(A) * w) @ B.T


def _rot(Q):
    """Block-diagonal D(Q) over degrees 0..P, coefficient index n^2 + n + m."""
    D = np.zeros(((P + 1) ** 2, (P + 1) ** 2), dtype=complex)
    for n in range(P + 1):
        D[n * n:(n + 1) ** 2, n * n:(n + 1) ** 2] = _rot_block(n, Q)
    return D


def _translation(t, rho=None):
    """T(t)[(n', m'), (n, m)]: coefficients of S_n^m(t + r) on R_n'^m'(r)."""
    rho = 0.25 * np.linalg.norm(t) if rho is None else rho
    th, ph, w = _grid(48, 96)
    x = _xyz(th, ph)
    r, tv, pv = _sph(t[None, :] + rho * x)
    Ybar = np.array([np.conj(_Y(n2, m2, th, ph)) * w
                     for n2 in range(P + 1) for m2 in range(-n2, n2 + 1)])
    jn = np.array([sp.spherical_jn(n2, K * rho)
                   for n2 in range(P + 1) for m2 in range(-n2, n2 + 1)])
    T = np.zeros(((P + 1) ** 2, (P + 1) ** 2), dtype=complex)
    for n in range(P + 1):
        h = sp.spherical_jn(n, K * r) + 1j * sp.spherical_yn(n, K * r)
        for m in range(-n, n + 1):
            T[:, n * n + n + m] = (Ybar @ (h * _Y(n, m, tv, pv))) / jn
    return T


def test_rotation_blocks_rotate_harmonics():
    rng = np.random.default_rng(1)
    Q = _Rz(0.9) @ _Ry(1.2) @ _Rz(-0.4)
    z = rng.normal(size=(50, 3))
    z /= np.linalg.norm(z, axis=1)[:, None]
    _, th, ph = _sph(z)
    _, thr, phr = _sph(z @ Q)
    for n in range(P + 1):
        D = _rot_block(n, Q)
        lhs = np.array([_Y(n, m2, thr, phr) for m2 in range(-n, n + 1)])   # Y^m'(Q^T z)
        rhs = D.T @ np.array([_Y(n, m, th, ph) for m in range(-n, n + 1)])
        assert np.max(np.abs(lhs - rhs)) < 1e-12
        assert np.max(np.abs(D.conj().T @ D - np.eye(2 * n + 1))) < 1e-12


def test_rotation_factors_into_phases_and_real_blocks():
    phi, theta = 0.7, 1.1
    for n in range(P + 1):
        Dz = _rot_block(n, _Rz(phi))
        assert np.max(np.abs(Dz - np.diag(np.exp(-1j * np.arange(-n, n + 1) * phi)))) < 1e-12
        d = _rot_block(n, _Ry(theta))
        assert np.max(np.abs(d.imag)) < 1e-13
        assert np.max(np.abs(d.real @ d.real.T - np.eye(2 * n + 1))) < 1e-12
        D = _rot_block(n, _Rz(phi) @ _Ry(theta))
        assert np.max(np.abs(D - Dz @ d)) < 1e-12


def test_translation_factorises_through_the_axis():
    """T(t) = D(Q) T(|t| e_z) D(Q)^H for t = |t| Q e_z, Q = R_z(phi) R_y(theta),
    and T(|t| e_z) is diagonal in the order m (checked for a translation across
    two boxes and one across three, as on a level of box side 1)."""
    for off in ((2, 1, -1), (3, -2, 1)):
        t = np.array(off, dtype=float)
        r, theta, phi = _sph(t)
        Q = _Rz(phi) @ _Ry(theta)
        assert np.allclose(Q @ np.array([0, 0, 1.0]), t / r)
        Tz = _translation(np.array([0.0, 0.0, r]))
        T = _translation(t)
        scale = np.max(np.abs(T))
        D = _rot(Q)
        err = np.max(np.abs(T - D @ Tz @ D.conj().T)) / scale
        assert err < 1e-10, err
        ms = np.array([m for n in range(P + 1) for m in range(-n, n + 1)])
        off_m = np.abs(Tz[ms[:, None] != ms[None, :]])
        assert np.max(off_m) < 1e-12 * np.max(np.abs(Tz))
