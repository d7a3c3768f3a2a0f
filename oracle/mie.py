"""Rigid-sphere plane-wave scattering series (oracle, closed-form reference).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper validates its solver against an analytic sphere solution (Sec. 3.1);
the analogue for the acoustic operator alone is the sound-hard sphere.  With
the time factor exp(-i omega t) (Sec. 2.1), the incident wave
exp(i k d.x) = sum_n i^n (2n+1) j_n(kr) P_n(cos t) and the outgoing spherical
Hankel functions h_n = j_n + i y_n, the rigid condition dp/dr = 0 at r = a
gives the scattered coefficients -j_n'(ka)/h_n'(ka), and the Wronskian
j_n h_n' - j_n' h_n = i/x^2 collapses the surface field to

    p(a, t) = (i / (ka)^2) sum_n i^n (2n+1) P_n(cos t) / h_n'(ka).
"""
from __future__ import annotations

import numpy as np
from scipy.special import eval_legendre, spherical_jn, spherical_yn


def _nmax(x):
    return int(x + 4.0 * np.cbrt(x) + 30)


def hankel1(n, x, derivative=False):
    return spherical_jn(n, x, derivative) + 1j * spherical_yn(n, x, derivative)


def surface_pressure(ka: float, cos_t):
    """Total pressure on the rigid sphere surface, unit incident amplitude."""
    cos_t = np.asarray(cos_t, dtype=np.float64)
    out = np.zeros(cos_t.shape, dtype=np.complex128)
    for n in range(_nmax(ka)):
        out += (1j ** n) * (2 * n + 1) * eval_legendre(n, cos_t) / hankel1(n, ka, True)
    return out * 1j / ka ** 2


def total_field(k: float, a: float, r, cos_t):
    """Incident + scattered field at radius r >= a (series form)."""
    r = np.asarray(r, dtype=np.float64)
    cos_t = np.asarray(cos_t, dtype=np.float64)
    out = np.zeros(np.broadcast(r, cos_t).shape, dtype=np.complex128)
    for n in range(_nmax(k * max(a, float(np.max(r))))):
        an = -spherical_jn(n, k * a, True) / hankel1(n, k * a, True)
        rad = spherical_jn(n, k * r) + an * hankel1(n, k * r)
        out += (1j ** n) * (2 * n + 1) * eval_legendre(n, cos_t) * rad
    return out


def incident_series(k: float, r, cos_t):
    """The plane wave through its partial-wave series (used to pin the
    series against exp(i k r cos t))."""
    r = np.asarray(r, dtype=np.float64)
    cos_t = np.asarray(cos_t, dtype=np.float64)
    out = np.zeros(np.broadcast(r, cos_t).shape, dtype=np.complex128)
    for n in range(_nmax(k * float(np.max(r)))):
        out += (1j ** n) * (2 * n + 1) * eval_legendre(n, cos_t) * spherical_jn(n, k * r)
    return out


def total_field_xyz(k: float, a: float, pts, d):
    """total_field at Cartesian points for incidence direction d."""
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    r = np.linalg.norm(pts, axis=1)
    return total_field(k, a, r, (pts @ np.asarray(d)) / r)
