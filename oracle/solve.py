"""Solvers, field representation, objective and gradient (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

* ``gmres``  - restarted GMRES(m) (the paper's iterative solver, Sec. 3,
  tolerance given there as 1e-5; the workloads use 1e-6): x0 = 0, Arnoldi by
  modified Gram-Schmidt, Givens rotations, exit on the true relative residual
  ||b - A x|| / ||b|| <= tol recomputed with the operator.
* ``dense_solve`` - LU (numpy.linalg.solve), the analogue of the paper's
  LAPACK direct solver (Sec. 3.1).
* ``represent`` - the integral representation at exterior points (solver
  step 5, Sec. 2.3):  p(x) = p_inc(x) + sum_j [Khat_j(x) p_j - Shat_j(x) q_j],
  with the 3-point rule (points well separated from the boundary).
* ``represent_grad`` / ``point_source_grad`` - gradients of the scattered
  and incident fields at exterior points; ``topological_derivative`` - the
  paper's T_Omega (Eq. danseitpoderi) from the state and adjoint fields;
* ``objective_and_gradient`` - J = sum_m |p(x_m)|^2 (Eq. obj with
  f = |p|^2) for an admittance boundary q = sigma p, sigma = -i k beta, and
  its gradient in beta by the discrete adjoint; the pairing
  dJ = Re[sum_m df/dp dp(x_m)] with df/dp = 2 conj(p) follows Eq. danseideltaJ.
"""
from __future__ import annotations

import numpy as np

from . import bem


def gmres(apply_A, b, tol=1e-6, restart=50, max_iter=2000, x0=None):
    """Returns (x, info) with info = dict(iters, resid, history, converged)."""
    b = np.asarray(b, dtype=np.complex128)
    n = len(b)
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, dict(iters=0, resid=0.0, history=[0.0], converged=True)
    history = []
    total = 0
    r = b - apply_A(x) if x0 is not None else b.copy()
    rel = np.linalg.norm(r) / bn
    history.append(rel)
    while total < max_iter and rel > tol:
        beta = np.linalg.norm(r)
        Vb = np.zeros((restart + 1, n), dtype=np.complex128)
        Hh = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        g[0] = beta
        Vb[0] = r / beta
        j_end = 0
        for j in range(restart):
            w = apply_A(Vb[j])
            total += 1
            for i in range(j + 1):           # modified Gram-Schmidt
                Hh[i, j] = np.vdot(Vb[i], w)
                w = w - Hh[i, j] * Vb[i]
            Hh[j + 1, j] = np.linalg.norm(w)
            if Hh[j + 1, j] != 0.0:
                Vb[j + 1] = w / Hh[j + 1, j]
            for i in range(j):               # previous rotations
                t = cs[i] * Hh[i, j] + sn[i] * Hh[i + 1, j]
                Hh[i + 1, j] = -np.conj(sn[i]) * Hh[i, j] + np.conj(cs[i]) * Hh[i + 1, j]
                Hh[i, j] = t
            a, c = Hh[j, j], Hh[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(c) ** 2)
            if den == 0.0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j] = a / den
                sn[j] = c / den
                cs[j], sn[j] = np.conj(cs[j]), np.conj(sn[j])
            Hh[j, j] = cs[j] * a + sn[j] * c
            Hh[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            j_end = j + 1
            history.append(abs(g[j + 1]) / bn)
            if abs(g[j + 1]) / bn <= tol or total >= max_iter or Hh[j, j] == 0.0:
                break
        y = np.linalg.solve(np.triu(Hh[:j_end, :j_end]), g[:j_end])
        x = x + Vb[:j_end].T @ y
        r = b - apply_A(x)
        rel = np.linalg.norm(r) / bn
        history[-1] = rel
    return x, dict(iters=total, resid=rel, history=history, converged=rel <= tol)


def dense_solve(A, b):
    return np.linalg.solve(A, b)


def represent_blocks(geom: bem.Geometry, k: float, pts):
    """Khat (M, N) and Shat (M, N): 3-point-rule integrals of G_y and G from
    the elements to exterior points."""
    pts = np.asarray(pts, dtype=np.float64)
    x = pts[:, None, None, :]
    dummy = np.zeros_like(x)
    y = geom.qpts[None]
    ny = geom.normal[None, :, None, :]
    G, Gy, _, _ = bem.kernels(x, dummy, y, ny, k)
    w = geom.qw[None]
    return (Gy * w).sum(2), (G * w).sum(2)


def represent(geom: bem.Geometry, k: float, pts, p, q, d):
    Kh, Sh = represent_blocks(geom, k, pts)
    pinc = np.exp(1j * k * (np.asarray(pts) @ np.asarray(d)))
    return pinc + Kh @ p - Sh @ q


def represent_grad_blocks(geom: bem.Geometry, k: float, pts):
    """Gradients in x of the representation's kernels (3-point rule):
    GK (M, N, 3) = grad_x int_j dG/dn_y(x - y), GS (M, N, 3) = grad_x int_j G.
    With rv = x - y, r = |rv|, G' = G (ik - 1/r), G'' = G ((ik - 1/r)^2 + 1/r^2):
    grad G = G' rv / r;  grad dG/dn_y = -(G'' - G'/r)(rv.n_y) rv / r^2 - G' n_y / r."""
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    rv = pts[:, None, None, :] - geom.qpts[None]            # (M, N, 3, 3)
    r2 = np.einsum("...i,...i->...", rv, rv)
    r = np.sqrt(r2)
    ik = 1j * k
    G = np.exp(ik * r) / (4.0 * np.pi * r)
    g1 = G * (ik - 1.0 / r)
    g2 = G * ((ik - 1.0 / r) ** 2 + 1.0 / r2)
    ny = geom.normal[None, :, None, :]
    rny = np.einsum("...i,...i->...", rv, ny)
    w = geom.qw[None, :, :, None]
    gS = (g1 / r)[..., None] * rv
    gK = (-(g2 - g1 / r) * rny / r2)[..., None] * rv - (g1 / r)[..., None] * ny
    return (gK * w).sum(2), (gS * w).sum(2)


def represent_grad(geom: bem.Geometry, k: float, pts, p, q):
    """grad_x of sum_j [Khat_j(x) p_j - Shat_j(x) q_j] (scattered part), (M, 3)."""
    GK, GS = represent_grad_blocks(geom, k, pts)
    out = np.einsum("mnc,n->mc", GK, p)
    if q is not None:
        out -= np.einsum("mnc,n->mc", GS, q)
    return out


def point_source_grad(k: float, pts, src, amp):
    """grad of sum_m A_m G(x - y_m), (M, 3)."""
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    src = np.asarray(src, dtype=np.float64).reshape(-1, 3)
    rv = pts[:, None, :] - src[None, :, :]
    r = np.linalg.norm(rv, axis=2)
    G = np.exp(1j * k * r) / (4.0 * np.pi * r)
    g1 = G * (1j * k - 1.0 / r)
    return ((g1 / r * np.asarray(amp)[None, :])[..., None] * rv).sum(1)


def topological_derivative(p, gp, pt, gpt, rho_f, rho_s, lam_f, lam_s, omega):
    """T_Omega at points (Eq. danseitpoderi): appearance of a small elastic
    sphere (density rho_s, bulk modulus lam_s) in the fluid (rho_f, lam_f)
    at frequency omega, from the state field p, grad p and the adjoint field
    pt, grad pt there:
      Re[3 (rho_s - rho_f) / (2 rho_s + rho_f) grad p . grad pt
         - (lam_s - lam_f) / (lam_s lam_f) rho_f omega^2 p pt].
    lam_s = inf, rho_s = inf is the sound-hard (rigid) limit."""
    if np.isinf(rho_s):
        cg = 1.5
    else:
        cg = 3.0 * (rho_s - rho_f) / (2.0 * rho_s + rho_f)
    cv = (1.0 / lam_f if np.isinf(lam_s) else (lam_s - lam_f) / (lam_s * lam_f)) * rho_f * omega ** 2
    return np.real(cg * np.einsum("mc,mc->m", gp, gpt) - cv * p * pt)


def point_source_field(k: float, pts, src, amp):
    """Incident field of point sources, sum_m A_m G(x - y_m) (Eq. hel)."""
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    src = np.asarray(src, dtype=np.float64).reshape(-1, 3)
    r = np.linalg.norm(pts[:, None, :] - src[None, :, :], axis=2)
    return (np.exp(1j * k * r) / (4.0 * np.pi * r) * np.asarray(amp)[None, :]).sum(1)


def objective_and_gradient(geom: bem.Geometry, k: float, alpha: complex, beta, d, pts,
                           Mp=None, Mq=None):
    """Dense discrete J(beta) and dJ/dRe(beta) + i dJ/dIm(beta).

    A(sigma) = Mp + Mq diag(sigma), sigma = -i k beta; A p = b (plane wave);
    p_obs = p_inc + (Kh - Sh diag(sigma)) p; J = sum |p_obs|^2.
    Adjoint: A^T lam = (Kh - Sh diag(sigma))^T conj(p_obs);
    g = -Mq^T lam - Sh^T conj(p_obs);  dJ/dRe beta_e = 2 Re(-i k g_e p_e),
    dJ/dIm beta_e = 2 Re(k g_e p_e).
    """
    if Mp is None:
        Mp, Mq = bem.bm_blocks(geom, k, alpha)
    sigma = -1j * k * np.asarray(beta)
    A = Mp + Mq * sigma[None, :]
    b = bem.plane_wave_rhs(geom, k, alpha, d)
    p = np.linalg.solve(A, b)
    Kh, Sh = represent_blocks(geom, k, pts)
    R = Kh - Sh * sigma[None, :]
    pinc = np.exp(1j * k * (np.asarray(pts) @ np.asarray(d)))
    pobs = pinc + R @ p
    J = float(np.sum(np.abs(pobs) ** 2))
    c = np.conj(pobs)
    lam = np.linalg.solve(A.T, R.T @ c)
    g = -(Mq.T @ lam) - Sh.T @ c
    dRe = 2.0 * np.real(-1j * k * g * p)
    dIm = 2.0 * np.real(k * g * p)
    return J, dRe + 1j * dIm, p
