"""Exact discrete Burton-Miller collocation operator, complex128 (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Discretisation (paper Sec. 2.3): the boundary is a union of flat triangles,
the pressure p and its normal derivative q are constant on each triangle and
the boundary integral equation is collocated at one point per triangle.  The
paper does not name that point; we take the centroid.  The normal ``n`` is the
unit normal exterior to the scatterer, i.e. pointing into the fluid (Sec. 2.1).

Kernel: G(x, y) = exp(i k r) / (4 pi r), r = |x - y| (Sec. 2.3, below Eq.
danseibie2).  With rv = x - y, G' = dG/dr = G (ik - 1/r) and
G'' = G ((ik - 1/r)^2 + 1/r^2):

    G_y  = dG/dn_y        = -G' (rv . n_y) / r
    G_x  = dG/dn_x        =  G' (rv . n_x) / r
    G_xy = d2G/dn_x dn_y  = -(G'' - G'/r)(rv.n_x)(rv.n_y)/r^2 - (G'/r)(n_x.n_y)

Discrete operators, element j, collocation point x_i:

    S_ij = int_j G,  K_ij = int_j G_y,  K'_ij = int_j G_x (n_x = n_i),
    H_ij = finite-part int_j G_xy.

How each integral is evaluated is part of the operator's definition:
* regular pairs (j != i and |x_i - c_j| >= eta * l_j, l_j = longest edge):
  the 3-point degree-2 rule (barycentric (2/3,1/6,1/6) and permutations,
  equal weights A_j/3);
* near pairs (j != i and |x_i - c_j| < eta * l_j, the test done on
  squared distances in float64): the exact integral, here to ~1e-13 relative
  by adaptive subdivision;
* self (j == i): closed reductions to edge integrals (``self_terms``).
eta = 2 unless stated.

The Burton-Miller matrix-vector product (the paper's acoustic block I/2 - D,
Eq. renritupu, plus a hypersingular equation weighted by alpha; alpha = 0 is
the paper's own operator):

    y = (I/2 - K - alpha H) p + (S + alpha K' + (alpha/2) I) q.
"""
from __future__ import annotations

import math
import multiprocessing
import os

import numpy as np

FOUR_PI = 4.0 * math.pi

# 3-point degree-2 rule on a triangle (barycentric coordinates, weight 1/3)
Q3_BARY = np.array([[2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0],
                    [1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0],
                    [1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0]])
Q3_W = np.full(3, 1.0 / 3.0)


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
class Geometry:
    """Per-element vertices, centroid (collocation point), unit normal,
    area, longest edge and the 3-point rule's points and weights."""

    def __init__(self, V: np.ndarray, T: np.ndarray):
        V = np.asarray(V, dtype=np.float64)
        T = np.asarray(T, dtype=np.int64)
        self.a = V[T[:, 0]]
        self.b = V[T[:, 1]]
        self.c = V[T[:, 2]]
        self.n_elem = len(T)
        self.cen = (self.a + self.b + self.c) / 3.0
        cr = np.cross(self.b - self.a, self.c - self.a)
        nrm = np.linalg.norm(cr, axis=1)
        self.area = 0.5 * nrm
        self.normal = cr / nrm[:, None]
        e1 = np.linalg.norm(self.b - self.a, axis=1)
        e2 = np.linalg.norm(self.c - self.b, axis=1)
        e3 = np.linalg.norm(self.a - self.c, axis=1)
        self.ell = np.maximum(np.maximum(e1, e2), e3)
        # quadrature points (N, 3, 3): element, point, xyz
        self.qpts = (Q3_BARY[None, :, 0, None] * self.a[:, None, :]
                     + Q3_BARY[None, :, 1, None] * self.b[:, None, :]
                     + Q3_BARY[None, :, 2, None] * self.c[:, None, :])
        self.qw = self.area[:, None] * Q3_W[None, :]


# --------------------------------------------------------------------------
# kernel
# --------------------------------------------------------------------------
def kernels(x, nx, y, ny, k):
    """G, G_y, G_x, G_xy for broadcastable arrays of points/normals (..., 3)."""
    rv = x - y
    r2 = np.einsum("...i,...i->...", rv, rv)
    r = np.sqrt(r2)
    ik = 1j * k
    G = np.exp(ik * r) / (FOUR_PI * r)
    g1 = G * (ik - 1.0 / r)                       # G'
    g2 = G * ((ik - 1.0 / r) ** 2 + 1.0 / r2)     # G''
    rnx = np.einsum("...i,...i->...", rv, nx)
    rny = np.einsum("...i,...i->...", rv, ny)
    nxny = np.einsum("...i,...i->...", nx, ny)
    Gy = -g1 * rny / r
    Gx = g1 * rnx / r
    Gxy = -(g2 - g1 / r) * rnx * rny / r2 - (g1 / r) * nxny
    return G, Gy, Gx, Gxy


# --------------------------------------------------------------------------
# near-singular integrals: adaptive subdivision with a collapsed Gauss rule
# --------------------------------------------------------------------------
def _gauss01(n):
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def _collapsed_rule(n):
    """Barycentric points/weights (sum 1) of an n x n Gauss rule on the
    triangle, from the square by (u, v) -> (u, (1-u) v, (1-u)(1-v))."""
    u, wu = _gauss01(n)
    U, Vv = np.meshgrid(u, u, indexing="ij")
    W = np.outer(wu, wu) * (1.0 - U) * 2.0
    l1 = U.ravel()
    l2 = ((1.0 - U) * Vv).ravel()
    l3 = 1.0 - l1 - l2
    return np.stack([l1, l2, l3], axis=1), W.ravel()


def _rule_on(bary, w, A, B, C, x, nx, ny, k):
    """Apply a barycentric rule to triangles (A,B,C) (M,3); returns (M,4)."""
    pts = (bary[None, :, 0, None] * A[:, None, :] + bary[None, :, 1, None] * B[:, None, :]
           + bary[None, :, 2, None] * C[:, None, :])
    area = 0.5 * np.linalg.norm(np.cross(B - A, C - A), axis=1)
    G, Gy, Gx, Gxy = kernels(x[:, None, :], nx[:, None, :], pts, ny[:, None, :], k)
    ww = w[None, :] * area[:, None]
    return np.stack([(G * ww).sum(1), (Gy * ww).sum(1), (Gx * ww).sum(1), (Gxy * ww).sum(1)], axis=1)


def near_integrals(x, nx, A, B, C, ny, k, tol=1e-13, order=8, max_depth=40):
    """Integrals of (G, G_y, G_x, G_xy) over triangles (A,B,C) seen from
    points x (not on the triangles).  Arrays have a leading pair axis M.

    Adaptive subdivision: a sub-triangle's rule value is compared with the
    sum over its four midpoint children; the children's sum is accepted when
    the difference is below ``tol`` times the pair's natural scale
    area / (4 pi d^m) (m = 1, 2, 2, 3 for the four kernels, d = distance from
    x to the triangle) times the sub-triangle's area share (or below 1e-15 of
    the value itself).
    Returns (M, 4) complex128.
    """
    bary, w = _collapsed_rule(order)
    M = len(x)
    out = np.zeros((M, 4), dtype=np.complex128)
    d = point_triangle_distance(x, A, B, C)
    area0 = 0.5 * np.linalg.norm(np.cross(B - A, C - A), axis=1)
    scale = area0[:, None] / (FOUR_PI * d[:, None] ** np.array([1.0, 2.0, 2.0, 3.0])[None, :])
    idx = np.arange(M)
    tA, tB, tC = A.copy(), B.copy(), C.copy()
    parent_val = _rule_on(bary, w, tA, tB, tC, x, nx, ny, k)
    for _ in range(max_depth):
        if len(idx) == 0:
            break
        mAB, mBC, mCA = 0.5 * (tA + tB), 0.5 * (tB + tC), 0.5 * (tC + tA)
        cA = np.concatenate([tA, tB, tC, mAB])
        cB = np.concatenate([mAB, mBC, mCA, mBC])
        cC = np.concatenate([mCA, mAB, mBC, mCA])
        cidx = np.tile(idx, 4)
        cval = _rule_on(bary, w, cA, cB, cC, x[cidx], nx[cidx], ny[cidx], k)
        m = len(idx)
        child_sum = cval[0:m] + cval[m:2 * m] + cval[2 * m:3 * m] + cval[3 * m:4 * m]
        sub_area = 0.5 * np.linalg.norm(np.cross(tB - tA, tC - tA), axis=1)
        frac = sub_area / area0[idx]
        err = np.abs(child_sum - parent_val)
        ok = np.all(err <= np.maximum(tol * scale[idx] * frac[:, None],
                                      1e-15 * np.abs(child_sum)), axis=1)
        np.add.at(out, idx[ok], child_sum[ok])
        bad = ~ok
        if not bad.any():
            idx = idx[:0]
            break
        if 4 * bad.sum() > 4_000_000:
            raise RuntimeError("near_integrals: too many sub-triangles")
        bad4 = np.tile(bad, 4)
        idx = cidx[bad4]
        tA, tB, tC = cA[bad4], cB[bad4], cC[bad4]
        parent_val = cval[bad4]
    if len(idx):
        raise RuntimeError("near_integrals: subdivision did not converge")
    return out


def _segment_distance(x, P, Q):
    t = np.einsum("ij,ij->i", x - P, Q - P) / np.einsum("ij,ij->i", Q - P, Q - P)
    t = np.clip(t, 0.0, 1.0)
    return np.linalg.norm(x - (P + t[:, None] * (Q - P)), axis=1)


def point_triangle_distance(x, A, B, C):
    """Euclidean distance from points x to triangles (A, B, C), (M, 3) each."""
    n = np.cross(B - A, C - A)
    n = n / np.linalg.norm(n, axis=1, keepdims=True)
    h = np.einsum("ij,ij->i", x - A, n)
    x0 = x - h[:, None] * n
    inside = np.ones(len(x), dtype=bool)
    for P, Q in ((A, B), (B, C), (C, A)):
        inside &= np.einsum("ij,ij->i", np.cross(Q - P, x0 - P), n) >= 0.0
    edge = np.minimum(np.minimum(_segment_distance(x, A, B), _segment_distance(x, B, C)),
                      _segment_distance(x, C, A))
    return np.where(inside, np.abs(h), edge)


NEAR_WORKERS = None   # process count for near integrals (None: all cores, max 16)


def _near_chunk(args):
    return near_integrals(*args[:7], tol=args[7])


def near_integrals_parallel(x, nx, A, B, C, ny, k, tol=1e-13, workers=None, chunk=2048):
    """``near_integrals`` split over a process pool (results identical: each
    pair is integrated independently)."""
    M = len(x)
    if workers is None:
        workers = NEAR_WORKERS or min(len(os.sched_getaffinity(0)), 16)
    if M <= chunk or workers <= 1:
        return near_integrals(x, nx, A, B, C, ny, k, tol=tol)
    jobs = [(x[s:s + chunk], nx[s:s + chunk], A[s:s + chunk], B[s:s + chunk], C[s:s + chunk],
             ny[s:s + chunk], k, tol) for s in range(0, M, chunk)]
    ctx = multiprocessing.get_context("fork")
    with ctx.Pool(workers) as pool:
        parts = pool.map(_near_chunk, jobs)
    return np.concatenate(parts, axis=0)


# --------------------------------------------------------------------------
# self terms (target = centroid of the source triangle)
# --------------------------------------------------------------------------
def _edge_polar(geom: Geometry, i: np.ndarray):
    """For each element in ``i`` and each edge: distance d_e from the centroid
    to the edge line and the polar angles phi-, phi+ of the edge ends
    measured from the foot of the perpendicular."""
    x = geom.cen[i]
    verts = [geom.a[i], geom.b[i], geom.c[i]]
    out = []
    for e in range(3):
        P0, P1 = verts[e], verts[(e + 1) % 3]
        L = np.linalg.norm(P1 - P0, axis=1)
        t = (P1 - P0) / L[:, None]
        s0 = np.einsum("ij,ij->i", x - P0, t)
        foot = P0 + s0[:, None] * t
        de = np.linalg.norm(x - foot, axis=1)
        sm, sp = -s0, L - s0
        out.append((de, np.arctan2(sm, de), np.arctan2(sp, de)))
    return out


def self_terms(geom: Geometry, k: float, i=None, n_gauss=64):
    """S_ii and H_ii for flat triangles collocated at their centroid
    (K_ii = K'_ii = 0 because rv . n = 0 in the plane).

    In polar coordinates about x with R(theta) the distance to the boundary:
      S_ii = (1/4pi) oint (exp(ikR) - 1)/(ik) dtheta         (k > 0; R if k = 0)
      H_ii = ik/2 - (1/4pi) oint exp(ikR)/R dtheta
    H is the Hadamard finite part (circular exclusion, 1/(2 eps) dropped),
    which equals the limit of the normal derivative of the double-layer
    potential for a density constant near x.  The angle integral is split
    per edge and written in the edge's own angle phi (R = d_e / cos phi),
    where the integrand is smooth, and done by Gauss-Legendre.
    """
    if i is None:
        i = np.arange(geom.n_elem)
    i = np.asarray(i)
    t, w = np.polynomial.legendre.leggauss(n_gauss)
    S = np.zeros(len(i), dtype=np.complex128)
    H = np.zeros(len(i), dtype=np.complex128)
    for de, pm, pp in _edge_polar(geom, i):
        half = 0.5 * (pp - pm)
        phi = 0.5 * (pp + pm)[:, None] + half[:, None] * t[None, :]
        ww = half[:, None] * w[None, :]
        R = de[:, None] / np.cos(phi)
        if k == 0.0:
            gS = R
        else:
            x_ = k * R
            gS = (np.sin(x_) + 2j * np.sin(0.5 * x_) ** 2) / k
        S += (gS * ww).sum(1) / FOUR_PI
        H -= (np.exp(1j * k * R) / R * ww).sum(1) / FOUR_PI
    H += 0.5j * k
    return S, H


# --------------------------------------------------------------------------
# operator blocks
# --------------------------------------------------------------------------
def near_mask(geom: Geometry, rows, cols, eta=2.0):
    """Boolean (len(rows), len(cols)): j != i and |x_i - c_j|^2 < eta^2 l_j^2."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    d = geom.cen[rows][:, None, :] - geom.cen[cols][None, :, :]
    d2 = np.einsum("ijk,ijk->ij", d, d)
    lim = (eta * geom.ell[cols]) ** 2
    m = d2 < lim[None, :]
    m &= rows[:, None] != cols[None, :]
    return m


def assemble_block(geom: Geometry, k: float, rows=None, cols=None, eta=2.0, near_tol=1e-13):
    """Dense blocks S, K, K', H (rows x cols) of the discrete operators."""
    N = geom.n_elem
    rows = np.arange(N) if rows is None else np.asarray(rows)
    cols = np.arange(N) if cols is None else np.asarray(cols)
    x = geom.cen[rows][:, None, None, :]
    nx = geom.normal[rows][:, None, None, :]
    y = geom.qpts[cols][None, :, :, :]
    ny = geom.normal[cols][None, :, None, :]
    w = geom.qw[cols][None, :, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        G, Gy, Gx, Gxy = kernels(x, nx, y, ny, k)
    blocks = [(G * w).sum(2), (Gy * w).sum(2), (Gx * w).sum(2), (Gxy * w).sum(2)]
    # near pairs: exact integrals
    nm = near_mask(geom, rows, cols, eta)
    ri, cj = np.nonzero(nm)
    if len(ri):
        gi, gj = rows[ri], cols[cj]
        vals = near_integrals_parallel(geom.cen[gi], geom.normal[gi], geom.a[gj], geom.b[gj],
                                       geom.c[gj], geom.normal[gj], k, tol=near_tol)
        for t in range(4):
            blocks[t][ri, cj] = vals[:, t]
    # self pairs
    same = rows[:, None] == cols[None, :]
    si, sj = np.nonzero(same)
    if len(si):
        S_ii, H_ii = self_terms(geom, k, rows[si])
        blocks[0][si, sj] = S_ii
        blocks[1][si, sj] = 0.0
        blocks[2][si, sj] = 0.0
        blocks[3][si, sj] = H_ii
    return blocks


def bm_blocks(geom: Geometry, k: float, alpha: complex, rows=None, cols=None, eta=2.0):
    """The two Burton-Miller blocks  Mp = I/2 - K - alpha H  and
    Mq = S + alpha K' + (alpha/2) I  restricted to rows x cols."""
    N = geom.n_elem
    rows = np.arange(N) if rows is None else np.asarray(rows)
    cols = np.arange(N) if cols is None else np.asarray(cols)
    S, K, Kp, H = assemble_block(geom, k, rows, cols, eta)
    eye = (rows[:, None] == cols[None, :]).astype(np.float64)
    Mp = 0.5 * eye - K - alpha * H
    Mq = S + alpha * Kp + 0.5 * alpha * eye
    return Mp, Mq


def matvec(geom: Geometry, k: float, alpha: complex, p, q=None, rows=None, eta=2.0, block=64):
    """y[rows] = Mp p + Mq q, assembled block-row by block-row (matrix-free)."""
    N = geom.n_elem
    rows = np.arange(N) if rows is None else np.asarray(rows)
    y = np.zeros(len(rows), dtype=np.complex128)
    for s in range(0, len(rows), block):
        r = rows[s:s + block]
        Mp, Mq = bm_blocks(geom, k, alpha, r, None, eta)
        y[s:s + block] = Mp @ p
        if q is not None:
            y[s:s + block] += Mq @ q
    return y


def matvec_adjoint(geom: Geometry, k: float, alpha: complex, yv, cols=None, eta=2.0, block=64):
    """u[cols] = (Mp^H y)[cols],  w[cols] = (Mq^H y)[cols], column blocks."""
    N = geom.n_elem
    cols = np.arange(N) if cols is None else np.asarray(cols)
    u = np.zeros(len(cols), dtype=np.complex128)
    w = np.zeros(len(cols), dtype=np.complex128)
    for s in range(0, len(cols), block):
        c = cols[s:s + block]
        Mp, Mq = bm_blocks(geom, k, alpha, None, c, eta)
        u[s:s + block] = Mp.conj().T @ yv
        w[s:s + block] = Mq.conj().T @ yv
    return u, w


def plane_wave_rhs(geom: Geometry, k: float, alpha: complex, d):
    """b_i = p_inc(x_i) + alpha q_inc(x_i) for p_inc = exp(i k d.x), unit
    amplitude; q_inc = dp_inc/dn = i k (d.n) p_inc."""
    d = np.asarray(d, dtype=np.float64)
    ph = np.exp(1j * k * (geom.cen @ d))
    return ph + alpha * (1j * k * (geom.normal @ d)) * ph


def point_source_rhs(geom: Geometry, k: float, alpha: complex, src, amp):
    """Right-hand side of point sources of intensity A_m at y_m (the paper's
    forward problem, Eq. hel: Helmholtz equation with sum_m A_m delta(x - y_m),
    whose incident field is p_inc(x) = sum_m A_m G(x - y_m)):
    b_i = p_inc(x_i) + alpha dp_inc/dn(x_i), dp_inc/dn = sum_m A_m dG/dn_x."""
    src = np.asarray(src, dtype=np.float64).reshape(-1, 3)
    amp = np.asarray(amp, dtype=np.complex128).reshape(-1)
    x = geom.cen[:, None, :]
    nx = geom.normal[:, None, :]
    y = src[None, :, :]
    G, _, Gx, _ = kernels(x, nx, y, np.zeros_like(y), k)
    return (G * amp[None, :]).sum(1) + alpha * (Gx * amp[None, :]).sum(1)
