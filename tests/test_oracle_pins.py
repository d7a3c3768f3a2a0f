"""Pins for oracle pieces that the other CPU tests reach only indirectly.

* ``tree.bounding_cube`` / ``quantise``: the extreme centroids of the widest
  axis land a fixed distance (2^10 / (1 + 2^-10) units) inside [0, 2^21) and
  the axis spans 2^21 / (1 + 2^-10) units; the mid-point of a narrower axis
  maps to the cube's centre, 2^20.  A factor-2 slip in the scale, a wrong
  half side or a shifted lower corner breaks these by thousands of units.
* ``Tree(..., ell_max=...)``: the leaf level is clamped to the largest level
  whose box side exceeds eta times the longest edge (derived here from a
  logarithm, independently of the oracle's loop), and with that clamp every
  near pair of ``bem.near_mask`` lies in neighbouring leaves (the property the
  clamp exists for), also on meshes where the clamp binds.
* ``bem.near_mask`` against a plain loop over pairs.
* ``bem.matvec`` / ``bem.matvec_adjoint`` (the row- and column-block
  wrappers every full-scale parity test uses as reference) against the dense
  blocks of ``bem.bm_blocks`` with p and q both non-zero.
"""
import math

import numpy as np
import pytest

from oracle import bem, tree
from workloads import complex_normal, cube_surface, icosphere

SPAN = 2.0 ** 21 / (1.0 + 2.0 ** -10)     # quantised width of the widest axis
MARGIN = 2.0 ** 10 / (1.0 + 2.0 ** -10)   # distance of its extremes from 0 / 2^21


def _cases():
    V, T = icosphere(2)
    Vc, Tc = cube_surface(5)
    Ve, Te = icosphere(2)
    Ve = Ve * np.array([1.7, 0.6, 1.1]) + np.array([0.3, -2.0, 5.0])
    return {"ico2": (V, T), "cube5": (Vc, Tc), "ellipsoid": (Ve, Te)}


@pytest.mark.parametrize("name", ["ico2", "cube5", "ellipsoid"])
def test_quantisation_extremes_and_centre(name):
    V, T = _cases()[name]
    cen = V[T].mean(axis=1)
    q = np.array(tree.quantise(cen), dtype=np.float64)
    ext = cen.max(axis=0) - cen.min(axis=0)
    wide = int(np.argmax(ext))
    lo, hi = q[:, wide].min(), q[:, wide].max()
    # floor() moves each end by less than one unit
    assert abs(lo - MARGIN) <= 1.0, (lo, MARGIN)
    assert abs(hi - (MARGIN + SPAN)) <= 1.0, (hi, MARGIN + SPAN)
    assert hi - lo >= 2.0 ** 21 * (1.0 - 2.0 ** -9)
    assert hi <= tree.QMAX and lo >= 0          # no clamping needed
    for a in range(3):
        # the axis mid-point sits at the cube centre: q of mn and mx straddle
        # 2^20 symmetrically (to rounding), whatever the axis width
        mid = 0.5 * (q[:, a].min() + q[:, a].max())
        assert abs(mid - 2.0 ** 20) <= 1.0, (a, mid)
        # widths scale with the axis extent: s = 2^21 / (2 R0)
        span_a = q[:, a].max() - q[:, a].min()
        assert abs(span_a - SPAN * ext[a] / ext[wide]) <= 2.0, (a, span_a)


def _leaf_of(t, i_sorted):
    sh = 3 * (tree.NBITS - t.L)
    return t.sorted_keys[i_sorted] >> sh


def _check_near_pairs_in_colleague_leaves(V, T, eta=2.0, cap=1):
    g = bem.Geometry(V, T)
    ell = float(g.ell.max())
    t = tree.Tree(g.cen, leaf_cap=cap, ell_max=ell, eta=eta)
    # independent derivation of the clamp: largest l >= 2 with
    # 2 R0 / 2^l > eta * ell, i.e. l < log2(2 R0 / (eta ell))
    ext = float((g.cen.max(axis=0) - g.cen.min(axis=0)).max())
    R0 = 0.5 * ext * (1.0 + 2.0 ** -10)
    ratio = 2.0 * R0 / (eta * ell)
    l_near = max(2, math.ceil(math.log2(ratio)) - 1)
    assert 2.0 * R0 / 2 ** (l_near + 1) <= eta * ell
    occ = tree.choose_leaf_level(t.sorted_keys, cap)
    assert t.L == min(occ, l_near), (t.L, occ, l_near)
    if not 2.0 * R0 / 2 ** l_near > eta * ell:
        # even level-2 boxes are narrower than the near radius: such a mesh
        # has no far field (every pair is summed directly), nothing to check
        assert l_near == 2
        return t, occ, l_near
    # every near pair (target i, source j) lies in colleague leaves
    pos = np.empty(len(T), dtype=np.int64)
    pos[np.array(t.perm)] = np.arange(len(T))
    n = len(T)
    m = bem.near_mask(g, np.arange(n), np.arange(n), eta)
    ii, jj = np.nonzero(m)
    assert len(ii) > 0
    for i, j in zip(ii, jj):
        a = tree.Tree.coords(_leaf_of(t, pos[i]), t.L)
        b = tree.Tree.coords(_leaf_of(t, pos[j]), t.L)
        assert max(abs(a[0] - b[0]), abs(a[1] - b[1]), abs(a[2] - b[2])) <= 1, (i, j)
    return t, occ, l_near


@pytest.mark.parametrize("name", ["ico3", "cube12"])
def test_near_pairs_lie_in_colleague_leaves(name):
    V, T = icosphere(3) if name == "ico3" else cube_surface(12)
    # leaf_cap 1 asks for the finest level: the clamp decides the level
    t, occ, l_near = _check_near_pairs_in_colleague_leaves(V, T, cap=1)
    assert occ > l_near          # the clamp binds here
    assert t.L == l_near


def test_coarse_mesh_clamps_to_level_two():
    # cube8: level-2 boxes (side 0.5) are narrower than 2 x the face
    # diagonal (0.71): the level is clamped to 2 (the direct-sum case)
    V, T = cube_surface(8)
    t, occ, l_near = _check_near_pairs_in_colleague_leaves(V, T, cap=1)
    assert t.L == 2 and l_near == 2


def test_near_pairs_clamp_binds_on_a_graded_mesh():
    # a cube whose one face is refined more finely than the others: the
    # longest edge sets the clamp while the occupancy rule wants finer leaves
    V, T = cube_surface(6)
    V = V.copy()
    V[:, 2] = np.sign(V[:, 2]) * np.abs(V[:, 2]) ** 1.5
    t, occ, l_near = _check_near_pairs_in_colleague_leaves(V, T, cap=4)
    assert t.L == min(occ, l_near)


def test_near_mask_equals_plain_loop():
    V, T = icosphere(2)
    g = bem.Geometry(V, T)
    n = len(T)
    rng = np.random.default_rng(7)
    rows = np.sort(rng.choice(n, 60, replace=False))
    cols = np.arange(n)
    got = bem.near_mask(g, rows, cols, eta=2.0)
    for a, i in enumerate(rows):
        for b, j in enumerate(cols):
            d2 = sum((float(g.cen[i][c]) - float(g.cen[j][c])) ** 2 for c in range(3))
            want = (i != j) and d2 < (2.0 * float(g.ell[j])) ** 2
            assert bool(got[a, b]) == want, (i, j)
    assert got.sum() > len(rows)      # the rows do have near pairs


def test_row_and_column_wrappers_equal_dense_blocks():
    V, T = icosphere(2)
    g = bem.Geometry(V, T)
    k, alpha = 1.7, 0.3 + 0.5j
    n = len(T)
    Mp, Mq = bem.bm_blocks(g, k, alpha)
    rng = np.random.default_rng(11)
    p, q, yv = complex_normal(rng, n), complex_normal(rng, n), complex_normal(rng, n)
    rows = np.sort(rng.choice(n, 45, replace=False))
    y = bem.matvec(g, k, alpha, p, q, rows=rows, block=7)
    ref = Mp[rows] @ p + Mq[rows] @ q
    assert np.linalg.norm(y - ref) <= 1e-14 * np.linalg.norm(ref)
    # without q: the p block alone
    y0 = bem.matvec(g, k, alpha, p, None, rows=rows, block=16)
    assert np.linalg.norm(y0 - Mp[rows] @ p) <= 1e-14 * np.linalg.norm(Mp[rows] @ p)
    # full matvec equals the dense product
    yf = bem.matvec(g, k, alpha, p, q, block=64)
    assert np.linalg.norm(yf - (Mp @ p + Mq @ q)) <= 1e-14 * np.linalg.norm(Mp @ p + Mq @ q)
    cols = np.sort(rng.choice(n, 30, replace=False))
    u, w = bem.matvec_adjoint(g, k, alpha, yv, cols=cols, block=9)
    assert np.linalg.norm(u - Mp.conj().T[cols] @ yv) <= 1e-14 * np.linalg.norm(u)
    assert np.linalg.norm(w - Mq.conj().T[cols] @ yv) <= 1e-14 * np.linalg.norm(w)
    # the identity terms sit on the diagonal of the two blocks
    S, K, Kp, H = bem.assemble_block(g, k)
    assert np.allclose(np.diag(Mp), 0.5 - np.diag(K) - alpha * np.diag(H), rtol=0, atol=1e-15)
    assert np.allclose(np.diag(Mq), np.diag(S) + alpha * np.diag(Kp) + 0.5 * alpha, rtol=0,
                       atol=1e-15)
