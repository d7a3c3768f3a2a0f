"""Morton order and uniform-depth octree, in Python integers (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper uses an FMM (Sec. 2.3) without stating its tree; this is the
reading the GPU path must reproduce bit for bit:

* bounding cube over the collocation points (element centroids):
  per axis mn, mx; centre c = (mn + mx) / 2; half side
  R0 = 0.5 * max_axis(mx - mn) * (1 + 2^-10); lower corner lo = c - R0;
  scale s = 2^20 / R0 (= 2^21 / (2 R0)); all in float64, each operation
  rounded separately (no fused multiply-add);
* integer coordinate q_a = clamp(floor((x_a - lo_a) * s), 0, 2^21 - 1);
* key bit 3b+2 <- x bit b, 3b+1 <- y bit b, 3b <- z bit b (b = 0..20);
* elements sorted stably by (key, original index);
* the box of a point at level l is key >> 3 (21 - l); all leaves sit at one
  level L (uniform depth), chosen as the smallest L >= 2 whose fullest leaf
  holds at most ``leaf_cap`` elements (at most level 21), but no finer than
  the largest level l >= 2 whose box side h_l = 2 R0 / 2^l exceeds
  eta * (longest element edge), so that near pairs lie in adjacent leaves
  whenever the mesh allows it;
* lists, per level l >= 2, over non-empty boxes only:
  colleagues(b)  = boxes at level l with max_a |i_a(b) - i_a(c)| <= 1;
  V(b)           = children of colleagues(parent(b)) that are not
                   colleagues of b (multipole-to-local partners);
  U(b), b a leaf = colleagues(b) (direct near-field partners).
"""
from __future__ import annotations

import math

import numpy as np

NBITS = 21
QMAX = (1 << NBITS) - 1


def bounding_cube(cen: np.ndarray):
    mn = [float(v) for v in cen.min(axis=0)]
    mx = [float(v) for v in cen.max(axis=0)]
    ext = max(mx[a] - mn[a] for a in range(3))
    R0 = (0.5 * ext) * (1.0 + 2.0 ** -10)
    lo = [(mn[a] + mx[a]) / 2.0 - R0 for a in range(3)]
    s = 2.0 ** 20 / R0
    return lo, s, R0


def quantise(cen: np.ndarray):
    lo, s, _ = bounding_cube(cen)
    q = []
    for p in cen:
        row = []
        for a in range(3):
            t = math.floor((float(p[a]) - lo[a]) * s)
            row.append(min(max(t, 0), QMAX))
        q.append(row)
    return q


def interleave(qx: int, qy: int, qz: int) -> int:
    key = 0
    for b in range(NBITS):
        key |= ((qx >> b) & 1) << (3 * b + 2)
        key |= ((qy >> b) & 1) << (3 * b + 1)
        key |= ((qz >> b) & 1) << (3 * b)
    return key


def deinterleave(key: int, nbits: int = NBITS):
    qx = qy = qz = 0
    for b in range(nbits):
        qx |= ((key >> (3 * b + 2)) & 1) << b
        qy |= ((key >> (3 * b + 1)) & 1) << b
        qz |= ((key >> (3 * b)) & 1) << b
    return qx, qy, qz


def morton_keys(cen: np.ndarray):
    return [interleave(*row) for row in quantise(cen)]


def sort_order(keys):
    return sorted(range(len(keys)), key=lambda i: (keys[i], i))


def choose_leaf_level(sorted_keys, leaf_cap: int) -> int:
    for L in range(2, NBITS + 1):
        sh = 3 * (NBITS - L)
        counts = {}
        for kk in sorted_keys:
            b = kk >> sh
            counts[b] = counts.get(b, 0) + 1
        if max(counts.values()) <= leaf_cap:
            return L
    return NBITS


class Tree:
    """Uniform-depth octree over Morton-sorted elements."""

    def __init__(self, cen: np.ndarray, leaf_cap: int = 32, leaf_level: int | None = None,
                 ell_max: float | None = None, eta: float = 2.0):
        self.keys = morton_keys(cen)
        self.perm = sort_order(self.keys)
        sk = [self.keys[i] for i in self.perm]
        self.sorted_keys = sk
        self.L = choose_leaf_level(sk, leaf_cap) if leaf_level is None else max(2, leaf_level)
        if ell_max is not None:
            _, _, R0 = bounding_cube(cen)
            L_near = 2
            for l in range(2, NBITS + 1):
                if 2.0 * R0 / float(1 << l) > eta * ell_max:
                    L_near = l
            self.L = min(self.L, L_near)
        # boxes per level: sorted unique box keys
        self.boxes = {}
        for l in range(0, self.L + 1):
            sh = 3 * (NBITS - l)
            seen = []
            for kk in sk:
                b = kk >> sh
                if not seen or seen[-1] != b:
                    seen.append(b)
            self.boxes[l] = seen
        # leaf ranges [start, end) in sorted order
        sh = 3 * (NBITS - self.L)
        self.leaf_start, self.leaf_end = [], []
        for i, kk in enumerate(sk):
            b = kk >> sh
            if i == 0 or (sk[i - 1] >> sh) != b:
                self.leaf_start.append(i)
                if i:
                    self.leaf_end.append(i)
        self.leaf_end.append(len(sk))

    @staticmethod
    def coords(bkey: int, level: int):
        return deinterleave(bkey, level)

    def _present(self, level: int):
        if not hasattr(self, "_sets"):
            self._sets = {}
        if level not in self._sets:
            self._sets[level] = set(self.boxes[level])
        return self._sets[level]

    def colleagues(self, level: int, bkey: int):
        """Non-empty boxes at ``level`` whose integer coordinates differ from
        those of ``bkey`` by at most one on every axis (itself included)."""
        bx, by, bz = self.coords(bkey, level)
        present = self._present(level)
        side = 1 << level
        out = []
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    cx, cy, cz = bx + dx, by + dy, bz + dz
                    if 0 <= cx < side and 0 <= cy < side and 0 <= cz < side:
                        c = interleave(cx, cy, cz)
                        if c in present:
                            out.append(c)
        return sorted(out)

    def vlist(self, level: int, bkey: int):
        """Multipole-to-local partners of box ``bkey`` at ``level`` (>= 2)."""
        mine = set(self.colleagues(level, bkey))
        present = self._present(level)
        out = []
        for pc in self.colleagues(level - 1, bkey >> 3):
            for ch in range(8):
                c = (pc << 3) | ch
                if c in present and c not in mine:
                    out.append(c)
        return sorted(out)

    def ulist(self, bkey: int):
        return self.colleagues(self.L, bkey)
