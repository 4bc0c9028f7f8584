"""Hierarchical boxes, neighbour lists and interaction lists (Theory section).

The paper partitions the system into boxes, each divided again, down to a
lowest level of about 2 bohr; the depth and the near/far parameters are left
to the implementation.  This oracle takes the following readings:

* Root (split dimensions only): E = largest extent of the pair centres over the
  split dimensions, delta = 0.05 E + 1 bohr, lo_d = min_d - 0.35 delta,
  width W = E + delta (cubic over the split dimensions).  Dimensions that are
  not split hold a single layer whose centre is the midpoint of the pair
  centres' range.
* ``depth`` subdivisions: level l has 2**l boxes per split dimension, box
  size h_l = W / 2**l; leaf index floor((x - lo)/h_depth), clamped.  A pair
  centre closer than 1e-8 h to a leaf boundary is rejected as ambiguous.
* Empty boxes are pruned.  Two boxes of one level are near when the Chebyshev
  distance of their integer indices is <= ws.
* Interaction list: the non-near boxes of the same level whose parents are
  near the box's parent.  Leaf pairs that are near are the near field and are
  not part of K^ff.

Extent rule (the paper's criterion: two charge distributions are separated
when the distance of their centres exceeds the sum of their extents, with a
slack ws): given the extent e_k of every pair distribution, the extent of a
box is the largest |P_k - X_box| + e_k over the distributions whose centres
lie in it; two boxes of one level are far when |X_a - X_b| > (1 + ws)(e_a +
e_b) and near otherwise.  Near lists are formed top down: the root is near
itself, and a box's candidates are the children of its parent's near boxes;
a candidate far from the box enters its interaction list, the others its
near list.
"""
from __future__ import annotations

import math

import numpy as np


class Tree:
    def __init__(self, centres: np.ndarray, split_mask: int, depth: int, ws, extents=None):
        centres = np.asarray(centres, dtype=np.float64)
        self.depth, self.ws = int(depth), ws
        self.split = [d for d in range(3) if (split_mask >> d) & 1]
        if not self.split:
            raise ValueError("no split dimension")
        mn, mx = centres.min(0), centres.max(0)
        E = max(mx[d] - mn[d] for d in self.split)
        delta = 0.05 * E + 1.0
        self.lo = np.zeros(3)
        self.mid = 0.5 * (mn + mx)
        for d in self.split:
            self.lo[d] = mn[d] - 0.35 * delta
        self.W = E + delta
        nside = 1 << depth
        hleaf = self.W / nside
        coords = np.zeros((len(centres), 3), dtype=np.int64)
        for d in self.split:
            u = (centres[:, d] - self.lo[d]) / hleaf
            f = np.floor(u)
            frac = u - f
            if np.any(np.minimum(frac, 1.0 - frac) < 1e-8):
                raise ValueError("pair centre on a leaf boundary")
            coords[:, d] = np.clip(f.astype(np.int64), 0, nside - 1)
        self.pair_leaf_coord = coords
        # boxes per level: sorted integer coordinates -> id
        self.boxes: list[list[tuple]] = []
        self.index: list[dict] = []
        for lev in range(depth + 1):
            sh = depth - lev
            cs = sorted({tuple(int(v) >> sh for v in c) for c in coords})
            self.boxes.append(cs)
            self.index.append({c: k for k, c in enumerate(cs)})
        leafidx = self.index[depth]
        self.pair_leaf = np.array([leafidx[tuple(int(v) for v in c)] for c in coords], dtype=np.int64)
        # interaction lists
        self.il: list[list[list[int]]] = [[[] for _ in self.boxes[lev]] for lev in range(depth + 1)]
        if extents is not None:
            self._extent_lists(centres, coords, np.asarray(extents, dtype=np.float64), float(ws))
            levels = [lev for lev in range(depth + 1) if any(self.il[lev][b] for b in range(len(self.boxes[lev])))]
            self.lmin = min(levels) if levels else None
            return
        for lev in range(1, depth + 1):
            for b, c in enumerate(self.boxes[lev]):
                pc = tuple(v >> 1 for v in c)
                for b2, c2 in enumerate(self.boxes[lev]):
                    pc2 = tuple(v >> 1 for v in c2)
                    if self.near(pc, pc2) and not self.near(c, c2):
                        self.il[lev][b].append(b2)
        levels = [lev for lev in range(depth + 1) if any(self.il[lev][b] for b in range(len(self.boxes[lev])))]
        self.lmin = min(levels) if levels else None

    def _extent_lists(self, centres, coords, extents, ws):
        D = self.depth
        self.box_ext = []
        for lev in range(D + 1):
            sh = D - lev
            ext = np.zeros(len(self.boxes[lev]))
            for k in range(len(centres)):
                b = self.index[lev][tuple(int(v) >> sh for v in coords[k])]
                d = np.linalg.norm(centres[k] - self.centre(lev, self.boxes[lev][b]))
                ext[b] = max(ext[b], d + extents[k])
            self.box_ext.append(ext)
        self.near_list = [[[0]]]
        for lev in range(1, D + 1):
            nl = []
            for b, c in enumerate(self.boxes[lev]):
                mine = []
                Xb = self.centre(lev, c)
                for q in self.near_list[lev - 1][self.parent(lev, b)]:
                    qc = self.boxes[lev - 1][q]
                    for b2, c2 in enumerate(self.boxes[lev]):
                        if tuple(v >> 1 for v in c2) != qc:
                            continue
                        dist = np.linalg.norm(Xb - self.centre(lev, c2))
                        if dist > (1.0 + ws) * (self.box_ext[lev][b] + self.box_ext[lev][b2]):
                            self.il[lev][b].append(b2)
                        else:
                            mine.append(b2)
                self.il[lev][b].sort()
                nl.append(sorted(mine))
            self.near_list.append(nl)

    def near_leaves(self, leaf: int) -> list:
        """Leaves near the given leaf (itself included): the near field."""
        if hasattr(self, "near_list"):
            return list(self.near_list[self.depth][leaf])
        c = self.boxes[self.depth][leaf]
        return [b for b, c2 in enumerate(self.boxes[self.depth]) if self.near(c, c2)]

    def near(self, c1, c2) -> bool:
        return max(abs(c1[d] - c2[d]) for d in range(3)) <= self.ws

    def h(self, lev: int) -> float:
        return self.W / (1 << lev)

    def centre(self, lev: int, c) -> np.ndarray:
        x = self.mid.copy()
        for d in self.split:
            x[d] = self.lo[d] + (c[d] + 0.5) * self.h(lev)
        return x

    def parent(self, lev: int, b: int) -> int:
        c = self.boxes[lev][b]
        return self.index[lev - 1][tuple(v >> 1 for v in c)]

    def ancestor(self, lev: int, leaf: int) -> int:
        c = self.boxes[self.depth][leaf]
        sh = self.depth - lev
        return self.index[lev][tuple(v >> sh for v in c)]

    def n_il(self) -> int:
        return sum(len(x) for lev in self.il for x in lev)

    def far_level(self, leaf1: int, leaf2: int):
        """Level at which the ancestors of two leaves are in each other's
        interaction list, or None when the leaves are near (near field)."""
        for lev in range(1, self.depth + 1):
            a, b = self.ancestor(lev, leaf1), self.ancestor(lev, leaf2)
            if b in self.il[lev][a]:
                return lev
        return None
