"""Balanced median-split 2^s tree (Sec. II.A, steps 1-4; Listing 2).

Oracle code (test infrastructure only).

Each box is split s times in a row by a binary median split; each binary
split
  1. takes the extent (max - min) of the box's points along x, y, z and picks
     the longest axis (Sec. II.A step 1; Listing 2 takes the first axis of
     equal maxima, as ``argmax`` does -- Reading: first axis wins ties);
  2. orders the points along that axis and gives the lower half the points
     below the median and the upper half those above (step 2).
     Reading: points are ordered by (coordinate, original index), and the
     lower child takes the first ceil(n/2) of them.  For rows without
     padding this is exactly the argpartition-at-n//2, pad-to-even, halve
     sequence of Listing 2; the result satisfies the balance property of
     Sec. II.A (boxes of level l hold ceil(N/2^{ls}) or floor(N/2^{ls})
     points).
Levels are added until every box holds at most N_max points (step 4):
the depth L is the smallest L with ceil(N / 2^{Ls}) <= N_max, optionally
capped at ``max_depth``.  Children of box b (level numbering) are
b * 2^s + c, c = 0 .. 2^s-1, in the order the binary splits produce them,
which is the row order of Listing 2's reshape.  Within each leaf, points are
sorted by original index (the final ``sort`` of Listing 2).

Box geometry (used by the admissibility test, eq. 4).  Reading: the paper
does not define centre and radius; a box's centre is the midpoint of the
tight bounding box of its points and its radius is half of that bounding
box's diagonal.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def tree_depth(n: int, leaf_max: int, s: int, max_depth: int = 64) -> int:
    """Smallest L with ceil(n / 2^{L s}) <= leaf_max, capped at max_depth
    (Sec. II.A step 4)."""
    L = 0
    while L < max_depth and -(-n // (1 << (L * s))) > leaf_max:
        L += 1
    return L


@dataclass
class Tree:
    """A built tree.

    perm        -- int64[N]; leaf-ordered slot i holds input point perm[i]
    leaf_start  -- int64[2^{Ls}+1]; points of leaf j are perm[leaf_start[j]:
                   leaf_start[j+1]]
    L, s        -- depth and splits per level
    level_off   -- int64[L+2]; global id of box b at level l is
                   level_off[l] + b
    centre      -- f64[B,3]; radius -- f64[B]   (B = level_off[L+1])
    """

    perm: np.ndarray
    leaf_start: np.ndarray
    L: int
    s: int
    level_off: np.ndarray
    centre: np.ndarray
    radius: np.ndarray

    @property
    def nbox(self) -> int:
        return int(self.level_off[-1])

    @property
    def nleaf(self) -> int:
        return 1 << (self.L * self.s)

    def box_range(self, level: int, b: int):
        """[start, end) of box b of ``level`` in leaf order."""
        k = 1 << (self.s * (self.L - level))
        return int(self.leaf_start[b * k]), int(self.leaf_start[(b + 1) * k])

    def level_of(self, gid: int) -> int:
        return int(np.searchsorted(self.level_off, gid, side="right") - 1)


def _level_offsets(L: int, s: int) -> np.ndarray:
    off = [0]
    for l in range(L + 1):
        off.append(off[-1] + (1 << (s * l)))
    return np.array(off, dtype=np.int64)


def split_order_recursive(pos: np.ndarray, L: int, s: int):
    """Plain recursive form of the splitting, for small inputs.

    Returns the list of leaves (each an ascending array of original indices)
    in tree order.  One function call per binary split."""
    def split(idx: np.ndarray, depth: int):
        if depth == L * s:
            return [np.sort(idx)]
        pts = pos[idx]
        ext = pts.max(axis=0) - pts.min(axis=0)
        ax = int(np.argmax(ext))  # first axis wins ties
        order = np.lexsort((idx, pts[:, ax]))  # by coordinate, then index
        half = (len(idx) + 1) // 2
        lo, hi = idx[order[:half]], idx[order[half:]]
        return split(lo, depth + 1) + split(hi, depth + 1)

    return split(np.arange(len(pos), dtype=np.int64), 0)


def split_order(pos: np.ndarray, L: int, s: int):
    """The same splitting as :func:`split_order_recursive`, done for all boxes
    of one binary-split depth at once.  Returns (perm, leaf_start)."""
    n = len(pos)
    order = np.arange(n, dtype=np.int64)
    seg_start = np.array([0, n], dtype=np.int64)  # boundaries of segments
    for _ in range(L * s):
        nseg = len(seg_start) - 1
        cnt = np.diff(seg_start)
        seg_id = np.repeat(np.arange(nseg), cnt)
        pts = pos[order]
        lo = np.minimum.reduceat(pts, seg_start[:-1], axis=0)
        hi = np.maximum.reduceat(pts, seg_start[:-1], axis=0)
        ax = np.argmax(hi - lo, axis=1)  # first axis wins ties
        key = pts[np.arange(n), ax[seg_id]]
        o = np.lexsort((order, key, seg_id))  # segment, coordinate, index
        order = order[o]
        half = (cnt + 1) // 2
        mid = seg_start[:-1] + half
        new = np.empty(2 * nseg + 1, dtype=np.int64)
        new[0:-1:2] = seg_start[:-1]
        new[1::2] = mid
        new[-1] = n
        seg_start = new
    # within each leaf, ascending original index
    nseg = len(seg_start) - 1
    seg_id = np.repeat(np.arange(nseg), np.diff(seg_start))
    order = order[np.lexsort((order, seg_id))]
    return order, seg_start


def box_geometry(pos_leaf: np.ndarray, starts: np.ndarray):
    """Centre and radius of boxes given as contiguous ranges of leaf-ordered
    points (Reading: bbox midpoint and half the bbox diagonal)."""
    lo = np.minimum.reduceat(pos_leaf, starts[:-1], axis=0)
    hi = np.maximum.reduceat(pos_leaf, starts[:-1], axis=0)
    centre = 0.5 * (lo + hi)
    e = hi - lo
    radius = 0.5 * np.sqrt(e[:, 0] * e[:, 0] + e[:, 1] * e[:, 1] + e[:, 2] * e[:, 2])
    return centre, radius


def build_tree(pos: np.ndarray, leaf_max: int, s: int = 2,
               max_depth: int = 64, recursive: bool = False) -> Tree:
    """Build the tree and the geometry of every box at every level."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = len(pos)
    if n < 1:
        raise ValueError("need at least one point")
    if leaf_max < (1 << s):
        raise ValueError("leaf_max must be >= 2^s so that no box is empty")
    L = tree_depth(n, leaf_max, s, max_depth)
    if recursive:
        leaves = split_order_recursive(pos, L, s)
        perm = np.concatenate(leaves)
        leaf_start = np.concatenate([[0], np.cumsum([len(x) for x in leaves])])
    else:
        perm, leaf_start = split_order(pos, L, s)
    leaf_start = leaf_start.astype(np.int64)
    off = _level_offsets(L, s)
    pos_leaf = pos[perm]
    centre = np.empty((off[-1], 3))
    radius = np.empty(off[-1])
    for l in range(L + 1):
        k = 1 << (s * (L - l))
        starts = leaf_start[::k]
        c, r = box_geometry(pos_leaf, starts)
        centre[off[l]:off[l + 1]] = c
        radius[off[l]:off[l + 1]] = r
    return Tree(perm=perm.astype(np.int64), leaf_start=leaf_start, L=L, s=s,
                level_off=off, centre=centre, radius=radius)
