"""Interaction lists by cross-level level marching (Sec. II.B).

Oracle code (test infrastructure only).

Admissibility (eq. 4): boxes a, b are well separated when
    R + theta * r <= theta * d,
R the larger and r the smaller of the two radii and d the distance of the
centres.  Reading: a pair with d = 0 is never admissible (the expansions are
singular there; this only matters for boxes whose points all coincide).

Level marching (Sec. II.B, enumerated rules after eq. 5): start with the pair
(root, root) at source level 0 and target level 0, then repeatedly
  * refine the side whose level has the larger average box radius;
  * on equal averages refine the source side (rule 2; the ``tie`` argument
    can select the target side instead);
  * when one side has no more levels, refine the other (rule 3);
  * after each refinement every admissible pair leaves the working set and
    joins the M2L list;
  * stop when the working set is empty or both sides are at the leaf level
    (rule 4).
The pairs left at the end are leaf-leaf pairs evaluated directly (P2P,
including each leaf with itself).
Reading: "average box radius" is the arithmetic mean of the radii of all
boxes of the level, summed sequentially in box order.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .tree import Tree


def admissible(ca, ra, cb, rb, theta):
    """Eq. (4) for arrays of box pairs: R + theta*r <= theta*d and d > 0."""
    dx = ca[..., 0] - cb[..., 0]
    dy = ca[..., 1] - cb[..., 1]
    dz = ca[..., 2] - cb[..., 2]
    d = np.sqrt(dx * dx + dy * dy + dz * dz)
    big = np.maximum(ra, rb)
    small = np.minimum(ra, rb)
    return (big + theta * small <= theta * d) & (d > 0.0)


def level_mean_radius(tree: Tree):
    """Arithmetic mean radius of each level, summed in box order."""
    out = []
    for l in range(tree.L + 1):
        acc = 0.0
        for r in tree.radius[tree.level_off[l]:tree.level_off[l + 1]].tolist():
            acc += r
        out.append(acc / float(tree.level_off[l + 1] - tree.level_off[l]))
    return out


@dataclass
class Lists:
    """Interaction lists, as global box ids sorted by (target, source).

    m2l_src/m2l_tgt -- admissible pairs (any levels)
    p2p_src/p2p_tgt -- leaf-leaf pairs, as leaf indices (0 .. 2^{Ls}-1)
    steps           -- the sequence of (source level, target level) visited
    """

    m2l_src: np.ndarray
    m2l_tgt: np.ndarray
    p2p_src: np.ndarray
    p2p_tgt: np.ndarray
    steps: list


def build_lists(tree: Tree, theta: float, tie: str = "src", mode: str = "cross") -> Lists:
    """Level-marching lists for sources = targets (``mode`` as in
    ``build_lists_st``)."""
    return build_lists_st(tree, tree, theta, tie, mode)


def build_lists_st(stree: Tree, ttree: Tree, theta: float, tie: str = "src",
                   mode: str = "cross") -> Lists:
    """Cross-level level-marching lists between a source hierarchy and a
    target hierarchy (Sec. II.B, the generalisation to separate sources and
    targets): source boxes of level ls are tested against target boxes of
    level lt, the march choosing which level to refine from the two trees'
    own level-mean radii; a tree that has reached its leaves stops being
    refined, so the trees may differ in depth.  M2L pairs are global box ids
    of their own trees (source id in ``stree``, target id in ``ttree``);
    P2P pairs are leaf indices of their own trees.

    ``mode="same"`` gives the same-level lists of the enumerated procedure
    at the start of Sec. II.B (the lists of Engblom's criterion): every step
    refines both sides, so boxes are only ever compared with boxes of their
    own level, and the children of well-separated pairs are skipped; once
    one tree has reached its leaves only the other is refined."""
    Ls, Lt = stree.L, ttree.L
    ns, nt = 1 << stree.s, 1 << ttree.s
    offs, offt = stree.level_off, ttree.level_off
    avg_s, avg_t = level_mean_radius(stree), level_mean_radius(ttree)
    src = np.zeros(1, dtype=np.int64)  # box index within its level
    tgt = np.zeros(1, dtype=np.int64)
    ls = lt = 0
    steps = [(0, 0)]
    m2l_s, m2l_t = [], []
    # Reading: the march starts by testing the pair of roots itself (two
    # separate hierarchies can be well separated as a whole); with sources =
    # targets the roots coincide (d = 0) and are never admissible.
    ok = admissible(stree.centre[:1], stree.radius[:1], ttree.centre[:1], ttree.radius[:1], theta)
    if ok[0]:
        m2l_s.append(np.zeros(1, np.int64))
        m2l_t.append(np.zeros(1, np.int64))
        src = tgt = np.zeros(0, np.int64)
    while len(src) and not (ls == Ls and lt == Lt):
        if ls == Ls:
            sides = ("tgt",)
        elif lt == Lt:
            sides = ("src",)
        elif mode == "same":
            sides = ("src", "tgt")
        elif avg_s[ls] > avg_t[lt]:
            sides = ("src",)
        elif avg_s[ls] < avg_t[lt]:
            sides = ("tgt",)
        else:
            sides = (tie,)
        for side in sides:
            if side == "src":
                src = (src[:, None] * ns + np.arange(ns)[None, :]).ravel()
                tgt = np.repeat(tgt, ns)
                ls += 1
            else:
                tgt = (tgt[:, None] * nt + np.arange(nt)[None, :]).ravel()
                src = np.repeat(src, nt)
                lt += 1
        steps.append((ls, lt))
        gs, gt = src + offs[ls], tgt + offt[lt]
        ok = admissible(stree.centre[gs], stree.radius[gs],
                        ttree.centre[gt], ttree.radius[gt], theta)
        m2l_s.append(gs[ok])
        m2l_t.append(gt[ok])
        src, tgt = src[~ok], tgt[~ok]
    m2l_s = np.concatenate(m2l_s) if m2l_s else np.zeros(0, np.int64)
    m2l_t = np.concatenate(m2l_t) if m2l_t else np.zeros(0, np.int64)
    o = np.lexsort((m2l_s, m2l_t))
    m2l_s, m2l_t = m2l_s[o], m2l_t[o]
    if ls != Ls or lt != Lt:
        # the working set emptied before the leaf levels: nothing is direct
        src = tgt = np.zeros(0, np.int64)
    o = np.lexsort((src, tgt))
    return Lists(m2l_src=m2l_s, m2l_tgt=m2l_t, p2p_src=src[o], p2p_tgt=tgt[o],
                 steps=steps)


def csr(tgt: np.ndarray, src: np.ndarray, ntgt: int):
    """CSR arrays (ptr[ntgt+1], src) of a list sorted by target."""
    ptr = np.zeros(ntgt + 1, dtype=np.int64)
    np.add.at(ptr, tgt + 1, 1)
    return np.cumsum(ptr), src
