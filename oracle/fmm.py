"""The FMM evaluation pass assembled from its definitions (Sec. II; stage
list of Sec. III.A).

Oracle code (test infrastructure only).

Same tree (Sec. II.A), same lists (Sec. II.B) and same order p as the GPU
path, but a different route to the same truncated result:

1. multipoles C of EVERY box by direct P2M about that box's centre (eq. 10,
   real form of Sec. II.C).  Equal to the M2M route because M2M is an exact
   re-centring of the degree-<=p multipole (App. B.3, M2M);
2. for every listed pair (a -> b), the direct O(p^4) multipole-to-local
   operator (``translations.m2l``), summed into D_b;
3. the far field at a point x in leaf lambda is the sum, over every box b
   on the path from the root to lambda, of the local expansion D_b
   evaluated at x about c_b.  Equal to the L2L route because L2L re-centres
   a degree-<=p local expansion exactly (App. B.3, L2L);
4. the near field is the direct sum over the P2P list, without r = 0 pairs;
5. u = far + near, field = -grad u.

With separate sources and targets (Sec. II.B, the generalisation to two
hierarchies) the same steps run on two trees: multipoles on the source tree,
locals and the far field on the target tree, the lists pairing boxes (and
leaves) of the two.
"""
from __future__ import annotations

import math

import numpy as np

from .basis import ncoef, regular
from .direct import FOUR_PI
from .expansions import eval_local
from .lists import Lists, build_lists, build_lists_st
from .translations import m2l
from .tree import Tree, build_tree


def multipoles(tree: Tree, pos: np.ndarray, q: np.ndarray, p: int,
               boxes: np.ndarray | None = None, chunk: int = 1 << 15) -> np.ndarray:
    """C[B, (p+1)^2]: direct P2M of every box (or of the global ids in
    ``boxes``; the others stay zero) about its own centre."""
    K = ncoef(p)
    C = np.zeros((tree.nbox, K))
    pl = pos[tree.perm]
    ql = q[tree.perm]
    leaf_of = np.repeat(np.arange(tree.nleaf), np.diff(tree.leaf_start))
    want = None
    if boxes is not None:
        want = np.zeros(tree.nbox, dtype=bool)
        want[np.asarray(boxes, dtype=np.int64)] = True
    for l in range(tree.L + 1):
        box = tree.level_off[l] + (leaf_of >> (tree.s * (tree.L - l)))
        sel = np.arange(len(pl)) if want is None else np.flatnonzero(want[box])
        for c0 in range(0, len(sel), chunk):
            ix = sel[c0:c0 + chunk]
            b = box[ix]
            d = pl[ix] - tree.centre[b]
            Rq = ql[ix, None] * regular(p, d[:, 0], d[:, 1], d[:, 2])
            cut = np.flatnonzero(np.diff(b)) + 1
            starts = np.concatenate([[0], cut])
            C[b[starts]] += np.add.reduceat(Rq, starts, axis=0)
    return C


def locals_from_m2l(tree: Tree, lists: Lists, C: np.ndarray, p: int,
                    targets_boxes: np.ndarray | None = None, chunk: int = 2048,
                    ttree: Tree | None = None):
    """D[B_t, (p+1)^2] = sum over listed (a -> b) of M2L(C_a; c_a - c_b);
    a is a box of ``tree`` and b of ``ttree`` (default the same tree)."""
    ttree = tree if ttree is None else ttree
    D = np.zeros((ttree.nbox, ncoef(p)))
    src, tgt = lists.m2l_src, lists.m2l_tgt
    if targets_boxes is not None:
        keep = np.isin(tgt, targets_boxes)
        src, tgt = src[keep], tgt[keep]
    for c0 in range(0, len(src), chunk):
        s = src[c0:c0 + chunk]
        t = tgt[c0:c0 + chunk]
        contrib = m2l(C[s], tree.centre[s] - ttree.centre[t], p)
        np.add.at(D, t, contrib)
    return D


def _ancestors(tree: Tree, leaf: np.ndarray):
    """Global ids of the boxes on the path root -> leaf, [L+1, len(leaf)]."""
    out = []
    for l in range(tree.L + 1):
        out.append(tree.level_off[l] + (leaf >> (tree.s * (tree.L - l))))
    return np.array(out)


def _evaluate(stree: Tree, spos: np.ndarray, q: np.ndarray, ttree: Tree, tpos: np.ndarray,
              lists: Lists, p: int, targets: np.ndarray, field: bool):
    """Steps 1-5 for the target points ``tpos[targets]`` of ``ttree`` and the
    charges ``q`` at the points ``spos`` of ``stree``."""
    nt = len(tpos)
    slot = np.empty(nt, dtype=np.int64)
    slot[ttree.perm] = np.arange(nt)
    tslot = slot[targets]
    tleaf = np.searchsorted(ttree.leaf_start, tslot, side="right") - 1
    anc = _ancestors(ttree, tleaf)
    need = np.unique(anc)
    srcs = np.unique(lists.m2l_src[np.isin(lists.m2l_tgt, need)])
    C = multipoles(stree, spos, q, p, boxes=srcs)
    D = locals_from_m2l(stree, lists, C, p, targets_boxes=need, ttree=ttree)
    x = tpos[targets]
    u = np.zeros(len(targets))
    g = np.zeros((len(targets), 3))
    for l in range(ttree.L + 1):
        b = anc[l]
        if field:
            uu, gg = eval_local(p, D[b], x, ttree.centre[b], grad=True)
            g += gg
        else:
            uu = eval_local(p, D[b], x, ttree.centre[b])
        u += uu
    # near field over the P2P list
    ptr = np.zeros(ttree.nleaf + 1, dtype=np.int64)
    np.add.at(ptr, lists.p2p_tgt + 1, 1)
    ptr = np.cumsum(ptr)
    pl, ql = spos[stree.perm], q[stree.perm]
    order = np.argsort(tleaf, kind="stable")
    for lam in np.unique(tleaf):
        sel = order[np.searchsorted(tleaf[order], lam):np.searchsorted(tleaf[order], lam, side="right")]
        srcl = lists.p2p_src[ptr[lam]:ptr[lam + 1]]
        if len(srcl) == 0:
            continue
        xs = x[sel]
        idx = np.concatenate([np.arange(stree.leaf_start[sl], stree.leaf_start[sl + 1])
                              for sl in srcl])
        d = xs[:, None, :] - pl[idx][None, :, :]
        r2 = (d * d).sum(-1)
        ok = r2 > 0
        inv = np.zeros_like(r2)
        inv[ok] = 1.0 / np.sqrt(r2[ok])
        u[sel] += -(inv @ ql[idx]) / FOUR_PI
        if field:
            g[sel] += np.einsum("ij,ijk->ik", inv ** 3 * ql[idx][None, :], d) / FOUR_PI
    return u, (-g if field else None)


def fmm(pos: np.ndarray, q: np.ndarray, p: int, leaf_max: int, s: int = 2,
        theta: float = 0.6, targets: np.ndarray | None = None,
        tree: Tree | None = None, lists: Lists | None = None,
        field: bool = True, max_depth: int = 64):
    """FMM potential (and field = -grad u) at the input points ``targets``
    (indices into ``pos``; default all).  Returns (u, field or None)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    if tree is None:
        tree = build_tree(pos, leaf_max, s, max_depth)
    if lists is None:
        lists = build_lists(tree, theta)
    targets = np.arange(len(pos)) if targets is None else np.asarray(targets, dtype=np.int64)
    return _evaluate(tree, pos, q, tree, pos, lists, p, targets, field)


def fmm_st(src: np.ndarray, q: np.ndarray, tgt: np.ndarray, p: int, leaf_max: int,
           s: int = 2, theta: float = 0.6, targets: np.ndarray | None = None,
           stree: Tree | None = None, ttree: Tree | None = None,
           lists: Lists | None = None, field: bool = True, max_depth: int = 64,
           tie: str = "src"):
    """FMM with separate sources and targets (Sec. II.B): potential (and
    field) at the points ``tgt[targets]`` (default all) of the charges ``q``
    at ``src``; a hierarchy per point set, lists between them.  Returns
    (u, field or None)."""
    src = np.ascontiguousarray(src, dtype=np.float64)
    tgt = np.ascontiguousarray(tgt, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    if stree is None:
        stree = build_tree(src, leaf_max, s, max_depth)
    if ttree is None:
        ttree = build_tree(tgt, leaf_max, s, max_depth)
    if lists is None:
        lists = build_lists_st(stree, ttree, theta, tie)
    targets = np.arange(len(tgt)) if targets is None else np.asarray(targets, dtype=np.int64)
    return _evaluate(stree, src, q, ttree, tgt, lists, p, targets, field)
