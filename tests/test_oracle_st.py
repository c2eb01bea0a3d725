"""Pins of the oracle's FMM with separate source and target hierarchies
(Sec. II.B, the generalisation to distinct sources and targets): brute-force
coverage of every (source, target) point pair, admissibility of the lists,
reduction to the single-hierarchy FMM when targets are the sources, accuracy
against the direct sum at arbitrary points, and the adjoint identity."""
import numpy as np
import pytest

from oracle.direct import direct
from oracle.fmm import _evaluate, fmm, fmm_st
from oracle.gradient import transpose_lists
from oracle.lists import admissible, build_lists, build_lists_st
from oracle.tree import build_tree


def _sets(kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "shells":      # sources on a sphere, targets on two others
        def sphere(n, r):
            v = rng.normal(size=(n, 3))
            return r * v / np.linalg.norm(v, axis=1, keepdims=True)
        return sphere(300, 2.0), np.concatenate([sphere(150, 1.5), sphere(150, 2.5)])
    if kind == "deep_vs_shallow":  # many sources, few targets: different depths
        return rng.random((3000, 3)), rng.random((40, 3)) * 0.5 + 0.25
    if kind == "shallow_vs_deep":
        return rng.random((40, 3)) * 0.5 + 0.25, rng.random((3000, 3))
    if kind == "disjoint":    # far-apart clouds
        return rng.random((500, 3)), rng.random((400, 3)) + np.array([3.0, 0.0, 0.0])
    if kind == "shared":      # targets include every source point
        src = rng.random((400, 3))
        return src, np.concatenate([src[::2], rng.random((200, 3))])
    raise KeyError(kind)


CASES = [("shells", 16, 2, 0.6), ("deep_vs_shallow", 16, 2, 0.6), ("shallow_vs_deep", 16, 2, 0.5),
         ("disjoint", 8, 3, 0.7), ("shared", 16, 1, 0.6)]


def _leaf_and_boxes(tree, n):
    """For every point: its leaf and the global id of its box at each level."""
    slot = np.empty(n, np.int64)
    slot[tree.perm] = np.arange(n)
    leaf = np.searchsorted(tree.leaf_start, slot, side="right") - 1
    boxes = np.array([tree.level_off[l] + (leaf >> (tree.s * (tree.L - l)))
                      for l in range(tree.L + 1)])
    return leaf, boxes


@pytest.mark.parametrize("kind,leaf,s,theta", CASES)
def test_every_source_target_pair_is_covered_exactly_once(kind, leaf, s, theta):
    src, tgt = _sets(kind, 1)
    st, tt = build_tree(src, leaf, s), build_tree(tgt, leaf, s)
    li = build_lists_st(st, tt, theta)
    sl, sb = _leaf_and_boxes(st, len(src))
    tl, tb = _leaf_and_boxes(tt, len(tgt))
    cover = np.zeros((len(src), len(tgt)), np.int64)
    # M2L: a source box a covers its points; a target box b covers its points
    for a, b in zip(li.m2l_src, li.m2l_tgt):
        ins = np.any(sb == a, axis=0)
        int_ = np.any(tb == b, axis=0)
        cover[np.ix_(ins, int_)] += 1
    for a, b in zip(li.p2p_src, li.p2p_tgt):
        cover[np.ix_(sl == a, tl == b)] += 1
    assert cover.min() == 1 and cover.max() == 1


@pytest.mark.parametrize("kind,leaf,s,theta", CASES)
def test_m2l_pairs_admissible_and_p2p_pairs_not(kind, leaf, s, theta):
    src, tgt = _sets(kind, 2)
    st, tt = build_tree(src, leaf, s), build_tree(tgt, leaf, s)
    li = build_lists_st(st, tt, theta)
    a, b = li.m2l_src, li.m2l_tgt
    assert np.all(admissible(st.centre[a], st.radius[a], tt.centre[b], tt.radius[b], theta))
    ga = st.level_off[st.L] + li.p2p_src
    gb = tt.level_off[tt.L] + li.p2p_tgt
    assert not np.any(admissible(st.centre[ga], st.radius[ga], tt.centre[gb], tt.radius[gb], theta))


def test_march_refines_by_level_mean_radius_and_stops_at_each_tree_depth():
    src, tgt = _sets("deep_vs_shallow", 3)
    st, tt = build_tree(src, 16, 2), build_tree(tgt, 16, 2)
    assert st.L > tt.L
    li = build_lists_st(st, tt, 0.6)
    ls, lt = zip(*li.steps)
    # one side advances by one level per step, never past its tree's depth
    assert all(abs((a1 - a0) + (b1 - b0)) == 1 for a0, b0, a1, b1 in
               zip(ls[:-1], lt[:-1], ls[1:], lt[1:]))
    assert max(ls) <= st.L and max(lt) <= tt.L


@pytest.mark.parametrize("n,leaf,s,theta", [(2000, 32, 2, 0.6), (1500, 16, 3, 0.7)])
def test_same_points_reduce_to_the_single_hierarchy_fmm(n, leaf, s, theta):
    rng = np.random.default_rng(4)
    pos, q = rng.random((n, 3)), rng.uniform(-1, 1, n)
    tr = build_tree(pos, leaf, s)
    l1, l2 = build_lists(tr, theta), build_lists_st(tr, tr, theta)
    for k in ("m2l_src", "m2l_tgt", "p2p_src", "p2p_tgt"):
        assert np.array_equal(getattr(l1, k), getattr(l2, k))
    u0, f0 = fmm(pos, q, 6, leaf, s, theta, tree=tr, lists=l1)
    u1, f1 = fmm_st(pos, q, pos.copy(), 6, leaf, s, theta, stree=tr, ttree=tr, lists=l2)
    assert np.array_equal(u0, u1) and np.array_equal(f0, f1)


@pytest.mark.parametrize("kind,leaf,s,theta", CASES)
def test_accuracy_against_the_direct_sum_at_the_targets(kind, leaf, s, theta):
    src, tgt = _sets(kind, 5)
    q = np.random.default_rng(6).uniform(-1, 1, len(src))
    ud, gd = direct(src, q, tgt, field=True)
    errs = []
    for p in (4, 8, 16):
        u, f = fmm_st(src, q, tgt, p, leaf, s, theta)
        errs.append(max(np.linalg.norm(u - ud) / np.linalg.norm(ud),
                        np.linalg.norm(f + gd) / np.linalg.norm(gd)))
    # geometric decay in p (eq. 5: the error bound shrinks like theta^(p+1))
    assert errs[0] > errs[1] > errs[2] or errs[2] < 1e-12
    assert errs[2] < 5e-5 and (errs[0] > 50 * errs[2] or errs[2] < 1e-12)
    if kind == "disjoint":
        assert errs[2] < 1e-8  # everything far field


def test_p20_reaches_roundoff_level():
    src, tgt = _sets("shells", 7)
    q = np.random.default_rng(8).uniform(-1, 1, len(src))
    ud, _ = direct(src, q, tgt)
    u, _ = fmm_st(src, q, tgt, 20, 16, 2, 0.5, field=False)
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 1e-9


@pytest.mark.parametrize("kind,leaf,s,theta", CASES)
def test_transposed_lists_give_the_adjoint(kind, leaf, s, theta):
    """<g, G q> = <G^T g, q> with G^T the same FMM from the target
    hierarchy to the source hierarchy over the reversed pairs."""
    src, tgt = _sets(kind, 9)
    rng = np.random.default_rng(10)
    q, g = rng.uniform(-1, 1, len(src)), rng.uniform(-1, 1, len(tgt))
    st, tt = build_tree(src, leaf, s), build_tree(tgt, leaf, s)
    li = build_lists_st(st, tt, theta)
    u, _ = _evaluate(st, src, q, tt, tgt, li, 6, np.arange(len(tgt)), False)
    v, _ = _evaluate(tt, tgt, g, st, src, transpose_lists(li), 6, np.arange(len(src)), False)
    lhs, rhs = float(np.dot(g, u)), float(np.dot(v, q))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-300) * 100


def test_coincident_source_and_target_points_contribute_nothing():
    src, tgt = _sets("shared", 11)
    q = np.random.default_rng(12).uniform(-1, 1, len(src))
    ud, _ = direct(src, q, tgt)
    u, _ = fmm_st(src, q, tgt, 12, 16, 2, 0.5, field=False)
    assert np.all(np.isfinite(u))
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 1e-6


def test_well_separated_roots_are_one_m2l_pair():
    """Two clouds whose roots pass eq. 4 interact through the single pair
    (source root, target root); sources = targets never do (d = 0)."""
    src, tgt = _sets("disjoint", 13)
    st, tt = build_tree(src, 8, 3), build_tree(tgt, 8, 3)
    li = build_lists_st(st, tt, 0.7)
    assert list(li.m2l_src) == [0] and list(li.m2l_tgt) == [0] and len(li.p2p_src) == 0
    li = build_lists(st, 0.7)
    assert 0 not in set(li.m2l_src) | set(li.m2l_tgt)
