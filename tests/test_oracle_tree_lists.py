"""Pins of the oracle's tree (Sec. II.A; Listing 2) and level-marching lists
(Sec. II.B; eq. 4): balance, the recursive definition, brute-force
coverage of every ordered point pair."""
import numpy as np
import pytest

from oracle.lists import admissible, build_lists
from oracle.tree import build_tree, split_order, split_order_recursive, tree_depth


@pytest.mark.parametrize("n,leaf,s,L", [(4096, 64, 2, 3), (1 << 20, 128, 2, 7), (1 << 20, 128, 3, 5),
                                        (1 << 18, 128, 2, 6), (100, 128, 2, 0), (129, 128, 1, 1),
                                        (10000, 128, 2, 4), (500000, 128, 2, 6)])
def test_depth(n, leaf, s, L):
    assert tree_depth(n, leaf, s) == L


def _inputs(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.random((n, 3))
    if kind == "lattice":  # many exact coordinate ties
        return rng.integers(0, 4, (n, 3)).astype(float)
    if kind == "flat":  # degenerate extent in z and x = y ties
        p = rng.random((n, 3))
        p[:, 2] = 0.5
        p[:, 1] = p[:, 0]
        return p
    raise KeyError(kind)


@pytest.mark.parametrize("kind", ["uniform", "lattice", "flat"])
@pytest.mark.parametrize("n,s", [(1000, 2), (777, 3), (4096, 2), (513, 1)])
def test_vectorised_split_matches_recursive_definition(kind, n, s):
    pos = _inputs(kind, n, n + s)
    L = tree_depth(n, 1 << s if s > 1 else 4, s)
    leaves = split_order_recursive(pos, L, s)
    perm, starts = split_order(pos, L, s)
    assert np.array_equal(np.concatenate(leaves), perm)
    assert np.array_equal(np.cumsum([0] + [len(x) for x in leaves]), starts)


@pytest.mark.parametrize("n,leaf,s", [(4096, 64, 2), (1000, 16, 2), (777, 8, 3), (513, 4, 1)])
def test_balance_and_structure(n, leaf, s):
    tr = build_tree(_inputs("uniform", n, 3), leaf, s)
    assert np.array_equal(np.sort(tr.perm), np.arange(n))
    for l in range(tr.L + 1):
        sizes = [np.subtract(*tr.box_range(l, b)[::-1]) for b in range(1 << (s * l))]
        lo, hi = n // (1 << (s * l)), -(-n // (1 << (s * l)))
        assert all(lo <= c <= hi for c in sizes)  # Sec. II.A balance property
    cnt = np.diff(tr.leaf_start)
    assert cnt.max() <= leaf
    for j in range(tr.nleaf):  # leaves sorted by original index
        seg = tr.perm[tr.leaf_start[j]:tr.leaf_start[j + 1]]
        assert np.all(np.diff(seg) > 0)


def test_split_picks_longest_axis_and_lower_half_gets_ceiling():
    # 5 points spread mostly along y: the first split is along y, lower half 3 points
    pos = np.array([[0.0, 0.0, 0.0], [0.1, 4.0, 0.0], [0.2, 1.0, 0.1], [0.0, 3.0, 0.0], [0.1, 2.0, 0.2]])
    leaves = split_order_recursive(pos, 1, 1)
    assert [list(x) for x in leaves] == [[0, 2, 4], [1, 3]]
    # equal extents in x and y: x (the first axis) wins
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 0.5, 0.0], [0.5, 1.0, 0.0], [0.2, 0.7, 0.0]])
    leaves = split_order_recursive(pos, 1, 1)
    assert [list(x) for x in leaves] == [[0, 3], [1, 2]]


def test_geometry_is_bbox_midpoint_and_half_diagonal():
    pos = _inputs("uniform", 300, 9)
    tr = build_tree(pos, 32, 2)
    pl = pos[tr.perm]
    for l in range(tr.L + 1):
        for b in range(1 << (2 * l)):
            a, e = tr.box_range(l, b)
            lo, hi = pl[a:e].min(0), pl[a:e].max(0)
            g = tr.level_off[l] + b
            assert np.array_equal(tr.centre[g], 0.5 * (lo + hi))
            assert tr.radius[g] == pytest.approx(0.5 * np.linalg.norm(hi - lo), rel=1e-15)


def _coverage(tr, li, n):
    """cover[i, j] = number of list entries through which source j reaches
    target i (leaf-ordered indices)."""
    cover = np.zeros((n, n), dtype=np.int16)
    for a, b in zip(li.m2l_src, li.m2l_tgt):
        la, lb = tr.level_of(a), tr.level_of(b)
        sa, ea = tr.box_range(la, a - tr.level_off[la])
        sb, eb = tr.box_range(lb, b - tr.level_off[lb])
        cover[sb:eb, sa:ea] += 1
    for a, b in zip(li.p2p_src, li.p2p_tgt):
        cover[tr.leaf_start[b]:tr.leaf_start[b + 1], tr.leaf_start[a]:tr.leaf_start[a + 1]] += 1
    return cover


@pytest.mark.parametrize("kind", ["uniform", "lattice"])
@pytest.mark.parametrize("theta", [0.3, 0.6, 0.77])
@pytest.mark.parametrize("n,leaf,s", [(2048, 32, 2), (1500, 16, 3), (999, 8, 1)])
def test_every_pair_covered_exactly_once(kind, theta, n, leaf, s):
    tr = build_tree(_inputs(kind, n, 11), leaf, s)
    li = build_lists(tr, theta)
    cover = _coverage(tr, li, n)
    assert np.all(cover == 1)
    # every M2L pair admissible, every direct pair not (eq. 4)
    c, r = tr.centre, tr.radius
    assert np.all(admissible(c[li.m2l_src], r[li.m2l_src], c[li.m2l_tgt], r[li.m2l_tgt], theta))
    gs = tr.level_off[tr.L] + li.p2p_src
    gt = tr.level_off[tr.L] + li.p2p_tgt
    assert not np.any(admissible(c[gs], r[gs], c[gt], r[gt], theta))
    # each leaf interacts directly with itself
    assert np.sum(li.p2p_src == li.p2p_tgt) == tr.nleaf


def test_march_alternates_for_equal_source_and_target_trees():
    tr = build_tree(_inputs("uniform", 4096, 2), 64, 2)
    li = build_lists(tr, 0.6)
    want = [(0, 0)]
    for l in range(1, tr.L + 1):
        want += [(l, l - 1), (l, l)]
    assert li.steps == want
    lt = build_lists(tr, 0.6, tie="tgt")
    assert len(lt.m2l_src) == len(li.m2l_src) and len(lt.p2p_src) == len(li.p2p_src)


def test_admissibility_boundary_and_zero_distance():
    c = np.array([[0.0, 0.0, 0.0]])
    # R + theta r <= theta d holds with equality: 1 + 0.5*1 = 0.5*3
    assert admissible(c, np.array([1.0]), np.array([[3.0, 0, 0]]), np.array([1.0]), 0.5)[0]
    assert not admissible(c, np.array([1.0]), np.array([[2.999, 0, 0]]), np.array([1.0]), 0.5)[0]
    # coincident point-like boxes are never admissible
    assert not admissible(c, np.array([0.0]), c, np.array([0.0]), 0.5)[0]
