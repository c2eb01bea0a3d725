"""Pins of the oracle's same-level interaction lists (the enumerated
procedure at the start of Sec. II.B: boxes compared only with boxes of
their own level, children of well-separated pairs skipped) beside the
cross-level level march: coverage of every point pair exactly once,
admissibility, equal levels, symmetry for one point set, fewer M2L pairs
for the cross-level lists (the comparison of Table I), and the FMM over
same-level lists (accuracy, and a symmetric operator)."""
import numpy as np
import pytest

from oracle.direct import direct
from oracle.fmm import _evaluate, fmm
from oracle.lists import admissible, build_lists, build_lists_st
from oracle.tree import build_tree
from test_oracle_tree_lists import _coverage, _inputs


@pytest.mark.parametrize("kind", ["uniform", "lattice"])
@pytest.mark.parametrize("theta", [0.4, 0.7])
@pytest.mark.parametrize("n,leaf,s", [(2048, 32, 2), (1500, 16, 3), (999, 8, 1)])
def test_same_level_lists_cover_every_pair_once_at_equal_levels(kind, theta, n, leaf, s):
    tr = build_tree(_inputs(kind, n, 21), leaf, s)
    li = build_lists(tr, theta, mode="same")
    assert np.all(_coverage(tr, li, n) == 1)
    c, r = tr.centre, tr.radius
    assert np.all(admissible(c[li.m2l_src], r[li.m2l_src], c[li.m2l_tgt], r[li.m2l_tgt], theta))
    lv = np.array([tr.level_of(a) for a in li.m2l_src])
    lw = np.array([tr.level_of(b) for b in li.m2l_tgt])
    assert np.array_equal(lv, lw)
    assert li.steps == [(l, l) for l in range(tr.L + 1)]
    # one point set: the lists are closed under exchanging source and target
    fwd = set(zip(li.m2l_src.tolist(), li.m2l_tgt.tolist()))
    assert fwd == set(zip(li.m2l_tgt.tolist(), li.m2l_src.tolist()))
    pp = set(zip(li.p2p_src.tolist(), li.p2p_tgt.tolist()))
    assert pp == set(zip(li.p2p_tgt.tolist(), li.p2p_src.tolist()))


@pytest.mark.parametrize("n,leaf,s,theta", [(1 << 14, 64, 2, 0.6), (1 << 14, 64, 3, 0.7),
                                            (20000, 32, 1, 0.5)])
def test_cross_level_lists_need_fewer_m2l_pairs(n, leaf, s, theta):
    """Sec. II.B (Table I): the cross-level march handles boxes at the
    earliest possible target level, so it lists fewer interactions."""
    tr = build_tree(_inputs("uniform", n, 22), leaf, s)
    same = build_lists(tr, theta, mode="same")
    cross = build_lists(tr, theta)
    assert len(cross.m2l_src) < len(same.m2l_src)
    assert len(cross.p2p_src) <= len(same.p2p_src)


def test_same_level_lists_between_two_trees():
    rng = np.random.default_rng(23)
    src, tgt = rng.random((3000, 3)), rng.random((60, 3)) * 0.5 + 0.25
    st, tt = build_tree(src, 16, 2), build_tree(tgt, 16, 2)
    li = build_lists_st(st, tt, 0.6, mode="same")
    # both trees refined together until the shallower reaches its leaves
    assert li.steps[:tt.L + 1] == [(l, l) for l in range(tt.L + 1)]
    assert li.steps[-1] == (st.L, tt.L)
    q = rng.uniform(-1, 1, len(src))
    ud, _ = direct(src, q, tgt)
    u, _ = _evaluate(st, src, q, tt, tgt, li, 10, np.arange(len(tgt)), False)
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 5e-5


@pytest.mark.parametrize("n,p,leaf,s,theta", [(3000, 6, 32, 2, 0.6), (2000, 8, 16, 3, 0.7)])
def test_same_level_fmm_accuracy_and_symmetry(n, p, leaf, s, theta):
    """FMM over same-level lists: as accurate as the cross-level FMM, and
    its operator is symmetric up to rounding, <g, G q> = <G g, q> (the
    lists are symmetric and the truncated two-centre kernel is symmetric
    under exchanging source and target)."""
    rng = np.random.default_rng(24)
    pos, q, g = rng.random((n, 3)), rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    tr = build_tree(pos, leaf, s)
    li = build_lists(tr, theta, mode="same")
    u, _ = fmm(pos, q, p, leaf, s, theta, tree=tr, lists=li, field=False)
    v, _ = fmm(pos, g, p, leaf, s, theta, tree=tr, lists=li, field=False)
    ud, _ = direct(pos, q)
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 1e-3
    lhs, rhs = float(np.dot(g, u)), float(np.dot(v, q))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
