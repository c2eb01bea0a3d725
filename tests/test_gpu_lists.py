"""GPU same-level interaction lists (the enumerated procedure at the start
of Sec. II.B) against the oracle: lists bit-identical for one point set and
for separate sources and targets, FP64 results within 1e-10 of the oracle
FMM over the same lists, and, for one point set, the transposed pass equal
to the forward pass (same-level lists are symmetric)."""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from _norms import parity as _rel  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_15269_amd as F
    return F


CASES = [("cube", 4096, 6, 64, 2, 0.6), ("cube", 5000, 8, 40, 3, 0.7),
         ("cluster", 20000, 7, 64, 2, 0.6), ("cube", 2000, 5, 16, 1, 0.5)]


def _inputs(kind, n, seed):
    return workloads.uniform_cube(n, seed) if kind == "cube" else workloads.clustered(n, seed)


@pytest.mark.parametrize("kind,n,p,leaf,s,theta", CASES)
def test_same_level_lists_and_results_match_oracle(fmm, kind, n, p, leaf, s, theta):
    from oracle.fmm import fmm as oracle_fmm
    from oracle.lists import build_lists
    from oracle.tree import build_tree
    _say(f"[same-level] {kind} n={n} p={p} leaf={leaf} s={s} theta={theta}")
    pos, q = _inputs(kind, n, 31)
    tr = build_tree(pos, leaf, s)
    li = build_lists(tr, theta, mode="same")
    plan = fmm.Plan(torch.from_numpy(pos).cuda(), p=p, leaf_max=leaf, splits=s, theta=theta,
                    lists="same")
    ms, mt, ps, pt = plan.lists()
    assert np.array_equal(ms, li.m2l_src) and np.array_equal(mt, li.m2l_tgt)
    assert np.array_equal(ps, li.p2p_src) and np.array_equal(pt, li.p2p_tgt)
    u0, f0 = oracle_fmm(pos, q, p, leaf, s, theta, tree=tr, lists=li)
    Q = torch.from_numpy(q).cuda()
    u, f = plan.evaluate(Q)
    v, fv = plan.evaluate_transposed(Q)
    torch.cuda.synchronize()
    assert _rel(u.cpu().numpy(), u0) <= 1e-10 and _rel(f.cpu().numpy(), f0) <= 1e-10
    # symmetric lists: the transposed pass is the forward pass
    assert torch.equal(u, v) and torch.equal(f, fv)


def test_same_level_lists_between_two_trees(fmm):
    from oracle.fmm import fmm_st
    from oracle.lists import build_lists_st
    from oracle.tree import build_tree
    _say("[same-level] separate sources and targets")
    rng = np.random.default_rng(32)
    src, tgt = rng.random((20000, 3)), rng.random((500, 3)) * 0.5 + 0.25
    q = rng.uniform(-1, 1, len(src))
    st, tt = build_tree(src, 32, 2), build_tree(tgt, 32, 2)
    li = build_lists_st(st, tt, 0.6, mode="same")
    plan = fmm.Plan(torch.from_numpy(src).cuda(), p=7, leaf_max=32, splits=2, theta=0.6,
                    lists="same", targets=torch.from_numpy(tgt).cuda())
    ms, mt, ps, pt = plan.lists()
    assert np.array_equal(ms, li.m2l_src) and np.array_equal(mt, st.nbox + li.m2l_tgt)
    assert np.array_equal(ps, li.p2p_src) and np.array_equal(pt, st.nleaf + li.p2p_tgt)
    u0, f0 = fmm_st(src, q, tgt, 7, 32, 2, 0.6, stree=st, ttree=tt, lists=li)
    u, f = plan.evaluate(torch.from_numpy(q).cuda())
    assert _rel(u.cpu().numpy(), u0) <= 1e-10 and _rel(f.cpu().numpy(), f0) <= 1e-10


def test_cross_level_lists_need_fewer_pairs_on_the_gpu(fmm):
    _say("[same-level] interaction counts, cube 2^17")
    pos, _ = workloads.uniform_cube(1 << 17, 33)
    P = torch.from_numpy(pos).cuda()
    a = fmm.Plan(P, p=6, leaf_max=64, splits=2, theta=0.6).info()
    b = fmm.Plan(P, p=6, leaf_max=64, splits=2, theta=0.6, lists="same").info()
    assert a["n_m2l"] < b["n_m2l"] and a["p2p_interactions"] <= b["p2p_interactions"]
