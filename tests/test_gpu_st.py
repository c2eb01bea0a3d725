"""GPU parity of plans with separate sources and targets (Sec. II.B, the
generalisation to distinct source and target points) against the CPU
oracle, through the C ABI: both trees and the lists between them
bit-identical, FP64 potentials and fields within 1e-10 (relative L2 and
relative max) of the oracle FMM with the same trees, lists and order, FP32
within 1e-5, the transposed pass against the oracle's FMM over the reversed
pairs, and the adjoint identity."""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from _norms import parity as _rel  # noqa: E402
from _norms import rel_l2  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_15269_amd as F
    return F


def _sets(kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "shield":
        g = workloads.shielding(seed)
        src = np.concatenate([g["shield"], g["ext"]])
        tgt = np.concatenate([g["inner"], g["outer"]])
        return src, tgt
    if kind == "cube_in_cube":   # targets inside the source cloud, other density
        return rng.random((20000, 3)), rng.random((7000, 3)) * 0.8 + 0.1
    if kind == "deep_vs_shallow":
        return rng.random((30000, 3)), rng.random((300, 3)) * 0.5 + 0.25
    if kind == "shallow_vs_deep":
        return rng.random((300, 3)) * 0.5 + 0.25, rng.random((30000, 3))
    if kind == "disjoint":
        return rng.random((5000, 3)), rng.random((4000, 3)) + np.array([3.0, 0.0, 0.0])
    if kind == "shared":         # every second source is also a target
        src = rng.random((6000, 3))
        return src, np.concatenate([src[::2], rng.random((2000, 3))])
    if kind == "clusters":
        src, _ = workloads.clustered(20000, seed)
        tgt, _ = workloads.sphere_surface(5000, seed, 0.5, (0.5, 0.5, 0.5))
        return src, tgt
    if kind == "single":
        return rng.random((1, 3)), rng.random((1, 3))
    raise KeyError(kind)


CASES = [("shield", 8, 16, 2, 0.6), ("cube_in_cube", 6, 64, 2, 0.6),
         ("deep_vs_shallow", 8, 64, 3, 0.7), ("shallow_vs_deep", 5, 32, 2, 0.5),
         ("disjoint", 8, 64, 2, 0.7), ("shared", 6, 32, 1, 0.6), ("clusters", 8, 64, 2, 0.6),
         ("single", 3, 8, 2, 0.6)]


def _plan(fmm, src, tgt, p, leaf, s, theta, precision="fp64"):
    return fmm.Plan(torch.from_numpy(src).cuda(), p=p, leaf_max=leaf, splits=s, theta=theta,
                    precision=precision, targets=torch.from_numpy(tgt).cuda())


@pytest.mark.parametrize("kind,p,leaf,s,theta", CASES)
def test_trees_and_lists_bit_identical(fmm, kind, p, leaf, s, theta):
    from oracle.lists import build_lists_st
    from oracle.tree import build_tree
    _say(f"[st tree/lists] {kind} leaf={leaf} s={s} theta={theta}")
    src, tgt = _sets(kind, 1)
    st, tt = build_tree(src, leaf, s), build_tree(tgt, leaf, s)
    li = build_lists_st(st, tt, theta)
    plan = _plan(fmm, src, tgt, p, leaf, s, theta)
    ns, nbs, nls = len(src), st.nbox, st.nleaf
    perm, ls, c, r = plan.tree()
    assert np.array_equal(perm[:ns], st.perm) and np.array_equal(perm[ns:], tt.perm)
    assert np.array_equal(ls[:nls + 1], st.leaf_start)
    assert np.array_equal(ls[nls:], ns + tt.leaf_start)
    assert np.array_equal(c[:nbs], st.centre) and np.array_equal(c[nbs:], tt.centre)
    assert np.array_equal(r[:nbs], st.radius) and np.array_equal(r[nbs:], tt.radius)
    ms, mt, ps, pt = plan.lists()
    assert np.array_equal(ms, li.m2l_src) and np.array_equal(mt, nbs + li.m2l_tgt)
    assert np.array_equal(ps, li.p2p_src) and np.array_equal(pt, nls + li.p2p_tgt)
    inf = plan.info()
    assert inf["n"] == ns + len(tgt) and inf["nbox"] == nbs + tt.nbox


@pytest.mark.parametrize("kind,p,leaf,s,theta", CASES)
def test_fp64_matches_oracle(fmm, kind, p, leaf, s, theta):
    from oracle.fmm import fmm_st
    _say(f"[st fp64 vs oracle] {kind} p={p} leaf={leaf} s={s} theta={theta}")
    src, tgt = _sets(kind, 2)
    q = np.random.default_rng(3).uniform(-1, 1, len(src))
    u0, f0 = fmm_st(src, q, tgt, p, leaf, s, theta)
    plan = _plan(fmm, src, tgt, p, leaf, s, theta)
    u, f = plan.evaluate(torch.from_numpy(q).cuda())
    torch.cuda.synchronize()
    u, f = u.cpu().numpy(), f.cpu().numpy()
    assert u.shape == (len(tgt),) and f.shape == (len(tgt), 3)
    if kind == "single":
        assert np.allclose(u, u0, rtol=1e-13) and np.allclose(f, f0, rtol=1e-13)
        return
    assert _rel(u, u0) <= 1e-10
    assert _rel(f, f0) <= 1e-10


@pytest.mark.parametrize("kind,p,leaf,s,theta", [c for c in CASES if c[0] != "single"])
def test_fp32_matches_fp64_oracle(fmm, kind, p, leaf, s, theta):
    from oracle.fmm import fmm_st
    _say(f"[st fp32 vs oracle] {kind} p={p}")
    src, tgt = _sets(kind, 4)
    q = np.random.default_rng(5).uniform(-1, 1, len(src))
    u0, f0 = fmm_st(src, q, tgt, p, leaf, s, theta)
    plan = _plan(fmm, src, tgt, p, leaf, s, theta, "fp32")
    u, f = plan.evaluate(torch.from_numpy(q).float().cuda())
    torch.cuda.synchronize()
    assert _rel(u.cpu().numpy(), u0) <= 1e-5
    assert _rel(f.cpu().numpy(), f0) <= 1e-5


@pytest.mark.parametrize("kind,p,leaf,s,theta", [c for c in CASES if c[0] != "single"])
def test_transposed_pass_and_adjoint_identity(fmm, kind, p, leaf, s, theta):
    """G-hat^T g (targets back to sources) against the oracle FMM over the
    reversed pairs, and <g, G-hat q> = <G-hat^T g, q>."""
    from oracle.fmm import _evaluate
    from oracle.gradient import transpose_lists
    from oracle.lists import build_lists_st
    from oracle.tree import build_tree
    _say(f"[st transposed] {kind} p={p}")
    src, tgt = _sets(kind, 6)
    rng = np.random.default_rng(7)
    q, g = rng.uniform(-1, 1, len(src)), rng.uniform(-1, 1, len(tgt))
    st, tt = build_tree(src, leaf, s), build_tree(tgt, leaf, s)
    li = transpose_lists(build_lists_st(st, tt, theta))
    v0, fv0 = _evaluate(tt, tgt, g, st, src, li, p, np.arange(len(src)), True)
    plan = _plan(fmm, src, tgt, p, leaf, s, theta)
    v, fv = plan.evaluate_transposed(torch.from_numpy(g).cuda())
    u, _ = plan.evaluate(torch.from_numpy(q).cuda(), field=False)
    gq, gx = plan.adjoint(None, torch.from_numpy(g).cuda(), None)
    torch.cuda.synchronize()
    v, fv, u, gq = v.cpu().numpy(), fv.cpu().numpy(), u.cpu().numpy(), gq.cpu().numpy()
    assert gx is None
    assert _rel(v, v0) <= 1e-10 and _rel(fv, fv0) <= 1e-10
    assert np.array_equal(gq, v)
    lhs, rhs = float(np.dot(g, u)), float(np.dot(v, q))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_same_points_as_targets_reproduce_the_single_plan(fmm):
    _say("[st] targets = sources vs one-set plan")
    pos, q = workloads.uniform_cube(30000, 8)
    P, Q = torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda()
    one = fmm.Plan(P, p=7, leaf_max=64, splits=2, theta=0.6)
    two = fmm.Plan(P, p=7, leaf_max=64, splits=2, theta=0.6, targets=P.clone())
    u1, f1 = one.evaluate(Q)
    u2, f2 = two.evaluate(Q)
    torch.cuda.synchronize()
    assert _rel(u2.cpu().numpy(), u1.cpu().numpy()) <= 1e-13
    assert _rel(f2.cpu().numpy(), f1.cpu().numpy()) <= 1e-13


def test_accuracy_against_direct_sum_at_targets(fmm):
    from oracle.direct import direct
    _say("[st] cube_in_cube vs direct sum")
    src, tgt = _sets("cube_in_cube", 9)
    q = np.random.default_rng(10).uniform(-1, 1, len(src))
    ud, gd = direct(src, q, tgt, field=True)
    plan = _plan(fmm, src, tgt, 8, 64, 2, 0.6)
    u, f = plan.evaluate(torch.from_numpy(q).cuda())
    assert rel_l2(u.cpu().numpy(), ud) <= 1e-4 and rel_l2(f.cpu().numpy(), -gd) <= 1e-4


def test_several_vectors_graph_and_errors(fmm):
    from paper_2511_15269_amd import FMMError
    _say("[st] vectors, graph replay, rejected position gradients")
    src, tgt = _sets("cube_in_cube", 11)
    rng = np.random.default_rng(12)
    Q = torch.from_numpy(rng.uniform(-1, 1, (3, len(src)))).cuda()
    plan = fmm.Plan(torch.from_numpy(src).cuda(), p=6, leaf_max=64, splits=2, theta=0.6,
                    max_rhs=3, targets=torch.from_numpy(tgt).cuda())
    U, F = plan.evaluate(Q)
    assert U.shape == (3, len(tgt)) and F.shape == (3, len(tgt), 3)
    for r in range(3):
        u, f = plan.evaluate(Q[r].contiguous())
        assert torch.equal(u, U[r]) and torch.equal(f, F[r])
    q0 = Q[0].contiguous().clone()
    gr = fmm.Graph(plan, q0)
    ref, _ = plan.evaluate(q0)
    for k in range(3):
        q0.copy_(Q[k])
        gr.launch()
        torch.cuda.synchronize()
        want, _ = plan.evaluate(Q[k].contiguous())
        assert torch.equal(gr.pot[0], want)
    with pytest.raises(FMMError):
        plan.adjoint(Q[0], torch.ones(len(tgt), dtype=torch.float64, device="cuda"),
                     torch.zeros((len(tgt), 3), dtype=torch.float64, device="cuda"))
