"""GPU parity of the HIP library against the CPU oracle (through the C ABI).

Tree and lists must be bit-identical to the oracle's; FP64 potentials and
fields must match the oracle FMM (same tree, lists and p) to 1e-10 in
relative L2 (the method is the same linear map up to rounding; the
rotation-based and nested-sum operators differ only in rounding order).
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_15269_amd as F
    return F


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _inputs(kind, n, seed):
    if kind == "cube":
        return workloads.uniform_cube(n, seed)
    if kind == "cluster":
        return workloads.clustered(n, seed)
    if kind == "plummer":
        return workloads.plummer(n, seed)
    if kind == "lattice":
        rng = np.random.default_rng(seed)
        return rng.integers(0, 5, (n, 3)).astype(float) * 0.25, rng.uniform(-1, 1, n)
    raise KeyError(kind)


TREE_CASES = [
    ("cube", 4096, 64, 2, 0.6),
    ("cube", 3001, 32, 2, 0.6),
    ("cube", 5000, 40, 3, 0.7),
    ("cube", 777, 8, 1, 0.5),
    ("lattice", 2000, 16, 2, 0.6),
    ("cluster", 20000, 64, 2, 0.6),
    ("plummer", 9000, 64, 3, 0.7),
    ("cube", 100, 128, 2, 0.6),
    ("cube", 1, 128, 2, 0.6),
]


@pytest.mark.parametrize("kind,n,leaf,s,theta", TREE_CASES)
def test_tree_and_lists_bit_identical(fmm, kind, n, leaf, s, theta):
    from oracle.lists import build_lists
    from oracle.tree import build_tree
    _say(f"[tree/lists] {kind} n={n} leaf={leaf} s={s} theta={theta}")
    pos, q = _inputs(kind, n, 1)
    tr = build_tree(pos, leaf, s)
    li = build_lists(tr, theta)
    plan = fmm.Plan(torch.from_numpy(pos).cuda(), p=4, leaf_max=leaf, splits=s, theta=theta)
    perm, ls, c, r = plan.tree()
    assert np.array_equal(perm, tr.perm)
    assert np.array_equal(ls, tr.leaf_start)
    assert np.array_equal(c, tr.centre)
    assert np.array_equal(r, tr.radius)
    ms, mt, ps, pt = plan.lists()
    assert np.array_equal(ms, li.m2l_src) and np.array_equal(mt, li.m2l_tgt)
    assert np.array_equal(ps, li.p2p_src) and np.array_equal(pt, li.p2p_tgt)
    inf = plan.info()
    assert inf["depth"] == tr.L and inf["n_m2l"] == len(li.m2l_src)


FMM_CASES = [
    # kind, n, p, leaf, s, theta
    ("cube", 4096, 6, 64, 2, 0.6),     # the small uniform-cube workload
    ("cube", 4096, 1, 64, 2, 0.6),
    ("cube", 4096, 8, 64, 2, 0.7),
    ("cube", 3001, 10, 32, 2, 0.5),
    ("cube", 5000, 5, 40, 3, 0.7),
    ("cube", 2500, 7, 16, 1, 0.6),
    ("cluster", 20000, 8, 64, 2, 0.6),
    ("plummer", 9000, 6, 64, 3, 0.7),
    ("lattice", 2000, 4, 16, 2, 0.6),
    ("cube", 100, 8, 128, 2, 0.6),     # one box: direct sum only
    ("cube", 1, 3, 128, 2, 0.6),       # a single point: zero potential
]


@pytest.mark.parametrize("kind,n,p,leaf,s,theta", FMM_CASES)
def test_fp64_matches_oracle_fmm(fmm, kind, n, p, leaf, s, theta):
    from oracle.fmm import fmm as oracle_fmm
    _say(f"[fp64 vs oracle] {kind} n={n} p={p} leaf={leaf} s={s} theta={theta}")
    pos, q = _inputs(kind, n, 2)
    u0, f0 = oracle_fmm(pos, q, p, leaf, s, theta)
    plan = fmm.Plan(torch.from_numpy(pos).cuda(), p=p, leaf_max=leaf, splits=s, theta=theta)
    u, f = plan.evaluate(torch.from_numpy(q).cuda())
    torch.cuda.synchronize()
    u, f = u.cpu().numpy(), f.cpu().numpy()
    if n == 1:
        assert u[0] == 0.0 and np.all(f == 0.0)
        return
    assert _rel(u, u0) <= 1e-10
    assert _rel(f, f0) <= 1e-10


def test_small_cube_against_direct_sum(fmm):
    from oracle.direct import direct
    _say("[fp64 vs direct] cube n=4096 p=6")
    pos, q = workloads.uniform_cube(4096, 0)
    plan = fmm.Plan(torch.from_numpy(pos).cuda(), p=6, leaf_max=64, splits=2, theta=0.6)
    u, f = plan.evaluate(torch.from_numpy(q).cuda())
    ud, gd = direct(pos, q, field=True)
    assert _rel(u.cpu().numpy(), ud) <= 1e-4
    assert _rel(f.cpu().numpy(), -gd) <= 3e-4


def test_repeat_is_bitwise_deterministic(fmm):
    _say("[determinism] cube n=20000 p=8")
    pos, q = workloads.uniform_cube(20000, 3)
    plan = fmm.Plan(torch.from_numpy(pos).cuda(), p=8, leaf_max=64, splits=2, theta=0.6)
    qt = torch.from_numpy(q).cuda()
    u1, f1 = plan.evaluate(qt)
    u2, f2 = plan.evaluate(qt)
    assert torch.equal(u1, u2) and torch.equal(f1, f2)


def test_potential_only_matches_field_run(fmm):
    pos, q = workloads.uniform_cube(5000, 4)
    plan = fmm.Plan(torch.from_numpy(pos).cuda(), p=5, leaf_max=64, splits=2, theta=0.6)
    qt = torch.from_numpy(q).cuda()
    u1, _ = plan.evaluate(qt, field=False)
    u2, _ = plan.evaluate(qt, field=True)
    assert torch.equal(u1, u2)


def test_bad_inputs_raise(fmm):
    pos, q = workloads.uniform_cube(100, 5)
    bad = pos.copy()
    bad[7, 1] = np.nan
    with pytest.raises(fmm.FMMError) as e:
        fmm.Plan(torch.from_numpy(bad).cuda(), p=4, leaf_max=16)
    assert e.value.code == 1
    plan = fmm.Plan(torch.from_numpy(pos).cuda(), p=4, leaf_max=16)
    qt = torch.from_numpy(q).cuda()
    with pytest.raises(fmm.FMMError):
        plan.evaluate(torch.stack([qt, qt]))  # nrhs above the plan's max_rhs
    u, f = plan.evaluate(qt)  # the plan still works
    assert torch.isfinite(u).all()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_direct_kernel_matches_oracle_direct(fmm, prec):
    from oracle.direct import direct
    _say(f"[direct kernel] {prec}")
    pos, q = workloads.uniform_cube(3000, 6)
    pos[5] = pos[9]  # a coincident pair contributes nothing
    tg = np.array([0, 5, 9, 17, 2999])
    dt = torch.float64 if prec == "fp64" else torch.float32
    u, f = fmm.direct(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda().to(dt),
                      torch.from_numpy(tg).cuda())
    ud, gd = direct(pos, q, pos[tg], field=True)
    tol = 1e-13 if prec == "fp64" else 1e-5
    assert _rel(u.double().cpu().numpy(), ud) <= tol
    assert _rel(f.double().cpu().numpy(), -gd) <= tol
    ua, fa = fmm.direct(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda().to(dt))
    ud, gd = direct(pos, q, field=True)
    assert _rel(ua.double().cpu().numpy(), ud) <= tol


def test_stage_profile_counts_passes(fmm):
    pos, q = workloads.uniform_cube(20000, 7)
    plan = fmm.Plan(torch.from_numpy(pos).cuda(), p=6, leaf_max=64, splits=2, theta=0.6)
    qt = torch.from_numpy(q).cuda()
    plan.set_profiling(True)
    for _ in range(3):
        plan.evaluate(qt)
    ms, passes = plan.read_profile()
    assert passes == 3 and all(v >= 0.0 for v in ms.values()) and ms["p2p"] > 0.0
    _, passes = plan.read_profile()
    assert passes == 0
    plan.set_profiling(False)
