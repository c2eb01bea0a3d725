"""GPU parity of the HIP library against the CPU oracle (through the C ABI).

Tree and lists must be bit-identical to the oracle's; FP64 potentials and
fields must match the oracle FMM (same tree, lists and p) to 1e-10 in both
the relative L2 and the relative max norm (the method is the same linear map
up to rounding; the rotation-based and nested-sum operators differ only in
rounding order), FP32 to 1e-5.
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


from _norms import parity as _rel  # noqa: E402  (rel-L2 and rel-max, both bounded)
from _norms import rel_l2, rel_max  # noqa: E402


def _inputs(kind, n, seed):
    if kind == "cube":
        return workloads.uniform_cube(n, seed)
    if kind == "cluster":
        return workloads.clustered(n, seed)
    if kind == "plummer":
        return workloads.plummer(n, seed)
    if kind == "dups":
        # a uniform cube in which 2% of the points repeat an earlier point
        pos, q = workloads.uniform_cube(n, seed)
        rng = np.random.default_rng(seed + 1000)
        k = max(1, n // 50)
        dst = rng.choice(np.arange(1, n), k, replace=False)
        pos[dst] = pos[rng.integers(0, n, k) % np.maximum(dst, 1)]
        return pos, q
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
    ("dups", 6000, 6, 32, 3, 0.7),     # coincident points across leaves
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
    u, f = u.cpu().numpy(), f.cpu().numpy()
    _say(f"    rel-L2 pot {rel_l2(u, ud):.2e} field {rel_l2(f, -gd):.2e}; rel-max pot "
         f"{rel_max(u, ud):.2e} field {rel_max(f, -gd):.2e}")
    assert rel_l2(u, ud) <= 1e-4
    assert rel_l2(f, -gd) <= 3e-4


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


def test_direct_rejects_out_of_range_targets_without_reading(fmm):
    """Through the C ABI (the Python wrapper refuses such indices first):
    target indices outside [0, n) read no memory and give NaN outputs; the
    valid ones are unaffected."""
    import ctypes
    from paper_2511_15269_amd import _lib
    pos, q = workloads.uniform_cube(500, 8)
    pt = torch.from_numpy(pos).cuda()
    qt = torch.from_numpy(q).cuda()
    tg = torch.tensor([-1, 7, 500, 1 << 40, 499], dtype=torch.int64, device="cuda")
    pot = torch.empty(5, dtype=torch.float64, device="cuda")
    fld = torch.empty((5, 3), dtype=torch.float64, device="cuda")
    _lib.check(_lib.lib().fmm_direct(ctypes.c_void_p(pt.data_ptr()), 500,
                                     ctypes.c_void_p(qt.data_ptr()), _lib.FMM_FP64,
                                     ctypes.c_void_p(tg.data_ptr()), 5,
                                     ctypes.c_void_p(pot.data_ptr()),
                                     ctypes.c_void_p(fld.data_ptr()), None))
    torch.cuda.synchronize()
    bad = torch.tensor([True, False, True, True, False], device="cuda")
    assert torch.isnan(pot[bad]).all() and torch.isnan(fld[bad]).all()
    u, f = fmm.direct(pt, qt, torch.tensor([7, 499], device="cuda"))
    assert torch.equal(pot[~bad], u) and torch.equal(fld[~bad], f)


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


FP32_CASES = [
    # kind, n, p, leaf, s, theta
    ("cube", 4096, 6, 64, 2, 0.6),
    ("cube", 20000, 8, 64, 2, 0.7),
    ("cube", 30000, 8, 128, 3, 0.7),
    ("cluster", 30000, 10, 128, 2, 0.6),   # clustered, sigma = 0.01: scaled expansions
    ("plummer", 20000, 8, 128, 2, 0.6),
    ("lattice", 3000, 6, 16, 2, 0.6),      # coincident points in different leaves
    ("dups", 8000, 8, 32, 3, 0.7),         # a few coincident pairs among uniform points
    ("cube", 100, 8, 128, 2, 0.6),
]


@pytest.mark.parametrize("kind,n,p,leaf,s,theta", FP32_CASES)
def test_fp32_matches_oracle_fmm(fmm, kind, n, p, leaf, s, theta):
    """FP32 form: within 1e-5 relative L2 of the FP64 oracle FMM (same tree,
    lists and order) for potential and field."""
    from oracle.fmm import fmm as oracle_fmm
    _say(f"[fp32 vs oracle] {kind} n={n} p={p} leaf={leaf} s={s} theta={theta}")
    pos, q = _inputs(kind, n, 8)
    u0, f0 = oracle_fmm(pos, q, p, leaf, s, theta)
    plan = fmm.Plan(torch.from_numpy(pos).cuda(), p=p, leaf_max=leaf, splits=s, theta=theta,
                    precision="fp32")
    u, f = plan.evaluate(torch.from_numpy(q).cuda().float())
    u, f = u.double().cpu().numpy(), f.double().cpu().numpy()
    eu, ef = _rel(u, u0), _rel(f, f0)
    _say(f"    rel-L2 pot {eu:.2e} field {ef:.2e}")
    assert eu <= 1e-5 and ef <= 1e-5


ADJ_CASES = [
    # kind, n, p, leaf, s, theta
    ("cube", 4096, 6, 64, 2, 0.6),
    ("plummer", 9000, 8, 128, 2, 0.6),
    ("cube", 5000, 5, 40, 3, 0.7),
    ("cluster", 8000, 7, 32, 1, 0.5),
]


@pytest.mark.parametrize("kind,n,p,leaf,s,theta", ADJ_CASES)
def test_transposed_pass_matches_oracle_and_is_the_adjoint(fmm, kind, n, p, leaf, s, theta):
    from oracle.fmm import fmm as oracle_fmm
    from oracle.gradient import transpose_lists
    from oracle.lists import build_lists
    from oracle.tree import build_tree
    _say(f"[transposed] {kind} n={n} p={p} leaf={leaf} s={s} theta={theta}")
    pos, q = _inputs(kind, n, 9)
    g = np.random.default_rng(10).uniform(-1, 1, n)
    tr = build_tree(pos, leaf, s)
    lt = transpose_lists(build_lists(tr, theta))
    v0, fv0 = oracle_fmm(pos, g, p, leaf, s, theta, tree=tr, lists=lt)
    plan = fmm.Plan(torch.from_numpy(pos).cuda(), p=p, leaf_max=leaf, splits=s, theta=theta)
    qt, gt = torch.from_numpy(q).cuda(), torch.from_numpy(g).cuda()
    v, fv = plan.evaluate_transposed(gt)
    assert _rel(v.cpu().numpy(), v0) <= 1e-10
    assert _rel(fv.cpu().numpy(), fv0) <= 1e-10
    u, _ = plan.evaluate(qt, field=False)
    lhs = float(torch.dot(gt, u))
    rhs = float(torch.dot(v, qt))
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_energy_gradient_matches_oracle(fmm, prec, tol):
    from oracle.gradient import energy_gradient_fmm
    from oracle.lists import build_lists
    from oracle.tree import build_tree
    n, p, leaf, s, theta = 6000, 8, 64, 2, 0.6
    _say(f"[energy gradient] plummer n={n} {prec}")
    pos, q = workloads.plummer(n, 18)
    tr = build_tree(pos, leaf, s)
    li = build_lists(tr, theta)
    dq0, dx0 = energy_gradient_fmm(pos, q, p, leaf, s, theta, tr, li)
    dt = torch.float64 if prec == "fp64" else torch.float32
    pos_t = torch.from_numpy(pos).cuda().requires_grad_(True)
    q_t = torch.from_numpy(q).cuda().to(dt).requires_grad_(True)
    plan = fmm.Plan(pos_t.detach(), p=p, leaf_max=leaf, splits=s, theta=theta, precision=prec)
    E = fmm.fmm_energy(plan, q_t, pos_t)
    gq, gx = torch.autograd.grad(E, (q_t, pos_t))
    eq = _rel(gq.double().cpu().numpy(), dq0)
    ex = _rel(gx.double().cpu().numpy(), dx0)
    _say(f"    rel-L2 dE/dq {eq:.2e} dE/dx {ex:.2e}")
    assert eq <= tol and ex <= tol


def test_fp32_energy_gradient_against_direct_gradient(fmm):
    """Plummer charges in (0,1]: FP32 forward + adjoint against the FP64
    direct-sum gradient on a 4096-point subset.  theta = 0.5: at p = 8 the
    Plummer tree needs it for 1e-4 on dE/dx (the FP64 oracle gives 1.1e-4
    at theta = 0.6)."""
    from oracle.gradient import energy_gradient_direct
    n = 60000
    _say(f"[fp32 gradient vs direct] plummer n={n}")
    pos, q = workloads.plummer(n, 0)
    sub = workloads.sample_targets(n, 4096, seed=3)
    dq0, dx0 = energy_gradient_direct(pos, q, targets=sub)
    pos_t = torch.from_numpy(pos).cuda().requires_grad_(True)
    q_t = torch.from_numpy(q).cuda().float().requires_grad_(True)
    plan = fmm.Plan(pos_t.detach(), p=8, leaf_max=128, splits=2, theta=0.5, precision="fp32")
    E = fmm.fmm_energy(plan, q_t, pos_t)
    gq, gx = torch.autograd.grad(E, (q_t, pos_t))
    eq = rel_l2(gq.double().cpu().numpy()[sub], dq0)
    ex = rel_l2(gx.double().cpu().numpy()[sub], dx0)
    _say(f"    rel-L2 dE/dq {eq:.2e} dE/dx {ex:.2e}; rel-max dE/dq "
         f"{rel_max(gq.double().cpu().numpy()[sub], dq0):.2e} dE/dx "
         f"{rel_max(gx.double().cpu().numpy()[sub], dx0):.2e}")
    assert eq <= 1e-4 and ex <= 1e-4


BATCH_CASES = [
    # kind, n, p, leaf, s, theta, R
    ("cube", 20000, 8, 128, 2, 0.7, 32),
    ("cube", 9000, 6, 64, 3, 0.6, 5),
    ("cluster", 15000, 10, 128, 2, 0.6, 40),   # two passes: 32 + 8 vectors
    ("cube", 100, 4, 128, 2, 0.6, 3),          # one box, direct only
]


@pytest.mark.parametrize("kind,n,p,leaf,s,theta,R", BATCH_CASES)
def test_batched_vectors_match_single_runs_and_oracle(fmm, kind, n, p, leaf, s, theta, R):
    """R charge vectors in one multi-vector pass (FP32, MFMA near field)
    equal R single-vector passes to 1e-6 and the FP64 oracle to 1e-5."""
    from oracle.fmm import fmm as oracle_fmm
    _say(f"[batched] {kind} n={n} p={p} leaf={leaf} s={s} theta={theta} R={R}")
    pos, _ = _inputs(kind, n, 19)
    Q = np.random.default_rng(20).uniform(-1, 1, (R, n))
    pt = torch.from_numpy(pos).cuda()
    plan = fmm.Plan(pt, p=p, leaf_max=leaf, splits=s, theta=theta, precision="fp32", max_rhs=R)
    single = fmm.Plan(pt, p=p, leaf_max=leaf, splits=s, theta=theta, precision="fp32")
    Qt = torch.from_numpy(Q).cuda().float()
    U, Fd = plan.evaluate(Qt)
    worst = 0.0
    for r in range(R):
        u1, f1 = single.evaluate(Qt[r])
        worst = max(worst, _rel(U[r].double().cpu().numpy(), u1.double().cpu().numpy()),
                    _rel(Fd[r].double().cpu().numpy(), f1.double().cpu().numpy()))
    _say(f"    batched vs single: {worst:.2e}")
    assert worst <= 1e-6
    for r in (0, R - 1):
        u0, f0 = oracle_fmm(pos, Q[r], p, leaf, s, theta)
        eu = _rel(U[r].double().cpu().numpy(), u0)
        ef = _rel(Fd[r].double().cpu().numpy(), f0)
        _say(f"    vector {r} vs oracle: pot {eu:.2e} field {ef:.2e}")
        assert eu <= 1e-5 and ef <= 1e-5
    Ut, _ = plan.evaluate_transposed(Qt)
    ut1, _ = single.evaluate_transposed(Qt[R - 1])
    assert _rel(Ut[R - 1].double().cpu().numpy(), ut1.double().cpu().numpy()) <= 1e-6


MULTI_CASES = [
    # precision, sizes, kinds, p, leaf, s, theta
    ("fp64", [2500, 1, 7000, 300, 4100], ["cube", "cube", "cluster", "cube", "plummer"],
     6, 64, 2, 0.6),
    ("fp32", [5000, 1200, 40, 9000], ["cluster", "cube", "cube", "plummer"], 8, 128, 3, 0.7),
]


def _multi_inputs(sizes, kinds, seed):
    ps, qs = [], []
    for j, (n, k) in enumerate(zip(sizes, kinds)):
        p_, q_ = _inputs(k, n, seed + j)
        ps.append(p_)
        qs.append(q_)
    return ps, qs


@pytest.mark.parametrize("prec,sizes,kinds,p,leaf,s,theta", MULTI_CASES)
def test_multi_plan_matches_separate_plans_and_oracle(fmm, prec, sizes, kinds, p, leaf, s,
                                                      theta):
    """Several independent problems of different depths in one plan: tree
    and lists are each problem's own (bit-identical to the oracle, indices
    shifted), results equal separate plans and the oracle FMM."""
    from oracle.fmm import fmm as oracle_fmm
    from oracle.lists import build_lists
    from oracle.tree import build_tree
    _say(f"[multi] {prec} sizes={sizes} p={p} leaf={leaf} s={s} theta={theta}")
    ps, qs = _multi_inputs(sizes, kinds, 40)
    dt = torch.float64 if prec == "fp64" else torch.float32
    pos = torch.from_numpy(np.concatenate(ps)).cuda()
    q = torch.from_numpy(np.concatenate(qs)).cuda().to(dt)
    plan = fmm.Plan(pos, p=p, leaf_max=leaf, splits=s, theta=theta, precision=prec,
                    sizes=sizes)
    u, f = plan.evaluate(q)
    ut, ft = plan.evaluate_transposed(q)
    torch.cuda.synchronize()
    perm, ls, c, r = plan.tree()
    ms, mt, pps, ppt = plan.lists()
    off = plan.offsets
    pb = bb = lb = 0
    m_all, p_all = [], []
    tol_sep, tol_or = (1e-12, 1e-10) if prec == "fp64" else (1e-6, 1e-5)
    for j, n in enumerate(sizes):
        sl = slice(off[j], off[j + 1])
        tr = build_tree(ps[j], leaf, s)
        li = build_lists(tr, theta)
        nb, nl = len(tr.radius), len(tr.leaf_start) - 1
        assert np.array_equal(perm[sl], tr.perm + pb)
        assert np.array_equal(ls[lb:lb + nl + 1], tr.leaf_start + pb)
        assert np.array_equal(c[bb:bb + nb], tr.centre)
        assert np.array_equal(r[bb:bb + nb], tr.radius)
        m_all.append(np.stack([li.m2l_src + bb, li.m2l_tgt + bb]))
        p_all.append(np.stack([li.p2p_src + lb, li.p2p_tgt + lb]))
        sep = fmm.Plan(pos[sl], p=p, leaf_max=leaf, splits=s, theta=theta, precision=prec)
        u1, f1 = sep.evaluate(q[sl])
        ut1, _ = sep.evaluate_transposed(q[sl])
        uj, fj = u[sl].double().cpu().numpy(), f[sl].double().cpu().numpy()
        if n == 1:
            assert np.all(uj == 0.0) and np.all(fj == 0.0)
        else:
            e_sep = max(_rel(uj, u1.double().cpu().numpy()), _rel(fj, f1.double().cpu().numpy()),
                        _rel(ut[sl].double().cpu().numpy(), ut1.double().cpu().numpy()))
            u0, f0 = oracle_fmm(ps[j], qs[j], p, leaf, s, theta)
            e_or = max(_rel(uj, u0), _rel(fj, f0))
            _say(f"    problem {j} n={n} depth {tr.L}: vs separate {e_sep:.2e} vs oracle {e_or:.2e}")
            assert e_sep <= tol_sep and e_or <= tol_or
        pb += n
        bb += nb
        lb += nl
    m_all = np.concatenate(m_all, axis=1)
    p_all = np.concatenate(p_all, axis=1)
    o = np.lexsort((m_all[0], m_all[1]))
    assert np.array_equal(ms, m_all[0][o]) and np.array_equal(mt, m_all[1][o])
    o = np.lexsort((p_all[0], p_all[1]))
    assert np.array_equal(pps, p_all[0][o]) and np.array_equal(ppt, p_all[1][o])


def test_batched_near_field_waves_give_identical_results_and_are_tuned(fmm):
    """The batched near field's waves per block only change how the 16-target
    tiles of a leaf are shared out: every choice gives the same bits, and
    autotune picks one of them."""
    _say("[batched waves]")
    pos, Q = workloads.uniform_cube(40000, 17, nrhs=8)
    pt = torch.from_numpy(pos).cuda()
    qt = torch.from_numpy(Q).cuda().float()
    plan = fmm.Plan(pt, p=6, leaf_max=96, splits=2, theta=0.7, precision="fp32", max_rhs=8)
    assert plan.tiles()["batch_p2p_waves"] in (1, 2, 4, 8)
    ref = None
    for w in (1, 2, 4, 8):
        plan.set_tiles(batch_p2p_waves=w)
        assert plan.tiles()["batch_p2p_waves"] == w
        u, f = plan.evaluate(qt)
        torch.cuda.synchronize()
        if ref is None:
            ref = (u, f)
        else:
            assert torch.equal(u, ref[0]) and torch.equal(f, ref[1])
    with pytest.raises(fmm.FMMError):
        plan.set_tiles(batch_p2p_waves=3)
    choice = plan.autotune(qt[0])
    assert choice["batch_p2p_waves"] in (1, 2, 4, 8)
    u, f = plan.evaluate(qt)
    assert torch.equal(u, ref[0]) and torch.equal(f, ref[1])


def test_multi_plan_batched_vectors(fmm):
    """Uneven problems and several charge vectors at once (FP32)."""
    sizes = [6000, 500, 13000]
    _say(f"[multi batched] sizes={sizes} R=6")
    ps, _ = _multi_inputs(sizes, ["cube", "cluster", "plummer"], 60)
    pos = torch.from_numpy(np.concatenate(ps)).cuda()
    Q = torch.from_numpy(np.random.default_rng(61).uniform(-1, 1, (6, sum(sizes)))).cuda().float()
    plan = fmm.Plan(pos, p=8, leaf_max=64, splits=2, theta=0.7, precision="fp32", max_rhs=6,
                    sizes=sizes)
    single = fmm.Plan(pos, p=8, leaf_max=64, splits=2, theta=0.7, precision="fp32",
                      sizes=sizes)
    U, Fd = plan.evaluate(Q)
    worst = 0.0
    for r in range(6):
        u1, f1 = single.evaluate(Q[r])
        worst = max(worst, _rel(U[r].double().cpu().numpy(), u1.double().cpu().numpy()),
                    _rel(Fd[r].double().cpu().numpy(), f1.double().cpu().numpy()))
    _say(f"    batched vs single: {worst:.2e}")
    assert worst <= 1e-6


GRAPH_CASES = [
    # precision, sizes (None = one problem), n, R, transposed
    ("fp64", None, 20000, 1, False),
    ("fp64", None, 9000, 1, True),
    ("fp32", [7000, 300, 12000, 1], None, 1, False),
    ("fp32", [4000, 9000], None, 32, False),
]


@pytest.mark.parametrize("prec,sizes,n,R,transposed", GRAPH_CASES)
def test_graph_replays_match_eager_runs(fmm, prec, sizes, n, R, transposed):
    """A captured evaluation replayed several times, with new charges
    written by ordinary eager work between replays, reproduces the eager
    evaluation bit for bit on every replay."""
    _say(f"[graph] {prec} sizes={sizes} n={n} R={R} transposed={transposed}")
    if sizes is None:
        pos, _ = workloads.uniform_cube(n, 70)
        kw = {}
    else:
        pos = np.concatenate(_multi_inputs(sizes, ["cube", "cluster", "plummer", "cube"][:len(sizes)], 71)[0])
        kw = {"sizes": sizes}
    N = len(pos)
    dt = torch.float64 if prec == "fp64" else torch.float32
    plan = fmm.Plan(torch.from_numpy(pos).cuda(), p=6, leaf_max=64, splits=2, theta=0.6,
                    precision=prec, max_rhs=R, **kw)
    q = torch.empty((R, N), dtype=dt, device="cuda")
    g = fmm.Graph(plan, q, field=True, transposed=transposed)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(72)
    for rep in range(4):
        q.uniform_(-1, 1, generator=gen)
        g.launch()
        torch.cuda.synchronize()
        ev = plan.evaluate_transposed if transposed else plan.evaluate
        u, f = ev(q)
        torch.cuda.synchronize()
        _say(f"    replay {rep}")
        assert torch.equal(g.pot, u) and torch.equal(g.field, f)


@pytest.mark.parametrize("prec,n,leaf,s,tol", [("fp64", 30000, 64, 2, 1e-12),
                                               ("fp32", 20000, 128, 3, 1e-6)])
def test_autotuned_tiles_give_the_same_results(fmm, prec, n, leaf, s, tol):
    """Tiles chosen by timing change only summation orders: results equal
    the default tiles' to rounding, and stay within the oracle bound."""
    _say(f"[autotune] {prec} n={n} leaf={leaf} s={s}")
    pos, q = workloads.uniform_cube(n, 80)
    dt = torch.float64 if prec == "fp64" else torch.float32
    pt = torch.from_numpy(pos).cuda()
    qt = torch.from_numpy(q).cuda().to(dt)
    a = fmm.Plan(pt, p=6, leaf_max=leaf, splits=s, theta=0.7, precision=prec)
    b = fmm.Plan(pt, p=6, leaf_max=leaf, splits=s, theta=0.7, precision=prec)
    choice = b.autotune(qt)
    _say(f"    chosen {choice}")
    assert choice["p2p_groups"] in (1, 2, 4) and choice["leaves_per_wave"] in (1, 2, 4, 8)
    assert choice["m2l_waves"] in ((1, 4) if prec == "fp64" else (1,))
    ua, fa = a.evaluate(qt)
    ub, fb = b.evaluate(qt)
    assert _rel(ub.double().cpu().numpy(), ua.double().cpu().numpy()) <= tol
    assert _rel(fb.double().cpu().numpy(), fa.double().cpu().numpy()) <= tol


@pytest.mark.parametrize("prec,p,n,leaf,s,theta", [
    ("fp64", 6, 30000, 64, 2, 0.5), ("fp64", 7, 40000, 64, 3, 0.8),
    ("fp32", 9, 30000, 64, 3, 0.7), ("fp32", 10, 20000, 32, 2, 0.6)])
def test_m2l_shared_form_is_identical_to_one_lane_form(fmm, prec, p, n, leaf, s, theta):
    """The M2L form whose translations are shared by several waves applies
    the same operations to every coefficient in the same order as the form
    with one lane per translation: forward and transposed results agree
    bit for bit."""
    _say(f"[m2l forms] {prec} p={p} n={n} leaf={leaf} s={s} theta={theta}")
    pos, q = workloads.clustered(n, 90 + p)
    dt = torch.float64 if prec == "fp64" else torch.float32
    pt = torch.from_numpy(pos).cuda()
    qt = torch.from_numpy(q).cuda().to(dt)
    plan = fmm.Plan(pt, p=p, leaf_max=leaf, splits=s, theta=theta, precision=prec)
    assert plan.tiles()["m2l_waves"] == 4
    u1, f1 = plan.evaluate(qt)
    t1 = plan.evaluate_transposed(qt)
    plan.set_tiles(m2l_waves=1)
    assert plan.tiles()["m2l_waves"] == 1
    u0, f0 = plan.evaluate(qt)
    t0 = plan.evaluate_transposed(qt)
    torch.cuda.synchronize()
    assert torch.equal(u0, u1) and torch.equal(f0, f1)
    assert torch.equal(t0[0], t1[0]) and torch.equal(t0[1], t1[1])
    with pytest.raises(fmm.FMMError):
        plan.set_tiles(m2l_waves=3)
    assert plan.tiles()["m2l_waves"] == 1


@pytest.mark.parametrize("prec,p,n,leaf,s,theta", [
    ("fp64", 5, 30000, 16, 1, 0.6), ("fp64", 8, 40000, 64, 3, 0.8), ("fp64", 10, 30000, 32, 2, 0.5),
    ("fp32", 6, 40000, 24, 2, 0.7), ("fp32", 9, 30000, 64, 3, 0.6)])
def test_chain_shared_form_is_identical_to_one_lane_form(fmm, prec, p, n, leaf, s, theta):
    """M2M and L2L translations shared by four waves give the same bits as
    one lane per translation, forward and transposed (s = 1, 2, 3 cover
    child groups of 2, 4 and 8 lanes; deep trees give long ancestor
    groups in the L2L lists)."""
    _say(f"[chain forms] {prec} p={p} n={n} leaf={leaf} s={s} theta={theta}")
    pos, q = workloads.clustered(n, 40 + p)
    dt = torch.float64 if prec == "fp64" else torch.float32
    pt = torch.from_numpy(pos).cuda()
    qt = torch.from_numpy(q).cuda().to(dt)
    plan = fmm.Plan(pt, p=p, leaf_max=leaf, splits=s, theta=theta, precision=prec)
    assert plan.tiles()["chain_waves"] == 4
    u1, f1 = plan.evaluate(qt)
    t1 = plan.evaluate_transposed(qt)
    plan.set_tiles(chain_waves=1)
    assert plan.tiles()["chain_waves"] == 1
    u0, f0 = plan.evaluate(qt)
    t0 = plan.evaluate_transposed(qt)
    torch.cuda.synchronize()
    assert torch.equal(u0, u1) and torch.equal(f0, f1)
    assert torch.equal(t0[0], t1[0]) and torch.equal(t0[1], t1[1])
    with pytest.raises(fmm.FMMError):
        plan.set_tiles(chain_waves=2)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_near_field_stream_choice_gives_identical_results(fmm, prec):
    """The near field on the plan's second stream (default) and on the
    caller's stream give the same bits, forward, transposed and in a graph
    replayed after eager passes on another stream."""
    _say(f"[near stream] {prec}")
    pos, q = workloads.uniform_cube(60000, 23)
    dt = torch.float64 if prec == "fp64" else torch.float32
    pt = torch.from_numpy(pos).cuda()
    qt = torch.from_numpy(q).cuda().to(dt)
    plan = fmm.Plan(pt, p=7, leaf_max=32, splits=3, theta=0.7, precision=prec)
    assert plan.tiles()["near_stream"] == 2
    u2, f2 = plan.evaluate(qt)
    t2 = plan.evaluate_transposed(qt)
    g = fmm.Graph(plan, qt, field=True)
    plan.set_tiles(near_stream=1)
    assert plan.tiles()["near_stream"] == 1
    u1, f1 = plan.evaluate(qt)
    t1 = plan.evaluate_transposed(qt)
    # one plan's passes share its workspace: the pass on another stream
    # starts once the passes above have finished
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        u3, f3 = plan.evaluate(qt, stream=side)
    side.synchronize()
    g.launch()
    torch.cuda.synchronize()
    plan.set_tiles()
    assert torch.equal(u1, u2) and torch.equal(f1, f2)
    assert torch.equal(t1[0], t2[0]) and torch.equal(t1[1], t2[1])
    assert torch.equal(u3, u2) and torch.equal(f3, f2)
    assert torch.equal(g.pot[0], u2) and torch.equal(g.field[0], f2)
    with pytest.raises(fmm.FMMError):
        plan.set_tiles(near_stream=3)


def test_m2l_one_lane_form_where_no_shared_form_is_built(fmm):
    pos, _ = workloads.uniform_cube(5000, 3)
    pt = torch.from_numpy(pos).cuda()
    for prec, p in (("fp64", 8), ("fp64", 5), ("fp32", 8)):
        plan = fmm.Plan(pt, p=p, leaf_max=64, splits=3, theta=0.7, precision=prec)
        assert plan.tiles()["m2l_waves"] == 1
        assert plan.tiles()["chain_waves"] == 4
        with pytest.raises(fmm.FMMError):
            plan.set_tiles(m2l_waves=4)
        plan.set_tiles(m2l_waves=1)
        assert plan.tiles()["m2l_waves"] == 1


def test_autotune_cache_file_is_written_and_reused(fmm, tmp_path):
    """A cache miss times the tiles and stores them; a second plan of the
    same kind takes them from the file without timing."""
    from paper_2511_15269_amd import _lib
    path = str(tmp_path / "tiles.json")
    pos, q = workloads.uniform_cube(30000, 81)
    pt = torch.from_numpy(pos).cuda()
    qt = torch.from_numpy(q).cuda()
    a = fmm.Plan(pt, p=6, leaf_max=32, splits=3, theta=0.7)
    chosen = a.autotune(qt, cache=path)
    stored = fmm.read_tile_cache(path)
    assert len(stored) == 1 and list(stored.values())[0] == chosen
    b = fmm.Plan(pt, p=6, leaf_max=32, splits=3, theta=0.7)
    lib = _lib.lib()
    real = lib.fmm_plan_autotune

    def refuse(*args):
        raise AssertionError("the cache hit must not time the tiles")
    lib.fmm_plan_autotune = refuse
    try:
        assert b.autotune(qt, cache=path) == chosen
    finally:
        lib.fmm_plan_autotune = real
    ua, fa = a.evaluate(qt)
    ub, fb = b.evaluate(qt)
    assert torch.equal(ua, ub) and torch.equal(fa, fb)


@pytest.mark.parametrize("prec,n,p,leaf,s,theta", [("fp64", 30000, 5, 64, 2, 0.6),
                                                   ("fp32", 25000, 6, 32, 2, 0.7)])
def test_split_near_field_lists_match_oracle(fmm, prec, n, p, leaf, s, theta):
    """Clustered points give some leaves direct lists far longer than the
    near-field work-item budget: those lists are cut into several items whose
    partial sums are added afterwards; the result must still match the
    oracle, which sums every list in one go."""
    from oracle.fmm import fmm as oracle_fmm
    _say(f"[split near field] clustered n={n} p={p} leaf={leaf} s={s} theta={theta} {prec}")
    pos, q = workloads.clustered(n, 5)
    u0, f0 = oracle_fmm(pos, q, p, leaf, s, theta)
    dt = torch.float64 if prec == "fp64" else torch.float32
    plan = fmm.Plan(torch.from_numpy(pos).cuda(), p=p, leaf_max=leaf, splits=s, theta=theta,
                    precision=prec)
    inf = plan.info()
    assert inf["p2p_items"] > inf["nleaf"], "no leaf was split: the case does not test splitting"
    Q = torch.from_numpy(q).to(dt).cuda()
    u, f = plan.evaluate(Q)
    v, _ = plan.evaluate(Q, field=False)
    torch.cuda.synchronize()
    bound = 1e-10 if prec == "fp64" else 1e-5
    assert _rel(u.cpu().numpy(), u0) <= bound and _rel(f.cpu().numpy(), f0) <= bound
    assert torch.equal(u, v)
