"""The evaluation entry point that allocates nothing (fmm_evaluate_noalloc),
called through the C ABI against fmm_evaluate on the same inputs: two calls
in a row on one device, the second with a smaller input, FP64 and FP32;
plans without their own workspace; the size limit and the state errors."""
import ctypes
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
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_15269_amd import _lib
    return _lib


def _create(L, pos, prec, flags, p=6, leaf=64, s=2, theta=0.6):
    prm = L.FmmParams(p=p, leaf_max=leaf, splits=s, theta=theta, max_depth=16,
                      precision=L.FMM_FP64 if prec == "fp64" else L.FMM_FP32,
                      tie_refine=0, max_rhs=2)
    h = ctypes.c_void_p()
    st = L.lib().fmm_plan_create_ex(ctypes.c_void_p(pos.data_ptr()), pos.shape[0],
                                    ctypes.byref(prm), None, flags, None, ctypes.byref(h))
    assert st == L.FMM_OK, L.lib().fmm_last_error()
    return h


def _eval(L, fn, h, q, n_out, dt):
    R = q.shape[0]
    pot = torch.full((R, n_out), float("nan"), dtype=dt, device="cuda")
    fld = torch.full((R, n_out, 3), float("nan"), dtype=dt, device="cuda")
    st = fn(h, ctypes.c_void_p(q.data_ptr()), R, ctypes.c_void_p(pot.data_ptr()),
            ctypes.c_void_p(fld.data_ptr()), None)
    assert st == L.FMM_OK, L.lib().fmm_last_error()
    torch.cuda.synchronize()
    return pot, fld


def _rel(a, b):
    a, b = a.double().cpu().numpy(), b.double().cpu().numpy()
    return max(np.linalg.norm(a - b) / np.linalg.norm(b), np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_evaluate_on_two_calls(L, prec):
    lib = L.lib()
    dt = torch.float64 if prec == "fp64" else torch.float32
    bound = 1e-10 if prec == "fp64" else 1e-5
    for n, seed in ((60000, 1), (7000, 2)):  # second call: smaller input
        _say(f"[noalloc] {prec} n={n}")
        pos, q = workloads.uniform_cube(n, seed)
        P = torch.from_numpy(pos).cuda()
        Q = torch.from_numpy(np.stack([q, -0.5 * q])).to(dt).cuda().contiguous()
        ha = _create(L, P, prec, 0)
        hb = _create(L, P, prec, L.FMM_PLAN_NO_WORKSPACE)
        try:
            # reference: one fmm_evaluate pass per vector (the no-allocation
            # path runs single-vector passes; FP32 plans for two vectors
            # would otherwise take the 32-vector kernels)
            parts = [_eval(L, lib.fmm_evaluate, ha, Q[r:r + 1].contiguous(), n, dt)
                     for r in range(2)]
            u0 = torch.cat([a for a, _ in parts])
            f0 = torch.cat([b for _, b in parts])
            u1, f1 = _eval(L, lib.fmm_evaluate_noalloc, hb, Q, n, dt)
            u2, f2 = _eval(L, lib.fmm_evaluate_noalloc, ha, Q, n, dt)
            assert _rel(u1, u0) <= bound and _rel(f1, f0) <= bound
            assert torch.equal(u1, u0) and torch.equal(f1, f0)  # same kernels, same order
            assert torch.equal(u2, u0) and torch.equal(f2, f0)
            # the plan without a workspace refuses the allocating entry points
            pot = torch.empty((2, n), dtype=dt, device="cuda")
            assert lib.fmm_evaluate(hb, ctypes.c_void_p(Q.data_ptr()), 2,
                                    ctypes.c_void_p(pot.data_ptr()), None, None) == L.FMM_ESTATE
            inf = L.FmmPlanInfo()
            assert lib.fmm_plan_get_info(hb, ctypes.byref(inf)) == L.FMM_OK
            assert inf.workspace_bytes == 0
        finally:
            lib.fmm_plan_destroy(ha)
            lib.fmm_plan_destroy(hb)


def test_noalloc_rejects_plans_beyond_the_limit(L):
    _say("[noalloc] size limit")
    lib = L.lib()
    n = 1 << 21  # FP64: 64 MiB of records + 64 MiB of near field alone
    pos, q = workloads.uniform_cube(n, 3)
    P = torch.from_numpy(pos).cuda()
    h = _create(L, P, "fp64", L.FMM_PLAN_NO_WORKSPACE, p=4, leaf=128)
    try:
        Q = torch.from_numpy(q).cuda()
        pot = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
        st = lib.fmm_evaluate_noalloc(h, ctypes.c_void_p(Q.data_ptr()), 1,
                                      ctypes.c_void_p(pot.data_ptr()), None, None)
        assert st == L.FMM_EINVAL
        assert "FMM_NOALLOC_MAX_BYTES" in lib.fmm_last_error().decode()
        torch.cuda.synchronize()
        assert bool(torch.all(pot == 7.0))  # outputs untouched
    finally:
        lib.fmm_plan_destroy(h)
