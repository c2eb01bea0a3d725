"""GPU checks of the boundary's memory interface: plans whose device memory
comes entirely from a caller-supplied allocator (fmm_plan_create_ex), the
workspace size query, and the plan info's memory figures."""
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
def fmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_15269_amd as F
    return F


class Tracking:
    """An fmm_allocator over torch's caching allocator that records every
    live block."""

    def __init__(self, L):
        self.live = {}
        self.calls = 0

        def _alloc(ctx, nbytes, stream):
            p = torch.cuda.caching_allocator_alloc(int(nbytes), 0, stream or 0)
            self.live[p] = int(nbytes)
            self.calls += 1
            return p

        def _free(ctx, ptr, stream):
            assert ptr in self.live, "free of a block alloc did not return"
            del self.live[ptr]
            torch.cuda.caching_allocator_delete(ptr)

        self._fns = (L.ALLOC_FN(_alloc), L.FREE_FN(_free))
        self.struct = L.FmmAllocator(self._fns[0], self._fns[1], None)


@pytest.mark.parametrize("prec,multi", [("fp64", False), ("fp32", False), ("fp64", True)])
def test_plan_from_callback_memory(fmm, prec, multi):
    from paper_2511_15269_amd import _lib as L
    _say(f"[allocator] {prec} multi={multi}")
    sizes = [3000, 500, 7000] if multi else None
    n = 10500 if multi else 20000
    pos, q = workloads.uniform_cube(n, 3)
    dt = torch.float64 if prec == "fp64" else torch.float32
    P = torch.from_numpy(pos).cuda()
    Q = torch.from_numpy(q).to(dt).cuda()
    kw = dict(p=6, leaf_max=64, splits=2, theta=0.6, precision=prec, sizes=sizes)
    ref = fmm.Plan(P, **kw)
    u0, f0 = ref.evaluate(Q)
    tr = Tracking(L)
    plan = fmm.Plan(P, allocator=tr.struct, **kw)
    inf = plan.info()
    assert tr.calls > 0
    assert inf["device_bytes"] == sum(tr.live.values())
    if not multi:
        assert inf["workspace_bytes"] == fmm.workspace_bytes(n, p=6, leaf_max=64, splits=2,
                                                             theta=0.6, precision=prec)
    u, f = plan.evaluate(Q)
    g, gx = plan.adjoint(Q, Q, f)
    g0, gx0 = ref.adjoint(Q, Q, f0)
    torch.cuda.synchronize()
    # same kernels, same order: identical results
    assert torch.equal(u, u0) and torch.equal(f, f0)
    assert torch.equal(g, g0) and torch.equal(gx, gx0)
    del plan
    torch.cuda.synchronize()
    assert tr.live == {}, "plan memory not returned at destroy"


def test_torch_allocator_option(fmm):
    _say("[allocator] Plan(allocator='torch')")
    pos, q = workloads.uniform_cube(5000, 4)
    P = torch.from_numpy(pos).cuda()
    Q = torch.from_numpy(q).cuda()
    u0, _ = fmm.Plan(P, p=5, leaf_max=32, splits=2, theta=0.6).evaluate(Q, field=False)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    plan = fmm.Plan(P, p=5, leaf_max=32, splits=2, theta=0.6, allocator="torch")
    held = torch.cuda.memory_allocated() - before
    assert held >= plan.info()["device_bytes"] > 0
    u, _ = plan.evaluate(Q, field=False)
    assert torch.equal(u, u0)
    del u
    del plan
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before


def test_allocator_failure_returns_everything(fmm):
    """An allocator that fails after k blocks: create reports FMM_ENOMEM and
    every block handed out so far comes back through free."""
    from paper_2511_15269_amd import _lib as L
    pos, _ = workloads.uniform_cube(20000, 5)
    P = torch.from_numpy(pos).cuda()
    prm = fmm.params(p=6, leaf_max=64, splits=2, theta=0.6)
    for k in (0, 3, 12, 40):
        _say(f"[allocator] failing after {k} blocks")
        tr = Tracking(L)
        inner = tr._fns[0]

        def _alloc(ctx, nbytes, stream, inner=inner, tr=tr, k=k):
            if tr.calls >= k:
                return None
            return inner(ctx, nbytes, stream)

        fn = L.ALLOC_FN(_alloc)
        a = L.FmmAllocator(fn, tr._fns[1], None)
        out = ctypes.c_void_p(4321)
        st = L.lib().fmm_plan_create_ex(ctypes.c_void_p(P.data_ptr()), P.shape[0],
                                        ctypes.byref(prm), ctypes.byref(a), 0,
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                        ctypes.byref(out))
        assert st == L.FMM_ENOMEM
        assert out.value == 4321
        assert tr.live == {}
