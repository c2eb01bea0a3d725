"""MI355X-native adaptive point-charge Laplace FMM (Kraft et al., jaxFMM,
arXiv 2511.15269), Python binding of the C ABI in ``include/fmm.h``.

PyTorch supplies device memory and the stream; the tree, lists and every
evaluation stage run inside ``libfmm.so`` (hand-written HIP kernels for
gfx950).  There is no fallback: without the built library or a GPU the
calls raise.

    plan = Plan(pos, p=8, leaf_max=128, splits=2, theta=0.7)
    pot, field = plan.evaluate(q)
"""
from __future__ import annotations

import contextlib
import ctypes

import numpy as np
import torch

from ._lib import (ALLOC_FN, FMM_FP32, FMM_FP64, FMM_NSTAGES, FMM_PLAN_NO_WORKSPACE,
                   FMM_TIE_SOURCE, FMM_TIE_TARGET,
                   FREE_FN, STAGES, FmmAllocator, FMMError, FmmParams, FmmPlanInfo, FmmTiles,
                   check, lib)

__all__ = ["Plan", "Graph", "FMMError", "params", "direct", "STAGES", "FMMPotential",
           "fmm_energy", "workspace_bytes", "torch_allocator", "tile_cache_key",
           "read_tile_cache", "write_tile_cache"]


@contextlib.contextmanager
def _on(device, stream):
    """Make ``device`` current and, when given, ``stream`` torch's current
    stream, so that every temporary and output tensor of a call is
    allocated on (and recorded against) the stream the library enqueues
    its kernels on."""
    with torch.cuda.device(device):
        if stream is None:
            yield
        else:
            with torch.cuda.stream(stream):
                yield


def _check_out(t, shape, dtype, device, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.device == device
            and t.dtype == dtype and tuple(t.shape) == tuple(shape) and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {tuple(shape)} "
                         f"on {device}")


def direct(pos: torch.Tensor, q: torch.Tensor, targets: torch.Tensor | None = None,
           field: bool = True, stream=None):
    """Direct-sum potential (and field) at ``targets`` (int64 indices into
    pos, CUDA) or at every point; runs in the library's direct kernel."""
    if not (pos.is_cuda and q.is_cuda):
        raise ValueError("pos and q must be CUDA tensors")
    if pos.dim() != 2 or pos.shape[1] != 3 or q.dim() != 1 or q.shape[0] != pos.shape[0]:
        raise ValueError("pos must be [N, 3] and q [N]")
    if q.dtype not in (torch.float64, torch.float32):
        raise ValueError("q must be float64 or float32")
    n = pos.shape[0]
    with _on(pos.device, stream):
        pos = pos.to(torch.float64).contiguous()
        q = q.contiguous()
        prec = FMM_FP64 if q.dtype == torch.float64 else FMM_FP32
        nt = n if targets is None else targets.numel()
        if targets is not None:
            targets = targets.to(device=pos.device, dtype=torch.int64).contiguous()
            if nt and (int(targets.min()) < 0 or int(targets.max()) >= n):
                raise ValueError("targets must index points in [0, N)")
        pot = torch.empty(nt, dtype=q.dtype, device=q.device)
        fld = torch.empty((nt, 3), dtype=q.dtype, device=q.device) if field else None
        check(lib().fmm_direct(ctypes.c_void_p(pos.data_ptr()), n, ctypes.c_void_p(q.data_ptr()),
                               prec, ctypes.c_void_p(targets.data_ptr()) if targets is not None else None,
                               nt, ctypes.c_void_p(pot.data_ptr()),
                               ctypes.c_void_p(fld.data_ptr()) if fld is not None else None,
                               _stream_ptr(None)))
    return pot, fld


TILE_FIELDS = ("p2p_groups", "leaves_per_wave", "m2l_waves", "chain_waves", "near_stream",
               "batch_p2p_waves")


def tile_cache_key(arch: str, prm: FmmParams, n: int, kind: str = "single") -> str:
    """Key of a tile choice in an autotune cache file: the GPU architecture
    (its name up to the first ':'), the order, precision, vectors per pass,
    splits, leaf size, theta, list kind and plan kind, and N rounded to a
    power of two."""
    size = int(round(np.log2(max(int(n), 1))))
    prec = "fp32" if prm.precision == FMM_FP32 else "fp64"
    lists = "same" if prm.lists == 1 else "cross"
    return (f"{arch.split(':')[0]}|p{prm.p}|{prec}|R{prm.max_rhs}|s{prm.splits}|"
            f"leaf{prm.leaf_max}|theta{prm.theta:.6g}|{lists}|{kind}|n2^{size}")


def read_tile_cache(path: str) -> dict:
    """The choices stored in an autotune cache file ({} when the file is
    missing or not a JSON object)."""
    import json
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return {}
    return data if isinstance(data, dict) else {}


def write_tile_cache(path: str, key: str, tiles: dict) -> None:
    """Add (or replace) one choice in an autotune cache file; the file is
    rewritten whole through a temporary file and a rename, so readers see
    either the old or the new contents."""
    import json
    import os
    import tempfile
    data = read_tile_cache(path)
    data[key] = {k: int(tiles[k]) for k in TILE_FIELDS if k in tiles}
    d = os.path.dirname(os.path.abspath(path))
    fd, tmp = tempfile.mkstemp(prefix=".tiles", dir=d)
    try:
        with os.fdopen(fd, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except BaseException:
        if os.path.exists(tmp):
            os.unlink(tmp)
        raise


def params(p=8, leaf_max=128, splits=2, theta=0.7, max_depth=16,
           precision="fp64", tie="source", max_rhs=1, lists="cross") -> FmmParams:
    if lists not in ("cross", "same"):
        raise ValueError("lists must be 'cross' (cross-level) or 'same' (same-level)")
    return FmmParams(p=p, leaf_max=leaf_max, splits=splits, theta=float(theta),
                     max_depth=max_depth,
                     precision=FMM_FP64 if precision == "fp64" else FMM_FP32,
                     tie_refine=FMM_TIE_SOURCE if tie == "source" else FMM_TIE_TARGET,
                     max_rhs=max_rhs, lists=1 if lists == "same" else 0)


def workspace_bytes(n: int, **kw) -> int:
    """Device bytes of the evaluation workspace of a plan of ``n`` points
    (fmm_plan_workspace_bytes; keywords as for ``params``)."""
    out = ctypes.c_int64()
    prm = params(**kw)
    check(lib().fmm_plan_workspace_bytes(int(n), ctypes.byref(prm), ctypes.byref(out)))
    return out.value


def torch_allocator(device) -> FmmAllocator:
    """An fmm_allocator whose callbacks take device memory from torch's
    caching allocator (on the stream the library names), so that plan
    memory is part of torch's pool.  Keep the returned object alive as long
    as any plan created with it."""
    dev = torch.device(device).index or 0

    def _alloc(ctx, nbytes, stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream or 0)
        except Exception:
            return None

    def _free(ctx, ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    a = FmmAllocator(ALLOC_FN(_alloc), FREE_FN(_free), None)
    a._keep = (_alloc, _free)
    return a


def _stream_ptr(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """Tree, geometry and interaction lists of a fixed point set (the
    paper's cached hierarchy), reusable for any number of charge vectors.

    With ``sizes`` (problem sizes summing to N), ``pos`` holds several
    independent problems back to back; each gets its own tree and lists and
    every evaluation covers all of them at once (fmm_multi_plan_create).

    With ``targets`` ([M, 3]), the charges sit at ``pos`` and potentials
    are evaluated at the M target points, each point set with its own tree
    (fmm_plan_create_st): evaluate takes q [N] and returns [M] values,
    evaluate_transposed the reverse."""

    def __init__(self, pos: torch.Tensor, p=8, leaf_max=128, splits=2, theta=0.7,
                 max_depth=16, precision="fp64", tie="source", max_rhs=1, stream=None,
                 sizes=None, allocator=None, targets=None, lists="cross", workspace=True):
        if not (isinstance(pos, torch.Tensor) and pos.is_cuda):
            raise ValueError("pos must be a CUDA tensor")
        if pos.dim() != 2 or pos.shape[1] != 3:
            raise ValueError("pos must have shape [N, 3]")
        pos = pos.to(torch.float64).contiguous()
        self.n = pos.shape[0]          # charges per vector
        self.n_out = self.n            # evaluation points
        self.separate = targets is not None
        self.device = pos.device
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.max_rhs = max_rhs
        self._prm = params(p, leaf_max, splits, theta, max_depth, precision, tie, max_rhs, lists)
        self._h = ctypes.c_void_p()
        # allocator: None (hipMalloc), "torch" (torch's caching allocator) or
        # an FmmAllocator; kept alive with the plan
        if allocator == "torch":
            allocator = torch_allocator(self.device)
        self._alloc = allocator
        ap = ctypes.byref(allocator) if allocator is not None else None
        # workspace=False: the plan holds tree and lists only and is
        # evaluated with evaluate_noalloc (FMM_PLAN_NO_WORKSPACE)
        flags = 0 if workspace else FMM_PLAN_NO_WORKSPACE
        with torch.cuda.device(self.device):
            if targets is not None:
                if sizes is not None:
                    raise ValueError("targets and sizes cannot be combined")
                if not (isinstance(targets, torch.Tensor) and targets.is_cuda
                        and targets.device == self.device and targets.dim() == 2
                        and targets.shape[1] == 3):
                    raise ValueError("targets must be a CUDA tensor of shape [M, 3] on the "
                                     "device of pos")
                tgt = targets.to(torch.float64).contiguous()
                self.n_out = tgt.shape[0]
                check(lib().fmm_plan_create_st(ctypes.c_void_p(pos.data_ptr()), self.n,
                                               ctypes.c_void_p(tgt.data_ptr()), self.n_out,
                                               ctypes.byref(self._prm), ap, flags,
                                               _stream_ptr(stream), ctypes.byref(self._h)))
            elif sizes is None:
                check(lib().fmm_plan_create_ex(ctypes.c_void_p(pos.data_ptr()), self.n,
                                               ctypes.byref(self._prm), ap, flags,
                                               _stream_ptr(stream), ctypes.byref(self._h)))
            else:
                off = np.concatenate([[0], np.cumsum(np.asarray(sizes, np.int64))])
                if off[-1] != self.n:
                    raise ValueError("sizes must sum to the number of points")
                self.offsets = off
                check(lib().fmm_multi_plan_create_ex(
                    ctypes.c_void_p(pos.data_ptr()),
                    off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(off) - 1,
                    ctypes.byref(self._prm), ap, flags, _stream_ptr(stream),
                    ctypes.byref(self._h)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().fmm_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    def info(self) -> dict:
        inf = FmmPlanInfo()
        check(lib().fmm_plan_get_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in FmmPlanInfo._fields_}

    def _vec(self, x: torch.Tensor, name: str, n: int | None = None):
        n = self.n if n is None else n
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == self.dtype
                and x.device == self.device):
            raise ValueError(f"{name} must be a CUDA {self.dtype} tensor on {self.device}")
        xx = x.reshape(1, -1) if x.dim() == 1 else x
        if xx.dim() != 2 or xx.shape[1] != n:
            raise ValueError(f"{name} has the wrong number of points")
        return xx.contiguous()

    def evaluate_transposed(self, q: torch.Tensor, field: bool = True, stream=None):
        """The adjoint operator: G-hat^T q (and its field), same shapes as
        evaluate."""
        single = q.dim() == 1
        with _on(self.device, stream):
            qq = self._vec(q, "q", self.n_out)
            R = qq.shape[0]
            pot = torch.empty((R, self.n), dtype=self.dtype, device=self.device)
            fld = (torch.empty((R, self.n, 3), dtype=self.dtype, device=self.device)
                   if field else None)
            check(lib().fmm_evaluate_transposed(self._h, ctypes.c_void_p(qq.data_ptr()), R,
                                                ctypes.c_void_p(pot.data_ptr()),
                                                ctypes.c_void_p(fld.data_ptr()) if fld is not None else None,
                                                _stream_ptr(None)))
        if single:
            return pot[0], (fld[0] if fld is not None else None)
        return pot, fld

    def adjoint(self, q: torch.Tensor, g: torch.Tensor, field_fwd: torch.Tensor | None,
                stream=None):
        """(grad_q, grad_x) of sum g * u-hat(q, x) with the hierarchy frozen:
        grad_q = G-hat^T g, grad_x = g grad u-hat + q grad(G-hat^T g)
        (grad_x is None when field_fwd is None)."""
        single = g.dim() == 1
        with _on(self.device, stream):
            gg = self._vec(g, "g", self.n_out)
            R = gg.shape[0]
            qq = self._vec(q, "q") if field_fwd is not None else None
            ff = None
            if field_fwd is not None:
                m = self.n_out
                if not (isinstance(field_fwd, torch.Tensor) and field_fwd.is_cuda
                        and field_fwd.dtype == self.dtype and field_fwd.numel() == 3 * R * m):
                    raise ValueError(f"field_fwd must be a CUDA {self.dtype} tensor of "
                                     f"{R} x {m} x 3 values")
                ff = field_fwd.reshape(R, m, 3).contiguous()
            gq = torch.empty((R, self.n), dtype=self.dtype, device=self.device)
            gx = (torch.empty((R, self.n, 3), dtype=self.dtype, device=self.device)
                  if ff is not None else None)
            vp = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
            check(lib().fmm_adjoint(self._h, vp(qq), vp(gg), R, vp(ff), vp(gq), vp(gx),
                                    _stream_ptr(None)))
        if single:
            return gq[0], (gx[0] if gx is not None else None)
        return gq, gx

    def evaluate(self, q: torch.Tensor, field: bool = True, out=None, stream=None):
        """Potentials (and fields = -grad u) for charges ``q`` ([N] or
        [R, N], CUDA, plan precision).  Returns (pot, field or None).
        ``out`` = (pot [R, N], field [R, N, 3] or None) reuses caller
        buffers (contiguous, plan dtype, plan device)."""
        if not (isinstance(q, torch.Tensor) and q.is_cuda and q.dtype == self.dtype):
            raise ValueError(f"q must be a CUDA {self.dtype} tensor")
        single = q.dim() == 1
        qq = q.reshape(1, -1) if single else q
        if qq.dim() != 2 or qq.shape[1] != self.n:
            raise ValueError("q has the wrong number of points")
        R = qq.shape[0]
        m = self.n_out
        with _on(self.device, stream):
            qq = qq.contiguous()
            if out is None:
                pot = torch.empty((R, m), dtype=self.dtype, device=self.device)
                fld = (torch.empty((R, m, 3), dtype=self.dtype, device=self.device)
                       if field else None)
            else:
                pot, fld = out
                _check_out(pot, (R, m), self.dtype, self.device, "out[0] (pot)")
                if fld is not None:
                    _check_out(fld, (R, m, 3), self.dtype, self.device, "out[1] (field)")
            check(lib().fmm_evaluate(self._h, ctypes.c_void_p(qq.data_ptr()), R,
                                     ctypes.c_void_p(pot.data_ptr()),
                                     ctypes.c_void_p(fld.data_ptr()) if fld is not None else None,
                                     _stream_ptr(None)))
        if single:
            return pot[0], (fld[0] if fld is not None else None)
        return pot, fld

    def evaluate_noalloc(self, q: torch.Tensor, out, stream=None) -> None:
        """evaluate into caller buffers ``out`` = (pot [R, M], field
        [R, M, 3] or None) with the library's static workspace
        (fmm_evaluate_noalloc): the call allocates nothing, also not here."""
        qq = self._vec(q, "q")
        R = qq.shape[0]
        if qq.data_ptr() != q.data_ptr():
            raise ValueError("q must be contiguous")
        pot, fld = out
        _check_out(pot, (R, self.n_out), self.dtype, self.device, "out[0] (pot)")
        if fld is not None:
            _check_out(fld, (R, self.n_out, 3), self.dtype, self.device, "out[1] (field)")
        with torch.cuda.device(self.device):
            check(lib().fmm_evaluate_noalloc(self._h, ctypes.c_void_p(qq.data_ptr()), R,
                                             ctypes.c_void_p(pot.data_ptr()),
                                             ctypes.c_void_p(fld.data_ptr()) if fld is not None
                                             else None, _stream_ptr(stream)))

    def autotune(self, q: torch.Tensor, stream=None, cache: str | None = None) -> dict:
        """Time the launch tiles (fmm_tiles) on charges ``q`` ([N], CUDA,
        plan precision) and keep the fastest (fmm_plan_autotune).  Returns
        the chosen values.

        ``cache``: path of a JSON file of earlier choices keyed by
        tile_cache_key (GPU architecture, order, precision, vectors per
        pass, splits, leaf size, theta, list kind, plan kind and the size
        class of N).  A hit sets the stored tiles without timing (unless
        this plan cannot use them); a miss times them and adds the choice
        to the file."""
        key = None
        if cache is not None:
            key = tile_cache_key(torch.cuda.get_device_properties(self.device).gcnArchName,
                                 self._prm, self.n, self._kind())
            hit = read_tile_cache(cache).get(key)
            if hit is not None:
                try:
                    self.set_tiles(**{k: int(hit[k]) for k in TILE_FIELDS if k in hit})
                    return self.tiles()
                except (FMMError, TypeError, ValueError):
                    pass  # stored for a plan whose leaves allowed other tiles
        g, lw = ctypes.c_int(), ctypes.c_int()
        with _on(self.device, stream):
            qq = self._vec(q, "q")
            check(lib().fmm_plan_autotune(self._h, ctypes.c_void_p(qq.data_ptr()),
                                          _stream_ptr(None), ctypes.byref(g),
                                          ctypes.byref(lw)))
        chosen = self.tiles()
        if key is not None:
            write_tile_cache(cache, key, chosen)
        return chosen

    def _kind(self) -> str:
        if self.separate:
            return "st"
        return "multi" if hasattr(self, "offsets") else "single"

    def tiles(self) -> dict:
        """Launch tiles the evaluations use (fmm_plan_get_tiles)."""
        t = FmmTiles()
        check(lib().fmm_plan_get_tiles(self._h, ctypes.byref(t)))
        return {"p2p_groups": t.p2p_groups, "leaves_per_wave": t.leaves_per_wave,
                "m2l_waves": t.m2l_waves, "chain_waves": t.chain_waves,
                "near_stream": t.near_stream, "batch_p2p_waves": t.batch_p2p_waves}

    def set_tiles(self, p2p_groups: int = 0, leaves_per_wave: int = 0,
                  m2l_waves: int = 0, chain_waves: int = 0, near_stream: int = 0,
                  batch_p2p_waves: int = 0) -> None:
        """Set the launch tiles (0: the plan's default; fmm_plan_set_tiles)."""
        t = FmmTiles(p2p_groups, leaves_per_wave, m2l_waves, chain_waves, near_stream,
                     batch_p2p_waves)
        check(lib().fmm_plan_set_tiles(self._h, ctypes.byref(t)))

    def set_profiling(self, on: bool = True) -> None:
        """Record per-stage HIP events in every evaluate (see
        read_profile)."""
        with torch.cuda.device(self.device):
            check(lib().fmm_plan_set_profiling(self._h, 1 if on else 0))

    def read_profile(self) -> tuple[dict, int]:
        """({stage: summed ms}, passes) since the last read; clears."""
        ms = (ctypes.c_double * FMM_NSTAGES)()
        passes = ctypes.c_int64()
        with torch.cuda.device(self.device):
            check(lib().fmm_plan_read_profile(self._h, ms, ctypes.byref(passes)))
        return {k: ms[i] for i, k in enumerate(STAGES)}, passes.value

    def tree(self):
        """(perm, leaf_start, centre[B,3], radius[B]) as numpy arrays."""
        inf = self.info()
        perm = np.empty(inf["n"], np.int64)
        ls = np.empty(inf["nleaf"] + 1, np.int64)
        c = np.empty((inf["nbox"], 3), np.float64)
        r = np.empty(inf["nbox"], np.float64)
        P64 = ctypes.POINTER(ctypes.c_int64)
        PD = ctypes.POINTER(ctypes.c_double)
        with torch.cuda.device(self.device):
            check(lib().fmm_plan_get_tree(self._h, perm.ctypes.data_as(P64), ls.ctypes.data_as(P64),
                                          c.ctypes.data_as(PD), r.ctypes.data_as(PD)))
        return perm, ls, c, r

    def lists(self):
        """(m2l_src, m2l_tgt, p2p_src, p2p_tgt), sorted by (target, source)."""
        inf = self.info()
        a = [np.empty(inf["n_m2l"], np.int64), np.empty(inf["n_m2l"], np.int64),
             np.empty(inf["n_p2p"], np.int64), np.empty(inf["n_p2p"], np.int64)]
        P64 = ctypes.POINTER(ctypes.c_int64)
        with torch.cuda.device(self.device):
            check(lib().fmm_plan_get_lists(self._h, *[x.ctypes.data_as(P64) for x in a]))
        return tuple(a)


class Graph:
    """One evaluation of ``plan`` captured as a HIP graph for fixed buffers
    (fmm_graph_create): ``launch()`` replays it, reading ``q``'s current
    contents and rewriting ``pot`` (and ``field``)."""

    def __init__(self, plan: Plan, q: torch.Tensor, field: bool = True,
                 transposed: bool = False):
        self.plan = plan
        nin, nout = (plan.n_out, plan.n) if transposed else (plan.n, plan.n_out)
        self.q = plan._vec(q, "q", nin)
        if self.q.data_ptr() != q.data_ptr():
            raise ValueError("q must be contiguous (the graph keeps its address)")
        R = self.q.shape[0]
        self.pot = torch.empty((R, nout), dtype=plan.dtype, device=q.device)
        self.field = (torch.empty((R, nout, 3), dtype=plan.dtype, device=q.device)
                      if field else None)
        self._h = ctypes.c_void_p()
        with torch.cuda.device(plan.device):
            check(lib().fmm_graph_create(
                plan._h, 1 if transposed else 0, ctypes.c_void_p(self.q.data_ptr()), R,
                ctypes.c_void_p(self.pot.data_ptr()),
                ctypes.c_void_p(self.field.data_ptr()) if self.field is not None else None,
                ctypes.byref(self._h)))

    def launch(self, stream=None) -> None:
        with torch.cuda.device(self.plan.device):
            check(lib().fmm_graph_launch(self._h, _stream_ptr(stream)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().fmm_graph_destroy(h)
            except Exception:
                pass
            self._h = None


class FMMPotential(torch.autograd.Function):
    """u-hat = FMM(q, x) on a fixed plan, differentiable in q and in the
    point positions x (hierarchy frozen: tree, lists and box centres do not
    move).  ``pos`` must hold the positions the plan was built from.  On a
    plan with separate targets only q is differentiable (pass pos=None)."""

    @staticmethod
    def forward(ctx, q, pos, plan):
        need_x = pos is not None and pos.requires_grad
        if need_x and plan.separate:
            raise ValueError("position gradients need a plan over one point set")
        u, f = plan.evaluate(q, field=need_x)
        ctx.plan = plan
        ctx.save_for_backward(q, f if need_x else None)
        return u

    @staticmethod
    def backward(ctx, gu):
        q, f = ctx.saved_tensors
        plan = ctx.plan
        gq, gx = plan.adjoint(q, gu.contiguous(), f)
        return gq, (gx.to(torch.float64) if gx is not None else None), None


def fmm_energy(plan: Plan, q: torch.Tensor, pos: torch.Tensor) -> torch.Tensor:
    """E = 1/2 sum_i q_i u-hat_i, differentiable in q and pos (frozen
    hierarchy)."""
    u = FMMPotential.apply(q, pos, plan)
    return 0.5 * torch.dot(q, u)
