#!/usr/bin/env python3
"""Throughput of the FMM evaluation pass on one MI355X.

Workload: N = 2^20 charges uniform in the unit cube, charges uniform in
[-1, 1), expansion order p = 8, leaf size <= 128, potential and field.  A
step is one evaluation pass (sort, P2M, M2M, M2L, L2L, L2P, P2P) of one
charge vector on a cached plan (tree and lists built once, as in the
paper's protocol), inputs resident in HBM, FP64.  ``value`` = N / step time
in Mpoints/s.  ``variants`` times the other parts of the metric on the same
workload: the FP32 form, and forward + backward (potential and field, then
the adjoint giving dE/dq and dE/dx of E = 1/2 sum q u) in both precisions.
Every variant's accuracy against the FP64 direct sum is measured on 8192
sampled targets with the library's direct kernel; the roofline object
reports the dominant kernel of the headline pass (per-stage HIP events over
the timed steps); ``cpu_baseline`` times the CPU oracle on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Mpoints/s fwd and fwd+bwd at rel-L2 ≤1e-4 vs direct sum; "
          "FP32/batched vs FP64")
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}  # MI355X vector peaks


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload_tag(n, p, precision, splits, theta) -> str:
    """Name of a benchmark configuration in profiles/ file names."""
    nl = "1m" if n == 1 << 20 else str(n)
    return f"cube{nl}_p{p}_{precision}_s{splits}_t{int(round(theta * 100))}"


def traffic_from_profile(kernel_prefix: str, tag: str):
    """HBM bytes per launch recorded for the dominant kernel under profiles/,
    if the kernel sources have not changed since (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel_prefix}_{tag}_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source_sha256:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (m and t):
        return None
    if kernel_source_hash() != m.group(1):
        return None
    return float(t.group(1))


KERNEL_SOURCES = ("csrc/eval.hip", "csrc/ops.h", "csrc/tables.h", "csrc/tables.cpp", "build.py")


def kernel_source_hash() -> str:
    """sha256 over the sources and build flags of the single-vector
    evaluation kernels."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2511_15269_amd", f), "rb").read())
    return h.hexdigest()


_CPU = {}


def _cpu_chunk(tg):
    """One worker's share of the CPU-baseline sample (forked worker: the
    tree and lists were built by the parent)."""
    import threadpoolctl
    from oracle.fmm import fmm as oracle_fmm
    c = _CPU
    with threadpoolctl.threadpool_limits(1):
        oracle_fmm(c["pos"], c["q"], c["p"], c["leaf"], c["s"], c["theta"], targets=tg,
                   tree=c["tree"], lists=c["lists"])
    return len(tg)


def cpu_baseline(pos, q, p, leaf, s, theta, per_worker=96, reps=3):
    """The CPU oracle FMM (as it stands: NumPy FP64, one thread per worker)
    on a bounded sample, spread over the host cores: every worker process
    evaluates the potential and field at its own ``per_worker`` sampled
    targets with the prebuilt hierarchy, all workers at once; the wall time
    of the slowest is the time of the sample.  Best of ``reps``.  Runs
    before the GPU is initialised, so the workers can be forked."""
    import multiprocessing as mp

    import threadpoolctl
    import workloads
    from oracle.lists import build_lists
    from oracle.tree import build_tree
    with threadpoolctl.threadpool_limits(1):
        tr = build_tree(pos, leaf, s)
        li = build_lists(tr, theta)
    cores = min(16, len(os.sched_getaffinity(0)))
    tg = workloads.sample_targets(len(pos), cores * per_worker, seed=7)
    _CPU.update(pos=pos, q=q, p=p, leaf=leaf, s=s, theta=theta, tree=tr, lists=li)
    chunks = [tg[w::cores] for w in range(cores)]
    best = None
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        for _ in range(reps):
            t0 = time.perf_counter()
            done = sum(pool.map(_cpu_chunk, chunks, chunksize=1))
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": done / best / 1e6, "unit": "Mpoints/s", "cores": cores,
            "kind": "oracle",
            "sample": f"FMM potential+field at {done} sampled targets of the same 2^20-point "
                      f"workload ({per_worker} per worker process, {cores} processes of one "
                      f"thread each), tree and lists prebuilt; best of {reps}: {best:.1f} s; "
                      f"host CPU {model or 'unknown'}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--p", type=int, default=8)
    ap.add_argument("--leaf", type=int, default=128)
    ap.add_argument("--splits", type=int, default=3)
    ap.add_argument("--theta", type=float, default=0.8)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"],
                    help="precision of the headline (value) pass")
    ap.add_argument("--samples", type=int, default=0,
                    help="targets of the accuracy check against the FP64 direct sum "
                         "(0: every point)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-targets-per-core", type=int, default=96)
    ap.add_argument("--only-headline", action="store_true",
                    help="skip the FP32 / forward+backward variants")
    ap.add_argument("--theta-uneven", type=float, default=0.6,
                    help="separation parameter of the uneven problem set (its small, shallow "
                         "trees need a smaller theta for 1e-4)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the multi-vector and uneven-problem-set variants")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (HBM counter scale)")
    ap.add_argument("--counters-batched", action="store_true",
                    help="with --counters: the 32-vector FP32 pass on 2^18 points instead")
    ap.add_argument("--counters", action="store_true",
                    help="only the headline pass (plan, autotune, warm-up, timed steps) and, with "
                         "--copy-calibration, the calibration copy: the program to run under "
                         "rocprofv3 --pmc")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the FMM library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import workloads

    pos, q = workloads.uniform_cube(args.n, 0)
    if args.counters:
        counters_run(args, pos, q)
        return
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(pos, q, args.p, args.leaf, args.splits, args.theta,
                           args.cpu_targets_per_core)
        log(f"cpu baseline: {cpu['value']:.3e} Mpoints/s ({cpu['sample']})")

    import torch

    import paper_2511_15269_amd as F

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pos_d = torch.from_numpy(pos).to(dev)
    q64 = torch.from_numpy(q).to(dev)
    stream = torch.cuda.current_stream()

    # FP64 direct sum at sampled targets: the accuracy reference of every variant
    tg = (np.arange(args.n) if args.samples <= 0
          else workloads.sample_targets(args.n, args.samples, seed=1))
    tg_d = torch.from_numpy(tg).to(dev)
    ud, fd = F.direct(pos_d, q64, tg_d)
    torch.cuda.synchronize()
    ud, fd = ud.cpu().numpy(), fd.cpu().numpy()
    qs = q[tg]
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    linf = lambda a, b: float(np.abs(a - b).max() / np.abs(b).max())

    def build(prec):
        t0 = time.perf_counter()
        plan = F.Plan(pos_d, p=args.p, leaf_max=args.leaf, splits=args.splits,
                      theta=args.theta, precision=prec)
        torch.cuda.synchronize()
        return plan, (time.perf_counter() - t0) * 1e3

    def timed(fn, steps, warmup, warm_s=0.0):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        # optional warm spell: passes of fn, untimed, for warm_s seconds, so
        # that a measurement taken after host-side work (accuracy checks,
        # plan builds) does not time the GPU's clocks ramping up again
        t_end = time.perf_counter() + warm_s
        while time.perf_counter() < t_end:
            for _ in range(max(warmup, 1)):
                fn()
            torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def vtimed(fn, steps, warmup):
        """timed() for the variants: after a 50 ms warm spell."""
        return timed(fn, steps, warmup, warm_s=0.05)

    res_variants = {}
    res_tiles = {}

    def run_forward(prec, profile):
        plan, plan_ms = build(prec)
        tdt = torch.float64 if prec == "fp64" else torch.float32
        qd = q64.to(tdt)
        pot = torch.empty((1, args.n), dtype=tdt, device=dev)
        fld = torch.empty((1, args.n, 3), dtype=tdt, device=dev)
        tiles = plan.autotune(qd[0] if qd.dim() > 1 else qd)
        res_tiles[prec] = tiles
        fn = lambda: plan.evaluate(qd, out=(pot, fld))
        # the timed steps record no stage events; the per-stage times come
        # from a second, profiled set of steps
        ms = timed(fn, args.steps, args.warmup)
        stages = None
        if profile:
            plan.set_profiling(True)
            timed(fn, args.steps, 0)
            st_ms, passes = plan.read_profile()
            plan.set_profiling(False)
            stages = {k: v / max(passes, 1) for k, v in st_ms.items()}
        up = pot[0].double().cpu().numpy()[tg]
        fp = fld[0].double().cpu().numpy()[tg]
        acc = {"rel_l2_pot": rel(up, ud), "rel_l2_field": rel(fp, fd),
               "rel_linf_pot": linf(up, ud), "rel_linf_field": linf(fp, fd)}
        return plan, plan_ms, ms, stages, acc

    def run_fwd_bwd(plan, prec):
        tdt = torch.float64 if prec == "fp64" else torch.float32
        qd = q64.to(tdt)
        half = 0.5 * qd
        out = {}

        def fn():
            u, f = plan.evaluate(qd)
            gq, gx = plan.adjoint(qd, half, f)
            out["u"], out["gq"], out["gx"] = u, gq, gx
        ms = vtimed(fn, args.steps, args.warmup)
        # E = 1/2 q.u-hat: dE/dq = u-hat/2 + G-hat^T(q/2), dE/dx = grad_x
        dq = (0.5 * out["u"] + out["gq"]).double().cpu().numpy()[tg]
        dx = out["gx"].double().cpu().numpy()[tg]
        acc = {"rel_l2_dEdq": rel(dq, ud), "rel_l2_dEdx": rel(dx, -qs[:, None] * fd),
               "rel_linf_dEdq": linf(dq, ud), "rel_linf_dEdx": linf(dx, -qs[:, None] * fd)}
        return ms, acc

    head = args.precision
    plan, plan_ms, ms_per_step, per_stage, acc = run_forward(head, True)
    info = plan.info()
    value = args.n / (ms_per_step * 1e-3) / 1e6
    log(f"plan ({head}): {plan_ms:.1f} ms, depth {info['depth']}, M2L {info['n_m2l']}, "
        f"P2P pairs {info['n_p2p']}, P2P interactions {info['p2p_interactions']}")
    log(f"fwd {head}: {ms_per_step:.3f} ms/step, {value:.1f} Mpoints/s, rel-L2 pot "
        f"{acc['rel_l2_pot']:.2e} field {acc['rel_l2_field']:.2e}, rel-Linf pot "
        f"{acc['rel_linf_pot']:.2e} field {acc['rel_linf_field']:.2e}")
    log("stages (ms/pass): " + ", ".join(f"{k} {v:.3f}" for k, v in per_stage.items()))
    if args.copy_calibration:
        a = torch.empty(1 << 25, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if not args.only_headline:
        # the same pass replayed from a captured HIP graph (one launch call)
        gq = q64.to(torch.float64 if head == "fp64" else torch.float32).reshape(1, -1).clone()
        graph = F.Graph(plan, gq, field=True)
        # eager launches timed in the same window, for a like-for-like ratio
        ms_g = vtimed(graph.launch, args.steps, args.warmup)
        ms_e = vtimed(lambda: plan.evaluate(gq), args.steps, args.warmup)
        same = bool(torch.equal(graph.pot, plan.evaluate(gq)[0]))
        res_variants[f"fwd_{head}_graph"] = {"ms_per_step": ms_g, "mpoints_s": args.n / ms_g / 1e3,
                                             "eager_ms_same_window": ms_e,
                                             "graph_equals_eager": same}
        log(f"fwd {head} graph replay: {ms_g:.3f} ms/step ({args.n / ms_g / 1e3:.1f} Mpoints/s)")
        del graph
        ms, a2 = run_fwd_bwd(plan, head)
        res_variants[f"fwd_bwd_{head}"] = {"ms_per_step": ms, "mpoints_s": args.n / ms / 1e3, **a2}
        log(f"fwd+bwd {head}: {ms:.3f} ms/step, {args.n / ms / 1e3:.1f} Mpoints/s, {a2}")
        other = "fp32" if head == "fp64" else "fp64"
        del plan
        plan2, pms2, ms2, _, acc2 = run_forward(other, False)
        res_variants[f"fwd_{other}"] = {"ms_per_step": ms2, "mpoints_s": args.n / ms2 / 1e3,
                                        "plan_build_ms": pms2, **acc2}
        log(f"fwd {other}: {ms2:.3f} ms/step, {args.n / ms2 / 1e3:.1f} Mpoints/s, {acc2}")
        ms3, a3 = run_fwd_bwd(plan2, other)
        res_variants[f"fwd_bwd_{other}"] = {"ms_per_step": ms3, "mpoints_s": args.n / ms3 / 1e3, **a3}
        log(f"fwd+bwd {other}: {ms3:.3f} ms/step, {args.n / ms3 / 1e3:.1f} Mpoints/s, {a3}")
        del plan2
    if not args.only_headline and not args.no_batched:
        res_variants.update(run_batched(F, torch, dev, args, vtimed, rel))
        res_variants.update(run_uneven(F, torch, dev, args, vtimed, rel))
    if not args.only_headline:
        res_variants.update(run_paper_sets(F, torch, dev, pos_d, q64, vtimed))
        res_variants.update(run_clustered(F, torch, dev, args, vtimed, rel, linf))
        res_variants.update(run_plummer(F, torch, dev, args, vtimed, rel, linf))

    # roofline of the dominant kernel of the headline pass (one launch per pass)
    dom = max(per_stage, key=per_stage.get)
    K = (args.p + 1) ** 2
    dtype = "f64" if head == "fp64" else "f32"
    if dom == "p2p":
        flops = 20.0 * info["p2p_interactions"]
    elif dom == "l2p":
        flops = 24.0 * K * args.n
    elif dom == "m2l":
        flops = info["n_m2l"] * m2l_flops(args.p)
    else:
        flops = None
    roof = None
    if flops is not None:
        achieved = flops / (per_stage[dom] * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS[dtype],
                "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[dtype],
                "traffic": traffic_from_profile(
                    dom, workload_tag(args.n, args.p, head, args.splits, args.theta)),
                "kernel": dom,
                "kernel_ms": per_stage[dom], "algorithmic_flops": flops}

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"uniform cube N={args.n}, charges U[-1,1), p={args.p}, "
                               f"leaf<={args.leaf}, s={args.splits}, theta={args.theta}, "
                               f"potential+field, {head} forward pass on a cached plan",
                   "n": args.n, "p": args.p, "leaf_max": args.leaf, "splits": args.splits,
                   "theta": args.theta, "precision": head,
                   "tiles": res_tiles.get(head)},
        "accuracy": {**acc, "targets": len(tg), "reference": "direct sum (FP64), library kernel"},
        "variants": res_variants,
        "stage_ms": per_stage,
        "plan_build_ms": plan_ms,
        "plan": {k: info[k] for k in ("depth", "nbox", "n_m2l", "n_p2p", "p2p_interactions")},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def run_batched(F, torch, dev, args, timed, rel, n=1 << 18, R=32):
    """One geometry, R charge vectors per pass (FP32): multi-vector pass
    against R single-vector passes, in point-evaluations per second."""
    import workloads
    pos, Q = workloads.uniform_cube(n, 0, nrhs=R)
    pos_d = torch.from_numpy(pos).to(dev)
    Qd = torch.from_numpy(Q).to(dev).float()
    kw = dict(p=args.p, leaf_max=args.leaf, splits=args.splits, theta=args.theta,
              precision="fp32")
    plan = F.Plan(pos_d, max_rhs=R, **kw)
    single = F.Plan(pos_d, **kw)
    tiles = plan.autotune(Qd[0])
    single.autotune(Qd[0])
    pot = torch.empty((R, n), dtype=torch.float32, device=dev)
    fld = torch.empty((R, n, 3), dtype=torch.float32, device=dev)
    ms_b = timed(lambda: plan.evaluate(Qd, out=(pot, fld)), args.steps, args.warmup)
    p1 = torch.empty((1, n), dtype=torch.float32, device=dev)
    f1 = torch.empty((1, n, 3), dtype=torch.float32, device=dev)

    def singles():
        for r in range(R):
            single.evaluate(Qd[r:r + 1], out=(p1, f1))
    ms_s = timed(singles, max(1, args.steps // 4), 1)
    tg = np.arange(n)
    tg_d = torch.from_numpy(tg).to(dev)
    acc = {}
    for r in (0, R - 1):
        ud, fd = F.direct(pos_d, torch.from_numpy(Q[r]).to(dev), tg_d)
        acc[f"rel_l2_pot_v{r}"] = rel(pot[r].double().cpu().numpy()[tg], ud.cpu().numpy())
        acc[f"rel_l2_field_v{r}"] = rel(fld[r].double().cpu().numpy()[tg], fd.cpu().numpy())
    out = {
        f"fwd_fp32_batched{R}_n{n}": {"ms_per_step": ms_b, "mpoints_s": R * n / ms_b / 1e3,
                                      "vectors": R, "tiles": tiles, **acc},
        f"fwd_fp32_{R}x_single_n{n}": {"ms_per_step": ms_s, "mpoints_s": R * n / ms_s / 1e3,
                                       "vectors": R},
    }
    log(f"batched {R}x{n} fp32: {ms_b:.3f} ms ({R * n / ms_b / 1e3:.1f} Mpoints/s); "
        f"{R} single passes {ms_s:.3f} ms ({R * n / ms_s / 1e3:.1f}); {acc}")
    return out


def run_paper_sets(F, torch, dev, pos_d, q64, timed):
    """The paper's own timed setting on the same 2^20-point uniform cube:
    potential only, relative L-infinity error against the direct sum, its
    three parameter sets (Sec. III.A, Tables II-III; s = 2).  Context for
    the paper's single-GPU figures, not the headline metric."""
    sets = {"paper_set1": (5, 0.70, 128, "fp32"), "paper_set2": (9, 0.50, 256, "fp32"),
            "paper_set3": (10, 0.27, 256, "fp64")}
    ud, _ = F.direct(pos_d, q64, field=False)
    ud = ud.cpu().numpy()
    n = len(ud)
    out = {}
    for name, (p, th, leaf, prec) in sets.items():
        dt = torch.float64 if prec == "fp64" else torch.float32
        plan = F.Plan(pos_d, p=p, leaf_max=leaf, splits=2, theta=th, precision=prec)
        qd = q64.to(dt).reshape(1, n)
        plan.autotune(qd[0])
        pot = torch.empty((1, n), dtype=dt, device=dev)
        ms = timed(lambda: plan.evaluate(qd, field=False, out=(pot, None)), 10, 2)
        u = pot[0].double().cpu().numpy()
        linf = float(np.abs(u - ud).max() / np.abs(ud).max())
        out[name] = {"p": p, "theta": th, "leaf_max": leaf, "splits": 2, "precision": prec,
                     "output": "potential", "ms_per_step": ms, "mpoints_s": n / ms / 1e3,
                     "rel_linf_pot": linf}
        log(f"{name} (p={p}, theta={th}, leaf<={leaf}, s=2, {prec}, potential only): "
            f"{ms:.3f} ms ({n / ms / 1e3:.1f} Mpoints/s), rel L-inf {linf:.2e}")
        del plan
    return out


def run_uneven(F, torch, dev, args, timed, rel, k=16):
    """Sixteen independent uniform-cube problems of log-uniform sizes in
    [1e4, 5e5] (FP32): one plan over all of them replayed as a captured
    graph, against the same plan launched eagerly and against separate
    plans evaluated one after another."""
    import workloads
    sizes = workloads.uneven_problem_sizes(k, seed=100)
    parts = [workloads.uniform_cube(m, 101 + j) for j, m in enumerate(sizes)]
    pos = np.concatenate([a for a, _ in parts])
    q = np.concatenate([b for _, b in parts])
    N = len(pos)
    pos_d = torch.from_numpy(pos).to(dev)
    qd = torch.from_numpy(q).to(dev).float()
    kw = dict(p=args.p, leaf_max=args.leaf, splits=args.splits, theta=args.theta_uneven,
              precision="fp32")
    plan = F.Plan(pos_d, sizes=sizes, **kw)
    qg = qd.reshape(1, N).clone()
    g = F.Graph(plan, qg, field=True)
    ms_g = timed(g.launch, args.steps, args.warmup)
    pot = torch.empty((1, N), dtype=torch.float32, device=dev)
    fld = torch.empty((1, N, 3), dtype=torch.float32, device=dev)
    ms_e = timed(lambda: plan.evaluate(qg, out=(pot, fld)), args.steps, args.warmup)
    off = np.concatenate([[0], np.cumsum(sizes)])
    seps = [F.Plan(pos_d[off[j]:off[j + 1]], **kw) for j in range(k)]
    outs = [(torch.empty((1, m), dtype=torch.float32, device=dev),
             torch.empty((1, m, 3), dtype=torch.float32, device=dev)) for m in sizes]

    def separate():
        for j in range(k):
            seps[j].evaluate(qg[:, off[j]:off[j + 1]].contiguous(), out=outs[j])
    ms_s = timed(separate, args.steps, args.warmup)
    torch.cuda.synchronize()
    eu = ef = 0.0
    for j in range(k):
        tg = np.arange(sizes[j])
        ud, fd = F.direct(pos_d[off[j]:off[j + 1]],
                          torch.from_numpy(parts[j][1]).to(dev), torch.from_numpy(tg).to(dev))
        eu = max(eu, rel(g.pot[0, off[j] + tg].double().cpu().numpy(), ud.cpu().numpy()))
        ef = max(ef, rel(g.field[0, off[j] + tg].double().cpu().numpy(), fd.cpu().numpy()))
    same = bool(torch.equal(g.pot, pot) and torch.equal(g.field, fld))
    out = {
        f"fwd_fp32_uneven{k}_graph": {"ms_per_step": ms_g, "mpoints_s": N / ms_g / 1e3,
                                      "n_total": N, "sizes": sizes, "theta": args.theta_uneven,
                                      "rel_l2_pot_max": eu,
                                      "rel_l2_field_max": ef, "graph_equals_eager": same},
        f"fwd_fp32_uneven{k}_eager": {"ms_per_step": ms_e, "mpoints_s": N / ms_e / 1e3},
        f"fwd_fp32_uneven{k}_separate_plans": {"ms_per_step": ms_s, "mpoints_s": N / ms_s / 1e3},
    }
    log(f"uneven {k} problems (N={N}) fp32: graph {ms_g:.3f} ms ({N / ms_g / 1e3:.1f} Mpoints/s), "
        f"eager {ms_e:.3f} ms, separate plans {ms_s:.3f} ms; rel-L2 pot {eu:.2e} field {ef:.2e}")
    return out


def counters_run(args, pos, q):
    """The headline pass alone, for hardware-counter runs: every kernel of
    one evaluation appears (steps + warmup) times, plus once per autotune
    candidate; then optionally one plain device copy of 256 MiB whose
    FETCH_SIZE / WRITE_SIZE calibrate the HBM byte counters."""
    import torch

    import paper_2511_15269_amd as F
    dev = torch.device("cuda:0")
    if args.counters_batched:
        import workloads
        n, R = 1 << 18, 32
        pos, Q = workloads.uniform_cube(n, 0, nrhs=R)
        plan = F.Plan(torch.from_numpy(pos).to(dev), p=args.p, leaf_max=args.leaf,
                      splits=args.splits, theta=args.theta, precision="fp32", max_rhs=R)
        Qd = torch.from_numpy(Q).to(dev).float()
        tiles = plan.autotune(Qd[0])
        pot = torch.empty((R, n), dtype=torch.float32, device=dev)
        fld = torch.empty((R, n, 3), dtype=torch.float32, device=dev)
        for _ in range(args.warmup + args.steps):
            plan.evaluate(Qd, out=(pot, fld))
    else:
        pos_d = torch.from_numpy(pos).to(dev)
        dt = torch.float64 if args.precision == "fp64" else torch.float32
        qd = torch.from_numpy(q).to(dev).to(dt)
        plan = F.Plan(pos_d, p=args.p, leaf_max=args.leaf, splits=args.splits, theta=args.theta,
                      precision=args.precision)
        tiles = plan.autotune(qd)
        pot = torch.empty((1, args.n), dtype=dt, device=dev)
        fld = torch.empty((1, args.n, 3), dtype=dt, device=dev)
        for _ in range(args.warmup + args.steps):
            plan.evaluate(qd.reshape(1, -1), out=(pot, fld))
    torch.cuda.synchronize()
    if args.copy_calibration:
        a = torch.empty(1 << 25, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
    print(json.dumps({"counters_run": True, "passes": args.warmup + args.steps, "tiles": tiles,
                      "source_sha256": kernel_source_hash()}), flush=True)


def dominant_roofline(stages, info, p, n, dtype, fwd_bwd=False):
    """Algorithmic rate of the slowest stage of a pass (M2L or P2P, whose
    work the plan's counts give) against the vector peak of ``dtype``."""
    dom = max(("m2l", "p2p"), key=lambda k: stages[k])
    if dom == "p2p":
        flops = 20.0 * info["p2p_interactions"]
    else:
        flops = info["n_m2l"] * m2l_flops(p)
    achieved = flops / (stages[dom] * 1e-3) / 1e12
    return {"bound": "alu", "kernel": dom, "kernel_ms": stages[dom], "achieved": achieved,
            "peak": PEAK_TFLOPS[dtype], "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[dtype]}


def profiled_stages(plan, fn, passes=5):
    """Mean per-stage milliseconds of ``passes`` calls of fn (each one pass)."""
    plan.set_profiling(True)
    for _ in range(passes):
        fn()
    st, n = plan.read_profile()
    plan.set_profiling(False)
    return {k: v / max(n, 1) for k, v in st.items()}


def run_clustered(F, torch, dev, args, timed, rel, linf, n=1 << 20):
    """The highly non-uniform set: 8 Gaussians (sigma = 0.01) plus 5% of the
    points on a sphere shell, charges +-1, p = 10, FP32, potential and field
    (theta = 0.7, s = 3, leaf <= 128), accuracy over every point against the
    FP64 direct sum."""
    import workloads
    pos, q = workloads.clustered(n, 0)
    pos_d = torch.from_numpy(pos).to(dev)
    q64 = torch.from_numpy(q).to(dev)
    p, th = 10, 0.7
    plan = F.Plan(pos_d, p=p, leaf_max=args.leaf, splits=args.splits, theta=th,
                  precision="fp32")
    qd = q64.float()
    plan.autotune(qd)
    pot = torch.empty((1, n), dtype=torch.float32, device=dev)
    fld = torch.empty((1, n, 3), dtype=torch.float32, device=dev)
    fn = lambda: plan.evaluate(qd.reshape(1, n), out=(pot, fld))
    ms = timed(fn, args.steps, args.warmup)
    stages = profiled_stages(plan, fn)
    ud, fd = F.direct(pos_d, q64)
    ud, fd = ud.cpu().numpy(), fd.cpu().numpy()
    u, f = pot[0].double().cpu().numpy(), fld[0].double().cpu().numpy()
    info = plan.info()
    out = {"ms_per_step": ms, "mpoints_s": n / ms / 1e3, "p": p, "theta": th,
           "splits": args.splits, "leaf_max": args.leaf, "precision": "fp32",
           "rel_l2_pot": rel(u, ud), "rel_l2_field": rel(f, fd), "rel_linf_pot": linf(u, ud),
           "rel_linf_field": linf(f, fd), "depth": info["depth"], "stage_ms": stages,
           "roofline": dominant_roofline(stages, info, p, n, "f32")}
    log(f"clustered 2^20 p=10 fp32: {ms:.3f} ms ({n / ms / 1e3:.1f} Mpoints/s), rel-L2 pot "
        f"{out['rel_l2_pot']:.2e} field {out['rel_l2_field']:.2e}, roofline "
        f"{out['roofline']['kernel']} {out['roofline']['frac']:.3f}")
    return {"fwd_fp32_clustered1m_p10": out}


def run_plummer(F, torch, dev, args, timed, rel, linf, n=1 << 20):
    """Plummer sphere (a = 0.1), charges in (0, 1], FP32 forward + adjoint of
    E = 1/2 sum q u (dE/dq, dE/dx), p = 8, theta = 0.5, s = 3, leaf <= 128;
    accuracy over every point against the direct-sum gradient
    (dE/dq = u, dE/dx = q grad u)."""
    import workloads
    pos, q = workloads.plummer(n, 0)
    pos_d = torch.from_numpy(pos).to(dev)
    q64 = torch.from_numpy(q).to(dev)
    p, th = 8, 0.5
    plan = F.Plan(pos_d, p=p, leaf_max=args.leaf, splits=args.splits, theta=th,
                  precision="fp32")
    qd = q64.float()
    plan.autotune(qd)
    half = 0.5 * qd
    res = {}

    def fn():
        u, f = plan.evaluate(qd)
        gq, gx = plan.adjoint(qd, half, f)
        res["u"], res["gq"], res["gx"] = u, gq, gx
    ms = timed(fn, args.steps, args.warmup)
    ms_fwd = timed(lambda: plan.evaluate(qd), args.steps, args.warmup)
    stages = profiled_stages(plan, lambda: plan.evaluate(qd))
    ud, fd = F.direct(pos_d, q64)
    ud, fd = ud.cpu().numpy(), fd.cpu().numpy()
    dq = (0.5 * res["u"] + res["gq"]).double().cpu().numpy()
    dx = res["gx"].double().cpu().numpy()
    want_dx = -q[:, None] * fd
    info = plan.info()
    out = {"ms_per_step": ms, "mpoints_s": n / ms / 1e3, "fwd_ms": ms_fwd,
           "p": p, "theta": th, "splits": args.splits, "leaf_max": args.leaf,
           "precision": "fp32", "rel_l2_dEdq": rel(dq, ud), "rel_l2_dEdx": rel(dx, want_dx),
           "rel_linf_dEdq": linf(dq, ud), "rel_linf_dEdx": linf(dx, want_dx),
           "depth": info["depth"], "stage_ms_fwd": stages,
           "roofline_fwd": dominant_roofline(stages, info, p, n, "f32")}
    log(f"plummer 2^20 fwd+bwd fp32: {ms:.3f} ms ({n / ms / 1e3:.1f} Mpoints/s), rel-L2 dE/dq "
        f"{out['rel_l2_dEdq']:.2e} dE/dx {out['rel_l2_dEdx']:.2e}")
    return {"fwd_bwd_fp32_plummer1m": out}


def m2l_flops(p: int) -> float:
    """Algorithmic flops of one rotation-based M2L: two polar rotations of
    sum_n (2n^2+2n+1) MACs, the z-axis translation of the same count, and
    O(p^2) azimuthal rotations and Wigner-matrix work."""
    rot = sum(2 * n * n + 2 * n + 1 for n in range(p + 1))
    az = 4 * p * (p + 1) // 2
    wig = (p + 1) * (p + 2) * (2 * p + 3) // 6 * 4
    return 2.0 * (3 * rot) + 2 * az + wig


if __name__ == "__main__":
    main()
