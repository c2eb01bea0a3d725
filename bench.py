#!/usr/bin/env python3
"""Throughput of the FMM evaluation pass on one MI355X.

Workload: N = 2^20 charges uniform in the unit cube, charges uniform in
[-1, 1), expansion order p = 8, leaf size <= 128, potential and field.  A
step is one evaluation pass (sort, P2M, M2M, M2L, L2L, L2P, P2P) of one
charge vector on a cached plan (tree and lists built once, as in the
paper's protocol), inputs resident in HBM.  ``value`` = N / step time in
Mpoints/s.  The accuracy against the direct sum is measured on 8192
sampled targets with the library's direct kernel; the roofline object
reports the dominant kernel (per-stage HIP events over the timed steps);
``cpu_baseline`` times the CPU oracle on a bounded sample.

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


def traffic_from_profile(kernel_prefix: str):
    """HBM bytes per launch recorded for the dominant kernel under profiles/,
    if the kernel source has not changed since (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel_prefix}_cube1m_p8_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source_sha256:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (m and t):
        return None
    src = open(os.path.join(ROOT, "paper_2511_15269_amd", "csrc", "eval.hip"), "rb").read()
    if hashlib.sha256(src).hexdigest() != m.group(1):
        return None
    return float(t.group(1))


def cpu_baseline(pos, q, p, leaf, s, theta, n_targets=256):
    """The CPU oracle FMM, one thread, on a bounded sample: the potential
    and field at ``n_targets`` sampled points with the hierarchy (tree and
    lists) built beforehand, as for the GPU plan."""
    import threadpoolctl
    import workloads
    from oracle.fmm import fmm as oracle_fmm
    from oracle.lists import build_lists
    from oracle.tree import build_tree
    with threadpoolctl.threadpool_limits(1):
        tr = build_tree(pos, leaf, s)
        li = build_lists(tr, theta)
        tg = workloads.sample_targets(len(pos), n_targets, seed=7)
        t0 = time.perf_counter()
        oracle_fmm(pos, q, p, leaf, s, theta, targets=tg, tree=tr, lists=li)
        dt = time.perf_counter() - t0
    return {"value": n_targets / dt / 1e6, "unit": "Mpoints/s", "cores": 1,
            "kind": "oracle",
            "sample": f"FMM potential+field at {n_targets} sampled targets of the same "
                      f"2^20-point workload, tree and lists prebuilt; {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--p", type=int, default=8)
    ap.add_argument("--leaf", type=int, default=128)
    ap.add_argument("--splits", type=int, default=3)
    ap.add_argument("--theta", type=float, default=0.7)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--samples", type=int, default=8192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-targets", type=int, default=1024)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (HBM counter scale)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the FMM library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2511_15269_amd as F
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pos, q = workloads.uniform_cube(args.n, 0)
    tdt = torch.float64 if args.precision == "fp64" else torch.float32
    pos_d = torch.from_numpy(pos).to(dev)
    q_d = torch.from_numpy(q).to(dev, tdt)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    plan = F.Plan(pos_d, p=args.p, leaf_max=args.leaf, splits=args.splits, theta=args.theta,
                  precision=args.precision)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    info = plan.info()
    log(f"plan: {plan_ms:.1f} ms, depth {info['depth']}, M2L {info['n_m2l']}, "
        f"P2P pairs {info['n_p2p']}, P2P interactions {info['p2p_interactions']}")

    pot = torch.empty(args.n, dtype=tdt, device=dev)
    fld = torch.empty((args.n, 3), dtype=tdt, device=dev)
    out = (pot.view(1, -1), fld.view(1, -1, 3))
    for _ in range(args.warmup):
        plan.evaluate(q_d, out=out)
    torch.cuda.synchronize()
    if args.copy_calibration:
        a = torch.empty(1 << 25, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    plan.set_profiling(True)
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        plan.evaluate(q_d, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - w0) * 1e3
    total_ms = ev0.elapsed_time(ev1)
    stage_ms, passes = plan.read_profile()
    plan.set_profiling(False)
    ms_per_step = total_ms / args.steps
    value = args.n / (ms_per_step * 1e-3) / 1e6
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step (wall {wall_ms / args.steps:.3f}), "
        f"{value:.1f} Mpoints/s")
    per_stage = {k: v / max(passes, 1) for k, v in stage_ms.items()}
    log("stages (ms/pass): " + ", ".join(f"{k} {v:.3f}" for k, v in per_stage.items()))

    # accuracy against the direct sum (library's direct kernel, FP64)
    tg = workloads.sample_targets(args.n, args.samples, seed=1)
    tg_d = torch.from_numpy(tg).to(dev)
    ud, fd = F.direct(pos_d, torch.from_numpy(q).to(dev), tg_d)
    torch.cuda.synchronize()
    ud, fd = ud.cpu().numpy(), fd.cpu().numpy()
    up = pot.double().cpu().numpy()[tg]
    fp = fld.double().cpu().numpy()[tg]
    rel_pot = float(np.linalg.norm(up - ud) / np.linalg.norm(ud))
    rel_fld = float(np.linalg.norm(fp - fd) / np.linalg.norm(fd))
    log(f"rel-L2 vs direct on {args.samples} targets: pot {rel_pot:.3e}, field {rel_fld:.3e}")

    # roofline of the dominant kernel (one launch per pass)
    dom = max(per_stage, key=per_stage.get)
    K = (args.p + 1) ** 2
    dtype = "f64" if args.precision == "fp64" else "f32"
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
                "traffic": traffic_from_profile(dom), "kernel": dom,
                "kernel_ms": per_stage[dom], "algorithmic_flops": flops}

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(pos, q, args.p, args.leaf, args.splits, args.theta, args.cpu_targets)
        log(f"cpu baseline: {cpu['value']:.3e} Mpoints/s ({cpu['sample']})")

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
                               f"potential+field, {args.precision}, cached plan",
                   "n": args.n, "p": args.p, "leaf_max": args.leaf, "splits": args.splits,
                   "theta": args.theta, "precision": args.precision},
        "accuracy": {"rel_l2_pot": rel_pot, "rel_l2_field": rel_fld,
                     "samples": args.samples, "reference": "direct sum (FP64)"},
        "stage_ms": per_stage,
        "plan_build_ms": plan_ms,
        "plan": {k: info[k] for k in ("depth", "nbox", "n_m2l", "n_p2p", "p2p_interactions")},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


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
