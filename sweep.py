#!/usr/bin/env python3
"""Parameter sweeps of the FMM evaluation pass on one MI355X: the paper's
experiments of Sec. III.A on its two distributions.

``sizes``: points uniform in the unit cube and uniform on the unit sphere
surface, N = 2^11 .. 2^22, the three parameter sets of Table II (s = 2,
potential only; set 1 p = 5, theta = 0.70, N_max = 128, FP32; set 2 p = 9,
theta = 0.50, N_max = 256, FP32; set 3 p = 10, theta = 0.27, N_max = 256,
FP64).  Per point: the fastest of ``--reps`` event-timed passes on a
cached plan (the paper reports the minimum of repeated evaluations), the
per-stage times, the relative L-infinity error against the FP64 direct sum
for N <= 2^20 (the paper's limit for its error figures), and parity with
the CPU oracle FMM (same tree, lists and order) at 64 sampled targets for
N <= 2^18.

``accuracy``: the uniform cube at N = 2^15 (FP64, s = 2, N_max = 128):
the relative L-infinity error against the direct sum for p = 1..10 at
theta = 0.7 and for theta = 0.3 .. 0.8 at p = 5, with the effective theta
of the plan's lists (eq. 4 solved for theta on every M2L pair,
R / (d - r), averaged) and the slope the bound of eq. 5 predicts with it;
every point also checked against the oracle at 64 targets.

    python sweep.py sizes [--max-log2 22] [--md profiles/sweep_sizes.md]
    python sweep.py accuracy [--md profiles/sweep_accuracy.md]

One JSON line per point on stdout; a markdown summary with ``--md``.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SETS = {1: (5, 0.70, 128, "fp32"), 2: (9, 0.50, 256, "fp32"), 3: (10, 0.27, 256, "fp64")}
PARITY_TARGETS = 64


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def inputs(dist: str, n: int, seed: int = 0):
    import workloads
    if dist == "cube":
        return workloads.uniform_cube(n, seed)
    if dist == "sphere":
        return workloads.sphere_surface(n, seed, 1.0)
    raise KeyError(dist)


def oracle_at_samples(job):
    """Oracle FMM potential at sampled targets (a forked worker, one thread)."""
    import threadpoolctl

    import workloads
    from oracle.fmm import fmm
    dist, n, p, theta, leaf, seed = job
    pos, q = inputs(dist, n, seed)
    tg = workloads.sample_targets(n, PARITY_TARGETS, seed=3)
    with threadpoolctl.threadpool_limits(1):
        u, _ = fmm(pos, q, p, leaf, 2, theta, targets=tg, field=False)
    return job, tg, u


def time_passes(plan, qd, pot, reps, torch):
    """Fastest of ``reps`` single passes, each between its own events."""
    plan.evaluate(qd, field=False, out=(pot, None))
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.evaluate(qd, field=False, out=(pot, None))
        e1.record()
        e1.synchronize()
        t = e0.elapsed_time(e1)
        best = t if best is None else min(best, t)
    return best


def theta_eff(plan) -> float:
    """Mean over the plan's M2L pairs of R / (d - r), the theta for which
    eq. 4 holds with equality (R, r the larger and smaller radius, d the
    distance of the centres)."""
    _, _, c, r = plan.tree()
    ms, mt, _, _ = plan.lists()
    if len(ms) == 0:
        return float("nan")
    d = np.linalg.norm(c[ms] - c[mt], axis=1)
    big, small = np.maximum(r[ms], r[mt]), np.minimum(r[ms], r[mt])
    return float(np.mean(big / (d - small)))


def run(points, args):
    """points: list of dicts (dist, n, p, theta, leaf, prec, label)."""
    jobs = [(pt["dist"], pt["n"], pt["p"], pt["theta"], pt["leaf"], 0)
            for pt in points if pt["n"] <= args.parity_max_n]
    ctx = mp.get_context("fork")
    pool = ctx.Pool(min(8, max(1, len(os.sched_getaffinity(0)) // 2)))
    pending = pool.map_async(oracle_at_samples, jobs, chunksize=1)

    import torch

    import paper_2511_15269_amd as F
    dev = torch.device("cuda:0")
    rows = []
    direct_cache = {}
    for pt in points:
        pos, q = inputs(pt["dist"], pt["n"], 0)
        dt = torch.float64 if pt["prec"] == "fp64" else torch.float32
        pos_d = torch.from_numpy(pos).to(dev)
        qd = torch.from_numpy(q).to(dev).to(dt).reshape(1, -1)
        t0 = time.perf_counter()
        plan = F.Plan(pos_d, p=pt["p"], leaf_max=pt["leaf"], splits=2, theta=pt["theta"],
                      precision=pt["prec"])
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - t0) * 1e3
        plan.autotune(qd[0])
        pot = torch.empty_like(qd)
        ms = time_passes(plan, qd, pot, args.reps, torch)
        plan.set_profiling(True)
        for _ in range(3):
            plan.evaluate(qd, field=False, out=(pot, None))
        st, npass = plan.read_profile()
        plan.set_profiling(False)
        inf = plan.info()
        row = dict(pt, ms=ms, mpoints_s=pt["n"] / ms / 1e3, build_ms=build_ms,
                   stages={k: v / npass for k, v in st.items()}, depth=inf["depth"],
                   n_m2l=inf["n_m2l"], p2p_interactions=inf["p2p_interactions"])
        if args.theta_eff:
            row["theta_eff"] = theta_eff(plan)
        u = pot[0].double().cpu().numpy()
        if pt["n"] <= args.error_max_n:
            key = (pt["dist"], pt["n"])
            if key not in direct_cache:
                ud, _ = F.direct(pos_d, torch.from_numpy(q).to(dev), field=False)
                direct_cache.clear()
                direct_cache[key] = ud.cpu().numpy()
            ud = direct_cache[key]
            row["rel_linf"] = float(np.abs(u - ud).max() / np.abs(ud).max())
        row["_u"] = u
        rows.append(row)
        log(f"{pt['label']} {pt['dist']} N={pt['n']}: {ms:.3f} ms ({row['mpoints_s']:.1f} Mpts/s)"
            + (f", rel Linf {row['rel_linf']:.2e}" if "rel_linf" in row else "")
            + (f", theta_eff {row['theta_eff']:.3f}" if "theta_eff" in row else ""))
        del plan
    # parity with the oracle at the sampled targets
    res = {j: (tg, u) for j, tg, u in pending.get()}
    pool.close()
    ok = True
    for row in rows:
        j = (row["dist"], row["n"], row["p"], row["theta"], row["leaf"], 0)
        u = row.pop("_u")
        if j not in res:
            continue
        tg, u0 = res[j]
        err = float(max(np.linalg.norm(u[tg] - u0) / np.linalg.norm(u0),
                        np.abs(u[tg] - u0).max() / np.abs(u0).max()))
        bound = 1e-10 if row["prec"] == "fp64" else 1e-5
        row["parity_vs_oracle"] = err
        row["parity_ok"] = err <= bound
        ok = ok and row["parity_ok"]
    for row in rows:
        print(json.dumps(row), flush=True)
    return rows, ok


def md_sizes(rows, cmd):
    out = ["# FMM pass vs N: uniform cube and sphere surface, paper parameter sets", "",
           "Command: `" + cmd + "`", "",
           "One MI355X; potential only, s = 2; time = fastest single pass on a cached plan "
           "(tree and lists built once); rel L-inf against the FP64 direct sum (N <= 2^20); "
           "parity = max(rel-L2, rel-max) against the CPU oracle FMM at 64 sampled targets "
           "(N <= 2^18; bound 1e-10 FP64, 1e-5 FP32).", "",
           "| dist | set | N | ms | Mpts/s | rel L-inf | parity | depth | M2L pairs | P2P interactions |",
           "|---|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| {r['dist']} | {r['label']} | 2^{int(round(math.log2(r['n'])))} | "
                   f"{r['ms']:.3f} | {r['mpoints_s']:.1f} | "
                   f"{r.get('rel_linf', float('nan')):.2e} | "
                   f"{r.get('parity_vs_oracle', float('nan')):.1e} | {r['depth']} | "
                   f"{r['n_m2l']} | {r['p2p_interactions']} |")
    return "\n".join(out) + "\n"


def md_accuracy(rows, cmd):
    out = ["# Error vs p and theta, uniform cube N = 2^15 (FP64, s = 2, N_max = 128)", "",
           "Command: `" + cmd + "`", "",
           "rel L-inf against the direct sum over all points; theta_eff = mean of R / (d - r) "
           "over the plan's M2L pairs; `bound slope` = theta_eff^(p+1) / (1 - theta_eff)^2 "
           "(eq. 5 without its constant); parity against the CPU oracle at 64 targets.", "",
           "| sweep | p | theta | theta_eff | rel L-inf | bound slope | parity | ms |",
           "|---|---|---|---|---|---|---|---|"]
    for r in rows:
        te = r["theta_eff"]
        slope = te ** (r["p"] + 1) / (1 - te) ** 2
        out.append(f"| {r['label']} | {r['p']} | {r['theta']} | {te:.3f} | "
                   f"{r['rel_linf']:.2e} | {slope:.2e} | "
                   f"{r.get('parity_vs_oracle', float('nan')):.1e} | {r['ms']:.3f} |")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["sizes", "accuracy"])
    ap.add_argument("--min-log2", type=int, default=11)
    ap.add_argument("--max-log2", type=int, default=22)
    ap.add_argument("--dists", default="cube,sphere")
    ap.add_argument("--sets", default="1,2,3")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--error-max-n", type=int, default=1 << 20)
    ap.add_argument("--parity-max-n", type=int, default=1 << 18)
    ap.add_argument("--md", default=None)
    args = ap.parse_args()
    cmd = "python sweep.py " + " ".join(sys.argv[1:])
    points = []
    if args.mode == "sizes":
        args.theta_eff = False
        for dist in args.dists.split(","):
            for k in (int(x) for x in args.sets.split(",")):
                p, th, leaf, prec = SETS[k]
                for e in range(args.min_log2, args.max_log2 + 1):
                    points.append(dict(dist=dist, n=1 << e, p=p, theta=th, leaf=leaf, prec=prec,
                                       label=f"set{k}"))
    else:
        args.theta_eff = True
        n = 1 << 15
        for p in range(1, 11):
            points.append(dict(dist="cube", n=n, p=p, theta=0.7, leaf=128, prec="fp64",
                               label="p"))
        for th in (0.3, 0.4, 0.5, 0.6, 0.7, 0.8):
            points.append(dict(dist="cube", n=n, p=5, theta=th, leaf=128, prec="fp64",
                               label="theta"))
    rows, ok = run(points, args)
    if args.md:
        text = (md_sizes if args.mode == "sizes" else md_accuracy)(rows, cmd)
        with open(args.md, "w") as f:
            f.write(text)
    if not ok:
        log("parity with the oracle FAILED for some point")
        sys.exit(1)


if __name__ == "__main__":
    main()
