"""Write the oracle values the full-size GPU parity tests compare against.

Calls only ``oracle/`` (and the seeded generators of ``workloads.py``): the
FP64 oracle FMM and direct sum at sampled targets of the 2^20-point
workloads, which take minutes on the host and are therefore computed once
here instead of on a GPU machine.  Each ``.npz`` holds the workload's
parameters, a SHA-256 of the generated positions and charges (the tests
regenerate the inputs and refuse a fixture whose hash differs), the target
indices and the oracle outputs.  ``tests/test_oracle_fixtures.py``
recomputes a sample of every fixture with the oracle.

    python tests/golden/make_oracle_fixtures.py [name ...]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import workloads  # noqa: E402
from _fixtures import input_hash  # noqa: E402
from oracle.direct import direct  # noqa: E402
from oracle.fmm import fmm as oracle_fmm  # noqa: E402
from oracle.gradient import energy_gradient_direct  # noqa: E402
from oracle.lists import build_lists  # noqa: E402
from oracle.tree import build_tree  # noqa: E402

N = 1 << 20
TARGETS = 1024


def fmm_case(pos, q, p, leaf, s, theta, tg, hier=None):
    if hier is None:
        tr = build_tree(pos, leaf, s)
        hier = (tr, build_lists(tr, theta))
    tr, li = hier
    u, f = oracle_fmm(pos, q, p, leaf, s, theta, targets=tg, tree=tr, lists=li)
    return u, f, hier


def cube():
    p, leaf, s, theta = 8, 128, 3, 0.8
    pos, q = workloads.uniform_cube(N, 0)
    tg = workloads.sample_targets(N, TARGETS, seed=11)
    u, f, (tr, li) = fmm_case(pos, q, p, leaf, s, theta, tg)
    ud, gd = direct(pos, q, pos[tg], field=True)
    return dict(p=p, leaf=leaf, s=s, theta=theta, hash=input_hash(pos, q), targets=tg,
                u=u, f=f, u_direct=ud, f_direct=-gd, depth=tr.L, n_m2l=len(li.m2l_src),
                n_p2p=len(li.p2p_src))


def clustered():
    p, leaf, s, theta = 10, 128, 3, 0.7
    pos, q = workloads.clustered(N, 0)
    tg = workloads.sample_targets(N, TARGETS, seed=12)
    u, f, (tr, li) = fmm_case(pos, q, p, leaf, s, theta, tg)
    ud, gd = direct(pos, q, pos[tg], field=True)
    return dict(p=p, leaf=leaf, s=s, theta=theta, hash=input_hash(pos, q), targets=tg,
                u=u, f=f, u_direct=ud, f_direct=-gd, depth=tr.L, n_m2l=len(li.m2l_src),
                n_p2p=len(li.p2p_src))


def plummer_gradient():
    pos, q = workloads.plummer(N, 0)
    sub = workloads.sample_targets(N, 4096, seed=13)
    dq, dx = energy_gradient_direct(pos, q, targets=sub)
    return dict(hash=input_hash(pos, q), targets=sub, dEdq=dq, dEdx=dx)


def batched():
    n, R, p, leaf, s, theta = 1 << 18, 32, 8, 128, 3, 0.8
    pos, Q = workloads.uniform_cube(n, 0, nrhs=R)
    tg = workloads.sample_targets(n, TARGETS, seed=15)
    out = dict(p=p, leaf=leaf, s=s, theta=theta, hash=input_hash(pos, Q), targets=tg,
               vectors=np.array([0, 17, R - 1]))
    hier = None
    us, fs = [], []
    for r in out["vectors"]:
        u, f, hier = fmm_case(pos, Q[r], p, leaf, s, theta, tg, hier)
        us.append(u)
        fs.append(f)
    out["u"] = np.stack(us)
    out["f"] = np.stack(fs)
    return out


def uneven():
    p, leaf, s, theta = 8, 128, 3, 0.6
    sizes = workloads.uneven_problem_sizes(16, seed=100)
    out = dict(p=p, leaf=leaf, s=s, theta=theta, sizes=np.array(sizes))
    hashes = []
    for j, m in enumerate(sizes):
        pj, qj = workloads.uniform_cube(m, 101 + j)
        hashes.append(input_hash(pj, qj))
        tg = workloads.sample_targets(m, 256, seed=16 + j)
        u, f, _ = fmm_case(pj, qj, p, leaf, s, theta, tg)
        ud, gd = direct(pj, qj, pj[tg], field=True)
        out[f"targets_{j}"] = tg
        out[f"u_{j}"] = u
        out[f"f_{j}"] = f
        out[f"u_direct_{j}"] = ud
        out[f"f_direct_{j}"] = -gd
    out["hashes"] = np.array(hashes)
    return out


CASES = {"oracle_cube1m_p8_s3_t80": cube, "oracle_clustered1m_p10_s3_t70": clustered,
         "oracle_plummer1m_direct_gradient": plummer_gradient,
         "oracle_batched256k_r32_p8_s3_t80": batched, "oracle_uneven16_p8_s3_t60": uneven}


def main(names):
    for name in names or CASES:
        t0 = time.time()
        data = CASES[name]()
        np.savez_compressed(os.path.join(HERE, name + ".npz"), **data)
        print(f"{name}: {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
