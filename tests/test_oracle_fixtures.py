"""The stored oracle values under tests/golden/ (used by the full-size GPU
parity tests) are the oracle's: the generated inputs hash to the recorded
value, and a sample of the stored outputs is recomputed here with the
oracle FMM and direct sum and must agree to rounding."""
import numpy as np
import pytest

import workloads
from _fixtures import input_hash, load
from _norms import parity

pytestmark = pytest.mark.slow

N = 1 << 20


def _oracle(pos, q, p, leaf, s, theta, tg):
    from oracle.fmm import fmm as oracle_fmm
    from oracle.lists import build_lists
    from oracle.tree import build_tree
    tr = build_tree(pos, leaf, s)
    li = build_lists(tr, theta)
    u, f = oracle_fmm(pos, q, p, leaf, s, theta, targets=tg, tree=tr, lists=li)
    return u, f, tr, li


def _pick(n, k, seed):
    return np.sort(np.random.default_rng(seed).choice(n, k, replace=False))


@pytest.mark.parametrize("name,gen", [("oracle_cube1m_p8_s3_t80", workloads.uniform_cube),
                                      ("oracle_clustered1m_p10_s3_t70", workloads.clustered)])
def test_single_problem_fixture(name, gen):
    from oracle.direct import direct
    pos, q = gen(N, 0)
    fx = load(name, pos, q)
    k = _pick(len(fx["targets"]), 6, 1)
    tg = fx["targets"][k]
    u, f, tr, li = _oracle(pos, q, int(fx["p"]), int(fx["leaf"]), int(fx["s"]),
                           float(fx["theta"]), tg)
    assert tr.L == fx["depth"] and len(li.m2l_src) == fx["n_m2l"]
    assert len(li.p2p_src) == fx["n_p2p"]
    assert parity(u, fx["u"][k]) <= 1e-13 and parity(f, fx["f"][k]) <= 1e-13
    ud, gd = direct(pos, q, pos[tg], field=True)
    assert parity(ud, fx["u_direct"][k]) <= 1e-13 and parity(-gd, fx["f_direct"][k]) <= 1e-13


def test_plummer_gradient_fixture():
    from oracle.gradient import energy_gradient_direct
    pos, q = workloads.plummer(N, 0)
    fx = load("oracle_plummer1m_direct_gradient", pos, q)
    k = _pick(len(fx["targets"]), 16, 2)
    dq, dx = energy_gradient_direct(pos, q, targets=fx["targets"][k])
    assert parity(dq, fx["dEdq"][k]) <= 1e-13 and parity(dx, fx["dEdx"][k]) <= 1e-13


def test_batched_fixture():
    pos, Q = workloads.uniform_cube(1 << 18, 0, nrhs=32)
    fx = load("oracle_batched256k_r32_p8_s3_t80", pos, Q)
    k = _pick(len(fx["targets"]), 8, 3)
    j = 1  # the middle stored vector
    u, f, _, _ = _oracle(pos, Q[fx["vectors"][j]], int(fx["p"]), int(fx["leaf"]), int(fx["s"]),
                         float(fx["theta"]), fx["targets"][k])
    assert parity(u, fx["u"][j][k]) <= 1e-13 and parity(f, fx["f"][j][k]) <= 1e-13


def test_uneven_fixture():
    from oracle.direct import direct
    sizes = workloads.uneven_problem_sizes(16, seed=100)
    fx = load("oracle_uneven16_p8_s3_t60")
    assert list(fx["sizes"]) == sizes
    for j in (int(np.argmin(sizes)), 3):
        pj, qj = workloads.uniform_cube(sizes[j], 101 + j)
        assert str(fx["hashes"][j]) == input_hash(pj, qj)
        k = _pick(len(fx[f"targets_{j}"]), 8, 4 + j)
        tg = fx[f"targets_{j}"][k]
        u, f, _, _ = _oracle(pj, qj, int(fx["p"]), int(fx["leaf"]), int(fx["s"]),
                             float(fx["theta"]), tg)
        assert parity(u, fx[f"u_{j}"][k]) <= 1e-13 and parity(f, fx[f"f_{j}"][k]) <= 1e-13
        ud, gd = direct(pj, qj, pj[tg], field=True)
        assert parity(ud, fx[f"u_direct_{j}"][k]) <= 1e-13
