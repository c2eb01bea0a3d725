"""Pins of the oracle's energy gradients (E = 1/2 sum q_i u_i): the adjoint
identity of the transposed-list FMM, central finite differences of the
frozen-hierarchy FMM energy, and the direct-sum gradient."""
import numpy as np
import pytest

import workloads
from oracle.direct import direct
from oracle.fmm import fmm
from oracle.gradient import (energy_direct, energy_fmm, energy_gradient_direct,
                             energy_gradient_fmm, transpose_lists)
from oracle.lists import build_lists
from oracle.tree import build_tree


@pytest.mark.parametrize("n,p,leaf,s,theta", [(1500, 5, 32, 2, 0.6), (2000, 4, 16, 3, 0.7),
                                              (1200, 6, 16, 1, 0.5)])
def test_transposed_fmm_is_the_adjoint(n, p, leaf, s, theta):
    pos, q = workloads.uniform_cube(n, 11)
    g = np.random.default_rng(12).uniform(-1, 1, n)
    tr = build_tree(pos, leaf, s)
    li = build_lists(tr, theta)
    lt = transpose_lists(li)
    Gq, _ = fmm(pos, q, p, leaf, s, theta, tree=tr, lists=li, field=False)
    GTg, _ = fmm(pos, g, p, leaf, s, theta, tree=tr, lists=lt, field=False)
    lhs, rhs = np.dot(g, Gq), np.dot(GTg, q)
    assert lhs == pytest.approx(rhs, rel=1e-12)
    # the operator is not symmetric, so the transposed run is a different map
    GTq, _ = fmm(pos, q, p, leaf, s, theta, tree=tr, lists=lt, field=False)
    assert np.abs(GTq - Gq).max() > 1e3 * 1e-16 * np.abs(Gq).max()


def test_direct_gradient_matches_finite_differences():
    pos, q = workloads.uniform_cube(300, 13)
    dq, dx = energy_gradient_direct(pos, q)
    h = 1e-6
    rng = np.random.default_rng(14)
    for i in rng.choice(300, 6, replace=False):
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, a] += h
            pm[i, a] -= h
            fd = (energy_direct(pp, q) - energy_direct(pm, q)) / (2 * h)
            assert fd == pytest.approx(dx[i, a], rel=1e-6, abs=1e-9)
        qp, qm = q.copy(), q.copy()
        qp[i] += h
        qm[i] -= h
        fd = (energy_direct(pos, qp) - energy_direct(pos, qm)) / (2 * h)
        assert fd == pytest.approx(dq[i], rel=1e-8)


def test_fmm_gradient_matches_finite_differences_of_frozen_energy():
    n, p, leaf, s, theta = 1000, 5, 32, 2, 0.6
    pos, q = workloads.uniform_cube(n, 15)
    tr = build_tree(pos, leaf, s)
    li = build_lists(tr, theta)
    dq, dx = energy_gradient_fmm(pos, q, p, leaf, s, theta, tr, li)
    h = 1e-6
    rng = np.random.default_rng(16)
    for i in rng.choice(n, 4, replace=False):
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, a] += h
            pm[i, a] -= h
            fd = (energy_fmm(pp, q, p, leaf, s, theta, tr, li) -
                  energy_fmm(pm, q, p, leaf, s, theta, tr, li)) / (2 * h)
            assert fd == pytest.approx(dx[i, a], rel=1e-6, abs=1e-8)
        qp, qm = q.copy(), q.copy()
        qp[i] += h
        qm[i] -= h
        fd = (energy_fmm(pos, qp, p, leaf, s, theta, tr, li) -
              energy_fmm(pos, qm, p, leaf, s, theta, tr, li)) / (2 * h)
        assert fd == pytest.approx(dq[i], rel=1e-8)


def test_fmm_gradient_close_to_direct_gradient():
    n, p, leaf, s, theta = 3000, 8, 64, 2, 0.6
    pos, q = workloads.plummer(n, 17)
    tr = build_tree(pos, leaf, s)
    li = build_lists(tr, theta)
    dq, dx = energy_gradient_fmm(pos, q, p, leaf, s, theta, tr, li)
    dq0, dx0 = energy_gradient_direct(pos, q)
    assert np.linalg.norm(dq - dq0) / np.linalg.norm(dq0) < 1e-4
    assert np.linalg.norm(dx - dx0) / np.linalg.norm(dx0) < 1e-4
