"""Pins of the oracle's direct sum (eqs. 1-3) and FMM (Sec. II) against
closed forms, symmetries and limiting cases."""
import math

import numpy as np
import pytest

import workloads
from oracle import basis as B
from oracle.direct import FOUR_PI, direct, direct_fsum
from oracle.fmm import fmm, multipoles
from oracle.lists import build_lists
from oracle.tree import build_tree


def test_coulomb_pair():
    src = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 2.0]])
    q = np.array([3.0, -5.0])
    u, g = direct(src, q, field=True)
    assert u[0] == pytest.approx(-(-5.0) / (FOUR_PI * 2.0), rel=1e-15)
    assert u[1] == pytest.approx(-3.0 / (FOUR_PI * 2.0), rel=1e-15)
    # grad u at point 0 = (1/4pi) q1 (x0 - x1)/r^3 = (1/4pi)(-5)(0,0,-2)/8
    assert np.allclose(g[0], [0, 0, 10.0 / (8 * FOUR_PI)], rtol=1e-15)


def test_matches_correctly_rounded_sum():
    pos, q = workloads.uniform_cube(64, 3)
    u, _ = direct(pos, q)
    assert np.allclose(u, direct_fsum(pos, q), rtol=1e-13, atol=0)


def test_reciprocity_and_linearity():
    pos, q = workloads.uniform_cube(700, 4)
    g = np.random.default_rng(5).uniform(-1, 1, 700)
    uq, _ = direct(pos, q)
    ug, _ = direct(pos, g)
    assert np.dot(g, uq) == pytest.approx(np.dot(q, ug), rel=1e-12)
    u2, _ = direct(pos, 2 * q - 3 * g)
    assert np.allclose(u2, 2 * uq - 3 * ug, rtol=1e-12, atol=1e-12)


def test_power_of_two_scaling_and_translation():
    pos, q = workloads.uniform_cube(500, 6)
    u, gu = direct(pos, q, field=True)
    u2, gu2 = direct(4.0 * pos, q, field=True)
    assert np.array_equal(u2, u / 4.0)
    assert np.allclose(gu2, gu / 16.0, rtol=1e-14, atol=0)
    u3, _ = direct(pos + 8.0, q)
    assert np.allclose(u3, u, rtol=1e-12, atol=1e-12)


def test_coincident_points_contribute_nothing():
    src = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    q = np.array([1.0, 2.0, 4.0])
    u, g = direct(src, q, field=True)
    assert u[0] == pytest.approx(-4.0 / FOUR_PI)
    assert np.all(np.isfinite(g))


def test_fmm_without_far_field_is_the_direct_sum():
    # N <= leaf size: a single box, everything direct
    pos, q = workloads.uniform_cube(100, 7)
    u, f = fmm(pos, q, p=4, leaf_max=128)
    ud, gd = direct(pos, q, field=True)
    assert np.allclose(u, ud, rtol=1e-13)
    assert np.allclose(f, -gd, rtol=1e-12, atol=1e-12)


def test_root_monopole_is_total_charge():
    pos, q = workloads.uniform_cube(3000, 8)
    tr = build_tree(pos, 64, 2)
    C = multipoles(tr, pos, q, 3)
    assert C[0, B.idx(0, 0)] == pytest.approx(q.sum(), rel=1e-12, abs=1e-12)
    for l in range(tr.L + 1):
        sl = slice(tr.level_off[l], tr.level_off[l + 1])
        assert C[sl, B.idx(0, 0)].sum() == pytest.approx(q.sum(), rel=1e-12, abs=1e-12)


def test_error_decays_with_order_and_reaches_roundoff():
    pos, q = workloads.uniform_cube(2048, 9)
    tr = build_tree(pos, 32, 2)
    li = build_lists(tr, 0.5)
    ud, gd = direct(pos, q, field=True)
    errs = []
    for p in (2, 4, 6, 8, 12, 20):
        u, f = fmm(pos, q, p, 32, tree=tr, lists=li)
        errs.append(np.linalg.norm(u - ud) / np.linalg.norm(ud))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    # eq. 5 with theta = 0.5: error ~ theta^{p+1}/(1-theta)^2
    assert errs[-1] < 1e-8


def test_config_scale_accuracy_vs_direct():
    pos, q = workloads.uniform_cube(4096, 0)
    u, f = fmm(pos, q, 6, 64, 2, 0.6)
    ud, gd = direct(pos, q, field=True)
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 1e-4
    assert np.linalg.norm(f + gd) / np.linalg.norm(gd) < 3e-4


def test_sampled_targets_equal_full_evaluation():
    pos, q = workloads.uniform_cube(3000, 10)
    u, f = fmm(pos, q, 5, 32, 2, 0.6)
    tg = workloads.sample_targets(3000, 100)
    us, fs = fmm(pos, q, 5, 32, 2, 0.6, targets=tg)
    assert np.allclose(us, u[tg], rtol=1e-13, atol=1e-15)
    assert np.allclose(fs, f[tg], rtol=1e-13, atol=1e-14)
