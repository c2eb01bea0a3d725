"""Pins of the oracle's expansions and translation operators (Sec. II.C;
App. B.3) against closed forms and the exact potential."""
import math

import numpy as np
import pytest

from oracle import basis as B
from oracle.expansions import FOUR_PI, eval_local, eval_multipole, p2l, p2m
from oracle.translations import m2l


def _coulomb(x, y, q):
    return -q / (FOUR_PI * np.linalg.norm(x - y))


@pytest.mark.parametrize("p", [2, 5, 8, 12])
def test_single_charge_multipole_within_bound(p):
    # error of the multipole expansion <= q (a/r)^{p+1} / (r - a) / (4 pi)
    rng = np.random.default_rng(p)
    c = rng.random(3)
    for _ in range(8):
        y = c + 0.3 * rng.standard_normal(3) / math.sqrt(3)
        a = np.linalg.norm(y - c)
        x = c + rng.standard_normal(3)
        x = c + (x - c) * (4 * a / np.linalg.norm(x - c))
        C = p2m(p, y[None], np.array([0.7]), c)
        got = eval_multipole(p, C, x, c)
        r = np.linalg.norm(x - c)
        bound = 0.7 * (a / r) ** (p + 1) / (r - a) / FOUR_PI
        assert abs(got - _coulomb(x, y, 0.7)) <= bound * (1 + 1e-9) + 1e-16


@pytest.mark.parametrize("p", [2, 5, 8, 12])
def test_single_charge_local_within_bound(p):
    rng = np.random.default_rng(10 + p)
    c = rng.random(3)
    for _ in range(8):
        y = c + rng.standard_normal(3)
        a = np.linalg.norm(y - c)
        x = c + rng.standard_normal(3)
        x = c + (x - c) * (0.25 * a / np.linalg.norm(x - c))
        D = p2l(p, y[None], np.array([-1.3]), c)
        got = eval_local(p, D, x, c)
        r = np.linalg.norm(x - c)
        bound = 1.3 * (r / a) ** (p + 1) / (a - r) / FOUR_PI
        assert abs(got - _coulomb(x, y, -1.3)) <= bound * (1 + 1e-9) + 1e-16


def test_multipole_error_decays_with_p():
    rng = np.random.default_rng(3)
    pts = rng.random((40, 3)) - 0.5
    q = rng.uniform(-1, 1, 40)
    x = np.array([2.0, 1.5, -1.0])
    exact = sum(_coulomb(x, y, qq) for y, qq in zip(pts, q))
    errs = [abs(eval_multipole(p, p2m(p, pts, q, np.zeros(3)), x, np.zeros(3)) - exact)
            for p in (2, 4, 6, 8, 10)]
    assert all(b < a for a, b in zip(errs, errs[1:]))


def test_monopole_and_dipole_coefficients():
    rng = np.random.default_rng(4)
    pts = rng.random((30, 3))
    q = rng.uniform(-1, 1, 30)
    c = np.array([0.5, 0.5, 0.5])
    C = p2m(3, pts, q, c)
    d = pts - c
    assert C[B.idx(0, 0)] == pytest.approx(q.sum(), rel=1e-14)
    assert C[B.idx(1, 0)] == pytest.approx((q * d[:, 2]).sum(), rel=1e-13)
    assert C[B.idx(1, 1)] == pytest.approx((q * d[:, 0]).sum() / 2, rel=1e-13)
    assert C[B.idx(1, -1)] == pytest.approx(-(q * d[:, 1]).sum() / 2, rel=1e-13)


@pytest.mark.parametrize("p", [3, 6, 8])
def test_m2l_single_charge_reaches_p2l(p):
    # M2L(P2M of one charge, high input order) -> exact P2L of that charge
    rng = np.random.default_rng(20 + p)
    for _ in range(5):
        rho = rng.standard_normal(3)
        rho *= 0.05 / np.linalg.norm(rho)
        t = rng.standard_normal(3)
        t /= np.linalg.norm(t)
        D = m2l(B.regular(30, *rho), t, 30, p)
        Dex = B.singular(p, *(rho + t))
        assert np.abs(D - Dex).max() <= 1e-13 * np.abs(Dex).max()


def test_m2l_along_z_is_the_printed_diagonal_operator():
    # App. B.3 (M2L): D^m_n = sum_k sgn(m) (-1)^{k+m} (n+k)!/r^{n+k+1} C^m_k
    # for a translation of length r along +z from the multipole centre to the
    # local centre's opposite side, i.e. c_src - c_tgt = (0, 0, r).
    p, r = 7, 2.3
    C = np.random.default_rng(5).standard_normal(B.ncoef(p))
    D = m2l(C, np.array([0.0, 0.0, r]), p)
    for n in range(p + 1):
        for m in range(-n, n + 1):
            sg = 1 if m >= 0 else -1
            want = sum(sg * (-1) ** (k + m) * math.factorial(n + k) / r ** (n + k + 1) * C[B.idx(k, m)]
                       for k in range(abs(m), p + 1))
            assert D[B.idx(n, m)] == pytest.approx(want, rel=1e-12, abs=1e-14 * np.abs(D).max())


def test_printed_m2m_operator_is_exact_recentering():
    # App. B.3 (M2M) with old centre - new centre = (0, 0, r):
    # C^m_n(new) = sum_{k=|m|}^n r^{n-k}/(n-k)! C^m_k(old) equals P2M at the new centre
    p, r = 8, 0.37
    rng = np.random.default_rng(6)
    pts = 0.2 * rng.standard_normal((12, 3))
    q = rng.uniform(-1, 1, 12)
    old = np.zeros(3)
    new = old - np.array([0.0, 0.0, r])
    Co, Cn = p2m(p, pts, q, old), p2m(p, pts, q, new)
    for n in range(p + 1):
        for m in range(-n, n + 1):
            v = sum(r ** (n - k) / math.factorial(n - k) * Co[B.idx(k, m)] for k in range(abs(m), n + 1))
            assert v == pytest.approx(Cn[B.idx(n, m)], rel=1e-12, abs=1e-14)


def test_printed_l2l_operator_is_exact_recentering():
    # App. B.3 (L2L) with old centre - new centre = (0, 0, r):
    # D^m_n(new) = sum_{k=n}^p (-r)^{k-n}/(k-n)! D^m_k(old); evaluating either
    # expansion gives the same degree-p polynomial
    p, r = 8, 0.21
    rng = np.random.default_rng(7)
    far = rng.standard_normal((6, 3)) + np.array([6.0, 0.0, 0.0])
    q = rng.uniform(-1, 1, 6)
    old = np.zeros(3)
    new = old - np.array([0.0, 0.0, r])
    Do = p2l(p, far, q, old)
    Dn = np.zeros_like(Do)
    for n in range(p + 1):
        for m in range(-n, n + 1):
            Dn[B.idx(n, m)] = sum((-r) ** (k - n) / math.factorial(k - n) * Do[B.idx(k, m)]
                                  for k in range(n, p + 1))
    x = new + 0.1 * rng.standard_normal((5, 3))
    assert np.allclose(eval_local(p, Dn, x, new), eval_local(p, Do, x, old), rtol=1e-12, atol=1e-16)
