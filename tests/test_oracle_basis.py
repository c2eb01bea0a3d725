"""Pins of the oracle's solid harmonics (App. A) against the definitions,
printed values, and exact identities."""
import math

import numpy as np
import pytest

from oracle import basis as B


def _pts(n=64, seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((3, n)) * scale


@pytest.mark.parametrize("p", [0, 1, 2, 5, 12])
def test_recursions_match_definitions(p):
    x, y, z = _pts()
    R1, R2 = B.regular_closed(p, x, y, z), B.regular(p, x, y, z)
    S1, S2 = B.singular_closed(p, x, y, z), B.singular(p, x, y, z)
    for a, b in ((R1, R2), (S1, S2)):
        scale = np.abs(a).max(axis=0) + 1e-300
        assert np.all(np.abs(a - b) <= 1e-12 * scale)


def test_printed_seed_values():
    # App. A.1/A.2 seeds and low-order check values
    x, y, z = 0.3, -0.7, 1.1
    r = math.sqrt(x * x + y * y + z * z)
    R = B.regular(3, x, y, z)
    S = B.singular(3, x, y, z)
    exp_R = {(0, 0): 1.0, (1, 1): x / 2, (1, -1): -y / 2, (1, 0): z,
             (2, 2): (x * x - y * y) / 8, (2, -2): -x * y / 4}
    exp_S = {(0, 0): 1 / r, (1, 1): x / r ** 3, (1, -1): y / r ** 3, (1, 0): z / r ** 3,
             (2, 2): 3 * (x * x - y * y) / r ** 5}
    for (n, m), v in exp_R.items():
        assert R[B.idx(n, m)] == pytest.approx(v, rel=1e-14, abs=1e-15)
    for (n, m), v in exp_S.items():
        assert S[B.idx(n, m)] == pytest.approx(v, rel=1e-14)


def test_regular_is_harmonic():
    p = 8
    x, y, z = _pts(16, 1)
    h = 1e-3
    lap = -6 * B.regular(p, x, y, z)
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        lap = lap + B.regular(p, x + e[0], y + e[1], z + e[2]) + B.regular(p, x - e[0], y - e[1], z - e[2])
    lap /= h * h
    mag = np.abs(B.regular(p, x, y, z)).max() / h ** 0 + 1.0
    assert np.abs(lap).max() < 1e-4 * mag


def test_singular_is_harmonic():
    p = 6
    x, y, z = _pts(16, 2) + 3.0
    h = 1e-3
    lap = -6 * B.singular(p, x, y, z)
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        lap = lap + B.singular(p, x + e[0], y + e[1], z + e[2]) + B.singular(p, x - e[0], y - e[1], z - e[2])
    lap /= h * h
    assert np.abs(lap).max() < 1e-5 * np.abs(B.singular(p, x, y, z)).max()


def test_gradient_euler_identity():
    # R-hat^m_n is homogeneous of degree n: r . grad R = n R (exact identity)
    p = 10
    x, y, z = _pts(32, 3)
    R, G = B.regular_grad(p, x, y, z)
    rdotg = G[..., 0] * x[:, None] + G[..., 1] * y[:, None] + G[..., 2] * z[:, None]
    n = np.array([n for n in range(p + 1) for m in range(-n, n + 1)])
    assert np.allclose(rdotg, n * R, rtol=1e-12, atol=1e-14 * np.abs(R).max())


def test_gradient_dz_identity():
    # d/dz R-hat^m_n = R-hat^m_{n-1} (zero when |m| = n)
    p = 9
    x, y, z = _pts(32, 4)
    R, G = B.regular_grad(p, x, y, z)
    for n in range(p + 1):
        for m in range(-n, n + 1):
            want = R[:, B.idx(n - 1, m)] if abs(m) <= n - 1 else 0.0
            assert np.allclose(G[:, B.idx(n, m), 2], want, rtol=1e-12, atol=1e-15)


def test_gradient_matches_finite_differences():
    p = 8
    x, y, z = _pts(16, 5)
    R, G = B.regular_grad(p, x, y, z)
    h = 1e-6
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd = (B.regular(p, x + e[0], y + e[1], z + e[2]) - B.regular(p, x - e[0], y - e[1], z - e[2])) / (2 * h)
        assert np.allclose(G[..., d], fd, rtol=1e-6, atol=1e-8)


def test_sectoral_gradient_sign_reading():
    # grad R-hat^2_2 = (x/4, -y/4, 0): the printed leading minus is dropped
    R, G = B.regular_grad(2, 0.5, 0.25, -0.3)
    assert np.allclose(G[B.idx(2, 2)], [0.5 / 4, -0.25 / 4, 0.0], rtol=1e-15)


@pytest.mark.parametrize("p", [4, 10, 30])
def test_real_addition_theorem(p):
    # 1/|x-y| = sum w_m R-hat(y) S-hat(x), truncation error <= (|y|/|x|)^{p+1}/(|x|-|y|)
    rng = np.random.default_rng(6)
    w = B.weights(p)
    for _ in range(10):
        X = rng.standard_normal(3)
        X *= 2.0 / np.linalg.norm(X)
        Y = rng.standard_normal(3)
        Y *= 0.5 / np.linalg.norm(Y)
        val = (w * B.regular(p, *Y) * B.singular(p, *X)).sum()
        exact = 1.0 / np.linalg.norm(X - Y)
        bound = (0.25) ** (p + 1) / 1.5
        assert abs(val - exact) <= bound + 1e-15
