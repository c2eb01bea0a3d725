"""Real solid harmonics of the Laplace kernel (Sec. II.C; App. A).

Oracle code (test infrastructure only).

Coefficient vectors are indexed by (n, m), 0 <= n <= p, -n <= m <= n, at
position ``idx(n, m) = n*n + n + m`` of a vector of length (p+1)^2.

Two independent evaluations are provided:

* closed forms built from the definitions in App. A (associated Legendre
  functions obtained by differentiating the Legendre polynomial, as in the
  definition of P^m_n there), and
* the App. A recursions (regular basis A.1, singular basis A.2, gradient of
  the regular basis A.3).

Each pins the other in the tests.  The FMM oracle uses the recursions
(faster); the closed forms are the definition.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre as npleg


def idx(n: int, m: int) -> int:
    return n * n + n + m


def ncoef(p: int) -> int:
    return (p + 1) * (p + 1)


def _assoc_legendre(n: int, m: int, x: np.ndarray) -> np.ndarray:
    """P^m_n(x) = (-1)^m (1-x^2)^{m/2} d^m/dx^m P_n(x), m >= 0 (App. A.1,
    definition including the (-1)^m phase)."""
    c = np.zeros(n + 1)
    c[n] = 1.0
    dm = npleg.legder(c, m) if m > 0 else c
    val = npleg.legval(x, dm)
    return (-1.0) ** m * (1.0 - x * x) ** (m / 2.0) * val


def _spherical(x, y, z):
    r = np.sqrt(x * x + y * y + z * z)
    safe = np.where(r > 0, r, 1.0)
    ct = np.where(r > 0, z / safe, 1.0)
    phi = np.arctan2(y, x)
    return r, ct, phi


def regular_closed(p: int, x, y, z) -> np.ndarray:
    """R-hat^m_n from the definition (App. A.1):
    R^m_n = alpha^m_n r^n P^{|m|}_n(cos theta) e^{i m phi},
    alpha^m_n = (-1)^m / (n+|m|)!, and R-hat = Re R (m >= 0), Im R (m < 0).
    Returns an array of shape x.shape + ((p+1)^2,)."""
    x, y, z = (np.asarray(a, dtype=np.float64) for a in (x, y, z))
    r, ct, phi = _spherical(x, y, z)
    out = np.empty(x.shape + (ncoef(p),))
    for n in range(p + 1):
        rn = r ** n
        for m in range(-n, n + 1):
            a = (-1.0) ** m / math.factorial(n + abs(m))
            R = a * rn * _assoc_legendre(n, abs(m), ct) * np.exp(1j * m * phi)
            out[..., idx(n, m)] = R.real if m >= 0 else R.imag
    return out


def singular_closed(p: int, x, y, z) -> np.ndarray:
    """S-hat^m_n from the definition (App. A.2):
    S^m_n = beta^m_n r^{-(n+1)} P^{|m|}_n(cos theta) e^{i m phi},
    beta^m_n = (-1)^m (n-|m|)!, and S-hat = Re S^m_n (m >= 0),
    Im S^{|m|}_n (m < 0).  Undefined at r = 0."""
    x, y, z = (np.asarray(a, dtype=np.float64) for a in (x, y, z))
    r, ct, phi = _spherical(x, y, z)
    out = np.empty(x.shape + (ncoef(p),))
    for n in range(p + 1):
        rn1 = r ** -(n + 1)
        for m in range(-n, n + 1):
            am = abs(m)
            b = (-1.0) ** am * math.factorial(n - am)
            S = b * rn1 * _assoc_legendre(n, am, ct) * np.exp(1j * am * phi)
            out[..., idx(n, m)] = S.real if m >= 0 else S.imag
    return out


def regular(p: int, x, y, z) -> np.ndarray:
    """R-hat^m_n by the App. A.1 recursions."""
    x, y, z = (np.asarray(a, dtype=np.float64) for a in (x, y, z))
    r2 = x * x + y * y + z * z
    R = np.zeros(x.shape + (ncoef(p),))
    R[..., idx(0, 0)] = 1.0
    if p >= 1:
        R[..., idx(1, 1)] = x / 2.0
        R[..., idx(1, -1)] = -y / 2.0
    for n in range(2, p + 1):  # sectoral
        a, b = R[..., idx(n - 1, n - 1)], R[..., idx(n - 1, 1 - n)]
        R[..., idx(n, n)] = (x * a + y * b) / (2 * n)
        R[..., idx(n, -n)] = (x * b - y * a) / (2 * n)
    for n in range(0, p):  # one above sectoral
        R[..., idx(n + 1, n)] = z * R[..., idx(n, n)]
        R[..., idx(n + 1, -n)] = z * R[..., idx(n, -n)]
    for n in range(2, p + 1):
        for m in range(2 - n, n - 1):
            R[..., idx(n, m)] = ((2 * n - 1) * z * R[..., idx(n - 1, m)]
                                 - r2 * R[..., idx(n - 2, m)]) / ((n - abs(m)) * (n + abs(m)))
    return R


def singular(p: int, x, y, z) -> np.ndarray:
    """S-hat^m_n by the App. A.2 recursions."""
    x, y, z = (np.asarray(a, dtype=np.float64) for a in (x, y, z))
    r2 = x * x + y * y + z * z
    S = np.zeros(x.shape + (ncoef(p),))
    S[..., idx(0, 0)] = 1.0 / np.sqrt(r2)
    if p >= 1:
        r3 = r2 * np.sqrt(r2)
        S[..., idx(1, 1)] = x / r3
        S[..., idx(1, -1)] = y / r3
    for n in range(2, p + 1):
        a, b = S[..., idx(n - 1, n - 1)], S[..., idx(n - 1, 1 - n)]
        S[..., idx(n, n)] = (2 * n - 1) * (x * a - y * b) / r2
        S[..., idx(n, -n)] = (2 * n - 1) * (x * b + y * a) / r2
    for n in range(0, p):
        S[..., idx(n + 1, n)] = (2 * n + 1) * z * S[..., idx(n, n)] / r2
        S[..., idx(n + 1, -n)] = (2 * n + 1) * z * S[..., idx(n, -n)] / r2
    for n in range(2, p + 1):
        for m in range(2 - n, n - 1):
            S[..., idx(n, m)] = ((2 * n - 1) * z * S[..., idx(n - 1, m)]
                                 - (n - 1 - m) * (n - 1 + m) * S[..., idx(n - 2, m)]) / r2
    return S


def regular_grad(p: int, x, y, z):
    """(R-hat, grad R-hat) by the App. A.1 and A.3 recursions.

    Reading: the sectoral gradient formula for grad R-hat^n_n is printed with
    a leading minus sign; the product rule applied to the sectoral recursion
    of A.1 gives it without that sign (e.g. R-hat^2_2 = (x^2-y^2)/8 has
    gradient (x/4, -y/4, 0)), so the sign is dropped.
    Returns (R[..., K], G[..., K, 3])."""
    x, y, z = (np.asarray(a, dtype=np.float64) for a in (x, y, z))
    R = regular(p, x, y, z)
    r2 = x * x + y * y + z * z
    G = np.zeros(x.shape + (ncoef(p), 3))
    ex = np.array([1.0, 0.0, 0.0])
    ey = np.array([0.0, 1.0, 0.0])
    ez = np.array([0.0, 0.0, 1.0])
    xv = x[..., None]
    yv = y[..., None]
    zv = z[..., None]
    rv = np.stack([x, y, z], axis=-1)
    if p >= 1:
        G[..., idx(1, 1), :] = 0.5 * ex
        G[..., idx(1, -1), :] = -0.5 * ey
    for n in range(2, p + 1):
        ga, gb = G[..., idx(n - 1, n - 1), :], G[..., idx(n - 1, 1 - n), :]
        a, b = R[..., idx(n - 1, n - 1), None], R[..., idx(n - 1, 1 - n), None]
        G[..., idx(n, n), :] = (xv * ga + yv * gb + a * ex + b * ey) / (2 * n)
        G[..., idx(n, -n), :] = (xv * gb - yv * ga + b * ex - a * ey) / (2 * n)
    for n in range(0, p):
        for m in (n, -n):
            G[..., idx(n + 1, m), :] = zv * G[..., idx(n, m), :] + R[..., idx(n, m), None] * ez
    for n in range(2, p + 1):
        for m in range(2 - n, n - 1):
            G[..., idx(n, m), :] = ((2 * n - 1) * (zv * G[..., idx(n - 1, m), :]
                                                   + R[..., idx(n - 1, m), None] * ez)
                                    - r2[..., None] * G[..., idx(n - 2, m), :]
                                    - 2.0 * R[..., idx(n - 2, m), None] * rv) / (n * n - m * m)
    return R, G


def weights(p: int) -> np.ndarray:
    """(2 - delta_{0m}) sgn(m), sgn(0) = 1: the weights with which local
    (and multipole) coefficients meet the real basis (Sec. II.C)."""
    w = np.empty(ncoef(p))
    for n in range(p + 1):
        for m in range(-n, n + 1):
            w[idx(n, m)] = 1.0 if m == 0 else (2.0 if m > 0 else -2.0)
    return w
