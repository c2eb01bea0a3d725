"""Multipole and local expansions in the real basis (Sec. II.C, eqs. 9-12).

Oracle code (test infrastructure only).

  multipole coefficients  C^m_n = sum_i q_i R-hat^m_n(r_i - c)
  local coefficients      D^m_n = sum_i q_i S-hat^m_n(r_i - c)   (P2L)
  local evaluation        u(x) = -1/(4 pi) sum w_m D^m_n R-hat^m_n(x - c)
  multipole evaluation    u(x) = -1/(4 pi) sum w_m C^m_n S-hat^m_n(x - c)
with w_m = (2 - delta_{0m}) sgn(m), sgn(0) = 1 (Sec. II.C).  Both forms
follow from the real addition theorem
  1/|x - y| = sum_{n,m} w_m R-hat^m_n(y) S-hat^m_n(x),  |y| < |x|.
"""
from __future__ import annotations

import math

import numpy as np

from .basis import regular, regular_grad, singular, weights

FOUR_PI = 4.0 * math.pi


def p2m(p: int, pts: np.ndarray, q: np.ndarray, centre: np.ndarray) -> np.ndarray:
    d = pts - centre
    return (q[:, None] * regular(p, d[:, 0], d[:, 1], d[:, 2])).sum(axis=0)


def p2l(p: int, pts: np.ndarray, q: np.ndarray, centre: np.ndarray) -> np.ndarray:
    d = pts - centre
    return (q[:, None] * singular(p, d[:, 0], d[:, 1], d[:, 2])).sum(axis=0)


def eval_local(p: int, D: np.ndarray, x: np.ndarray, centre: np.ndarray,
               grad: bool = False):
    """u (and grad u) at points x[..., 3] of the local expansion D about
    centre (D and centre broadcast against x's leading axes)."""
    d = x - centre
    w = weights(p)
    if not grad:
        R = regular(p, d[..., 0], d[..., 1], d[..., 2])
        return -(R * (w * D)).sum(axis=-1) / FOUR_PI
    R, G = regular_grad(p, d[..., 0], d[..., 1], d[..., 2])
    wd = w * D
    u = -(R * wd).sum(axis=-1) / FOUR_PI
    g = -(G * wd[..., None]).sum(axis=-2) / FOUR_PI
    return u, g


def eval_multipole(p: int, C: np.ndarray, x: np.ndarray, centre: np.ndarray):
    d = x - centre
    S = singular(p, d[..., 0], d[..., 1], d[..., 2])
    return -(S * (weights(p) * C)).sum(axis=-1) / FOUR_PI
