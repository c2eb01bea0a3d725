"""Direct O(N^2) sum of the Laplace point-charge potential (eqs. 1-3).

Oracle code (test infrastructure only).

  u(x_i)      = -1/(4 pi) sum_{j : r_ij > 0} q_j / r_ij
  grad u(x_i) =  1/(4 pi) sum_{j : r_ij > 0} q_j (x_i - x_j) / r_ij^3
  field       = -grad u
Reading: pairs at distance 0 (a point with itself, or coincident points)
contribute nothing; the paper's kernel (eq. 2) is singular there.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

FOUR_PI = 4.0 * math.pi


def _block(src, q, tgt, field):
    d = tgt[:, None, :] - src[None, :, :]
    r2 = (d * d).sum(axis=-1)
    ok = r2 > 0.0
    inv = np.zeros_like(r2)
    inv[ok] = 1.0 / np.sqrt(r2[ok])
    u = -(inv @ q) / FOUR_PI
    if not field:
        return u, None
    inv3 = inv * inv * inv
    g = np.einsum("ij,ijk->ik", inv3 * q[None, :], d) / FOUR_PI
    return u, g


def direct(src: np.ndarray, q: np.ndarray, tgt: np.ndarray | None = None,
           field: bool = False, threads: int | None = None, block: int = 8):
    """Potential (and grad u) at ``tgt`` (default: the sources) from charges
    ``q`` at ``src``.  Returns (u[T], grad_u[T,3] or None)."""
    src = np.asarray(src, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    tgt = src if tgt is None else np.asarray(tgt, dtype=np.float64)
    T = len(tgt)
    u = np.empty(T)
    g = np.empty((T, 3)) if field else None
    # keep temporaries near 64 MB whatever the source count
    block = max(1, min(block, (1 << 23) // max(1, len(src))))
    starts = list(range(0, T, block))
    if threads is None:
        threads = min(16, len(os.sched_getaffinity(0)))

    def work(s0):
        uu, gg = _block(src, q, tgt[s0:s0 + block], field)
        u[s0:s0 + block] = uu
        if field:
            g[s0:s0 + block] = gg

    if threads <= 1 or len(starts) == 1:
        for s0 in starts:
            work(s0)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(work, starts))
    return u, g


def direct_fsum(src, q, tgt=None):
    """Correctly rounded sums (math.fsum) of the potential, for tiny N."""
    src = np.asarray(src, dtype=np.float64)
    tgt = src if tgt is None else np.asarray(tgt, dtype=np.float64)
    out = np.empty(len(tgt))
    for i, x in enumerate(tgt):
        terms = []
        for j, y in enumerate(src):
            r = math.sqrt(math.fsum((a - b) ** 2 for a, b in zip(x, y)))
            if r > 0.0:
                terms.append(q[j] / r)
        out[i] = -math.fsum(terms) / FOUR_PI
    return out
