"""Direct ("nested-sum") multipole-to-local operator, O(p^4) per pair.

Oracle code (test infrastructure only).

The paper avoids this operator and uses rotations instead (Sec. II.D); the
oracle uses it on purpose, so that the oracle and the GPU path reach the
same truncated operator by different methods.  It is written in the complex
basis of Sec. II.C (eqs. 6-12) and converted to and from the real
coefficients of the paper:

  complex regular   R^m_n = r^n P~^{|m|}_n(cos t) e^{i m phi} / (n+|m|)!
  complex singular  S^m_n = (n-|m|)! P~^{|m|}_n(cos t) e^{i m phi} / r^{n+1}
  (P~ is the associated Legendre function without the (-1)^m phase; the
  phases of App. A cancel against alpha^m_n and beta^m_n),
  multipole         M^m_n = sum q conj(R^m_n(rho))       (eq. 10)
  local             L^m_n = sum q conj(S^m_n(y - c))      (eq. 12)
  real <-> complex  M^m = C^m + i C^{-m},   L^m = D^m - i D^{-m}   (m > 0)

Translation of the singular harmonics (|rho| < |t|):
  S^m_n(t + rho) = eps_m sum_{k,l} (-1)^k eps_l eps_{m+l} conj(R^l_k(rho))
                   S^{m+l}_{n+k}(t),     eps_j = 1 (j >= 0), (-1)^j (j < 0),
so that for a multipole about c_a and a local expansion about c_b,
t = c_a - c_b:
  L^m_n = eps_m sum_{k<=p} sum_{|l|<=k} (-1)^k eps_l eps_{m+l}
          M^{-l}_k conj(S^{m+l}_{n+k}(t)).
This is pinned by the single-charge test: M2L applied to the multipole of
one charge reproduces the charge's exact local expansion as the multipole
order grows.
"""
from __future__ import annotations

import numpy as np

from .basis import idx, ncoef, singular


def _eps(j: int) -> int:
    return 1 if j >= 0 else (-1) ** (-j)


def real_to_complex_multipole(C: np.ndarray, p: int) -> np.ndarray:
    """M[..., n, m + p] (complex) from real C[..., (p+1)^2]."""
    M = np.zeros(C.shape[:-1] + (p + 1, 2 * p + 1), dtype=np.complex128)
    for n in range(p + 1):
        M[..., n, p] = C[..., idx(n, 0)]
        for m in range(1, n + 1):
            v = C[..., idx(n, m)] + 1j * C[..., idx(n, -m)]
            M[..., n, p + m] = v
            M[..., n, p - m] = np.conj(v)
    return M


def complex_local_to_real(Lc: np.ndarray, p: int) -> np.ndarray:
    """Real D[..., (p+1)^2] from complex L[..., n, m + p]: D^m = Re L^m,
    D^{-m} = -Im L^m (m > 0)."""
    D = np.zeros(Lc.shape[:-2] + (ncoef(p),))
    for n in range(p + 1):
        D[..., idx(n, 0)] = Lc[..., n, p].real
        for m in range(1, n + 1):
            D[..., idx(n, m)] = Lc[..., n, p + m].real
            D[..., idx(n, -m)] = -Lc[..., n, p + m].imag
    return D


def complex_singular(P: int, t: np.ndarray) -> np.ndarray:
    """S^m_n(t) (complex) for n <= P as array [..., n, m + P]."""
    Sh = singular(P, t[..., 0], t[..., 1], t[..., 2])
    S = np.zeros(t.shape[:-1] + (P + 1, 2 * P + 1), dtype=np.complex128)
    for n in range(P + 1):
        S[..., n, P] = Sh[..., idx(n, 0)]
        for m in range(1, n + 1):
            v = Sh[..., idx(n, m)] + 1j * Sh[..., idx(n, -m)]
            S[..., n, P + m] = v
            S[..., n, P - m] = np.conj(v)
    return S


_PLAN_CACHE: dict = {}


def _m2l_plan(p_in: int, p_out: int):
    """Index arrays of the nested sum, as [row = (n, m >= 0), column = (k, l)]:
    the factor eps_m (-1)^k eps_l eps_{m+l}, the position of M^{-l}_k and the
    position of S^{m+l}_{n+k} in the degree-(p_in+p_out) table."""
    key = (p_in, p_out)
    if key in _PLAN_CACHE:
        return _PLAN_CACHE[key]
    P = p_in + p_out
    cols = [(k, l) for k in range(p_in + 1) for l in range(-k, k + 1)]
    outs = [(n, m) for n in range(p_out + 1) for m in range(0, n + 1)]
    mk = np.array([k for k, l in cols])
    ml = np.array([-l + p_in for k, l in cols])
    sn = np.array([[n + k for k, l in cols] for n, m in outs])
    sm = np.array([[m + l + P for k, l in cols] for n, m in outs])
    coef = np.array([[_eps(m) * (-1) ** k * _eps(l) * _eps(m + l) for k, l in cols]
                     for n, m in outs], dtype=np.float64)
    plan = (outs, mk, ml, sn, sm, coef)
    _PLAN_CACHE[key] = plan
    return plan


def m2l(C: np.ndarray, t: np.ndarray, p_in: int, p_out: int | None = None) -> np.ndarray:
    """Local coefficients D[..., (p_out+1)^2] about c_b of the multipole
    C[..., (p_in+1)^2] about c_a, with t = c_a - c_b (batched over the
    leading axes of C and t)."""
    if p_out is None:
        p_out = p_in
    C = np.asarray(C, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    lead = np.broadcast_shapes(C.shape[:-1], t.shape[:-1])
    M = real_to_complex_multipole(np.broadcast_to(C, lead + C.shape[-1:]), p_in)
    S = np.conj(complex_singular(p_in + p_out, np.broadcast_to(t, lead + (3,))))
    outs, mk, ml, sn, sm, coef = _m2l_plan(p_in, p_out)
    Mv = M[..., mk, ml]                      # lead + (ncols,)
    G = S[..., sn, sm]                       # lead + (nrows, ncols)
    Lrow = np.einsum("...rj,rj,...j->...r", G, coef, Mv)
    Lfull = np.zeros(lead + (p_out + 1, 2 * p_out + 1), dtype=np.complex128)
    for r, (n, m) in enumerate(outs):
        Lfull[..., n, p_out + m] = Lrow[..., r]
    return complex_local_to_real(Lfull, p_out)
