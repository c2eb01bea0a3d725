"""Derivatives of the energy E = 1/2 sum_i q_i u_i (the inverse-design use of
autodiff, Sec. III.B, differentiating the FMM evaluation pass).

Oracle code (test infrastructure only).

Direct sum (eqs. 1-3): u = G q with G symmetric, so
    dE/dq_i = u_i,        dE/dx_i = q_i grad u(x_i).

FMM with a frozen hierarchy (tree, lists, box centres fixed; only the
points move): u-hat = G-hat q is linear in q and G-hat is not symmetric
(cross-level lists pair a source level with a different target level).
    dE/dq = 1/2 (G-hat + G-hat^T) q
    dE/dx_k = 1/2 q_k (grad u-hat(x_k) + grad v-hat(x_k)),  v-hat = G-hat^T q,
where the first gradient acts on x_k as a target and the second as a
source.  G-hat^T is the same FMM over the transposed lists (every
(source, target) pair reversed, M2L and P2P): the truncated two-centre
kernel is symmetric under swapping source and target offsets with the
translation reversed (the truncation n <= p, k <= p is square), and M2M and
L2L are exact re-centrings.  The dot-product test <g, G-hat q> =
<G-hat^T g, q> against the forward FMM pins this.
"""
from __future__ import annotations

import numpy as np

from .direct import direct
from .fmm import fmm
from .lists import Lists


def transpose_lists(lists: Lists) -> Lists:
    """Every (source, target) pair reversed, sorted by (target, source)."""
    o = np.lexsort((lists.m2l_tgt, lists.m2l_src))
    p = np.lexsort((lists.p2p_tgt, lists.p2p_src))
    return Lists(m2l_src=lists.m2l_tgt[o], m2l_tgt=lists.m2l_src[o],
                 p2p_src=lists.p2p_tgt[p], p2p_tgt=lists.p2p_src[p], steps=lists.steps)


def energy_gradient_direct(pos, q, targets=None):
    """(E-contribution terms) dE/dq and dE/dx of the direct-sum energy at
    ``targets`` (default all): u_i and q_i grad u(x_i)."""
    pos = np.asarray(pos, dtype=np.float64)
    idx = np.arange(len(pos)) if targets is None else np.asarray(targets)
    u, g = direct(pos, q, pos[idx], field=True)
    return u, q[idx, None] * g


def energy_direct(pos, q):
    u, _ = direct(pos, q)
    return 0.5 * float(np.dot(q, u))


def energy_gradient_fmm(pos, q, p, leaf_max, s, theta, tree, lists, targets=None):
    """dE/dq and dE/dx of the frozen-hierarchy FMM energy (see module
    docstring) at ``targets`` (default all)."""
    u, fu = fmm(pos, q, p, leaf_max, s, theta, targets=targets, tree=tree, lists=lists)
    v, fv = fmm(pos, q, p, leaf_max, s, theta, targets=targets, tree=tree,
                lists=transpose_lists(lists))
    idx = np.arange(len(pos)) if targets is None else np.asarray(targets)
    # fields are -grad
    return 0.5 * (u + v), -0.5 * q[idx, None] * (fu + fv)


def energy_fmm(pos, q, p, leaf_max, s, theta, tree, lists):
    u, _ = fmm(pos, q, p, leaf_max, s, theta, tree=tree, lists=lists, field=False)
    return 0.5 * float(np.dot(q, u))
