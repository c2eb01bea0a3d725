"""The active-shielding inverse design of Sec. III.B on the GPU: separate
source and target hierarchies, two charge vectors, the adjoint through
torch.autograd.  The loss gradient with respect to the shield charges is
checked against the gradient the CPU oracle gives (its FMM with the same
trees and lists, transposed, FP64: 1e-10) and against the exact gradient of
the direct-sum loss (FMM accuracy); gradient descent must lower the loss."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def shield():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import shielding
    return shielding.Shield(seed=0, precision="fp64")


def _reference_gradient(q, potentials, transpose, n_in, w):
    """dL/dq from the potentials phi(Q) and the transposed operator, for
    Q = [q, q_ext] and [q, 0] (numpy)."""
    w_in, w_out, w_reg = w
    phi0, phi1 = potentials
    a0 = np.zeros_like(phi0)
    a1 = np.zeros_like(phi1)
    a0[:n_in] = 2 * w_in * (phi0[:n_in] - phi0[:n_in].mean())
    a1[n_in:] = 2 * w_out * phi1[n_in:]
    g0, g1 = transpose(a0), transpose(a1)
    n_sh = len(q)
    return g0[:n_sh] + g1[:n_sh] + 2 * w_reg * q


def test_gradient_matches_oracle_and_direct_sum(shield):
    import shielding
    import workloads
    from oracle.direct import direct
    from oracle.fmm import _evaluate
    from oracle.gradient import transpose_lists
    from oracle.lists import build_lists_st
    from oracle.tree import build_tree
    _say("[shielding] gradient vs oracle and direct sum")
    g = workloads.shielding(0)
    src = np.concatenate([g["shield"], g["ext"]])
    tgt = np.concatenate([g["inner"], g["outer"]])
    n_sh, n_in = len(g["shield"]), len(g["inner"])
    q = np.random.default_rng(5).uniform(-0.5, 0.5, n_sh)
    Q = [np.concatenate([q, g["q_ext"]]), np.concatenate([q, np.zeros(len(g["ext"]))])]
    w = (shielding.W_IN, shielding.W_OUT, shielding.W_REG)
    # oracle: same trees and lists, its own FMM and transposed FMM
    st, tt = build_tree(src, 16, 2), build_tree(tgt, 16, 2)
    li = build_lists_st(st, tt, 0.6)
    lt = transpose_lists(li)
    fwd = lambda x: _evaluate(st, src, x, tt, tgt, li, 8, np.arange(len(tgt)), False)[0]
    adj = lambda y: _evaluate(tt, tgt, y, st, src, lt, 8, np.arange(len(src)), False)[0]
    g_or = _reference_gradient(q, [fwd(Q[0]), fwd(Q[1])], adj, n_in, w)
    # exact: direct sums (the operator is symmetric, so the transpose is the
    # direct sum from the targets back to the sources)
    dfwd = lambda x: direct(src, x, tgt)[0]
    dadj = lambda y: direct(tgt, y, src)[0]
    g_ex = _reference_gradient(q, [dfwd(Q[0]), dfwd(Q[1])], dadj, n_in, w)
    L, gq = shield.gradient(torch.from_numpy(q).cuda())
    gq = gq.cpu().numpy()
    e_or = np.abs(gq - g_or).max() / np.abs(g_or).max()
    e_ex = np.linalg.norm(gq - g_ex) / np.linalg.norm(g_ex)
    _say(f"    vs oracle {e_or:.2e}, vs direct-sum gradient {e_ex:.2e}")
    assert e_or <= 1e-10
    assert e_ex <= 1e-4


def test_gradient_descent_lowers_the_loss(shield):
    _say("[shielding] 20 descent steps from q = 0")
    q0 = torch.zeros(shield.n_sh, dtype=torch.float64, device="cuda")
    L0 = [float(x) for x in shield.loss(q0)]
    q, hist = shield.optimise(20, q0)
    Ls = [L0[0]] + [h["L"] for h in hist]
    _say(f"    L {Ls[0]:.4e} -> {Ls[-1]:.4e}; L_in {L0[1]:.4e} -> {hist[-1]['L_in']:.4e}; "
         f"L_out {hist[-1]['L_out']:.4e}")
    assert all(b <= a * (1 + 1e-12) for a, b in zip(Ls[:-1], Ls[1:]))
    assert Ls[-1] < 0.5 * Ls[0]
    assert hist[-1]["L_in"] < 0.2 * L0[1]
