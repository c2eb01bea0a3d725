#!/usr/bin/env python3
"""Active-shielding inverse design (Sec. III.B), on the GPU FMM with
separate source and target hierarchies and its adjoint.

128 shield charges sit regularly on a sphere of radius 2, 256 external
charges of random position and charge on a sphere of radius 5; probes lie
evenly on spheres of radius 1.5 (inside, 1024) and 2.5 (outside, 1024).
The shield charges q minimise
    L = w_in  sum_inner (phi_tot - mean phi_tot)^2
      + w_out sum_outer phi_shield^2
      + w_reg sum q^2,                 w = (1.0, 0.2, 0.1),
where phi_tot is the potential of all charges and phi_shield that of the
shield alone.  Both potentials come from one plan (sources: shield and
external charges; targets: both probe spheres) evaluated for two charge
vectors, [q, q_ext] and [q, 0]; dL/dq comes from the plan's adjoint through
torch.autograd.  L is quadratic in q, so plain gradient descent takes the
exact step along -dL/dq (one extra evaluation gives the curvature).

    python shielding.py [--iters 30] [--precision fp64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

W_IN, W_OUT, W_REG = 1.0, 0.2, 0.1


class Shield:
    def __init__(self, seed=0, p=8, leaf_max=16, splits=2, theta=0.6, precision="fp64"):
        import torch

        import paper_2511_15269_amd as F
        import workloads
        g = workloads.shielding(seed)
        self.torch = torch
        dev = torch.device("cuda:0")
        self.dt = torch.float64 if precision == "fp64" else torch.float32
        self.n_sh, self.n_in = len(g["shield"]), len(g["inner"])
        src = torch.cat([torch.from_numpy(g["shield"]), torch.from_numpy(g["ext"])]).to(dev)
        tgt = torch.cat([torch.from_numpy(g["inner"]), torch.from_numpy(g["outer"])]).to(dev)
        self.q_ext = torch.from_numpy(g["q_ext"]).to(dev, self.dt)
        self.plan = F.Plan(src, p=p, leaf_max=leaf_max, splits=splits, theta=theta,
                           precision=precision, max_rhs=2, targets=tgt)
        self.F = F

    def charges(self, q):
        """The two charge vectors [q, q_ext] and [q, 0] (differentiable in q)."""
        torch = self.torch
        zero = torch.zeros_like(self.q_ext)
        return torch.stack([torch.cat([q, self.q_ext]), torch.cat([q, zero])])

    def loss(self, q):
        """(L, L_in, L_out, L_reg) as tensors, differentiable in q."""
        u = self.F.FMMPotential.apply(self.charges(q), None, self.plan)
        tot_in = u[0, :self.n_in]
        sh_out = u[1, self.n_in:]
        l_in = ((tot_in - tot_in.mean()) ** 2).sum()
        l_out = (sh_out ** 2).sum()
        l_reg = (q ** 2).sum()
        return W_IN * l_in + W_OUT * l_out + W_REG * l_reg, l_in, l_out, l_reg

    def gradient(self, q):
        q = q.detach().clone().requires_grad_(True)
        L = self.loss(q)[0]
        (g,) = self.torch.autograd.grad(L, q)
        return L.detach(), g

    def optimise(self, iters=30, q0=None, log=None):
        """Gradient descent with the exact step of the quadratic loss."""
        torch = self.torch
        q = torch.zeros(self.n_sh, dtype=self.dt, device=self.q_ext.device) if q0 is None else q0
        hist = []
        for it in range(iters):
            L, g = self.gradient(q)
            with torch.no_grad():
                # L(q - a g) = L - a |g|^2 + a^2 c/2 with c = g^T H g,
                # c = 2 (L(q - g) - L + |g|^2)
                gg = float((g * g).sum())
                L1 = float(self.loss(q - g)[0])
                c = 2.0 * (L1 - float(L) + gg)
                a = gg / c if c > 0 else 0.0
                q = q - a * g
            parts = [float(x) for x in self.loss(q)]
            hist.append({"iter": it + 1, "L": parts[0], "L_in": parts[1], "L_out": parts[2],
                         "L_reg": parts[3], "step": a})
            if log:
                log(hist[-1])
        return q, hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=30)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    sh = Shield(seed=args.seed, precision=args.precision)
    q0 = sh.torch.zeros(sh.n_sh, dtype=sh.dt, device="cuda:0")
    L0 = [float(x) for x in sh.loss(q0)]
    print(json.dumps({"iter": 0, "L": L0[0], "L_in": L0[1], "L_out": L0[2], "L_reg": L0[3]}))
    q, hist = sh.optimise(args.iters, q0, log=lambda h: print(json.dumps(h), flush=True))


if __name__ == "__main__":
    main()
