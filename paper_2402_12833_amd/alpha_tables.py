"""Step-size (alpha) tables of Sec. 3, Example 1, from the device solver.

For each anisotropy kxx of the sweep, MPCG with m = 5 and nu = 6 (damped
Jacobi, omega = 1/2) is run on the 160 x 160-element bilinear FEM problem
(4 levels) with the per-iteration alpha history recorded; alpha_k has one
entry per level correction (coarsest first, the finest smoother's last).
The paper shows these as heatmaps (level x iteration); this prints the same
data binned: the mean |alpha_l| over each fifth of the iterations.

  python -m paper_2402_12833_amd.alpha_tables   (needs the GPU)
"""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def alpha_histories():
    sys.path.insert(0, ROOT)
    import torch
    import paper_2402_12833_amd as amg
    import workloads as W
    n = W.EXAMPLE1_ELEMENTS - 1
    b = torch.as_tensor(W.example1_rhs(), device="cuda")
    out = {}
    for kxx in W.EXAMPLE1_KXX:
        s = amg.Solver(2, n, W.EXAMPLE1_LEVELS, stencil=W.example1_stencil(kxx), omega=0.5, maxit=5000, m=5, nu=6,
                       record_history=1)
        x = torch.zeros_like(b)
        _, info = s.solve(b, x, tol=1e-8)
        assert info["status"] == amg.OK, (kxx, info)
        alpha, res = s.history()
        out[kxx] = (alpha, res, info["iterations"])
        s.close()
    return out


def table(hist, bins: int = 5) -> str:
    lines = []
    for kxx, (alpha, res, its) in hist.items():
        nb = alpha.shape[1]
        edges = np.linspace(0, alpha.shape[0], bins + 1).astype(int)
        lines.append(f"kxx = {kxx:.0e}: {its} iterations; mean |alpha_l| per fifth of the iterations "
                     f"(rows: level 0 = coarsest .. {nb - 1} = finest)")
        lines.append("| level | " + " | ".join(f"its {edges[q] + 1}-{edges[q + 1]}" for q in range(bins)) + " |")
        lines.append("|---" * (bins + 1) + "|")
        for lvl in range(nb):
            cells = [f"{np.mean(np.abs(alpha[edges[q]:edges[q + 1], lvl])):.3g}" if edges[q + 1] > edges[q] else "-"
                     for q in range(bins)]
            lines.append(f"| {lvl} | " + " | ".join(cells) + " |")
        lines.append("")
    return "\n".join(lines)


if __name__ == "__main__":
    print(table(alpha_histories()))
