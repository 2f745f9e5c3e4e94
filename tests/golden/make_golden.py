"""Write the oracle's reference values for the full-size GPU parity tests.

Calls only the CPU oracle (oracle/) and the seeded generators (workloads/).
For each full-size workload it stores the iteration count and residual
history of the FP64 oracle at tol 1e-8, and x_k at k = 1, 5 and the final k
sampled at 1024 fixed indices (seed 12345), plus the 2-norm of each x_k.

    python tests/golden/make_golden.py [poisson3d_127] [diffusion3d_127] [diffusion3d_127:m5]

A name suffix ":mK" runs the truncation window m = K (file oracle_<name>_mK.json).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import hierarchy, mpcg  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def make(spec):
    name, _, msuf = spec.partition(":")
    m = int(msuf[1:]) if msuf else 1
    prob = W.PROBLEMS[name]
    t0 = time.time()
    h = hierarchy.build(prob.dim, prob.n, prob.nlevels, kappa=W.kappa_field(prob))
    b = W.problem_rhs(prob)
    res = mpcg.mpcg(h, b, tol=1e-8, m=m)
    k = res.iterations
    snaps = mpcg.mpcg(h, b, tol=0.0, maxit=k, snapshots=(1, 5, k), m=m)
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(prob.ndof, size=1024, replace=False))
    out = {
        "source": f"oracle/ (FP64 CPU oracle), Algorithm 1 with m={m}, nu=2, omega=2/3; written by tests/golden/make_golden.py",
        "m": m,
        "workload": name,
        "tol": 1e-8,
        "iterations": k,
        "status": res.status,
        "resnorms": res.resnorms,
        "bnorm": res.bnorm,
        "alphas": [a.tolist() for a in res.alphas],
        "sample_idx": idx.tolist(),
        "x": {str(kk): snaps.snapshots[kk][idx].tolist() for kk in (1, 5, k)},
        "xnorm": {str(kk): float(np.linalg.norm(snaps.snapshots[kk])) for kk in (1, 5, k)},
    }
    fname = f"oracle_{name}.json" if m == 1 else f"oracle_{name}_m{m}.json"
    with open(os.path.join(HERE, fname), "w") as f:
        json.dump(out, f)
    print(spec, "iterations", k, "time %.1fs" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or ["poisson3d_127", "diffusion3d_127"]
    for n in names:
        make(n)
