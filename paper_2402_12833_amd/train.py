"""Training and evaluation driver of the learned search direction.

Training pairs (r_k, e_k = x* - x_k) come from plain MPCG solves (the
library's own iterates, ``Solver.make_pairs``) on fresh heterogeneous
diffusion instances kappa = exp(2 g), g a unit-variance Gaussian field with
correlation length 1/16 (training kappa seeds 10000 + j).  Every step of
the forward and backward pass and the Adam update runs in the library's HIP
kernels; this module only schedules them.

Data flow: a CPU thread synthesises the kappa fields and right-hand sides
ahead of the GPU; per field the main thread sets up the hierarchy, solves to
a tight tolerance for x*, replays the iteration to emit the pairs into a
device buffer holding the most recent fields, and takes Adam steps on pairs
drawn at random from that buffer.

    python -m paper_2402_12833_amd.train --fields 200 --out weights.f32
"""
from __future__ import annotations

import argparse
import math
import os
import queue
import sys
import threading
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
import workloads as W  # noqa: E402

DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                               "unet_diffusion3d_127.f32")


def save_weights(net: B.Network, path: str) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    net.get_weights().astype("<f4").tofile(path)


def load_weights(net: B.Network, path: str = DEFAULT_WEIGHTS) -> None:
    w = np.fromfile(path, dtype="<f4")
    if w.size != B.cnn_weight_count():
        raise ValueError(f"{path}: {w.size} weights, expected {B.cnn_weight_count()}")
    net.set_weights(w)


def _fields(seeds: List[int], n: int, nlevels: int, workers: int, out: "queue.Queue"):
    for sd in seeds:
        prob = W.diffusion_instance(sd, n, nlevels)
        kap = W.kappa_field(prob, workers=workers)
        out.put((sd, kap, W.problem_rhs(prob)))
    out.put(None)


def pair_iterations(iters: int, count: int) -> List[int]:
    """count iteration indices spread over 0 .. iters - 1 (unique, sorted)."""
    if iters <= 1:
        return [0]
    ks = np.unique(np.round(np.linspace(0, iters - 1, count)).astype(int))
    return [int(k) for k in ks]


def train(n: int = 127, nlevels: int = 6, fields: int = 200, pairs_per_field: int = 24,
          steps_per_field: int = 24, buffer_fields: int = 8, lr: float = 1e-3, lr_min: float = 5e-5,
          warmup: int = 100, seed: int = 0, tol_star: float = 1e-12, workers: int = 8,
          net: Optional[B.Network] = None, log: Callable[[str], None] = print,
          seed0: int = W.TRAIN_KAPPA_SEED0, loss: str = "marginal") -> Dict:
    """Train a network on `fields` fresh instances; returns a summary dict.

    loss "energy": 1 - (d.r)^2 / ((d.A d)(e.r)), the A-norm error fraction
    left by the best step along d = N(r); "marginal": the same on top of the
    level-correction block of r (the error left by the energy-minimising
    step over [MG(r), d] relative to the step over MG(r) alone); both need
    the field's operator, so the buffer keeps each field's handle; "mse":
    mean squared error against e / rms(e).  Learning rate: linear warm-up over `warmup` steps to `lr`,
    then cosine decay to `lr_min` over the remaining steps.
    """
    import torch
    B.load()
    net = net or B.Network(n, seed=seed)
    rng = np.random.default_rng(seed)
    total_steps = fields * steps_per_field
    q: "queue.Queue" = queue.Queue(maxsize=4)
    th = threading.Thread(target=_fields, args=([seed0 + j for j in range(fields)], n, nlevels, workers, q),
                          daemon=True)
    th.start()
    buf: List = []
    losses: List[float] = []
    step = 0
    t0 = time.time()
    npairs = 0
    fi = 0
    while True:
        item = q.get()
        if item is None:
            break
        sd, kap, b_h = item
        s = B.Solver(3, n, nlevels, kappa=kap)
        b = torch.as_tensor(b_h, device="cuda")
        xs, info = s.solve(b, tol=tol_star)
        ks = pair_iterations(info["iterations"], pairs_per_field)
        R, E = s.make_pairs(b, xs, ks)
        lk = s.log_kappa()
        del xs, b
        if loss == "mse":
            s.close()
            s = None
        buf.append((R, E, lk, s))
        npairs += len(ks)
        if len(buf) > buffer_fields:
            old = buf.pop(0)
            if old[3] is not None:
                old[3].close()
        fl = []
        for _ in range(steps_per_field):
            if step < warmup:
                cur = lr * (step + 1) / warmup
            else:
                p = (step - warmup) / max(1, total_steps - warmup)
                cur = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * min(p, 1.0)))
            f = int(rng.integers(len(buf)))
            Rf, Ef, lkf, sf = buf[f]
            k = int(rng.integers(Rf.shape[0]))
            if loss in ("energy", "marginal"):
                fl.append(net.energy_step(sf, Rf[k], Ef[k], cur, lkf, marginal=loss == "marginal"))
            else:
                fl.append(net.train_step(Rf[k], Ef[k], cur, lkf))
            step += 1
        losses.extend(fl)
        fi += 1
        log(f"field {fi}/{fields} seed {sd}: {info['iterations']} its to {tol_star:g}, {len(ks)} pairs, "
            f"mean loss {np.mean(fl):.4f}, step {step}, {time.time() - t0:.0f}s")
    th.join()
    for item in buf:
        if item[3] is not None:
            item[3].close()
    return {"net": net, "steps": step, "pairs": npairs, "fields": fi, "losses": losses,
            "seconds": time.time() - t0}


def evaluate(net: Optional[B.Network], seeds: List[int], n: int = 127, nlevels: int = 6, tol: float = 1e-8,
             precision: int = 0, repeats: int = 1, workers: int = 8,
             log: Callable[[str], None] = print) -> List[Dict]:
    """Plain vs learned solves on the given kappa seeds (same b, x0 = 0)."""
    import torch
    B.load()
    out = []
    for sd in seeds:
        prob = W.diffusion_instance(sd, n, nlevels)
        kap = W.kappa_field(prob, workers=workers)
        b = torch.as_tensor(W.problem_rhs(prob), device="cuda")
        s = B.Solver(3, n, nlevels, kappa=kap, precision=precision)
        row = {"seed": sd}
        for tag, attach in (("plain", None), ("learned", net)):
            if tag == "learned" and net is None:
                continue
            s.attach(attach)
            ms, info = [], None
            for _ in range(repeats + 1):
                x = torch.zeros_like(b)
                torch.cuda.synchronize()
                _, info = s.solve(b, x, tol=tol)
                ms.append(info["solve_ms"])
            rtrue = s.residual(b, x)
            row[tag] = {"iterations": info["iterations"], "status": info["status"],
                        "ms": float(np.mean(ms[1:])),
                        "true_relres": float(torch.linalg.norm(rtrue) / torch.linalg.norm(b))}
        s.attach(None)
        s.close()
        log(f"seed {sd}: " + ", ".join(f"{k} {v['iterations']} its {v['ms']:.2f} ms"
                                       for k, v in row.items() if k != "seed"))
        out.append(row)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=127)
    ap.add_argument("--levels", type=int, default=6)
    ap.add_argument("--fields", type=int, default=200)
    ap.add_argument("--pairs-per-field", type=int, default=24)
    ap.add_argument("--steps-per-field", type=int, default=24)
    ap.add_argument("--buffer-fields", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--loss", choices=("marginal", "energy", "mse"), default="marginal")
    ap.add_argument("--eval", type=int, default=5, help="held-out instances to evaluate after training")
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    res = train(n=args.n, nlevels=args.levels, fields=args.fields, pairs_per_field=args.pairs_per_field,
                steps_per_field=args.steps_per_field, buffer_fields=args.buffer_fields, lr=args.lr,
                seed=args.seed, log=log, loss=args.loss)
    save_weights(res["net"], args.out)
    log(f"trained {res['steps']} steps on {res['pairs']} pairs from {res['fields']} fields in "
        f"{res['seconds']:.0f}s; weights -> {args.out}")
    if args.eval > 0:
        rows = evaluate(res["net"], [W.TEST_KAPPA_SEED0 + i for i in range(args.eval)], n=args.n,
                        nlevels=args.levels, log=log)
        ip = np.mean([r["plain"]["iterations"] for r in rows])
        il = np.mean([r["learned"]["iterations"] for r in rows])
        log(f"held-out mean iterations: plain {ip:.1f}, learned {il:.1f}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
