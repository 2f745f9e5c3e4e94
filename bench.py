#!/usr/bin/env python3
"""Benchmark: time-to-1e-8 relative residual and HBM GB/s of additive-MG MPCG.

One step = one complete solve (setup excluded) of the 3D Poisson problem on
127^3 interior nodes (2,048,383 DoF, 6 levels, 7-point FD, Galerkin coarse
levels, damped Jacobi nu=2 omega=2/3, b ~ U[-1,1] seed 2, x0 = 0) to
||r|| <= 1e-8 ||b|| in FP64, with b and x resident in device memory.
``value`` is the mean time per solve (ms, lower is better).  The same
protocol is applied to the FP32-bulk form, to the heterogeneous-kappa
workload (truncation window m = 1 and m = 5), to the comparison methods of
Sec. 3 (additive MG-PCG, MG(V)-PCG) and to the learned direction; they are
reported under ``variants``.

The roofline entry is for the fine-level kernel with the largest time per
iteration; its average launch duration is measured with HIP events on the
solver's stream inside the iterations of one more solve of the same
workload (amgmpcg_profile_solve: the iterations launched one by one, every
kernel on the data its predecessor just wrote), for the x/P update with
events bound to its dispatch (its own duration), and its algorithmic bytes
come from the per-DoF traffic model below.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--no-cpu] [--no-variants]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "time-to-1e-8 rel. residual & HBM GB/s, 3D Poisson 2.1M DoF, plain vs learned/FP32"


def traffic_model(dim, n, nlevels, bulk, var):
    """Algorithmic HBM bytes per launch of each kernel of one iteration.

    bulk: bytes of the bulk type (8 FP64, 4 FP32).  var: face arrays stored
    for the finest operator (heterogeneous kappa).  x, r, b are FP64.
    Every array a kernel touches is counted once (compulsory traffic).
    """
    L = nlevels - 1
    b = nlevels
    sizes = [n // (2 ** (L - l)) for l in range(nlevels)]
    N = [s ** dim for s in sizes]
    S = 3 ** dim
    Nf = N[L]
    faces = (dim + 1) * bulk * Nf if var else 0
    faces64 = (dim + 1) * 8 * Nf if var else 0
    # coarse level l keeps one constant stencil (no coefficient arrays) when
    # the fine operator has constant coefficients and every finer grid size
    # is odd (the setup checks this exactly)
    cst = [not var and all(sz % 2 == 1 for sz in sizes[l + 1:]) for l in range(nlevels)]
    coefb = [0 if cst[l] else S * bulk * N[l] for l in range(nlevels)]
    diagb = [0 if cst[l] else bulk * N[l] for l in range(nlevels)]
    m = {}
    m["update_r"] = (b * bulk + 16) * Nf
    m["fine_smooth"] = (8 + bulk) * Nf + faces
    if L > 0:
        # restriction: read the finer vector, write g and the first sweep c1 (reads D)
        m["restrict_fine"] = 8 * Nf + 2 * bulk * N[L - 1] + diagb[L - 1]
        m["restrict_coarse"] = sum(bulk * N[l + 1] + 2 * bulk * N[l] + diagb[l] for l in range(L - 1))
        # smoothing: read g, c1 and the coefficients, write the result
        m["coarse_smooth"] = sum(3 * bulk * N[l] + coefb[l] for l in range(L))
        m["prolong_top"] = (L - 1) * bulk * (N[L - 2] + N[L - 1]) if L >= 2 else 0
        m["prolong_all"] = sum((l + 1) * bulk * (N[l] + N[l + 1]) for l in range(L - 1))
        coarse_cols = L * bulk * N[L - 1]
    else:
        coarse_cols = 0
    m["fine_W"] = (b * bulk + bulk) * Nf + coarse_cols
    m["update_xP"] = (2 * b * bulk + 16 + bulk) * Nf + coarse_cols
    m["spmm_gram"] = (2 * b * bulk + 8) * Nf + faces
    m["residual"] = 24 * Nf + faces64
    per_iter = sum(v for k, v in m.items() if k not in ("prolong_top", "residual"))
    return m, per_iter


def unet_gflop(S, padded=True):
    """Work of one U-Net forward on an S^3 grid: with the padded channel
    counts (w1 stored with 16 input channels of which 2 are real, w11 with 16
    outputs of which 1 is used), or the network's own work (padded=False)."""
    from paper_2402_12833_amd import CNN_LAYERS
    level = {"w1": 0, "w2": 0, "w3": 1, "w4": 1, "w5": 2, "w6": 2, "w7": 1, "w8": 1, "w9": 0, "w10": 0, "w11": 0}
    real = {} if padded else {"w1": (2, None), "w11": (None, 1)}
    tot = 0.0
    for name, taps, cin, cout in CNN_LAYERS:
        ci, co = real.get(name, (None, None))
        tot += 2.0 * (S >> level[name]) ** 3 * taps * (ci or cin) * (co or cout)
    return tot / 1e9


def unet_line(fms, S):
    """The U-Net timing fields: work and rate against the BF16 dense peak,
    on the padded and on the real channel counts."""
    gp, gu = unet_gflop(S), unet_gflop(S, padded=False)
    return {"ms": round(fms, 4), "gflop": round(gu, 1), "TFLOPs": round(gu / fms, 1),
            "bf16_peak_frac": round(gu / fms / 2500.0, 4), "gflop_padded": round(gp, 1),
            "bf16_peak_frac_padded": round(gp / fms / 2500.0, 4)}


def kernel_source_hash():
    """Hash of the device sources the counters were taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2402_12833_amd", "csrc")
    for f in ("common.hpp", "grid_kernels.hpp", "small_kernels.hpp", "host_common.hpp", "solver_grid.hpp"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain-copy calibration), or
    None when the summary is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "counters_poisson3d_127.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except OSError:
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("traffic_bytes")


def per_dof(dim, nlevels, bulk, var):
    """Per fine DoF bytes of the fine kernels (the units of the model)."""
    b = nlevels
    faces = (dim + 1) * bulk if var else 0
    return {"update_r": b * bulk + 16, "fine_smooth": 8 + bulk + faces, "spmm_gram": 2 * b * bulk + 8 + faces,
            "update_xP": 2 * b * bulk + 16 + bulk, "fine_W": b * bulk + bulk}


def poisson_csr(n, nlevels):
    """The 3D 7-point Poisson operator on n^3 interior nodes (h = 1/(n+1),
    Dirichlet) and the tensor-product linear interpolations of the grid
    hierarchy (coarse node J on fine node 2J+1), as CSR inputs for the
    general entry point; with R = P^T / 8 this is the structured workload."""
    import scipy.sparse as sp

    def lap1(m):
        h = 1.0 / (m + 1)
        return sp.diags([-np.ones(m - 1), 2.0 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1]) / h ** 2

    def interp1(nc):
        j = np.arange(nc)
        rows = np.concatenate([2 * j + 1, 2 * j, 2 * j + 2])
        vals = np.concatenate([np.ones(nc), np.full(nc, 0.5), np.full(nc, 0.5)])
        return sp.csr_matrix((vals, (rows, np.concatenate([j, j, j]))), shape=(2 * nc + 1, nc))

    L1, I = lap1(n), sp.identity(n)
    A = (sp.kron(sp.kron(I, I), L1) + sp.kron(sp.kron(I, L1), I) + sp.kron(sp.kron(L1, I), I)).tocsr()
    sizes = [n]
    for _ in range(nlevels - 1):
        sizes.append(sizes[-1] // 2)
    sizes = sizes[::-1]
    Ps = []
    for l in range(nlevels - 1):
        P1 = interp1(sizes[l])
        Ps.append(sp.kron(sp.kron(P1, P1), P1).tocsr())
    return A, Ps


def run_solver(amg, torch, prob, precision, steps, warmup, kappa=None, net=None, m=1, method=0):
    import workloads as W
    b = torch.as_tensor(W.problem_rhs(prob), device="cuda")
    t0 = time.time()
    s = amg.Solver(prob.dim, prob.n, prob.nlevels, kappa=kappa, precision=precision, m=m, method=method)
    setup_s = time.time() - t0
    if net is not None:
        s.attach(net)
    x = torch.zeros_like(b)
    for _ in range(warmup):
        x.zero_()
        s.solve(b, x, tol=1e-8)
    torch.cuda.synchronize()
    infos = []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    tot = 0.0
    for _ in range(steps):
        x.zero_()
        torch.cuda.synchronize()
        ev0.record()
        _, info = s.solve(b, x, tol=1e-8)
        ev1.record()
        torch.cuda.synchronize()
        tot += ev0.elapsed_time(ev1)
        infos.append(info)
    ms = tot / steps
    it = infos[-1]["iterations"]
    assert all(i["status"] == amg.OK for i in infos), infos[-1]
    return s, b, x, ms, it, setup_s, infos[-1]


def run_batched(amg, torch, precision, steps, warmup, persistent=0):
    """The batched workload: 512 2D Poisson problems (sides U{31..255}), all
    solved by one graph of batched launches per k_poll iterations (or, with
    persistent=1, by one persistent launch: a workgroup per problem)."""
    import workloads as W
    table = W.batched_instances()
    bcat = torch.as_tensor(np.concatenate([W.batched_rhs(t) for t in table]), device="cuda")
    bsolv = amg.BatchedSolver([(2, t.n, t.nlevels) for t in table], precision=precision, persistent=persistent)
    xb = torch.zeros_like(bcat)
    for _ in range(warmup):
        xb.zero_()
        bsolv.solve(bcat, xb, tol=1e-8)
    tms = []
    binfos = []
    for _ in range(steps):
        xb.zero_()
        torch.cuda.synchronize()
        _, binfos, bms = bsolv.solve(bcat, xb, tol=1e-8)
        tms.append(bms)
    its = [i["iterations"] for i in binfos]
    assert all(i["status"] == amg.OK for i in binfos)
    # algorithmic bytes of the whole batch: per problem its iterations of the
    # per-iteration model (2D, its own side and levels) plus the initial and
    # refresh residuals
    bulk = 4 if precision == 1 else 8
    nbytes = 0
    for t, inf in zip(table, binfos):
        m, per_iter = traffic_model(2, t.n, t.nlevels, bulk, False)
        nbytes += inf["iterations"] * per_iter + (1 + inf.get("refreshes", 0)) * m["residual"]
    ms = float(np.mean(tms))
    gbs = nbytes / (ms * 1e-3) / 1e9
    out = {"ms": round(ms, 4), "problems": len(table), "dofs": int(bsolv.N),
           "iterations_min": int(min(its)), "iterations_max": int(max(its)),
           "iterations_mean": round(float(np.mean(its)), 2), "bytes_model": int(nbytes),
           "hbm_GBps_algorithmic": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
    offs = bsolv.offsets
    xs = (xb.clone(), [xb[offs[i]:offs[i + 1]].clone() for i in range(len(table))])
    bsolv.close()
    return out, xs


def run_example1(amg, torch):
    """Sec. 3, Example 1 (bilinear FEM, anisotropic diffusion, 160 x 160
    elements, 4 levels): iterations to 1e-8 for kxx = 1e-7 .. 1 of additive-MG
    MPCG (m = 5, nu = 6), additive MG-PCG (nu = 6) and MG(V)-PCG (3 + 3
    sweeps), damped Jacobi omega = 1/2, FP64; device ms of one solve each."""
    import workloads as W
    n = W.EXAMPLE1_ELEMENTS - 1
    b = torch.as_tensor(W.example1_rhs(), device="cuda")
    methods = (("mpcg_m5", dict(m=5, nu=6)), ("additive_pcg", dict(method=amg.ADDITIVE_PCG, nu=6)),
               ("vcycle_pcg", dict(method=amg.VCYCLE_PCG, nu_pre=3, nu_post=3)))
    out = {"elements": W.EXAMPLE1_ELEMENTS, "levels": W.EXAMPLE1_LEVELS, "omega": 0.5, "kxx": W.EXAMPLE1_KXX}
    for tag, opts in methods:
        its, ms = [], []
        for kxx in W.EXAMPLE1_KXX:
            s = amg.Solver(2, n, W.EXAMPLE1_LEVELS, stencil=W.example1_stencil(kxx), omega=0.5, maxit=5000, **opts)
            x = torch.zeros_like(b)
            _, info = s.solve(b, x, tol=1e-8)
            assert info["status"] == amg.OK, (tag, kxx, info)
            its.append(info["iterations"])
            ms.append(round(info["solve_ms"], 3))
            s.close()
        out[f"{tag}_iterations"] = its
        out[f"{tag}_ms"] = ms
    return out


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo, as lscpu reports it)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def host_threads():
    """Host CPUs this process may run on (its affinity set)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(prob, threads, max_iters=None):
    """The FP64 oracle (numpy/scipy, as it stands) on the same workload with
    at most `threads` library threads: (ms, iterations, cores it used =
    process CPU time / wall time of the solve, oracle x).  Setup excluded."""
    from threadpoolctl import threadpool_limits
    import workloads as W
    from oracle import hierarchy, mpcg
    with threadpool_limits(limits=threads):
        h = hierarchy.build(prob.dim, prob.n, prob.nlevels, kappa=W.kappa_field(prob))
        b = W.problem_rhs(prob)
        t0, c0 = time.perf_counter(), time.process_time()
        res = mpcg.mpcg(h, b, tol=1e-8, maxit=max_iters or 1000)
        dt, dc = time.perf_counter() - t0, time.process_time() - c0
    return dt * 1e3, res.iterations, dc / dt, res.x


def rel_err(x, ref):
    """Full-vector relative error ||x - ref|| / ||ref|| (device tensors or arrays)."""
    import torch
    x = torch.as_tensor(x, dtype=torch.float64)
    ref = torch.as_tensor(ref, dtype=torch.float64, device=x.device)
    return float(torch.linalg.norm(x - ref) / torch.linalg.norm(ref))


def x1_fields(x32, info32, x64, it64):
    """The mixed-precision result against the FP64 one: full-vector relative
    error, FP64 iteration count, true FP64 residual of the FP32-bulk x."""
    return {"err_vs_fp64": float(f"{rel_err(x32, x64):.3e}"), "iterations_fp64": it64,
            "relres_true": float(f"{info32['relres_true']:.3e}")}


def calibration_kernel(torch):
    """One plain elementwise kernel reading and writing 512 MiB each, the
    known-size reference for the HBM byte counters."""
    a = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    c = a * 2.0
    torch.cuda.synchronize()
    del a, c


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--unet-only", action="store_true",
                    help="time only the U-Net inference on the 128^3 grid (committed weights) and print its line")
    ap.add_argument("--batched-only", action="store_true",
                    help="time only the 512-problem batched workload (FP32 bulk) and print its line")
    ap.add_argument("--large-only", action="store_true",
                    help="time only the 255^3 Poisson solve (FP64, 16.6 M DoF) and print its line")
    ap.add_argument("--csr-only", action="store_true",
                    help="time only the 127^3 Poisson solve through the CSR entry point (FP64) and print its line")
    ap.add_argument("--calibrate", action="store_true",
                    help="end with one plain 512 MiB read + 512 MiB write elementwise kernel (counter calibration)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); multi-GPU runs are not "
              f"part of this build", file=sys.stderr)
        return 2
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    import paper_2402_12833_amd as amg
    import workloads as W
    amg.load()
    if args.unet_only:
        from paper_2402_12833_amd import train as T
        dprob = W.DIFFUSION3D_127
        sol = amg.Solver(dprob.dim, dprob.n, dprob.nlevels, kappa=W.kappa_field(dprob))
        net = amg.Network(dprob.n)
        T.load_weights(net)
        b = torch.as_tensor(W.problem_rhs(dprob), device="cuda")
        fms = net.time_forward(b, sol.log_kappa(), reps=max(args.steps, 1))
        print(json.dumps({"workload": "unet_forward_128", **unet_line(fms, (dprob.n + 3) // 4 * 4)}), flush=True)
        net.close()
        sol.close()
        return 0
    if args.large_only:
        bprob = W.POISSON3D_255
        sb, _, _, msb, itb, _, _ = run_solver(amg, torch, bprob, 0, max(args.steps, 1), args.warmup)
        _, pib = traffic_model(3, bprob.n, bprob.nlevels, 8, False)
        print(json.dumps({"workload": "poisson3d_255", "dtype": "f64", "ms": round(msb, 4), "iterations": itb,
                          "hbm_GBps_algorithmic": round(pib * itb / (msb * 1e-3) / 1e9, 1)}), flush=True)
        sb.close()
        if args.calibrate:
            calibration_kernel(torch)
        return 0
    if args.csr_only:
        cprob = W.POISSON3D_127
        Ac, Psc = poisson_csr(cprob.n, cprob.nlevels)
        bc = torch.as_tensor(W.problem_rhs(cprob), device="cuda")
        sc = amg.Solver.from_csr(Ac, Psc, 0.125)
        xc = torch.zeros_like(bc)
        for _ in range(args.warmup):
            xc.zero_()
            sc.solve(bc, xc, tol=1e-8)
        tms = []
        for _ in range(max(args.steps, 1)):
            xc.zero_()
            torch.cuda.synchronize()
            _, ci = sc.solve(bc, xc, tol=1e-8)
            assert ci["status"] == amg.OK, ci
            tms.append(ci["solve_ms"])
        print(json.dumps({"workload": "poisson3d_127_csr", "dtype": "f64", "ms": round(float(np.mean(tms)), 4),
                          "iterations": ci["iterations"], "nnz": int(Ac.nnz)}), flush=True)
        sc.close()
        return 0
    if args.batched_only:
        res, _ = run_batched(amg, torch, 1, args.steps, args.warmup)
        print(json.dumps({"workload": "batched2d_512", "dtype": "f32 bulk / f64 Gram", **res}), flush=True)
        return 0

    prob = W.POISSON3D_127
    s, b, x, ms, iters, setup_s, info = run_solver(amg, torch, prob, 0, args.steps, args.warmup)
    x64 = x.clone()
    m, per_iter = traffic_model(prob.dim, prob.n, prob.nlevels, 8, False)
    gbs = per_iter * iters / (ms * 1e-3) / 1e9
    # kernel durations inside real iterations (each kernel on the data the
    # previous one just wrote), HIP events on the solver's stream
    x.zero_()
    _, pinfo, sec, samples = s.profile_solve(b, x, tol=1e-8)
    assert pinfo["status"] == amg.OK and pinfo["iterations"] == iters, pinfo
    # with nu = 2 the smoothers run inside the restriction launches (the fine
    # one beside the first restriction, both reading r once)
    m["restrict"] = (m.get("restrict_fine", 0) + m.get("restrict_coarse", 0) + m["fine_smooth"]
                     + m.get("coarse_smooth", 0) - 8 * prob.ndof)
    m["prolong"] = m.get("prolong_all", 0)
    fine = {k: sec[k] for k in ("update_r", "fine_smooth", "fine_W", "update_xP", "spmm_gram")}
    dom = max(fine, key=lambda k: fine[k])
    dom_bytes = m[dom]
    # the x/P update also carries events bound to its dispatch (its own
    # duration, without the launch latency the span between stream events adds)
    own = sec.get(dom + "_kernel", 0.0)
    dom_ms = own if own > 0 else sec[dom]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    m[dom + "_kernel"] = dom_bytes
    # every section of the iteration with its algorithmic bytes, rate and
    # fraction of the 8 TB/s peak (spans between stream events: launch
    # latency included, so these understate the kernels' own rates)
    kernels = {k: {"ms": round(v, 5), "bytes": m.get(k),
                   "GB/s": round(m[k] / (v * 1e-3) / 1e9, 1) if m.get(k) and v > 0 else None,
                   "frac": round(m[k] / (v * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if m.get(k) and v > 0 else None}
               for k, v in sec.items() if v > 0}
    out = {
        "metric": METRIC,
        "value": round(ms, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "poisson3d_127", "dofs": prob.ndof, "levels": prob.nlevels, "stencil": "7-point FD",
                   "coarse": "Galerkin 27-point", "smoother": "damped Jacobi nu=2 omega=2/3", "m": 1,
                   "tol": 1e-8, "rhs": "U[-1,1] seed 2", "x0": 0},
        "iterations": iters,
        "relres_true": float(f"{info['relres_true']:.3e}"),
        "ms_per_iteration": round(ms / max(iters, 1), 5),
        "hbm_GBps_algorithmic": round(gbs, 1),
        "bytes_per_iteration_model": per_iter,
        "setup_s": round(setup_s, 3),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom),
                     "bytes_per_launch": dom_bytes, "bytes_per_dof": per_dof(3, prob.nlevels, 8, False)[dom],
                     "avg_launch_ms": round(dom_ms, 5), "avg_span_ms": round(sec[dom], 5),
                     "launches_averaged": samples,
                     "timing": ("HIP events bound to the kernel's dispatch (hipExtLaunchKernel start/stop) "
                                "inside the iterations of a solve of this workload; avg_span_ms: span between "
                                "stream events around the launch") if own > 0 else
                               "HIP events around the kernel inside the iterations of a solve of this workload"},
        "kernels_in_solve": kernels,
    }
    s.close()
    if not args.no_variants:
        var = {}
        s2, _, x2, ms2, it2, _, info2 = run_solver(amg, torch, prob, 1, args.steps, args.warmup)
        _, pi2 = traffic_model(3, prob.n, prob.nlevels, 4, False)
        var["poisson3d_127_fp32bulk"] = {"ms": round(ms2, 4), "iterations": it2, "refreshes": info2["refreshes"],
                                        "hbm_GBps_algorithmic": round(pi2 * it2 / (ms2 * 1e-3) / 1e9, 1),
                                        "speedup_vs_fp64": round(ms / ms2, 3), **x1_fields(x2, info2, x64, iters)}
        x32_headline = x2.clone()
        s2.close()
        # the same problem at 255^3: 16.6 M DoF, 7 levels, a working set far
        # beyond the 256 MB Infinity Cache
        bprob = W.POISSON3D_255
        for prec, tag, bulk in ((0, "fp64", 8), (1, "fp32bulk", 4)):
            sb, _, xb_, msb, itb, setb, infb = run_solver(amg, torch, bprob, prec, max(2, args.steps // 2), 1)
            _, pib = traffic_model(3, bprob.n, bprob.nlevels, bulk, False)
            var[f"poisson3d_255_{tag}"] = {"ms": round(msb, 4), "iterations": itb, "refreshes": infb["refreshes"],
                                           "dofs": bprob.ndof, "levels": bprob.nlevels,
                                           "hbm_GBps_algorithmic": round(pib * itb / (msb * 1e-3) / 1e9, 1),
                                           "setup_s": round(setb, 3)}
            if prec == 0:
                x255, it255 = xb_.clone(), itb
            else:
                var[f"poisson3d_255_{tag}"].update(x1_fields(xb_, infb, x255, it255))
                del x255
            sb.close()
        dprob = W.DIFFUSION3D_127
        kap = W.kappa_field(dprob)
        dref = {}
        for prec, tag, bulk in ((0, "fp64", 8), (1, "fp32bulk", 4)):
            s3, _, x3, ms3, it3, _, info3 = run_solver(amg, torch, dprob, prec, args.steps, args.warmup, kappa=kap)
            _, pi3 = traffic_model(3, dprob.n, dprob.nlevels, bulk, True)
            var[f"diffusion3d_127_{tag}"] = {"ms": round(ms3, 4), "iterations": it3, "refreshes": info3["refreshes"],
                                             "hbm_GBps_algorithmic": round(pi3 * it3 / (ms3 * 1e-3) / 1e9, 1)}
            if prec == 0:
                dref["m1"] = (x3.clone(), it3)
            else:
                var[f"diffusion3d_127_{tag}"].update(x1_fields(x3, info3, *dref["m1"]))
            s3.close()
            # truncation window m = 5: each new direction block A-orthogonalised
            # against the last four blocks as well
            s5, _, x5, ms5, it5, _, info5 = run_solver(amg, torch, dprob, prec, args.steps, args.warmup, kappa=kap,
                                                       m=5)
            plain = var[f"diffusion3d_127_{tag}"]
            var[f"diffusion3d_127_m5_{tag}"] = {"ms": round(ms5, 4), "iterations": it5, "refreshes": info5["refreshes"],
                                                "iterations_m1": plain["iterations"],
                                                "time_vs_m1": round(ms5 / plain["ms"], 3)}
            if prec == 0:
                dref["m5"] = (x5.clone(), it5)
            else:
                var[f"diffusion3d_127_m5_{tag}"].update(x1_fields(x5, info5, *dref["m5"]))
            s5.close()
        # the comparison methods of Sec. 3 on the same hierarchy and kernels:
        # CG preconditioned by the summed additive correction and by one
        # V-cycle (1 + 1 damped-Jacobi sweeps, the additive nu = 2 per level)
        for pname, pr, kp in (("poisson3d_127", prob, None), ("diffusion3d_127", dprob, kap)):
            ref = var.get(f"{pname}_fp64") if pname == "diffusion3d_127" else {"ms": round(ms, 4), "iterations": iters}
            for meth, tag in ((amg.ADDITIVE_PCG, "additive_pcg"), (amg.VCYCLE_PCG, "vcycle_pcg")):
                s6, _, _, ms6, it6, _, _ = run_solver(amg, torch, pr, 0, args.steps, args.warmup, kappa=kp,
                                                      method=meth)
                var[f"{pname}_{tag}_fp64"] = {"ms": round(ms6, 4), "iterations": it6,
                                              "mpcg_iterations": ref["iterations"], "mpcg_ms": ref["ms"]}
                s6.close()
        bx = {}
        for prec, tag in ((1, "fp32bulk"), (0, "fp64")):
            var[f"batched2d_512_{tag}"], bx[prec] = run_batched(amg, torch, prec, args.steps, args.warmup)
        var["batched2d_512_fp32bulk"]["err_vs_fp64"] = float(f"{rel_err(bx[1][0], bx[0][0]):.3e}")
        var["batched2d_512_fp32bulk"]["err_vs_fp64_max_problem"] = float(f"{max(rel_err(a, c) for a, c in zip(bx[1][1], bx[0][1])):.3e}")
        var["batched2d_512_fp32bulk"]["iterations_fp64_mean"] = var["batched2d_512_fp64"]["iterations_mean"]
        # the same batch in one persistent launch (the other launch form)
        var["batched2d_512_fp32bulk_persistent"], bpx = run_batched(amg, torch, 1, args.steps, args.warmup,
                                                                    persistent=1)
        var["batched2d_512_fp32bulk_persistent"]["err_vs_fp64"] = float(f"{rel_err(bpx[0], bx[0][0]):.3e}")
        var["batched2d_512_fp32bulk_persistent"]["iterations_fp64_mean"] = var["batched2d_512_fp64"]["iterations_mean"]
        del bx, bpx
        var["example1_160"] = run_example1(amg, torch)
        # the general (CSR) entry point on an unstructured graph problem
        A, Ps, bg = W.graph_problem()
        bt = torch.as_tensor(bg, device="cuda")
        for prec, tag in ((0, "fp64"), (1, "fp32bulk")):
            sc = amg.Solver.from_csr(A, Ps, 1.0, precision=prec, maxit=5000)
            xc = torch.zeros_like(bt)
            sc.solve(bt, xc, tol=1e-8)
            tms = []
            for _ in range(args.steps):
                xc.zero_()
                torch.cuda.synchronize()
                _, ci = sc.solve(bt, xc, tol=1e-8)
                tms.append(ci["solve_ms"])
            assert ci["status"] == amg.OK, ci
            var[f"graph2d_20000_csr_{tag}"] = {"ms": round(float(np.mean(tms)), 4), "iterations": ci["iterations"],
                                               "unknowns": int(A.shape[0]), "nnz": int(A.nnz), "levels": len(Ps) + 1}
            if prec == 0:
                gref = (xc.clone(), ci["iterations"])
            else:
                var[f"graph2d_20000_csr_{tag}"].update(x1_fields(xc, ci, *gref))
            sc.close()
        # the 127^3 Poisson workload through the general entry point: the
        # fine operator as a 14.2 M-nonzero CSR matrix (the cost of generality)
        Ac, Psc = poisson_csr(prob.n, prob.nlevels)
        bc = torch.as_tensor(W.problem_rhs(prob), device="cuda")
        for prec, tag in ((0, "fp64"), (1, "fp32bulk")):
            t0 = time.time()
            sc = amg.Solver.from_csr(Ac, Psc, 0.125, precision=prec)
            set_c = time.time() - t0
            xc = torch.zeros_like(bc)
            sc.solve(bc, xc, tol=1e-8)
            tms = []
            for _ in range(max(2, args.steps // 2)):
                xc.zero_()
                torch.cuda.synchronize()
                _, ci = sc.solve(bc, xc, tol=1e-8)
                tms.append(ci["solve_ms"])
            assert ci["status"] == amg.OK, ci
            ref = ms if prec == 0 else var["poisson3d_127_fp32bulk"]["ms"]
            var[f"poisson3d_127_csr_{tag}"] = {"ms": round(float(np.mean(tms)), 4), "iterations": ci["iterations"],
                                               "nnz": int(Ac.nnz), "setup_s": round(set_c, 3),
                                               "time_vs_structured": round(float(np.mean(tms)) / ref, 3)}
            if prec == 1:
                var[f"poisson3d_127_csr_{tag}"].update(x1_fields(xc, ci, x64, iters))
            sc.close()
        # the learned direction (committed trained weights) on the same problem
        from paper_2402_12833_amd import train as T
        net = amg.Network(dprob.n)
        T.load_weights(net)
        for prec, tag in ((0, "fp64"), (1, "fp32bulk")):
            s4, b4, x4, ms4, it4, _, info4 = run_solver(amg, torch, dprob, prec, args.steps, args.warmup, kappa=kap,
                                                        net=net)
            plain = var[f"diffusion3d_127_{tag}"]
            var[f"diffusion3d_127_learned_{tag}"] = {
                "ms": round(ms4, 4), "iterations": it4, "refreshes": info4["refreshes"], "nb": info4["nb"],
                "iterations_plain": plain["iterations"], "time_vs_plain": round(ms4 / plain["ms"], 3)}
            if prec == 0:
                lref = (x4.clone(), it4)
            else:
                var[f"diffusion3d_127_learned_{tag}"].update(x1_fields(x4, info4, *lref))
            if prec == 0:
                lk = s4.log_kappa()
                fms = net.time_forward(b4, lk, reps=20)
                var["unet_forward_128"] = unet_line(fms, (dprob.n + 3) // 4 * 4)
            s4.close()
        net.close()
        out["variants"] = var
    if not args.no_cpu:
        nthr = host_threads()
        cpu_ms, cpu_it, used, xo = cpu_baseline(prob, nthr)
        cpu1_ms, _, used1, _ = cpu_baseline(prob, 1)
        out["cpu_baseline"] = {"value": round(cpu_ms, 1), "unit": "ms", "cores": max(1, round(used)), "kind": "oracle",
                               "sample": f"FP64 oracle (numpy/scipy as it stands) full solve of poisson3d_127 to 1e-8, "
                                         f"{cpu_it} iterations, setup excluded, library threads limited to the "
                                         f"{nthr} host CPUs; cores = process CPU time / wall time of the solve",
                               "threads_allowed": nthr, "cores_measured": round(used, 2),
                               "value_1thread": round(cpu1_ms, 1), "cores_measured_1thread": round(used1, 2),
                               "cpu": cpu_model()}
        # the benchmarked solution against the oracle's, full vector
        out["err_vs_fp64_oracle"] = float(f"{rel_err(x64, xo):.3e}")
        if "variants" in out:
            out["variants"]["poisson3d_127_fp32bulk"]["err_vs_fp64_oracle"] = float(f"{rel_err(x32_headline, xo):.3e}")
    if args.calibrate:
        calibration_kernel(torch)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
