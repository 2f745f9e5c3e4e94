"""Text summaries of rocprofv3 output for the benchmarked workloads.

Reads the CSV files of `rocprofv3 --kernel-trace --output-format csv` and of
`rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs and prints a markdown
table per kernel (calls, average duration, algorithmic bytes and rate for the
fine-level kernels of the structured solver, HBM bytes from the counters).

  python -m paper_2402_12833_amd.profile_summary trace WORKLOAD KERNEL_TRACE_CSV \
      [--fetch FETCH_CSV --write WRITE_CSV --json OUT.json]

WORKLOAD: poisson3d_127 or poisson3d_255 (structured FP64 solve: byte model
and counters), or any other name (plain per-kernel table).  The counter runs
must end with the plain 512 MiB read + 512 MiB write calibration kernel
(`bench.py --calibrate`), whose counter values give the scale factors.
"""
from __future__ import annotations

import argparse
import collections
import csv
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# fine-level kernels of one iteration and their entries in the byte model
FINE = {"update_xP": "update_xP", "spmm_gram_z": "spmm_gram", "spmm_gram": "spmm_gram", "fine_W": "fine_W",
        "update_r": "update_r", "restrict_fine_smooth": "restrict_fine_smooth",
        "restrict_fine_smooth_tile": "restrict_fine_smooth"}
GRID = {"poisson3d_127": (3, 127, 6), "poisson3d_255": (3, 255, 7)}
CAL_BYTES = 512 * 1024 * 1024   # the calibration kernel reads and writes this many bytes


def short_name(name: str) -> str:
    s = name.split("(")[0].replace("void ", "").strip()
    s = s.split("amg::")[-1]
    return s


def base_name(short: str) -> str:
    s = short.split("<")[0]
    return s[2:] if s.startswith("k_") else s


def load_trace(path):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        d[short_name(r["Kernel_Name"])].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0)
    return d


def load_counter(path, counter):
    """Per kernel, the counter value of every dispatch, in dispatch order."""
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    d = collections.defaultdict(list)
    for r in rows:
        d[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return d


def calibration(d, expect_kib):
    """Scale factor of a counter: known bytes / the value the last large
    elementwise kernel of the run reads."""
    cands = [v[-1] for k, v in d.items() if "elementwise" in k and v and v[-1] > 0.25 * expect_kib]
    if not cands:
        raise SystemExit("no calibration kernel in the counter run (run bench.py with --calibrate)")
    return expect_kib / cands[-1], cands[-1]


def byte_model(workload):
    sys.path.insert(0, ROOT)
    import bench
    dim, n, nl = GRID[workload]
    m, _ = bench.traffic_model(dim, n, nl, 8, False)
    m["restrict_fine_smooth"] = m["restrict_fine"] + m["fine_smooth"] - 8 * n ** dim
    return m, bench.kernel_source_hash()


def full(v, frac):
    med = statistics.median(v)
    return [x for x in v if x >= frac * med]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["trace"])
    ap.add_argument("workload")
    ap.add_argument("trace_csv")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--json")
    args = ap.parse_args(argv)
    tr = load_trace(args.trace_csv)
    total = sum(sum(v) for v in tr.values())
    out = []
    if args.workload not in GRID:
        out.append("| kernel | calls | avg us | total ms | share |")
        out.append("|---|---|---|---|---|")
        for k, v in sorted(tr.items(), key=lambda kv: -sum(kv[1])):
            out.append(f"| `{k}` | {len(v)} | {sum(v) / len(v):.2f} | {sum(v) / 1e3:.3f} | "
                       f"{100 * sum(v) / total:.1f} % |")
        print("\n".join(out))
        return 0
    m, src_hash = byte_model(args.workload)
    cnt = None
    if args.fetch and args.write:
        fd, wd = load_counter(args.fetch, "FETCH_SIZE"), load_counter(args.write, "WRITE_SIZE")
        ff, fcal = calibration(fd, CAL_BYTES / 1024)
        wf, wcal = calibration(wd, CAL_BYTES / 1024)
        cnt = (fd, wd, ff, wf, fcal, wcal)
    rec = {"workload": f"{args.workload} FP64", "source_hash": src_hash, "kernels": {}}
    hdr = "| kernel | calls (full of all) | avg us (full) | algorithmic MB | GB/s | frac of 8 TB/s"
    hdr += " | FETCH KiB | WRITE KiB | scaled traffic MB | traffic / algorithmic |" if cnt else " |"
    out.append(hdr)
    out.append("|---" * (hdr.count("|") - 1) + "|")
    for k, v in sorted(tr.items(), key=lambda kv: -sum(kv[1])):
        b = base_name(k)
        key = FINE.get(b)
        # fine kernels: full launches only (a solve's first and last x/P
        # update and the SpMM/Gram launches after the stop flag do part of
        # the work or none); the others: every launch
        fv = full(v, 0.75) if key else v
        avg = sum(fv) / len(fv)
        row = f"| `{k}` | {len(fv)} of {len(v)} | {avg:.2f}"
        if key is None:
            out.append(row + " |" + " |" * (hdr.count("|") - 4))
            continue
        alg = m[key]
        gbs = alg / (avg * 1e-6) / 1e9
        row += f" | {alg / 1e6:.1f} | {gbs:.0f} | {gbs / 8000:.3f}"
        krec = {"launches": len(fv), "avg_us": round(avg, 3), "algorithmic_bytes": int(alg)}
        if cnt:
            fd, wd, ff, wf, _, _ = cnt
            fk = full(fd.get(k, [0.0]), 0.9)
            wk = full(wd.get(k, [0.0]), 0.9)
            fkib, wkib = sum(fk) / len(fk), sum(wk) / len(wk)
            traffic = (fkib * ff + wkib * wf) * 1024
            row += f" | {fkib:.0f} | {wkib:.0f} | {traffic / 1e6:.1f} | {traffic / alg:.2f}"
            krec.update({"dispatches": len(fk), "fetch_kib": round(fkib, 1), "write_kib": round(wkib, 1),
                         "traffic_bytes": int(traffic)})
        out.append(row + " |")
        rec["kernels"][key] = krec
    print("\n".join(out))
    if cnt:
        _, _, ff, wf, fcal, wcal = cnt
        print(f"\nCalibration (plain elementwise kernel, 512 MiB read + 512 MiB written): FETCH_SIZE {fcal:.0f} KiB "
              f"(factor {ff:.3f}), WRITE_SIZE {wcal:.0f} KiB (factor {wf:.3f}).  Source hash of the kernel sources: "
              f"{src_hash}.")
        rec["calibration"] = {"kernel": "torch elementwise a*2.0 over 64Mi doubles (512 MiB read + 512 MiB written)",
                              "fetch_kib": fcal, "write_kib": wcal, "fetch_factor": round(ff, 4),
                              "write_factor": round(wf, 4)}
    if args.json:
        with open(args.json, "w") as f:
            json.dump(rec, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
