"""Profiling driver and summariser for rocprofv3.

Run under the profiler (the program itself follows ``--``):

    rocprofv3 --kernel-trace --stats --output-format csv -d OUT -o run -- \\
        python3 -m paper_2608_15781_amd.profile_run --precision fp32 --steps 50
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT -o fetch -- python3 -m ... (same args)
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT -o write -- python3 -m ... (same args)

The driver runs the benchmark workload for the given number of steps, then a plain device-to-
device copy of a known size (``--copy-mib``), whose counter readings calibrate the byte counters.
``python3 -m paper_2608_15781_amd.profile_run summarize OUT`` turns the CSV files into the short
text summary kept under ``profiles/``.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def run(args):
    sys.path.insert(0, ROOT)
    import torch

    from paper_2608_15781_amd import core, inputs

    w, solid, theta, rr0, rp0 = inputs.workload_inputs(args.workload, device="cuda:0")
    kw = dict(tau=w["tau"], sigma=w["sigma"], beta=w["beta"], xi=w["xi"], accel=[(w["accel"], 0, 0)] * 2,
              species=w["species"], x_open=w["x_open"], tau_species=w["tau_c"], c_inlet=w["c_in"])
    sim = core.Lbm(w["shape"], solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, precision=args.precision, **kw)
    sim.step(args.warmup, reductions=False)
    sim.step(args.steps)
    torch.cuda.synchronize()
    n = args.copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    # evict the source from the 256 MB last-level cache before the calibration copy
    flush = torch.ones(2 * n, dtype=torch.float32, device="cuda:0")
    del flush
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps(dict(workload=args.workload, precision=args.precision, steps=args.steps,
                          fluid_nodes=int((solid == 0).sum()), copy_bytes=4 * n)), flush=True)


def _rows(pattern):
    out = []
    for path in glob.glob(pattern, recursive=True):
        with open(path) as f:
            out.extend(csv.DictReader(f))
    return out


def summarize(out_dir, kernel="k_collide<1", copy_bytes=None):
    """Average kernel durations and per-dispatch FETCH_SIZE / WRITE_SIZE (KiB), calibrated by the copy."""
    res = {}
    stats = _rows(os.path.join(out_dir, "**", "*kernel_stats.csv"))
    res["kernels"] = {r["Name"]: dict(calls=int(r["Calls"]), avg_us=float(r["AverageNs"]) / 1e3) for r in stats}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        rows = [r for r in _rows(os.path.join(out_dir, "**", "*counter_collection.csv")) if r.get("Counter_Name") == ctr]
        if not rows:
            continue
        per = {}
        for r in rows:
            per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        res[ctr] = {k: sum(v) / len(v) for k, v in per.items()}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", nargs="?", default="run")
    ap.add_argument("out", nargs="?")
    ap.add_argument("--workload", default="bijel128")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--copy-mib", type=int, default=512)
    args = ap.parse_args()
    if args.cmd == "summarize":
        print(json.dumps(summarize(args.out), indent=1))
    else:
        run(args)


if __name__ == "__main__":
    main()
