"""Profiling program and summariser for rocprofv3.

Run under the profiler (the program itself follows ``--``):

    rocprofv3 --kernel-trace --stats --output-format csv -d OUT -o run -- \\
        python3 -m paper_2608_15781_amd.profile_run --precision fp32 --steps 50
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT -o fetch -- python3 -m ... (same args)
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT -o write -- python3 -m ... (same args)

The program runs the benchmark workload for the given number of steps, then a plain device-to-
device copy of a known size (``--copy-mib``), whose counter readings calibrate the byte counters.
``python3 -m paper_2608_15781_amd.profile_run report --precision P --fluid-nodes F TRACE FETCH WRITE``
turns the three CSV folders into the short markdown summary kept under ``profiles/``;
``profile_run bench-trace TRACE BENCH_JSON`` summarises a kernel trace of bench.py itself.
``profile_run counters PASS_A PASS_B`` summarises two hardware-counter runs (the counter sets of
COUNTER_PASSES, one run each) into what bounds each step kernel.
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


def run_adjoint(args):
    """Forward with checkpoints and the checkpointed backward of the 96^3 adjoint workload."""
    sys.path.insert(0, ROOT)
    import torch

    from paper_2608_15781_amd import autograd as ag
    from paper_2608_15781_amd import core, inputs

    w, solid, theta, rr0, rp0 = inputs.workload_inputs("adjoint96", device="cuda:0")
    kw = dict(tau=w["tau"], sigma=w["sigma"], beta=w["beta"], xi=w["xi"], accel=[(w["accel"], 0, 0)] * 2,
              species=w["species"], x_open=w["x_open"], tau_species=w["tau_c"], c_inlet=w["c_in"])
    sim = core.Lbm(w["shape"], solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, precision=args.precision, **kw)
    steps = args.steps
    L, cps, final = ag.forward_states(sim, steps, w["checkpoint"])
    gth, gxi, _ = ag.adjoint_gradients(sim, steps, w["checkpoint"], cps, final)
    res = dict(workload="adjoint96", precision=args.precision, steps=steps, fluid_nodes=int((solid == 0).sum()),
               L=L, dxi=float(gxi))
    torch.cuda.synchronize()
    _calibration_copy(args, torch)  # the last dispatch of the run
    print(json.dumps(res), flush=True)


def _calibration_copy(args, torch):
    """A plain device copy of known size, with its source evicted from the last-level cache."""
    n = args.copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    flush = torch.ones(2 * n, dtype=torch.float32, device="cuda:0")
    del flush
    dst.copy_(src)
    torch.cuda.synchronize()


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
    _calibration_copy(args, torch)
    print(json.dumps(dict(workload=args.workload, precision=args.precision, steps=args.steps,
                          fluid_nodes=int((solid == 0).sum()), copy_bytes=args.copy_mib << 20)), flush=True)


def _rows(pattern):
    out = []
    for path in sorted(glob.glob(pattern, recursive=True)):
        with open(path) as f:
            out.extend(csv.DictReader(f))
    return out


def _short(name):
    """Kernel name without the return type and argument list."""
    name = name.strip()
    if name.startswith("void "):
        name = name[5:]
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def summarize(out_dir, copy_bytes):
    """Average kernel durations, and per-dispatch FETCH_SIZE / WRITE_SIZE calibrated by the copy.

    The calibration copy is the last dispatch of the run; its counters read (in KiB) what the
    hardware reports for copy_bytes bytes read and written, and every kernel's counters are scaled
    by copy_bytes / (1024 * that reading).
    """
    res = {"kernels": {}, "counters": {}}
    for r in _rows(os.path.join(out_dir, "**", "*kernel_stats.csv")):
        res["kernels"][_short(r["Name"])] = dict(calls=int(r["Calls"]), avg_us=float(r["AverageNs"]) / 1e3,
                                                 min_us=float(r["MinNs"]) / 1e3, max_us=float(r["MaxNs"]) / 1e3)
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        rows = [r for r in _rows(os.path.join(out_dir, "**", "*counter_collection.csv"))
                if r.get("Counter_Name") == ctr]
        if not rows:
            continue
        by_dispatch = {}
        for r in rows:
            key = int(r["Dispatch_Id"])
            name, val = by_dispatch.get(key, (_short(r["Kernel_Name"]), 0.0))
            by_dispatch[key] = (name, val + float(r["Counter_Value"]))
        last = max(by_dispatch)
        copy_kib = by_dispatch[last][1]
        scale = copy_bytes / (1024.0 * copy_kib)
        per = {}
        for key, (name, val) in by_dispatch.items():
            if key != last:
                per.setdefault(name, []).append(val)
        res["counters"][ctr] = dict(copy_kernel=by_dispatch[last][0], copy_kib=copy_kib, scale=scale,
                                    kib_per_dispatch={k: sum(v) / len(v) for k, v in per.items()})
    return res


def report(args):
    """Markdown summary of one kernel-trace run and the FETCH_SIZE / WRITE_SIZE runs of a precision."""
    sys.path.insert(0, ROOT)
    from paper_2608_15781_amd import build

    copy_bytes = args.copy_mib * (1 << 20)
    kt = summarize(args.trace, copy_bytes)["kernels"]
    fe = summarize(args.fetch, copy_bytes)["counters"]["FETCH_SIZE"]
    wr = summarize(args.write, copy_bytes)["counters"]["WRITE_SIZE"]
    fluid = args.fluid_nodes
    adj = args.mode == "adjoint"
    drv = "python3 -m paper_2608_15781_amd.profile_run %s--precision %s --steps " % (
        "adjoint " if adj else "--workload %s " % args.workload, args.precision)
    steps = (200, 40) if adj else (50, 20)
    title = ("Adjoint kernels, adjoint96 (forward with checkpoints every 20 steps, then the checkpointed backward)"
             if adj else "Step kernels, %s" % args.workload)
    lines = ["# %s, %s storage" % (title, args.precision), "",
             "Commands (repository root, `cd /tmp && export TMPDIR=/tmp` first, `PYTHONPATH` = repository root):", "",
             "```",
             "rocprofv3 --kernel-trace --stats --output-format csv -d OUT/prof -o run -- %s%d" % (drv, steps[0]),
             "rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/fetch -o run -- %s%d" % (drv, steps[1]),
             "rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/write -o run -- %s%d" % (drv, steps[1]),
             "python3 -m paper_2608_15781_amd.profile_run report %s--precision %s --fluid-nodes %d "
             "OUT/prof OUT/fetch OUT/write" % ("--mode adjoint " if adj else "--workload %s " % args.workload,
                                               args.precision, fluid),
             "```", "",
             "Counter calibration: the run ends with a %d MiB device copy (source evicted from the last-level "
             "cache first); it reads FETCH_SIZE = %.0f KiB and WRITE_SIZE = %.0f KiB for %.0f KiB moved each way, "
             "so FETCH_SIZE is scaled by %.4f and WRITE_SIZE by %.4f." % (
                 args.copy_mib, fe["copy_kib"], wr["copy_kib"], copy_bytes / 1024, fe["scale"], wr["scale"]), "",
             "| kernel | calls | avg us | min us | FETCH KiB/dispatch | WRITE KiB/dispatch | HBM MB/launch "
             "(calibrated) | B/fluid node | GB/s |",
             "|---|---|---|---|---|---|---|---|---|"]
    traffic = {}
    for name, k in sorted(kt.items(), key=lambda kv: -kv[1]["avg_us"] * kv[1]["calls"]):
        if not name.startswith("lbm::"):
            continue
        f = fe["kib_per_dispatch"].get(name)
        w = wr["kib_per_dispatch"].get(name)
        if f is None or w is None:
            continue
        b = 1024 * (f * fe["scale"] + w * wr["scale"])
        traffic[name] = b
        lines.append("| `%s` | %d | %.2f | %.2f | %.1f | %.1f | %.2f | %.1f | %.0f |" % (
            name, k["calls"], k["avg_us"], k["min_us"], f, w, b / 1e6, b / fluid, b / (k["avg_us"] * 1e3)))
    if adj:
        nsteps = kt["lbm::k_adj_collide<%d>" % {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3}[args.precision]]["calls"]
        tot = sum(k["avg_us"] * k["calls"] for n, k in kt.items() if n.startswith("lbm::"))
        lines += ["", "Fluid nodes: %d. Library kernel time per adjoint step (all launches of the run, forward "
                  "recomputation included, divided by the %d adjoint steps): %.1f us." % (fluid, nsteps, tot / nsteps),
                  ""]
    else:
        step_us = sum(k["avg_us"] for n, k in kt.items() if n.startswith("lbm::"))
        step_b = sum(traffic.values())
        lines += ["", "Fluid nodes: %d. Sum over the step kernels: %.2f us, %.1f MB, %.1f B per fluid node." % (
            fluid, step_us, step_b / 1e6, step_b / fluid), ""]
    lines += [
        "Machine-readable (read by bench.py; valid only while the HIP sources hash to the digest):", "",
        "- source_digest: %s" % build.source_digest()]
    for name, b in traffic.items():
        lines.append("- traffic_bytes_per_launch %s: %.0f" % (name, b))
    print("\n".join(lines))


BENCH_ARGS = "--steps 20 --warmup 5 --no-cpu --no-adjoint --no-side"
STEP_KERNELS = ("lbm::k_colour<%d>", "lbm::k_extrap<%d>", "lbm::k_normal<%d>", "lbm::k_collide<%d, false>")


def bench_trace(args):
    """Markdown summary of a kernel trace of bench.py itself (args.out: the trace folder,
    args.fetch: the JSON line that run printed): the average duration of each step kernel of the
    FP32 headline's profiled pass beside the bench's own event timing of the same kernels."""
    kt = summarize(args.out, 0)["kernels"]
    with open(args.fetch) as f:
        bench = json.loads(f.read().strip().splitlines()[-1])
    roof = bench["roofline"]
    lines = ["# bench.py under the kernel tracer: the 512^3 headline workload, FP32 and FP16 storage", "",
             "Command (repository root, `cd /tmp && export TMPDIR=/tmp` first, `PYTHONPATH` = repository root):", "",
             "```",
             "rocprofv3 --kernel-trace --stats --output-format csv -d OUT/prof -o run -- python3 bench.py %s "
             "> OUT/bench.json" % BENCH_ARGS,
             "python3 -m paper_2608_15781_amd.profile_run bench-trace OUT/prof OUT/bench.json",
             "```", "",
             "| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
    for name, k in sorted(kt.items(), key=lambda kv: -kv[1]["avg_us"] * kv[1]["calls"]):
        if name.startswith("lbm::"):
            lines.append("| `%s` | %d | %.2f | %.2f | %.2f |" % (name, k["calls"], k["avg_us"], k["min_us"],
                                                                k["max_us"]))
    # the FP32 headline's profiled pass: the last `steps` launches of each FP32 step kernel before the
    # FP16 run starts (every FP32 launch of the run comes first)
    trace = sorted(_rows(os.path.join(args.out, "**", "*kernel_trace.csv")), key=lambda r: int(r["Start_Timestamp"]))
    rows = ["", "| kernel (FP32 headline, profiled pass) | tracer avg us | bench.py event avg us |", "|---|---|---|"]
    tracer_sum = 0.0
    for name, key in zip(STEP_KERNELS, ("colour", "extrap", "normal", "collide")):
        kname = name % 1
        dur = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in trace
               if _short(r["Kernel_Name"]) == kname]
        timed = dur[-bench["steps"]:]
        avg = sum(timed) / max(1, len(timed))
        tracer_sum += avg
        rows.append("| `%s` | %.2f | %.2f |" % (kname, avg, 1e3 * roof["kernel_ms"].get(key, 0.0)))
    lines += rows
    lines += ["", "Same run, bench.py's own figures: %.1f MFLUPS over %d timed steps; step %.2f us from HIP events "
              "on the library's stream (tracer: %.2f us, the sum of the four kernels' averages over the same "
              "launches); roofline achieved %.1f GB/s = %.4f of %.0f GB/s at %d algorithmic bytes per fluid "
              "update. Under the tracer each event bracket also holds the tracer's own per-dispatch work." % (
                  bench["value"], bench["steps"], 1e3 * roof["avg_step_ms"], tracer_sum, roof["achieved"],
                  roof["frac"], roof["peak"], roof["alg_bytes_per_fluid_update"]), ""]
    print("\n".join(lines))


# Two counter sets, each within one run's per-block limits (8 SQ; 2 TA, 4 TCP, 2 TCC).
COUNTER_PASSES = (
    "SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_INST_ANY SQ_ACTIVE_INST_VMEM SQ_INST_LEVEL_VMEM "
    "SQ_INSTS_VMEM_RD SQ_LEVEL_WAVES",
    "TA_TA_BUSY TA_ADDR_STALLED_BY_TC_CYCLES TCP_PENDING_STALL_CYCLES TCP_TCC_READ_REQ "
    "TCP_READ_TAGCONFLICT_STALL_CYCLES TCP_PERF_SEL_TOTAL_READ TCC_HIT TCC_MISS",
)
CLOCK_HZ = 2.4e9  # MI355X peak engine clock
N_CU = 256        # one texture-address unit per compute unit


def _counters_per_kernel(out_dir):
    """Per kernel: dispatch count, mean duration (the counter run's own timestamps) and the mean
    of each counter per dispatch (summed over the counter's hardware instances)."""
    disp = {}
    for r in _rows(os.path.join(out_dir, "**", "*counter_collection.csv")):
        d = disp.setdefault(int(r["Dispatch_Id"]), dict(
            name=_short(r["Kernel_Name"]), dur=(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9, c={}))
        d["c"][r["Counter_Name"]] = d["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    agg = {}
    for d in disp.values():
        a = agg.setdefault(d["name"], dict(n=0, dur=0.0, c={}))
        a["n"] += 1
        a["dur"] += d["dur"]
        for k, v in d["c"].items():
            a["c"][k] = a["c"].get(k, 0.0) + v
    return {k: dict(n=a["n"], dur=a["dur"] / a["n"], c={c: v / a["n"] for c, v in a["c"].items()})
            for k, a in agg.items()}


def counters(args):
    """Markdown summary of the two hardware-counter runs of COUNTER_PASSES."""
    sys.path.insert(0, ROOT)
    from paper_2608_15781_amd import build

    pa, pb = _counters_per_kernel(args.out), _counters_per_kernel(args.fetch)
    lines = ["# Hardware counters of the step kernels, %s, %s storage" % (args.workload, args.precision), "",
             "Commands (repository root, `cd /tmp && export TMPDIR=/tmp` first, `PYTHONPATH` = repository root):", "",
             "```"]
    for k, ctrs in enumerate(COUNTER_PASSES):
        lines.append("rocprofv3 --pmc %s --output-format csv -d OUT/pass%s -o run -- python3 -m "
                     "paper_2608_15781_amd.profile_run --workload %s --precision %s --steps %d"
                     % (ctrs, "AB"[k], args.workload, args.precision, args.steps))
    lines += ["python3 -m paper_2608_15781_amd.profile_run counters --workload %s --precision %s --steps %d "
              "OUT/passA OUT/passB" % (args.workload, args.precision, args.steps), "```", "",
              "| kernel | dispatches | us (counter run) | TA busy | TA stalled on L2 | L2 hit | VMEM reads per wave |",
              "|---|---|---|---|---|---|---|"]

    def pct(x):
        return "%.0f%%" % (100 * x)

    for name in sorted(pb, key=lambda k: -pb[k]["dur"]):
        if not name.startswith("lbm::k_"):
            continue
        b, a = pb[name], pa.get(name)
        ta = b["c"].get("TA_TA_BUSY", 0.0)
        busy = ta / (b["dur"] * CLOCK_HZ * N_CU) if b["dur"] > 0 else 0.0
        stalled = b["c"].get("TA_ADDR_STALLED_BY_TC_CYCLES", 0.0) / ta if ta else 0.0
        hit, miss = b["c"].get("TCC_HIT", 0.0), b["c"].get("TCC_MISS", 0.0)
        l2 = hit / (hit + miss) if hit + miss else 0.0
        rd = "-"
        if a and a["c"].get("SQ_WAVES"):
            rd = "%.1f" % (a["c"].get("SQ_INSTS_VMEM_RD", 0.0) / a["c"]["SQ_WAVES"])
        lines.append("| `%s` | %d | %.2f | %s | %s | %s | %s |"
                     % (name, b["n"], b["dur"] * 1e6, pct(busy), pct(stalled), pct(l2), rd))
    lines += ["", "TA busy = TA_TA_BUSY / (duration x %.1f GHz x %d units): the share of the texture-address "
              "units' cycles spent processing vector-memory addresses (gathers, loads and stores); TA stalled on "
              "L2 = TA_ADDR_STALLED_BY_TC_CYCLES / TA_TA_BUSY; L2 hit = TCC_HIT / (TCC_HIT + TCC_MISS); VMEM reads "
              "per wave = SQ_INSTS_VMEM_RD / SQ_WAVES. Counter runs serialise the dispatches, so their durations read somewhat above the kernel trace's."
              % (CLOCK_HZ / 1e9, N_CU), "",
              "- source_digest: %s" % build.source_digest()]
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", nargs="?", default="run")
    ap.add_argument("out", nargs="?")
    ap.add_argument("fetch", nargs="?")
    ap.add_argument("write", nargs="?")
    ap.add_argument("--fluid-nodes", type=int, default=0)
    ap.add_argument("--mode", default="step", choices=["step", "adjoint"])
    ap.add_argument("--workload", default="bijel128")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--copy-mib", type=int, default=512)
    args = ap.parse_intermixed_args()
    if args.cmd == "summarize":
        print(json.dumps(summarize(args.out, args.copy_mib * (1 << 20)), indent=1))
    elif args.cmd == "report":
        args.trace = args.out
        report(args)
    elif args.cmd == "adjoint":
        run_adjoint(args)
    elif args.cmd == "bench-trace":
        bench_trace(args)
    elif args.cmd == "counters":
        counters(args)
    else:
        run(args)


if __name__ == "__main__":
    main()
