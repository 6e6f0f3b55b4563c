#!/usr/bin/env python3
"""Throughput of the reactive colour-gradient lattice Boltzmann step on one MI355X.

Workload: 128^3 porous mask (thresholded Gaussian random field, 512 plane waves of wavelength 16,
seed 2, ~50% porosity), two colours on D3Q19 with the central-moment collision, surface tension
0.01, Akai wetting at 60 degrees, body force 1e-6 along x on both colours, wall reaction xi = 1e-3,
D3Q7 species with inlet C = 1 at x = 0, all-reactant start. FP32 populations (the headline), and
FP16 / BF16 deviation storage with FP32 arithmetic; errors of each after the timed steps against
an FP64 run of the same library. One step = one pass of the whole step over the lattice; the
state is resident in HBM before the timed region starts.

Adjoint: 96^3 mask (wavelength 12, seed 4), contact angles 90 +- 10 degrees per node, 200 FP32
steps with a checkpoint every 20; the backward pass (recompute + adjoint steps) of the gas
production L = m^p(200) - m^p(0) is timed, and its gradients are compared with the FP64 ones.

Prints one JSON line. value = million fluid-node updates per second (MFLUPS).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and % HBM roofline, FP32 vs FP16-storage vs adjoint, at stated error"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
WORKLOAD = "bijel128"


def bytes_per_fluid_update(precision):
    """Algorithmic bytes per fluid node of each kernel (each array element moved once).

    State per node: 19 colour-blind populations and 7 species populations in storage precision
    (s bytes), 4 colour scalars (a, v) in arithmetic precision (r bytes); info word 4 bytes.
    """
    s = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}[precision]
    r = 8 if precision == "fp64" else 4
    colour = 19 * s + 4 * r + 4 + r                  # pull f^m, (a, v); info; write rho^N
    normal = r + 4 + 4 * r + 4 * r                   # rho^N; info; wetting data; write n*, |G|
    collide = 26 * s + r + 4 * r + 4 + 26 * s + 4 * r  # pull f^m, g; rho^N; n*, |G|; info; write state
    step_min = 2 * (26 * s + 4 * r) + 4              # state read once and written once, info
    naive = 2 * 45 * s + 1                           # 45 per-colour populations in and out, flag byte
    return dict(colour=colour, normal=normal, collide=collide, step_min=step_min, naive45=naive)


def measured_traffic(precision, kernel):
    """Calibrated HBM bytes per launch of a kernel from the committed counter summary, or None.

    The summary records the hash of the HIP sources it was taken on; a different hash means the
    kernels changed since, and the figure no longer applies.
    """
    path = os.path.join(ROOT, "profiles", "step_kernels_bijel128_%s.md" % precision)
    if not os.path.exists(path):
        return None
    from paper_2608_15781_amd import build as lbm_build

    digest, val = None, None
    with open(path) as f:
        for line in f:
            if line.startswith("- source_digest: "):
                digest = line.split(": ", 1)[1].strip()
            elif line.startswith("- traffic_bytes_per_launch %s: " % kernel):
                val = float(line.rsplit(": ", 1)[1])
    return val if digest == lbm_build.source_digest() else None


def make_inputs(device):
    from paper_2608_15781_amd import inputs

    w, solid, theta, rr0, rp0 = inputs.workload_inputs(WORKLOAD, device=device)
    return w, solid, theta, rr0, rp0


def sim_kwargs(w):
    return dict(tau=w["tau"], sigma=w["sigma"], beta=w["beta"], xi=w["xi"], accel=[(w["accel"], 0, 0)] * 2,
                species=w["species"], x_open=w["x_open"], tau_species=w["tau_c"], c_inlet=w["c_in"])


def run_mode(core, torch, w, solid, theta, rr0, rp0, precision, steps, warmup, profile):
    sim = core.Lbm(w["shape"], solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, precision=precision,
                   **sim_kwargs(w))
    sim.step(warmup, reductions=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    red = sim.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    mom = {k: v.clone() for k, v in sim.moments().items()}  # fields after warmup + steps
    kern = None
    if profile:
        sim.set_profiling(True)
        sim.step(steps, reductions=False)
        ms, n = sim.kernel_times()
        kern = {k: v / n for k, v in ms.items()}
        sim.set_profiling(False)
    return sim, red, dt, kern, mom


def adjoint_mode(core, torch, precision):
    """Forward + checkpointed backward of the gas production on the 96^3 adjoint workload."""
    from paper_2608_15781_amd import autograd as ag
    from paper_2608_15781_amd import inputs

    w, solid, theta, rr0, rp0 = inputs.workload_inputs("adjoint96", device="cuda:0")
    steps, ck = w["steps"], w["checkpoint"]
    sim = core.Lbm(w["shape"], solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, precision=precision,
                   **sim_kwargs(w))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L, cps, final = ag.forward_states(sim, steps, ck)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gth, gxi, _ = ag.adjoint_gradients(sim, steps, ck, cps, final)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    nfluid = int((solid == 0).sum())
    return dict(nfluid=nfluid, steps=steps, L=L, gth=gth, gxi=float(gxi), fwd_s=t1 - t0, bwd_s=t2 - t1)


def adjoint_keep_all(core, torch, precision):
    """The same gradient with every level kept by the forward pass (no recomputation). Timed
    with the kept levels' memory already in torch's cache (a second run)."""
    from paper_2608_15781_amd import autograd as ag
    from paper_2608_15781_amd import inputs

    w, solid, theta, rr0, rp0 = inputs.workload_inputs("adjoint96", device="cuda:0")
    steps = w["steps"]
    sim = core.Lbm(w["shape"], solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, precision=precision,
                   **sim_kwargs(w))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L, levels, final = ag.forward_keep_all(sim, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gth, gxi, _ = ag.adjoint_gradients_keep_all(sim, levels, final)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    kept = steps * (sim.state_bytes + sim.fields_bytes())
    del levels, final
    torch.cuda.empty_cache()
    return dict(L=L, gth=gth, gxi=float(gxi), fwd_s=t1 - t0, bwd_s=t2 - t1, kept_bytes=kept)


def rel_l2(a, b):
    a = a.double()
    b = b.double()
    return float(((a - b).norm() / b.norm()).item()) if b.norm() > 0 else float((a - b).norm().item())


def device_copy_gbs(torch, nbytes=1 << 30, reps=10):
    """Achievable streaming rate: bytes read + written per second by a device-to-device copy of a
    buffer four times the last-level cache, timed with events on the current stream."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0").fill_(1)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / sec / 1e9


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, solid, theta, rr0, rp0, nfluid, steps):
    import oracle

    kw = dict(tau=w["tau"], sigma=w["sigma"], beta=w["beta"], accel=[(w["accel"], 0, 0)] * 2,
              species=w["species"], x_open=w["x_open"], tau_c=w["tau_c"], c_in=w["c_in"])
    o = oracle.Oracle(w["shape"], solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, xi=w["xi"], **kw)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return dict(value=nfluid * steps / dt / 1e6, unit="MFLUPS", cores=oracle.get_threads(), kind="oracle",
                sample="%d steps of the full 128^3 workload (FP64, OpenMP over z), %.1f s" % (steps, dt),
                cpu_model=cpu_model())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=64)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--modes", default="fp16,bf16", help="extra storage precisions to time")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path (the step would shard by "
              "spatial domain decomposition with face exchanges between GPUs; that is not implemented).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2608_15781_amd import core

    core.lib()
    print("bench: building %s inputs" % WORKLOAD, file=sys.stderr, flush=True)
    w, solid, theta, rr0, rp0 = make_inputs("cuda:0")
    nfluid = int((solid == 0).sum())
    nx, ny, nz = w["shape"]
    nall = nx * ny * nz

    print("bench: fp32 headline, %d warmup + %d timed steps" % (args.warmup, args.steps), file=sys.stderr, flush=True)
    sim32, red32, dt32, kern32, mom32 = run_mode(core, torch, w, solid, theta, rr0, rp0, "fp32", args.steps, args.warmup,
                                          profile=True)
    mflups = nfluid * args.steps / dt32 / 1e6
    ms_step = dt32 * 1e3 / args.steps
    b = bytes_per_fluid_update("fp32")
    coll_s = kern32["collide"] * 1e-3
    achieved = b["collide"] * nfluid / coll_s / 1e9

    # Reference: the same steps in FP64 storage and arithmetic.
    print("bench: fp64 reference run", file=sys.stderr, flush=True)
    sim64, red64, dt64, _, m64 = run_mode(core, torch, w, solid, theta, rr0, rp0, "fp64", args.steps, args.warmup,
                                     profile=False)
    conv64 = red64[:, 2].sum()

    def errors(m, red):
        rm = m["rho_r"] + m["rho_p"]
        rm64 = m64["rho_r"] + m64["rho_p"]
        return dict(rho_m=rel_l2(rm, rm64), u=rel_l2(m["u"], m64["u"]), rho_n=rel_l2(m["rho_n"], m64["rho_n"]),
                    c=rel_l2(m["c"], m64["c"]), conversion=float(abs(red[:, 2].sum() - conv64) / conv64))

    err32 = errors(mom32, red32)
    modes = {"fp32": dict(mflups=mflups, ms_per_step=ms_step, error_vs_fp64=err32, kernel_ms=kern32),
             "fp64": dict(mflups=nfluid * args.steps / dt64 / 1e6, ms_per_step=dt64 * 1e3 / args.steps)}
    del sim32
    for prec in [m for m in args.modes.split(",") if m]:
        print("bench: %s mode" % prec, file=sys.stderr, flush=True)
        sim, red, dt, kern, mom = run_mode(core, torch, w, solid, theta, rr0, rp0, prec, args.steps, args.warmup,
                                           profile=True)
        bp = bytes_per_fluid_update(prec)
        modes[prec] = dict(mflups=nfluid * args.steps / dt / 1e6, ms_per_step=dt * 1e3 / args.steps,
                           error_vs_fp64=errors(mom, red), kernel_ms=kern,
                           collide_gbs=bp["collide"] * nfluid / (kern["collide"] * 1e-3) / 1e9)
        del sim
    del sim64

    adjoint = None
    if not args.no_adjoint:
        print("bench: adjoint (96^3, 200 steps, checkpoint 20), fp32 and fp64", file=sys.stderr, flush=True)
        # each timed on its second run, with its buffers already in torch's cache
        adjoint_mode(core, torch, "fp32")
        a32 = adjoint_mode(core, torch, "fp32")
        adjoint_mode(core, torch, "fp64")
        a64 = adjoint_mode(core, torch, "fp64")
        adjoint_keep_all(core, torch, "fp32")  # first run maps the kept levels' memory
        k32 = adjoint_keep_all(core, torch, "fp32")
        adjoint = dict(
            workload="96^3 porous GRF mask (wavelength 12, seed 4), theta 90 +- 10 deg per node, %d steps, "
                     "checkpoint every 20, dL/dtheta and dL/dxi of the gas production" % a32["steps"],
            timed="second run of each mode (its buffers already in torch's memory cache)",
            fluid_nodes=a32["nfluid"],
            mflups=round(a32["nfluid"] * a32["steps"] / a32["bwd_s"] / 1e6, 1),
            mflups_forward_with_checkpoints=round(a32["nfluid"] * a32["steps"] / a32["fwd_s"] / 1e6, 1),
            backward_s=round(a32["bwd_s"], 4), forward_s=round(a32["fwd_s"], 4),
            fp64_backward_s=round(a64["bwd_s"], 4),
            error_vs_fp64=dict(L=abs(a32["L"] - a64["L"]) / abs(a64["L"]), dtheta=rel_l2(a32["gth"], a64["gth"]),
                               dxi=abs(a32["gxi"] - a64["gxi"]) / abs(a64["gxi"])),
            keep_all_levels=dict(
                mflups=round(a32["nfluid"] * a32["steps"] / k32["bwd_s"] / 1e6, 1),
                backward_s=round(k32["bwd_s"], 4), forward_s=round(k32["fwd_s"], 4),
                kept_gb=round(k32["kept_bytes"] / 1e9, 2),
                same_gradient_as_checkpointed=bool(torch.equal(k32["gth"], a32["gth"]) and k32["gxi"] == a32["gxi"])))
        del a32, a64, k32

    cpu = None
    if not args.no_cpu:
        print("bench: cpu baseline (oracle, %d steps)" % args.cpu_steps, file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, solid, theta, rr0, rp0, nfluid, args.cpu_steps)

    traffic = measured_traffic("fp32", "lbm::k_collide<1, false>")
    copy_gbs = device_copy_gbs(torch)

    out = {
        "metric": METRIC,
        "value": round(mflups, 1),
        "unit": "MFLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "128^3 porous GRF mask (wavelength 16, seed 2, porosity %.3f), D3Q19 two-colour "
                               "CG-LBM + D3Q7 species, FP32 storage" % (nfluid / nall),
                   "lattice": [nx, ny, nz], "fluid_nodes": nfluid, "parallelism": "single GPU"},
        "mlups_all_nodes": round(nall * args.steps / dt32 / 1e6, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": "k_collide",
                     "alg_bytes_per_fluid_node": b["collide"], "avg_launch_ms": round(kern32["collide"], 5),
                     "device_copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)},
        "step_roofline": {"alg_bytes_per_fluid_update": b["step_min"],
                          "frac": round(mflups * 1e6 * b["step_min"] / (HBM_PEAK_GBS * 1e9), 4),
                          "naive45_bytes_per_fluid_update": b["naive45"],
                          "naive45_equiv_frac": round(mflups * 1e6 * b["naive45"] / (HBM_PEAK_GBS * 1e9), 4)},
        "modes": modes,
        "adjoint": adjoint,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
