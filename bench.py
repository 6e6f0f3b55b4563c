#!/usr/bin/env python3
"""Throughput of the reactive colour-gradient lattice Boltzmann step on one MI355X.

Headline workload: 512^3 porous mask (thresholded Gaussian random field, 512 plane waves of
wavelength 32, seed 5, porosity 0.55), two colours on D3Q19 with the central-moment collision,
surface tension 0.01, Akai wetting at 30 degrees, body force 1e-6 along x on both colours, wall
reaction xi = 1e-3, D3Q7 species with inlet C = 1 at x = 0, all-reactant start. FP32 populations
(the headline value) and FP16 deviation storage with FP32 arithmetic beside it (its fields and
conversion compared with the FP32 run). One step = one pass of the whole step over the lattice;
the state is resident in HBM before the timed region starts.

Roofline: the whole step against HBM, with the algorithmic bytes per fluid update of the
45-population representation (each population read once and written once, plus a flag byte:
2 x 45 x 4 + 1 = 361 B in FP32, 181 B with 2-byte storage), divided by the step's device time
measured with HIP events on the library's stream.

Beside the headline: the 128^3 workload (wavelength 16, seed 2, 60 degrees) in FP32, FP16 and BF16
storage with errors against an FP64 run of the same library; the adjoint on the 96^3 workload
(wavelength 12, seed 4), contact angles 90 +- 10 degrees per node, 200 FP32 steps with a checkpoint
every 20: the backward pass (recompute + adjoint steps) of the gas production
L = m^p(200) - m^p(0) is timed and its gradients compared with the FP64 ones; and the FP64 CPU
oracle on a 128^3 crop of the headline mask.

Prints one JSON line. value = million fluid-node updates per second (MFLUPS).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and % HBM roofline, FP32 vs FP16-storage vs adjoint, at stated error"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
HEADLINE = "bijel512"  # the largest single-GPU workload
SIDE = "bijel128"      # error modes against FP64


def bytes_per_fluid_update(precision):
    """Algorithmic bytes per fluid update.

    naive45: the 45-population representation (38 colour + 7 species), each population read once
    and written once in storage precision s, plus a flag byte. step_min: the compact state this
    library stores (19 colour-blind + 7 species populations in s bytes, 4 colour scalars in
    arithmetic precision r), read once and written once, plus the 4-byte info word.
    """
    s = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}[precision]
    r = 8 if precision == "fp64" else 4
    return dict(naive45=2 * 45 * s + 1, step_min=2 * (26 * s + 4 * r) + 4)


def measured_step_traffic(workload, precision, kernels):
    """Calibrated HBM bytes of one step (sum over its kernels) from the committed counter summary
    of that workload, or None. The summary records the hash of the HIP sources it was taken on;
    a different hash means the kernels changed since, and the figure no longer applies."""
    path = os.path.join(ROOT, "profiles", "step_kernels_%s_%s.md" % (workload, precision))
    if not os.path.exists(path):
        return None
    from paper_2608_15781_amd import build as lbm_build

    digest, vals = None, {}
    with open(path) as f:
        for line in f:
            if line.startswith("- source_digest: "):
                digest = line.split(": ", 1)[1].strip()
            elif line.startswith("- traffic_bytes_per_launch "):
                name, val = line[len("- traffic_bytes_per_launch "):].rsplit(": ", 1)
                vals[name] = float(val)
    if digest != lbm_build.source_digest():
        return None
    picked = [v for k, v in vals.items() if any(k.startswith(kn) for kn in kernels)]
    return sum(picked) if picked else None


def sim_kwargs(w):
    return dict(tau=w["tau"], sigma=w["sigma"], beta=w["beta"], xi=w["xi"], accel=[(w["accel"], 0, 0)] * 2,
                species=w["species"], x_open=w["x_open"], tau_species=w["tau_c"], c_inlet=w["c_in"])


def run_mode(core, torch, w, solid, theta, rr0, rp0, precision, steps, warmup, profile, fields=True):
    """W untimed steps, then K steps timed with the host clock between device synchronisations;
    then (profile) K more steps with HIP events around every kernel on the library's stream."""
    sim = core.Lbm(w["shape"], solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, precision=precision,
                   **sim_kwargs(w))
    sim.step(warmup, reductions=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    red = sim.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    mom = {k: v.clone() for k, v in sim.moments().items()} if fields else None  # after warmup + steps
    kern = None
    if profile:
        sim.set_profiling(True)
        sim.step(steps, reductions=False)
        ms, n = sim.kernel_times()
        kern = {k: v / n for k, v in ms.items() if v > 0}
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


def cpu_baseline(w, solid, theta, rr0, rp0, steps, size=128):
    """The FP64 oracle on the leading size^3 corner of the headline mask (same wavelength,
    threshold, angle and physics), timed on all host cores."""
    import oracle
    from paper_2608_15781_amd import inputs

    c = [inputs.crop(a, size) for a in (solid, theta, rr0, rp0)]
    nfluid = int((c[0] == 0).sum())
    kw = dict(tau=w["tau"], sigma=w["sigma"], beta=w["beta"], accel=[(w["accel"], 0, 0)] * 2,
              species=w["species"], x_open=w["x_open"], tau_c=w["tau_c"], c_in=w["c_in"])
    o = oracle.Oracle((size, size, size), solid=c[0], theta=c[1], rho_r0=c[2], rho_p0=c[3], xi=w["xi"], **kw)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return dict(value=nfluid * steps / dt / 1e6, unit="MFLUPS", cores=oracle.get_threads(), kind="oracle",
                sample="%d steps of the leading %d^3 corner of the 512^3 mask (%d fluid nodes; FP64, OpenMP "
                       "over z), %.1f s" % (steps, size, nfluid, dt),
                cpu_model=cpu_model())


def step_roofline(mflups, kern, nfluid, precision, workload, copy_gbs):
    """The whole step against HBM: algorithmic bytes of the 45-population representation per
    fluid update, over the step's device time (sum of its kernels' HIP-event averages)."""
    b = bytes_per_fluid_update(precision)
    step_s = sum(kern.values()) * 1e-3
    achieved = b["naive45"] * nfluid / step_s / 1e9
    traffic = measured_step_traffic(workload, precision, ["lbm::k_"])
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "kernel": "one step (%s)" % " + ".join("k_" + k for k in kern),
           "alg_bytes_per_fluid_update": b["naive45"], "fluid_nodes_per_launch": nfluid,
           "avg_step_ms": round(step_s * 1e3, 5),
           "frac_from_mflups": round(mflups * 1e6 * b["naive45"] / (HBM_PEAK_GBS * 1e9), 4),
           "compact_state_bytes_per_fluid_update": b["step_min"],
           "compact_state_frac": round(b["step_min"] * nfluid / step_s / 1e9 / HBM_PEAK_GBS, 4),
           "device_copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
           "kernel_ms": {k: round(v, 5) for k, v in kern.items()}}
    if traffic is not None:
        out["traffic_bytes_per_fluid_update"] = round(traffic / nfluid, 1)
    per = {}
    for k, ms in kern.items():
        alg = kernel_alg_bytes(precision).get(k)
        e = {"ms": round(ms, 5)}
        if alg is not None:
            gbs = alg * nfluid / (ms * 1e-3) / 1e9
            e.update(alg_bytes_per_fluid_node=alg, achieved_gbs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4))
        t = measured_step_traffic(workload, precision, ["lbm::k_%s<" % k])
        if t is not None:
            e.update(traffic_bytes_per_fluid_node=round(t / nfluid, 1),
                     traffic_gbs=round(t / (ms * 1e-3) / 1e9, 1))
        per[k] = e
    out["per_kernel"] = per
    return out


def kernel_alg_bytes(precision):
    """Algorithmic bytes per fluid node of the colour, normal and collide passes (each array element
    they need moved once; s = storage bytes, r = arithmetic bytes): colour pulls 19 colour-blind
    populations and the 4 colour scalars and writes rho^N; normal reads rho^N and the wetting
    data and writes (n*, |G|); collide pulls and writes the 26 populations and 4 scalars and reads
    rho^N and the normals (plus the species totals with 2-byte storage). The extrapolation pass
    works on solid nodes and has no per-fluid-node figure."""
    s = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}[precision]
    r = 8 if precision == "fp64" else 4
    extra = 2 * r if s == 2 else 0
    return {"colour": 19 * s + 4 * r + 4 + r, "normal": r + 4 + 4 * r + 4 * r,
            "collide": 26 * s + r + 4 * r + 4 + 26 * s + 4 * r + extra}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--side-steps", type=int, default=2000, help="steps of the 128^3 error modes")
    ap.add_argument("--cpu-steps", type=int, default=48)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-side", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path (the step would shard by "
              "spatial domain decomposition with face exchanges between GPUs; that is not implemented).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2608_15781_amd import core, inputs

    core.lib()
    print("bench: building %s inputs" % HEADLINE, file=sys.stderr, flush=True)
    w, solid, theta, rr0, rp0 = inputs.workload_inputs(HEADLINE, device="cuda:0")
    nfluid = int((solid == 0).sum())
    nx, ny, nz = w["shape"]
    nall = nx * ny * nz
    # the achievable streaming rate, measured first: it also brings the GPU out of idle before
    # the timed region
    copy_gbs = device_copy_gbs(torch)

    print("bench: fp32 headline, %d warmup + %d timed steps" % (args.warmup, args.steps), file=sys.stderr, flush=True)
    sim32, red32, dt32, kern32, mom32 = run_mode(core, torch, w, solid, theta, rr0, rp0, "fp32", args.steps,
                                                 args.warmup, profile=True)
    mflups = nfluid * args.steps / dt32 / 1e6
    ms_step = dt32 * 1e3 / args.steps
    del sim32
    print("bench: fp16 storage, %d warmup + %d timed steps" % (args.warmup, args.steps), file=sys.stderr, flush=True)
    sim16, red16, dt16, kern16, mom16 = run_mode(core, torch, w, solid, theta, rr0, rp0, "fp16", args.steps,
                                                 args.warmup, profile=True)
    del sim16
    mfl16 = nfluid * args.steps / dt16 / 1e6
    conv32, conv16 = float(red32[:, 2].sum()), float(red16[:, 2].sum())
    fp16 = dict(mflups=round(mfl16, 1), ms_per_step=round(dt16 * 1e3 / args.steps, 5),
                roofline=step_roofline(mfl16, kern16, nfluid, "fp16", HEADLINE, copy_gbs),
                vs_fp32=dict(steps=args.warmup + args.steps,
                             rho_m=rel_l2(mom16["rho_r"] + mom16["rho_p"], mom32["rho_r"] + mom32["rho_p"]),
                             u=rel_l2(mom16["u"], mom32["u"]), rho_n=rel_l2(mom16["rho_n"], mom32["rho_n"]),
                             c=rel_l2(mom16["c"], mom32["c"]),
                             conversion_efficiency=conv16 / conv32 if conv32 else None))
    del mom16, mom32
    torch.cuda.empty_cache()

    side = None
    if not args.no_side:
        print("bench: %s modes (fp64 reference, fp32, fp16, bf16), %d steps" % (SIDE, args.side_steps),
              file=sys.stderr, flush=True)
        ws, ss, ths, rrs, rps = inputs.workload_inputs(SIDE, device="cuda:0")
        nfs = int((ss == 0).sum())
        _, red64, dt64, _, m64 = run_mode(core, torch, ws, ss, ths, rrs, rps, "fp64", args.side_steps, 100,
                                          profile=False)
        conv64 = red64[:, 2].sum()
        side = dict(workload="128^3 porous GRF mask (wavelength 16, seed 2, porosity %.3f), theta 60 deg, "
                             "errors after %d steps against the library's FP64 run" % (nfs / ss.size,
                                                                                        100 + args.side_steps),
                    fluid_nodes=nfs,
                    modes={"fp64": dict(mflups=round(nfs * args.side_steps / dt64 / 1e6, 1))})
        for prec in ("fp32", "fp16", "bf16"):
            sim, red, dt, kern, m = run_mode(core, torch, ws, ss, ths, rrs, rps, prec, args.side_steps, 100,
                                             profile=True)
            del sim
            mfl = nfs * args.side_steps / dt / 1e6
            side["modes"][prec] = dict(
                mflups=round(mfl, 1), roofline=step_roofline(mfl, kern, nfs, prec, SIDE, copy_gbs),
                error_vs_fp64=dict(rho_m=rel_l2(m["rho_r"] + m["rho_p"], m64["rho_r"] + m64["rho_p"]),
                                   u=rel_l2(m["u"], m64["u"]), rho_n=rel_l2(m["rho_n"], m64["rho_n"]),
                                   c=rel_l2(m["c"], m64["c"]),
                                   conversion=float(abs(red[:, 2].sum() - conv64) / conv64)))
        del m64
        torch.cuda.empty_cache()

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
        print("bench: cpu baseline (oracle, %d steps on a 128^3 corner)" % args.cpu_steps, file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, solid, theta, rr0, rp0, args.cpu_steps)

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
        "config": {"workload": "512^3 porous GRF mask (wavelength 32, seed 5, porosity %.3f), contact angle 30 deg, "
                               "D3Q19 two-colour CG-LBM + D3Q7 species, FP32 storage" % (nfluid / nall),
                   "lattice": [nx, ny, nz], "fluid_nodes": nfluid, "parallelism": "single GPU"},
        "mlups_all_nodes": round(nall * args.steps / dt32 / 1e6, 1),
        "roofline": step_roofline(mflups, kern32, nfluid, "fp32", HEADLINE, copy_gbs),
        "fp16_storage": fp16,
        "side_128": side,
        "adjoint": adjoint,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
