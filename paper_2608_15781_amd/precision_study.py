"""Storage-precision studies on the large porous workloads (one GPU).

    python3 -m paper_2608_15781_amd.precision_study storage256 [--steps 5000]
        256^3 mask (wavelength 16, seed 3): FP32, FP16-deviation and BF16-deviation storage against
        the library's FP64 run of the same steps. Relative L2 errors of rho^m, u_phys, rho^N and C,
        relative error of the total conversion, and the throughput of each mode.

    python3 -m paper_2608_15781_amd.precision_study large512 [--steps 10000]
        512^3 mask (wavelength 32, porosity 0.55, theta 30 deg): FP32 and FP16-deviation storage.
        Sustained MFLUPS, algorithmic HBM GB/s of the step, conversion efficiency
        sum(conversion FP16) / sum(conversion FP32), and the FP16 field errors against FP32.

Both print progress lines to stderr and one JSON object to stdout. The FP64 library run used as
the reference is validated against the FP64 oracle by the GPU parity tests (crops of the same
masks and the full 128^3 workload).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def _kwargs(w):
    return dict(tau=w["tau"], sigma=w["sigma"], beta=w["beta"], xi=w["xi"], accel=[(w["accel"], 0, 0)] * 2,
                species=w["species"], x_open=w["x_open"], tau_species=w["tau_c"], c_inlet=w["c_in"])


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _run(core, torch, w, solid, theta, rr0, rp0, precision, steps, chunk=1000, tag=""):
    """Runs `steps` steps in chunks (progress line per chunk); returns (sim, conversion sum, seconds)."""
    sim = core.Lbm(w["shape"], solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, precision=precision,
                   **_kwargs(w))
    torch.cuda.synchronize()
    conv = 0.0
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        red = sim.step(n)
        conv += float(red[:, 2].sum())
        done += n
        _log("%s %s: %d / %d steps, %.1f s" % (tag, precision, done, steps, time.perf_counter() - t0))
    torch.cuda.synchronize()
    return sim, conv, time.perf_counter() - t0


def _fields(sim):
    m = sim.moments()
    return dict(rho_m=(m["rho_r"] + m["rho_p"]).double(), u=m["u"].double(), rho_n=m["rho_n"].double(),
                c=m["c"].double())


def _rel_l2(a, b):
    nb = float(b.norm())
    return float((a - b).norm()) / nb if nb > 0 else float((a - b).norm())


def _errors(f, ref):
    return {k: _rel_l2(f[k], ref[k]) for k in ref}


def storage256(args):
    import torch

    from paper_2608_15781_amd import core, inputs

    w, solid, theta, rr0, rp0 = inputs.workload_inputs("bijel256", device="cuda:0")
    nfluid = int((solid == 0).sum())
    out = dict(workload="256^3 porous GRF mask (wavelength 16, seed 3, porosity %.3f), theta 60 deg, %d steps"
               % (nfluid / solid.size, args.steps), fluid_nodes=nfluid, modes={})
    sim, conv64, dt = _run(core, torch, w, solid, theta, rr0, rp0, "fp64", args.steps, tag="256")
    ref = _fields(sim)
    del sim
    out["modes"]["fp64"] = dict(mflups=nfluid * args.steps / dt / 1e6, conversion=conv64)
    for prec in ("fp32", "fp16", "bf16"):
        sim, conv, dt = _run(core, torch, w, solid, theta, rr0, rp0, prec, args.steps, tag="256")
        err = _errors(_fields(sim), ref)
        err["conversion"] = abs(conv - conv64) / abs(conv64)
        out["modes"][prec] = dict(mflups=nfluid * args.steps / dt / 1e6, conversion=conv, error_vs_fp64=err)
        del sim
        torch.cuda.empty_cache()
    return out


def large512(args):
    import torch

    from paper_2608_15781_amd import core, inputs

    _log("512: building inputs")
    w, solid, theta, rr0, rp0 = inputs.workload_inputs("bijel512", device="cuda:0")
    nfluid = int((solid == 0).sum())
    out = dict(workload="512^3 porous GRF mask (wavelength 32, seed 5, porosity %.3f), theta 30 deg, %d steps"
               % (nfluid / solid.size, args.steps), fluid_nodes=nfluid, modes={})
    bytes_step = {"fp32": 2 * (26 * 4 + 16) + 4, "fp16": 2 * (26 * 2 + 16) + 4}
    fields = {}
    for prec in ("fp32", "fp16"):
        sim, conv, dt = _run(core, torch, w, solid, theta, rr0, rp0, prec, args.steps, tag="512")
        sim.set_profiling(True)
        sim.step(100, reductions=False)
        ms, n = sim.kernel_times()
        sim.set_profiling(False)
        mflups = nfluid * args.steps / dt / 1e6
        out["modes"][prec] = dict(mflups=mflups, conversion=conv, seconds=dt,
                                  step_alg_gbs=mflups * 1e6 * bytes_step[prec] / 1e9,
                                  kernel_us={k: 1e3 * v / n for k, v in ms.items()})
        fields[prec] = _fields(sim)
        del sim
        torch.cuda.empty_cache()
    out["conversion_efficiency_fp16_over_fp32"] = out["modes"]["fp16"]["conversion"] / out["modes"]["fp32"]["conversion"]
    out["fp16_error_vs_fp32"] = _errors(fields["fp16"], fields["fp32"])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["storage256", "large512"])
    ap.add_argument("--steps", type=int, default=None)
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 5000 if args.study == "storage256" else 10000
    res = storage256(args) if args.study == "storage256" else large512(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
