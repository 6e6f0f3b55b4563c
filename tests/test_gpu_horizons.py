"""The 256^3 and 512^3 workloads at their full horizons against the oracle, on crops the oracle
steps in about 20 s: the leading 40^3 corner of the 256^3 mask (wavelength 16, seed 3, theta
60 deg) over 5000 steps, and the leading 32^3 corner of the 512^3 mask (wavelength 32, porosity
0.55 over the whole mask, theta 30 deg) over 10^4 steps, both with the species, open x faces,
xi = 1e-3 and the all-reactant start. Every storage the workload is run in is compared with the
same oracle state: densities, colour function, species, populations and the per-step sums in max
norm relative to the field's maximum, the velocity in relative L2.

Measured (max norm / velocity L2): 256^3 crop FP64 2.9e-11 / 7e-12, FP32 2.9e-4 / 1.1e-4, FP16
2.8e-3 / 9.1e-4, BF16 1.9e-2 / 5.6e-3; 512^3 crop FP64 1.2e-11 / 9e-12, FP32 1.8e-4 / 2.1e-4, FP16
2.4e-3 / 1.4e-3. The FP64 bound is the parity tolerance; the others leave a factor of 3 to 7:
FP32 rounding (6e-8 per operation) and the 11-bit (FP16) or 8-bit (BF16) deviations grow along
the interfaces over these horizons."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

BOUNDS = {"fp64": (1e-10, 1e-10), "fp32": (2e-3, 2e-3), "fp16": (1e-2, 6e-3), "bf16": (6e-2, 2.5e-2)}


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / np.abs(b).max())


def _l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def core():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_15781_amd import core as c

    c.lib()
    return c


def _horizon(core, oracle_mod, workload, n, T, precisions):
    from paper_2608_15781_amd import inputs

    w, solid, theta, rr0, rp0 = inputs.workload_inputs(workload, size=n, device="cuda:0")
    kw = dict(tau=w["tau"], sigma=w["sigma"], beta=w["beta"], accel=[(w["accel"], 0, 0)] * 2, species=True,
              x_open=True, xi=w["xi"])
    ref = oracle_mod.Oracle((n, n, n), solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, tau_c=w["tau_c"], **kw)
    rr = ref.step(T)
    assert rr[-1, 1] > 0  # gas was produced
    r = ref.moments()
    rfr, rfp, rgg = ref.get_state()
    for prec in precisions:
        g = core.Lbm((n, n, n), solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, precision=prec,
                     tau_species=w["tau_c"], **kw)
        red = g.step(T)
        m = g.moments()
        fr, fp, gg = g.populations()
        mx = {k: _rel(m[k].cpu().numpy(), r[k]) for k in ("rho_r", "rho_p", "rho_n", "c")}
        mx["pops"] = max(_rel(fr.cpu().numpy(), rfr), _rel(fp.cpu().numpy(), rfp), _rel(gg.cpu().numpy(), rgg))
        mx["sums"] = max(_rel(red[:, j], rr[:, j]) for j in (0, 1, 2, 3))
        u_l2 = _l2(m["u"].cpu().numpy(), r["u"])
        print("%s crop %d^3 %s t=%d max: %s | u L2 %.2e" % (workload, n, prec, T,
              " ".join("%s=%.1e" % kv for kv in mx.items()), u_l2), flush=True)
        tol, tol_u = BOUNDS[prec]
        for k, e in mx.items():
            assert e < tol, (prec, k, e)
        assert u_l2 < tol_u, (prec, u_l2)
        del g


def test_bijel256_crop40_5000_steps(core, oracle_mod):
    _horizon(core, oracle_mod, "bijel256", 40, 5000, ("fp64", "fp32", "fp16", "bf16"))


def test_bijel512_crop32_10000_steps(core, oracle_mod):
    _horizon(core, oracle_mod, "bijel512", 32, 10000, ("fp64", "fp32", "fp16"))
