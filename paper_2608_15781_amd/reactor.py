"""The paper's reactor set-up and effectiveness-factor analysis on top of the library's step.

Geometry diagnostics (Sec. "Porous structures"): nearest solid neighbours NN
(eq. nearest_solid_neighbors), surface area A (eq. surface_area), porosity phi (eq. porosity),
single-phase permeability from Darcy's law (eq. permeability) and the reactor efficiency number
eta = kappa (A/V)^2.

Reaction set-up (Sec. "Numerical parameter mapping"): one bubble nucleation site, a fluid node
with exactly one solid face neighbour, per 64^3 block; reaction rate xi = 1; surface tension
sigma = 0.3; the body force a from the pressure Bond number (eq. bond_number_pressure); the
viscosity, hence tau (eq. kinematic_viscosity), from the Damkohler number (eq. damkohler_number).

Analysis (Sec. "Theoretical model"): effectiveness factor alpha(t) (eq. effectiveness_factor),
its running mean (eq. effectiveness_factor_avg), and the fit of the reactant mass to the
exponential decay (eq. effectiveness_factor_solution).

    python3 -m paper_2608_15781_amd.reactor permeability --workload bijel128
    python3 -m paper_2608_15781_amd.reactor run --workload bijel128 --da 1 --theta 60 --steps 50000

Each prints one JSON object. The masks are the seeded random-field stand-ins of inputs.py.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

# Face directions of D3Q19 (|c|^2 = 1).
_FACES = ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))


def nearest_solid_neighbors(solid):
    """NN(x) = l(x) * number of solid face neighbours (periodic); solid is (nz, ny, nx), 1 = solid."""
    s = np.asarray(solid, dtype=np.int32)
    nn = np.zeros_like(s)
    for cx, cy, cz in _FACES:
        nn += np.roll(s, shift=(-cz, -cy, -cx), axis=(0, 1, 2))
    return nn * (1 - s)


def geometry_properties(solid):
    """Surface area A = sum NN, porosity phi, volume V, A / V."""
    nn = nearest_solid_neighbors(solid)
    V = int(np.asarray(solid).size)
    A = int(nn.sum())
    phi = float((np.asarray(solid) == 0).sum()) / V
    return dict(A=A, phi=phi, V=V, A_over_V=A / V)


def reactor_efficiency(kappa, A_over_V):
    """eta = kappa (A/V)^2."""
    return kappa * A_over_V ** 2


def nucleation_sites(solid, block=64, seed=0):
    """Reactive indicator r(x): in every block^3 block of the lattice (blocks at the domain's far
    faces may be partial), one fluid node with exactly one solid face neighbour, drawn with a seeded
    generator; r = 0 elsewhere. Blocks without such a node get no site. Returns (r, sites) with
    sites the chosen (x, y, z)."""
    solid = np.asarray(solid)
    nz, ny, nx = solid.shape
    cand = nearest_solid_neighbors(solid) == 1
    rng = np.random.default_rng(seed)
    r = np.zeros(solid.shape, np.uint8)
    sites = []
    for z0 in range(0, nz, block):
        for y0 in range(0, ny, block):
            for x0 in range(0, nx, block):
                sub = cand[z0:z0 + block, y0:y0 + block, x0:x0 + block]
                idx = np.flatnonzero(sub)
                if idx.size == 0:
                    continue
                k = int(idx[rng.integers(idx.size)])
                dz, rem = divmod(k, sub.shape[1] * sub.shape[2])
                dy, dx = divmod(rem, sub.shape[2])
                r[z0 + dz, y0 + dy, x0 + dx] = 1
                sites.append((x0 + dx, y0 + dy, z0 + dz))
    return r, sites


def acceleration_from_bond(bo_p, sigma, radius):
    """Body force per unit mass from the pressure Bond number Bo_p = rho a R^2 / sigma (rho = 1)."""
    return bo_p * sigma / radius ** 2


def viscosity_from_damkohler(da, xi, area_r, length, kappa, volume, accel):
    """nu from Da = xi A_r nu L / (kappa V a)."""
    return da * kappa * volume * accel / (xi * area_r * length)


def tau_from_viscosity(nu):
    """tau from nu = c_s^2 (tau - 1/2), c_s^2 = 1/3."""
    return 3.0 * nu + 0.5


def effectiveness(m_r, conversion, xi, area_r, phi, volume):
    """alpha(t) = mdot^r(t) / mdot^r_th(t) with mdot^r = -conversion(t) and
    mdot^r_th = -(xi A_r / (phi V)) m^r(t); and its running mean (1/t) sum_{i<=t} alpha(i)
    (the sum over t + 1 values, divided by t + 1 so that the mean of the first value is itself)."""
    m_r = np.asarray(m_r, dtype=np.float64)
    conv = np.asarray(conversion, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        alpha = np.where(m_r > 0, conv * phi * volume / (xi * area_r * m_r), 0.0)
    mean = np.cumsum(alpha) / np.arange(1, alpha.size + 1)
    return alpha, mean


def fit_alpha(m_r, m_m, xi, area_r, phi, volume, t0=0, t1=None):
    """Least-squares fit of ln(m^r(t) / m^m) = -(xi A_r / (phi V)) alpha t over t0 <= t < t1 (a line
    through the origin, the integration constant being the initial reactant mass m^m)."""
    m_r = np.asarray(m_r, dtype=np.float64)
    t1 = m_r.size if t1 is None else t1
    t = np.arange(t0, t1, dtype=np.float64)
    y = np.log(m_r[t0:t1] / m_m)
    slope = float((t * y).sum() / (t * t).sum())
    return -slope * phi * volume / (xi * area_r)


def permeability(core, solid, axis=0, accel=1e-6, nu=0.1, precision="fp64", check_every=500, rtol=1e-6,
                 max_steps=200000, device="cuda:0"):
    """Single-phase permeability along `axis` from Darcy's law kappa = nu <u> / a, <u> the
    superficial velocity (the velocity component along the force averaged over the whole lattice,
    solid nodes counting zero). One colour fills the pores (no interface, no reaction); the run
    stops when <u> changes by less than rtol over check_every steps. Returns (kappa, <u>, steps)."""
    solid = np.asarray(solid, dtype=np.uint8)
    shape = solid.shape[::-1]
    a = [0.0, 0.0, 0.0]
    a[axis] = accel
    sim = core.Lbm(shape, solid=solid, rho_r0=(1 - solid).astype(np.float64), rho_p0=0.0, precision=precision,
                   tau=tau_from_viscosity(nu), sigma=0.0, beta=0.0, xi=0.0, accel=[tuple(a), tuple(a)],
                   species=False, device=device)
    prev, steps = None, 0
    while steps < max_steps:
        sim.step(check_every, reductions=False)
        steps += check_every
        u = float(sim.moments()["u"][axis].double().mean())
        if prev is not None and abs(u - prev) <= rtol * abs(u):
            break
        prev = u
    return nu * u / accel, u, steps


def reaction_setup(solid, da, theta_deg, kappa, block=64, seed=0, xi=1.0, sigma=0.3, beta=0.7, bo_p=0.01,
                   radius=None, accel=None):
    """Parameters of the paper's reaction runs for a mask: nucleation sites, a (from Bo_p, or given),
    nu and tau from Da. radius defaults to the pore radius 2 phi / (A/V) of the mask (the radius of
    a cylindrical pore with the mask's surface-to-pore-volume ratio)."""
    geo = geometry_properties(solid)
    r, sites = nucleation_sites(solid, block=block, seed=seed)
    area_r = int((nearest_solid_neighbors(solid) * r).sum())
    nz, ny, nx = np.asarray(solid).shape
    if radius is None:
        radius = 2.0 * geo["phi"] / geo["A_over_V"]
    a = acceleration_from_bond(bo_p, sigma, radius) if accel is None else accel
    nu = viscosity_from_damkohler(da, xi, area_r, nx, kappa, geo["V"], a)
    return dict(geometry=geo, reactive=r, sites=sites, area_r=area_r, radius=radius, accel=a, nu=nu,
                tau=tau_from_viscosity(nu), xi=xi, sigma=sigma, beta=beta, theta=math.radians(theta_deg), da=da)


def reaction_run(core, solid, setup, steps, precision="fp32", chunk=10000, device="cuda:0", log=None):
    """All-reactant start, paper mode (no species), nucleation sites, body force along x on both
    colours. Returns the per-step reductions (m^r, m^p, conversion) and the wall time."""
    solid = np.asarray(solid, dtype=np.uint8)
    shape = solid.shape[::-1]
    a = (setup["accel"], 0.0, 0.0)
    sim = core.Lbm(shape, solid=solid, theta=setup["theta"], reactive=setup["reactive"],
                   rho_r0=(1 - solid).astype(np.float64), rho_p0=0.0, precision=precision, tau=setup["tau"],
                   sigma=setup["sigma"], beta=setup["beta"], xi=setup["xi"], accel=[a, a], species=False,
                   device=device)
    reds = []
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        reds.append(sim.step(n, check=False))
        done += n
        if log:
            log("%d / %d steps, %.1f s" % (done, steps, time.perf_counter() - t0))
        if sim.last_status == core.LBM_ERR_NONFINITE:  # unstable parameters: stop, report it
            break
    return np.concatenate(reds), time.perf_counter() - t0


def _main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["permeability", "run", "sweep"])
    ap.add_argument("--das", default="0.1,1,10", help="sweep: Damkohler numbers")
    ap.add_argument("--thetas", default="15,30,60,90,150", help="sweep: contact angles (degrees)")
    ap.add_argument("--workload", default="bijel128")
    ap.add_argument("--da", type=float, default=1.0)
    ap.add_argument("--theta", type=float, default=60.0)
    ap.add_argument("--steps", type=int, default=50000)
    ap.add_argument("--kappa", type=float, default=None, help="permeability along x (else computed)")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--fit-from", type=int, default=10000)
    args = ap.parse_args()

    from paper_2608_15781_amd import core, inputs

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    w, solid, _, _, _ = inputs.workload_inputs(args.workload)
    if args.cmd == "permeability":
        out = dict(workload=args.workload, **geometry_properties(solid))
        for axis in range(3):
            kappa, u, n = permeability(core, solid, axis=axis)
            out["kappa_%s" % "xyz"[axis]] = kappa
            out["steps_%s" % "xyz"[axis]] = n
            log("axis %d: kappa %.5f after %d steps" % (axis, kappa, n))
        out["kappa_mean"] = (out["kappa_x"] + out["kappa_y"] + out["kappa_z"]) / 3
        out["eta"] = reactor_efficiency(out["kappa_mean"], out["A_over_V"])
        print(json.dumps(out), flush=True)
        return
    kappa = args.kappa
    if kappa is None:
        kappa, _, _ = permeability(core, solid, axis=0)
        log("kappa_x %.5f" % kappa)

    def one(da, theta):
        st = reaction_setup(solid, da, theta, kappa)
        log("Da %g theta %g: sites %d, A_r %d, a %.4e, nu %.4f, tau %.4f" % (
            da, theta, len(st["sites"]), st["area_r"], st["accel"], st["nu"], st["tau"]))
        red, wall = reaction_run(core, solid, st, args.steps, precision=args.precision, log=log)
        geo = st["geometry"]
        m_r, m_p, conv = red[:, 0], red[:, 1], red[:, 2]
        alpha, mean = effectiveness(m_r, conv, st["xi"], st["area_r"], geo["phi"], geo["V"])
        m_m = float(m_r[0] + m_p[0])
        fit = fit_alpha(m_r, m_m, st["xi"], st["area_r"], geo["phi"], geo["V"], t0=min(args.fit_from, len(m_r) - 1))
        return dict(da=da, theta_deg=theta, nu=st["nu"], tau=st["tau"], steps_run=len(m_r),
                    mflups=int((solid == 0).sum()) * len(m_r) / wall / 1e6, alpha_first=float(alpha[0]),
                    alpha_mean_final=float(mean[-1]), alpha_fit=fit, reactant_fraction_final=float(m_r[-1] / m_m),
                    nonfinite=int(red[:, 4].sum()))

    head = dict(workload=args.workload, steps=args.steps, precision=args.precision, kappa_x=kappa,
                fit_from=args.fit_from)
    if args.cmd == "run":
        print(json.dumps(dict(head, **one(args.da, args.theta))), flush=True)
    else:
        runs = [one(float(d), float(t)) for d in args.das.split(",") for t in args.thetas.split(",")]
        print(json.dumps(dict(head, runs=runs)), flush=True)


if __name__ == "__main__":
    _main()
