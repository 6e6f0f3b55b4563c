"""Physics pins of the oracle: closed-form flows, the Laplace law, the imposed contact angle,
species diffusion, exact bookkeeping of mass and conversion, lattice symmetries, and the
dual-number gradient against finite differences."""
import numpy as np
import pytest
from scipy.optimize import brentq

from paper_2608_15781_amd import inputs


def test_poiseuille_profile(oracle_mod):
    """Body-force-driven channel between halfway bounce-back walls: parabolic profile with
    nu = c_s^2 (tau - 1/2) (eq. kinematic_viscosity); walls half-way between nodes."""
    ny = 34
    solid = np.zeros((1, ny, 1), np.uint8)
    solid[0, 0, 0] = solid[0, ny - 1, 0] = 1
    a = 1e-6
    for tau in (0.8, 1.0):
        nu = (tau - 0.5) / 3
        o = oracle_mod.Oracle((1, ny, 1), solid=solid, rho_r0=1.0, rho_p0=0.0, tau=tau, accel=[(a, 0, 0), (a, 0, 0)])
        o.step(12000)
        ux = o.moments()["u"][0, 0, :, 0]
        y = np.arange(1, ny - 1)
        exact = a / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)
        err = np.linalg.norm(ux[1:-1] - exact) / np.linalg.norm(exact)
        assert err < 5e-3, (tau, err)


def test_shear_wave_viscosity(oracle_mod):
    """u_y = U sin(kx) decays as exp(-nu k^2 t) with nu = (tau - 1/2)/3."""
    L = 64
    c, w, _ = oracle_mod.lattice()
    x = np.arange(L)
    k = 2 * np.pi / L
    U = 1e-4
    for tau in (0.6, 0.8, 1.2):
        o = oracle_mod.Oracle((L, 1, 1), rho_r0=1.0, rho_p0=0.0, tau=tau)
        fr = np.stack([oracle_mod.feq(1.0, [0, U * np.sin(k * xx), 0]) for xx in x], axis=1)
        o.set_state(fr, np.zeros_like(fr))
        o.step(100)
        a0 = o.moments()["u"][1, 0, 0, :] @ np.sin(k * x)
        o.step(400)
        a1 = o.moments()["u"][1, 0, 0, :] @ np.sin(k * x)
        nu_meas = -np.log(a1 / a0) / (k * k * 400)
        nu = (tau - 0.5) / 3
        assert abs(nu_meas / nu - 1) < 2e-3, (tau, nu_meas, nu)


def test_laplace_law_static_droplet(oracle_mod):
    """Static droplet, 32^3 periodic, R = 8, tau = 1, sigma = 0.01, beta = 0.7, 500 steps:
    pressure jump c_s^2 (rho_in - rho_out) equals 2 sigma / R (CSF force of
    eq. continuum_surface_force with the curvature of eq. interface_curvature), and each
    colour's mass is conserved exactly."""
    n = 32
    rr0, rp0 = inputs.droplet((n, n, n), 8.0, centre=(15.5, 15.5, 15.5))
    o = oracle_mod.Oracle((n, n, n), rho_r0=rr0, rho_p0=rp0, tau=1.0, sigma=0.01, beta=0.7)
    s = o.step(500)
    assert abs(s[-1, 0] / s[0, 0] - 1) < 1e-12 and abs(s[-1, 1] / s[0, 1] - 1) < 1e-12
    m = o.moments()
    rm = m["rho_r"] + m["rho_p"]
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    r = np.sqrt((x - 15.5) ** 2 + (y - 15.5) ** 2 + (z - 15.5) ** 2)
    reff = (3 * ((1 + m["rho_n"]) / 2).sum() / (4 * np.pi)) ** (1 / 3)
    dp = (rm[r < reff - 3].mean() - rm[r > reff + 3].mean()) / 3
    assert dp > 0
    assert abs(dp / (2 * 0.01 / reff) - 1) < 0.10
    # the drop stays put and round: red centre of mass at the centre
    red = (1 + m["rho_n"]) / 2
    for coord in (x, y, z):
        assert abs((red * coord).sum() / red.sum() - 15.5) < 1e-6


def _cap_angle(rn, nx, nz):
    """Contact angle of a 2D cap from its area and apex height (circular-arc geometry)."""
    area = ((1 + rn[1:nz - 2]) / 2).sum()
    col = (rn[:, nx // 2] + rn[:, nx // 2 - 1]) / 2
    zt = None
    for zz in range(1, nz - 3):
        if col[zz] > 0 and col[zz + 1] <= 0:
            zt = zz + col[zz] / (col[zz] - col[zz + 1])
            break
    h = zt - 0.5
    f = lambda th: (th - np.sin(th) * np.cos(th)) / (1 - np.cos(th)) ** 2 - area / h ** 2
    return np.degrees(brentq(f, 1e-3, np.pi - 1e-3))


@pytest.mark.parametrize("theta_deg", [60.0, 90.0, 120.0])
def test_contact_angle_flat_wall(oracle_mod, theta_deg):
    """Akai wetting (eq. realigned_normal_vectors) on a flat wall: a red cap relaxes to the
    imposed angle, measured through the red colour. Quasi-2D (ny = 1), wall three nodes thick
    so that the colour extrapolated into it only sees the cap's side."""
    nx, nz = 100, 42
    solid = np.zeros((nz, 1, nx), np.uint8)
    solid[0] = solid[nz - 1] = solid[nz - 2] = 1
    z, x = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    r = np.sqrt((x - nx / 2 + 0.5) ** 2 + (z - 0.5) ** 2)
    red = ((r < 14) & (solid[:, 0] == 0)).astype(float)[:, None, :]
    o = oracle_mod.Oracle((nx, 1, nz), solid=solid, theta=np.deg2rad(theta_deg), rho_r0=red, rho_p0=1 - red,
                          tau=1.0, sigma=0.01, beta=0.7)
    o.step(6000)
    th = _cap_angle(o.moments()["rho_n"][:, 0, :], nx, nz)
    assert abs(th - theta_deg) < 5.0, th


def _segment_cap(nx, nz, area, theta_deg):
    """Red circular segment of the given area whose arc meets the wall z = 0.5 at theta_deg
    (through red), centred in x; walls at z = 0 and z = nz - 2, nz - 1 (three nodes thick with
    the periodic image)."""
    th = np.radians(theta_deg)
    R = np.sqrt(area / (th - np.sin(th) * np.cos(th)))
    zc = 0.5 - R * np.cos(th)
    z, x = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    red = (np.sqrt((x - nx / 2 + 0.5) ** 2 + (z - zc) ** 2) < R) & (z >= 1) & (z <= nz - 3)
    solid = np.zeros((nz, 1, nx), np.uint8)
    solid[0] = solid[nz - 1] = solid[nz - 2] = 1
    return solid, red.astype(float)[:, None, :]


def _circle_angle(rn, zmin):
    """Contact angle through red of a cap on the wall z = 0.5: circle fit (algebraic least squares)
    to the rho^N = 0 crossings along rows and columns at z >= zmin, then cos(theta) = -(z_c - 0.5)/R."""
    nz, nx = rn.shape
    xs, zs = [], []
    for x in range(nx):
        for z in range(1, nz - 3):
            a, b = rn[z, x], rn[z + 1, x]
            if (a > 0) != (b > 0) and z + a / (a - b) >= zmin:
                xs.append(x); zs.append(z + a / (a - b))
    for z in range(int(np.ceil(zmin)), nz - 2):
        for x in range(nx):
            a, b = rn[z, x], rn[z, (x + 1) % nx]
            if (a > 0) != (b > 0):
                xs.append(x + a / (a - b)); zs.append(z)
    x, z = np.array(xs, float), np.array(zs, float)
    sol = np.linalg.lstsq(np.stack([x, z, np.ones_like(x)], 1), x * x + z * z, rcond=None)[0]
    xc, zc = sol[0] / 2, sol[1] / 2
    R = np.sqrt(sol[2] + xc * xc + zc * zc)
    return float(np.degrees(np.arccos(np.clip(-(zc - 0.5) / R, -1.0, 1.0))))


# Caps at the sweep's extreme angles. Started 10 to 25 degrees away from the imposed angle, each
# must move toward it and end within 5 degrees. The low-angle caps are wide and flat (large x
# extent, apex height 11-15 nodes); tau = 0.6 and sigma = 0.06 make the contact lines relax within
# a few thousand steps (with tau = 1, sigma = 0.01 a 15 degree cap still spreads after 10^4 steps).
# Measured: 15 deg from 25 -> 17.9 after 8000 steps (15.7 when started at 15), 30 from 50 -> 30.6,
# 150 from 125 -> 152.2. The deviation of the static angle is first order in 1/R (at tau = 1,
# sigma = 0.01, 150 deg: 12.6 deg at R = 10, 5.6 at R = 20, 3.7 at R = 30).
EXTREME_CAPS = {15.0: dict(nx=240, nz=42, area=1200.0, start=25.0, steps=8000, zmin=2.0),
                30.0: dict(nx=200, nz=42, area=1200.0, start=50.0, steps=4000, zmin=3.5),
                150.0: dict(nx=100, nz=42, area=308.0, start=125.0, steps=4000, zmin=3.5)}


@pytest.mark.parametrize("theta_deg", sorted(EXTREME_CAPS))
def test_contact_angle_extreme_angles(oracle_mod, theta_deg):
    """Akai wetting (eq. realigned_normal_vectors) at the sweep's extreme contact angles: a quasi-2D
    red cap started away from the imposed angle relaxes to within 5 degrees of it, measured
    through red by a circle fit of the interface away from the wall."""
    c = EXTREME_CAPS[theta_deg]
    solid, red = _segment_cap(c["nx"], c["nz"], c["area"], c["start"])
    o = oracle_mod.Oracle((c["nx"], 1, c["nz"]), solid=solid, theta=np.deg2rad(theta_deg), rho_r0=red,
                          rho_p0=(1 - solid) - red, tau=0.6, sigma=0.06, beta=0.7)
    th0 = _circle_angle(o.moments()["rho_n"][:, 0, :], c["zmin"])
    o.step(c["steps"])
    th = _circle_angle(o.moments()["rho_n"][:, 0, :], c["zmin"])
    print("cap %g deg: started at %.2f, %.2f after %d steps" % (theta_deg, th0, th, c["steps"]))
    assert abs(th - theta_deg) < 5.0, th
    assert abs(th0 - theta_deg) - abs(th - theta_deg) > 5.0, (th0, th)  # it moved toward the angle


def test_akai_cone_does_not_set_the_contact_angle(oracle_mod):
    """The realignment keeps n inside a cone sin(theta') < 1e-2 around +-n_s (the rotation plane is
    undefined there). That cone is a guard against rounding, not part of the wetting physics: caps at
    15 deg (the interface nearest to parallel with the wall) and at 150 deg give the same contact
    angle, to 0.01 deg, with the cone, with a cone ten times narrower and with none, and the colour
    fields differ by less than 1e-5 (measured: 1.2e-6 and 4e-9 at 15 deg, where a few nodes enter
    the cone for a while; bitwise equal at 150 deg). So the angles pinned above do not depend on
    the cone's size."""
    runs = [(15.0, dict(nx=240, nz=42, area=1200.0, start=15.0, steps=1500, zmin=2.0)),
            (150.0, dict(nx=100, nz=42, area=308.0, start=125.0, steps=1500, zmin=3.5))]
    try:
        for theta_deg, c in runs:
            solid, red = _segment_cap(c["nx"], c["nz"], c["area"], c["start"])
            out = []
            for cone in (1e-2, 1e-3, 0.0):
                oracle_mod.set_akai_cone(cone)
                o = oracle_mod.Oracle((c["nx"], 1, c["nz"]), solid=solid, theta=np.deg2rad(theta_deg), rho_r0=red,
                                      rho_p0=(1 - solid) - red, tau=0.6, sigma=0.06, beta=0.7)
                o.step(c["steps"])
                rn = o.moments()["rho_n"]
                out.append((rn, _circle_angle(rn[:, 0, :], c["zmin"])))
            for rn, th in out[1:]:
                print("cone check %g deg: angle %.4f vs %.4f, max |d rho^N| %.2e" % (
                    theta_deg, th, out[0][1], np.abs(rn - out[0][0]).max()))
                assert abs(th - out[0][1]) < 0.01
                assert np.abs(rn - out[0][0]).max() < 1e-5
    finally:
        oracle_mod.set_akai_cone(1e-2)


def test_species_decay_matches_fourier_evolution(oracle_mod):
    """D3Q7 species at rest (u = 0): C = 1 + A sin(kx) evolves exactly by the 7x7 one-step
    Fourier matrix of pull + BGK, and decays like exp(-D k^2 t), D = (tau_C - 1/2)/4."""
    L, A, tau_c, T = 32, 0.1, 0.9, 300
    x = np.arange(L)
    k = 2 * np.pi / L
    c0 = 1 + A * np.sin(k * x)
    o = oracle_mod.Oracle((L, 1, 1), rho_r0=1.0, rho_p0=0.0, c0=c0, species=True, tau_c=tau_c)
    o.step(T)
    C = o.moments()["c"][0, 0, :]
    # Independent linear evolution of the e^{ikx} mode with the D3Q7 velocities along x.
    cx = np.array([1, -1, 0, 0, 0, 0, 0])
    w = np.array([1, 1, 1, 1, 1, 1, 2]) / 8.0
    Mc = np.eye(7) - (np.eye(7) - np.outer(w, np.ones(7))) / tau_c
    P = np.diag(np.exp(-1j * k * cx))
    g0 = w * (A / 2j)                   # coefficient of e^{ikx} in w_i C_0(x)
    gt = np.linalg.matrix_power(P @ Mc, T) @ (P @ g0)
    expect = 1 + 2 * np.real(gt.sum() * np.exp(1j * k * x))
    assert np.abs(C - expect).max() < 1e-13
    D = (tau_c - 0.5) / 4
    amp = (C - 1) @ np.sin(k * x) / (L / 2)
    assert abs(amp / (A * np.exp(-D * k * k * T)) - 1) < 0.02


def test_species_inlet_and_outflow_diffusion(oracle_mod):
    """Species at rest entering through the inlet plane (C = C_in at x = 0) into C = 0, with the
    zero-gradient outflow plane at x = L-1 (the outflow node takes its own S_1): C follows the series
    solution of C_t = D C_xx with C(0) = 1 and C_x(L - 1/2) = 0, to first order in the lattice
    spacing (the error halves when L doubles at fixed D t / L^2). A Dirichlet point half a node
    off, or the outflow condition at L - 1 or L, fits worse."""
    tau_c = 0.9
    D = (tau_c - 0.5) / 4

    def err(L, T, x0=0.0, Lb=None):
        o = oracle_mod.Oracle((L, 1, 1), rho_r0=1.0, rho_p0=0.0, c0=np.zeros(L), species=True, x_open=True,
                              tau_c=tau_c, c_in=1.0)
        o.step(T)
        C = o.moments()["c"][0, 0, :]
        x = np.arange(L, dtype=float)
        Lb = L - 0.5 if Lb is None else Lb
        k = np.arange(4000)
        lam = (2 * k + 1) * np.pi / (2 * (Lb - x0))
        ser = 1 - (4 / ((2 * k + 1) * np.pi) * np.sin(np.outer(x - x0, lam)) * np.exp(-D * lam ** 2 * T)).sum(1)
        assert C[0] == 1.0
        return np.abs(C[1:] - ser[1:]).max()

    e40, e80 = err(40, 6000), err(80, 24000)
    assert e40 < 6e-3 and e80 < 3e-3 and e80 < 0.6 * e40, (e40, e80)
    for x0, Lb in ((0.0, 79.0), (0.0, 80.0), (0.5, 79.5), (-0.5, 79.5)):
        assert err(80, 24000, x0, Lb) > 1.4 * e80, (x0, Lb)


def test_solid_normal_flat_walls_and_sphere(oracle_mod):
    """E8 solid normal (eq. normal_vector_solid) at wetting nodes: exactly the wall normal,
    pointing into the solid, next to a flat wall of each orientation; within the staircase error
    of the radial direction next to a voxelised sphere."""
    n = 16
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    for axis, coord in enumerate((x, y, z)):
        solid = (coord < 3).astype(np.uint8)
        g = oracle_mod.Oracle((n, n, n), solid=solid).geometry()
        ok = g["ns_ok"].astype(bool) & (solid.ravel() == 0)
        lo = coord.ravel()[ok] == 3      # solid below: normal points to -axis
        hi = coord.ravel()[ok] == n - 1  # periodic image of the solid above
        assert lo.sum() == n * n and hi.sum() == n * n and (lo | hi).all()
        e = np.zeros(3)
        e[axis] = 1.0
        assert np.abs(g["ns"][:, ok][:, lo] + e[:, None]).max() < 1e-15
        assert np.abs(g["ns"][:, ok][:, hi] - e[:, None]).max() < 1e-15
    c = 7.5
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    solid = (r < 4.5).astype(np.uint8)
    g = oracle_mod.Oracle((n, n, n), solid=solid).geometry()
    ok = g["ns_ok"].astype(bool) & (solid.ravel() == 0)
    d = np.stack([(c - a).ravel()[ok] for a in (x, y, z)])
    d /= np.linalg.norm(d, axis=0)
    ang = np.degrees(np.arccos(np.clip((g["ns"][:, ok] * d).sum(0), -1, 1)))
    assert ok.sum() > 300 and ang.mean() < 10 and ang.max() < 20, (ang.mean(), ang.max())


def _grf_case(n=16, wavelength=8.0, seed=7):
    solid, _ = inputs.grf_mask((n, n, n), wavelength, seed)
    return solid


def test_mass_and_conversion_bookkeeping(oracle_mod):
    """With the wall reaction: m^r + m^p is constant and m^p(t+1) - m^p(t) = conversion(t)
    (eq. total_mass, eq. production_rate); in the species mode the species loses the same."""
    n = 16
    solid = _grf_case(n)
    rr0 = (1 - solid).astype(float)
    for species in (False, True):
        o = oracle_mod.Oracle((n, n, n), solid=solid, theta=np.deg2rad(60), rho_r0=rr0, rho_p0=0.0, xi=0.05,
                              tau=0.8, sigma=0.01, accel=[(1e-5, 0, 0), (1e-5, 0, 0)], species=species, tau_c=0.9)
        s = o.step(60)
        tot = s[:, 0] + s[:, 1]
        assert np.abs(tot / tot[0] - 1).max() < 1e-12
        assert np.abs(np.diff(s[:, 1]) - s[:-1, 2]).max() < 1e-11
        assert s[:, 2].min() > 0
        if species:
            assert np.abs(np.diff(s[:, 3]) + s[:-1, 2]).max() < 1e-11


def test_initial_conversion_equals_xi_times_reactive_area(oracle_mod):
    """All-reactant start: conversion(0) = xi * A_r (eq. production_rate with rho^r = 1, i.e. an
    effectiveness factor of exactly one, eq. effectiveness_factor)."""
    n = 16
    solid = _grf_case(n)
    o = oracle_mod.Oracle((n, n, n), solid=solid, rho_r0=(1 - solid).astype(float), rho_p0=0.0, xi=0.01, tau=0.8)
    geo = o.geometry()
    area_r = (geo["react"].astype(float) * geo["nn"]).sum()
    assert area_r > 0
    s = o.step(1)
    assert abs(s[0, 2] / (0.01 * area_r) - 1) < 1e-13


def test_uniform_flow_is_a_fixed_point(oracle_mod):
    """A uniform equilibrium in motion, without force, is left unchanged."""
    n = 6
    o = oracle_mod.Oracle((n, n, n), rho_r0=0.7, rho_p0=0.3, tau=0.7)
    u = np.array([0.02, -0.01, 0.03])
    fr = np.repeat(oracle_mod.feq(0.7, u)[:, None], n ** 3, axis=1)
    fp = np.repeat(oracle_mod.feq(0.3, u)[:, None], n ** 3, axis=1)
    o.set_state(fr, fp)
    o.step(5)
    sr, sp, _ = o.get_state()
    assert np.abs(sr - fr).max() < 1e-15 and np.abs(sp - fp).max() < 1e-15


def _sym_case(n=14):
    solid = _grf_case(n, wavelength=7.0, seed=11)
    rng = np.random.default_rng(12)
    rr0 = (1 - solid) * (rng.uniform(size=solid.shape) > 0.5)
    rp0 = (1 - solid) - rr0
    theta = np.deg2rad(rng.uniform(40, 140, solid.shape))
    return solid, theta, rr0.astype(float), rp0.astype(float)


def _sym_run(oracle_mod, solid, theta, rr0, rp0, accel, steps=12):
    nz, ny, nx = solid.shape
    o = oracle_mod.Oracle((nx, ny, nz), solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, xi=0.02, tau=0.7,
                          sigma=0.02, accel=accel, species=True, tau_c=0.8)
    o.step(steps)
    return o.moments()


def test_mirror_and_transpose_equivariance(oracle_mod):
    """Mirroring x, or swapping x and y, of geometry and initial state mirrors or swaps the
    result (catches wrong lattice indices anywhere in the step)."""
    solid, theta, rr0, rp0 = _sym_case()
    acc = [(2e-4, 1e-4, -5e-5), (2e-4, 1e-4, -5e-5)]
    ref = _sym_run(oracle_mod, solid, theta, rr0, rp0, acc)
    # mirror x -> n-1-x (the lattice is closed under it)
    f = lambda a: np.ascontiguousarray(a[..., ::-1])
    acc_m = [(-a[0], a[1], a[2]) for a in acc]
    mir = _sym_run(oracle_mod, f(solid), f(theta), f(rr0), f(rp0), acc_m)
    for key in ("rho_r", "rho_p", "c"):
        assert np.abs(mir[key] - f(ref[key])).max() < 1e-12, key
    assert np.abs(mir["u"][0] + f(ref["u"][0])).max() < 1e-12
    assert np.abs(mir["u"][1:] - f(ref["u"][1:])).max() < 1e-12
    # swap x <-> y
    t = lambda a: np.ascontiguousarray(np.swapaxes(a, -1, -2))
    acc_t = [(a[1], a[0], a[2]) for a in acc]
    tr = _sym_run(oracle_mod, t(solid), t(theta), t(rr0), t(rp0), acc_t)
    for key in ("rho_r", "rho_p", "c"):
        assert np.abs(tr[key] - t(ref[key])).max() < 1e-12, key
    assert np.abs(tr["u"][0] - t(ref["u"][1])).max() < 1e-12
    assert np.abs(tr["u"][1] - t(ref["u"][0])).max() < 1e-12
    assert np.abs(tr["u"][2] - t(ref["u"][2])).max() < 1e-12


def test_dual_gradient_matches_finite_differences(oracle_mod):
    """Forward-mode duals through the whole step agree with central differences of the plain
    FP64 oracle, for the reaction rate and for a contact-angle direction."""
    n = 10
    solid = _grf_case(n, wavelength=6.0, seed=21)
    rng = np.random.default_rng(22)
    theta = np.deg2rad(rng.uniform(70, 110, solid.shape))
    dth = rng.normal(size=solid.shape) * (1 - solid)
    kw = dict(tau=0.8, sigma=0.01, accel=[(1e-5, 0, 0), (1e-5, 0, 0)], species=True, tau_c=0.9, x_open=True)
    rr0 = (1 - solid).astype(float)
    xi, steps = 0.02, 25
    L, dL = oracle_mod.grad((n, n, n), solid, theta, xi, steps, dtheta=[dth.ravel(), np.zeros(n ** 3)],
                            dxi=[0.0, 1.0], rho_r0=rr0, **kw)

    def run(th, x):
        o = oracle_mod.Oracle((n, n, n), solid=solid, theta=th, rho_r0=rr0, rho_p0=0.0, xi=x, **kw)
        return o.step(steps)[:, 2].sum()

    assert abs(run(theta, xi) - L) < 1e-12 * L
    h = 1e-4
    fd_th = (run(theta + h * dth, xi) - run(theta - h * dth, xi)) / (2 * h)
    fd_xi = (run(theta, xi + 1e-6) - run(theta, xi - 1e-6)) / 2e-6
    assert abs(dL[1] / fd_xi - 1) < 1e-6
    assert abs(dL[0] - fd_th) < 1e-5 * abs(dL[0]) + 1e-12
