"""Reactor pipeline on the GPU: single-phase permeability of a slit against the plane-Poiseuille
closed form, and the paper's reaction set-up (nucleation sites, xi = 1, sigma = 0.3, paper mode
without species) against the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def core():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_15781_amd import core as c

    c.lib()
    return c


def test_slit_permeability_matches_plane_poiseuille(core):
    """Fluid layers z = 1..H between periodic solid layers z = 0: with halfway bounce-back the
    walls sit half a node outside the fluid, the mean fluid velocity is a H^2 / (12 nu), and the
    superficial (whole-lattice) permeability is phi H^2 / 12 with phi = H / nz."""
    from paper_2608_15781_amd import reactor

    nz, H = 18, 17
    solid = np.zeros((nz, 6, 8), np.uint8)
    solid[0] = 1
    for axis in (0, 1):
        kappa, u, steps = reactor.permeability(core, solid, axis=axis, accel=1e-6, nu=0.1, rtol=1e-9)
        expect = (H / nz) * H * H / 12.0
        print("slit axis %d: kappa %.6f closed form %.6f (%d steps)" % (axis, kappa, expect, steps), flush=True)
        assert abs(kappa / expect - 1) < 5e-3


def test_paper_reaction_setup_against_oracle(core, oracle_mod):
    """24^3 random-field mask with one nucleation site per 12^3 block, xi = 1 (full conversion at a
    site), sigma = 0.3, beta = 0.7, body force from Bo_p = 0.01, tau from Da = 1 (kappa taken as
    1), contact angle 60 deg, FP64, 150 steps: per-step m^r, m^p and conversion, and the fields,
    against the oracle; the effectiveness factor of the first step is 1 (all-reactant start)."""
    from paper_2608_15781_amd import inputs, reactor

    n = 24
    solid, _ = inputs.grf_mask((n, n, n), 8.0, 11)
    st = reactor.reaction_setup(solid, da=1.0, theta_deg=60.0, kappa=1.0, block=12, seed=4)
    assert len(st["sites"]) == 8 and st["area_r"] == 8
    a = (st["accel"], 0.0, 0.0)
    kw = dict(theta=st["theta"], reactive=st["reactive"], rho_r0=(1 - solid).astype(float), rho_p0=0.0,
              tau=st["tau"], sigma=st["sigma"], beta=st["beta"], xi=st["xi"], accel=[a, a], species=False)
    sim = core.Lbm((n, n, n), solid=solid, precision="fp64", **kw)
    ref = oracle_mod.Oracle((n, n, n), solid=solid, **kw)
    T = 150
    rg = sim.step(T)
    rr = ref.step(T)
    for j in (0, 1, 2):
        assert np.abs(rg[:, j] - rr[:, j]).max() <= 1e-10 * np.abs(rr[:, j]).max(), j
    m = sim.moments()
    mr = ref.moments()
    for key in ("rho_r", "rho_p", "rho_n", "u"):
        g = m[key].cpu().numpy()
        assert np.abs(g - mr[key]).max() <= 1e-10 * np.abs(mr[key]).max(), key
    geo = st["geometry"]
    alpha, mean = reactor.effectiveness(rg[:, 0], rg[:, 2], st["xi"], st["area_r"], geo["phi"], geo["V"])
    assert abs(alpha[0] - 1) < 1e-12
    print("paper set-up: tau %.4f a %.3e; alpha(0) %.6f, mean alpha over %d steps %.4f" %
          (st["tau"], st["accel"], alpha[0], T, mean[-1]), flush=True)


def test_paper_setup_gradient_against_oracle_duals(core, oracle_mod):
    """The adjoint on the paper's reaction set-up (paper mode: no species; nucleation sites with
    full conversion, xi = 1; sigma = 0.3) against the oracle's dual numbers: directional
    derivatives of L along two random per-node contact-angle perturbations and along a uniform
    one, 24^3, 120 FP64 steps with checkpoints every 40."""
    from paper_2608_15781_amd import autograd as ag
    from paper_2608_15781_amd import inputs, reactor

    n, T = 24, 120
    solid, _ = inputs.grf_mask((n, n, n), 8.0, 11)
    st = reactor.reaction_setup(solid, da=1.0, theta_deg=60.0, kappa=1.0, block=12, seed=4)
    a = (st["accel"], 0.0, 0.0)
    kw = dict(tau=st["tau"], sigma=st["sigma"], beta=st["beta"], accel=[a, a], species=False)
    theta = np.full(solid.shape, st["theta"])
    rng = np.random.default_rng(2)
    d1 = rng.normal(size=solid.shape) * (1 - solid)
    d2 = np.ones(solid.shape) * (1 - solid)
    L, dL = oracle_mod.grad((n, n, n), solid, theta, st["xi"], T, dtheta=[d1.ravel(), d2.ravel()],
                            dxi=[0.0, 0.0], reactive=st["reactive"], rho_r0=(1 - solid).astype(float), **kw)
    sim = core.Lbm((n, n, n), solid=solid, theta=theta, reactive=st["reactive"], rho_r0=(1 - solid).astype(float),
                   rho_p0=0.0, xi=st["xi"], precision="fp64", **kw)
    Lg, cps, final = ag.forward_states(sim, T, 40)
    gth, gxi, _ = ag.adjoint_gradients(sim, T, 40, cps, final)
    g = gth.cpu().numpy()
    ad = [float(g @ d1.ravel()), float(g @ d2.ravel())]
    print("paper set-up: L gpu %.12e oracle %.12e; dL adjoint %s oracle %s" % (Lg, L, ad, list(dL)), flush=True)
    assert abs(Lg - L) < 1e-10 * abs(L)
    for x, y in zip(ad, dL):
        assert abs(x - y) < 1e-8 * abs(y) + 1e-12, (x, y)


# The contact-angle x Damkohler sweep's extremes: angles 15 and 150 deg, and the relaxation times
# that Da = 0.1 and Da = 10 give on the 128^3 stand-in (tau 0.569 and 7.36).
SWEEP_TAU = {0.1: 0.569, 10.0: 7.36}


@pytest.mark.parametrize("theta_deg", [15.0, 150.0])
@pytest.mark.parametrize("da", [0.1, 10.0])
def test_sweep_slice_against_oracle(core, oracle_mod, theta_deg, da):
    """A two-angle x two-Da slice of the sweep pipeline (reaction_run, then the effectiveness
    factor, its running mean and the exponential fit) on a 24^3 mask with one nucleation site per
    12^3 block, xi = 1, sigma = 0.3, paper mode, FP64, 300 steps: the per-step m^r, m^p and
    conversion against the oracle within 1e-10, and the analysis of the GPU sums equal to that of
    the oracle's within 1e-10."""
    from paper_2608_15781_amd import inputs, reactor

    n, T = 24, 300
    solid, _ = inputs.grf_mask((n, n, n), 8.0, 13)
    st = reactor.reaction_setup(solid, da=da, theta_deg=theta_deg, kappa=1.0, block=12, seed=6)
    st["tau"] = SWEEP_TAU[da]
    print("sweep slice: theta %g deg, tau %.3f, %d sites" % (theta_deg, st["tau"], len(st["sites"])), flush=True)
    red, _ = reactor.reaction_run(core, solid, st, T, precision="fp64", chunk=100)
    a = (st["accel"], 0.0, 0.0)
    ref = oracle_mod.Oracle((n, n, n), solid=solid, theta=st["theta"], reactive=st["reactive"],
                            rho_r0=(1 - solid).astype(float), rho_p0=0.0, tau=st["tau"], sigma=st["sigma"],
                            beta=st["beta"], xi=st["xi"], accel=[a, a], species=False)
    rr = ref.step(T)
    assert red.shape[0] == T and red[:, 4].max() == 0
    for j in (0, 1, 2):
        assert np.abs(red[:, j] - rr[:, j]).max() <= 1e-10 * np.abs(rr[:, j]).max(), j
    assert rr[-1, 1] > 0  # gas was produced
    geo = st["geometry"]
    out = []
    for r in (red, rr):
        alpha, mean = reactor.effectiveness(r[:, 0], r[:, 2], st["xi"], st["area_r"], geo["phi"], geo["V"])
        fit = reactor.fit_alpha(r[:, 0], float(r[0, 0] + r[0, 1]), st["xi"], st["area_r"], geo["phi"], geo["V"],
                                t0=100)
        out.append((alpha, mean, fit))
    assert np.abs(out[0][0] - out[1][0]).max() <= 1e-10 * np.abs(out[1][0]).max()
    assert abs(out[0][1][-1] / out[1][1][-1] - 1) < 1e-10
    assert abs(out[0][2] / out[1][2] - 1) < 1e-10
    assert abs(out[1][0][0] - 1) < 1e-12  # all-reactant start
    print("sweep slice: alpha mean %.6f fit %.6f (oracle %.6f)" % (out[0][1][-1], out[0][2], out[1][2]), flush=True)


def test_sweep_angle_gradient_sign_against_difference_quotients(core):
    """The adjoint's sum of dL/dtheta over the wetting nodes at 60 deg (the direction of a uniform
    change of the coating's angle) against central difference quotients of uniform-angle runs, on
    the leading 32^3 corner of the 128^3 mask with the paper's set-up (Da = 1, one site per 16^3
    block), FP64, 300 steps: the quotients for eps = 1e-5 and 1e-6 rad agree with each other
    (converged at this horizon), and the adjoint agrees with them to 1e-5 in relative terms, sign
    included."""
    import math

    from paper_2608_15781_amd import autograd as ag
    from paper_2608_15781_amd import inputs, reactor

    n, T = 32, 300
    w, solid, _, _, _ = inputs.workload_inputs("bijel128", size=n)
    st = reactor.reaction_setup(solid, da=1.0, theta_deg=60.0, kappa=1.0, block=16, seed=3)
    a = (st["accel"], 0.0, 0.0)
    kw = dict(reactive=st["reactive"], rho_r0=(1 - solid).astype(float), rho_p0=0.0, xi=st["xi"], tau=st["tau"],
              sigma=st["sigma"], beta=st["beta"], accel=[a, a], species=False, precision="fp64")

    def L(theta):
        sim = core.Lbm((n, n, n), solid=solid, theta=np.full(solid.shape, theta), **kw)
        m0 = sim.state_sums()["mass_p"]
        sim.step(T, reductions=False)
        return sim.state_sums()["mass_p"] - m0

    sim = core.Lbm((n, n, n), solid=solid, theta=np.full(solid.shape, st["theta"]), **kw)
    L0, cps, final = ag.forward_states(sim, T, 50)
    gth, _, _ = ag.adjoint_gradients(sim, T, 50, cps, final)
    ad = float(gth.sum())
    th = math.radians(60.0)
    fd = {eps: (L(th + eps) - L(th - eps)) / (2 * eps) for eps in (1e-5, 1e-6)}
    print("angle gradient at 60 deg: L %.10e adjoint %.10e fd %s" % (L0, ad, fd), flush=True)
    assert abs(fd[1e-5] / fd[1e-6] - 1) < 1e-4
    assert ad * fd[1e-6] > 0
    assert abs(ad / fd[1e-6] - 1) < 1e-5
