"""GPU adjoint (lbm_adjoint_seed / lbm_adjoint_step) and the checkpointed autograd function.

FP64 storage unless stated. Pins, independent of the adjoint code:
  * one step: <lambda_t, dS> against central differences of the forward step (FP64 library);
    theta and xi parts likewise;
  * many steps: directional derivatives of L = m^p(T) - m^p(0) against the oracle's forward-mode
    dual numbers (exact derivatives of the FP64 reference step);
  * checkpoint-and-recompute gives the same gradient bit for bit as keeping every level;
  * per-node contact-angle derivatives on sampled wetting nodes against central differences
    (eps = 1e-4 rad) of the FP64 forward run;
  * the FP32-arithmetic adjoint (FP32, FP16 and BF16 storage) against the FP64 adjoint.
"""
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


def _case(n, seed, wavelength=7.0):
    from paper_2608_15781_amd import inputs

    solid, _ = inputs.grf_mask((n, n, n), wavelength, seed)
    rng = np.random.default_rng(seed + 1)
    theta = np.deg2rad(rng.uniform(60, 120, solid.shape))
    rr0 = (1 - solid).astype(float)
    return solid, theta, rr0, np.zeros_like(rr0)


KW = dict(tau=0.7, sigma=0.02, beta=0.7, accel=[(2e-5, 0, 0), (2e-5, 0, 0)], species=True, x_open=True)


def _sim(core, n, solid, theta, rr0, rp0, xi):
    return core.Lbm((n, n, n), solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, xi=xi, precision="fp64",
                    tau_species=0.8, **KW)


def _flat(sim, buf):
    import torch

    f, a, g = sim.state_parts(buf)
    return torch.cat([f, a, g], 0)


def _unflat(sim, vec, like):
    buf = like.clone()
    f, a, g = sim.state_parts(buf)
    f.copy_(vec[:19])
    a.copy_(vec[19:23])
    g.copy_(vec[23:30])
    return buf


def test_adjoint_one_step_against_finite_differences(core):
    import torch

    n, xi = 14, 0.05
    solid, theta, rr0, rp0 = _case(n, 31)
    sim = _sim(core, n, solid, theta, rr0, rp0, xi)
    sim.step(12)
    S = sim.get_state()
    NF = sim.nfluid
    gen = torch.Generator(device="cuda:0").manual_seed(5)
    lam1 = sim.new_adjoint()
    lam1[:, :NF] = torch.randn(30, NF, dtype=torch.float64, device="cuda:0", generator=gen)
    dS = torch.randn(30, NF, dtype=torch.float64, device="cuda:0", generator=gen)
    dS[:19] *= 1e-2
    dS[19] *= 1e-2
    # the colour scalar e holds -b or +a by its sign: keep the perturbed value on the same side
    dS[19][_flat(sim, S)[19].abs() < 1e-6] = 0
    dS[20:23] *= 1e-3
    dS[23:] *= 1e-2
    lam0 = sim.new_adjoint()
    scratch = sim.new_scratch()
    gth = torch.zeros(sim.N, dtype=torch.float64, device="cuda:0")
    gxi = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    sim.adjoint_step(S, lam1, lam0, scratch, gth, gxi)
    torch.cuda.synchronize()
    x0 = _flat(sim, S).clone()

    def F(buf, model=sim):
        model.set_state(buf, 12)
        model.step(1, reductions=False)
        return float((lam1[:, :NF] * _flat(model, model.get_state())).sum())

    h = 1e-6
    fd = (F(_unflat(sim, x0 + h * dS, S)) - F(_unflat(sim, x0 - h * dS, S))) / (2 * h)
    ad = float((lam0[:, :NF] * dS).sum())
    print("one-step state: adjoint %.12e fd %.12e" % (ad, fd), flush=True)
    assert abs(ad - fd) < 1e-6 * abs(fd)
    # contact angle and reaction rate
    rng = np.random.default_rng(7)
    dth = rng.normal(size=solid.shape) * (1 - solid)
    ht = 1e-6
    Fp = F(S, _sim(core, n, solid, theta + ht * dth, rr0, rp0, xi))
    Fm = F(S, _sim(core, n, solid, theta - ht * dth, rr0, rp0, xi))
    fd_th = (Fp - Fm) / (2 * ht)
    ad_th = float((gth.cpu().numpy() * dth.ravel()).sum())
    print("one-step theta: adjoint %.12e fd %.12e" % (ad_th, fd_th), flush=True)
    assert abs(ad_th - fd_th) < 1e-6 * abs(fd_th)
    hx = 1e-7
    fd_xi = (F(S, _sim(core, n, solid, theta, rr0, rp0, xi + hx)) -
             F(S, _sim(core, n, solid, theta, rr0, rp0, xi - hx))) / (2 * hx)
    print("one-step xi: adjoint %.12e fd %.12e" % (float(gxi[0]), fd_xi), flush=True)
    assert abs(float(gxi[0]) - fd_xi) < 1e-6 * abs(fd_xi)


def test_gradient_matches_oracle_duals_and_checkpointing(core, oracle_mod):
    import torch

    from paper_2608_15781_amd import autograd as ag

    n, xi, T = 12, 0.05, 30
    solid, theta, rr0, rp0 = _case(n, 41, wavelength=6.0)
    rng = np.random.default_rng(3)
    d1 = rng.normal(size=solid.shape) * (1 - solid)
    d2 = rng.normal(size=solid.shape) * (1 - solid)
    L, dL = oracle_mod.grad((n, n, n), solid, theta, xi, T, dtheta=[d1.ravel(), d2.ravel(), np.zeros(n ** 3)],
                            dxi=[0.0, 0.0, 1.0], rho_r0=rr0, tau_c=0.8, **KW)
    sim = _sim(core, n, solid, theta, rr0, rp0, xi)
    Lg, cps, final = ag.forward_states(sim, T, T)
    gth, gxi, _ = ag.adjoint_gradients(sim, T, T, cps, final)
    g = gth.cpu().numpy()
    ad = [float(g @ d1.ravel()), float(g @ d2.ravel()), float(gxi)]
    print("L gpu %.12e oracle %.12e" % (Lg, L), flush=True)
    print("dL adjoint", ad, "oracle duals", list(dL), flush=True)
    assert abs(Lg - L) < 1e-10 * abs(L)
    for a, b in zip(ad, dL):
        assert abs(a - b) < 1e-8 * abs(b) + 1e-14, (a, b)
    # checkpoint-and-recompute (every 7 steps) reproduces the gradient exactly, and so does
    # recomputing the level fields inside each adjoint step instead of keeping them
    sim2 = _sim(core, n, solid, theta, rr0, rp0, xi)
    L2, cps2, final2 = ag.forward_states(sim2, T, 7)
    gth2, gxi2, _ = ag.adjoint_gradients(sim2, T, 7, cps2, final2)
    assert torch.equal(gth2, gth) and float(gxi2) == float(gxi)
    gth3, gxi3, _ = ag.adjoint_gradients(sim2, T, 7, cps2, final2, keep_fields=False)
    assert torch.equal(gth3, gth) and float(gxi3) == float(gxi)
    # keeping every level in the forward pass instead: the same gradient bit for bit, the same
    # final state, and L (read from the end states' product mass) equal to the conversion sum
    sim3 = _sim(core, n, solid, theta, rr0, rp0, xi)
    L3, levels, final3 = ag.forward_keep_all(sim3, T)
    gth4, gxi4, _ = ag.adjoint_gradients_keep_all(sim3, levels, final3)
    assert torch.equal(gth4, gth) and float(gxi4) == float(gxi)
    assert sim3.steps_done == T
    for a_, b_ in zip(sim3.state_parts(final3), sim.state_parts(final)):
        assert torch.equal(a_, b_)
    assert abs(L3 - Lg) <= 1e-11 * abs(Lg), (L3, Lg)
    # the autograd function
    th_t = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    xi_t = torch.tensor(xi, dtype=torch.float64, requires_grad=True)
    problem = dict(shape=(n, n, n), solid=solid, rho_r0=rr0, rho_p0=rp0, precision="fp64", steps=T, checkpoint=7,
                   params=dict(tau_species=0.8, **KW))
    Lt = ag.gas_production(th_t, xi_t, problem)
    Lt.backward()
    assert abs(float(Lt.detach()) - Lg) <= 1e-12 * abs(Lg)
    assert np.array_equal(th_t.grad.numpy().ravel(), g)
    assert float(xi_t.grad) == float(gxi)
    th_k = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    xi_k = torch.tensor(xi, dtype=torch.float64, requires_grad=True)
    Lk = ag.gas_production(th_k, xi_k, dict(problem, checkpoint=0))
    Lk.backward()
    assert np.array_equal(th_k.grad.numpy().ravel(), g) and float(xi_k.grad) == float(gxi)


@pytest.mark.parametrize("nx", [1, 2])
def test_thin_x_gradient_against_oracle_duals(core, oracle_mod, nx):
    """Lattices one and two nodes wide in x with scattered solids: the adjoint passes take the
    pull-source ids from a row neighbour's or a y/z partner's fluid id, which must fall back to
    the id map where a row wraps onto the node itself or onto its other neighbour."""
    from paper_2608_15781_amd import autograd as ag

    shape, xi, T = (nx, 9, 8), 0.05, 15
    rng = np.random.default_rng(60 + nx)
    solid = (rng.uniform(size=(8, 9, nx)) < 0.3).astype(np.uint8)
    theta = np.deg2rad(rng.uniform(60, 120, solid.shape))
    rr0 = ((1 - solid) * (rng.uniform(size=solid.shape) > 0.5)).astype(float)
    rp0 = (1 - solid) - rr0
    d1 = rng.normal(size=solid.shape) * (1 - solid)
    kw = dict(KW, x_open=nx >= 2)
    L, dL = oracle_mod.grad(shape, solid, theta, xi, T, dtheta=[d1.ravel(), np.zeros(solid.size)], dxi=[0.0, 1.0],
                            rho_r0=rr0, rho_p0=rp0, tau_c=0.8, **kw)
    sim = core.Lbm(shape, solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, xi=xi, precision="fp64",
                   tau_species=0.8, **kw)
    Lg, cps, final = ag.forward_states(sim, T, 5)
    gth, gxi, _ = ag.adjoint_gradients(sim, T, 5, cps, final)
    ad = [float(gth.cpu().numpy() @ d1.ravel()), float(gxi)]
    print("nx=%d L gpu %.12e oracle %.12e; dL adjoint %s oracle duals %s" % (nx, Lg, L, ad, list(dL)), flush=True)
    assert abs(Lg - L) < 1e-10 * abs(L)
    for a, b in zip(ad, dL):
        assert abs(a - b) < 1e-8 * abs(b) + 1e-14, (a, b)


def test_contact_angle_gradient_finite_differences_on_wall_nodes(core):
    from paper_2608_15781_amd import autograd as ag

    n, xi, T = 18, 0.05, 40
    solid, theta, rr0, rp0 = _case(n, 51)
    sim = _sim(core, n, solid, theta, rr0, rp0, xi)
    L0, cps, final = ag.forward_states(sim, T, 10)
    gth, gxi, _ = ag.adjoint_gradients(sim, T, 10, cps, final)
    g = gth.cpu().numpy()
    order = np.argsort(-np.abs(g))
    rng = np.random.default_rng(9)
    wet = np.flatnonzero(g != 0)
    picks = list(order[:4]) + list(rng.choice(wet, 4, replace=False))
    eps = 1e-4
    for k in picks:
        tp = theta.ravel().copy()
        tm = theta.ravel().copy()
        tp[k] += eps
        tm[k] -= eps
        Lp = float(_sim(core, n, solid, tp.reshape(solid.shape), rr0, rp0, xi).step(T)[:, 2].sum())
        Lm = float(_sim(core, n, solid, tm.reshape(solid.shape), rr0, rp0, xi).step(T)[:, 2].sum())
        fd = (Lp - Lm) / (2 * eps)
        print("node %d adjoint %.10e fd %.10e" % (k, g[k], fd), flush=True)
        assert abs(g[k] - fd) < 1e-5 * abs(g[order[0]]) + 1e-6 * abs(fd), (k, g[k], fd)


def _adjoint96():
    from paper_2608_15781_amd import inputs

    w, solid, theta, rr0, rp0 = inputs.workload_inputs("adjoint96")
    kw = dict(tau=w["tau"], sigma=w["sigma"], beta=w["beta"], accel=[(w["accel"], 0, 0)] * 2, species=w["species"],
              x_open=w["x_open"])
    return w, solid, theta, rr0, rp0, kw


def test_adjoint96_gradient_against_finite_differences(core):
    """The 96^3 adjoint workload at full size (200 steps, checkpoint every 20), FP64: dL/dtheta on
    32 wetting nodes (the 16 largest |dL/dtheta| and 16 drawn at random) against central
    differences, and dL/dxi against a central difference in xi.

    L is strongly nonlinear in theta at the nodes of largest gradient: there the central quotient
    with eps = 1e-4 rad is still far from its limit (13.6 at eps -> 0, 18.2 at 1e-4, 11.6 at 1e-3
    on the largest node), so the comparison uses eps = 1e-7, where the quotient has converged to
    about 1e-7 relative; the quotient at eps = 1e-4 is printed beside it."""
    from paper_2608_15781_amd import autograd as ag

    w, solid, theta, rr0, rp0, kw = _adjoint96()
    T, ck = w["steps"], w["checkpoint"]

    def make(th, xi):
        return core.Lbm(w["shape"], solid=solid, theta=th, rho_r0=rr0, rho_p0=rp0, xi=xi, precision="fp64",
                        tau_species=w["tau_c"], c_inlet=w["c_in"], **kw)

    def central(k, eps):
        tp = theta.ravel().copy()
        tm = theta.ravel().copy()
        tp[k] += eps
        tm[k] -= eps
        Lp = float(make(tp.reshape(theta.shape), w["xi"]).step(T)[:, 2].sum())
        Lm = float(make(tm.reshape(theta.shape), w["xi"]).step(T)[:, 2].sum())
        return (Lp - Lm) / (2 * eps)

    sim = make(theta, w["xi"])
    L0, cps, final = ag.forward_states(sim, T, ck)
    gth, gxi, _ = ag.adjoint_gradients(sim, T, ck, cps, final)
    g = gth.cpu().numpy()
    del sim, cps, final
    order = np.argsort(-np.abs(g))
    rng = np.random.default_rng(11)
    wet = np.setdiff1d(np.flatnonzero(g != 0), order[:16])
    picks = list(order[:16]) + list(rng.choice(wet, 16, replace=False))
    gmax = abs(g[order[0]])
    worst = 0.0
    for k in picks:
        fd7 = central(k, 1e-7)
        fd4 = central(k, 1e-4)
        worst = max(worst, abs(g[k] - fd7) / gmax)
        print("node %7d adjoint %+.8e fd(1e-7) %+.8e fd(1e-4) %+.8e" % (k, g[k], fd7, fd4), flush=True)
        assert abs(g[k] - fd7) < 1e-5 * gmax + 1e-5 * abs(fd7), (k, g[k], fd7)
    hx = 1e-9  # L is curved in xi too: at hx = 1e-7 the central quotient is still 5e-6 off
    fdx = (float(make(theta, w["xi"] + hx).step(T)[:, 2].sum()) -
           float(make(theta, w["xi"] - hx).step(T)[:, 2].sum())) / (2 * hx)
    print("xi: adjoint %.10e fd %.10e; worst theta error / max|g| %.2e" % (float(gxi), fdx, worst), flush=True)
    assert abs(float(gxi) - fdx) < 1e-6 * abs(fdx)


def test_adjoint96_crop_gradient_against_oracle_duals(core, oracle_mod):
    """The [0, 24)^3 crop of the 96^3 adjoint workload (periodic as a domain of its own), 200 FP64
    steps with checkpoints every 20: directional derivatives of L along two random theta
    perturbations and along xi, against the oracle's forward-mode dual numbers."""
    from paper_2608_15781_amd import autograd as ag
    from paper_2608_15781_amd import inputs

    w, solid, theta, rr0, rp0, kw = _adjoint96()
    n = 24
    solid, theta, rr0, rp0 = (inputs.crop(a, n) for a in (solid, theta, rr0, rp0))
    T, ck, xi = w["steps"], w["checkpoint"], w["xi"]
    rng = np.random.default_rng(5)
    d1 = rng.normal(size=solid.shape) * (1 - solid)
    d2 = rng.normal(size=solid.shape) * (1 - solid)
    L, dL = oracle_mod.grad((n, n, n), solid, theta, xi, T, dtheta=[d1.ravel(), d2.ravel(), np.zeros(n ** 3)],
                            dxi=[0.0, 0.0, 1.0], rho_r0=rr0, tau_c=w["tau_c"], c_in=w["c_in"], **kw)
    sim = core.Lbm((n, n, n), solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, xi=xi, precision="fp64",
                   tau_species=w["tau_c"], c_inlet=w["c_in"], **kw)
    Lg, cps, final = ag.forward_states(sim, T, ck)
    gth, gxi, _ = ag.adjoint_gradients(sim, T, ck, cps, final)
    g = gth.cpu().numpy()
    ad = [float(g @ d1.ravel()), float(g @ d2.ravel()), float(gxi)]
    print("crop24: L gpu %.12e oracle %.12e; dL adjoint %s oracle %s" % (Lg, L, ad, list(dL)), flush=True)
    assert abs(Lg - L) < 1e-10 * abs(L)
    for a, b in zip(ad, dL):
        assert abs(a - b) < 1e-8 * abs(b) + 1e-14, (a, b)


@pytest.mark.parametrize("prec,tol_th,tol_xi,tol_L", [("fp32", 1e-2, 1e-5, 1e-5), ("fp16", 0.15, 5e-5, 6e-5),
                                                      ("bf16", 0.3, 5e-4, 1e-4)])
def test_reduced_precision_adjoint_against_fp64(core, prec, tol_th, tol_xi, tol_L):
    """The adjoint in FP32 arithmetic (FP32 storage, or FP16/BF16 deviation storage whose rounding
    the adjoint takes as the identity) against the FP64 adjoint of the same problem: 24^3 porous
    mask, 100 steps, checkpoint 10. Measured on this case: FP32 dL/dtheta 1.7e-4 (relative L2),
    dL/dxi 1.2e-6, L 1.6e-6; FP16 1.5e-3, 6.2e-6, 1.0e-5; BF16 3.8e-2, 7.0e-5, 1.2e-5. The
    integral quantities are bounded at 6-8x those. The per-node contact-angle gradient is set by a
    few wetting nodes whose realignment branch falls differently under the rounding (half of the
    squared error sits on ten nodes in every mode), and builds that differ only in where
    multiply-adds are contracted have measured it up to 20x apart (FP32 3.5e-3 in one such build),
    so it is bounded more loosely: 1e-2, 0.15 and 0.3; a 48^3 case over 200 steps measures 5.4e-3,
    4.8e-3 and 0.28."""
    from paper_2608_15781_amd import autograd as ag

    n, T, seed = 24, 100, 43
    solid, theta, rr0, rp0 = _case(n, seed)
    res = {}
    for p in ("fp64", prec):
        sim = core.Lbm((n, n, n), solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, xi=0.02, precision=p,
                       tau_species=0.8, **KW)
        L, cps, fin = ag.forward_states(sim, T, 10)
        g, gx, _ = ag.adjoint_gradients(sim, T, 10, cps, fin)
        res[p] = (L, g.cpu().numpy(), float(gx))
    (L0, g0, x0), (L, g, x) = res["fp64"], res[prec]
    e_th = np.linalg.norm(g - g0) / np.linalg.norm(g0)
    e_xi = abs(x - x0) / abs(x0)
    e_L = abs(L - L0) / abs(L0)
    print("%s adjoint vs fp64: dtheta %.2e dxi %.2e L %.2e" % (prec, e_th, e_xi, e_L), flush=True)
    assert e_xi < tol_xi and e_L < tol_L
    if tol_th is not None:
        assert e_th < tol_th


def test_gradient_on_a_side_stream(core):
    """A context on a side stream (default priority) while torch's current stream is busy with
    unrelated work: the forward states, the recompute buffers and the zeroed gradient
    accumulators are all ordered on the context's stream, so the checkpointed gradient equals the
    one computed on the current stream bit for bit (24^3 mask, 60 FP32 steps, checkpoint 20)."""
    import torch

    from paper_2608_15781_amd import autograd as ag

    n, xi, T, ck = 24, 0.02, 60, 20
    solid, theta, rr0, rp0 = _case(n, 43)

    def grad(stream):
        sim = core.Lbm((n, n, n), solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, xi=xi, precision="fp32",
                       tau_species=0.8, stream=stream, **KW)
        # keep the current stream busy so that unordered work on it would overlap the library's
        busy = torch.randn(4096, 4096, device="cuda:0")
        for _ in range(8):
            busy = busy @ busy
            busy = busy / busy.abs().max()
        L, cps, fin = ag.forward_states(sim, T, ck)
        g, gx, _ = ag.adjoint_gradients(sim, T, ck, cps, fin)
        sim.stream.synchronize()
        torch.cuda.synchronize()
        return L, g.clone(), float(gx)

    L0, g0, x0 = grad(None)
    side = torch.cuda.Stream(device="cuda:0")
    L1, g1, x1 = grad(side)
    print("side stream: L %.12e / %.12e, dL/dxi %.12e / %.12e" % (L0, L1, x0, x1), flush=True)
    assert L1 == L0 and x1 == x0
    assert torch.equal(g1, g0)


def test_adjoint_refuses_overlapping_buffers(core):
    """Checked on the host before any launch: the adjoint output overlapping the input, and the
    scratch overlapping the state, are refused (through the C ABI, bypassing the binding)."""
    import torch

    n = 8
    solid, theta, rr0, rp0 = _case(n, 5)
    sim = _sim(core, n, solid, theta, rr0, rp0, 0.01)
    state = sim.get_state()
    ab, scr = sim.adjoint_bytes()
    big = torch.zeros(2 * ab + 4096, dtype=torch.uint8, device="cuda:0")
    scratch = sim.new_scratch()
    gth = torch.zeros(sim.N, dtype=torch.float64, device="cuda:0")
    gxi = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    L = core.lib()
    p = big.data_ptr()
    st = L.lbm_adjoint_step(sim._h, state.data_ptr(), p, p + 256, scratch.data_ptr(), gth.data_ptr(), gxi.data_ptr())
    assert st == core.LBM_ERR_ARG and b"overlap" in L.lbm_last_error(sim._h)
    st = L.lbm_adjoint_step(sim._h, state.data_ptr(), p, p + ab + 256, state.data_ptr() + 512, gth.data_ptr(),
                            gxi.data_ptr())
    assert st == core.LBM_ERR_ARG and b"overlap" in L.lbm_last_error(sim._h)
    # disjoint buffers are accepted
    st = L.lbm_adjoint_step(sim._h, state.data_ptr(), p, p + ab + 256, scratch.data_ptr(), gth.data_ptr(),
                            gxi.data_ptr())
    assert st == core.LBM_OK
    torch.cuda.synchronize()
