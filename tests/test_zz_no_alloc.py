"""The allocation-free adjoint step (lbm_adjoint_step_static) against lbm_adjoint_step.

Both run the same kernels on the same inputs; only where the scratch lives differs (the library's
fixed device array instead of a caller buffer), so the outputs must agree bit for bit. Two calls in
a row on different problems, the second smaller, show that nothing the first call left in the
shared array leaks into the second. A third context whose scratch need exceeds the array must be
refused with LBM_ERR_ARG.
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


KW = dict(tau=0.7, sigma=0.02, beta=0.7, accel=[(2e-5, 0, 0), (2e-5, 0, 0)], species=True, x_open=True,
          tau_species=0.8)


def _problem(core, n, seed, precision):
    from paper_2608_15781_amd import inputs

    solid, _ = inputs.grf_mask((n, n, n), 7.0, seed)
    rng = np.random.default_rng(seed + 1)
    theta = np.deg2rad(rng.uniform(60, 120, solid.shape))
    rr0 = (1 - solid).astype(float)
    sim = core.Lbm((n, n, n), solid=solid, theta=theta, rho_r0=rr0, rho_p0=np.zeros_like(rr0), xi=0.05,
                   precision=precision, **KW)
    sim.step(9)
    return sim


def _both(sim, seed):
    """One reverse step from a random lambda_{t+1} through both entry points."""
    import torch

    S = sim.get_state()
    gen = torch.Generator(device=sim.device).manual_seed(seed)
    lam1 = sim.new_adjoint()
    lam1[:, :sim.nfluid] = torch.randn(30, sim.nfluid, dtype=sim.real, device=sim.device, generator=gen)
    out = []
    for static in (False, True):
        lam0 = sim.new_adjoint()
        gth, gxi = sim.new_gradients()
        if static:
            sim.adjoint_step_static(S, lam1, lam0, gth, gxi)
        else:
            sim.adjoint_step(S, lam1, lam0, sim.new_scratch(), gth, gxi)
        torch.cuda.synchronize()
        out.append((lam0[:, :sim.nfluid].clone(), gth.clone(), gxi.clone()))
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_static_adjoint_step_matches_caller_scratch(core, precision):
    import torch

    for n, seed in ((20, 3), (11, 5)):  # the second call on a smaller lattice
        print("static adjoint: %s %d^3 seed %d" % (precision, n, seed), flush=True)
        sim = _problem(core, n, seed, precision)
        (l_ref, g_ref, x_ref), (l_st, g_st, x_st) = _both(sim, seed)
        assert torch.equal(l_ref, l_st)
        assert torch.equal(g_ref, g_st)
        assert torch.equal(x_ref, x_st)
        assert float(l_ref.abs().max()) > 0 and float(x_ref.abs().max()) > 0


def test_static_adjoint_step_refuses_oversized_problem(core):
    import torch

    n = 96
    solid = np.zeros((n, n, n), np.uint8)
    sim = core.Lbm((n, n, n), solid=solid, rho_r0=1.0, rho_p0=0.0, precision="fp64", **KW)
    assert sim.adjoint_bytes()[1] > core.lib().lbm_adjoint_static_scratch_bytes()
    S = sim.get_state()
    lam1, lam0 = sim.new_adjoint(), sim.new_adjoint()
    gth, gxi = sim.new_gradients()
    with pytest.raises(core.LbmError) as e:
        sim.adjoint_step_static(S, lam1, lam0, gth, gxi)
    assert e.value.status == core.LBM_ERR_ARG
    torch.cuda.synchronize()
