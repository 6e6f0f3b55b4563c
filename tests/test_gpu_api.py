"""Guarantees of the C ABI that the other GPU tests use but do not state: the enqueue-only step
(lbm_step_async) advances the state exactly as lbm_step does, kernel timing changes no result and
accounts for every timed step, and steps without host reductions (lbm_step with no per-step array)
leave the same state as steps with them."""
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


def _sim(core, prec):
    from paper_2608_15781_amd import inputs

    w, solid, theta, rr0, rp0 = inputs.workload_inputs("bijel128", size=40)
    return core.Lbm(w["shape"], solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, precision=prec, tau=w["tau"],
                    sigma=w["sigma"], beta=w["beta"], xi=w["xi"], accel=[(w["accel"], 0, 0)] * 2, species=True,
                    x_open=True, tau_species=w["tau_c"], c_inlet=w["c_in"])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_async_and_unreduced_steps_match_lbm_step(core, prec):
    a, b, c = _sim(core, prec), _sim(core, prec), _sim(core, prec)
    a.step(37)
    b.advance(20)
    b.advance(17)
    b.stream.synchronize()
    c.step(37, reductions=False)
    sa = a.get_state().cpu().numpy().tobytes()
    assert b.get_state().cpu().numpy().tobytes() == sa
    assert c.get_state().cpu().numpy().tobytes() == sa
    assert a.steps_done == b.steps_done == c.steps_done == 37


def test_kernel_timing_changes_no_result(core):
    a, b = _sim(core, "fp32"), _sim(core, "fp32")
    ra = a.step(30)
    b.set_profiling(True)
    rb = b.step(30)
    ms, n = b.kernel_times()
    b.set_profiling(False)
    assert np.array_equal(ra, rb)
    assert a.get_state().cpu().numpy().tobytes() == b.get_state().cpu().numpy().tobytes()
    assert n == 30
    assert set(ms) == {"colour", "extrap", "normal", "collide"}
    assert all(v > 0 for v in ms.values()), ms
    # enabling again resets the totals
    b.set_profiling(True)
    ms2, n2 = b.kernel_times()
    assert n2 == 0 and all(v == 0 for v in ms2.values())
    b.set_profiling(False)
