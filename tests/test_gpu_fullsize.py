"""The large workloads at full size, on sampled nodes the oracle computes one by one.

256^3 (wavelength 16, seed 3) in FP64, FP16 and BF16 and 512^3 (wavelength 32, porosity 0.55,
theta 30 deg) in FP32 and FP16 storage, in the launch configuration of the library's step. After
a few steps the GPU's populations around each sampled node are cut out (a 13^3 box, periodic indexing), the oracle is
started from them on a 13^3 periodic domain with the same mask and contact angles, and both take
one step. The post-collision populations of the sampled node after that step depend on the state
within 4 nodes and on the mask within 4 nodes (solid normal, extrapolated colour), and the
densities of the next level on the state within 5, so the box's wrapped edges (6 nodes away)
cannot reach them.

Samples: wetting nodes, reactive nodes and interior nodes, away from the inlet and outflow planes.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

R = 6


@pytest.fixture(scope="module")
def core():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_15781_amd import core as c

    c.lib()
    return c


def _box(a, c):
    """(..., nz, ny, nx) array -> (..., 2R+1, 2R+1, 2R+1) periodic box around c = (x, y, z)."""
    import torch

    x, y, z = c
    nz, ny, nx = a.shape[-3:]
    dev = a.device if isinstance(a, torch.Tensor) else None
    rng = np.arange(-R, R + 1)
    if dev is None:
        return a[..., ((z + rng) % nz)[:, None, None], ((y + rng) % ny)[None, :, None], ((x + rng) % nx)[None, None, :]]
    zi = torch.tensor((z + rng) % nz, device=dev)
    yi = torch.tensor((y + rng) % ny, device=dev)
    xi = torch.tensor((x + rng) % nx, device=dev)
    return a.index_select(-3, zi).index_select(-2, yi).index_select(-1, xi)


def _samples(info, shape, seed, count=6):
    nx, ny, nz = shape
    info = info.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    n = np.arange(info.size)
    x = n % nx
    fluid = ((info >> 18) & 1).astype(bool) & (x >= R) & (x < nx - R)
    wet = fluid & ((info >> 19) & 1).astype(bool)
    react = fluid & (((info >> 20) & 7) > 0)
    interior = fluid & ~wet
    rng = np.random.default_rng(seed)
    picks = []
    for mask in (wet, react, interior):
        cand = np.flatnonzero(mask)
        picks += list(rng.choice(cand, count, replace=False))
    return [(int(k % nx), int((k // nx) % ny), int(k // (nx * ny))) for k in picks]


def _run(core, oracle_mod, name, precision, warm, tol_pop, tol_rho):
    import torch

    from paper_2608_15781_amd import inputs

    w, solid, theta, rr0, rp0 = inputs.workload_inputs(name, device="cuda:0")
    nx, ny, nz = w["shape"]
    print("%s: %d fluid nodes, %s" % (name, int((solid == 0).sum()), precision), flush=True)
    kw = dict(tau=w["tau"], sigma=w["sigma"], beta=w["beta"], accel=[(w["accel"], 0, 0)] * 2, species=True,
              x_open=True)
    sim = core.Lbm(w["shape"], solid=solid, theta=theta, rho_r0=rr0, rho_p0=rp0, xi=w["xi"], precision=precision,
                   tau_species=w["tau_c"], c_inlet=w["c_in"], **kw)
    sim.step(warm)
    info, _ = sim.geometry()
    samples = _samples(info, w["shape"], seed=nx)
    fr, fp, g = sim.populations()
    grid = lambda t, k: t.view(k, nz, ny, nx)  # noqa: E731
    boxes = [(_box(grid(fr, 19), c).double().cpu().numpy(), _box(grid(fp, 19), c).double().cpu().numpy(),
              _box(grid(g, 7), c).double().cpu().numpy()) for c in samples]
    del fr, fp, g
    torch.cuda.empty_cache()
    sim.step(1)
    fr, fp, g = sim.populations()
    m = sim.moments()
    gpu = []
    for (x, y, z) in samples:
        k = x + nx * (y + ny * z)
        gpu.append((fr[:, k].double().cpu().numpy(), fp[:, k].double().cpu().numpy(), g[:, k].double().cpu().numpy(),
                    np.array([float(m[f][z, y, x]) for f in ("rho_r", "rho_p", "rho_n", "c")])))
    del fr, fp, g, m, sim
    torch.cuda.empty_cache()
    worst_pop, worst_rho = 0.0, 0.0
    c0 = R + (2 * R + 1) * (R + (2 * R + 1) * R)
    for (x, y, z), (bfr, bfp, bg), (gfr, gfp, gg, gm) in zip(samples, boxes, gpu):
        mask = _box(solid, (x, y, z))
        th = _box(theta, (x, y, z))
        ref = oracle_mod.Oracle((2 * R + 1,) * 3, solid=mask, theta=th, xi=w["xi"], tau_c=w["tau_c"], c_in=w["c_in"],
                                **kw)
        ref.set_state(bfr, bfp, bg)
        ref.step(1)
        rfr, rfp, rg = ref.get_state()
        rm = ref.moments()
        rmv = np.array([rm[f].ravel()[c0] for f in ("rho_r", "rho_p", "rho_n", "c")])
        e_pop = max(np.abs(gfr - rfr[:, c0]).max(), np.abs(gfp - rfp[:, c0]).max(), np.abs(gg - rg[:, c0]).max())
        e_rho = np.abs(gm - rmv).max()
        worst_pop, worst_rho = max(worst_pop, e_pop), max(worst_rho, e_rho)
        assert e_pop < tol_pop and e_rho < tol_rho, ((x, y, z), e_pop, e_rho)
    print("%s %s: %d samples, max |population error| %.2e, max |density error| %.2e"
          % (name, precision, len(samples), worst_pop, worst_rho), flush=True)


def test_bijel256_fp64_sampled_against_oracle(core, oracle_mod):
    _run(core, oracle_mod, "bijel256", "fp64", warm=5, tol_pop=1e-12, tol_rho=1e-12)


@pytest.mark.parametrize("precision,tol_pop,tol_rho", [
    # half precision: at most 2^-12 of a deviation (species deviations reach 0.25): 6.1e-5 per
    # population, 4.3e-4 for a sum of 7
    ("fp16", 1e-4, 5e-4),
    # bfloat16: at most 2^-8 of a deviation: 9.8e-4 per population, 6.8e-3 for a sum of 7
    ("bf16", 2e-3, 1e-2),
])
def test_bijel256_reduced_storage_sampled_against_oracle(core, oracle_mod, precision, tol_pop, tol_rho):
    _run(core, oracle_mod, "bijel256", precision, warm=5, tol_pop=tol_pop, tol_rho=tol_rho)


def test_bijel512_fp32_sampled_against_oracle(core, oracle_mod):
    # the oracle steps the FP32 state exactly (FP64); the GPU rounds to FP32 once
    _run(core, oracle_mod, "bijel512", "fp32", warm=5, tol_pop=1e-6, tol_rho=2e-6)


def test_bijel512_fp16_sampled_against_oracle(core, oracle_mod):
    # FP16 deviation storage, the configuration compared with FP32 at 512^3: the GPU rounds each
    # stored deviation to half precision (at most 2^-12 of it after the 2^12 scaling); species
    # deviations reach 0.25 (C between 0 and 1), so a population is off by at most 6.1e-5 plus
    # FP32 arithmetic, and a density (at most 7 such terms for C) by at most 4.3e-4
    _run(core, oracle_mod, "bijel512", "fp16", warm=5, tol_pop=1e-4, tol_rho=5e-4)
