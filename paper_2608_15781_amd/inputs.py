"""Seeded synthetic inputs: porous masks, initial colour fields and contact-angle maps.

This module holds none of the lattice Boltzmann arithmetic. It only draws the geometry and
initial conditions that the HIP library and the reference implementation both consume, so the
two always see identical bytes.

The paper's bijel geometry (a 1024^3 bijel simulation subsampled to 256^3, Sec. III) is not
available. Its stand-in is a Gaussian random field: a sum of plane waves of one wavelength with
isotropically distributed directions and uniform phases, thresholded into solid and fluid. This
gives a bicontinuous structure with a single dominant pore size, like a bijel.
"""
from __future__ import annotations

import numpy as np


def grf_field(shape, wavelength: float, seed: int, n_waves: int = 512, device=None):
    """phi(x) = sum_j cos(k_j . x + psi_j), |k_j| = 2 pi / wavelength, on integer node coordinates.

    shape = (nx, ny, nz); returns float64 array of shape (nz, ny, nx). Directions are uniform on
    the sphere (cos(polar) ~ U(-1, 1), azimuth ~ U(0, 2 pi)), phases psi ~ U(0, 2 pi), all drawn
    from numpy's default_rng(seed). The sum is evaluated as a separable complex product per
    wave, contracted over waves with a matrix product (torch, float64/complex128).
    """
    import torch

    nx, ny, nz = (int(s) for s in shape)
    rng = np.random.default_rng(seed)
    cz = rng.uniform(-1.0, 1.0, n_waves)
    az = rng.uniform(0.0, 2.0 * np.pi, n_waves)
    psi = rng.uniform(0.0, 2.0 * np.pi, n_waves)
    kmag = 2.0 * np.pi / wavelength
    sz = np.sqrt(1.0 - cz * cz)
    k = kmag * np.stack([sz * np.cos(az), sz * np.sin(az), cz], axis=1)
    dev = torch.device(device) if device is not None else torch.device("cpu")
    kt = torch.tensor(k, dtype=torch.float64, device=dev)
    pt = torch.tensor(psi, dtype=torch.float64, device=dev)
    xs = torch.arange(nx, dtype=torch.float64, device=dev)
    ys = torch.arange(ny, dtype=torch.float64, device=dev)
    zs = torch.arange(nz, dtype=torch.float64, device=dev)
    X = torch.polar(torch.ones(n_waves, nx, dtype=torch.float64, device=dev), kt[:, 0:1] * xs[None, :])
    Y = torch.polar(torch.ones(n_waves, ny, dtype=torch.float64, device=dev), kt[:, 1:2] * ys[None, :])
    Z = torch.polar(torch.ones(n_waves, nz, dtype=torch.float64, device=dev), kt[:, 2:3] * zs[None, :] + pt[:, None])
    out = torch.empty((nz, ny, nx), dtype=torch.float64, device=dev)
    zb = max(1, min(nz, (1 << 24) // max(1, ny * n_waves)))
    for z0 in range(0, nz, zb):
        z1 = min(nz, z0 + zb)
        zy = Z[:, z0:z1, None] * Y[:, None, :]                 # (J, bz, ny)
        zy = zy.permute(1, 2, 0).reshape((z1 - z0) * ny, n_waves)
        out[z0:z1] = (zy @ X).real.reshape(z1 - z0, ny, nx)
    return out.cpu().numpy()


def grf_mask(shape, wavelength: float, seed: int, porosity: float | None = None, threshold: float = 0.0,
             n_waves: int = 512, device=None):
    """Solid mask (uint8, 1 = solid) of shape (nz, ny, nx) from the thresholded random field.

    Fluid where phi > t; t = threshold, or the (1 - porosity) quantile of phi when porosity is
    given. Returns (solid, t).
    """
    phi = grf_field(shape, wavelength, seed, n_waves, device)
    t = float(np.quantile(phi, 1.0 - porosity)) if porosity is not None else float(threshold)
    return (phi <= t).astype(np.uint8), t


def droplet(shape, radius: float, centre=None):
    """Sharp sphere of red colour in blue: rho_r0 = 1 inside |x - c| < R, rho_p0 = 1 outside."""
    nx, ny, nz = shape
    if centre is None:
        centre = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2)
    inside = (r < radius).astype(np.float64)
    return inside, 1.0 - inside


def theta_noise(shape, base_deg: float, spread_deg: float, seed: int):
    """Per-node contact angle in radians, uniform on [base - spread, base + spread] degrees."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    th = rng.uniform(base_deg - spread_deg, base_deg + spread_deg, size=(nz, ny, nx))
    return np.deg2rad(th)


def crop(a, size):
    """Leading size^3 corner of a (nz, ny, nx) array."""
    return np.ascontiguousarray(a[:size, :size, :size])


# Workloads used by the tests and the benchmark, named by what they are. Physical parameters
# the paper leaves unstated take these values: tau = 0.8 (kinematic viscosity 0.1),
# sigma = 0.01, tau_C = 0.9, C_in = C_0 = 1, beta = 0.7, all-reactant start.
WORKLOADS = {
    "droplet32": dict(shape=(32, 32, 32), radius=8.0, tau=1.0, sigma=0.01, beta=0.7, steps=500,
                      precision="fp64", species=False, xi=0.0),
    "bijel128": dict(shape=(128, 128, 128), wavelength=16.0, seed=2, threshold=0.0, tau=0.8, sigma=0.01,
                     beta=0.7, tau_c=0.9, accel=1e-6, xi=1e-3, theta_deg=60.0, species=True, x_open=True,
                     c_in=1.0, steps=2000, precision="fp32"),
    "bijel256": dict(shape=(256, 256, 256), wavelength=16.0, seed=3, threshold=0.0, tau=0.8, sigma=0.01,
                     beta=0.7, tau_c=0.9, accel=1e-6, xi=1e-3, theta_deg=60.0, species=True, x_open=True,
                     c_in=1.0, steps=5000, precision="fp16"),
    "adjoint96": dict(shape=(96, 96, 96), wavelength=12.0, seed=4, threshold=0.0, tau=0.8, sigma=0.01,
                      beta=0.7, tau_c=0.9, accel=1e-6, xi=1e-3, theta_deg=90.0, theta_spread_deg=10.0,
                      species=True, x_open=True, c_in=1.0, steps=200, checkpoint=20, precision="fp32"),
    "bijel512": dict(shape=(512, 512, 512), wavelength=32.0, seed=5, porosity=0.55, tau=0.8, sigma=0.01,
                     beta=0.7, tau_c=0.9, accel=1e-6, xi=1e-3, theta_deg=30.0, species=True, x_open=True,
                     c_in=1.0, steps=10000, precision="fp16"),
}


def workload_inputs(name: str, size: int | None = None, device=None):
    """Mask, contact angles and initial fields of a named workload (optionally cropped to size^3)."""
    w = dict(WORKLOADS[name])
    shape = w["shape"]
    if "wavelength" in w:
        solid, _ = grf_mask(shape, w["wavelength"], w["seed"], porosity=w.get("porosity"),
                            threshold=w.get("threshold", 0.0), device=device)
        rho_r0 = (1 - solid).astype(np.float64)
        rho_p0 = np.zeros_like(rho_r0)
    else:
        solid = np.zeros(shape[::-1], np.uint8)
        rho_r0, rho_p0 = droplet(shape, w["radius"])
    if "theta_spread_deg" in w:
        theta = theta_noise(shape, w["theta_deg"], w["theta_spread_deg"], w["seed"] + 1000)
    else:
        theta = np.full(shape[::-1], np.deg2rad(w.get("theta_deg", 90.0)))
    if size is not None:
        solid, theta, rho_r0, rho_p0 = (crop(a, size) for a in (solid, theta, rho_r0, rho_p0))
        w["shape"] = (size, size, size)
    return w, solid, theta, rho_r0, rho_p0
