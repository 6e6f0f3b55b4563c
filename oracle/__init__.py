"""FP64 CPU oracle of the reactive colour-gradient lattice Boltzmann step (test infrastructure).

This package is the slow, plain reference that the HIP library is checked against. Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may import it; the
product library never does. The arithmetic lives in ``lbm_oracle.cpp`` (plain C++ loops, one
function per step of the paper's Sec. II and Appendix A); this module only marshals arrays.

Parity status: every function is pinned by CPU tests against closed forms, invariants or
library routines (lattice isotropy, equilibrium moments, a numerical solve of the central-moment
transform, the Akai construction, Poiseuille flow, shear-wave decay, the Laplace law, the
contact angle on a flat wall (60, 90 and 120 deg from a semicircle; 15, 30 and 150 deg from caps started
10 to 25 deg away; the same angles with the realignment cone narrowed or removed), D3Q7 species decay, the species inlet and outflow planes against
the diffusion series, mass and conversion bookkeeping, symmetry).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.cpp")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (FP64, IEEE semantics, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
               "-ffp-contract=off", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("species", ctypes.c_int32), ("x_open", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("tau", ctypes.c_double), ("tau_c", ctypes.c_double), ("sigma", ctypes.c_double),
        ("beta", ctypes.c_double), ("accel", (ctypes.c_double * 3) * 2),
        ("c_in", ctypes.c_double), ("grad_eps", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        d, i32, vp = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        _lib.orc_create.restype = vp
        _lib.orc_create.argtypes = [P(Params), d, vp, vp, vp, vp, vp, vp]
        _lib.orc_destroy.argtypes = [vp]
        _lib.orc_step.argtypes = [vp, i32, vp]
        _lib.orc_step.restype = i32
        _lib.orc_moments.argtypes = [vp] * 6
        _lib.orc_normals.argtypes = [vp] * 3
        _lib.orc_get_state.argtypes = [vp] * 4
        _lib.orc_set_state.argtypes = [vp] * 4
        _lib.orc_geometry.argtypes = [vp] * 6
        _lib.orc_lattice.argtypes = [vp] * 3
        _lib.orc_e8.argtypes = [vp, vp]
        _lib.orc_e8.restype = i32
        _lib.orc_feq.argtypes = [d, vp, vp]
        _lib.orc_cm_back.argtypes = [vp, vp, vp]
        _lib.orc_wetting.argtypes = [vp, vp, d, vp, vp, vp]
        _lib.orc_set_akai_cone.argtypes = [d]
        _lib.orc_set_akai_cone.restype = d
        _lib.orc_set_threads.argtypes = [i32]
        _lib.orc_get_threads.restype = i32
        _lib.orc_max_dirs.restype = i32
        _lib.orc_grad.restype = i32
        _lib.orc_grad.argtypes = [P(Params), d, vp, vp, vp, vp, vp, vp, i32, i32, vp, vp, vp, vp]
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        a = np.broadcast_to(a, (n,)).copy() if a.size == 1 else a.reshape(n)
    return a


def make_params(shape, tau=1.0, tau_c=0.9, sigma=0.0, beta=0.7, accel=((0, 0, 0), (0, 0, 0)),
                species=False, x_open=False, c_in=1.0, grad_eps=1e-6) -> Params:
    nx, ny, nz = shape
    p = Params()
    p.nx, p.ny, p.nz = nx, ny, nz
    p.species, p.x_open = int(bool(species)), int(bool(x_open))
    p.tau, p.tau_c, p.sigma, p.beta = tau, tau_c, sigma, beta
    for k in range(2):
        for a in range(3):
            p.accel[k][a] = float(accel[k][a])
    p.c_in, p.grad_eps = c_in, grad_eps
    return p


class Oracle:
    """Stateful FP64 oracle simulation.

    Arrays are flat in node order ``x + nx*(y + ny*z)``; numpy arrays of shape (nz, ny, nx)
    are accepted and returned.
    """

    def __init__(self, shape, solid=None, theta=np.pi / 2, reactive=None, rho_r0=1.0, rho_p0=0.0,
                 c0=None, xi=0.0, **kw):
        self.shape = tuple(int(s) for s in shape)
        nx, ny, nz = self.shape
        self.N = nx * ny * nz
        self.params = make_params(self.shape, **kw)
        self.solid = np.zeros(self.N, np.uint8) if solid is None else np.ascontiguousarray(solid, np.uint8).reshape(self.N)
        self.theta = _f64(theta, self.N)
        self.reactive = None if reactive is None else np.ascontiguousarray(reactive, np.uint8).reshape(self.N)
        self.rho_r0, self.rho_p0 = _f64(rho_r0, self.N), _f64(rho_p0, self.N)
        self.c0 = None if c0 is None else _f64(c0, self.N)
        self.xi = float(xi)
        self._h = lib().orc_create(ctypes.byref(self.params), self.xi, _ptr(self.solid), _ptr(self.theta),
                                   _ptr(self.reactive), _ptr(self.rho_r0), _ptr(self.rho_p0), _ptr(self.c0))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def _grid(self, a):
        nx, ny, nz = self.shape
        return a.reshape(-1, nz, ny, nx) if a.size != self.N else a.reshape(nz, ny, nx)

    def step(self, nsteps=1):
        """Advance; returns per-step level-t sums [mass_r, mass_p, conversion, species, nonfinite]."""
        sums = np.zeros((nsteps, 5))
        rc = lib().orc_step(self._h, nsteps, _ptr(sums))
        self.last_status = rc
        return sums

    def moments(self):
        N = self.N
        rr, rp, rn, c = (np.zeros(N) for _ in range(4))
        u = np.zeros(3 * N)
        lib().orc_moments(self._h, _ptr(rr), _ptr(rp), _ptr(rn), _ptr(u), _ptr(c))
        return dict(rho_r=self._grid(rr), rho_p=self._grid(rp), rho_n=self._grid(rn),
                    u=self._grid(u), c=self._grid(c))

    def normals(self):
        """Realigned unit normal and colour gradient of the level computed by the last moments()."""
        ns, g = np.zeros(3 * self.N), np.zeros(3 * self.N)
        lib().orc_normals(self._h, _ptr(ns), _ptr(g))
        return self._grid(ns), self._grid(g)

    def get_state(self):
        N = self.N
        fr, fp, g = np.zeros(19 * N), np.zeros(19 * N), np.zeros(7 * N)
        lib().orc_get_state(self._h, _ptr(fr), _ptr(fp), _ptr(g))
        return fr.reshape(19, N), fp.reshape(19, N), g.reshape(7, N)

    def set_state(self, fr, fp, g=None):
        fr = _f64(fr).reshape(-1)
        fp = _f64(fp).reshape(-1)
        g = None if g is None else _f64(g).reshape(-1)
        lib().orc_set_state(self._h, _ptr(fr), _ptr(fp), _ptr(g))

    def geometry(self):
        N = self.N
        wet, nn, react, ok = (np.zeros(N, np.uint8) for _ in range(4))
        ns = np.zeros(3 * N)
        lib().orc_geometry(self._h, _ptr(wet), _ptr(nn), _ptr(react), _ptr(ok), _ptr(ns))
        return dict(wet=wet, nn=nn, react=react, ns_ok=ok, ns=ns.reshape(3, N))


def lattice():
    c, w, opp = np.zeros((19, 3), np.int32), np.zeros(19), np.zeros(19, np.int32)
    lib().orc_lattice(_ptr(c), _ptr(w), _ptr(opp))
    return c, w, opp


def e8():
    e, w = np.zeros((92, 3), np.int32), np.zeros(92)
    n = lib().orc_e8(_ptr(e), _ptr(w))
    return e[:n], w[:n]


def feq(rho, u):
    out = np.zeros(19)
    lib().orc_feq(float(rho), _ptr(_f64(u)), _ptr(out))
    return out


def cm_back(u, k5_9):
    out = np.zeros(19)
    lib().orc_cm_back(_ptr(_f64(u)), _ptr(_f64(k5_9)), _ptr(out))
    return out


def wetting(n, ns, theta):
    """Returns (n*, n+, n-) of the Akai construction."""
    out, np_, nm = np.zeros(3), np.zeros(3), np.zeros(3)
    lib().orc_wetting(_ptr(_f64(n)), _ptr(_f64(ns)), float(theta), _ptr(out), _ptr(np_), _ptr(nm))
    return out, np_, nm


def set_akai_cone(s: float) -> float:
    """Sets the sine of the half-angle of the cone around +-n_s inside which the Akai
    realignment keeps n (1e-2 by default, as in the library); returns the previous value."""
    return float(lib().orc_set_akai_cone(float(s)))


def set_threads(n: int):
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def grad(shape, solid, theta, xi, nsteps, dtheta=None, dxi=None, reactive=None, rho_r0=1.0, rho_p0=0.0,
         c0=None, **kw):
    """Gas production L and its directional derivatives (forward-mode duals, exact).

    dtheta: (ndir, N) directions in contact angle (radians); dxi: (ndir,) directions in xi.
    """
    nx, ny, nz = shape
    N = nx * ny * nz
    p = make_params(shape, **kw)
    ndir = 0 if dtheta is None and dxi is None else (len(dtheta) if dtheta is not None else len(dxi))
    if ndir > lib().orc_max_dirs():
        raise ValueError("too many directions")
    dth = None if dtheta is None else np.ascontiguousarray(dtheta, np.float64).reshape(ndir * N)
    dx = None if dxi is None else np.ascontiguousarray(dxi, np.float64).reshape(ndir)
    solid = np.ascontiguousarray(solid, np.uint8).reshape(N)
    th = _f64(theta, N)
    rr, rp = _f64(rho_r0, N), _f64(rho_p0, N)
    c0a = None if c0 is None else _f64(c0, N)
    react = None if reactive is None else np.ascontiguousarray(reactive, np.uint8).reshape(N)
    L = np.zeros(1)
    dL = np.zeros(max(ndir, 1))
    rc = lib().orc_grad(ctypes.byref(p), float(xi), _ptr(solid), _ptr(th), _ptr(react), _ptr(rr), _ptr(rp),
                        _ptr(c0a), int(nsteps), int(ndir), _ptr(dth), _ptr(dx), _ptr(L), _ptr(dL))
    if rc != 0:
        raise RuntimeError("oracle gradient run failed (%d)" % rc)
    return float(L[0]), dL[:ndir].copy()
