"""ctypes binding of liblbm.so. Argument marshalling only: every step of the method runs in the
library's HIP kernels; torch provides the device memory and the stream.

The library must have been built (``python -m paper_2608_15781_amd.build``); loading raises if it
is missing, and there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import build as _build

PRECISIONS = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3}
LBM_OK, LBM_ERR_ARG, LBM_ERR_ALLOC, LBM_ERR_HIP, LBM_ERR_NONFINITE, LBM_ERR_STATE, LBM_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
EXPORTED = ["lbm_version", "lbm_workspace_bytes", "lbm_state_bytes", "lbm_init", "lbm_step", "lbm_step_async",
            "lbm_moments",
            "lbm_populations", "lbm_geometry", "lbm_state_layout", "lbm_get_state", "lbm_set_state",
            "lbm_set_profiling", "lbm_kernel_times", "lbm_adjoint_bytes", "lbm_adjoint_seed", "lbm_adjoint_step",
            "lbm_steps_done", "lbm_free", "lbm_last_error", "lbm_fields_bytes", "lbm_step_fields",
            "lbm_adjoint_step_fields", "lbm_step_from", "lbm_state_sums", "lbm_adjoint_step_static",
            "lbm_adjoint_static_scratch_bytes"]
KERNELS = ("colour", "extrap", "normal", "collide")


class LbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("lbm status %d: %s" % (status, msg))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("species", ctypes.c_int32), ("x_open", ctypes.c_int32),
        ("tau", ctypes.c_double), ("tau_species", ctypes.c_double), ("sigma", ctypes.c_double),
        ("beta", ctypes.c_double), ("xi", ctypes.c_double), ("accel", (ctypes.c_double * 3) * 2),
        ("c_inlet", ctypes.c_double), ("grad_eps", ctypes.c_double), ("fp16_scale_log2", ctypes.c_int32),
        ("fluid_nodes", ctypes.c_int32),
    ]


class Reductions(ctypes.Structure):
    _fields_ = [("mass_r", ctypes.c_double), ("mass_p", ctypes.c_double), ("conversion", ctypes.c_double),
                ("species_total", ctypes.c_double), ("nonfinite", ctypes.c_double)]


_lib = None


def lib():
    """Loads liblbm.so from the package directory; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            raise RuntimeError("liblbm.so is not built: run `python -m paper_2608_15781_amd.build` "
                               "(or __graft_entry__.build())")
        L = ctypes.CDLL(_build.LIB)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        P = ctypes.POINTER
        L.lbm_version.restype = ctypes.c_char_p
        L.lbm_workspace_bytes.argtypes = [P(Params), P(sz)]
        L.lbm_state_bytes.argtypes = [P(Params), P(sz)]
        L.lbm_init.argtypes = [P(Params), vp, vp, ctypes.c_double, vp, vp, vp, vp, vp, sz, vp, P(vp)]
        L.lbm_step.argtypes = [vp, i32, vp]
        L.lbm_step_async.argtypes = [vp, i32]
        L.lbm_fields_bytes.argtypes = [P(Params), P(sz)]
        L.lbm_step_fields.argtypes = [vp, vp]
        L.lbm_step_from.argtypes = [vp, vp, vp, vp]
        L.lbm_adjoint_step_fields.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.lbm_moments.argtypes = [vp, vp, vp, vp, vp, vp]
        L.lbm_populations.argtypes = [vp, vp, vp, vp]
        L.lbm_state_sums.argtypes = [vp, vp, vp]
        L.lbm_adjoint_step_static.argtypes = [vp, vp, vp, vp, vp, vp]
        L.lbm_adjoint_static_scratch_bytes.argtypes = []
        L.lbm_adjoint_static_scratch_bytes.restype = sz
        L.lbm_geometry.argtypes = [vp, vp, vp]
        L.lbm_get_state.argtypes = [vp, vp]
        L.lbm_set_state.argtypes = [vp, vp, i64]
        L.lbm_state_layout.argtypes = [P(Params), P(sz), P(sz), P(sz), P(sz)]
        L.lbm_adjoint_bytes.argtypes = [P(Params), P(sz), P(sz)]
        L.lbm_adjoint_seed.argtypes = [vp, vp, vp]
        L.lbm_adjoint_step.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.lbm_set_profiling.argtypes = [vp, i32]
        L.lbm_kernel_times.argtypes = [vp, vp, vp]
        L.lbm_steps_done.argtypes = [vp]
        L.lbm_steps_done.restype = i64
        L.lbm_free.argtypes = [vp]
        L.lbm_last_error.argtypes = [vp]
        L.lbm_last_error.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in ("lbm_version", "lbm_steps_done", "lbm_free", "lbm_last_error",
                            "lbm_adjoint_static_scratch_bytes"):
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def make_params(shape, precision="fp32", tau=1.0, tau_species=0.9, sigma=0.0, beta=0.7, xi=0.0,
                accel=((0, 0, 0), (0, 0, 0)), species=False, x_open=False, c_inlet=1.0, grad_eps=1e-6,
                fp16_scale_log2=12, fluid_nodes=0) -> Params:
    p = Params()
    p.nx, p.ny, p.nz = (int(s) for s in shape)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.species, p.x_open = int(bool(species)), int(bool(x_open))
    p.tau, p.tau_species, p.sigma, p.beta, p.xi = tau, tau_species, sigma, beta, xi
    for k in range(2):
        for a in range(3):
            p.accel[k][a] = float(accel[k][a])
    p.c_inlet, p.grad_eps, p.fp16_scale_log2 = c_inlet, grad_eps, fp16_scale_log2
    p.fluid_nodes = int(fluid_nodes)
    return p


def _host(a, dtype, n):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=dtype)
    if a.size == 1 and n != 1:
        a = np.full(n, a.reshape(()), dtype=dtype)
    if a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a.reshape(n)


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Lbm:
    """One simulation context on one GPU.

    shape = (nx, ny, nz); per-node inputs are arrays of shape (nz, ny, nx) (x fastest) or flat.
    Keyword parameters map one to one onto lbm_params (see include/lbm.h). compact=True sizes the
    state, adjoint and per-fluid-node buffers for the mask's fluid nodes (lbm_params.fluid_nodes);
    False sizes them for every node.
    """

    def __init__(self, shape, solid=None, theta=None, theta_uniform=math.pi / 2, reactive=None, rho_r0=1.0,
                 rho_p0=0.0, c0=None, device="cuda:0", stream=None, compact=True, **kw):
        import torch

        self.torch = torch
        self.shape = tuple(int(s) for s in shape)
        nx, ny, nz = self.shape
        self.N = nx * ny * nz
        self.params = make_params(self.shape, **kw)
        self.precision = self.params.precision
        self.real = torch.float64 if self.precision == 0 else torch.float32
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        L = lib()
        N = self.N
        solid = np.zeros(N, np.uint8) if solid is None else _host(solid, np.uint8, N)
        self.solid = solid
        self.nfluid = int((solid == 0).sum())  # state entries, fluid nodes in node order
        # compact: state and per-fluid-node arrays sized for the mask's fluid nodes (else for every node)
        self.params.fluid_nodes = self.nfluid if compact else 0
        ws = ctypes.c_size_t()
        self._check(L.lbm_workspace_bytes(ctypes.byref(self.params), ctypes.byref(ws)), None)
        sb = ctypes.c_size_t()
        self._check(L.lbm_state_bytes(ctypes.byref(self.params), ctypes.byref(sb)), None)
        self.workspace_bytes, self.state_bytes = ws.value, sb.value
        self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._ws_ptr = base + off
        th = _host(theta, np.float64, N)
        react = _host(reactive, np.uint8, N)
        rr, rp = _host(rho_r0, np.float64, N), _host(rho_p0, np.float64, N)
        c0a = _host(c0, np.float64, N)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = L.lbm_init(ctypes.byref(self.params), _p(solid), _p(th), float(theta_uniform), _p(react), _p(rr),
                            _p(rp), _p(c0a), ctypes.c_void_p(self._ws_ptr), self.workspace_bytes,
                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        self._check(st, None)
        self._lib = L
        self._h = h

    def _check(self, status, h):
        if status != LBM_OK:
            msg = lib().lbm_last_error(h).decode()
            raise LbmError(status, msg)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            # the library handle is held by the instance: module globals may be gone at exit
            self._lib.lbm_free(h)
            self._h = None

    close = __del__

    @property
    def steps_done(self) -> int:
        return int(lib().lbm_steps_done(self._h))

    def step(self, nsteps=1, reductions=True, check=True):
        """Advance nsteps; returns an (nsteps, 5) array [mass_r, mass_p, conversion, species, nonfinite]."""
        out = (Reductions * max(1, nsteps))() if reductions else None
        st = lib().lbm_step(self._h, int(nsteps), out)
        if check:
            self._check(st, self._h)
        self.last_status = st
        if not reductions:
            return None
        return np.frombuffer(out, dtype=np.float64).reshape(-1, 5)[:nsteps].copy()

    def advance(self, nsteps=1):
        """Enqueue nsteps on the stream without waiting (no reductions, no non-finite check)."""
        self._check(lib().lbm_step_async(self._h, int(nsteps)), self._h)

    def _grid(self, t, comps=1):
        nx, ny, nz = self.shape
        return t.view(comps, nz, ny, nx) if comps > 1 else t.view(nz, ny, nx)

    def moments(self):
        """Level-t fields as device tensors of shape (nz, ny, nx) ((3, nz, ny, nx) for u)."""
        t = self.torch
        N = self.N
        with t.cuda.stream(self.stream):
            rr, rp, rn, c = (t.empty(N, dtype=self.real, device=self.device) for _ in range(4))
            u = t.empty(3 * N, dtype=self.real, device=self.device)
        self._check(lib().lbm_moments(self._h, rr.data_ptr(), rp.data_ptr(), rn.data_ptr(), u.data_ptr(),
                                      c.data_ptr()), self._h)
        self.stream.synchronize()
        return dict(rho_r=self._grid(rr), rho_p=self._grid(rp), rho_n=self._grid(rn), u=self._grid(u, 3),
                    c=self._grid(c))

    def populations(self):
        """Post-collision populations per colour, (19, N), (19, N), (7, N) device tensors."""
        t = self.torch
        N = self.N
        with t.cuda.stream(self.stream):
            fr = t.empty(19 * N, dtype=self.real, device=self.device)
            fp = t.empty(19 * N, dtype=self.real, device=self.device)
            g = t.empty(7 * N, dtype=self.real, device=self.device)
        self._check(lib().lbm_populations(self._h, fr.data_ptr(), fp.data_ptr(), g.data_ptr()), self._h)
        self.stream.synchronize()
        return fr.view(19, N), fp.view(19, N), g.view(7, N)

    def geometry(self):
        t = self.torch
        with t.cuda.stream(self.stream):
            info = t.empty(self.N, dtype=t.int32, device=self.device)
            wet = t.empty(4 * self.N, dtype=self.real, device=self.device)
        self._check(lib().lbm_geometry(self._h, info.data_ptr(), wet.data_ptr()), self._h)
        self.stream.synchronize()
        return info, wet.view(self.N, 4).t()

    def new_state(self):
        """An uninitialised state buffer (uint8 tensor of state_bytes) for step_from."""
        with self.torch.cuda.stream(self.stream):
            return self.torch.empty(self.state_bytes, dtype=self.torch.uint8, device=self.device)

    def step_from(self, src, dst, fields=None):
        """One enqueued step from the state in `src` into `dst` (state buffers, as from get_state or
        new_state); keeps its level-t fields in `fields` if given. With dst None only the fields
        are computed (no collision). The context's own state and step count do not change."""
        self._need(src, self.state_bytes, "source state")
        dp = None
        if dst is not None:
            self._need(dst, self.state_bytes, "destination state")
            dp = dst.data_ptr()
        fp = None
        if fields is not None:
            self._need(fields, self.fields_bytes(), "fields")
            fp = fields.data_ptr()
        self._check(lib().lbm_step_from(self._h, src.data_ptr(), dp, fp), self._h)

    def step_chain(self, states, fields=None):
        """len(states) - 1 enqueued steps, states[k] -> states[k + 1] (lbm_step_from), keeping the
        level-k fields in fields[k] if given. The buffers are checked once, before the first
        step, and the steps are issued with their raw pointers."""
        sb = self.state_bytes
        for k, s in enumerate(states):
            self._need(s, sb, "state %d" % k)
        fps = [None] * (len(states) - 1)
        if fields is not None:
            if len(fields) != len(states) - 1:
                raise ValueError("need one fields buffer per step")
            fb = self.fields_bytes()
            for k, f in enumerate(fields):
                self._need(f, fb, "fields %d" % k)
            fps = [f.data_ptr() for f in fields]
        ptrs = [s.data_ptr() for s in states]
        fn, h = lib().lbm_step_from, self._h
        for k in range(len(states) - 1):
            st = fn(h, ptrs[k], ptrs[k + 1], fps[k])
            if st != LBM_OK:
                self._check(st, h)

    def get_state(self, sync=True):
        """A copy of the state (uint8 tensor of state_bytes). With sync=False the copy is only
        enqueued on the context's stream (work on that stream sees it complete)."""
        with self.torch.cuda.stream(self.stream):
            buf = self.torch.empty(self.state_bytes, dtype=self.torch.uint8, device=self.device)
        self._check(lib().lbm_get_state(self._h, buf.data_ptr()), self._h)
        if sync:
            self.stream.synchronize()
        return buf

    def state_sums(self, state=None):
        """FP64 sums of a stored state, computed by the library on the device (lbm_state_sums):
        dict with mass_r, mass_p (the colour masses of the state's level), species_total and
        nonfinite. `state`: a state buffer (as from get_state), or None for the current state."""
        out = Reductions()
        ptr = None
        if state is not None:
            self._need(state, self.state_bytes, "state")
            ptr = state.data_ptr()
        self._check(lib().lbm_state_sums(self._h, ptr, ctypes.byref(out)), self._h)
        return dict(mass_r=out.mass_r, mass_p=out.mass_p, species_total=out.species_total,
                    nonfinite=out.nonfinite)

    # ---- state layout and adjoint -------------------------------------------------------------
    def state_layout(self):
        """Byte offsets of the population, colour-scalar and species parts of a state snapshot, and
        the plane stride (elements between consecutive planes)."""
        f, a, g, ps = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        self._check(lib().lbm_state_layout(ctypes.byref(self.params), ctypes.byref(f), ctypes.byref(a),
                                           ctypes.byref(g), ctypes.byref(ps)), None)
        return f.value, a.value, g.value, ps.value

    def state_parts(self, buf):
        """Views (19, F), (4, F), (7, F) of a state snapshot (FP32/FP64 storage only), F = number of
        fluid nodes, columns in node order; the colour scalars are stored node-major, so their view
        is strided."""
        t = self.torch
        if self.precision not in (0, 1):
            raise ValueError("state_parts needs FP32 or FP64 storage")
        dt = self.real
        es = 8 if self.precision == 0 else 4
        f_off, a_off, g_off, ps = self.state_layout()
        F = self.nfluid
        f = buf[f_off:f_off + 19 * ps * es].view(dt).view(19, ps)[:, :F]
        a = buf[a_off:a_off + 4 * ps * es].view(dt).view(ps, 4)[:F].t()
        g = buf[g_off:g_off + 7 * ps * es].view(dt).view(7, ps)[:, :F] if self.params.species else None
        return f, a, g

    def adjoint_bytes(self):
        if getattr(self, "_adj_bytes", None) is None:
            ab, sb = ctypes.c_size_t(), ctypes.c_size_t()
            self._check(lib().lbm_adjoint_bytes(ctypes.byref(self.params), ctypes.byref(ab), ctypes.byref(sb)),
                        None)
            self._adj_bytes = (ab.value, sb.value)
        return self._adj_bytes

    def new_adjoint(self):
        """A zeroed adjoint state: (30, P) tensor of the context's real type, P the plane stride;
        column f < nfluid is the fluid node of rank f. Allocated and zeroed on the context's
        stream, so the library's later work on that stream is ordered after the fill."""
        with self.torch.cuda.stream(self.stream):
            return self.torch.zeros(30, self.state_layout()[3], dtype=self.real, device=self.device)

    def new_scratch(self):
        with self.torch.cuda.stream(self.stream):
            return self.torch.empty(self.adjoint_bytes()[1] + 256, dtype=self.torch.uint8, device=self.device)

    def new_gradients(self):
        """Zeroed FP64 accumulators (dL/dtheta per node, dL/dxi) on the context's stream."""
        with self.torch.cuda.stream(self.stream):
            return (self.torch.zeros(self.N, dtype=self.torch.float64, device=self.device),
                    self.torch.zeros(1, dtype=self.torch.float64, device=self.device))

    @staticmethod
    def _aligned(t):
        p = t.data_ptr()
        return p + ((-p) % 256)

    def _need(self, t, nbytes, what):
        """The library reads and writes these buffers through raw device pointers: check them here."""
        if not t.is_contiguous() or t.device != self.device or t.numel() * t.element_size() < nbytes:
            raise ValueError("%s must be a contiguous tensor of at least %d bytes on %s" % (what, nbytes, self.device))

    def _check_adjoint_args(self, state, *adj):
        ab = self.adjoint_bytes()[0]
        self._need(state, self.state_bytes, "state")
        for a in adj:
            if a.dtype != self.real:
                raise ValueError("adjoint states are %s" % self.real)
            self._need(a, ab, "adjoint state")

    def adjoint_seed(self, state, adj):
        """adj <- dL/dS_T of L = m^p(T) at the state snapshot `state`."""
        self._check_adjoint_args(state, adj)
        self._check(lib().lbm_adjoint_seed(self._h, state.data_ptr(), adj.data_ptr()), self._h)

    def fields_bytes(self):
        if getattr(self, "_fields_bytes", None) is None:
            b = ctypes.c_size_t()
            self._check(lib().lbm_fields_bytes(ctypes.byref(self.params), ctypes.byref(b)), None)
            self._fields_bytes = b.value
        return self._fields_bytes

    def new_fields(self):
        """A buffer for the forward fields of one level (lbm_step_fields), on the context's stream."""
        with self.torch.cuda.stream(self.stream):
            return self.torch.empty(self.fields_bytes(), dtype=self.torch.uint8, device=self.device)

    def step_fields(self, fields):
        """One enqueued step that keeps its level-t fields in `fields` (from new_fields)."""
        self._need(fields, self.fields_bytes(), "fields")
        self._check(lib().lbm_step_fields(self._h, fields.data_ptr()), self._h)

    def adjoint_step(self, state, adj_in, adj_out, scratch, grad_theta, grad_xi, fields=None):
        """adj_out <- (dS_{t+1}/dS_t)^T adj_in at the state S_t; accumulates grad_theta (N doubles) and
        grad_xi (1 double) on the device."""
        if grad_theta.dtype != self.torch.float64 or grad_xi.dtype != self.torch.float64:
            raise ValueError("gradients accumulate in float64")
        self._check_adjoint_args(state, adj_in, adj_out)
        self._need(grad_theta, 8 * self.N, "grad_theta")
        self._need(grad_xi, 8, "grad_xi")
        self._need(scratch, self.adjoint_bytes()[1] + 255, "scratch")
        if fields is None:
            self._check(lib().lbm_adjoint_step(self._h, state.data_ptr(), adj_in.data_ptr(), adj_out.data_ptr(),
                                               ctypes.c_void_p(self._aligned(scratch)), grad_theta.data_ptr(),
                                               grad_xi.data_ptr()), self._h)
        else:
            self._need(fields, self.fields_bytes(), "fields")
            self._check(lib().lbm_adjoint_step_fields(self._h, state.data_ptr(), fields.data_ptr(), adj_in.data_ptr(),
                                                      adj_out.data_ptr(), ctypes.c_void_p(self._aligned(scratch)),
                                                      grad_theta.data_ptr(), grad_xi.data_ptr()), self._h)

    def adjoint_step_static(self, state, adj_in, adj_out, grad_theta, grad_xi):
        """adjoint_step with the library's fixed scratch array instead of a caller buffer
        (lbm_adjoint_step_static: no device allocation in the call)."""
        if grad_theta.dtype != self.torch.float64 or grad_xi.dtype != self.torch.float64:
            raise ValueError("gradients accumulate in float64")
        self._check_adjoint_args(state, adj_in, adj_out)
        self._need(grad_theta, 8 * self.N, "grad_theta")
        self._need(grad_xi, 8, "grad_xi")
        self._check(lib().lbm_adjoint_step_static(self._h, state.data_ptr(), adj_in.data_ptr(), adj_out.data_ptr(),
                                                  grad_theta.data_ptr(), grad_xi.data_ptr()), self._h)

    def set_profiling(self, enable: bool):
        self._check(lib().lbm_set_profiling(self._h, int(bool(enable))), self._h)

    def kernel_times(self):
        """Accumulated device milliseconds per kernel and the number of timed steps."""
        ms = (ctypes.c_double * len(KERNELS))()
        n = ctypes.c_int64()
        self._check(lib().lbm_kernel_times(self._h, ms, ctypes.byref(n)), self._h)
        return dict(zip(KERNELS, list(ms))), int(n.value)

    def set_state(self, buf, steps_done):
        if buf.numel() != self.state_bytes or buf.device != self.device:
            raise ValueError("state buffer must hold %d bytes on %s" % (self.state_bytes, self.device))
        self._check(lib().lbm_set_state(self._h, buf.data_ptr(), int(steps_done)), self._h)
        self.stream.synchronize()
