"""Gas production as a differentiable function of the contact angles and the reaction rate.

GasProduction.apply(theta, xi, problem) runs the lattice Boltzmann step ``problem["steps"]``
times from the problem's initial state and returns L = m^p(T) - m^p(0), the product (gas) mass
created, as a float64 scalar tensor. Its backward pass is the hand-written discrete adjoint of
the library (lbm_adjoint_seed / lbm_adjoint_step) with checkpoint-and-recompute over time: the
forward pass keeps the state every ``problem["checkpoint"]`` steps, and the last segment whole;
the backward pass runs the adjoint steps backwards through that segment, then restores each
earlier checkpoint in reverse order, recomputes that segment's states, and runs the adjoint steps
backwards through it. Memory: one state per checkpoint plus one segment of states and fields
(the kept last segment's buffers are reused for the recomputation once its sweep is done).
``problem["checkpoint"] = 0`` keeps every level instead (state and forward fields, written
straight into buffers of their own by the forward pass), and the backward pass recomputes
nothing: faster, for T levels of memory.

theta: per-node contact angles in radians, shape (nz, ny, nx) (only wetting nodes matter);
xi: scalar reaction rate. Both are float64 tensors; gradients come back in float64 on the same
device as the inputs.
"""
from __future__ import annotations

import numpy as np
import torch

from . import core


def _build(theta, xi, problem):
    kw = dict(problem.get("params", {}))
    kw["xi"] = float(xi)
    return core.Lbm(problem["shape"], solid=problem["solid"], theta=theta.detach().cpu().numpy().astype(np.float64),
                    reactive=problem.get("reactive"), rho_r0=problem["rho_r0"], rho_p0=problem["rho_p0"],
                    c0=problem.get("c0"), precision=problem.get("precision", "fp32"),
                    device=problem.get("device", "cuda:0"), **kw)


class Checkpoints(dict):
    """States at the checkpoint levels, {t: state}. `last` is the last segment as the forward pass
    kept it: (s0, [state of each level s0 .. T-1], [the fields of those levels])."""
    last = None


def forward_states(sim, steps, checkpoint):
    """Runs `steps` steps; returns (L, checkpoints, final state) with L = m^p(T) - m^p(0). The
    last segment goes from buffer to buffer keeping every level's state and fields
    (lbm_step_from), so the reverse sweep, which starts there, need not recompute it."""
    mp0 = _product_mass(sim)
    t0 = sim.steps_done
    cps = Checkpoints({0: sim.get_state()})
    s_last = (steps - 1) // checkpoint * checkpoint if steps > 0 else 0
    t = 0
    while t < s_last:
        n = min(checkpoint, s_last - t)
        sim.step(n)
        t += n
        cps[t] = sim.get_state()
    if steps > 0:
        n = steps - s_last
        states = [cps[s_last]] + [sim.new_state() for _ in range(n)]
        fields = [sim.new_fields() for _ in range(n)]
        sim.step_chain(states, fields)
        final = states.pop()
        sim.set_state(final, t0 + steps)
        cps.last = (s_last, states, fields)
    else:
        final = sim.get_state()
    return _product_mass(sim) - mp0, cps, final


def _product_mass(sim):
    """m^p of the current level, summed in FP64 on the device by the library (lbm_state_sums): the
    quantity whose derivative the adjoint seed writes."""
    return sim.state_sums()["mass_p"]


def forward_keep_all(sim, steps):
    """Runs `steps` steps keeping every level: returns (L, (states S_0..S_{T-1}, their level
    fields), final state S_T) and leaves the context at S_T. The steps go from buffer to buffer
    (lbm_step_from), so nothing is copied; the colour mass changes only by the wall reaction, so
    L = m^p(T) - m^p(0) is read from the end states. Memory: T states and T field buffers."""
    mp0 = _product_mass(sim)
    t0 = sim.steps_done
    sb, fb = sim.state_bytes, sim.fields_bytes()  # multiples of 256 bytes
    # one allocation for all levels, sliced: levels 1..T, then the fields of levels 0..T-1
    with torch.cuda.stream(sim.stream):
        block = torch.empty(steps * (sb + fb), dtype=torch.uint8, device=sim.device)
    states = [sim.get_state(sync=False)] + [block[k * sb:(k + 1) * sb] for k in range(steps)]
    base = steps * sb
    fields = [block[base + k * fb:base + (k + 1) * fb] for k in range(steps)]
    sim.step_chain(states, fields)
    final = states.pop()
    sim.set_state(final, t0 + steps)
    return _product_mass(sim) - mp0, (states, fields), final


def adjoint_gradients_keep_all(sim, levels, final_state):
    """Reverse sweep over levels kept by forward_keep_all (no recomputation); returns
    (dL/dtheta per node, dL/dxi, lambda_0), bitwise the same as adjoint_gradients."""
    states, fields = levels
    dev = sim.device
    lam = sim.new_adjoint()
    lam2 = sim.new_adjoint()
    scratch = sim.new_scratch()
    gth, gxi = sim.new_gradients()
    sim.adjoint_seed(final_state, lam)
    for t in range(len(states) - 1, -1, -1):
        sim.adjoint_step(states[t], lam, lam2, scratch, gth, gxi, fields=fields[t])
        lam, lam2 = lam2, lam
    torch.cuda.synchronize(dev)
    return gth, gxi[0], lam


def adjoint_gradients(sim, steps, checkpoint, cps, final_state, keep_fields=True):
    """Reverse sweep with checkpoint-and-recompute; returns (dL/dtheta per node, dL/dxi, lambda_0).

    Each segment is recomputed from its checkpoint with enqueue-only steps between state buffers
    (lbm_step_from): the checkpoint itself is level s0 and every later level is written straight
    into a buffer of its own, so no state is copied. With keep_fields the recomputation also keeps
    every level's rho^N, n* and rho^m, which the adjoint steps then reuse instead of recomputing
    (same values bit for bit). The last segment, when the forward pass kept it (forward_states),
    is not recomputed; its sweep consumes it (cps.last is cleared) and its buffers then serve the
    recomputation, so a second sweep over the same checkpoints recomputes that segment from its
    checkpoint instead (same gradient bit for bit). Memory: one segment of `checkpoint` state
    buffers and as many field buffers."""
    dev = sim.device
    lam = sim.new_adjoint()
    lam2 = sim.new_adjoint()
    scratch = sim.new_scratch()
    gth, gxi = sim.new_gradients()
    kept = getattr(cps, "last", None)
    bufs = fields = None
    spare_states, spare_fields = [], []
    sim.adjoint_seed(final_state, lam)
    starts = sorted(cps)
    for s0 in reversed(starts):
        s1 = min(s0 + checkpoint, steps)
        if kept is not None and s0 == kept[0]:
            # kept whole by the forward pass: no recomputation
            seg, segf = kept[1], kept[2]
            for t in range(s1 - 1, s0 - 1, -1):
                sim.adjoint_step(seg[t - s0], lam, lam2, scratch, gth, gxi, fields=segf[t - s0])
                lam, lam2 = lam2, lam
            # seg[0] is the checkpoint itself and stays; the other buffers are free now
            spare_states, spare_fields = list(seg[1:]), list(segf)
            cps.last = kept = None
            continue
        if bufs is None:
            def state_buf():
                return spare_states.pop() if spare_states else sim.new_state()

            def fields_buf():
                return spare_fields.pop() if spare_fields else sim.new_fields()

            bufs = [None] + [state_buf() for _ in range(checkpoint - 1)]  # bufs[k]: level s0 + k
            if keep_fields:
                fields = [fields_buf() for _ in range(checkpoint)]
            spare_states = spare_fields = None
        seg = [cps[s0]] + bufs[1:s1 - s0]
        for t in range(s0, s1):
            k = t - s0
            if t < s1 - 1:
                sim.step_from(seg[k], seg[k + 1], fields[k] if keep_fields else None)
            elif keep_fields:
                sim.step_from(seg[k], None, fields[k])  # the segment's last level: its fields only
        for t in range(s1 - 1, s0 - 1, -1):
            sim.adjoint_step(seg[t - s0], lam, lam2, scratch, gth, gxi,
                             fields=fields[t - s0] if keep_fields else None)
            lam, lam2 = lam2, lam
    torch.cuda.synchronize(dev)
    return gth, gxi[0], lam


class GasProduction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, xi, problem):
        sim = _build(theta, xi, problem)
        steps, ck = int(problem["steps"]), int(problem.get("checkpoint", 20))
        if ck == 0:
            L, cps, final = forward_keep_all(sim, steps)
        else:
            L, cps, final = forward_states(sim, steps, ck)
        ctx.sim, ctx.cps, ctx.final, ctx.steps, ctx.ck = sim, cps, final, steps, ck
        ctx.theta_shape, ctx.theta_device, ctx.xi_device = theta.shape, theta.device, xi.device
        return torch.tensor(L, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(ctx, gL):
        if ctx.ck == 0:
            gth, gxi, _ = adjoint_gradients_keep_all(ctx.sim, ctx.cps, ctx.final)
        else:
            gth, gxi, _ = adjoint_gradients(ctx.sim, ctx.steps, ctx.ck, ctx.cps, ctx.final)
        g = gL.to(torch.float64)
        dtheta = (g.to(gth.device) * gth).view(ctx.theta_shape).to(ctx.theta_device)
        dxi = (g.to(gxi.device) * gxi).reshape(()).to(ctx.xi_device)
        ctx.sim = ctx.cps = ctx.final = None
        return dtheta, dxi, None


def gas_production(theta, xi, problem):
    """L = m^p(T) - m^p(0) with autograd support for theta (radians, per node) and xi."""
    return GasProduction.apply(theta, xi, problem)
