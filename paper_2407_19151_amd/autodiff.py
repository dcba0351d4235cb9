"""Differentiated form of the collision step, in both modes.

One step maps (v, ln Lambda) to v' with every random number and every
discrete choice fixed by (seed, step): the pairing, the acceptances, the
correction order, the cut pair of the energy correction and the failure
decision.  On the GPU, `mcc_collide_sorted_jvp` carries a tangent through
that map (forward mode, riding along the primal inside the collide kernel)
and `mcc_collide_adjoint` returns the vector-Jacobian product (reverse
mode: the step recomputed per cell and swept back through the correction,
the energy partition, the momentum restore and the scatter chains).

- `CollideStep` is the step as a `torch.autograd.Function` with both rules:
  `jvp` (for `torch.autograd.forward_ad`) and `backward`.
- `RelaxationAdjoint` gives d(T_e, T_i)_final / d(T_e0, T_i0, lnL) of the
  reparameterised relaxation v0 = sqrt(T0/m) xi (fixed xi) in reverse mode:
  the forward keeps the state every `checkpoint_every` steps, the backward
  recomputes each segment from its checkpoint and sweeps the step adjoints
  back through it.  Memory: the checkpoints plus one segment's states.
- `relaxation_jacobian` gives the same 2 x 3 Jacobian by three tangent
  sweeps carried with one primal run (no stored trajectory), and
  `Relaxation` wraps it as a Function whose backward is J^T g.
"""
from __future__ import annotations

import numpy as np
import torch

from . import native
from .runner import DeviceWorkload, collide_adjoint, params_for


def _step(ctx, dw: DeviceWorkload, v, t, step, lnl, lnl_t, params, update_primal):
    wl = dw.wl
    ctx.collide_sorted_jvp(dw.offsets, dw.w, v[0], v[1], v[2], t[0], t[1], t[2],
                           n_cells=wl.n_cells, mass=wl.mass, charge=wl.charge,
                           collisions=wl.collisions, dt=wl.dt, coulomb_log=float(lnl),
                           coulomb_log_tangent=float(lnl_t), seed=wl.seed, step=int(step),
                           params=params, cell_volume=wl.cell_volume,
                           update_primal=update_primal)


class CollideStep(torch.autograd.Function):
    """v' = step(v, lnL) for v a (3, n) float64 device tensor in the sorted
    layout of `dw`; lnL a 0-dim tensor.  Forward-mode only."""

    @staticmethod
    def forward(v, lnl, ctx_, dw, step, params):
        out = v.contiguous().clone()
        t = torch.zeros_like(out)
        _step(ctx_, dw, out, t, step, lnl.item(), 0.0, params, True)
        return out

    @staticmethod
    def setup_context(ctx, inputs, output):
        v, lnl, ctx_, dw, step, params = inputs
        ctx.save_for_forward(v, lnl)
        ctx.save_for_backward(v, lnl)
        ctx.mcc = (ctx_, dw, step, params)

    @staticmethod
    def jvp(ctx, v_t, lnl_t, *_):
        v, lnl = ctx.saved_tensors
        ctx_, dw, step, params = ctx.mcc
        vin = v.contiguous().clone()
        t = (v_t if v_t is not None else torch.zeros_like(vin)).contiguous().clone()
        dl = 0.0 if lnl_t is None else float(lnl_t)
        _step(ctx_, dw, vin, t, step, lnl.item(), dl, params, False)
        return t

    @staticmethod
    def backward(ctx, g_out):
        v, lnl = ctx.saved_tensors
        ctx_, dw, step, params = ctx.mcc
        g = g_out.contiguous().clone()
        gl = torch.zeros(1, dtype=torch.float64, device=g.device)
        collide_adjoint(ctx_, dw, v.contiguous(), g, step, g_lnl=gl, params=params,
                        coulomb_log=lnl.item())
        return g, gl[0].to(lnl.dtype), None, None, None, None


def species_temperatures(wl, v):
    """Per-species weighted temperature about the species' mean velocity,
    averaged over the three components; v a (3, n) device tensor."""
    w = torch.as_tensor(wl.w, device=v.device)
    out = []
    for sp in range(wl.n_species):
        k = torch.as_tensor(wl.species == sp, device=v.device)
        ws = w[k]
        vs = v[:, k]
        mean = (vs * ws).sum(1, keepdim=True) / ws.sum()
        out.append(wl.mass[sp] * (ws * ((vs - mean) ** 2).sum(0)).sum() / (3.0 * ws.sum()))
    return torch.stack(out)


def species_temperature_tangents(wl, v, t):
    """Tangent of species_temperatures along t (the mean term drops out since
    sum w (v - mean) = 0)."""
    w = torch.as_tensor(wl.w, device=v.device)
    out = []
    for sp in range(wl.n_species):
        k = torch.as_tensor(wl.species == sp, device=v.device)
        ws = w[k]
        vs = v[:, k]
        mean = (vs * ws).sum(1, keepdim=True) / ws.sum()
        out.append(2.0 * wl.mass[sp] * (ws * ((vs - mean) * t[:, k]).sum(0)).sum() /
                   (3.0 * ws.sum()))
    return torch.stack(out)


def _primal_step(ctx, dw: DeviceWorkload, v, step, lnl, params):
    wl = dw.wl
    ctx.collide_sorted(dw.offsets, dw.w, v[0], v[1], v[2], n_cells=wl.n_cells, mass=wl.mass,
                       charge=wl.charge, collisions=wl.collisions, dt=wl.dt,
                       coulomb_log=float(lnl), seed=wl.seed, step=int(step), params=params,
                       cell_volume=wl.cell_volume)


def relaxation_jacobian(ctx, wl, xi, Te0: float, Ti0: float, lnl: float, steps: int,
                        params=None):
    """T_final = (T_e, T_i) after `steps` steps from v0 = sqrt(T0_s/m_s) xi, and
    J = d T_final / d (T_e0, T_i0, lnL) (2 x 3), on the GPU."""
    params = params if params is not None else params_for(wl)
    dw = DeviceWorkload(wl)
    xi_d = torch.as_tensor(np.ascontiguousarray(xi), device="cuda", dtype=torch.float64)
    sp = torch.as_tensor(wl.species, device="cuda")
    T0 = torch.where(sp == 0, torch.tensor(Te0, device="cuda", dtype=torch.float64),
                     torch.tensor(Ti0, device="cuda", dtype=torch.float64))
    m = torch.as_tensor(wl.mass, device="cuda")[sp]
    v = (torch.sqrt(T0 / m) * xi_d).contiguous()
    # dv0/dT0_s = v0 / (2 T0_s) on species s
    tangents = [torch.where(sp == 0, v / (2.0 * Te0), torch.zeros_like(v)).contiguous(),
                torch.where(sp == 1, v / (2.0 * Ti0), torch.zeros_like(v)).contiguous(),
                torch.zeros_like(v)]
    dlnl = [0.0, 0.0, 1.0]
    for k in range(steps):
        # the tangents at the step's input, then the step itself (the same
        # primal stepper as RelaxationAdjoint, so both follow one trajectory)
        for d in range(3):
            _step(ctx, dw, v, tangents[d], k, lnl, dlnl[d], params, False)
        _primal_step(ctx, dw, v, k, lnl, params)
    T = species_temperatures(wl, v)
    J = torch.stack([species_temperature_tangents(wl, v, tangents[d]) for d in range(3)], 1)
    return T, J


def _initial_state(wl, xi, Te0: float, Ti0: float):
    """v0 = sqrt(T0_s / m_s) xi on the device, and the species index."""
    xi_d = torch.as_tensor(np.ascontiguousarray(xi), device="cuda", dtype=torch.float64)
    sp = torch.as_tensor(wl.species, device="cuda")
    T0 = torch.where(sp == 0, torch.tensor(Te0, device="cuda", dtype=torch.float64),
                     torch.tensor(Ti0, device="cuda", dtype=torch.float64))
    m = torch.as_tensor(wl.mass, device="cuda")[sp]
    return (torch.sqrt(T0 / m) * xi_d).contiguous(), sp


def species_temperature_adjoint(wl, v, gT):
    """Adjoint of species_temperatures: d(sum_s gT_s T_s)/dv (the mean term
    drops out since sum w (v - mean) = 0)."""
    w = torch.as_tensor(wl.w, device=v.device)
    g = torch.zeros_like(v)
    for sp in range(wl.n_species):
        k = torch.as_tensor(wl.species == sp, device=v.device)
        ws = w[k]
        vs = v[:, k]
        mean = (vs * ws).sum(1, keepdim=True) / ws.sum()
        g[:, k] = gT[sp] * 2.0 * wl.mass[sp] * ws * (vs - mean) / (3.0 * ws.sum())
    return g


class RelaxationAdjoint(torch.autograd.Function):
    """(T_e, T_i) after `steps` steps from v0 = sqrt(T0/m) xi as a
    differentiable function of (T_e0, T_i0, lnL) (0-dim float64 tensors),
    differentiated in reverse mode with checkpoints every
    `checkpoint_every` steps.  `params` selects the precision form (the FP32
    kinematics form is differentiated at its own states and choices).

        Te, Ti = RelaxationAdjoint.apply(Te0, Ti0, lnl, ctx, wl, xi, steps)
    """

    @staticmethod
    def forward(ctx, Te0, Ti0, lnl, ctx_, wl, xi, steps, checkpoint_every=10, params=None):
        params = params if params is not None else params_for(wl)
        dw = DeviceWorkload(wl)
        v, _ = _initial_state(wl, xi, Te0.item(), Ti0.item())
        checkpoints = []
        for k in range(steps):
            if k % checkpoint_every == 0:
                checkpoints.append(v.clone())
            _primal_step(ctx_, dw, v, k, lnl.item(), params)
        T = species_temperatures(wl, v)
        ctx.mcc = (ctx_, wl, xi, steps, checkpoint_every, checkpoints, dw, params, Te0.item(),
                   Ti0.item(), lnl.item())
        ctx.save_for_backward(v)
        return T[0].clone(), T[1].clone()

    @staticmethod
    def backward(ctx, gTe, gTi):
        (v,) = ctx.saved_tensors
        ctx_, wl, xi, steps, every, checkpoints, dw, params, Te0, Ti0, lnl = ctx.mcc
        gT = torch.stack([gTe, gTi]).to(torch.float64)
        g = species_temperature_adjoint(wl, v, gT).contiguous()
        gl = torch.zeros(1, dtype=torch.float64, device=g.device)
        g_lnl = torch.zeros((), dtype=torch.float64, device=g.device)
        for seg in reversed(range(len(checkpoints))):
            start = seg * every
            end = min(start + every, steps)
            states = [checkpoints[seg]]
            for k in range(start, end - 1):  # the segment's states, recomputed
                nxt = states[-1].clone()
                _primal_step(ctx_, dw, nxt, k, lnl, params)
                states.append(nxt)
            for k in reversed(range(start, end)):
                collide_adjoint(ctx_, dw, states[k - start], g, k, g_lnl=gl, params=params,
                                coulomb_log=lnl)
                g_lnl = g_lnl + gl[0]
        v0, sp = _initial_state(wl, xi, Te0, Ti0)
        ge = (g * v0)[:, sp == 0].sum() / (2.0 * Te0)
        gi = (g * v0)[:, sp == 1].sum() / (2.0 * Ti0)
        return (ge.to(gTe.device), gi.to(gTe.device), g_lnl.to(gTe.device), None, None, None,
                None, None, None)


class Relaxation(torch.autograd.Function):
    """(T_e, T_i)_final as a differentiable function of (T_e0, T_i0, lnL)
    (0-dim float64 tensors); the Jacobian comes from the forward sweep and
    backward returns J^T g."""

    @staticmethod
    def forward(Te0, Ti0, lnl, ctx_, wl, xi, steps):
        T, J = relaxation_jacobian(ctx_, wl, xi, Te0.item(), Ti0.item(), lnl.item(), steps)
        return T[0].clone(), T[1].clone(), J

    @staticmethod
    def setup_context(ctx, inputs, output):
        ctx.save_for_backward(output[2])
        ctx.mark_non_differentiable(output[2])

    @staticmethod
    def backward(ctx, gTe, gTi, _gJ):
        (J,) = ctx.saved_tensors
        g = torch.stack([gTe, gTi]).to(J.dtype) @ J
        return (g[0].to(gTe.device), g[1].to(gTe.device), g[2].to(gTe.device), None, None,
                None, None)
