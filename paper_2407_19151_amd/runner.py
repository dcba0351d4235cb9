"""Device-resident copy of a workload and one-call helpers around the C ABI."""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from . import native
from .workloads import Workload


class DeviceWorkload:
    """The arrays of a Workload as torch device tensors (SoA, FP64)."""

    def __init__(self, wl: Workload, device: str = "cuda", unsorted: bool = False):
        import torch
        self.wl = wl
        self.device = device
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
        self.offsets = t(wl.offsets, torch.int64)
        self.cells = t(wl.cells, torch.int32)
        self.species = t(wl.species, torch.int32)
        self.w = t(wl.w, torch.float64)
        self.vx = t(wl.vx, torch.float64)
        self.vy = t(wl.vy, torch.float64)
        self.vz = t(wl.vz, torch.float64)
        self.cell_corr = torch.zeros(max(wl.n_cells, 1), dtype=torch.int32, device=device)[: wl.n_cells]
        self.stats = native.new_stats(device)

    def velocities(self) -> np.ndarray:
        return np.stack([self.vx.cpu().numpy(), self.vy.cpu().numpy(), self.vz.cpu().numpy()])

    def set_velocities(self, v: np.ndarray):
        import torch
        for dst, src in zip((self.vx, self.vy, self.vz), v):
            dst.copy_(torch.from_numpy(np.ascontiguousarray(src)))


def params_for(wl: Workload, **over) -> native.mcc_params:
    kw = dict(method=wl.method, relativistic=wl.relativistic, f_E=wl.f_E, eps0=wl.eps0,
              c=wl.c if wl.relativistic else 0.0)
    kw.update(over)
    return native.make_params(**kw)


def collide_sorted(ctx: native.Context, dw: DeviceWorkload, step: int,
                   params: Optional[native.mcc_params] = None, with_stats: bool = True):
    wl = dw.wl
    ctx.collide_sorted(dw.offsets, dw.w, dw.vx, dw.vy, dw.vz, n_cells=wl.n_cells,
                       mass=wl.mass, charge=wl.charge, collisions=wl.collisions, dt=wl.dt,
                       coulomb_log=wl.coulomb_log, seed=wl.seed, step=step,
                       params=params if params is not None else params_for(wl),
                       cell_volume=wl.cell_volume,
                       stats=dw.stats if with_stats else None,
                       cell_corr_pairs=dw.cell_corr if with_stats else None)


def collide_sorted_jvp(ctx: native.Context, dw: DeviceWorkload, tangent, step: int,
                       coulomb_log_tangent: float = 0.0,
                       params: Optional[native.mcc_params] = None, update_primal: bool = True):
    """One step of dw and its tangent; `tangent` is a (3, n) float64 device tensor,
    updated in place."""
    wl = dw.wl
    ctx.collide_sorted_jvp(dw.offsets, dw.w, dw.vx, dw.vy, dw.vz, tangent[0], tangent[1],
                           tangent[2], n_cells=wl.n_cells, mass=wl.mass, charge=wl.charge,
                           collisions=wl.collisions, dt=wl.dt, coulomb_log=wl.coulomb_log,
                           coulomb_log_tangent=coulomb_log_tangent, seed=wl.seed, step=step,
                           params=params if params is not None else params_for(wl),
                           cell_volume=wl.cell_volume, update_primal=update_primal)


def collide_adjoint(ctx: native.Context, dw: DeviceWorkload, v, g, step: int,
                    g_lnl=None, params: Optional[native.mcc_params] = None,
                    coulomb_log: Optional[float] = None):
    """g <- g J for the step of dw's population from the state v ((3, n)
    float64 device tensors; g in place); g_lnl (1-element device tensor or
    None) receives g dv'/dlnL."""
    wl = dw.wl
    ctx.collide_adjoint(dw.offsets, dw.w, v[0], v[1], v[2], g[0], g[1], g[2],
                        n_cells=wl.n_cells, mass=wl.mass, charge=wl.charge,
                        collisions=wl.collisions, dt=wl.dt,
                        coulomb_log=wl.coulomb_log if coulomb_log is None else coulomb_log,
                        seed=wl.seed, step=step,
                        params=params if params is not None else params_for(wl),
                        cell_volume=wl.cell_volume, g_coulomb_log=g_lnl)


def collide_unsorted(ctx: native.Context, dw: DeviceWorkload, step: int,
                     params: Optional[native.mcc_params] = None):
    wl = dw.wl
    ctx.collide(dw.cells, dw.species, dw.w, dw.vx, dw.vy, dw.vz, n_cells=wl.n_cells,
                mass=wl.mass, charge=wl.charge, collisions=wl.collisions, dt=wl.dt,
                coulomb_log=wl.coulomb_log, seed=wl.seed, step=step,
                params=params if params is not None else params_for(wl),
                cell_volume=wl.cell_volume, stats=dw.stats, cell_corr_pairs=dw.cell_corr)


def make_plan(ctx: native.Context, dw: DeviceWorkload, params=None, autotune=True,
              with_stats=False) -> native.Plan:
    wl = dw.wl
    return native.Plan(ctx, dw.offsets, dw.w, dw.vx, dw.vy, dw.vz, n_cells=wl.n_cells,
                       mass=wl.mass, charge=wl.charge, collisions=wl.collisions, dt=wl.dt,
                       coulomb_log=wl.coulomb_log, seed=wl.seed,
                       params=params if params is not None else params_for(wl),
                       cell_volume=wl.cell_volume, stats=dw.stats if with_stats else None,
                       cell_corr_pairs=dw.cell_corr if with_stats else None,
                       autotune=autotune)
