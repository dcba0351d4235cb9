"""Seeded synthetic plasmas shaped like the paper's test problems.

This module only draws inputs (velocities, weights, per-cell counts).  It
holds none of the collision method's arithmetic, so both the GPU path and
the CPU oracle can be fed from it.

Units are normalized: eps0 = 1, electron mass 1, electron charge magnitude 1,
cell volume 1.  Relative weights are scaled by one common factor per workload
so that the mean electron density per cell is 1 (weight ratios unchanged).
The time step is a fraction of the electron collision time

    tau_e = 3 (2 pi)^{3/2} eps0^2 sqrt(m_e) T_e^{3/2} / (Z n_e e^4 lnL),

the Braginskii form of the paper's tau_e used with the 0D Spitzer model of
Sec. 5.3 (there in practical units).

Workloads (one particle array per workload, grouped by (cell, species)):
  1  one electron species, 16 cells x 200, anisotropic Maxwellian
     (T_x = T_y = 1, T_z = 2), lognormal(0, 1) weights, N97, lnL = 10,
     dt = 0.05 tau_e(T = 1).
  2  electrons + ions (m_i = 100, q = +1), 4096 cells, Poisson(256) particles
     per species per cell, T_e = 2, T_i = 1, w_e = 1, w_i = 10^U(1,2),
     lnL = 10, dt = 0.05 tau_e(T_e = 2).
  3  as 2, 65536 cells, N_cell = clip(round(lognormal(ln 200, 1)), 16, 4096)
     split ceil(N/2) electrons / floor(N/2) ions.
  4  relativistic beam-plasma, c = 1: 448 background electrons
     (Maxwell-Juettner, T = 0.05 m c^2), 128 beam electrons (gamma = 3 along
     x, same thermal spread, weight 1e-2 relative), 448 ions (m = 1836,
     T_i = T_e, neutralizing weight), 16384 cells, dt = 0.05 tau_e(bg).
  5  as 2 with 1024 cells x (256 e + 256 i), v0 = sqrt(T0/m) xi.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

TA77 = 0
N97 = 1
HARD_SPHERE = 2   # elastic, isotropic, constant cross-section (collision tuples (a, b, sigma))

PHILOX_SEED_BASE = 0x2407_1915_1000_0000


def tau_e(T: float, n_e: float = 1.0, lnL: float = 10.0, Z: float = 1.0,
          eps0: float = 1.0, m_e: float = 1.0, e: float = 1.0) -> float:
    """Electron collision time in the normalized units of this module."""
    return (3.0 * (2.0 * math.pi) ** 1.5 * eps0 ** 2 * math.sqrt(m_e) * T ** 1.5
            / (Z * n_e * e ** 4 * lnL))


@dataclasses.dataclass
class Workload:
    name: str
    n_cells: int
    n_species: int
    offsets: np.ndarray          # int64 [n_cells*n_species + 1]
    cells: np.ndarray            # int32 [n]
    species: np.ndarray          # int32 [n]
    w: np.ndarray                # float64 [n]
    vx: np.ndarray               # float64 [n] (proper velocity if relativistic)
    vy: np.ndarray
    vz: np.ndarray
    mass: np.ndarray             # float64 [n_species]
    charge: np.ndarray           # float64 [n_species]
    collisions: List[Tuple[int, int]]
    dt: float
    coulomb_log: float
    method: int
    relativistic: bool = False
    c: float = math.inf
    eps0: float = 1.0
    cell_volume: float = 1.0
    seed: int = PHILOX_SEED_BASE
    steps: int = 1
    f_E: float = 0.05
    extra: Optional[dict] = None

    @property
    def n(self) -> int:
        return int(self.w.shape[0])

    def copy(self) -> "Workload":
        d = dataclasses.replace(self)
        for k in ("offsets", "cells", "species", "w", "vx", "vy", "vz", "mass", "charge"):
            setattr(d, k, getattr(self, k).copy())
        return d

    def velocities(self) -> np.ndarray:
        return np.stack([self.vx, self.vy, self.vz])

    def particle_collisions_per_step(self) -> int:
        """Particle-collisions per step: each particle counts once for every
        collision in the list that includes its species (and that has pairs
        in its cell)."""
        cnt = np.diff(self.offsets).reshape(self.n_cells, self.n_species)
        tot = 0
        for c in self.collisions:
            a, b = c[0], c[1]
            if a == b:
                na = cnt[:, a]
                tot += int(na[na >= 2].sum())
            else:
                na, nb = cnt[:, a], cnt[:, b]
                ok = (na > 0) & (nb > 0)
                tot += int(na[ok].sum() + nb[ok].sum())
        return tot

    def unsorted(self, seed: int = 12345) -> "Workload":
        """Same particles in a random order (for the unsorted entry point)."""
        rng = np.random.Generator(np.random.PCG64(seed))
        perm = rng.permutation(self.n)
        d = self.copy()
        for k in ("cells", "species", "w", "vx", "vy", "vz"):
            setattr(d, k, getattr(self, k)[perm].copy())
        d.extra = dict(self.extra or {}, perm=perm)
        return d


def _assemble(name, counts, mass, charge, draw, collisions, dt, lnL, method,
              seed_data, **kw) -> Workload:
    """counts: int [n_cells, S]; draw(rng, s, n) -> (w_rel, vx, vy, vz)."""
    rng = np.random.Generator(np.random.PCG64(seed_data))
    n_cells, S = counts.shape
    flat = counts.reshape(-1).astype(np.int64)
    offsets = np.zeros(flat.size + 1, dtype=np.int64)
    np.cumsum(flat, out=offsets[1:])
    n = int(offsets[-1])
    cells = np.repeat(np.repeat(np.arange(n_cells, dtype=np.int32), S), flat)
    species = np.repeat(np.tile(np.arange(S, dtype=np.int32), n_cells), flat)
    w = np.empty(n)
    vx = np.empty(n)
    vy = np.empty(n)
    vz = np.empty(n)
    for s in range(S):
        idx = np.nonzero(species == s)[0]
        ws, x, y, z = draw(rng, s, idx.size)
        w[idx], vx[idx], vy[idx], vz[idx] = ws, x, y, z
    return Workload(name=name, n_cells=n_cells, n_species=S, offsets=offsets,
                    cells=cells, species=species, w=w, vx=vx, vy=vy, vz=vz,
                    mass=np.asarray(mass, dtype=np.float64),
                    charge=np.asarray(charge, dtype=np.float64),
                    collisions=list(collisions), dt=dt, coulomb_log=lnL,
                    method=method, **kw)


def _scale_electron_density(wl: Workload, electron_species=(0,)) -> Workload:
    """Common weight factor so that the mean electron density per cell is 1."""
    tot = sum(wl.w[wl.species == s].sum() for s in electron_species)
    scale = wl.n_cells * wl.cell_volume / tot
    wl.w *= scale
    wl.extra = dict(wl.extra or {}, weight_scale=scale)
    return wl


def config1(n_cells: int = 16, ppc: int = 200, seed_data: int = 1,
            method: int = N97) -> Workload:
    counts = np.full((n_cells, 1), ppc, dtype=np.int64)

    def draw(rng, s, n):
        w = rng.lognormal(0.0, 1.0, n)
        return (w, rng.normal(0, 1.0, n), rng.normal(0, 1.0, n),
                rng.normal(0, math.sqrt(2.0), n))

    wl = _assemble("1: one species, anisotropic Maxwellian, lognormal weights",
                   counts, [1.0], [-1.0], draw, [(0, 0)],
                   dt=0.05 * tau_e(1.0), lnL=10.0, method=method,
                   seed_data=seed_data, seed=PHILOX_SEED_BASE + 1, steps=100)
    return _scale_electron_density(wl)


def _two_species_draw(Te=2.0, Ti=1.0, mi=100.0):
    def draw(rng, s, n):
        if s == 0:
            w = np.ones(n)
            sig = math.sqrt(Te / 1.0)
        else:
            w = 10.0 ** rng.uniform(1.0, 2.0, n)
            sig = math.sqrt(Ti / mi)
        return w, rng.normal(0, sig, n), rng.normal(0, sig, n), rng.normal(0, sig, n)
    return draw


def config2(n_cells: int = 4096, mean_ppc: float = 256.0, seed_data: int = 2,
            method: int = N97) -> Workload:
    rng = np.random.Generator(np.random.PCG64(seed_data + 1000))
    counts = rng.poisson(mean_ppc, size=(n_cells, 2)).astype(np.int64)
    wl = _assemble("2: electrons + ions (m_i = 100), Poisson(256) per species",
                   counts, [1.0, 100.0], [-1.0, 1.0], _two_species_draw(),
                   [(0, 0), (1, 1), (0, 1)], dt=0.05 * tau_e(2.0), lnL=10.0,
                   method=method, seed_data=seed_data,
                   seed=PHILOX_SEED_BASE + 2, steps=200)
    return _scale_electron_density(wl)


def config3_counts(n_cells: int = 65536, seed_data: int = 3) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed_data + 1000))
    ncell = np.clip(np.rint(rng.lognormal(math.log(200.0), 1.0, n_cells)), 16, 4096)
    ncell = ncell.astype(np.int64)
    return np.stack([(ncell + 1) // 2, ncell // 2], axis=1)


def config3(n_cells: int = 65536, seed_data: int = 3, method: int = N97) -> Workload:
    counts = config3_counts(n_cells, seed_data)
    wl = _assemble("3: 65536 uneven cells, lognormal counts clipped to [16, 4096]",
                   counts, [1.0, 100.0], [-1.0, 1.0], _two_species_draw(),
                   [(0, 0), (1, 1), (0, 1)], dt=0.05 * tau_e(2.0), lnL=10.0,
                   method=method, seed_data=seed_data,
                   seed=PHILOX_SEED_BASE + 3, steps=20)
    return _scale_electron_density(wl)


def hard_sphere(wl: Workload, collision_prob: float = 0.05) -> Workload:
    """The same population under the hard-sphere process: collision (a, b)
    gets the cross-section with which a particle of species a expects about
    `collision_prob` collisions per step, at the mean density of species b
    and the mean relative speed of two Maxwellians with the populations'
    velocity variances (sqrt(8 / pi) g, g^2 the sum of the per-component
    variances)."""
    dV = np.broadcast_to(np.asarray(wl.cell_volume, dtype=np.float64), (wl.n_cells,))
    var = [float((wl.vx[wl.species == s] ** 2 + wl.vy[wl.species == s] ** 2
                  + wl.vz[wl.species == s] ** 2).mean()) / 3.0 for s in range(wl.n_species)]
    coll = []
    for c in wl.collisions:
        a, b = c[0], c[1]
        dens_b = float(np.bincount(wl.cells[wl.species == b], wl.w[wl.species == b],
                                   wl.n_cells).sum() / dV.sum())
        mean_u = math.sqrt(8.0 / math.pi) * math.sqrt(var[a] + var[b])
        coll.append((a, b, collision_prob / (dens_b * mean_u * wl.dt)))
    return dataclasses.replace(wl, name=wl.name + ", hard spheres", method=HARD_SPHERE,
                               collisions=coll)


def maxwell_juttner_speed(rng, theta: float, n: int) -> np.ndarray:
    """|u|/c of a Maxwell-Juettner distribution f(u) ~ u^2 exp(-gamma/theta),
    by inverse CDF on a fine grid."""
    umax = max(40.0 * math.sqrt(theta), 40.0 * theta + 1.0)
    grid = np.linspace(0.0, umax, 200001)
    gam = np.sqrt(1.0 + grid ** 2)
    pdf = grid ** 2 * np.exp(-(gam - 1.0) / theta)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(grid))])
    cdf /= cdf[-1]
    return np.interp(rng.uniform(0.0, 1.0, n), cdf, grid)


def _iso(rng, speed):
    n = speed.size
    mu = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * math.pi, n)
    st = np.sqrt(1.0 - mu * mu)
    return speed * st * np.cos(ph), speed * st * np.sin(ph), speed * mu


def config4(n_cells: int = 16384, n_bg: int = 448, n_beam: int = 128,
            n_ion: int = 448, seed_data: int = 4, method: int = N97) -> Workload:
    theta = 0.05
    gb = 3.0
    mi = 1836.0
    counts = np.tile(np.array([[n_bg + n_beam, n_ion]], dtype=np.int64), (n_cells, 1))
    w_ion = 1.0 + 0.01 * n_beam / n_ion

    def draw(rng, s, n):
        if s == 0:
            per = n_bg + n_beam
            u = maxwell_juttner_speed(rng, theta, n)
            ux, uy, uz = _iso(rng, u)
            k = np.arange(n) % per
            beam = k >= n_bg
            w = np.where(beam, 1e-2, 1.0)
            # boost the beam particles' thermal proper velocity by gamma = 3 along x
            bb = math.sqrt(1.0 - 1.0 / gb ** 2)
            g = np.sqrt(1.0 + ux * ux + uy * uy + uz * uz)
            ux = np.where(beam, gb * (ux + bb * g), ux)
            return w, ux, uy, uz
        u = maxwell_juttner_speed(rng, theta / mi, n)
        ux, uy, uz = _iso(rng, u)
        return np.full(n, w_ion), ux, uy, uz

    wl = _assemble("4: relativistic beam through Maxwell-Juettner e-i background",
                   counts, [1.0, mi], [-1.0, 1.0], draw,
                   [(0, 0), (1, 1), (0, 1)], dt=0.05 * tau_e(theta), lnL=10.0,
                   method=method, seed_data=seed_data,
                   seed=PHILOX_SEED_BASE + 4, steps=500, relativistic=True, c=1.0)
    # mean background-electron density 1 per cell
    scale = 1.0 / n_bg
    wl.w *= scale
    wl.extra = dict(weight_scale=scale)
    return wl


def config5(n_cells: int = 1024, ppc: int = 256, Te0: float = 2.0, Ti0: float = 1.0,
            seed_data: int = 5, method: int = N97) -> Workload:
    counts = np.full((n_cells, 2), ppc, dtype=np.int64)
    wl = _assemble("5: differentiated relaxation, 1024 cells x (256 e + 256 i)",
                   counts, [1.0, 100.0], [-1.0, 1.0],
                   _two_species_draw(Te0, Ti0), [(0, 0), (1, 1), (0, 1)],
                   dt=0.05 * tau_e(2.0), lnL=10.0, method=method,
                   seed_data=seed_data, seed=PHILOX_SEED_BASE + 5, steps=50)
    return _scale_electron_density(wl)


# SI constants (CODATA 2018) for the paper's own test problems
E_CHARGE = 1.602176634e-19      # C
M_ELECTRON = 9.1093837015e-31   # kg
M_U = 1.66053906660e-27         # kg
EPS0_SI = 8.8541878128e-12      # F/m

# Test 1 of the numerical tests (Sec. 5.1 and its table): two populations of
# fully ionized carbon 12 in one species; per case N_A, N_B per cell, dt [s]
# and f_E (the weight ratio follows from the densities and counts)
PAPER_T1_CASES = {
    "T1a": (400, 4000, 50e-15, 0.05),
    "T1b": (400, 400, 50e-15, 0.05),
    "T1c": (4000, 400, 15e-15, 0.02),
    "T1d": (200, 8000, 50e-15, 0.05),
}


def paper_test1(case: str = "T1b", n_cells: int = 180, seed_data: int = 11,
                method: int = N97, cell_volume: float = 1e-18) -> Workload:
    """Test 1 in SI units: populations A (n = 1e19 cm^-3, T = 500 eV,
    U = +655 km/s along x) and B (n = 1e20 cm^-3, T = 500 eV, at rest) of
    C^6+ (m = 12 m_u - 6 m_e), lnL = 10, quasi-0D (cells independent).  Each
    cell holds N_A particles of A, then N_B of B, all one species; weights
    are physical particles per macro-particle, n * dV / N.  extra["population"]
    is 0 for A and 1 for B."""
    n_a, n_b, dt, f_e = PAPER_T1_CASES[case]
    m = 12.0 * M_U - 6.0 * M_ELECTRON
    q = 6.0 * E_CHARGE
    dens = (1e25, 1e26)            # m^-3
    temp_ev = (500.0, 500.0)
    drift = (655e3, 0.0)           # m/s along x
    counts = np.full((n_cells, 1), n_a + n_b, dtype=np.int64)
    rng = np.random.Generator(np.random.PCG64(seed_data))
    n = n_cells * (n_a + n_b)
    pop = np.tile(np.concatenate([np.zeros(n_a, np.int8), np.ones(n_b, np.int8)]), n_cells)
    w = np.empty(n)
    v = np.empty((3, n))
    for k, npk in enumerate((n_a, n_b)):
        sel = pop == k
        w[sel] = dens[k] * cell_volume / npk
        sig = math.sqrt(temp_ev[k] * E_CHARGE / m)
        v[:, sel] = rng.normal(0.0, sig, size=(3, int(sel.sum())))
        v[0, sel] += drift[k]

    offsets = np.zeros(n_cells + 1, dtype=np.int64)
    np.cumsum(counts.reshape(-1), out=offsets[1:])
    wl = Workload(name="paper Test 1 (%s), %d cells x (%d A + %d B) C6+" % (case, n_cells, n_a, n_b),
                  n_cells=n_cells, n_species=1, offsets=offsets,
                  cells=np.repeat(np.arange(n_cells, dtype=np.int32), n_a + n_b),
                  species=np.zeros(n, dtype=np.int32), w=w, vx=v[0].copy(), vy=v[1].copy(),
                  vz=v[2].copy(), mass=np.array([m]), charge=np.array([q]),
                  collisions=[(0, 0)], dt=dt, coulomb_log=10.0, method=method,
                  eps0=EPS0_SI, cell_volume=cell_volume, f_E=f_e,
                  seed=PHILOX_SEED_BASE + 0x71, steps=1)
    wl.extra = dict(population=pop, densities=dens, temperatures_ev=temp_ev, drifts=drift)
    return wl


# Test 2 (Sec. 5.2 and its table): A in species alpha, B and C in species
# beta; per case N_A, N_B, N_C per cell (dt = 50 fs, f_E = 0.05 throughout)
PAPER_T2_CASES = {
    "T2a": (400, 4000, 200),
    "T2b": (400, 4000, 800),
    "T2c": (400, 800, 4000),
    "T2d": (4000, 500, 100),
    "T2e": (4000, 100, 500),
}


def _populations(rng, m, counts, dens, temps_ev, drifts, cell_volume, n_cells):
    """Per population k: N_k particles per cell, weights n_k dV / N_k,
    Maxwellian velocities about a drift along x."""
    out = []
    for npk, n_k, t_k, u_k in zip(counts, dens, temps_ev, drifts):
        total = npk * n_cells
        sig = math.sqrt(t_k * E_CHARGE / m)
        v = rng.normal(0.0, sig, size=(3, total))
        v[0] += u_k
        out.append((np.full(total, n_k * cell_volume / npk), v))
    return out


def paper_test2(case: str = "T2a", n_cells: int = 180, seed_data: int = 12,
                method: int = N97, cell_volume: float = 1e-18, scale: int = 1) -> Workload:
    """Test 2 in SI units: populations A (species alpha: n = 1e19 cm^-3,
    U = +655 km/s), B and C (species beta: n = 1e20 cm^-3 at rest, and the
    low-density C at U = -655 km/s), all C^6+ at T = 500 eV, lnL = 10,
    dt = 50 fs, f_E = 0.05.  n_C = 5e18 cm^-3: every row of the paper's table
    gives n_A : n_B : n_C = 2 : 20 : 1 through its counts and weight ratios.
    Collisions (alpha, alpha), (beta, beta), (alpha, beta).
    extra["population"] is 0, 1, 2 for A, B, C.  `scale` multiplies every
    per-cell count (the weight ratios stay those of the table)."""
    n_a, n_b, n_c = (scale * k for k in PAPER_T2_CASES[case])
    m = 12.0 * M_U - 6.0 * M_ELECTRON
    q = 6.0 * E_CHARGE
    dens = (1e25, 1e26, 5e24)        # m^-3
    temps = (500.0, 500.0, 500.0)
    drifts = (655e3, 0.0, -655e3)
    rng = np.random.Generator(np.random.PCG64(seed_data))
    pops = _populations(rng, m, (n_a, n_b, n_c), dens, temps, drifts, cell_volume, n_cells)
    per_cell = [n_a, n_b + n_c]      # species alpha, beta
    n = n_cells * (n_a + n_b + n_c)
    w = np.empty(n)
    v = np.empty((3, n))
    pop = np.empty(n, np.int8)
    species = np.empty(n, np.int32)
    cells = np.empty(n, np.int32)
    pos = 0
    cursor = [0, 0, 0]
    for c in range(n_cells):
        for k, npk in ((0, n_a), (1, n_b), (2, n_c)):
            sl = slice(pos, pos + npk)
            src = slice(cursor[k], cursor[k] + npk)
            w[sl] = pops[k][0][src]
            v[:, sl] = pops[k][1][:, src]
            pop[sl] = k
            species[sl] = 0 if k == 0 else 1
            cells[sl] = c
            cursor[k] += npk
            pos += npk
    offsets = np.zeros(2 * n_cells + 1, dtype=np.int64)
    np.cumsum(np.tile(per_cell, n_cells), out=offsets[1:])
    wl = Workload(name="paper Test 2 (%s), %d cells x (%d A | %d B + %d C) C6+"
                  % (case, n_cells, n_a, n_b, n_c),
                  n_cells=n_cells, n_species=2, offsets=offsets, cells=cells, species=species,
                  w=w, vx=v[0].copy(), vy=v[1].copy(), vz=v[2].copy(),
                  mass=np.array([m, m]), charge=np.array([q, q]),
                  collisions=[(0, 0), (1, 1), (0, 1)], dt=50e-15, coulomb_log=10.0,
                  method=method, eps0=EPS0_SI, cell_volume=cell_volume, f_E=0.05,
                  seed=PHILOX_SEED_BASE + 0x72, steps=1)
    wl.extra = dict(population=pop, densities=dens, temperatures_ev=temps, drifts=drifts)
    return wl


# Test 3 (Sec. 5.3): N_i, N_e per cell and whether the moment correction runs
PAPER_T3_CASES = {
    "T3a": (512, 3072, True),
    "T3b": (512, 512, False),
    "T3c": (512, 512, True),
}
PAPER_T3_DX = 1.3285e-9  # m, the grid spacing


def paper_test3(case: str = "T3a", n_cells: int = 1600, seed_data: int = 13,
                method: int = N97) -> Workload:
    """Test 3 in SI units: electron-ion thermalization of fully ionized
    carbon (Z = 6, M_i = 12 m_u - 6 m_e), non-drifting Maxwellians with
    n_i = 1e23 cm^-3, T_i = 50 eV, n_e = 6e23 cm^-3, T_e = 150 eV; lnL = 3,
    dt = 3.54e-4 fs, on the 40 x 40 grid of cells of side 1.3285 nm (taken as
    cubes).  Species 0 is the electrons, 1 the ions; collisions (e, e),
    (i, i), (e, i).  T3a weighs both species equally (N_e = 6 N_i); T3b and
    T3c use N_e = N_i, so w_e = 6 w_i, without and with the correction
    (extra["moment_correction"])."""
    n_i, n_e, corr = PAPER_T3_CASES[case]
    m_i = 12.0 * M_U - 6.0 * M_ELECTRON
    dv = PAPER_T3_DX ** 3
    rng = np.random.Generator(np.random.PCG64(seed_data))
    (w_e, v_e), (w_i, v_i) = _populations(rng, M_ELECTRON, (n_e,), (6e29,), (150.0,), (0.0,),
                                          dv, n_cells) + \
        _populations(rng, m_i, (n_i,), (1e29,), (50.0,), (0.0,), dv, n_cells)
    per = n_e + n_i
    n = n_cells * per
    w = np.empty(n)
    v = np.empty((3, n))
    lay = np.concatenate([np.zeros(n_e, np.int32), np.ones(n_i, np.int32)])
    species = np.tile(lay, n_cells)
    cells = np.repeat(np.arange(n_cells, dtype=np.int32), per)
    ie = species == 0
    w[ie], w[~ie] = w_e, w_i
    v[:, ie], v[:, ~ie] = v_e, v_i
    offsets = np.zeros(2 * n_cells + 1, dtype=np.int64)
    np.cumsum(np.tile([n_e, n_i], n_cells), out=offsets[1:])
    wl = Workload(name="paper Test 3 (%s), %d cells x (%d e + %d C6+)" % (case, n_cells, n_e, n_i),
                  n_cells=n_cells, n_species=2, offsets=offsets, cells=cells, species=species,
                  w=w, vx=v[0].copy(), vy=v[1].copy(), vz=v[2].copy(),
                  mass=np.array([M_ELECTRON, m_i]), charge=np.array([-E_CHARGE, 6.0 * E_CHARGE]),
                  collisions=[(0, 0), (1, 1), (0, 1)], dt=3.54e-19, coulomb_log=3.0,
                  method=method, eps0=EPS0_SI, cell_volume=dv, f_E=0.05,
                  seed=PHILOX_SEED_BASE + 0x73, steps=1)
    wl.extra = dict(moment_correction=corr, densities=(6e29, 1e29), temperatures_ev=(150.0, 50.0))
    return wl


def species_temperatures(wl: Workload, v: np.ndarray) -> Tuple[float, float]:
    """Weighted temperatures [eV] of species 0 and 1 over the whole grid,
    each about its own mean velocity."""
    out = []
    for s in (0, 1):
        sel = wl.species == s
        w = wl.w[sel]
        vv = v[:, sel]
        u = (vv * w).sum(1) / w.sum()
        d = vv - u[:, None]
        out.append(wl.mass[s] * (w * (d * d).sum(0)).sum() / w.sum() / 3.0 / E_CHARGE)
    return out[0], out[1]


def population_moments(wl: Workload, v: np.ndarray) -> dict:
    """Per population of a paper test: density-weighted mean x-velocity [m/s]
    and temperature [eV] about that mean (all cells together)."""
    pop = wl.extra["population"]
    m = wl.mass[wl.species]
    out = {}
    for k in np.unique(pop):
        sel = pop == k
        wk = wl.w[sel]
        mean = (v[:, sel] * wk).sum(1) / wk.sum()
        d2 = ((v[:, sel] - mean[:, None]) ** 2).sum(0)
        out[int(k)] = (mean[0], (m[sel] * wk * d2).sum() / (3.0 * wk.sum()) / E_CHARGE)
    return out


def standard_normal_state(wl: Workload, seed_data: int) -> np.ndarray:
    """Fixed xi ~ N(0,1)^{3 x n} for the reparameterized initial state
    v0 = sqrt(T0/m) xi of the differentiated relaxation."""
    rng = np.random.Generator(np.random.PCG64(seed_data + 777))
    return rng.normal(0.0, 1.0, size=(3, wl.n))


def make(config: int, **kw) -> Workload:
    return {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}[config](**kw)


def temperature(wl: Workload, species: int, vx=None, vy=None, vz=None) -> np.ndarray:
    """Weighted per-species temperature components (T_x, T_y, T_z) about the
    species' weighted mean velocity (diagnostic)."""
    vx = wl.vx if vx is None else vx
    vy = wl.vy if vy is None else vy
    vz = wl.vz if vz is None else vz
    sel = wl.species == species
    w = wl.w[sel]
    m = wl.mass[species]
    out = []
    for v in (vx[sel], vy[sel], vz[sel]):
        mean = np.sum(w * v) / np.sum(w)
        out.append(m * np.sum(w * (v - mean) ** 2) / np.sum(w))
    return np.array(out)
