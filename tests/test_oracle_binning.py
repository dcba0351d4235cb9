"""Pins of the oracle's grouping (the unsorted entry) and of its options
that do not change the arithmetic of a cell.

- Binning: the offsets of every (cell, species) group are the prefix sums of
  the group counts, and the permutation is numpy's stable argsort of the
  group key cell * S + species: groups ascending, ascending particle index
  inside a group (the particles of a cell, Sec. 2; the order inside a group
  is the canonical one every random number is keyed from).
- The unsorted step is the sorted step on the gathered arrays, scattered
  back: checked bit for bit against a gather and scatter done with numpy.
- Threads: cells are independent and every random number is keyed by its
  cell, so the cell loop's thread count changes nothing, bit for bit.
- The FP32-kinematics uniforms: the 23-bit form keeps N97's mean deflection
  <cos chi> = exp(-s) (the pin of the 32-bit form) and bounds the sampled
  1 - cos chi by ln(2^24) / A (the top uniform is 1 - 2^-24).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2407_19151_amd import workloads as W


def _random_ids(n, n_cells, S, seed, clustered=False):
    rng = np.random.default_rng(seed)
    if clustered:  # runs of equal keys, as a particle code's arrays often hold
        cells = np.repeat(rng.integers(0, n_cells, size=n // 8 + 1), 8)[:n]
    else:
        cells = rng.integers(0, n_cells, size=n)
    species = rng.integers(0, S, size=n)
    return cells.astype(np.int32), species.astype(np.int32)


@pytest.mark.parametrize("n,n_cells,S,clustered", [(0, 3, 1, False), (1, 1, 1, False),
                                                   (1000, 7, 2, False), (5000, 300, 3, True),
                                                   (20000, 64, 8, False)])
def test_bin_is_numpy_stable_argsort(n, n_cells, S, clustered):
    cells, species = _random_ids(n, n_cells, S, seed=n + S, clustered=clustered)
    off, perm = oracle.bin_particles(cells, species, n_cells, S)
    key = cells.astype(np.int64) * S + species
    assert np.array_equal(perm, np.argsort(key, kind="stable"))
    want = np.zeros(n_cells * S + 1, dtype=np.int64)
    want[1:] = np.cumsum(np.bincount(key, minlength=n_cells * S))
    assert np.array_equal(off, want)


def test_bin_rejects_ids_out_of_range():
    cells = np.array([0, 3], dtype=np.int32)
    species = np.array([0, 0], dtype=np.int32)
    with pytest.raises(oracle.OracleError):
        oracle.bin_particles(cells, species, 3, 1)


@pytest.mark.parametrize("relativistic", [False, True])
def test_unsorted_step_is_sorted_step_on_gathered_arrays(relativistic):
    base = W.config4(n_cells=6) if relativistic else W.config2(n_cells=12)
    wl = base.unsorted(seed=7)
    key = wl.cells.astype(np.int64) * wl.n_species + wl.species
    perm = np.argsort(key, kind="stable")
    off = np.zeros(wl.n_cells * wl.n_species + 1, dtype=np.int64)
    off[1:] = np.cumsum(np.bincount(key, minlength=wl.n_cells * wl.n_species))
    kw = dict(dt=wl.dt, coulomb_log=wl.coulomb_log, seed=wl.seed, step=3, method=wl.method,
              relativistic=wl.relativistic, c=wl.c, eps0=wl.eps0,
              cell_volume=wl.cell_volume, f_E=wl.f_E)
    g = [np.ascontiguousarray(a[perm]) for a in (wl.w, wl.vx, wl.vy, wl.vz)]
    so = oracle.collide_sorted(off, wl.mass, wl.charge, wl.collisions, *g, **kw)
    want = [np.empty_like(wl.vx) for _ in range(3)]
    for d in range(3):
        want[d][perm] = g[d + 1]
    su = oracle.collide(wl.cells, wl.species, wl.n_cells, wl.mass, wl.charge, wl.collisions,
                        wl.w, wl.vx, wl.vy, wl.vz, **kw)
    for d, v in enumerate((wl.vx, wl.vy, wl.vz)):
        assert np.array_equal(v, want[d])
    assert su["pairs"] == so["pairs"] and su["corr_pairs"] == so["corr_pairs"]
    assert np.array_equal(su["cell_corr_pairs"], so["cell_corr_pairs"])


@pytest.mark.parametrize("maker", [lambda: W.config2(n_cells=48), lambda: W.config4(n_cells=8),
                                   lambda: W.config3(n_cells=64)])
def test_thread_count_changes_nothing(maker):
    runs = []
    for threads in (1, 5):
        wl = maker()
        oracle.set_threads(threads)
        try:
            st = oracle.run_workload(wl, steps=2, first_step=4)
        finally:
            oracle.set_threads(1)
        runs.append((wl.velocities(), st))
    (v1, s1), (v5, s5) = runs
    assert np.array_equal(v1, v5)
    for k in ("pairs", "corr_pairs", "failed", "collisions"):
        assert s1[k] == s5[k]
    assert np.array_equal(s1["cell_corr_pairs"], s5["cell_corr_pairs"])


def test_uniform23_keeps_the_n97_mean_deflection():
    """One e-e pair per cell, many cells: with the 23-bit uniforms the mean
    cos of the deflection of u is exp(-s) (s known per pair), and no pair
    deflects past 1 - cos chi = ln(2^24)/A."""
    ncell = 40000
    rng = np.random.default_rng(3)
    u = rng.normal(size=(ncell, 3))
    v = np.zeros((2 * ncell, 3))
    v[0::2] = 0.5 * u
    v[1::2] = -0.5 * u
    vx, vy, vz = (np.ascontiguousarray(v[:, d]) for d in range(3))
    w = np.ones(2 * ncell)
    off = np.arange(ncell + 1, dtype=np.int64) * 2
    dt = 0.02
    oracle.collide_sorted(off, [1.0], [-1.0], [(0, 0)], w, vx, vy, vz, dt=dt, coulomb_log=10.0,
                          seed=5, step=0, correction=False, uniform23=True)
    un = np.stack([vx[0::2] - vx[1::2], vy[0::2] - vy[1::2], vz[0::2] - vz[1::2]], 1)
    um = np.linalg.norm(u, axis=1)
    cosx = np.sum(un * u, 1) / (um * np.linalg.norm(un, axis=1))
    s = 10.0 * 1.0 * dt / (4 * math.pi * 0.25 * um ** 3)  # Eq. (12), N_min w_max / dV = 1
    # E[cos chi | s] = exp(-s): the mean of cos - exp(-s) is 0 within its sampling sd
    r = cosx - np.exp(-s)
    assert abs(r.mean()) < 5 * r.std() / math.sqrt(ncell)
    A = np.array([oracle.n97_A(x) for x in s])
    big = A > 0  # (A = 0: isotropic, no bound)
    assert np.all(1 - cosx[big] <= math.log(2.0 ** 24) / A[big] * (1 + 1e-9) + 1e-12)
