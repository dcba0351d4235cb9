"""Parity at the benchmark's full size.

The 65,536-cell lognormal workload (2.15e7 electrons and ions, cells of 16 to
4096 particles) is stepped by a plan exactly as the benchmark times it: one
graph replay with the built-in variant table, in the FP32-kinematics and in
the FP64 form.  Two checks follow.

- Sampled outputs: the oracle recomputes a seeded sample of cells one by one
  (every size bucket, plus the largest cells), from the same state and with
  the same global cell ids.  Those cells' velocities are compared at the
  parity bars of the smaller tests.
- Properties of the whole state, which hold at any size: every velocity is
  finite, and every cell conserves its momentum and kinetic energy to
  rounding, whether its collisions were corrected or reset.
"""
import dataclasses

import numpy as np
import pytest

from paper_2407_19151_amd import workloads as W

from gpu_helpers import FP64_TOL, check_parity, oracle_step

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-4
FIRST_STEP = 1000  # the benchmark's first timed step
BUCKETS = [16, 128, 256, 512, 1024, 2048, 4096]


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_19151_amd import native
    c = native.Context()
    yield c
    c.close()


@pytest.fixture(scope="module")
def full():
    return W.config3()


def _sample_cells(wl, per_bucket=6, largest=2, seed=21):
    sizes = np.diff(wl.offsets[::wl.n_species])
    rng = np.random.default_rng(seed)
    out = []
    for lo, hi in zip(BUCKETS[:-1], BUCKETS[1:]):
        ids = np.nonzero((sizes > lo) & (sizes <= hi))[0]
        if ids.size:
            out.extend(rng.choice(ids, size=min(per_bucket, ids.size), replace=False).tolist())
    out.extend(np.argsort(sizes)[-largest:].tolist())
    return np.unique(np.asarray(out, dtype=np.int64))


def _subset(wl, cells):
    """The sampled cells' particles in a workload of the same n_cells (all
    other cells empty), so that the oracle sees the global cell ids."""
    S = wl.n_species
    grp = (cells[:, None] * S + np.arange(S)[None, :]).reshape(-1)
    starts, ends = wl.offsets[grp], wl.offsets[grp + 1]
    idx = np.concatenate([np.arange(a, b) for a, b in zip(starts, ends)])
    counts = np.zeros(wl.n_cells * S, dtype=np.int64)
    counts[grp] = ends - starts
    offsets = np.zeros(counts.size + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    sub = dataclasses.replace(wl, offsets=offsets, cells=wl.cells[idx].copy(),
                              species=wl.species[idx].copy(), w=wl.w[idx].copy(),
                              vx=wl.vx[idx].copy(), vy=wl.vy[idx].copy(), vz=wl.vz[idx].copy())
    return sub, idx


def _cell_moments(wl, v):
    """Per cell: total momentum (3) and kinetic energy, and the scales
    sum m w |v| and sum m w |v|^2 / 2 they are compared against."""
    m = wl.mass[wl.species] * wl.w
    c = wl.cells.astype(np.int64)
    P = np.stack([np.bincount(c, m * v[k], wl.n_cells) for k in range(3)])
    sp2 = (v * v).sum(0)
    E = np.bincount(c, 0.5 * m * sp2, wl.n_cells)
    Ps = np.bincount(c, m * np.sqrt(sp2), wl.n_cells)
    return P, E, Ps


@pytest.mark.parametrize("mode", ["fp32", "fp64"])
def test_full_workload_sampled_cells_and_conservation(ctx, full, mode):
    from paper_2407_19151_amd import native, runner
    wl = full
    prec = native.MCC_FP32_KINEMATICS if mode == "fp32" else native.MCC_FP64
    dw = runner.DeviceWorkload(wl)
    plan = runner.make_plan(ctx, dw, params=runner.params_for(wl, precision=prec),
                            autotune=False)
    try:
        plan.run(FIRST_STEP, 1)
        vg = dw.velocities()
    finally:
        plan.close()
    assert ctx.device_error() == 0
    v0 = wl.velocities()
    print("%s: %d cells, %d particles stepped" % (mode, wl.n_cells, wl.n), flush=True)

    # properties of the whole state
    assert np.all(np.isfinite(vg))
    P0, E0, Ps = _cell_moments(wl, v0)
    P1, E1, _ = _cell_moments(wl, vg)
    dP = np.abs(P1 - P0).max(0) / np.maximum(Ps, 1e-300)
    dE = np.abs(E1 - E0) / np.maximum(E0, 1e-300)
    print("  per-cell conservation: max |dP|/sum m w |v| %.2e, max |dE|/E %.2e"
          % (dP.max(), dE.max()), flush=True)
    assert dP.max() < 1e-13 and dE.max() < 1e-13

    # sampled cells against the oracle
    cells = _sample_cells(wl)
    sub, idx = _subset(wl, cells)
    ref = sub.copy()
    oracle_step(ref, FIRST_STEP, uniform23=(mode == "fp32"))

    def rerun(p):
        oracle_step(p, FIRST_STEP, uniform23=(mode == "fp32"))
        return p.velocities()

    info = check_parity(sub, vg[:, idx], ref.velocities(), sub.velocities(),
                        tol=FP32_TOL if mode == "fp32" else FP64_TOL,
                        cond_tol=FP32_TOL if mode == "fp32" else 1e-6, rerun=rerun)
    print("  %d sampled cells (%d particles, largest %d): %s"
          % (cells.size, idx.size, int(np.diff(wl.offsets[::wl.n_species])[cells].max()), info),
          flush=True)


def test_sharded_calls_equal_one_call(ctx, full):
    """Cells are independent and every random number is keyed by the global
    cell id and the particle's index in its cell, so a population split into
    cell ranges (here 4, balanced by particle count) and stepped in separate
    calls gives the one-call result bit for bit.  A shard passes its own
    particles with the full-length offsets array, in which the cells of the
    other shards are empty (they are bucketed out and cost nothing); this is
    how a rank of a multi-GPU run would call the library."""
    import torch
    from paper_2407_19151_amd import native, runner
    wl = full
    S = wl.n_species
    params = runner.params_for(wl, precision=native.MCC_FP32_KINEMATICS)
    one = runner.DeviceWorkload(wl)
    runner.collide_sorted(ctx, one, FIRST_STEP, params=params)
    v_one = one.velocities()
    st_one = native.read_stats(one.stats)
    cc_one = one.cell_corr.cpu().numpy()
    del one
    cell_start = wl.offsets[::S]
    bounds = np.searchsorted(cell_start, np.linspace(0, wl.n, 5)[1:-1])
    ranges = list(zip(np.r_[0, bounds], np.r_[bounds, wl.n_cells]))
    v_sh = np.zeros_like(v_one)
    pairs = 0
    cc_sh = np.zeros(wl.n_cells, dtype=np.int32)
    for c0, c1 in ranges:
        p0, p1 = int(wl.offsets[c0 * S]), int(wl.offsets[c1 * S])
        print("shard cells [%d, %d) particles [%d, %d)" % (c0, c1, p0, p1), flush=True)
        sub = wl.copy()
        sub.offsets = np.clip(wl.offsets - p0, 0, p1 - p0)
        for k in ("cells", "species", "w", "vx", "vy", "vz"):
            setattr(sub, k, getattr(wl, k)[p0:p1].copy())
        dw = runner.DeviceWorkload(sub)
        runner.collide_sorted(ctx, dw, FIRST_STEP, params=params)
        v_sh[:, p0:p1] = dw.velocities()
        pairs += native.read_stats(dw.stats)["pairs"]
        cc = dw.cell_corr.cpu().numpy()
        cc_sh[c0:c1] = cc[c0:c1]
        assert np.all(cc[:c0] == 0) and np.all(cc[c1:] == 0)
        del dw
        torch.cuda.empty_cache()
    assert ctx.device_error() == 0
    assert np.array_equal(v_sh, v_one)
    assert pairs == st_one["pairs"]
    assert np.array_equal(cc_sh, cc_one)
