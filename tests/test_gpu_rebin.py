"""Incremental re-binning (mcc_rebin) against the oracle's stable binning.

After a push, the particle at grouped position p goes to cell cells_new[p]
(its species unchanged).  The new grouping must be exactly what binning the
current order from scratch gives: offsets by (cell, species) and, inside
every group, ascending current position.  The oracle's counting sort is
that definition; offsets and permutation are compared bit for bit, and the
payload must come out as the old arrays gathered through the permutation,
in place (mcc_rebin) and into separate output arrays (mcc_rebin_out, which
must leave its inputs untouched).
Cases: no movers, neighbour moves at several rates, far jumps, every
particle moving, emptied and newly filled groups, one cell, three species,
no particles, long arrival lists (sorted in LDS and in place), long runs of
empty groups, a cells array that is not 16-byte aligned, and cell ids out of
range (reported; such particles stay).
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_19151_amd import native
    c = native.Context()
    yield c
    c.close()


def _population(rng, n_cells, S, mean, empty_frac=0.1):
    counts = rng.poisson(mean, size=(n_cells, S))
    counts[rng.uniform(size=(n_cells, S)) < empty_frac] = 0
    flat = counts.reshape(-1)
    off = np.zeros(flat.size + 1, dtype=np.int64)
    np.cumsum(flat, out=off[1:])
    cell = np.repeat(np.repeat(np.arange(n_cells, dtype=np.int32), S), flat)
    sp = np.repeat(np.tile(np.arange(S, dtype=np.int32), n_cells), flat)
    return off, cell, sp


def _push(rng, cell, n_cells, frac, far=0.1):
    new = cell.copy()
    mv = rng.uniform(size=cell.size) < frac
    jump = rng.uniform(size=cell.size) < far
    step = np.where(rng.uniform(size=cell.size) < 0.5, -1, 1)
    new[mv] = (cell[mv] + step[mv]) % n_cells
    sel = mv & jump
    new[sel] = rng.integers(0, n_cells, size=int(sel.sum()))
    return new.astype(np.int32)


def _check(ctx, off, sp, cells_new, n_cells, S, expect_err=0, keep=None):
    import torch
    n = cells_new.size
    rng = np.random.default_rng(n)
    pay = [rng.normal(size=n) for _ in range(4)]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    tp = [dev(a) for a in pay]
    print("rebin case: n=%d cells=%d S=%d movers=%d" % (n, n_cells, S, int(
        (cells_new != np.repeat(np.repeat(np.arange(n_cells), S), np.diff(off))).sum())),
        flush=True)
    off_new, perm = ctx.rebin(dev(off), dev(cells_new), n_cells, S, *tp)
    torch.cuda.synchronize()
    assert ctx.device_error() == expect_err
    ref_cells = cells_new if keep is None else keep
    ref_off, ref_perm = oracle.bin_particles(ref_cells, sp, n_cells, S)
    assert np.array_equal(off_new.cpu().numpy(), ref_off)
    assert np.array_equal(perm.cpu().numpy().astype(np.int64), ref_perm)
    for a, t in zip(pay, tp):
        assert np.array_equal(t.cpu().numpy(), a[ref_perm])
    # out of place, from the original payload
    tin = [dev(a) for a in pay]
    tout = [torch.full_like(t, np.nan) for t in tin]
    off2, perm2 = ctx.rebin_out(dev(off), dev(cells_new), n_cells, S, *tin, *tout)
    torch.cuda.synchronize()
    assert ctx.device_error() == expect_err
    assert np.array_equal(off2.cpu().numpy(), ref_off)
    assert np.array_equal(perm2.cpu().numpy().astype(np.int64), ref_perm)
    for a, ti, to in zip(pay, tin, tout):
        assert np.array_equal(ti.cpu().numpy(), a)
        assert np.array_equal(to.cpu().numpy(), a[ref_perm])


@pytest.mark.parametrize("frac", [0.0, 0.01, 0.05, 0.3, 1.0])
def test_rebin_is_the_stable_binning(ctx, frac):
    rng = np.random.default_rng(int(frac * 1000) + 1)
    n_cells, S = 3000, 2
    off, cell, sp = _population(rng, n_cells, S, 40)
    _check(ctx, off, sp, _push(rng, cell, n_cells, frac), n_cells, S)


def test_rebin_edge_cases(ctx):
    rng = np.random.default_rng(7)
    # one cell, three species: nobody can move
    off, cell, sp = _population(rng, 1, 3, 50, empty_frac=0.0)
    _check(ctx, off, sp, cell.copy(), 1, 3)
    # everybody leaves cell 0 for cell 5, which was empty; others jump far
    off, cell, sp = _population(rng, 8, 3, 30, empty_frac=0.0)
    counts = np.diff(off).reshape(8, 3)
    assert counts[5].sum() > 0
    new = cell.copy()
    new[cell == 0] = 5
    new[cell == 5] = 1
    _check(ctx, off, sp, new.astype(np.int32), 8, 3)
    # many arrivals into one group (about 2500 per species: the sort of long
    # arrival lists in LDS), and about 12000 (the same sort in place)
    off, cell, sp = _population(rng, 50, 2, 100, empty_frac=0.0)
    new = np.where(rng.uniform(size=cell.size) < 0.5, 7, cell).astype(np.int32)
    _check(ctx, off, sp, new, 50, 2)
    off, cell, sp = _population(rng, 240, 2, 100, empty_frac=0.0)
    new = np.where(rng.uniform(size=cell.size) < 0.5, 11, cell).astype(np.int32)
    _check(ctx, off, sp, new, 240, 2)
    # long runs of empty groups (hundreds inside one chunk of positions, and
    # chunks that start inside a run), some movers landing in them
    n_cells, S = 6000, 2
    counts = rng.poisson(30, size=(n_cells, S))
    counts[500:2500] = 0
    counts[3000:3400, 1] = 0
    counts[rng.uniform(size=(n_cells, S)) < 0.3] = 0
    flat = counts.reshape(-1)
    off = np.zeros(flat.size + 1, dtype=np.int64)
    np.cumsum(flat, out=off[1:])
    cell = np.repeat(np.repeat(np.arange(n_cells, dtype=np.int32), S), flat)
    sp = np.repeat(np.tile(np.arange(S, dtype=np.int32), n_cells), flat)
    new = _push(rng, cell, n_cells, 0.05, far=0.5)
    _check(ctx, off, sp, new, n_cells, S)
    # no particles
    off = np.zeros(2 * 4 + 1, dtype=np.int64)
    _check(ctx, off, np.zeros(0, np.int32), np.zeros(0, np.int32), 4, 2)


def test_rebin_cell_out_of_range_is_reported_and_kept(ctx):
    rng = np.random.default_rng(9)
    n_cells, S = 200, 2
    off, cell, sp = _population(rng, n_cells, S, 20)
    new = _push(rng, cell, n_cells, 0.05)
    bad = rng.choice(cell.size, size=5, replace=False)
    new[bad[:3]] = n_cells + 3
    new[bad[3:]] = -1
    keep = new.copy()
    keep[bad] = cell[bad]
    _check(ctx, off, sp, new, n_cells, S, expect_err=3, keep=keep)


def test_rebin_out_rejects_an_output_that_is_an_input(ctx):
    import torch
    from paper_2407_19151_amd import native
    rng = np.random.default_rng(12)
    off, cell, sp = _population(rng, 10, 2, 5, empty_frac=0.0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    tin = [dev(rng.normal(size=cell.size)) for _ in range(4)]
    tout = [torch.empty_like(t) for t in tin]
    tout[2] = tin[0]
    with pytest.raises(native.MCCError) as e:
        ctx.rebin_out(dev(off), dev(cell), 10, 2, *tin, *tout)
    assert e.value.code == -1


def test_rebin_full_size_population(ctx):
    """The benchmark's population (65 536 cells, 2.15e7 particles) with 2 % of
    the particles moving to a neighbouring cell."""
    from paper_2407_19151_amd import workloads as W
    wl = W.config3()
    rng = np.random.default_rng(11)
    cell = wl.cells.astype(np.int32)
    _check(ctx, wl.offsets, wl.species.astype(np.int32), _push(rng, cell, wl.n_cells, 0.02),
           wl.n_cells, wl.n_species)


def test_rebin_reads_cells_at_any_alignment(ctx):
    """cells_new one element into a larger array (4-byte aligned only)."""
    import torch
    rng = np.random.default_rng(13)
    n_cells, S = 700, 2
    off, cell, sp = _population(rng, n_cells, S, 30)
    new = _push(rng, cell, n_cells, 0.05)
    big = torch.from_numpy(np.concatenate([[0], new]).astype(np.int32)).cuda()
    view = big[1:]
    assert view.data_ptr() % 16 != 0
    off_new, perm = ctx.rebin(torch.from_numpy(off).cuda(), view, n_cells, S)
    torch.cuda.synchronize()
    assert ctx.device_error() == 0
    ref_off, ref_perm = oracle.bin_particles(new, sp, n_cells, S)
    assert np.array_equal(off_new.cpu().numpy(), ref_off)
    assert np.array_equal(perm.cpu().numpy().astype(np.int64), ref_perm)
