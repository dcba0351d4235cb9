"""GPU parity: the HIP library against the CPU FP64 oracle on the same seeded
inputs and the same Philox draws, called through the C ABI."""
import math

import numpy as np
import pytest

import oracle
from paper_2407_19151_amd import workloads as W

from gpu_helpers import (FP64_TOL, check_counts, check_parity, custom_workload, oracle_step,
                         rel_err)

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


def _gpu_step(ctx, wl, step, **pover):
    from paper_2407_19151_amd import native, runner
    dw = runner.DeviceWorkload(wl)
    runner.collide_sorted(ctx, dw, step, params=runner.params_for(wl, **pover))
    v = dw.velocities()
    st = native.read_stats(dw.stats)
    cc = dw.cell_corr.cpu().numpy()
    assert ctx.device_error() == 0
    return v, st, cc


def _parity(ctx, wl, step=0, tol=FP64_TOL, counts_exact=True, **over):
    v0 = wl.velocities().copy()
    print("parity case: %s cells=%d n=%d step=%d %s" % (wl.name, wl.n_cells, wl.n, step, over),
          flush=True)
    vg, sg, cg = _gpu_step(ctx, wl, step, **over)
    ref = wl.copy()
    oover = {k: v for k, v in over.items() if k not in ("precision", "diagnostics")}
    if "on_failure" in oover:
        oover["keep_on_fail"] = oover.pop("on_failure") == 1
    if "moment_correction" in oover:
        oover["correction"] = oover.pop("moment_correction")
    so = oracle_step(ref, step, **oover)
    vr = ref.velocities()

    def rerun(p):
        oracle_step(p, step, **oover)
        return p.velocities()

    info = check_parity(wl, vg, vr, v0, tol=tol, rerun=rerun)
    print("  parity:", info, flush=True)
    assert sg["pairs"] == so["pairs"]
    assert sg["collisions"] == so["collisions"]
    if counts_exact:
        assert sg["failed"] == so["failed"]

        def rerun_counts(p):
            return oracle_step(p, step, **oover)["cell_corr_pairs"]

        nd = check_counts(wl, cg, so["cell_corr_pairs"], rerun_counts)
        assert int(sg["corr_pairs"]) == int(np.sum(cg))
        if nd == 0:
            assert int(sg["corr_pairs"]) == so["corr_pairs"]
    return info, sg, so


@pytest.mark.parametrize("method", [W.N97, W.TA77])
def test_parity_config1_one_species_lognormal(ctx, method):
    wl = W.config1(method=method)
    for step in (0, 7):
        _parity(ctx, wl.copy(), step)


@pytest.mark.parametrize("method", [W.N97, W.TA77])
def test_parity_config2_subset_two_species(ctx, method):
    wl = W.config2(n_cells=48, method=method)
    _parity(ctx, wl, 3)


def test_parity_every_bucket_and_ragged_edges(ctx):
    """Cells spanning every size bucket and variant (LDS and global
    scratch), odd and even counts, empty species, single particles, N_min = 1."""
    sizes = [(0, 0), (1, 0), (0, 1), (1, 1), (2, 0), (3, 0), (2, 1), (1, 5), (5, 1), (3, 3),
             (7, 9), (64, 63), (65, 64), (100, 27), (129, 128), (200, 55), (255, 256),
             (300, 211), (511, 512), (700, 300), (1000, 1), (1023, 1024), (1500, 547),
             (2047, 2048), (2500, 1500), (1, 3000)]
    wl = custom_workload(sizes, seed=4)
    _parity(ctx, wl, 1)


def test_parity_large_global_scratch_cells(ctx):
    sizes = [(3000, 1095), (5000, 4000), (100, 16000)]
    wl = custom_workload(sizes, seed=5)
    _parity(ctx, wl, 2)


def test_degenerate_steps_leave_the_state_unchanged(ctx):
    """dt = 0 and lnL = 0 make every s zero; a cold cell (all velocities
    equal) has no relative velocity: the step must return the input bit for
    bit, with no correction pairs and no failures.  A cell where a pair has
    identical velocities is otherwise stepped like any other (against the
    oracle)."""
    from paper_2407_19151_amd import native, runner
    wl = custom_workload([(20, 10), (5, 5), (300, 200)], seed=49)
    for over in (dict(dt=0.0), dict(coulomb_log=0.0)):
        w2 = wl.copy()
        for k, v in over.items():
            setattr(w2, k, v)
        dw = runner.DeviceWorkload(w2)
        runner.collide_sorted(ctx, dw, 0)
        assert ctx.device_error() == 0
        assert np.array_equal(dw.velocities(), w2.velocities()), over
        st = native.read_stats(dw.stats)
        assert st["corr_pairs"] == 0 and st["failed"] == 0
    cold = wl.copy()
    cold.vx = np.full(cold.n, 0.3)
    cold.vy = np.full(cold.n, -0.1)
    cold.vz = np.full(cold.n, 0.2)
    dw = runner.DeviceWorkload(cold)
    runner.collide_sorted(ctx, dw, 0)
    assert np.array_equal(dw.velocities(), cold.velocities())
    twin = wl.copy()
    twin.vx = twin.vx.copy()
    twin.vy = twin.vy.copy()
    twin.vz = twin.vz.copy()
    for a in (twin.vx, twin.vy, twin.vz):
        a[1] = a[0]   # two particles of cell 0, species 0, at one velocity
    _parity(ctx, twin, 3)


@pytest.mark.parametrize("bad", [0.0, -1.0, float("nan"), float("inf")])
def test_weight_not_positive_and_finite_is_reported(ctx, bad):
    """Weights are densities (sum w / dV): a zero, negative, NaN or infinite
    weight is a data error (code 4), reported by the plain call and once by a
    plan's creation; the oracle rejects the same input."""
    import oracle as orc
    from paper_2407_19151_amd import runner
    wl = custom_workload([(20, 10), (5, 5)], seed=50)
    wl.w = wl.w.copy()
    wl.w[7] = bad
    dw = runner.DeviceWorkload(wl)
    runner.collide_sorted(ctx, dw, 0)
    assert ctx.device_error() == 4
    plan = runner.make_plan(ctx, runner.DeviceWorkload(wl), autotune=False)
    plan.close()
    assert ctx.device_error() == 4
    with pytest.raises(orc.OracleError):
        oracle_step(wl.copy(), 0)


def test_parity_at_the_maximum_cell_and_one_past_it(ctx):
    """A cell of exactly MCC_MAX_CELL particles is stepped like any other; a
    cell one particle larger is skipped (left unchanged) and reported as code
    2, while the cells around it are still stepped."""
    from paper_2407_19151_amd import native
    sizes = [(16384, 16384), (50, 30)]
    wl = custom_workload(sizes, seed=47)
    _parity(ctx, wl, 1)
    over = custom_workload([(40, 20), (16385, 16384), (70, 35)], seed=48)
    v0 = over.velocities().copy()
    vg, _, _ = _gpu_step_unchecked(ctx, over, 2)
    assert ctx.device_error() == 2
    big = over.cells == 1
    assert np.array_equal(vg[:, big], v0[:, big])
    ref = over.copy()
    oracle_step(ref, 2, cells=[0, 2])
    info = check_parity(over, vg, ref.velocities(), v0)
    print("  cells around the over-size one: %s" % info, flush=True)


def _gpu_step_unchecked(ctx, wl, step, **pover):
    from paper_2407_19151_amd import native, runner
    dw = runner.DeviceWorkload(wl)
    runner.collide_sorted(ctx, dw, step, params=runner.params_for(wl, **pover))
    return dw.velocities(), native.read_stats(dw.stats), dw.cell_corr.cpu().numpy()


@pytest.mark.parametrize("wmode", ["lognormal", "two", "clustered", "equal"])
def test_parity_weight_orders(ctx, wmode):
    """Distinct weights (bucket order), two weight classes (crowded bucket:
    one pass per weight value), 40 clustered values (crowded bucket with too
    many values: bitonic network), equal weights (shuffled order)."""
    sizes = [(300, 200), (97, 64), (512, 512), (40, 3)]
    wl = custom_workload(sizes, seed=6, weight_mode=wmode)
    _parity(ctx, wl, 0)
    _parity(ctx, wl.copy(), 5, sort_by_weight=False)


def test_parity_options(ctx):
    wl = W.config2(n_cells=16)
    _parity(ctx, wl.copy(), 1, moment_correction=False)
    _parity(ctx, wl.copy(), 1, on_failure=1)
    _parity(ctx, wl.copy(), 1, max_passes=3)
    _parity(ctx, wl.copy(), 1, f_E=0.02)


def test_parity_three_species_and_collision_order(ctx):
    sizes = [(40, 30, 20), (7, 0, 5), (100, 101, 3)]
    wl = custom_workload(sizes, seed=7, masses=(1.0, 4.0, 50.0), charges=(-1.0, 2.0, 3.0),
                         collisions=((2, 0), (0, 0), (1, 2), (1, 1), (0, 1), (2, 2)))
    _parity(ctx, wl, 4)


def test_parity_consecutive_intra_collisions(ctx):
    """Back-to-back intra-species collisions of different species touch
    disjoint particles; the kernel runs such a pair as one pass.  Each keeps
    its own counters, restore, correction and failure decision, so the
    result is the oracle's sequential one.  Covered: chains of such pairs,
    a repeated species (never merged), species with fewer than two
    particles, odd counts, and forced failures with both failure policies."""
    sizes = [(40, 30, 21), (1, 50, 33), (0, 2, 7), (3, 3, 3), (1501, 1000, 600), (2, 1, 0)]
    coll = ((0, 0), (1, 1), (2, 2), (0, 0), (0, 0), (1, 0), (2, 2), (1, 1))
    wl = custom_workload(sizes, seed=11, masses=(1.0, 4.0, 50.0), charges=(-1.0, 2.0, 3.0),
                         collisions=coll)
    _parity(ctx, wl.copy(), 2)
    _parity(ctx, wl.copy(), 3, f_E=0.01, max_passes=1)
    _parity(ctx, wl.copy(), 3, f_E=0.01, max_passes=1, on_failure=1)


def test_parity_relativistic_subset(ctx):
    wl = W.config4(n_cells=8)
    _parity(ctx, wl, 0)
    wl2 = custom_workload([(50, 40), (13, 2), (300, 300)], seed=8, masses=(1.0, 1836.0),
                          relativistic=True, c=1.0, dt=0.003)
    _parity(ctx, wl2, 1)


def test_parity_relativistic_global_layout(ctx):
    """Relativistic cells in global scratch: 2049 to 4096 particles (four
    waves in the order-N step) and above 4096 (8 waves by default, one wave
    forced)."""
    wl = custom_workload([(1500, 1200), (3000, 2500), (60, 40)], seed=9, masses=(1.0, 1836.0),
                         relativistic=True, c=1.0, dt=0.003)
    _parity(ctx, wl.copy(), 1)
    try:
        ctx.set_variant(6, 10)
        _parity(ctx, wl.copy(), 1)
    finally:
        ctx.set_variant(6, -1)


def test_relativistic_one_wave_global_forms(ctx):
    """Relativistic cells of 2049-4096 particles: the order-N step runs the
    four-wave global kernel, its diagnostic and duplicity forms the one-wave
    one.  Both forms against the oracle; the diagnostics also measure the
    residual momentum and energy of the relativistic correction (Appendix A)
    at FP64 rounding."""
    wl = custom_workload([(1500, 1200), (60, 40)], seed=13, masses=(1.0, 1836.0),
                         relativistic=True, c=1.0, dt=0.003)
    _, sg, so = _parity(ctx, wl.copy(), 1, diagnostics=True)
    print("  relativistic residuals: dP %.2e dE %.2e (oracle %.2e %.2e)"
          % (sg["max_rel_dP"], sg["max_rel_dE"], so["max_rel_dP"], so["max_rel_dE"]), flush=True)
    assert sg["max_rel_dP"] < 1e-14 and sg["max_rel_dE"] < 1e-14
    _parity(ctx, wl.copy(), 2, pairing=2)


@pytest.mark.parametrize("wmode", ["lognormal", "equal"])
def test_pairwise_momentum_sums_conserve_at_the_maximum_cell(ctx, wmode):
    """The momentum sums of Eq. (17) and the species energies of Eq. (24)
    are plain FP64 per thread and then a pairwise (butterfly) tree, not
    compensated as the oracle's: at the largest cell (MCC_MAX_CELL
    particles, 16384 per species) the residual momentum and energy after the
    correction still sit at FP64 rounding in both kinematics forms, with
    lognormal weights (rejections leave a large momentum change to restore)
    and with equal weights (the change to restore is itself rounding noise,
    so the tree's error and the compensated sum's differ most)."""
    from paper_2407_19151_amd import native
    wl = custom_workload([(16384, 16384), (60, 40)], seed=49, weight_mode=wmode)
    _, sg, so = _parity(ctx, wl.copy(), 1, diagnostics=True)
    print("  FP64 residuals: dP %.2e dE %.2e (oracle, compensated: %.2e %.2e)"
          % (sg["max_rel_dP"], sg["max_rel_dE"], so["max_rel_dP"], so["max_rel_dE"]), flush=True)
    assert sg["max_rel_dP"] < 1e-14 and sg["max_rel_dE"] < 1e-14
    _, s32, _ = _gpu_step(ctx, wl.copy(), 1, diagnostics=True,
                          precision=native.MCC_FP32_KINEMATICS)
    print("  FP32-kinematics residuals: dP %.2e dE %.2e" % (s32["max_rel_dP"], s32["max_rel_dE"]),
          flush=True)
    assert s32["max_rel_dP"] < 1e-14 and s32["max_rel_dE"] < 1e-14


def test_diagnostics_show_roundoff_conservation(ctx):
    wl = W.config2(n_cells=32)
    _, sg, so = _parity(ctx, wl, 0, diagnostics=True)
    assert sg["max_rel_dP"] < 1e-14 and sg["max_rel_dE"] < 1e-14


@pytest.mark.parametrize("prec", [0, 1])
def test_diagnostics_on_cells_in_global_scratch(ctx, prec):
    """Diagnostics on cells above 4096 particles (one-wave global kernel):
    FP64 against the oracle; FP32 kinematics against the FP64 residual bar
    (the correction is FP64 in both forms)."""
    from paper_2407_19151_amd import native
    wl = custom_workload([(3000, 2500), (60, 40)], seed=12)
    if prec == 0:
        _, sg, so = _parity(ctx, wl, 1, diagnostics=True)
    else:
        _, sg, _ = _gpu_step(ctx, wl, 1, diagnostics=True,
                             precision=native.MCC_FP32_KINEMATICS)
    assert sg["max_rel_dP"] < 1e-14 and sg["max_rel_dE"] < 1e-14


def test_unsorted_entry_matches_oracle(ctx):
    from paper_2407_19151_amd import native, runner
    base = W.config2(n_cells=40)
    wl = base.unsorted(seed=3)
    v0 = wl.velocities().copy()
    dw = runner.DeviceWorkload(wl)
    runner.collide_unsorted(ctx, dw, 2)
    vg = dw.velocities()
    assert ctx.device_error() == 0
    ref = wl.copy()
    oracle.collide(ref.cells, ref.species, ref.n_cells, ref.mass, ref.charge, ref.collisions,
                   ref.w, ref.vx, ref.vy, ref.vz, dt=ref.dt, coulomb_log=ref.coulomb_log,
                   seed=ref.seed, step=2, method=ref.method)
    check_parity(wl, vg, ref.velocities(), v0)


def test_bin_is_bit_exact(ctx):
    import torch
    base = custom_workload([(5, 3), (0, 0), (300, 2), (4000, 1), (1, 1)], seed=9)
    wl = base.unsorted(seed=4)
    off, perm = ctx.bin(torch.from_numpy(wl.cells).cuda(), torch.from_numpy(wl.species).cuda(),
                        wl.n_cells, wl.n_species)
    ro, rp = oracle.bin_particles(wl.cells, wl.species, wl.n_cells, wl.n_species)
    assert np.array_equal(off.cpu().numpy(), ro)
    assert np.array_equal(perm.cpu().numpy().astype(np.int64), rp)


def test_bin_at_full_size_and_with_bad_ids(ctx):
    """The radix-sort binning on the 65,536-cell population in random order
    (2.15e7 particles, two 9-bit passes) equals the oracle's stable
    counting sort bit for bit; with ids out of range it latches data error 3,
    groups the valid particles exactly as numpy's stable argsort and puts
    the bad ones last, in index order."""
    import torch
    wl = W.config3().unsorted(seed=9)
    off, perm = ctx.bin(torch.from_numpy(wl.cells).cuda(), torch.from_numpy(wl.species).cuda(),
                        wl.n_cells, wl.n_species)
    assert ctx.device_error() == 0
    ro, rp = oracle.bin_particles(wl.cells, wl.species, wl.n_cells, wl.n_species)
    assert np.array_equal(off.cpu().numpy(), ro)
    assert np.array_equal(perm.cpu().numpy().astype(np.int64), rp)
    rng = np.random.default_rng(3)
    n_cells, S, n = 700, 3, 20000
    cells = rng.integers(0, n_cells, n).astype(np.int32)
    species = rng.integers(0, S, n).astype(np.int32)
    cells[::53] = n_cells + 2
    species[7::101] = -1
    off, perm = ctx.bin(torch.from_numpy(cells).cuda(), torch.from_numpy(species).cuda(),
                        n_cells, S)
    assert ctx.device_error() == 3
    bad = (cells >= n_cells) | (species < 0)
    key = np.where(bad, n_cells * S, cells.astype(np.int64) * S + species)
    assert np.array_equal(perm.cpu().numpy().astype(np.int64), np.argsort(key, kind="stable"))
    want = np.zeros(n_cells * S + 1, dtype=np.int64)
    want[1:] = np.cumsum(np.bincount(key[~bad], minlength=n_cells * S))
    assert np.array_equal(off.cpu().numpy(), want)


def test_deterministic_reruns(ctx):
    wl = W.config2(n_cells=24)
    a, _, _ = _gpu_step(ctx, wl, 11)
    b, _, _ = _gpu_step(ctx, wl, 11)
    assert np.array_equal(a, b)


def test_plan_graph_replay_equals_plain_steps(ctx):
    """A plan with the default variants replays exactly the plain steps
    (bitwise); an autotuned plan agrees to the parity bar (its per-cell sums
    may run with another threads-per-cell, hence another rounding order).
    The population has cells in the 2048 and the 4096 buckets, so the graph's
    branch (the 4096 bucket beside the 2048 one) is part of the replay."""
    import json
    from paper_2407_19151_amd import runner
    wl = W.config3(n_cells=512)
    dw1 = runner.DeviceWorkload(wl)
    dw2 = runner.DeviceWorkload(wl)
    dw3 = runner.DeviceWorkload(wl)
    plan = runner.make_plan(ctx, dw1, autotune=False)
    tuned = runner.make_plan(ctx, dw3, autotune=True)
    try:
        cells = {b["max_cell"]: b["cells"] for b in json.loads(plan.describe())["buckets"]}
        assert cells[2048] > 0 and cells[4096] > 0, cells
        print(tuned.describe(), flush=True)
        plan.run(first_step=5, n_steps=3)
        tuned.run(first_step=5, n_steps=1)
        for s in (5, 6, 7):
            runner.collide_sorted(ctx, dw2, s, with_stats=False)
            if s == 5:
                v_after_5 = dw2.velocities()
        assert np.array_equal(dw1.velocities(), dw2.velocities())
        check_parity(wl, dw3.velocities(), v_after_5, wl.velocities())
    finally:
        plan.close()
        tuned.close()


def test_plan_scratch_survives_later_context_calls(ctx):
    """A plan's graph holds the address of its large-cell scratch.  Calls on
    the same context that need a larger scratch (the tangent form's stride
    is larger: a 2000-particle cell takes global scratch there, a 5000 one
    the largest stride) must not move it: the plan's replay after them still
    equals the plain steps, bit for bit (cells of 5000 and 2600 particles use
    the plan's global-scratch kernels)."""
    import torch
    from paper_2407_19151_amd import runner
    wl = custom_workload([(3000, 2000), (1300, 1300), (40, 30)], seed=14)
    dwp = runner.DeviceWorkload(wl)
    dwr = runner.DeviceWorkload(wl)
    plan = runner.make_plan(ctx, dwp, autotune=False)
    try:
        plan.run(first_step=3, n_steps=1)
        for sizes in ([(1100, 900)], [(2600, 2400)]):
            wj = custom_workload(sizes, seed=15)
            dj = runner.DeviceWorkload(wj)
            tan = torch.ones((3, wj.n), dtype=torch.float64, device="cuda")
            runner.collide_sorted_jvp(ctx, dj, tan, 0)
            torch.cuda.synchronize()
        plan.run(first_step=4, n_steps=1)
        torch.cuda.synchronize()
        for s in (3, 4):
            runner.collide_sorted(ctx, dwr, s, with_stats=False)
        assert ctx.device_error() == 0
        assert np.array_equal(dwp.velocities(), dwr.velocities())
    finally:
        plan.close()


VARIANTS = [(64, 128), (64, 256), (128, 256), (128, 512), (256, 512), (256, 1024),
            (512, 1024), (512, 2048), (1024, 2048), (1024, 4096), (64, 32768), (256, 2048),
            (512, 4096), (256, 4096), (256, 32768), (512, 32768)]
BUCKET_CAP = [128, 256, 512, 1024, 2048, 4096, 32768]


@pytest.mark.parametrize("v", range(len(VARIANTS)))
def test_every_kernel_variant_matches_oracle(ctx, v):
    """Every compiled (threads per cell, capacity) variant on every bucket it
    can serve, against the oracle."""
    cap = VARIANTS[v][1]
    sizes = [(60, 40), (111, 80), (300, 130), (600, 350), (1200, 700), (2300, 1600),
             (3000, 3200)]
    sizes = [s for s in sizes if sum(s) <= cap]
    wl = custom_workload(sizes, seed=40 + v)
    try:
        for b, bc in enumerate(BUCKET_CAP):
            if bc <= cap:
                ctx.set_variant(b, v)
        _parity(ctx, wl, 3)
    finally:
        for b in range(len(BUCKET_CAP)):
            ctx.set_variant(b, -1)


def test_invalid_offsets_flagged_not_faulting(ctx):
    import torch
    wl = W.config1(n_cells=4)
    from paper_2407_19151_amd import runner
    dw = runner.DeviceWorkload(wl)
    bad = dw.offsets.clone()
    bad[2] = bad[3] + 5  # not monotone
    dw.offsets = bad
    runner.collide_sorted(ctx, dw, 0)
    assert ctx.device_error() == 1


def test_fp32_angle_sampler_top_of_the_uniform_range(ctx):
    """FP32 N97 sampling takes its uniform from the top 23 bits of the word,
    (k + 1/2) 2^-23, which never rounds to 1: words at the top of the 32-bit
    range give the far tail of the inverse CDF (1 - cos theta = -ln(1 - u0)
    / A for large A, at most 16.6 / A), not a reversal.  Top words and
    random words, s over 12 decades, against the oracle's inverse CDF at the
    same quantized uniform, to FP32 accuracy."""
    import torch
    from paper_2407_19151_amd import native
    rng = np.random.default_rng(23)
    top = np.array([2 ** 32 - 1, 2 ** 32 - 2, 2 ** 32 - 64, 2 ** 32 - 128, 2 ** 32 - 129,
                    2 ** 32 - 256, 2 ** 32 - 300, 2 ** 32 - 4096], dtype=np.uint64)
    s = np.repeat(10.0 ** np.linspace(-10, 2, 25), top.size)
    a0 = np.tile(top, 25)
    s = np.concatenate([s, 10.0 ** rng.uniform(-10, 2, 4000)])
    a0 = np.concatenate([a0, rng.integers(0, 2 ** 32, 4000, dtype=np.uint64)]).astype(np.uint32)
    a1 = rng.integers(0, 2 ** 32, s.size, dtype=np.uint64).astype(np.uint32)
    oc, st, _ = ctx.sample_angles(W.N97, native.MCC_FP32_KINEMATICS, torch.from_numpy(s).cuda(),
                                  torch.from_numpy(a0.view(np.int32)).cuda(),
                                  torch.from_numpy(a1.view(np.int32)).cuda())
    oc, st = oc.cpu().numpy(), st.cpu().numpy()
    # at the top words 1 + u0 (e^-2A - 1) is about 2^-24 and FP32 keeps only
    # its leading bits (measured: 7.5e-4 of 1 - cos theta at s = 0.1); the
    # bar there is 3e-3
    ntop = 25 * top.size
    bad = []
    for i in range(s.size):
        u0 = (float(int(a0[i]) >> 9) + 0.5) * 2.0 ** -23
        u1 = (float(int(a1[i]) >> 9) + 0.5) * 2.0 ** -23
        ro, rs = oracle.sample_angle(W.N97, float(s[i]), u0, u1)
        if i < ntop:
            # the change of the unit relative velocity, (st cos phi, st sin phi,
            # -oc), has length sqrt(2 oc): its error against that length (near
            # a reversal st comes from the cancellation in 2 - oc)
            if math.hypot(oc[i] - ro, st[i] - rs) > 3e-3 * math.sqrt(2 * ro) + 1e-30:
                bad.append((i, s[i], int(a0[i]), oc[i], ro, st[i], rs))
        elif abs(oc[i] - ro) > 1e-4 * ro + 1e-30 or abs(st[i] - rs) > 1e-4 * max(rs, 1e-3):
            bad.append((i, s[i], int(a0[i]), oc[i], ro, st[i], rs))
    assert not bad, bad[:10]
    # no reversal at small s
    small = s < 1e-2
    assert np.all(oc[small] < 0.2)


@pytest.mark.parametrize("method", [W.N97, W.TA77])
def test_device_angle_sampler_matches_oracle_over_s_range(ctx, method):
    """The map s -> (1 - cos theta, sin theta) on the device against the
    oracle, over 16 decades of s and random uniforms (FP64)."""
    import torch
    rng = np.random.default_rng(17)
    n = 20000
    s = 10.0 ** rng.uniform(-12, 4, n)
    a0 = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    a1 = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    oc, st, A = ctx.sample_angles(method, 0, torch.from_numpy(s).cuda(),
                                  torch.from_numpy(a0.view(np.int32)).cuda(),
                                  torch.from_numpy(a1.view(np.int32)).cuda())
    oc, st, A = oc.cpu().numpy(), st.cpu().numpy(), A.cpu().numpy()
    bad = []
    for i in range(n):
        u0 = (float(a0[i]) + 0.5) * 2.0 ** -32
        u1 = (float(a1[i]) + 0.5) * 2.0 ** -32
        ro, rs = oracle.sample_angle(method, float(s[i]), u0, u1)
        if method == W.N97:
            ra = oracle.n97_A(float(s[i]))
            if not (abs(A[i] - ra) <= 1e-13 * abs(ra) or (ra == 0 and A[i] < 1e-300)):
                bad.append(("A", i, s[i], A[i], ra))
        if abs(oc[i] - ro) > 1e-12 * max(ro, 1e-300) + 1e-15 or abs(st[i] - rs) > 1e-12:
            bad.append(("angle", i, s[i], u0, oc[i], ro, st[i], rs))
    assert not bad, bad[:10]


def test_per_call_step_on_a_caller_stream_equals_the_default_stream(ctx):
    """The sorted step runs the kernel of its 2049-4096-particle cells on the
    context's side stream beside the 1025-2048 one, forked from and joined to
    the caller's stream.  Enqueued on a stream of the caller's (default
    priority), with the caller's own work before and after it on that stream,
    the step must equal the same step on the default stream, bit for bit, and
    the caller's later work must see its result."""
    import torch
    from paper_2407_19151_amd import runner
    wl = custom_workload([(1300, 900), (2600, 1300), (700, 600), (90, 40), (2000, 1900)],
                         seed=16)
    d0 = runner.DeviceWorkload(wl)
    d1 = runner.DeviceWorkload(wl)
    for k in range(3):
        runner.collide_sorted(ctx, d0, 30 + k, with_stats=False)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        d1.vx.mul_(1.0)  # caller work before the step, on the same stream
        for k in range(3):
            runner.collide_sorted(ctx, d1, 30 + k, with_stats=False)
        after = d1.vx * 1.0  # caller work after the step reads its result
    s.synchronize()
    assert ctx.device_error() == 0
    assert np.array_equal(d0.velocities(), d1.velocities())
    assert np.array_equal(after.cpu().numpy(), d0.vx.cpu().numpy())
