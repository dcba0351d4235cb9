"""The hard-sphere process (method MCC_HARD_SPHERE) on the GPU against the
oracle's.

The process is the non-Coulomb use of the paper's weighting and moment
correction: elastic scattering with a constant cross-section per collision,
s = sigma n_eff |u| dt read as the expected number of collisions, a
collision with probability 1 - exp(-s) and an isotropic centre-of-mass
direction.  Element-by-element parity at the FP64 bar over every size
bucket and layout, the weight classes, the correction options, the three
pairings and a plan's graph replays; at the benchmark's full size, sampled
cells against the oracle and per-cell conservation of the whole state; and
the forms the library does not take (FP32 kinematics, relativistic, the
tangent entry point) and invalid cross-sections rejected on the host.

The collide-or-not decision compares a uniform on the 2^-32 grid with
1 - exp(-s) in FP64 on both sides; the two values of s differ by a few ulp
(operation order), so a decision differs only when the uniform falls within
~1e-16 of the threshold.
"""
import math

import numpy as np
import pytest

from paper_2407_19151_amd import workloads as W

from gpu_helpers import FP64_TOL, check_parity, custom_workload, oracle_step
from test_gpu_parity import _gpu_step, _parity

pytestmark = pytest.mark.gpu

HS = W.HARD_SPHERE
SIZES = [(1, 0), (0, 1), (1, 1), (2, 1), (3, 5), (7, 2), (16, 16), (33, 64), (100, 27),
         (128, 129), (255, 1), (1, 300), (300, 700), (1024, 1000), (2100, 1900)]


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_19151_amd import native
    c = native.Context()
    yield c
    c.close()


def _hs(sizes, seed, prob=0.05, **kw):
    return W.hard_sphere(custom_workload(sizes, seed=seed, **kw), prob)


def test_hs_parity_every_bucket(ctx):
    wl = _hs(SIZES, 41)
    for step in (0, 3):
        info, sg, so = _parity(ctx, wl.copy(), step)
        assert sg["pairs"] > 0


@pytest.mark.parametrize("wmode", ["equal", "lognormal", "two", "clustered"])
def test_hs_parity_weight_classes(ctx, wmode):
    sizes = [(5, 4), (64, 63), (200, 9), (513, 40), (700, 900)]
    _parity(ctx, _hs(sizes, 42, weight_mode=wmode, prob=0.2), 1)


def test_hs_parity_options(ctx):
    sizes = [(9, 7), (130, 70), (400, 400), (1500, 1200)]
    wl = _hs(sizes, 43, weight_mode="lognormal", prob=0.1)
    _parity(ctx, wl.copy(), 2, max_passes=20)
    _parity(ctx, wl.copy(), 2, sort_by_weight=False, f_E=0.2)
    _parity(ctx, wl.copy(), 2, moment_correction=False)
    _parity(ctx, wl.copy(), 2, on_failure=1)


def test_hs_parity_certain_collisions(ctx):
    """s >> 1: every pair collides (probability 1 - exp(-s) rounds to 1)."""
    _parity(ctx, _hs([(40, 30), (300, 200)], 44, prob=50.0), 0)


@pytest.mark.parametrize("pairing", [1, 2])
def test_hs_parity_nxn_and_duplicity(ctx, pairing):
    from paper_2407_19151_amd import native
    sizes = [(1, 1), (3, 5), (16, 16), (33, 64), (100, 27), (255, 1), (300, 280)]
    wl = _hs(sizes, 45 + pairing, prob=0.1)
    v0 = wl.velocities().copy()
    print("hard-sphere parity, pairing %d: cells=%d n=%d" % (pairing, wl.n_cells, wl.n),
          flush=True)
    vg, sg, _ = _gpu_step(ctx, wl, 1, pairing=pairing)
    ref = wl.copy()
    so = oracle_step(ref, 1, pairing=pairing)

    def rerun(p):
        oracle_step(p, 1, pairing=pairing)
        return p.velocities()

    tol = FP64_TOL * math.sqrt(max(a + b for a, b in sizes))
    info = check_parity(wl, vg, ref.velocities(), v0, tol=tol, rerun=rerun)
    print("  parity (tol %.1e): %s" % (tol, info), flush=True)
    assert sg["pairs"] == so["pairs"] and sg["collisions"] == so["collisions"]
    assert sg["failed"] == so["failed"]
    if pairing == native.MCC_PAIRING_NXN:
        assert sg["pairs"] == sum(a * (a - 1) // 2 + b * (b - 1) // 2 + a * b for a, b in sizes)


def test_hs_plan_replays_equal_oracle_steps(ctx):
    import torch
    from paper_2407_19151_amd import runner
    sizes = [(30, 20), (129, 127), (600, 500), (3, 0), (2000, 1500)]
    wl = _hs(sizes, 47, weight_mode="lognormal", prob=0.05)
    dw = runner.DeviceWorkload(wl)
    plan = runner.make_plan(ctx, dw, params=runner.params_for(wl), autotune=False)
    try:
        plan.run(20, 3)
        torch.cuda.synchronize()
        vg = dw.velocities()
    finally:
        plan.close()
    assert ctx.device_error() == 0
    ref = wl.copy()
    for s in range(20, 23):
        oracle_step(ref, s)
    info = check_parity(wl, vg, ref.velocities(), wl.velocities(), tol=3 * FP64_TOL)
    print("plan, 3 replays: %s" % info, flush=True)


def test_hs_unsupported_and_invalid(ctx):
    import torch
    from paper_2407_19151_amd import native, runner
    wl = _hs([(10, 10)], 48)
    dw = runner.DeviceWorkload(wl)
    for over, code in ((dict(precision=native.MCC_FP32_KINEMATICS), -4),
                       (dict(relativistic=True, c=10.0), -4)):
        with pytest.raises(native.MCCError) as e:
            runner.collide_sorted(ctx, dw, 0, params=runner.params_for(wl, **over))
        assert e.value.code == code, over
    tan = torch.zeros((3, wl.n), dtype=torch.float64, device="cuda")
    with pytest.raises(native.MCCError) as e:
        runner.collide_sorted_jvp(ctx, dw, tan, 0, params=runner.params_for(wl))
    assert e.value.code == -4
    for bad in (-1.0, math.nan, math.inf):
        wb = W.dataclasses.replace(wl, collisions=[(0, 0, bad), (1, 1, 1.0), (0, 1, 1.0)])
        with pytest.raises(native.MCCError) as e:
            runner.collide_sorted(ctx, runner.DeviceWorkload(wb), 0, params=runner.params_for(wb))
        assert e.value.code == -1, bad
    # a zero cross-section changes nothing; a Coulomb method ignores it
    wz = W.dataclasses.replace(wl, collisions=[(0, 0, 0.0), (1, 1, 0.0), (0, 1, 0.0)])
    vz, _, _ = _gpu_step(ctx, wz, 0)
    assert np.array_equal(vz, wl.velocities())
    wc = W.dataclasses.replace(wl, method=W.N97)
    vc, _, _ = _gpu_step(ctx, wc, 0)
    wc2 = W.dataclasses.replace(wl, method=W.N97, collisions=[(0, 0), (1, 1), (0, 1)])
    vc2, _, _ = _gpu_step(ctx, wc2, 0)
    assert np.array_equal(vc, vc2)


def test_hs_full_population_sampled_cells_and_conservation(ctx):
    """The benchmark's 65,536-cell population under the hard-sphere process,
    stepped by a plan as the benchmark times it (FP64)."""
    from paper_2407_19151_amd import runner
    from test_gpu_full import FIRST_STEP, _cell_moments, _sample_cells, _subset
    wl = W.hard_sphere(W.config3())
    dw = runner.DeviceWorkload(wl)
    plan = runner.make_plan(ctx, dw, params=runner.params_for(wl), autotune=False)
    try:
        plan.run(FIRST_STEP, 1)
        vg = dw.velocities()
    finally:
        plan.close()
    assert ctx.device_error() == 0
    v0 = wl.velocities()
    assert np.all(np.isfinite(vg))
    moved = np.any(vg != v0, axis=0)   # scattered, or shifted by the correction
    print("hard spheres, %d particles: %.2f %% moved" % (wl.n, 100 * moved.mean()), flush=True)
    assert moved.mean() > 0.02
    P0, E0, Ps = _cell_moments(wl, v0)
    P1, E1, _ = _cell_moments(wl, vg)
    dP = np.abs(P1 - P0).max(0) / np.maximum(Ps, 1e-300)
    dE = np.abs(E1 - E0) / np.maximum(E0, 1e-300)
    print("  per-cell conservation: max |dP|/sum m w |v| %.2e, max |dE|/E %.2e"
          % (dP.max(), dE.max()), flush=True)
    assert dP.max() < 1e-13 and dE.max() < 1e-13
    cells = _sample_cells(wl)
    sub, idx = _subset(wl, cells)
    ref = sub.copy()
    oracle_step(ref, FIRST_STEP)

    def rerun(p):
        oracle_step(p, FIRST_STEP)
        return p.velocities()

    info = check_parity(sub, vg[:, idx], ref.velocities(), sub.velocities(), tol=FP64_TOL,
                        rerun=rerun)
    print("  %d sampled cells (%d particles): %s" % (cells.size, idx.size, info), flush=True)


def test_hs_maxwellian_energy_exchange_at_scale(ctx):
    """Independent of the oracle: 20 000 cells of 32 + 16 particles (masses 1
    and 4, T 2 and 1, equal densities), inter-species hard spheres at about
    3 % collision probability per particle.  One GPU step moves the energy
    of species a at the textbook rate d(3 T_a / 2)/dt = -n_b sigma (mu / M)
    8 sqrt(2 / pi) g (T_a - T_b), g^2 = T_a / m_a + T_b / m_b, within 3 %
    plus four standard errors of the per-cell gains."""
    from paper_2407_19151_amd import native
    n_cells, na, nb = 20000, 32, 16
    base = custom_workload([(na, nb)] * n_cells, seed=49, masses=(1.0, 4.0),
                           collisions=((0, 1),), weight_mode="equal")
    base.w[base.species == 1] *= na / nb          # equal densities
    wl = W.hard_sphere(base, 0.03)
    sigma = wl.collisions[0][2]
    v0 = wl.velocities().copy()
    vg, _, _ = _gpu_step(ctx, wl, 0, moment_correction=False, precision=native.MCC_FP64)
    ma, mb = wl.mass
    a = wl.species == 0
    ta = ma * (v0[:, a] ** 2).sum() / (3 * a.sum())
    tb = mb * (v0[:, ~a] ** 2).sum() / (3 * (~a).sum())
    dV = float(np.mean(wl.cell_volume))
    n_b = wl.w[~a].sum() / (n_cells * dV)
    g = math.sqrt(ta / ma + tb / mb)
    want = -n_b * sigma * (ma * mb / (ma + mb) ** 2) * 8 * math.sqrt(2 / math.pi) * g \
        * (ta - tb) * wl.dt
    e = lambda v: (0.5 * ma * (v[:, a] ** 2).sum(0)).reshape(n_cells, na).sum(1)
    gain = (e(vg) - e(v0)) / na
    se = gain.std() / math.sqrt(n_cells)
    print("energy gain per a particle %.4e +- %.1e, hard-sphere rate x dt %.4e"
          % (gain.mean(), se, want), flush=True)
    assert abs(gain.mean() - want) < 0.03 * abs(want) + 4 * se
    assert 4 * se < 0.15 * abs(want)
