"""The paper's Test 2 (Sec. 5.2, its parameter table and figures) on the GPU,
in SI units, 180 cells, FP64.

- Parity: two steps of every case against the oracle at the FP64 bar.
- Relaxation against the equal-weight case T2a at 25 ps: T2b-T2d carry the
  drifts and temperatures of all three populations to within bars about
  twice the measured deviation (U_A 0.9 %, T_A 0.8 %, U_B 3 %, T_B 0.4 %,
  U_C 2 %, T_C 1.4 %).
- T2e (weights 1 : 400 : 4) departs further at the table's 50 fs step: each
  A particle takes one A-B kick per step with a normalized scattering length
  w_max N_min / dV about 60 times that of T2a's pairs, where the angle's mean
  response is no longer linear in s.  That is a first-order time-step error
  of the order-N pairing: the gap in U_A roughly halves with the step
  (measured 10.4, 5.3, 3.2 km/s at 50, 25, 12.5 fs) and does not shrink with
  five times the particles.
- The weight sort of the energy pairs keeps the correction on the heavy
  particles: in T2e without it the correction lands on the light population
  C and overheats it (measured +29 % at 25 ps), with it T_C stays with T2a.
- Equilibrium: after 6000 steps every population of every case sits at the
  drift and temperature that conservation fixes for its own sampled initial
  state, and total momentum and energy are unchanged to rounding.
"""
import math

import numpy as np
import pytest

from paper_2407_19151_amd import workloads as W

from gpu_helpers import FP64_TOL, check_parity, oracle_step
from test_paper_test1 import closed_form_end_state

pytestmark = pytest.mark.gpu

T_STAR = 25e-12  # s


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_19151_amd import native
    c = native.Context()
    yield c
    c.close()


def _run_plan(ctx, wl, n, **over):
    import torch
    from paper_2407_19151_amd import runner
    dw = runner.DeviceWorkload(wl)
    plan = runner.make_plan(ctx, dw, params=runner.params_for(wl, **over), autotune=False)
    try:
        plan.run(0, n)
        torch.cuda.synchronize()
        return dw.velocities()
    finally:
        plan.close()


def _moments_at(ctx, wl, t, **over):
    v = _run_plan(ctx, wl, int(round(t / wl.dt)), **over)
    return W.population_moments(wl, v)


def _fmt(mo):
    return " ".join("%s: U %.2f km/s T %.1f eV" % ("ABC"[k], u / 1e3, T)
                    for k, (u, T) in sorted(mo.items()))


@pytest.mark.parametrize("case", sorted(W.PAPER_T2_CASES))
def test_paper_test2_parity(ctx, case):
    from paper_2407_19151_amd import runner
    wl = W.paper_test2(case)
    dw = runner.DeviceWorkload(wl)
    for s in range(2):
        runner.collide_sorted(ctx, dw, s)
    assert ctx.device_error() == 0
    ref = wl.copy()
    for s in range(2):
        oracle_step(ref, s)
    info = check_parity(wl, dw.velocities(), ref.velocities(), wl.velocities(), tol=FP64_TOL)
    print("%s parity over 2 steps: %s" % (case, info), flush=True)


def test_paper_test2_relaxation_independent_of_weighting(ctx):
    res = {case: _moments_at(ctx, W.paper_test2(case), T_STAR) for case in sorted(W.PAPER_T2_CASES)}
    for case, r in res.items():
        print("%s at 25 ps: %s" % (case, _fmt(r)), flush=True)
    base = res["T2a"]
    # the relaxation is well under way at 25 ps
    assert 0.45 < base[0][0] / 655e3 < 0.6 and 0.45 < -base[2][0] / 655e3 < 0.6
    assert base[0][1] > 2.0 * 500.0 and base[1][1] > 1.5 * 500.0
    bars = {0: (0.02, 0.02), 1: (0.06, 0.015), 2: (0.04, 0.03)}  # (U, T) per population
    for case in ("T2b", "T2c", "T2d"):
        for k, (bu, bt) in bars.items():
            assert abs(res[case][k][0] / base[k][0] - 1) < bu, (case, k)
            assert abs(res[case][k][1] / base[k][1] - 1) < bt, (case, k)


def test_paper_test2e_gap_is_a_time_step_error(ctx):
    gaps = {}
    for dt in (50e-15, 25e-15, 12.5e-15):
        mo = {}
        for case in ("T2a", "T2e"):
            wl = W.paper_test2(case)
            wl.dt = dt
            mo[case] = _moments_at(ctx, wl, T_STAR)
        gaps[dt] = mo["T2e"][0][0] - mo["T2a"][0][0]
        print("dt %.1f fs: T2a %s | T2e %s | gap in U_A %.2f km/s"
              % (dt * 1e15, _fmt(mo["T2a"]), _fmt(mo["T2e"]), gaps[dt] / 1e3), flush=True)
    g50, g25, g12 = gaps[50e-15], gaps[25e-15], gaps[12.5e-15]
    assert g50 > 0.015 * 340e3            # a visible lag at the table's step
    assert g25 < 0.7 * g50 and g12 < 0.45 * g50
    assert g12 < 0.015 * 340e3            # within the bars of the other cases


def test_paper_test2e_weight_sort_protects_the_light_population(ctx):
    base = _moments_at(ctx, W.paper_test2("T2a"), T_STAR)
    wl = W.paper_test2("T2e")
    srt = _moments_at(ctx, wl, T_STAR, sort_by_weight=1)
    nos = _moments_at(ctx, wl, T_STAR, sort_by_weight=0)
    print("T2e with sort: %s\nT2e without:   %s" % (_fmt(srt), _fmt(nos)), flush=True)
    assert abs(srt[2][1] / base[2][1] - 1) < 0.03
    assert nos[2][1] / base[2][1] - 1 > 0.1


@pytest.mark.parametrize("case", sorted(W.PAPER_T2_CASES))
def test_paper_test2_equilibrium_and_conservation(ctx, case):
    wl = W.paper_test2(case)
    m = wl.mass[0]
    pop = wl.extra["population"]
    v0 = wl.velocities()
    mom0 = W.population_moments(wl, v0)
    dens = [wl.w[pop == k].sum() / (wl.n_cells * wl.cell_volume) for k in range(3)]
    u_f, t_f = closed_form_end_state(m, dens, [mom0[k][1] for k in range(3)],
                                     [mom0[k][0] for k in range(3)])
    v = _run_plan(ctx, wl, 6000)
    mom = W.population_moments(wl, v)
    print("%s after 6000 steps: %s; conserved end state %.2f km/s, %.1f eV"
          % (case, _fmt(mom), u_f / 1e3, t_f), flush=True)
    for k in range(3):
        count = W.PAPER_T2_CASES[case][k] * wl.n_cells
        sig_v = math.sqrt(t_f * W.E_CHARGE / m)
        assert abs(mom[k][0] - u_f) < 5 * sig_v / math.sqrt(count), k
        assert abs(mom[k][1] / t_f - 1) < max(0.01, 5 * math.sqrt(2.0 / (3.0 * count))), k

    def totals(vv):
        return (wl.w * vv[0]).sum(), (0.5 * m * wl.w * (vv * vv).sum(0)).sum()

    p0, e0 = totals(v0)
    p1, e1 = totals(v)
    print("  relative change over 6000 steps: P_x %.1e, E %.1e"
          % (abs(p1 - p0) / abs(p0), abs(e1 - e0) / e0), flush=True)
    assert abs(p1 - p0) / abs(p0) < 1e-12
    assert abs(e1 - e0) / e0 < 1e-12
