"""The paper's Test 3 (Sec. 5.3, its figures) on the GPU, in SI units,
1600 cells, FP64.

- Parity: two steps of every case against the oracle at the FP64 bar, with
  the correction on (T3a, T3c) and off (T3b).
- The relaxation rate: over 20 000 steps (7.1 fs) the ions heat at the
  paper's 0D Spitzer rate, integrated from the sampled initial temperatures,
  times the finite-step factor of N97 computed by quadrature (no fit).  The
  paper's step is about tau_e / 165, where an electron-ion pair at the
  electron thermal speed still has s = 0.023 (T3a) or 0.14 (T3b, T3c, where
  w_e = 6 w_i makes every pair six times stronger and the electron accepts
  one in six); the factor is 0.948 and 0.858.  Measured: 0.950, 0.877 and
  0.866 of the Spitzer gain.  The full relaxation to the printed 136 eV
  takes about 2.6e5 steps per e-fold and is not run.
- Conservation: with the correction (T3a, T3c) total momentum and energy are
  unchanged to rounding; without it (T3b) both drift by many orders more,
  which is what the correction is for.
"""
import numpy as np
import pytest

from paper_2407_19151_amd import workloads as W

from gpu_helpers import FP64_TOL, check_parity, oracle_step
from test_paper_test3 import n97_saturation, pair_k, spitzer_0d

pytestmark = pytest.mark.gpu

STEPS = 20000


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_19151_amd import native
    c = native.Context()
    yield c
    c.close()


@pytest.mark.parametrize("case", sorted(W.PAPER_T3_CASES))
def test_paper_test3_parity(ctx, case):
    from paper_2407_19151_amd import runner
    wl = W.paper_test3(case)
    corr = bool(wl.extra["moment_correction"])
    dw = runner.DeviceWorkload(wl)
    for s in range(2):
        runner.collide_sorted(ctx, dw, s, params=runner.params_for(wl, moment_correction=int(corr)))
    assert ctx.device_error() == 0
    ref = wl.copy()
    for s in range(2):
        oracle_step(ref, s, correction=corr)
    info = check_parity(wl, dw.velocities(), ref.velocities(), wl.velocities(), tol=FP64_TOL)
    print("%s parity over 2 steps: %s" % (case, info), flush=True)


@pytest.mark.parametrize("case", sorted(W.PAPER_T3_CASES))
def test_paper_test3_spitzer_rate_and_conservation(ctx, case):
    import torch
    from paper_2407_19151_amd import runner
    wl = W.paper_test3(case)
    corr = bool(wl.extra["moment_correction"])
    n_i, n_e, _ = W.PAPER_T3_CASES[case]
    m = wl.mass[wl.species] * wl.w
    v0 = wl.velocities()
    te0, ti0 = W.species_temperatures(wl, v0)
    dw = runner.DeviceWorkload(wl)
    plan = runner.make_plan(ctx, dw, params=runner.params_for(wl, moment_correction=int(corr)),
                            autotune=False)
    try:
        plan.run(0, STEPS)
        torch.cuda.synchronize()
        v = dw.velocities()
    finally:
        plan.close()
    te, ti = W.species_temperatures(wl, v)
    _, ti_sp = spitzer_0d(te0, ti0, STEPS * wl.dt)
    # the target density of an e-i pair: w_max N_min / dV
    n_eff = max(wl.w[wl.species == 0][0], wl.w[wl.species == 1][0]) * min(n_i, n_e) / wl.cell_volume
    sat = n97_saturation(pair_k(n_eff), te0)
    ratio = (ti - ti0) / (ti_sp - ti0)
    print("%s after %d steps: T_e %.3f -> %.3f eV, T_i %.3f -> %.3f eV; Spitzer T_i %.3f; "
          "gain / Spitzer gain %.4f, N97 factor %.4f" % (case, STEPS, te0, te, ti0, ti, ti_sp,
                                                          ratio, sat), flush=True)
    assert abs(ratio / sat - 1) < 0.04
    # energy moves from the electrons to the ions in the density ratio
    assert (te0 - te) * 6.0 == pytest.approx(ti - ti0, rel=0.02 if corr else 0.2)

    def totals(vv):
        return (m * vv).sum(1), (0.5 * m * (vv * vv).sum(0)).sum(), (m * np.linalg.norm(vv, axis=0)).sum()

    p0, e0, ps = totals(v0)
    p1, e1, _ = totals(v)
    dp, de = np.abs(p1 - p0).max() / ps, abs(e1 - e0) / e0
    print("  over %d steps: max |dP| / sum m w |v| %.1e, |dE| / E %.1e" % (STEPS, dp, de), flush=True)
    if corr:
        assert dp < 1e-14 and de < 1e-12
    else:
        assert dp > 1e-6 and de > 1e-7
