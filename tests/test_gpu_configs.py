"""Whole runs at the full sizes of the two-species workload (4096 cells, 200
steps, N97 and TA77) and of the relativistic beam workload (16384 cells of
1024 particles, 500 steps) against the oracle's committed references
(tests/golden/make_config_references.py, oracle only).

After the first steps the GPU run and the oracle's part ways at the level of
single particles (rounding differences of the same draws grow through the
collisions), so the runs are compared by their moments: the first step
closely (the same draws from the same state), the whole trajectory and its
relaxation rate against the spread that the collision noise alone gives
(the oracle's runs with the Philox seed + 1 and + 2)."""
import os

import numpy as np
import pytest

from paper_2407_19151_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_19151_amd import native
    c = native.Context()
    yield c
    c.close()


def _load(name, per_run):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip("reference %s not written (tests/golden/make_config_references.py)" % name)
    a = np.loadtxt(path)
    runs = [a[:, 1 + i * per_run:1 + (i + 1) * per_run] for i in range((a.shape[1] - 1) // per_run)]
    return runs[0], runs[1:]


def _rate(T):
    """Relaxation rate per step: slope of log(T_e - T_i)."""
    return -np.polyfit(np.arange(T.shape[0]), np.log(T[:, 0] - T[:, 1]), 1)[0]


def _noise_scale(main, alts):
    """Largest per-step RMS (over the alternate seeds) of the relative
    deviation from the main run."""
    d = np.stack([np.abs(a / main - 1.0) for a in alts])
    return float(np.sqrt((d ** 2).mean(0)).max())


@pytest.mark.parametrize("method", ["n97", "ta77"])
def test_two_species_relaxation_at_full_size(ctx, method):
    import torch
    from paper_2407_19151_amd import autodiff, native, runner
    main, alts = _load("c2_%s_relaxation_oracle.txt" % method, 2)
    steps = main.shape[0] - 1
    scale = _noise_scale(main, alts)
    r_main = _rate(main)
    r_spread = float(np.sqrt(np.mean([(_rate(a) - r_main) ** 2 for a in alts])))
    for prec in (native.MCC_FP64, native.MCC_FP32_KINEMATICS):
        wl = W.config2(method=W.N97 if method == "n97" else W.TA77)
        dw = runner.DeviceWorkload(wl)
        plan = runner.make_plan(ctx, dw, params=runner.params_for(wl, precision=prec),
                                autotune=False)
        T = [autodiff.species_temperatures(wl, torch.stack([dw.vx, dw.vy, dw.vz]))]
        for k in range(steps):
            plan.run(k, 1)
            T.append(autodiff.species_temperatures(wl, torch.stack([dw.vx, dw.vy, dw.vz])))
        plan.close()
        assert ctx.device_error() == 0
        T = torch.stack(T).cpu().numpy()
        dev = np.abs(T / main - 1.0)
        r = _rate(T)
        print("  %s %s: step-1 deviation %.2e, largest %.2e (noise scale %.2e); rate %.5f vs "
              "oracle %.5f (seed spread %.5f)" % (method, "fp64" if prec == 0 else "fp32", dev[1].max(),
                                                 dev.max(), scale, r, r_main, r_spread), flush=True)
        # the first step: the same draws from the same state (FP64 parity;
        # FP32 kinematics within their own bar)
        assert dev[1].max() < (1e-10 if prec == native.MCC_FP64 else 1e-5)
        assert dev.max() < 4.0 * scale
        assert abs(r - r_main) < 4.0 * r_spread + 1e-3 * r_main


def test_relativistic_beam_at_full_size(ctx):
    import torch
    from paper_2407_19151_amd import native, runner
    main, alts = _load("c4_beam_oracle.txt", 4)
    steps = main.shape[0] - 1
    wl = W.config4()
    dw = runner.DeviceWorkload(wl)
    e = wl.species == 0
    beam = e & (wl.w < 0.5 * wl.w[e].max())
    masks = [torch.as_tensor(m, device="cuda") for m in (beam, e & ~beam, wl.species == 1)]
    mass = torch.as_tensor(wl.mass[wl.species], device="cuda")

    def observe():
        u2 = dw.vx * dw.vx + dw.vy * dw.vy + dw.vz * dw.vz
        kin = mass * u2 / (torch.sqrt(1.0 + u2) + 1.0)
        out = [(dw.w[masks[0]] * dw.vx[masks[0]]).sum() / dw.w[masks[0]].sum()]
        out += [(dw.w[m] * kin[m]).sum() / dw.w[m].sum() for m in masks]
        return torch.stack(out)

    plan = runner.make_plan(ctx, dw, params=runner.params_for(wl), autotune=False)
    obs = [observe()]
    for k in range(steps):
        plan.run(k, 1)
        obs.append(observe())
    plan.close()
    assert ctx.device_error() == 0
    obs = torch.stack(obs).cpu().numpy()
    dev = np.abs(obs / main - 1.0)
    scale = _noise_scale(main, alts)
    # the beam's slowing: its mean proper velocity along x lost over the run
    lost = 1.0 - obs[-1, 0] / obs[0, 0]
    lost_or = 1.0 - main[-1, 0] / main[0, 0]
    lost_spread = float(np.sqrt(np.mean([(1.0 - a[-1, 0] / a[0, 0] - lost_or) ** 2 for a in alts])))
    print("  beam: step-1 deviation %.2e, largest %.2e (noise scale %.2e); <u_x> lost %.5f vs "
          "oracle %.5f (seed spread %.5f)" % (dev[1].max(), dev.max(), scale, lost, lost_or,
                                              lost_spread), flush=True)
    assert dev[1].max() < 1e-10
    assert dev.max() < 4.0 * scale
    assert abs(lost - lost_or) < 4.0 * lost_spread + 1e-3 * abs(lost_or)
