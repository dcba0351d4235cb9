"""Duplicity pairing (the s of Higginson et al. that the paper describes
after Sec. 3.2) on the GPU against the oracle.

The pairs and their order are the order-N ones; an inter-species pair's s
takes N_max / D for N_min, D its chain length (the pairs of its
fewer-population particle).  The step is as well conditioned as the
order-N one, so the parity bars are those of the order-N tests: FP64 at
1e-12 of the cell scale with the order-N cut-off allowance, FP32 kinematics
at 1e-4.  With N_max a multiple of N_min the step is the order-N step.
"""
import numpy as np
import pytest

from paper_2407_19151_amd import workloads as W

from gpu_helpers import FP64_TOL, check_parity, custom_workload, oracle_step
from test_gpu_parity import _gpu_step, _parity

pytestmark = pytest.mark.gpu

DUP = 2
RAGGED = [(1, 0), (1, 1), (3, 2), (2, 3), (7, 3), (100, 27), (27, 100), (255, 1), (300, 700),
          (1024, 999), (1900, 2100), (2500, 2000)]


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_19151_amd import native
    c = native.Context()
    yield c
    c.close()


@pytest.mark.parametrize("method", [W.N97, W.TA77])
def test_duplicity_parity_every_bucket(ctx, method):
    wl = custom_workload(RAGGED, seed=41, method=method)
    _parity(ctx, wl, 3, pairing=DUP)


@pytest.mark.parametrize("wmode", ["equal", "lognormal", "two"])
def test_duplicity_parity_weight_classes(ctx, wmode):
    wl = custom_workload([(5, 3), (70, 40), (513, 300)], seed=42, weight_mode=wmode)
    _parity(ctx, wl, 1, pairing=DUP)


def test_duplicity_fp32_and_relativistic(ctx):
    from paper_2407_19151_amd import native
    wl = custom_workload([(9, 4), (130, 70), (700, 300)], seed=43)
    v0 = wl.velocities().copy()
    vg, _, _ = _gpu_step(ctx, wl, 2, pairing=DUP, precision=native.MCC_FP32_KINEMATICS)
    ref = wl.copy()
    oracle_step(ref, 2, pairing=DUP, uniform23=True)
    info = check_parity(wl, vg, ref.velocities(), v0, tol=1e-4, cond_tol=1e-4)
    print("fp32 duplicity parity: %s" % info, flush=True)
    wr = custom_workload([(50, 40), (13, 2), (300, 200)], seed=44, masses=(1.0, 1836.0),
                         relativistic=True, c=1.0, dt=0.003)
    _parity(ctx, wr, 1, pairing=DUP)


def test_duplicity_integer_ratio_is_order_n(ctx):
    wl = custom_workload([(6, 2), (2, 6), (90, 30), (400, 400)], seed=45)
    v0 = wl.velocities().copy()
    va, _, _ = _gpu_step(ctx, wl, 4, pairing=DUP)
    vb, _, _ = _gpu_step(ctx, wl, 4, pairing=0)
    info = check_parity(wl, va, vb, v0, tol=FP64_TOL, cond_tol=FP64_TOL)
    print("duplicity vs order-N at integer ratios: %s" % info, flush=True)


def test_duplicity_plan_replays(ctx):
    import torch
    from paper_2407_19151_amd import runner
    wl = custom_workload([(30, 20), (129, 61), (600, 500)], seed=46)
    dw = runner.DeviceWorkload(wl)
    plan = runner.make_plan(ctx, dw, params=runner.params_for(wl, pairing=DUP), autotune=False)
    try:
        plan.run(7, 3)
        torch.cuda.synchronize()
        vg = dw.velocities()
    finally:
        plan.close()
    ref = wl.copy()
    for s in range(7, 10):
        oracle_step(ref, s, pairing=DUP)
    info = check_parity(wl, vg, ref.velocities(), wl.velocities(), tol=3 * FP64_TOL,
                        cond_tol=1e-6)
    print("duplicity plan, 3 replays: %s" % info, flush=True)
