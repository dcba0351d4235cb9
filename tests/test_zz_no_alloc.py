"""The allocation-free step (mcc_collide_sorted_noalloc) against
mcc_collide_sorted, through the C ABI: the same velocities, counters and
per-cell correction-pair counts bit for bit, on two calls in a row (the
second with fewer cells and particles than the first, so the fixed array
holds the first call's lists), in the FP64 and FP32-kinematics forms; the
limits are refused or reported."""
import numpy as np
import pytest

from paper_2407_19151_amd import workloads as W

from gpu_helpers import custom_workload

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


def _run(ctx, wl, step, noalloc, **pover):
    from paper_2407_19151_amd import native, runner
    dw = runner.DeviceWorkload(wl)
    fn = ctx.collide_sorted_noalloc if noalloc else ctx.collide_sorted
    fn(dw.offsets, dw.w, dw.vx, dw.vy, dw.vz, n_cells=wl.n_cells, mass=wl.mass,
       charge=wl.charge, collisions=wl.collisions, dt=wl.dt, coulomb_log=wl.coulomb_log,
       seed=wl.seed, step=step, params=runner.params_for(wl, **pover),
       cell_volume=wl.cell_volume, stats=dw.stats, cell_corr_pairs=dw.cell_corr)
    return dw.velocities(), native.read_stats(dw.stats), dw.cell_corr.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_equals_the_sorted_step_on_two_calls(ctx, prec):
    big = W.config3(n_cells=3000)       # every size bucket up to 4096 particles
    small = custom_workload([(3, 2), (40, 33), (1, 0), (700, 512)], seed=71)
    for wl, step in ((big, 5), (small, 6)):
        print("noalloc case: cells %d n %d precision %d" % (wl.n_cells, wl.n, prec), flush=True)
        a = _run(ctx, wl, step, False, precision=prec)
        b = _run(ctx, wl, step, True, precision=prec)
        assert ctx.device_error() == 0
        assert np.array_equal(a[0], b[0])
        assert a[1] == b[1]
        assert np.array_equal(a[2], b[2])


def test_noalloc_limits(ctx):
    from paper_2407_19151_amd import native
    wl = custom_workload([(3000, 2000), (30, 20)], seed=72)
    v, st, _ = _run(ctx, wl, 1, True)
    assert ctx.device_error() == 2   # the 5000-particle cell is not stepped
    n0 = 5000
    assert np.array_equal(v[:, :n0], wl.velocities()[:, :n0])
    ref, _, _ = _run(ctx, wl, 1, False)
    assert np.array_equal(v[:, n0:], ref[:, n0:])
    rel = custom_workload([(10, 10)], seed=73, masses=(1.0, 1836.0), relativistic=True, c=1.0,
                          dt=0.003)
    with pytest.raises(native.MCCError) as e:
        _run(ctx, rel, 0, True)
    assert e.value.code == -4
    many = W.config1(n_cells=(1 << 18) + 1, ppc=1)
    with pytest.raises(native.MCCError) as e:
        _run(ctx, many, 0, True)
    assert e.value.code == -1
