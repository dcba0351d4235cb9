"""The differentiated form (forward mode) against the oracle.

The reference derivative is a same-seed central difference of the CPU
oracle: with every random number fixed by (seed, step), the step is a smooth
map of the velocities and of ln(Lambda) away from its discrete switches (the
cut pair of the energy correction, the failure decision).  Cells whose
correction-pair count differs between the perturbed oracle runs crossed a
switch and are left out.  Bar per particle: |J t - FD| <= 1e-6 of the
tangent's (cell, species) scale plus 10x the difference's own error, which is
estimated from two step sizes (h and h/2; central differences are
second-order).  Measured: median 7e-11, largest 3e-8 (electrons that scatter
500 times in one step)."""
import numpy as np
import pytest

from paper_2407_19151_amd import workloads as W

from gpu_helpers import custom_workload, oracle_step

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


def _scale(wl, x):
    key = wl.cells.astype(np.int64) * wl.n_species + wl.species
    ss = np.bincount(key, (x * x).sum(0), wl.n_cells * wl.n_species)
    c = np.bincount(key, None, wl.n_cells * wl.n_species)
    return np.sqrt(ss / np.maximum(c, 1))[key]


def _gpu_tangent(ctx, wl, t, step, dlnl, update_primal=True):
    import torch
    from paper_2407_19151_amd import runner
    dw = runner.DeviceWorkload(wl)
    T = torch.as_tensor(t, device="cuda").contiguous()
    runner.collide_sorted_jvp(ctx, dw, T, step, coulomb_log_tangent=dlnl,
                              update_primal=update_primal)
    assert ctx.device_error() == 0
    return T.cpu().numpy(), dw.velocities()


def _oracle_fd(wl, t, step, dlnl, h):
    v0 = wl.velocities()
    out = []
    for sgn in (1.0, -1.0):
        w2 = wl.copy()
        w2.vx, w2.vy, w2.vz = (v0 + sgn * h * t)
        so = oracle_step(w2, step, coulomb_log=wl.coulomb_log + sgn * h * dlnl)
        out.append((w2.velocities(), so["cell_corr_pairs"].copy()))
    (vp, cp), (vm, cm) = out
    return (vp - vm) / (2.0 * h), cp != cm


CASES = {
    "c5_velocity": (lambda: W.config5(n_cells=16), 0, 0.0),
    "c5_velocity_and_lnL": (lambda: W.config5(n_cells=16), 3, 1.0),
    "c2_TA77": (lambda: W.config2(n_cells=16, method=W.TA77), 2, 0.5),
    "c2_N97": (lambda: W.config2(n_cells=16), 2, 0.5),
    "cell_4095": (lambda: custom_workload([(2047, 2048)], seed=4), 1, 0.5),
    "mixed_cells": (lambda: custom_workload([(700, 300), (60, 50), (5000, 10), (3, 2)], seed=4),
                    1, 0.5),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_tangent_matches_oracle_central_differences(ctx, case):
    make, step, dlnl = CASES[case]
    wl = make()
    rng = np.random.default_rng(3)
    v0 = wl.velocities().copy()
    t = rng.normal(size=v0.shape) * _scale(wl, v0)
    jt, _ = _gpu_tangent(ctx, wl, t, step, dlnl)
    fd1, flip1 = _oracle_fd(wl, t, step, dlnl, 1e-6)
    fd2, flip2 = _oracle_fd(wl, t, step, dlnl, 5e-7)
    keep = ~(flip1 | flip2)[wl.cells]
    sc = np.maximum(_scale(wl, fd2), 1e-300)
    err = np.abs(jt - fd2).max(0) / sc
    est = np.abs(fd1 - fd2).max(0) / sc
    print("%s: %d of %d cells crossed a switch; |Jt - FD| median %.2e max %.2e" % (
        case, int((flip1 | flip2).sum()), wl.n_cells, np.median(err[keep]), err[keep].max()),
        flush=True)
    assert keep.mean() > 0.9
    assert np.all(np.isfinite(jt))
    assert np.all(err[keep] <= 1e-6 + 10.0 * est[keep])


def test_tangent_is_linear_and_zero_at_zero(ctx):
    wl = W.config5(n_cells=8)
    rng = np.random.default_rng(5)
    n = wl.n
    t1, t2 = rng.normal(size=(3, n)), rng.normal(size=(3, n))
    z, _ = _gpu_tangent(ctx, wl, np.zeros((3, n)), 1, 0.0)
    assert np.all(z == 0.0)
    j1, _ = _gpu_tangent(ctx, wl, t1, 1, 0.3)
    j2, _ = _gpu_tangent(ctx, wl, t2, 1, -0.7)
    j12, _ = _gpu_tangent(ctx, wl, 2.0 * t1 - 3.0 * t2, 1, 2.0 * 0.3 - 3.0 * -0.7)
    sc = np.abs(j12).max()
    assert np.abs(j12 - (2.0 * j1 - 3.0 * j2)).max() <= 1e-11 * sc


def test_tangent_primal_flag(ctx):
    from paper_2407_19151_amd import runner
    wl = W.config5(n_cells=8)
    t = np.random.default_rng(2).normal(size=(3, wl.n))
    _, v_kept = _gpu_tangent(ctx, wl, t, 4, 0.0, update_primal=False)
    assert np.array_equal(v_kept, wl.velocities())
    _, v_step = _gpu_tangent(ctx, wl, t, 4, 0.0, update_primal=True)
    dw = runner.DeviceWorkload(wl)
    runner.collide_sorted(ctx, dw, 4, with_stats=False)
    assert np.abs(v_step - dw.velocities()).max() <= 1e-13 * np.abs(wl.velocities()).max()


def _temps(wl, v):
    out = []
    for sp in range(2):
        k = wl.species == sp
        w, vs = wl.w[k], v[:, k]
        mean = (vs * w).sum(1, keepdims=True) / w.sum()
        out.append(wl.mass[sp] * (w * ((vs - mean) ** 2).sum(0)).sum() / (3.0 * w.sum()))
    return np.array(out)


def test_relaxation_jacobian_matches_oracle_differences(ctx):
    """d(T_e, T_i)_final / d(T_e0, T_i0, lnL) over 10 steps of the
    reparameterised relaxation v0 = sqrt(T0/m) xi, against central differences
    of the oracle run from the same xi and seed."""
    from paper_2407_19151_amd import autodiff
    steps, Te0, Ti0, lnl = 10, 2.0, 1.0, 10.0
    wl = W.config5(n_cells=8, Te0=Te0, Ti0=Ti0)
    xi = W.standard_normal_state(wl, 5)
    T, J = autodiff.relaxation_jacobian(ctx, wl, xi, Te0, Ti0, lnl, steps)
    T, J = T.cpu().numpy(), J.cpu().numpy()
    m = wl.mass[wl.species]

    def oracle_T(te0, ti0, ll):
        w2 = wl.copy()
        T0 = np.where(wl.species == 0, te0, ti0)
        w2.vx, w2.vy, w2.vz = np.sqrt(T0 / m) * xi
        for k in range(steps):
            oracle_step(w2, k, coulomb_log=ll)
        return _temps(wl, w2.velocities())

    T_or = oracle_T(Te0, Ti0, lnl)
    assert np.allclose(T, T_or, rtol=1e-10, atol=0)
    base = np.array([Te0, Ti0, lnl])
    Jfd = np.zeros((2, 3))
    for d in range(3):
        h = 1e-6 * base[d]
        e = np.zeros(3)
        e[d] = h
        Jfd[:, d] = (oracle_T(*(base + e)) - oracle_T(*(base - e))) / (2.0 * h)
    print("J gpu:\n", J, "\nJ oracle FD:\n", Jfd, flush=True)
    assert np.allclose(J, Jfd, rtol=1e-5, atol=1e-7 * np.abs(Jfd).max())


def test_torch_functions(ctx):
    """Relaxation's backward is J^T g; CollideStep's jvp rule is the tangent
    kernel (checked through torch.autograd.forward_ad)."""
    import torch
    from paper_2407_19151_amd import autodiff, runner
    wl = W.config5(n_cells=4)
    xi = W.standard_normal_state(wl, 5)
    te = torch.tensor(2.0, dtype=torch.float64, device="cuda", requires_grad=True)
    ti = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    ll = torch.tensor(10.0, dtype=torch.float64, device="cuda", requires_grad=True)
    Te, Ti, J = autodiff.Relaxation.apply(te, ti, ll, ctx, wl, xi, 5)
    (3.0 * Te - 2.0 * Ti).backward()
    g = torch.stack([te.grad, ti.grad, ll.grad]).cpu().numpy()
    assert np.allclose(g, np.array([3.0, -2.0]) @ J.cpu().numpy(), rtol=1e-14, atol=0)

    dw = runner.DeviceWorkload(wl)
    params = runner.params_for(wl)
    v = torch.stack([dw.vx, dw.vy, dw.vz]).contiguous()
    t = torch.as_tensor(np.random.default_rng(9).normal(size=(3, wl.n)), device="cuda")
    lnl = torch.tensor(wl.coulomb_log, dtype=torch.float64)
    import torch.autograd.forward_ad as fwAD
    with fwAD.dual_level():
        dv = fwAD.make_dual(v, t)
        dl = fwAD.make_dual(lnl, torch.tensor(0.5, dtype=torch.float64))
        out, tout = fwAD.unpack_dual(autodiff.CollideStep.apply(dv, dl, ctx, dw, 2, params))
    jt, vstep = _gpu_tangent(ctx, wl, t.cpu().numpy(), 2, 0.5)
    assert np.array_equal(tout.cpu().numpy(), jt)
    assert np.abs(out.cpu().numpy() - vstep).max() <= 1e-13 * np.abs(vstep).max()
