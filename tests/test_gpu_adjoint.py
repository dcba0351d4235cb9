"""The reverse-mode form (mcc_collide_adjoint) against the forward mode, the
oracle's central differences and, for the relaxation of the fifth synthetic
workload, the forward-mode Jacobian.

- Transpose: the step's Jacobian is block-diagonal over cells, so for every
  cell <g, J t> (forward mode) equals <J^T g, t> (reverse mode), and the lnL
  parts agree: g dv'/dlnL against <g, J_lnL>.  Both run the same discrete
  choices (the reverse kernel takes the forward-mode kernel's threads per
  cell, so its sums round and its cut pairs fall alike); they differ in the
  association of the products only.  Bar: 1e-11 of sum |g||Jt| + |J^T g||t|
  per cell.
- Central differences of the oracle, with every random number fixed by
  (seed, step): <g, (F(v + h t) - F(v - h t)) / 2h> per cell, cells whose
  correction-pair count changes between the perturbed runs excluded (they
  crossed a switch).  Bar: 1e-6 of the cell's scale plus 10 times the
  difference's own error (two step sizes).
- The FP32-kinematics form against the oracle's differences with the form's
  23-bit uniforms, at 1e-4.
- The relaxation of 1024 cells x (256 e + 256 i) over 50 steps with
  checkpoints every 10: the gradient of (T_e, T_i)_final with respect to
  (T_e0, T_i0, lnL) from the reverse sweep equals J^T g of the forward-mode
  Jacobian along the same trajectory.  Over 50 steps this pathwise gradient
  (every random number fixed) is dominated by the chaotic growth of
  perturbations through the collisions: across Philox seeds it ranges over
  -170..+570 for a component whose 10-step value is 2.79 +- 0.01, while the
  temperatures agree to 0.2 %.  So the FP32 form, whose 23-bit uniforms make
  its path a different realization, is compared with the FP64 form over 10
  steps (1e-3), and the 10-step reverse-mode gradient is checked against the
  oracle's same-seed central differences.
"""
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


def _percell(wl, x):
    return np.bincount(wl.cells, x, wl.n_cells)


def _gpu_vjp(ctx, wl, g, step, **pover):
    """(J^T g, g dv'/dlnL) of the step of wl from its current state."""
    import torch
    from paper_2407_19151_amd import runner
    dw = runner.DeviceWorkload(wl)
    v = torch.stack([dw.vx, dw.vy, dw.vz]).contiguous()
    G = torch.as_tensor(np.ascontiguousarray(g), device="cuda").contiguous()
    gl = torch.zeros(1, dtype=torch.float64, device="cuda")
    runner.collide_adjoint(ctx, dw, v, G, step, g_lnl=gl,
                           params=runner.params_for(wl, **pover))
    assert ctx.device_error() == 0
    assert np.array_equal(torch.stack([dw.vx, dw.vy, dw.vz]).cpu().numpy(), wl.velocities())
    return G.cpu().numpy(), float(gl.item())


def _gpu_jvp(ctx, wl, t, step, dlnl, **pover):
    import torch
    from paper_2407_19151_amd import runner
    dw = runner.DeviceWorkload(wl)
    T = torch.as_tensor(np.ascontiguousarray(t), device="cuda").contiguous()
    runner.collide_sorted_jvp(ctx, dw, T, step, coulomb_log_tangent=dlnl,
                              params=runner.params_for(wl, **pover), update_primal=False)
    assert ctx.device_error() == 0
    return T.cpu().numpy()


CASES = {
    "c5": (lambda: W.config5(n_cells=16), 0, {}),
    "c2_TA77": (lambda: W.config2(n_cells=16, method=W.TA77), 2, {}),
    "c2_N97": (lambda: W.config2(n_cells=16), 3, {}),
    "c1_lognormal": (lambda: W.config1(), 1, {}),
    "cell_4095": (lambda: custom_workload([(2047, 2048)], seed=4), 1, {}),
    "mixed_cells": (lambda: custom_workload([(700, 300), (60, 50), (5000, 10), (3, 2), (1, 1),
                                             (0, 7), (2, 0)], seed=4), 1, {}),
    "no_correction": (lambda: W.config2(n_cells=8), 2, {"moment_correction": 0}),
    "no_sort": (lambda: custom_workload([(300, 200), (41, 17)], seed=6,
                                        weight_mode="lognormal"), 2, {"sort_by_weight": 0}),
    "two_weight_classes": (lambda: custom_workload([(300, 200), (41, 17)], seed=7,
                                                   weight_mode="two"), 0, {}),
    "forced_failures_keep": (lambda: W.config2(n_cells=12), 3, {"f_E": 0.01, "on_failure": 1}),
    "forced_failures_reset": (lambda: W.config2(n_cells=12), 3, {"f_E": 0.01}),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_adjoint_is_the_transpose_of_the_tangent(ctx, case):
    make, step, pover = CASES[case]
    wl = make()
    print("adjoint transpose case %s: cells %d n %d" % (case, wl.n_cells, wl.n), flush=True)
    rng = np.random.default_rng(11)
    v0 = wl.velocities()
    sc = _scale(wl, v0)
    g = rng.normal(size=v0.shape) / np.maximum(sc, 1e-300)
    t = rng.normal(size=v0.shape) * sc
    jt = _gpu_jvp(ctx, wl, t, step, 0.0, **pover)
    jl = _gpu_jvp(ctx, wl, np.zeros_like(t), step, 1.0, **pover)
    gj, gl = _gpu_vjp(ctx, wl, g, step, **pover)
    a = _percell(wl, (g * jt).sum(0))
    b = _percell(wl, (gj * t).sum(0))
    size = _percell(wl, np.abs(g * jt).sum(0) + np.abs(gj * t).sum(0))
    err = np.abs(a - b) / np.maximum(size, 1e-300)
    print("  <g, Jt> vs <J^T g, t> per cell: max %.2e; lnL: %.15e vs %.15e"
          % (err.max(), float((g * jl).sum()), gl), flush=True)
    assert np.all(np.isfinite(gj))
    assert err.max() <= 1e-11
    jls = float((g * jl).sum())
    assert abs(jls - gl) <= 1e-11 * (np.abs(g * jl).sum() + 1e-300)


def _oracle_dir(wl, g, t, step, dlnl, h, **over):
    """<g, (F(v + h t, lnL + h dlnl) - F(v - h t, lnL - h dlnl)) / 2h> per cell,
    and the cells whose correction-pair count differs between the runs."""
    v0 = wl.velocities()
    out = []
    for sgn in (1.0, -1.0):
        w2 = wl.copy()
        w2.vx, w2.vy, w2.vz = (v0 + sgn * h * t)
        so = oracle_step(w2, step, coulomb_log=wl.coulomb_log + sgn * h * dlnl, **over)
        out.append((w2.velocities(), so["cell_corr_pairs"].copy()))
    (vp, cp), (vm, cm) = out
    return _percell(wl, (g * (vp - vm)).sum(0)) / (2.0 * h), cp != cm


@pytest.mark.parametrize("case,fp32", [("c5", False), ("mixed", False), ("c5", True)])
def test_adjoint_matches_oracle_central_differences(ctx, case, fp32):
    from paper_2407_19151_amd import native
    if case == "c5":
        wl, step = W.config5(n_cells=16), 2
    else:
        wl, step = custom_workload([(700, 300), (60, 50), (2100, 10), (3, 2)], seed=8), 1
    pover = {"precision": native.MCC_FP32_KINEMATICS} if fp32 else {}
    oover = {"uniform23": True} if fp32 else {}
    rng = np.random.default_rng(21)
    v0 = wl.velocities()
    sc = _scale(wl, v0)
    g = rng.normal(size=v0.shape) / np.maximum(sc, 1e-300)
    t = rng.normal(size=v0.shape) * sc
    gj, _ = _gpu_vjp(ctx, wl, g, step, **pover)
    b = _percell(wl, (gj * t).sum(0))
    fd1, flip1 = _oracle_dir(wl, g, t, step, 0.0, 1e-6, **oover)
    fd2, flip2 = _oracle_dir(wl, g, t, step, 0.0, 5e-7, **oover)
    keep = ~(flip1 | flip2)
    size = _percell(wl, np.abs(gj * t).sum(0))
    err = np.abs(b - fd2) / np.maximum(size, 1e-300)
    est = np.abs(fd1 - fd2) / np.maximum(size, 1e-300)
    bar = 1e-4 if fp32 else 1e-6
    print("%s fp32=%s: %d of %d cells crossed a switch; |<J^T g,t> - FD| max %.2e "
          "(FD error est. %.2e)" % (case, fp32, int((~keep).sum()), wl.n_cells,
                                    err[keep].max(), est[keep].max()), flush=True)
    assert keep.mean() > 0.8
    assert np.all(err[keep] <= bar + 10.0 * est[keep])
    if not fp32:
        # the lnL adjoint against the oracle's difference in lnL alone
        _, gl = _gpu_vjp(ctx, wl, g, step, **pover)
        l1, f1 = _oracle_dir(wl, g, np.zeros_like(t), step, 1.0, 1e-6 * wl.coulomb_log)
        l2, f2 = _oracle_dir(wl, g, np.zeros_like(t), step, 1.0, 5e-7 * wl.coulomb_log)
        if not (f1 | f2).any():
            e = abs(gl - l2.sum()) / (np.abs(l2).sum() + 1e-300)
            print("  lnL: adjoint %.10e FD %.10e rel %.2e" % (gl, l2.sum(), e), flush=True)
            assert e <= 1e-6 + 10.0 * abs(l1.sum() - l2.sum()) / (np.abs(l2).sum() + 1e-300)


def test_torch_collide_step_backward(ctx):
    """CollideStep's backward is the adjoint kernel: <g, J t> from the jvp
    rule equals <backward(g), t>, and the lnL gradient matches."""
    import torch
    from paper_2407_19151_amd import autodiff, runner
    wl = W.config5(n_cells=4)
    dw = runner.DeviceWorkload(wl)
    params = runner.params_for(wl)
    v = torch.stack([dw.vx, dw.vy, dw.vz]).contiguous().requires_grad_(True)
    lnl = torch.tensor(wl.coulomb_log, dtype=torch.float64, device="cuda", requires_grad=True)
    rng = np.random.default_rng(4)
    g = torch.as_tensor(rng.normal(size=(3, wl.n)), device="cuda")
    t = rng.normal(size=(3, wl.n))
    out = autodiff.CollideStep.apply(v, lnl, ctx, dw, 3, params)
    (out * g).sum().backward()
    jt = _gpu_jvp(ctx, wl, t, 3, 0.0)
    jl = _gpu_jvp(ctx, wl, np.zeros_like(t), 3, 1.0)
    a = float((g.cpu().numpy() * jt).sum())
    b = float((v.grad.cpu().numpy() * t).sum())
    assert abs(a - b) <= 1e-11 * np.abs(g.cpu().numpy() * jt).sum()
    c = float((g.cpu().numpy() * jl).sum())
    assert abs(c - lnl.grad.item()) <= 1e-11 * np.abs(g.cpu().numpy() * jl).sum()


def test_unsupported_forms(ctx):
    from paper_2407_19151_amd import native
    wl = custom_workload([(10, 10)], seed=38)
    g = np.ones((3, wl.n))
    for over, code in (({"pairing": 1}, -4), ({"pairing": 2}, -4), ({"max_passes": 2}, -4),
                       ({"method": 2}, -4)):
        with pytest.raises(native.MCCError) as e:
            _gpu_vjp(ctx, wl, g, 0, **over)
        assert e.value.code == code, over
    wr = custom_workload([(10, 10)], seed=38, masses=(1.0, 1836.0), relativistic=True, c=1.0,
                         dt=0.003)
    with pytest.raises(native.MCCError) as e:
        _gpu_vjp(ctx, wr, g, 0)
    assert e.value.code == -4


def _relax_grad(ctx, wl, xi, steps, prec, gT, Te0=2.0, Ti0=1.0, lnl0=10.0):
    import torch
    from paper_2407_19151_amd import autodiff, runner
    te = torch.tensor(Te0, dtype=torch.float64, device="cuda", requires_grad=True)
    ti = torch.tensor(Ti0, dtype=torch.float64, device="cuda", requires_grad=True)
    ll = torch.tensor(lnl0, dtype=torch.float64, device="cuda", requires_grad=True)
    Te, Ti = autodiff.RelaxationAdjoint.apply(te, ti, ll, ctx, wl, xi, steps, 10,
                                              runner.params_for(wl, precision=prec))
    (gT[0] * Te + gT[1] * Ti).backward()
    return (np.array([te.grad.item(), ti.grad.item(), ll.grad.item()]),
            np.array([Te.item(), Ti.item()]))


def test_c5_relaxation_gradient_reverse_and_forward(ctx):
    """The fifth synthetic workload at its size: 1024 cells x (256 e + 256 i),
    50 steps, checkpoints every 10.  Reverse mode (checkpointed adjoint
    sweep) against the forward-mode Jacobian J along the same trajectory:
    the gradient of gTe T_e + gTi T_i with respect to (T_e0, T_i0, lnL)
    equals (gTe, gTi) J to 1e-9 of its largest component (FP64; the two
    accumulate a product of 50 step Jacobians in opposite orders).  The
    FP32-kinematics form's 10-step gradient agrees with the FP64 one to
    1e-3."""
    from paper_2407_19151_amd import autodiff, native
    Te0, Ti0, lnl0 = 2.0, 1.0, 10.0
    wl = W.config5(Te0=Te0, Ti0=Ti0)
    assert wl.n_cells == 1024 and wl.n == 1024 * 512
    xi = W.standard_normal_state(wl, 5)
    gT = np.array([3.0, -2.0])
    T, J = autodiff.relaxation_jacobian(ctx, wl, xi, Te0, Ti0, lnl0, 50)
    want = gT @ J.cpu().numpy()
    g64, T64 = _relax_grad(ctx, wl, xi, 50, native.MCC_FP64, gT)
    assert np.all(np.abs(T64 / T.cpu().numpy() - 1) < 1e-13)
    rel = np.abs(g64 - want) / np.abs(want).max()
    g10, _ = _relax_grad(ctx, wl, xi, 10, native.MCC_FP64, gT)
    g10f, _ = _relax_grad(ctx, wl, xi, 10, native.MCC_FP32_KINEMATICS, gT)
    r32 = np.abs(g10f - g10) / np.abs(g10).max()
    assert ctx.device_error() == 0
    print("C5 gradient of 3 T_e - 2 T_i by (Te0, Ti0, lnL), 50 steps: forward %s, reverse %s "
          "(max rel %.2e); 10 steps: fp64 %s, fp32 %s (max rel %.2e)"
          % (want, g64, rel.max(), g10, g10f, r32.max()), flush=True)
    assert rel.max() <= 1e-9
    assert r32.max() <= 1e-3


def test_relaxation_adjoint_matches_oracle_differences(ctx):
    """The reverse-mode relaxation gradient over 10 steps (checkpoints every
    4, so three segments are recomputed) on 8 cells of the fifth workload,
    against central differences of the oracle from the same xi and seed."""
    from paper_2407_19151_amd import autodiff, native, runner
    import torch
    steps, Te0, Ti0, lnl = 10, 2.0, 1.0, 10.0
    wl = W.config5(n_cells=8, Te0=Te0, Ti0=Ti0)
    xi = W.standard_normal_state(wl, 5)
    gT = np.array([1.5, 0.5])
    te = torch.tensor(Te0, dtype=torch.float64, device="cuda", requires_grad=True)
    ti = torch.tensor(Ti0, dtype=torch.float64, device="cuda", requires_grad=True)
    ll = torch.tensor(lnl, dtype=torch.float64, device="cuda", requires_grad=True)
    Te, Ti = autodiff.RelaxationAdjoint.apply(te, ti, ll, ctx, wl, xi, steps, 4,
                                              runner.params_for(wl))
    (gT[0] * Te + gT[1] * Ti).backward()
    g = np.array([te.grad.item(), ti.grad.item(), ll.grad.item()])
    m = wl.mass[wl.species]

    def oracle_L(te0, ti0, l):
        w2 = wl.copy()
        T0 = np.where(wl.species == 0, te0, ti0)
        w2.vx, w2.vy, w2.vz = np.sqrt(T0 / m) * xi
        for k in range(steps):
            oracle_step(w2, k, coulomb_log=l)
        v = w2.velocities()
        out = []
        for sp in range(2):
            k = wl.species == sp
            w, vs = wl.w[k], v[:, k]
            mean = (vs * w).sum(1, keepdims=True) / w.sum()
            out.append(wl.mass[sp] * (w * ((vs - mean) ** 2).sum(0)).sum() / (3.0 * w.sum()))
        return float(gT @ np.array(out))

    base = np.array([Te0, Ti0, lnl])
    fd = np.zeros(3)
    for d in range(3):
        h = 1e-6 * base[d]
        e = np.zeros(3)
        e[d] = h
        fd[d] = (oracle_L(*(base + e)) - oracle_L(*(base - e))) / (2.0 * h)
    print("10-step gradient: reverse %s, oracle FD %s" % (g, fd), flush=True)
    assert np.allclose(g, fd, rtol=1e-5, atol=1e-7 * np.abs(fd).max())
