"""The paper's Test 1 (Sec. 5.1 and its parameter table) in SI units: what
the workload and the conservation laws fix, on the CPU.

The equilibrium of two populations of one species follows from conservation
alone: the common drift is the density-weighted mean of the drifts, and the
common temperature is what remains of the total energy after that drift.
From the specified initial state this gives the paper's printed values
(59.55 km/s, 1.97 keV).  The sampled workload must carry the specified
densities exactly (through its weights) and the specified drifts and
temperatures to within sampling noise.  The oracle, run on a few cells,
conserves momentum and energy to rounding over many steps (the behaviour the
paper shows for the moment-corrected method)."""
import math

import numpy as np
import pytest

from paper_2407_19151_amd import workloads as W

from gpu_helpers import oracle_step


def closed_form_end_state(m, dens, temps_ev, drifts):
    """(U_f [m/s], T_f [eV]) from momentum and energy conservation."""
    n_tot = sum(dens)
    u_f = sum(n * u for n, u in zip(dens, drifts)) / n_tot
    e_tot = sum(n * (1.5 * t * W.E_CHARGE + 0.5 * m * u * u)
                for n, t, u in zip(dens, temps_ev, drifts))
    t_f = (e_tot / n_tot - 0.5 * m * u_f * u_f) / 1.5 / W.E_CHARGE
    return u_f, t_f


def test_specified_end_state_is_the_papers():
    m = 12.0 * W.M_U - 6.0 * W.M_ELECTRON
    u_f, t_f = closed_form_end_state(m, (1e25, 1e26), (500.0, 500.0), (655e3, 0.0))
    assert abs(u_f / 1e3 - 59.55) < 0.005       # printed: 59.55 km/s
    assert abs(t_f / 1e3 - 1.97) < 0.005        # printed: 1.97 keV


@pytest.mark.parametrize("case", sorted(W.PAPER_T1_CASES))
def test_workload_carries_the_specified_populations(case):
    wl = W.paper_test1(case)
    n_a, n_b, dt, f_e = W.PAPER_T1_CASES[case]
    pop = wl.extra["population"]
    assert wl.n == wl.n_cells * (n_a + n_b) and wl.n_cells == 180
    assert wl.dt == dt and wl.f_E == f_e and wl.coulomb_log == 10.0
    # densities exactly, through the weights
    for k, (npk, dens) in enumerate(((n_a, 1e25), (n_b, 1e26))):
        per_cell = np.bincount(wl.cells[pop == k], wl.w[pop == k], wl.n_cells)
        assert np.allclose(per_cell / wl.cell_volume, dens, rtol=1e-12)
    # the weight ratio of the table
    ratio = {"T1a": 1.0, "T1b": 0.1, "T1c": 0.01, "T1d": 4.0}[case]
    assert math.isclose(wl.w[pop == 0][0] / wl.w[pop == 1][0], ratio, rel_tol=1e-12)
    # drifts and temperatures within 5 sigma of the sample size
    mom = W.population_moments(wl, wl.velocities())
    m = wl.mass[0]
    for k, (npk, u0, t0) in enumerate(((n_a, 655e3, 500.0), (n_b, 0.0, 500.0))):
        count = npk * wl.n_cells
        sig_v = math.sqrt(t0 * W.E_CHARGE / m)
        assert abs(mom[k][0] - u0) < 5 * sig_v / math.sqrt(count)
        assert abs(mom[k][1] / t0 - 1.0) < 5 * math.sqrt(2.0 / (3.0 * count))


def test_oracle_conserves_to_rounding_over_many_steps():
    wl = W.paper_test1("T1b", n_cells=4)
    ref = wl.copy()
    m = wl.mass[0]

    def totals(v):
        return (wl.w * v[0]).sum(), (0.5 * m * wl.w * (v * v).sum(0)).sum()

    p0, e0 = totals(ref.velocities())
    for s in range(300):
        oracle_step(ref, s)
    p1, e1 = totals(ref.velocities())
    assert abs(p1 - p0) / abs(p0) < 1e-13
    assert abs(e1 - e0) / e0 < 1e-13
    # and the drift has relaxed measurably (the collisions act)
    assert W.population_moments(wl, ref.velocities())[0][0] < 0.9 * 655e3
