"""The paper's Test 2 (Sec. 5.2 and its parameter table) in SI units: what
the workload and the conservation laws fix, on the CPU.

Three populations of C^6+ in two species: A alone in species alpha, B and C
in species beta.  The table prints, per case, the counts N_A, N_B, N_C, their
ratios, N_alpha : N_beta and the weight ratios w_A : w_B : w_C.  Weights are
n_k dV / N_k, so the printed weight ratios fix the density ratio
n_A : n_B : n_C; every row gives 2 : 20 : 1, i.e. n_C = 5e18 cm^-3 next to
the specified n_A = 1e19 and n_B = 1e20 (the text's 1e18 would give weight
ratios five times off for C in every row).  The workload must reproduce the
printed ratio columns exactly.

The equilibrium follows from conservation alone (all three populations have
one mass): the common drift is the density-weighted mean drift and the common
temperature is what remains of the total energy after it.  The oracle, on a
few cells of the most unequal weighting (1 : 400 : 4), conserves momentum and
energy to rounding over many steps."""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2407_19151_amd import workloads as W

from gpu_helpers import oracle_step
from test_paper_test1 import closed_form_end_state

# the table's printed ratio columns: N_A:N_B:N_C, N_alpha:N_beta, w_A:w_B:w_C
TABLE_RATIOS = {
    "T2a": ((2, 20, 1), (1, 10.5), (1, 1, 1)),
    "T2b": ((1, 10, 2), (1, 12), (4, 4, 1)),
    "T2c": ((1, 2, 10), (1, 12), (20, 100, 1)),
    "T2d": ((40, 5, 1), (40, 6), (1, 80, 20)),
    "T2e": ((40, 1, 5), (40, 6), (1, 400, 4)),
}


def _same_ratio(a, b):
    fa = [Fraction(x).limit_denominator(1000) for x in a]
    fb = [Fraction(x).limit_denominator(1000) for x in b]
    return all(x * fb[0] == y * fa[0] for x, y in zip(fa, fb))


@pytest.mark.parametrize("case", sorted(W.PAPER_T2_CASES))
def test_workload_reproduces_the_table(case):
    wl = W.paper_test2(case)
    n_a, n_b, n_c = W.PAPER_T2_CASES[case]
    pop = wl.extra["population"]
    counts_r, species_r, weights_r = TABLE_RATIOS[case]
    assert _same_ratio((n_a, n_b, n_c), counts_r)
    assert _same_ratio((n_a, n_b + n_c), species_r)
    w = [wl.w[pop == k][0] for k in range(3)]
    for k in range(3):
        assert np.all(wl.w[pop == k] == w[k])
    assert all(math.isclose(w[k] / w[0], weights_r[k] / weights_r[0], rel_tol=1e-12)
               for k in range(3))
    # species layout: A alone in alpha, B and C in beta
    assert np.all(wl.species[pop == 0] == 0) and np.all(wl.species[pop > 0] == 1)
    assert wl.collisions == [(0, 0), (1, 1), (0, 1)]
    assert wl.dt == 50e-15 and wl.f_E == 0.05 and wl.coulomb_log == 10.0


def test_the_texts_density_of_c_contradicts_the_table():
    """With n_C = 1e18 cm^-3 no row's weight ratios come out as printed."""
    for case, (n_a, n_b, n_c) in W.PAPER_T2_CASES.items():
        w = (1e25 / n_a, 1e26 / n_b, 1e24 / n_c)
        assert not _same_ratio(w, TABLE_RATIOS[case][2])


@pytest.mark.parametrize("case", ["T2a", "T2e"])
def test_workload_carries_the_specified_populations(case):
    wl = W.paper_test2(case)
    pop = wl.extra["population"]
    m = wl.mass[0]
    counts = W.PAPER_T2_CASES[case]
    mom = W.population_moments(wl, wl.velocities())
    for k, (npk, dens, u0) in enumerate(zip(counts, (1e25, 1e26, 5e24), (655e3, 0.0, -655e3))):
        per_cell = np.bincount(wl.cells[pop == k], wl.w[pop == k], wl.n_cells)
        assert np.allclose(per_cell / wl.cell_volume, dens, rtol=1e-12)
        count = npk * wl.n_cells
        sig_v = math.sqrt(500.0 * W.E_CHARGE / m)
        assert abs(mom[k][0] - u0) < 5 * sig_v / math.sqrt(count)
        assert abs(mom[k][1] / 500.0 - 1.0) < 5 * math.sqrt(2.0 / (3.0 * count))


def test_end_state_from_conservation():
    m = 12.0 * W.M_U - 6.0 * W.M_ELECTRON
    u_f, t_f = closed_form_end_state(m, (1e25, 1e26, 5e24), (500.0,) * 3, (655e3, 0.0, -655e3))
    # drift: (n_A - n_C) U / n_total exactly; the temperature gains the drift
    # energy lost, (n_A + n_C) m U^2 / 2 less n m U_f^2 / 2, over 3 n / 2
    n = 1.15e26
    assert math.isclose(u_f, 5e24 * 655e3 / n, rel_tol=1e-12)
    gain = (1.5e25 * 0.5 * m * 655e3 ** 2 - n * 0.5 * m * u_f ** 2) / (1.5 * n) / W.E_CHARGE
    assert math.isclose(t_f, 500.0 + gain, rel_tol=1e-12)
    assert abs(u_f / 1e3 - 28.48) < 0.01 and abs(t_f - 2785.7) < 0.1


def test_oracle_conserves_to_rounding_over_many_steps():
    wl = W.paper_test2("T2e", n_cells=3)
    ref = wl.copy()
    m = wl.mass[0]

    def totals(v):
        return (wl.w * v[0]).sum(), (0.5 * m * wl.w * (v * v).sum(0)).sum()

    p0, e0 = totals(ref.velocities())
    for s in range(200):
        oracle_step(ref, s)
    p1, e1 = totals(ref.velocities())
    assert abs(p1 - p0) / abs(p0) < 1e-13
    assert abs(e1 - e0) / e0 < 1e-13
    mom = W.population_moments(wl, ref.velocities())
    # the beams have slowed measurably
    assert mom[0][0] < 0.9 * 655e3 and mom[2][0] > -0.9 * 655e3
