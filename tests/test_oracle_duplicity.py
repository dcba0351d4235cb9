"""The oracle's duplicity pairing (the variant of Higginson et al. that the
paper describes after Sec. 3.2) pinned to what the paper fixes.

The pairs are the order-N pairs; an inter-species pair's s is Eq. (12)
with N_max / D in place of N_min, D the number of pairs its fewer-population
particle takes in the step.

- When N_max is a multiple of N_min every D equals N_max / N_min, the
  average the paper names, and the step is the order-N step bit for bit.
- Otherwise D depends on the shuffle.  For a 3 + 2 cell the second particle
  of the shorter list takes one pair (D = 1) and the first takes two
  (D = 2).  Grouping replica cells by their shuffled lists, the mean velocity
  change of every particle in every group is the drag sum of Eq. (8)
  over that group's pairs with the duplicity s; the order-N s (N_min), the
  N_max s without the division by D, and the N x N s (1) each fit far worse.
"""
import math

import numpy as np
import pytest

import oracle

MASS = (1.0, 4.0)
CHARGE = (-1.0, 2.0)
LNL, DT, DV, SEED = 10.0, 0.004, 1.0, 7


@pytest.mark.parametrize("na,nb", [(6, 2), (2, 6), (9, 3), (4, 4), (5, 1)])
@pytest.mark.parametrize("correction", [False, True])
def test_integer_ratio_is_the_order_n_step(na, nb, correction):
    rng = np.random.default_rng(na * 10 + nb)
    n = na + nb
    off = np.array([0, na, n], dtype=np.int64)
    w = np.concatenate([np.full(na, 1.0), np.full(nb, 2.5)])
    v = rng.normal(size=(3, n))
    res = []
    for pairing in (oracle.ORDER_N, oracle.DUPLICITY):
        vx, vy, vz = (v[k].copy() for k in range(3))
        oracle.collide_sorted(off, MASS, CHARGE, [(0, 0), (1, 1), (0, 1)], w, vx, vy, vz,
                              dt=0.2, coulomb_log=LNL, seed=3, step=1, pairing=pairing,
                              correction=correction)
        res.append(np.stack([vx, vy, vz]))
    assert np.array_equal(res[0], res[1])


def _cell():
    w = np.array([1.0, 2.0, 1.5, 1.5, 3.0])
    v = np.array([[1.0, -0.5, -0.5, 0.0, 0.0],
                  [0.0, 0.866, -0.866, 0.0, 0.0],
                  [0.0, 0.0, 0.0, 1.2, -1.2]])
    return w, v


def _predict(w, v, L0, L1, nfac_of_k):
    """First-order mean change of the 5 particles for the pairs of one
    shuffle: pair k = (L0[k], 3 + L1[k mod 2])."""
    out = np.zeros((3, 5))
    m = np.array([MASS[0]] * 3 + [MASS[1]] * 2)
    q = np.array([CHARGE[0]] * 3 + [CHARGE[1]] * 2)
    for k in range(3):
        i, j = L0[k], 3 + L1[k % 2]
        mu = m[i] * m[j] / (m[i] + m[j])
        u = v[:, i] - v[:, j]
        s = (q[i] ** 2 * q[j] ** 2 * LNL * DT / (4 * math.pi * mu ** 2)) \
            * max(w[i], w[j]) * nfac_of_k(k) / DV / np.linalg.norm(u) ** 3
        mean_du = -(1.0 - math.exp(-s)) * u
        pi = 1.0 if w[i] <= w[j] else w[j] / w[i]
        pj = 1.0 if w[j] <= w[i] else w[i] / w[j]
        out[:, i] += pi * mu / m[i] * mean_du
        out[:, j] -= pj * mu / m[j] * mean_du
    return out


def test_drag_per_shuffle_uses_the_duplicity():
    w, v = _cell()
    n_cells, steps = 20000, 16
    groups = {}
    for step in range(steps):
        off = np.zeros(2 * n_cells + 1, dtype=np.int64)
        np.cumsum(np.tile([3, 2], n_cells), out=off[1:])
        vx, vy, vz = (np.tile(v[k], n_cells) for k in range(3))
        oracle.collide_sorted(off, MASS, CHARGE, [(0, 1)], np.tile(w, n_cells), vx, vy, vz,
                              dt=DT, coulomb_log=LNL, seed=SEED, step=step, cell_volume=DV,
                              pairing=oracle.DUPLICITY, correction=False)
        dv = np.stack([vx, vy, vz]).reshape(3, n_cells, 5) - v[:, None, :]
        for c in range(n_cells):
            key = (tuple(oracle.shuffle(3, c, SEED, step, 0, 0)),
                   tuple(oracle.shuffle(2, c, SEED, step, 0, 1)))
            g = groups.setdefault(key, [np.zeros((3, 5)), np.zeros((3, 5)), 0])
            g[0] += dv[:, c]
            g[1] += dv[:, c] ** 2
            g[2] += 1
    assert len(groups) == 12   # every ordering of both lists occurs

    models = {
        "duplicity": lambda k: 3.0 / (2 if k % 2 == 0 else 1),
        "order-N (N_min)": lambda k: 2.0,
        "N_max without D": lambda k: 3.0,
        "N x N (1)": lambda k: 1.0,
    }
    dist = {}
    for name, nf in models.items():
        worst = 0.0
        for (L0, L1), (acc, acc2, cnt) in groups.items():
            mean = acc / cnt
            se = np.sqrt(np.maximum(acc2 / cnt - mean * mean, 0.0) / cnt)
            want = _predict(w, v, L0, L1, nf)
            # first order in s leaves O(s) relative terms: 3 % of the
            # group's largest term is allowed, then standard errors
            excess = (np.abs(mean - want) - 0.03 * np.abs(want).max()) / se
            worst = max(worst, float(excess.max()))
        dist[name] = worst
    print("largest excess over the allowance, in standard errors:", dist)
    assert dist["duplicity"] < 3.0
    for name in ("order-N (N_min)", "N_max without D", "N x N (1)"):
        assert dist[name] > 6.0, name
