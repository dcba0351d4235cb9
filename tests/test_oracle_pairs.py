"""Pair-level pins of the oracle: conservation by one scattered pair, the
w_min/w_max acceptance frequency, the closed forms of the zero-angle
inelastic energy correction (Eqs. (19)-(23), (26)-(28)) and of its
relativistic version (Eqs. (A.2)-(A.6))."""
import math

import numpy as np
import pytest

import oracle

RNG = np.random.default_rng(20240719)


def _pair_kw(**over):
    kw = dict(mi=1.0, qi=-1.0, mj=7.3, qj=2.0, wi=1.0, wj=1.0, nmin=50.0, dt=0.5,
              lnL=10.0, method=oracle.N97, seed=77, step=3, cell=5, coll=1)
    kw.update(over)
    return kw


@pytest.mark.parametrize("method", [oracle.TA77, oracle.N97])
def test_equal_weight_pair_conserves_momentum_and_energy(method):
    kw = _pair_kw(method=method)
    for k in range(300):
        vi, vj = RNG.normal(size=3), RNG.normal(size=3) * 0.4
        ni, nj = oracle.scatter_pair(vi, vj, pair=k, **kw)
        mi, mj = kw["mi"], kw["mj"]
        dp = mi * (ni - vi) + mj * (nj - vj)
        assert np.max(np.abs(dp)) <= 1e-15 * (mi * np.abs(vi).max() + mj * np.abs(vj).max())
        e0 = mi * vi @ vi + mj * vj @ vj
        e1 = mi * ni @ ni + mj * nj @ nj
        assert e1 == pytest.approx(e0, rel=1e-14)
        # the relative speed is unchanged (elastic)
        assert np.linalg.norm(ni - nj) == pytest.approx(np.linalg.norm(vi - vj), rel=1e-14)


def test_acceptance_frequency_is_weight_ratio():
    """The lighter particle always moves; the heavier one with probability
    w_min/w_max (Sec. 3.1 rejection; Alg. 1 update steps)."""
    kw = _pair_kw(wi=1.0, wj=4.0, method=oracle.N97, dt=5.0)
    trials = 20000
    moved_i = moved_j = 0
    for k in range(trials):
        vi, vj = np.array([1.0, 0.2, -0.3]), np.array([-0.5, 0.1, 0.4])
        ni, nj = oracle.scatter_pair(vi, vj, pair=k, **kw)
        moved_i += not np.array_equal(ni, vi)
        moved_j += not np.array_equal(nj, vj)
    assert moved_i == trials
    p = 0.25
    z = (moved_j - p * trials) / math.sqrt(trials * p * (1 - p))
    assert abs(z) < 5.0
    # swapped roles
    kw = _pair_kw(wi=8.0, wj=2.0, method=oracle.TA77, dt=5.0)
    moved_i = moved_j = 0
    for k in range(trials):
        vi, vj = np.array([1.0, 0.2, -0.3]), np.array([-0.5, 0.1, 0.4])
        ni, nj = oracle.scatter_pair(vi, vj, pair=k, **kw)
        moved_i += not np.array_equal(ni, vi)
        moved_j += not np.array_equal(nj, vj)
    assert moved_j == trials
    z = (moved_i - p * trials) / math.sqrt(trials * p * (1 - p))
    assert abs(z) < 5.0


def test_coincident_velocities_are_skipped():
    kw = _pair_kw()
    v = np.array([0.3, 0.3, 0.3])
    ni, nj = oracle.scatter_pair(v, v, **kw)
    assert np.array_equal(ni, v) and np.array_equal(nj, v)


def test_energy_pair_equal_mass_closed_form():
    """m1 = m2, U = -f_E K: v'_R = v_R sqrt(1 + f_E) (Eq. (22)) so
    v1' = v1 + (sqrt(1+f_E) - 1)/2 (v1 - v2) exactly, which is the
    f_E/4 rule of Eqs. (27)-(28) to first order."""
    for fE in (0.02, 0.05, 0.3):
        v1, v2 = RNG.normal(size=3), RNG.normal(size=3)
        m = 2.7
        K = 0.5 * (m / 2) * np.sum((v1 - v2) ** 2)
        n1, n2 = oracle.energy_pair_nr(m, m, -fE * K, v1, v2)
        k = 0.5 * (math.sqrt(1 + fE) - 1)
        assert np.allclose(n1, v1 + k * (v1 - v2), rtol=0, atol=1e-15 * np.abs(v1 - v2).max() + 1e-16)
        assert np.allclose(n2, v2 - k * (v1 - v2), rtol=0, atol=1e-15 * np.abs(v1 - v2).max() + 1e-16)
        assert np.allclose(n1 - v1, fE / 4 * (v1 - v2), rtol=0, atol=fE ** 2 * np.abs(v1 - v2).max())


def test_energy_pair_general_masses_conserves_momentum_moves_energy_by_U():
    for _ in range(200):
        m1, m2 = 10 ** RNG.uniform(-2, 2, size=2)
        v1, v2 = RNG.normal(size=3), RNG.normal(size=3)
        mu = m1 * m2 / (m1 + m2)
        K = 0.5 * mu * np.sum((v1 - v2) ** 2)
        U = RNG.uniform(-0.05, 0.05) * K
        n1, n2 = oracle.energy_pair_nr(m1, m2, U, v1, v2)
        p0, p1 = m1 * v1 + m2 * v2, m1 * n1 + m2 * n2
        assert np.allclose(p0, p1, rtol=0, atol=1e-15 * (np.abs(m1 * v1).max() + np.abs(m2 * v2).max()))
        # Eq. (21): relative kinetic energy drops by U; total changes by -U
        K1 = 0.5 * mu * np.sum((n1 - n2) ** 2)
        assert K1 == pytest.approx(K - U, rel=1e-13)
        dE = 0.5 * m1 * ((n1 - v1) @ (n1 + v1)) + 0.5 * m2 * ((n2 - v2) @ (n2 + v2))
        scale = m1 * (v1 @ v1) + m2 * (v2 @ v2)
        assert dE == pytest.approx(-U, rel=1e-11, abs=1e-14 * scale)
        # zero-angle: the relative velocity keeps its direction
        c = (n1 - n2) @ (v1 - v2) / (np.linalg.norm(n1 - n2) * np.linalg.norm(v1 - v2))
        assert c == pytest.approx(1.0, abs=1e-14)


def _rel_energy(m, u, c):
    return m * c * c * math.sqrt(1 + u @ u / (c * c))


@pytest.mark.parametrize("c", [1.0, 3.0, 30.0])
def test_relativistic_energy_pair_conserves_momentum_and_removes_U(c):
    for _ in range(200):
        m1, m2 = 10 ** RNG.uniform(-1, 1, size=2)
        u1, u2 = RNG.normal(size=3) * 2.0, RNG.normal(size=3) * 2.0
        K = oracle.rel_kecm(m1, m2, u1, u2, c)
        U = RNG.uniform(-0.05, 0.05) * K
        ok, n1, n2 = oracle.energy_pair_rel(m1, m2, U, c, u1, u2)
        if not ok:
            continue
        p0, p1 = m1 * u1 + m2 * u2, m1 * n1 + m2 * n2
        assert np.allclose(p0, p1, rtol=0, atol=2e-15 * (m1 * np.abs(u1).max() + m2 * np.abs(u2).max()))
        # (A.2)/(A.5): total energy drops by U; compare in difference form
        dE = 0.0
        for m, a, b in ((m1, n1, u1), (m2, n2, u2)):
            ga = math.sqrt(1 + a @ a / c ** 2)
            gb = math.sqrt(1 + b @ b / c ** 2)
            dE += m * ((a - b) @ (a + b)) / (ga + gb)
        assert dE == pytest.approx(-U, rel=1e-9, abs=1e-14 * K)
        # zero-angle: p1' - p1 is along u1 - u2
        d = m1 * (n1 - u1)
        du = u1 - u2
        rnd = 4e-16 * m1 * np.linalg.norm(u1) * np.linalg.norm(du)  # rounding of n1 - u1
        assert np.linalg.norm(np.cross(d, du)) <= 1e-12 * np.linalg.norm(d) * np.linalg.norm(du) + rnd


def test_relativistic_pair_satisfies_paper_quadratic():
    """The alpha found must be a root of the quadratic Eq. (A.6), and the one
    with the smaller magnitude (continuous with the non-relativistic root)."""
    c = 1.0
    for _ in range(100):
        m1, m2 = 10 ** RNG.uniform(-0.5, 0.5, size=2)
        u1, u2 = RNG.normal(size=3) * 1.5, RNG.normal(size=3) * 1.5  # gamma ~ up to 3-4
        K = oracle.rel_kecm(m1, m2, u1, u2, c)
        U = 0.05 * K * RNG.choice([-1.0, 1.0])
        ok, n1, n2 = oracle.energy_pair_rel(m1, m2, U, c, u1, u2)
        assert ok
        du = u1 - u2
        alpha = m1 * (n1 - u1) @ du / (du @ du)
        p1, p2 = m1 * u1, m2 * u2
        E1, E2 = _rel_energy(m1, u1, c), _rel_energy(m2, u2, c)
        A = (E1 + E2 - U) / c ** 2
        D = A * A + (E2 ** 2 - E1 ** 2) / c ** 4
        pt = p1 + p2
        a2 = 4 / c ** 4 * (A * A * (du @ du) * c * c - (pt @ du) ** 2)
        a1 = 4 / c ** 2 * (du @ (D * pt - 2 * A * A * p2))
        a0 = 4 / c ** 4 * A * A * E2 ** 2 - D * D
        scale = abs(a2 * alpha * alpha) + abs(a1 * alpha) + abs(4 / c ** 4 * A * A * E2 ** 2) + D * D
        assert abs(a2 * alpha ** 2 + a1 * alpha + a0) <= 1e-9 * scale
        roots = np.roots([a2, a1, a0])
        other = roots[np.argmax(np.abs(roots - alpha))]
        assert abs(alpha) < abs(other)


def test_relativistic_pair_nonrelativistic_limit():
    c = 1e5
    for _ in range(50):
        m1, m2 = 10 ** RNG.uniform(-1, 1, size=2)
        u1, u2 = RNG.normal(size=3), RNG.normal(size=3)
        mu = m1 * m2 / (m1 + m2)
        K = 0.5 * mu * np.sum((u1 - u2) ** 2)
        U = 0.04 * K
        ok, r1, r2 = oracle.energy_pair_rel(m1, m2, U, c, u1, u2)
        n1, n2 = oracle.energy_pair_nr(m1, m2, U, u1, u2)
        assert ok
        assert np.allclose(r1, n1, rtol=0, atol=1e-8 * np.abs(u1 - u2).max())
        assert np.allclose(r2, n2, rtol=0, atol=1e-8 * np.abs(u1 - u2).max())


@pytest.mark.parametrize("c", [1.0, 4.0])
def test_relativistic_scatter_conserves_four_momentum(c):
    kw = _pair_kw(method=oracle.N97, relativistic=True, c=c, dt=0.05)
    for k in range(200):
        ui, uj = RNG.normal(size=3) * 1.2, RNG.normal(size=3) * 0.3
        ni, nj = oracle.scatter_pair(ui, uj, pair=k, **kw)
        mi, mj = kw["mi"], kw["mj"]
        dp = mi * (ni - ui) + mj * (nj - uj)
        assert np.max(np.abs(dp)) <= 4e-15 * (mi * np.abs(ui).max() + mj * np.abs(uj).max())
        dE = 0.0
        for m, a, b in ((mi, ni, ui), (mj, nj, uj)):
            ga = math.sqrt(1 + a @ a / c ** 2)
            gb = math.sqrt(1 + b @ b / c ** 2)
            dE += m * ((a - b) @ (a + b)) / (ga + gb)
        etot = _rel_energy(mi, ui, c) + _rel_energy(mj, uj, c) - (mi + mj) * c * c
        assert abs(dE) <= 1e-13 * etot


def test_relativistic_scatter_nonrelativistic_limit():
    kw_nr = _pair_kw(method=oracle.TA77, dt=0.05)
    kw_r = dict(kw_nr, relativistic=True, c=1e6)
    for k in range(100):
        vi, vj = RNG.normal(size=3), RNG.normal(size=3) * 0.4
        a = oracle.scatter_pair(vi, vj, pair=k, **kw_nr)
        b = oracle.scatter_pair(vi, vj, pair=k, **kw_r)
        for x, y in zip(a, b):
            assert np.allclose(x, y, rtol=0, atol=1e-9)


def test_relativistic_scatter_off_fixed_heavy_target_matches_textbook_deflection():
    """A light charge with momentum p and speed v crossing a fixed heavy
    charge is deflected by dp_perp / p = 2 q_i q_j / (4 pi eps0 b v p)
    (straight-line relativistic Coulomb impulse), so
    s = <Theta^2>/2 = n dt q_i^2 q_j^2 lnL / (4 pi eps0^2 p^2 v).
    With N97 the mean change along u_i is then exactly -u_i (1 - e^{-s})."""
    c, lnL, dt, n = 1.0, 10.0, 0.02, 50.0
    mi, qi, mj, qj = 1.0, -1.0, 1e9, 3.0
    ui = np.array([1.2, -0.9, 1.1])  # gamma ~ 2
    g = math.sqrt(1 + ui @ ui / c ** 2)
    p = mi * np.linalg.norm(ui)
    v = np.linalg.norm(ui) / g
    s = n * dt * qi ** 2 * qj ** 2 * lnL / (4 * math.pi * p ** 2 * v)
    uhat = ui / np.linalg.norm(ui)
    par, perp = [], []
    for k in range(20000):
        ni, _ = oracle.scatter_pair(ui, np.zeros(3), mi=mi, qi=qi, mj=mj, qj=qj, wi=1.0,
                                    wj=1.0, nmin=n, dt=dt, lnL=lnL, method=oracle.N97,
                                    relativistic=True, c=c, pair=k, seed=5)
        d = (ni - ui) / np.linalg.norm(ui)
        par.append(d @ uhat)
        perp.append(d - (d @ uhat) * uhat)
    par = np.array(par)
    want = -(-math.expm1(-s))
    assert abs(par.mean() - want) < 5 * par.std() / math.sqrt(par.size)
    assert abs(par.mean() / want - 1) < 0.05
    pm = np.mean(perp, axis=0)
    assert np.linalg.norm(pm) < 5 * np.sqrt(np.var(perp, axis=0).sum() / len(perp))
