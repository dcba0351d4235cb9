"""Pins of the oracle's angle sampling and rotation against closed forms.

N97: <cos chi> = coth A - 1/A must equal exp(-s); the sampler must follow the
exp(A cos chi) law (checked through its survival function written
independently) and the Langevin function is checked against a 60-digit
decimal evaluation (120 digits).  TA77: tan(Theta/2) must be Normal(0, s/2) (KS test
against scipy's normal law) so that <Theta^2> = 2 s (Eq. (6), s = <Theta^2>/2
of Eq. (9)).  The rotation must keep |u| and turn u by Theta."""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy import stats

import oracle

getcontext().prec = 120


def _langevin_decimal(A: float) -> Decimal:
    a = Decimal(A)
    if A < 1e-6:  # Taylor series of coth a - 1/a; next term is -a^7/4725
        return a / 3 - a ** 3 / 45 + 2 * a ** 5 / 945
    em = (-2 * a).exp()  # coth a = (1 + e^{-2a}) / (1 - e^{-2a})
    return (1 + em) / (1 - em) - 1 / a


@pytest.mark.parametrize("A", [1e-8, 1e-4, 0.01, 0.1, 0.3, 0.49, 0.5, 0.51, 1.0,
                               2.0, 5.0, 20.0, 37.0, 100.0, 1e4])
def test_langevin_function_against_decimal(A):
    ref = _langevin_decimal(A)
    L = oracle.n97_L(A)
    assert abs(Decimal(L) - ref) <= Decimal(4e-16) * abs(ref)
    M = oracle.n97_M(A)
    refM = 1 - ref
    assert abs(Decimal(M) - refM) <= Decimal(4e-16) * abs(refM)


@pytest.mark.parametrize("s", [1e-10, 1e-6, 1e-3, 0.05, 0.3, 0.6931, 0.7, 1.0, 2.5,
                               5.0, 12.0, 40.0, 49.9])
def test_n97_A_solves_mean_cosine(s):
    """<cos chi> = coth A - 1/A = exp(-s) (Nanbu's defining relation)."""
    A = oracle.n97_A(s)
    assert A > 0.0
    ref = _langevin_decimal(A)
    if s <= math.log(2.0):
        # compare 1 - <cos chi> with 1 - exp(-s), where the information is
        target = Decimal(-math.expm1(-s))
        got = 1 - ref
    else:
        target = Decimal(math.exp(-s))
        got = ref
    assert abs(got - target) <= Decimal(8e-16) * target


def test_n97_A_asymptotics():
    for s in (1e-9, 1e-6, 1e-4):
        assert oracle.n97_A(s) == pytest.approx(1.0 / s, rel=2 * s)
    for s in (20.0, 30.0, 45.0):
        assert oracle.n97_A(s) == pytest.approx(3.0 * math.exp(-s), rel=1e-9)
    # s > 50: A < 6e-22, the isotropic limit to far below an ulp
    for s in (50.5, 60.0, 720.0, 745.0, 1000.0):
        assert oracle.n97_A(s) == 0.0
    assert math.isinf(oracle.n97_A(0.0))


@pytest.mark.parametrize("s", [1e-4, 0.02, 0.3, 1.0, 4.0, 30.0])
def test_n97_sampler_follows_exp_A_cos_law(s):
    """The sampled cos chi = x must satisfy P(cos chi > x) = u0 for the
    density proportional to exp(A x) on [-1, 1]."""
    A = oracle.n97_A(s)
    rng = np.random.default_rng(3)
    for u0 in rng.uniform(0.0, 1.0, 200):
        oc, st = oracle.sample_angle(oracle.N97, s, float(u0), 0.5)
        assert 0.0 <= oc <= 2.0
        assert st == pytest.approx(math.sqrt(oc * (2.0 - oc)), rel=1e-14, abs=1e-300)
        # survival function: (1 - exp(-A oc)) / (1 - exp(-2A))
        surv = math.expm1(-A * oc) / math.expm1(-2.0 * A) if A > 0 else oc / 2.0
        assert surv == pytest.approx(u0, rel=1e-11, abs=1e-14)


@pytest.mark.parametrize("s", [0.01, 0.2, 1.5])
def test_n97_mean_and_second_moment_monte_carlo(s):
    rng = np.random.default_rng(11)
    u = rng.uniform(0.0, 1.0, 100000)
    x = np.array([1.0 - oracle.sample_angle(oracle.N97, s, float(a), 0.5)[0] for a in u])
    A = oracle.n97_A(s)
    m1, m2 = math.exp(-s), 1.0 - 2.0 * math.exp(-s) / A
    se1 = x.std() / math.sqrt(x.size)
    se2 = (x * x).std() / math.sqrt(x.size)
    assert abs(x.mean() - m1) < 5 * se1 + 1e-12
    assert abs((x * x).mean() - m2) < 5 * se2 + 1e-12


@pytest.mark.parametrize("s", [1e-3, 0.05, 0.5])
def test_ta77_tan_half_angle_is_gaussian_with_variance_s_over_2(s):
    rng = np.random.default_rng(5)
    u0 = rng.uniform(0.0, 1.0, 40000)
    u1 = rng.uniform(0.0, 1.0, 40000)
    d = np.empty(u0.size)
    oc_all = np.empty(u0.size)
    for k in range(u0.size):
        oc, st = oracle.sample_angle(oracle.TA77, s, float(u0[k]), float(u1[k]))
        d[k] = st / (2.0 - oc)  # tan(Theta/2) = sin(Theta)/(1 + cos(Theta))
        oc_all[k] = oc
    z = d / math.sqrt(0.5 * s)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # <1 - cos Theta> against a direct quadrature over the Gaussian law
    from scipy import integrate
    sig = math.sqrt(0.5 * s)
    ref = integrate.quad(lambda t: 2 * t * t / (1 + t * t) * stats.norm.pdf(t, scale=sig),
                         -40 * sig, 40 * sig, limit=400)[0]
    se = oc_all.std() / math.sqrt(oc_all.size)
    assert abs(oc_all.mean() - ref) < 5 * se


def test_ta77_huge_s_is_backscatter():
    oc, st = oracle.sample_angle(oracle.TA77, math.inf, 0.3, 0.1)
    assert oc == 2.0 and st == 0.0
    oc, st = oracle.sample_angle(oracle.TA77, 1e300, 0.3, 0.1)
    assert oc == pytest.approx(2.0, rel=1e-15) and abs(st) < 1e-140


def test_rotation_invariants():
    rng = np.random.default_rng(2)
    for _ in range(500):
        u = rng.normal(size=3) * 10 ** rng.uniform(-3, 3)
        th = rng.uniform(0, math.pi)
        phi = rng.uniform(0, 2 * math.pi)
        st, oc = math.sin(th), 1.0 - math.cos(th)
        du = oracle.rotate(u, st, oc, phi)
        un = u + du
        uu = float(u @ u)
        assert float(un @ un) == pytest.approx(uu, rel=4e-15)
        assert float(un @ u) == pytest.approx(uu * math.cos(th), abs=8e-15 * uu)


def test_rotation_azimuthal_average_is_parallel_drag():
    """Averaged over a uniform azimuth only the component along u survives:
    <du> = -u (1 - cos Theta) (the step behind the drag of Eqs. (7)-(8))."""
    u = np.array([0.3, -1.2, 0.7])
    st, oc = math.sin(0.4), 1.0 - math.cos(0.4)
    phis = (np.arange(64) + 0.5) * 2 * math.pi / 64
    mean = np.mean([oracle.rotate(u, st, oc, p) for p in phis], axis=0)
    assert np.allclose(mean, -u * oc, rtol=0, atol=1e-15)


def test_rotation_along_z_axis():
    for uz in (2.5, -2.5):
        u = np.array([0.0, 0.0, uz])
        th, phi = 0.7, 1.1
        du = oracle.rotate(u, math.sin(th), 1 - math.cos(th), phi)
        un = u + du
        assert float(un @ un) == pytest.approx(uz * uz, rel=1e-15)
        assert float(un @ u) == pytest.approx(uz * uz * math.cos(th), rel=1e-14)


@pytest.mark.parametrize("s", [40.0, 49.9, 50.1, 300.0, 716.0, 744.6])
def test_n97_large_s_is_isotropic_to_rounding(s):
    """For large s the sampled 1 - cos chi equals 2 u to rounding (no
    subnormal arithmetic on the way)."""
    for u0 in (0.0427, 0.2427, 0.5369, 0.999):
        oc, st = oracle.sample_angle(oracle.N97, s, u0, 0.5)
        assert oc == pytest.approx(2.0 * u0, rel=1e-15)
