"""Pins of the oracle's super-time-stepping tables and stage counts: the
printed App. A constants, the closed-form stability polynomials of RKL2
(Legendre) and RKG2 (Gegenbauer, alpha = 3/2), second-order consistency,
the odd-stage rule of Sec. 3.1, and the Fig. 1 set-up (1-D uniform heat
equation at 500 x the explicit Euler limit)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.special import eval_gegenbauer, eval_legendre

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def scalar_recurrence(oracle_mod, kind, s, z):
    """The App. A recurrence applied to u' = lambda u with z = lambda dt."""
    mu, nu, mut, gam = oracle_mod.sts_coeffs(kind, s)
    u0 = 1.0
    y0 = z * u0
    um2, um1 = u0, u0 + mut[1] * y0
    for k in range(2, s + 1):
        uk = mu[k] * um1 + nu[k] * um2 + (1 - mu[k] - nu[k]) * u0 + mut[k] * z * um1 + gam[k] * y0
        um2, um1 = um1, uk
    return um1


def poly(kind, s, z):
    """Closed-form stability polynomials: RKL2 a_s + b_s P_s(1 + w1 z) with
    b_s = (s^2+s-2)/(2 s (s+1)), w1 = 4/(s^2+s-2) (Meyer et al. 2014);
    RKG2 1 - b_s C_s(1) + b_s C_s^(3/2)(1 + w z), w = 6/((s+4)(s-1))."""
    if kind == "rkl2":
        b = (s * s + s - 2) / (2 * s * (s + 1))
        w1 = 4 / (s * s + s - 2)
        return 1 - b + b * eval_legendre(s, 1 + w1 * z)
    b = 4 * (s - 1) * (s + 4) / (3 * s * (s + 1) * (s + 2) * (s + 3))
    w = 6 / ((s + 4) * (s - 1))
    return 1 - b * eval_gegenbauer(s, 1.5, 1.0) + b * eval_gegenbauer(s, 1.5, 1 + w * z)


def edge(kind, s):
    return -(s * s + s - 2) / 2 if kind == "rkl2" else -(s + 4) * (s - 1) / 3


def test_appendix_a_constants(oracle_mod):
    rows = [l.split() for l in open(os.path.join(GOLD, "rkg2_appendix_a.txt"))
            if l.strip() and not l.startswith("#")]
    for s in (3, 8, 21):
        w = 6 / ((s + 4) * (s - 1))
        mu, nu, mut, gam = oracle_mod.sts_coeffs("rkg2", s)
        got = {"mu1": mu[1], "mut1": mut[1], "mu2": mu[2], "nu2": nu[2], "mut2": mut[2],
               "gamma2": gam[2]}
        # b_0..b_2 enter through mu_3, nu_3: mu_3 = (2+1/3) b_3/b_2, nu_3 = -(4/3) b_3/b_1
        b3 = 4 * 2 * 7 / (3 * 3 * 4 * 5 * 6)
        for name, num, den, tw in rows:
            val = float(Fraction(int(num), int(den))) * (w if int(tw) else 1.0)
            if name in got:
                assert abs(got[name] - val) <= 1e-15 * max(1, abs(val)), name
            elif name == "b2":
                assert abs(mu[3] - (2 + 1 / 3) * b3 / val) < 1e-14
            elif name == "b1":
                assert abs(nu[3] + (1 / 3 + 1) * b3 / val) < 1e-14


def test_stage_formula_golden(oracle_mod):
    rows = [l.split() for l in open(os.path.join(GOLD, "rkg2_stage_formula.txt"))
            if l.strip() and not l.startswith("#")]
    for ratio, s_plain, s_odd in rows:
        assert oracle_mod.sts_stages("rkg2", float(ratio), False) == int(s_plain)
        assert oracle_mod.sts_stages("rkg2", float(ratio), True) == int(s_odd)


@pytest.mark.parametrize("kind", ["rkl2", "rkg2"])
def test_recurrence_equals_stability_polynomial(oracle_mod, kind):
    for s in list(range(2, 40)) + [45, 55, 101]:
        zs = np.linspace(edge(kind, s), 0.0, 9)
        err = max(abs(scalar_recurrence(oracle_mod, kind, s, z) - poly(kind, s, z)) for z in zs)
        assert err < 1e-12, (s, err)


@pytest.mark.parametrize("kind", ["rkl2", "rkg2"])
def test_second_order(oracle_mod, kind):
    """R(z) = 1 + z + z^2/2 + O(z^3): second-order accuracy.  Taylor
    coefficients from the recurrence evaluated on a small complex circle."""
    for s in (3, 9, 16):
        N, rad = 64, 0.05
        th = 2 * math.pi * np.arange(N) / N
        vals = np.array([scalar_recurrence(oracle_mod, kind, s, rad * np.exp(1j * t)) for t in th])
        c = np.fft.fft(vals) / N / rad ** np.arange(N)
        assert abs(c[0] - 1) < 1e-14 and abs(c[1] - 1) < 1e-12 and abs(c[2] - 0.5) < 1e-10
        assert abs(c[3] - 1 / 6) > 1e-6          # not third order


@pytest.mark.parametrize("kind", ["rkl2", "rkg2"])
def test_stability_interval(oracle_mod, kind):
    """|R| <= 1 on [edge, 0]; the edge is where the stage-count formula puts
    dt = ratio * dt_E with lambda_max dt_E = 2."""
    for s in (3, 10, 15, 17, 30):
        zs = np.linspace(edge(kind, s), 0.0, 2001)
        vals = np.array([poly(kind, s, z) for z in zs])
        assert np.abs(vals).max() <= 1 + 1e-12
        # ratio at the edge is -edge/2; the formula must return exactly s there
        ratio = -edge(kind, s) / 2
        assert oracle_mod.sts_stages(kind, ratio * (1 - 1e-12), False) == s


@pytest.mark.parametrize("kind", ["rkl2", "rkg2"])
def test_odd_stage_rule(oracle_mod, kind):
    """Sec. 3.1 / App. A: with an even stage count the amplification factor at
    the highest mode tends to one; odd counts damp it."""
    for s in (4, 10, 16, 30):
        assert abs(scalar_recurrence(oracle_mod, kind, s, edge(kind, s)) - 1.0) < 1e-11
    for s in (5, 11, 17, 31):
        Re = scalar_recurrence(oracle_mod, kind, s, edge(kind, s))
        assert abs(Re) < 0.5
        if kind == "rkl2":   # a_s + b_s P_s(-1) = 1 - 2 b_s = 2/(s(s+1)) for odd s
            assert abs(Re - 2 / (s * (s + 1))) < 1e-12
    # RKG2 saturates near -1/3 at the highest mode (Fig. 1 discussion)
    if kind == "rkg2":
        assert abs(scalar_recurrence(oracle_mod, kind, 101, edge(kind, 101)) + 1 / 3) < 0.01
    # the odd rule lifts even counts by one
    for ratio in (3.0, 24.3, 50.0, 500.0):
        s0 = oracle_mod.sts_stages(kind, ratio, False)
        s1 = oracle_mod.sts_stages(kind, ratio, True)
        assert s1 == s0 + (1 - s0 % 2) and s1 % 2 == 1


def test_fig1_setup(oracle_mod):
    """Fig. 1 (middle): 1-D uniform second-order heat equation at 500 x the
    Euler limit.  Its eigenvalues times dt are z_m = -1000 sin^2(m pi/(2n))
    (lambda_max dt_E = 2, dt = 500 dt_E).  Stage counts 45 (RKL2) and 55
    (RKG2, odd rule), both stable on the whole spectrum; BE is 1/(1-z)."""
    sl = oracle_mod.sts_stages("rkl2", 500.0)
    sg = oracle_mod.sts_stages("rkg2", 500.0)
    assert (sl, sg) == (45, 55)
    n = 200
    z = -1000.0 * np.sin(np.arange(1, n + 1) * math.pi / (2 * n)) ** 2
    for kind, s in (("rkl2", sl), ("rkg2", sg)):
        R = np.array([scalar_recurrence(oracle_mod, kind, s, zz) for zz in z])
        assert np.abs(R).max() <= 1.0
        assert np.allclose(R, [poly(kind, s, zz) for zz in z], atol=1e-11)
    be = 1 / (1 - z)
    assert np.all((be > 0) & (be < 1))
