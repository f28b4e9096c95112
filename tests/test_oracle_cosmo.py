"""Pins of the oracle's cosmology, growth and BullFrog coefficients against
closed forms and the paper's printed series (CPU only)."""
import math

import numpy as np
import pytest

from oracle import cosmo


@pytest.fixture(scope="module")
def growth():
    return cosmo.Growth(0.31)


@pytest.mark.parametrize("a", [0.02, 0.1, 0.3, 0.6, 1.0])
def test_growth_matches_closed_form_integral(growth, a):
    # flat-LCDM growing mode D = 5/2 Om H int da/(aH)^3 (D ~ a early): pins the
    # (2 - 3 gamma) friction reading of eq. growth_odes
    assert abs(float(growth.D(a)) / cosmo.growth_closed_form(a, 0.31) - 1) < 1e-10


@pytest.mark.parametrize("a", [0.02, 0.05, 0.1])
def test_second_order_growth_matches_paper_series(growth, a):
    # Sec. "Time stepping": E = -(3/7) D^2 - (3/1001) Lambda D^5 + O(Lambda^2 D^8)
    lam = (1 - 0.31) / 0.31
    D = float(growth.D(a))
    series = -3 / 7 * D ** 2 - 3 / 1001 * lam * D ** 5
    assert abs(float(growth.E(a)) / series - 1) < 1e-7


def test_second_order_growth_within_one_percent_today(growth):
    # App. growth: the D^n approximation of E errs by < 1% at z = 0
    D1 = float(growth.D(1.0))
    dev = abs(float(growth.E(1.0)) / (-3 / 7 * D1 ** 2) - 1)
    assert 0.001 < dev < 0.01


def test_eds_growth_is_exact():
    g = cosmo.Growth(1.0)
    for a in (0.02, 0.3, 1.0):
        assert abs(float(g.D(a)) / a - 1) < 1e-11
        assert abs(float(g.E(a)) / (-3 / 7 * a * a) - 1) < 1e-10
        assert abs(g.dEdD(float(g.D(a))) / (-6 / 7 * a) - 1) < 1e-10


def _bullfrog_toy_run(steps, D0):
    """2LPT test trajectory in EdS with the linear toy force along
    (psi1, psi2) = (e1, e2): X = D e1 + c e2 feels A = X / D^2 - e2, which has
    X = D e1 + E(D) e2, E = -(3/7) D^2, as an exact solution of the D-time
    equation of motion dV/dD = (3/2)(A - V/D)."""
    X = np.array([D0, -3 / 7 * D0 ** 2])
    V = np.array([1.0, -6 / 7 * D0])
    for st in steps:
        X = X + st.tau1 * V
        A = X * st.s - np.array([0.0, 1.0])
        V = st.alpha * V + st.beta * A
        X = X + st.tau2 * V
    return X, V


def _leapfrog_toy_run(steps, a0):
    """The same toy in canonical variables (EdS, H0 = 1): p = a^2 dX/dt =
    a^(3/2) dX/dD, dp/dt = (3/2) F / a with the toy field F = X - a^2 e2
    (D^2 A of the D-time toy), whose exact solution is again
    X = a e1 - (3/7) a^2 e2.  Kick p += beta s F(X^{n+1/2}, a_{n+1/2})."""
    X = np.array([a0, -3 / 7 * a0 ** 2])
    p = a0 ** 1.5 * np.array([1.0, -6 / 7 * a0])
    for st in steps:
        X = X + st.tau1 * p
        F = X - st.D_half ** 2 * np.array([0.0, 1.0])
        p = st.alpha * p + st.beta * st.s * F
        X = X + st.tau2 * p
    return X, p


@pytest.mark.parametrize("a0,a1,n", [(0.02, 1.0, 6), (0.5, 1.0, 1), (0.1, 0.11, 1), (0.02, 1.0, 1),
                                     (0.05, 0.8, 13)])
def test_bullfrog_is_2lpt_exact_in_eds(a0, a1, n):
    # BullFrog aligns the trajectory with 2LPT after every step; in EdS the
    # 2LPT trajectory is exact for the toy force, so any step size reproduces it
    steps = cosmo.bullfrog_steps(1.0, a0, a1, n)
    X, V = _bullfrog_toy_run(steps, a0)
    assert np.allclose(X, [a1, -3 / 7 * a1 ** 2], rtol=1e-12, atol=1e-15)
    assert np.allclose(V, [1.0, -6 / 7 * a1], rtol=1e-12, atol=1e-15)


def test_bullfrog_zeldovich_consistency_and_schedule():
    steps = cosmo.bullfrog_steps(0.31, 0.02, 1.0, 10)
    D0 = cosmo.D_of_a(0.31, 0.02)
    D1 = cosmo.D_of_a(0.31, 1.0)
    assert abs(steps[0].D_n - D0) < 1e-15 and abs(steps[-1].D_np1 - D1) < 1e-12
    for st in steps:
        # a linear-theory state V = psi, A = psi / D_half stays V = psi
        assert abs(st.alpha + st.beta / st.D_half - 1) < 1e-13
        assert abs(st.tau1 - st.tau2) < 1e-13
        assert abs(st.s * st.D_half ** 2 - 1) < 1e-14


def test_bbks_limits_and_sigma8_normalisation():
    # parity unpinned against the paper (BBKS is not used there): pinned only
    # by the published formula's limits and an independent quadrature
    assert abs(float(cosmo.bbks_transfer(1e-7, 0.31, 0.68)) - 1) < 1e-5
    assert float(cosmo.bbks_transfer(10.0, 0.31, 0.68)) < 1e-3
    sp = cosmo.bbks_spectrum(0.31, 0.68, 0.965, 0.81)
    from scipy import integrate
    f = lambda lnk: math.exp(lnk) ** 3 * float(sp(math.exp(lnk))) * float(
        cosmo.tophat_window(8 * math.exp(lnk))) ** 2
    v = sum(integrate.quad(f, lo, lo + 0.5, limit=200)[0]
            for lo in np.arange(math.log(1e-6), math.log(1e3), 0.5))
    assert abs(math.sqrt(v / (2 * math.pi ** 2)) / 0.81 - 1) < 1e-6


def _zeta_closed(a, om):
    """H a^3 dD/da from the closed-form growth integral
    D = (5/2) Om H(a) I(a), I = int_0^a dx / (x H)^3 (independent of the ODE)."""
    H = float(cosmo.hubble(a, om))
    I = cosmo.growth_closed_form(a, om) / (2.5 * om * H)
    dH = -1.5 * om * a ** -4 / H
    dD = 2.5 * om * (dH * I + H / (a * H) ** 3)
    return H * a ** 3 * dD


def test_fastpm_alpha_closed_forms():
    # EdS: zeta = a^(3/2) (H = a^-3/2, D = a)
    for st in cosmo.step_table(1.0, 0.02, 1.0, 7, "fastpm", "D"):
        assert abs(st.alpha - (st.D_n / st.D_np1) ** 1.5) < 1e-14
        assert abs(st.alpha + st.beta / st.D_half - 1) < 1e-13
    # LCDM, steps uniform in a (the nodes are known scale factors)
    a0, a1, n, om = 0.02, 1.0, 5, 0.31
    steps = cosmo.step_table(om, a0, a1, n, "fastpm", "a")
    for i, st in enumerate(steps):
        an, ap = a0 + i * (a1 - a0) / n, a0 + (i + 1) * (a1 - a0) / n
        assert abs(st.alpha / (_zeta_closed(an, om) / _zeta_closed(ap, om)) - 1) < 1e-8


@pytest.mark.parametrize("tv", ["a", "lna"])
def test_time_variable_nodes_and_midpoints(tv):
    om, a0, a1, n = 0.31, 0.02, 1.0, 6
    steps = cosmo.step_table(om, a0, a1, n, "bullfrog", tv)
    if tv == "a":
        t = lambda x: a0 + x * (a1 - a0) / n
    else:
        t = lambda x: a0 * (a1 / a0) ** (x / n)
    for i, st in enumerate(steps):
        for D, x in ((st.D_n, i), (st.D_half, i + 0.5), (st.D_np1, i + 1)):
            assert abs(D / cosmo.growth_closed_form(t(x), om) - 1) < 1e-9
        assert abs(st.tau1 - (st.D_half - st.D_n)) < 1e-15 and abs(st.tau2 - (st.D_np1 - st.D_half)) < 1e-15
    # in EdS steps uniform in a are steps uniform in D: BullFrog stays 2LPT exact
    X, V = _bullfrog_toy_run(cosmo.step_table(1.0, 0.05, 0.8, 5, "bullfrog", "a"), 0.05)
    assert np.allclose(X, [0.8, -3 / 7 * 0.8 ** 2], rtol=1e-12)


def test_fastpm_is_first_order_consistent_only():
    # the toy 2LPT trajectory: FastPM keeps the Zel'dovich component exactly
    # but misses the second-order one, by less as the steps shrink (BullFrog
    # hits it exactly for any step)
    errs = []
    for n in (4, 8, 16):
        X, V = _bullfrog_toy_run(cosmo.step_table(1.0, 0.02, 1.0, n, "fastpm", "D"), 0.02)
        assert abs(X[0] - 1.0) < 1e-13 and abs(V[0] - 1.0) < 1e-13
        errs.append(abs(X[1] + 3 / 7))
    assert errs[0] > 1e-2 and errs[0] / errs[1] > 2.0 and errs[1] / errs[2] > 2.0


def test_leapfrog_coefficients_closed_forms():
    # canonical momentum in EdS (H = a^-3/2): the drift integrals
    # int da / (a^3 H) = 2 (a^-1/2 - b^-1/2), the kick int da / (a^2 H)
    # = 2 (b^1/2 - a^1/2), alpha = 1, s = 3/2 Omega_m
    for tv in ("a", "superconft"):
        for st in cosmo.step_table(1.0, 0.02, 1.0, 6, "leapfrog", tv):
            a, h, b = st.D_n, st.D_half, st.D_np1  # D = a in EdS
            assert st.alpha == 1.0 and st.s == 1.5
            assert abs(st.tau1 / (2 * (a ** -0.5 - h ** -0.5)) - 1) < 1e-11
            assert abs(st.tau2 / (2 * (h ** -0.5 - b ** -0.5)) - 1) < 1e-11
            assert abs(st.beta / (2 * (b ** 0.5 - a ** 0.5)) - 1) < 1e-11
    # LCDM: the drift over the whole run is the superconformal interval, and a
    # superconformal spacing gives equal drifts
    om = 0.31
    steps = cosmo.step_table(om, 0.02, 1.0, 5, "leapfrog", "superconft")
    tau = [st.tau1 + st.tau2 for st in steps]
    assert abs(sum(tau) / cosmo.superconformal(om, 0.02, 1.0) - 1) < 1e-9
    assert max(tau) / min(tau) - 1 < 1e-8 and all(abs(st.tau1 / st.tau2 - 1) < 1e-8 for st in steps)


def test_superconformal_nodes_closed_form():
    # EdS: t(a) = 2 (a0^-1/2 - a^-1/2), so the nodes are a = (a0^-1/2 - t/2)^-2
    a0, a1, n = 0.02, 1.0, 6
    T = 2 * (a0 ** -0.5 - a1 ** -0.5)
    a_of = lambda x: (a0 ** -0.5 - x * T / n / 2) ** -2
    for i, st in enumerate(cosmo.step_table(1.0, a0, a1, n, "bullfrog", "superconft")):
        for D, x in ((st.D_n, i), (st.D_half, i + 0.5), (st.D_np1, i + 1)):
            assert abs(D / a_of(x) - 1) < 1e-10


def test_leapfrog_converges_at_second_order():
    # the toy 2LPT trajectory of EdS with the canonical momentum
    # p = a^2 dX/dt = zeta V_D (zeta = a^3/2): the leapfrog is neither
    # Zel'dovich nor 2LPT consistent, and with steps uniform in ln a its
    # error falls as the step squared (uniform steps in a from a = 0.02 are
    # far from that regime: the first step is six times a_start)
    errs = []
    for n in (8, 16, 32):
        X, V = _leapfrog_toy_run(cosmo.step_table(1.0, 0.02, 1.0, n, "leapfrog", "lna"), 0.02)
        errs.append(abs(X[0] - 1.0) + abs(X[1] + 3 / 7))
    assert errs[0] < 0.05 and 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5
