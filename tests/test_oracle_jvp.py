"""Pins of the forward-mode oracle (oracle/jvp.py): the force JVP and the
run's tangent against central differences of the oracle's own forward, the
force JVP against the independently pinned VJP by duality, the P(k) tangent
against differences of the estimator, and the large-scale limit of
d log P / d log sigma8 (Sec. "Correctness of the adjoint method and custom
derivatives": 2 on linear scales, since the linear spectrum scales as
sigma8^2)."""
import numpy as np
import pytest

from oracle import adjoint, force, jvp, nbody
from oracle.force import PMConfig


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


@pytest.mark.parametrize("order,dec,g,inter", [(2, False, 4, False), (3, True, 2, False), (4, True, 6, False),
                                               (2, True, 4, True), (3, False, 4, True)])
def test_force_jvp_matches_differences_and_vjp(order, dec, g, inter):
    cfg = PMConfig(8, 16, 40.0, order=order, deconvolve=dec, grad_order=g, interlace=inter)
    rng = np.random.default_rng(20 + order)
    psi = rng.normal(0, 1.0, (3, cfg.N))
    xd = rng.normal(size=(3, cfg.N))
    u = rng.normal(size=(3, cfg.N))
    J = jvp.force_jvp(cfg, psi, 2.0, xd)
    eps = 1e-6
    fd = (force.pm_force(cfg, psi + eps * xd, 2.0) - force.pm_force(cfg, psi - eps * xd, 2.0)) / (2 * eps)
    assert rel(J, fd) < 1e-7
    lhs = np.sum(u * J)
    rhs = np.sum(adjoint.force_vjp(cfg, psi, 2.0, u) * xd)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _problem(n_p=8, box=40.0, spectrum="bbks", stepper="bullfrog", time_var="D"):
    cfg = PMConfig(n_p, 2 * n_p, box, order=2, deconvolve=False, grad_order=4)
    return nbody.Problem(cfg, omega_m=0.31, a_start=0.02, a_end=1.0, n_steps=3, sigma8=0.9, spectrum=spectrum,
                         stepper=stepper, time_var=time_var)


@pytest.mark.parametrize("stepper,tv", [("bullfrog", "D"), ("leapfrog", "superconft")])
def test_run_tangent_matches_differences(stepper, tv):
    prob = _problem(stepper=stepper, time_var=tv)
    n = prob.pm.n_p
    rng = np.random.default_rng(1)
    w = nbody.white_noise(prob, 3).astype(np.float64)
    wd = rng.normal(size=n ** 3)
    _, _, delta, dd = jvp.run_jvp(prob, w, wd, 0.3)

    def dens(wv, s8):
        p = nbody.Problem(prob.pm, omega_m=0.31, a_start=0.02, a_end=1.0, n_steps=3, sigma8=s8,
                          stepper=stepper, time_var=tv)
        x, _ = nbody.run(p, w=wv.reshape(n, n, n))
        return adjoint.final_density(p, x)

    eps = 1e-6
    fd = (dens(w.reshape(-1) + eps * wd, 0.9 + 0.3 * eps) - dens(w.reshape(-1) - eps * wd, 0.9 - 0.3 * eps)) / (2 * eps)
    assert rel(dd, fd) < 1e-7
    assert np.array_equal(delta, dens(w.reshape(-1), 0.9))


def test_powerlaw_tangent_ignores_sigma8():
    prob = _problem(spectrum="powerlaw")
    w = nbody.white_noise(prob, 4).astype(np.float64)
    _, _, _, dd = jvp.run_jvp(prob, w, np.zeros(prob.pm.N), 1.0)
    assert not np.any(dd)


def test_pk_tangent_matches_differences():
    rng = np.random.default_rng(2)
    n = 16
    d = rng.normal(size=n ** 3)
    dd = rng.normal(size=n ** 3)
    for dec in (False, True):
        k, p, pdot, cnt = jvp.power_spectrum_jvp(d, dd, 100.0, 8, dec)
        eps = 1e-6
        from oracle.pk import power_spectrum
        fd = (power_spectrum(d + eps * dd, 100.0, 8, dec)[1] - power_spectrum(d - eps * dd, 100.0, 8, dec)[1]) / (2 * eps)
        assert rel(pdot, fd) < 1e-8


def test_sigma8_log_derivative_is_two_on_linear_scales():
    # 16^3 particles in a 1000 Mpc/h box: the lowest bins are linear at z = 0
    cfg = PMConfig(16, 32, 1000.0, order=2, deconvolve=False, grad_order=4)
    prob = nbody.Problem(cfg, omega_m=0.31, a_start=0.02, a_end=1.0, n_steps=4, sigma8=0.81)
    w = nbody.white_noise(prob, 5).astype(np.float64)
    _, _, d, dd = jvp.run_jvp(prob, w, np.zeros(cfg.N), prob.sigma8)
    k, p, pdot, _ = jvp.power_spectrum_jvp(d, dd, cfg.box, 16)
    logd = pdot / p
    assert abs(logd[0] - 2.0) < 0.03
    assert np.all(np.abs(logd[:3] - 2.0) < 0.1)


def test_nufft_force_jvp_matches_differences_and_vjp():
    from oracle import nufft
    rng = np.random.default_rng(40)
    n_p, n_f = 8, 16
    psi = rng.normal(0, 0.8, (3, n_p ** 3))
    xd = rng.normal(size=(3, n_p ** 3))
    u = rng.normal(size=(3, n_p ** 3))
    J = nufft.nufft_force_jvp(n_p, n_f, psi, 1.3, xd)
    eps = 1e-6
    fd = (nufft.nufft_force(n_p, n_f, psi + eps * xd, 1.3) - nufft.nufft_force(n_p, n_f, psi - eps * xd, 1.3)) / (2 * eps)
    assert rel(J, fd) < 1e-6
    lhs = np.sum(u * J)
    rhs = np.sum(nufft.nufft_force_vjp(n_p, n_f, psi, 1.3, u) * xd)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
