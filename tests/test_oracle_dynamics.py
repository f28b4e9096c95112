"""Pins of the oracle's N-body run, NUFFT force, power spectrum and
store-all adjoint (CPU only)."""
import math

import numpy as np
from scipy.integrate import quad
import pytest

from oracle import adjoint, cosmo, force, ics, mesh, nbody, nufft, pk
from oracle.force import PMConfig


def _plane_wave_run(n_g, A_w=0.5, order=3, stepper="bullfrog"):
    n_p, box = 32, 100.0
    cfg = PMConfig(n_p, n_g, box, order=order, deconvolve=False, grad_order=4, lap_order=0)
    prob = nbody.Problem(cfg, omega_m=1.0, spectrum="powerlaw", a_start=0.02, a_end=1.0, n_steps=6,
                         stepper=stepper)
    kw = 2 * math.pi / box
    q = mesh.lattice(n_p)[0] * (box / n_p)
    dq = box / n_p
    psi = np.zeros((3, n_p ** 3))
    psi[0] = -(A_w / kw) * np.sin(kw * q) / dq
    out, _ = nbody.run_from(prob, 0.02 * psi, psi)
    return out, 1.0 * psi, A_w / kw / dq


@pytest.mark.parametrize("stepper", ["bullfrog", "fastpm"])
def test_plane_wave_follows_zeldovich_before_shell_crossing(stepper):
    # EdS, D = a; BullFrog and FastPM are Zel'dovich consistent, so only PM
    # force error remains, and it must shrink with the mesh.  TSC keeps the
    # lattice's aliasing error below 1%; CIC errs by a few per cent
    # (discreteness) and is checked only for convergence
    errs = []
    for n_g in (64, 128):
        out, exact, amp = _plane_wave_run(n_g, stepper=stepper)
        errs.append(np.abs(out - exact).max() / amp)
    assert errs[0] < 0.015 and errs[1] < errs[0]
    e64 = _plane_wave_run(64, order=2)
    e128 = _plane_wave_run(128, order=2)
    c = [np.abs(o - e).max() / a for o, e, a in (e64, e128)]
    assert c[0] < 0.06 and c[1] < 0.7 * c[0]


def test_low_k_power_grows_as_D_squared():
    cfg = PMConfig(32, 64, 100.0, order=2, deconvolve=False, grad_order=4, lap_order=0)
    # C1 geometry; the lowest bin grows as D^2 up to a mode-coupling
    # correction that itself grows with D (0.5% at a = 0.05, 1.2% at 0.1)
    dev = []
    for a1 in (0.05, 0.1):
        prob = nbody.Problem(cfg, omega_m=1.0, spectrum="powerlaw", a_start=0.02, a_end=a1, n_steps=4)
        w = nbody.white_noise(prob, 54321)
        psi0, v0, _ = nbody.initial_state(prob, w)
        psi, _ = nbody.run_from(prob, psi0, v0)
        p0 = pk.power_spectrum(adjoint.final_density(prob, psi0), 100.0, 4)[1]
        p1 = pk.power_spectrum(adjoint.final_density(prob, psi), 100.0, 4)[1]
        dev.append(abs(p1[0] / p0[0] / (a1 / 0.02) ** 2 - 1))
    assert dev[0] < 0.01 and dev[0] < dev[1] < 0.02


def test_reverse_integration_recovers_initial_state():
    # primal rows of tab. adjoint_dkd undo the forward step (time reversibility)
    cfg = PMConfig(16, 32, 50.0, order=3, deconvolve=True, grad_order=4, lap_order=0)
    prob = nbody.Problem(cfg, omega_m=0.31, a_start=0.02, a_end=1.0, n_steps=5)
    psi0, v0, _ = nbody.initial_state(prob, nbody.white_noise(prob, 11))
    psi, vel = nbody.run_from(prob, psi0, v0)
    force = prob.force_fn()
    for st in reversed(prob.steps()):
        psi = psi - st.tau2 * vel
        vel = (vel - st.beta * force(psi, st.s)) / st.alpha
        psi = psi - st.tau1 * vel
    assert np.abs(psi - psi0).max() < 1e-9 * np.abs(psi0).max()
    assert np.abs(vel - v0).max() < 1e-9 * np.abs(v0).max()


# ---------------------------------------------------------------- NUFFT ----

def test_nufft_spreading_matches_direct_nudft():
    n_p, n_f = 8, 16
    psi = np.random.default_rng(1).normal(0, 0.7, (3, n_p ** 3))
    A1 = nufft.nudft_force_direct(n_p, n_f, psi, 1.0)
    A2 = nufft.nufft_force(n_p, n_f, psi, 1.0, 6, 13.8)
    assert np.linalg.norm(A1 - A2) / np.linalg.norm(A1) < 1.5e-5


def test_nufft_uniform_lattice_reduces_to_dft():
    # particles on the lattice: the NUDFT is the plain DFT of a constant, so
    # every kept mode but m = 0 vanishes and the force is zero
    n_p, n_f = 8, 16
    A = nufft.nufft_force(n_p, n_f, np.zeros((3, n_p ** 3)), 1.0)
    assert np.abs(A).max() < 1e-12


def test_nufft_net_force_and_linear_displacement():
    n_p, n_f = 8, 16
    psi = np.random.default_rng(2).normal(0, 0.5, (3, n_p ** 3))
    A = nufft.nufft_force(n_p, n_f, psi, 1.0)
    assert np.abs(A.sum(axis=1)).max() < 1e-10 * np.abs(A).sum()
    # a single low Fourier mode of small displacement: -grad Lap^-1 delta
    # equals the displacement itself to first order
    q = mesh.lattice(n_p)
    eps = 1e-4
    psi = np.zeros((3, n_p ** 3))
    psi[1] = eps * np.sin(2 * math.pi * q[1] / n_p)
    # the direct sums are exact here (the spreading path errs by ~1e-5 of the
    # total mass per mode, which swamps a 1e-4 perturbation)
    A = nufft.nudft_force_direct(n_p, n_f, psi, 1.0)
    assert np.abs(A[1] - psi[1]).max() < 1e-6 * eps


def test_es_fixedpoint_spread_matches_float_spread():
    n_p, n_f = 8, 16
    psi = np.random.default_rng(3).normal(0, 1.0, (3, n_p ** 3)).astype(np.float32)
    fx = nufft.deposit_fixedpoint_es(psi, n_p, n_f)
    fl = nufft._spread_float(mesh.mesh_coords(psi.astype(np.float64), n_p, n_f), n_f, 6, 13.8)
    assert np.linalg.norm(fx / nufft.ES_UNIT - fl) / np.linalg.norm(fl) < 2e-6


def test_es_fixedpoint_peak_and_support():
    """A particle on a node puts phi(0)^3 = 2^31 units on it; the nodes 3
    cells away lie on the edge of the support (phi = 0 there); a half-cell
    offset along z weighs the two nearest nodes equally."""
    n_f = 16
    st = {int(l[0]): int(w[0]) for l, w in nufft.es_fixed_stencil(np.zeros((3, 1), dtype=np.int64), n_f)}
    assert st[0] == 2 ** 31
    assert st[3] == 0 and st[(3 * n_f) * n_f] == 0 and st[n_f - 2] > 0
    U = np.array([[0], [0], [1 << 19]], dtype=np.int64)
    st = {int(l[0]): int(w[0]) for l, w in nufft.es_fixed_stencil(U, n_f)}
    assert st[0] == st[1] and st[n_f - 1] == st[2] and st[0] > st[2] > 0


# ------------------------------------------------------------------ P(k) ---

def test_pk_single_cosine_mode():
    n, box, amp = 16, 80.0, 0.3
    m0 = np.array([1, 2, 3])
    j = np.indices((n, n, n)).reshape(3, -1)
    delta = amp * np.cos(2 * math.pi * (m0 @ j) / n)
    kb, p, cnt = pk.power_spectrum(delta, box, 8)
    b = int(pk.bin_index(np.array([m0 @ m0]))[0])
    th = 2 * math.pi * m0 / n
    # the CIC window by quadrature of the triangle kernel's Fourier integral
    W = np.prod([quad(lambda x, t=t: (1.0 - abs(x)) * math.cos(t * x), -1.0, 1.0, points=[0.0])[0] for t in th])
    assert abs(p[b - 1] / (amp ** 2 * box ** 3 / (2 * W * W * cnt[b - 1])) - 1) < 1e-12
    others = np.delete(p, b - 1)
    assert np.all(np.abs(others) < 1e-20)


def test_pk_bin_counts_match_brute_force_full_grid():
    n = 12
    m = np.fft.fftfreq(n, 1.0 / n)
    mx, my, mz = np.meshgrid(m, m, m, indexing="ij")
    t = 4 * (mx ** 2 + my ** 2 + mz ** 2)
    _, _, cnt = pk.power_spectrum(np.zeros(n ** 3) + 1e-3 * np.arange(n ** 3) % 1, 1.0, n // 2)
    # modes with m_z = -n/2 are folded onto +n/2 in the half spectrum
    for b in range(1, n // 2 + 1):
        brute = np.sum(((2 * b - 1) ** 2 <= t) & (t < (2 * b + 1) ** 2))
        assert cnt[b - 1] == brute


def test_pk_white_noise_level():
    n, box = 32, 100.0
    rng = np.random.default_rng(4)
    ps = np.mean([pk.power_spectrum(rng.normal(size=n ** 3), box, 16, deconvolve_cic=False)[1]
                  for _ in range(4)], axis=0)
    assert abs(np.sum(ps[4:]) / (12 * box ** 3 / n ** 3) - 1) < 0.03


# --------------------------------------------------------------- adjoint ---

def _small_problem():
    cfg = PMConfig(8, 16, 40.0, order=2, deconvolve=False, grad_order=4, lap_order=0)
    return nbody.Problem(cfg, omega_m=0.31, a_start=0.02, a_end=1.0, n_steps=3, sigma8=0.9)


def test_force_vjp_matches_finite_differences():
    prob = _small_problem()
    cfg = prob.pm
    rng = np.random.default_rng(5)
    psi = rng.normal(0, 1.0, (3, cfg.N))
    u = rng.normal(size=(3, cfg.N))
    v = rng.normal(size=(3, cfg.N))
    jt = adjoint.force_vjp(cfg, psi, 2.0, u)
    eps = 1e-6
    fd = (np.sum(u * prob.force_fn()(psi + eps * v, 2.0))
          - np.sum(u * prob.force_fn()(psi - eps * v, 2.0))) / (2 * eps)
    assert abs(np.sum(jt * v) - fd) < 1e-6 * abs(fd)


@pytest.mark.parametrize("order,dec,g", [(2, False, 4), (3, True, 2), (4, True, 6)])
def test_interlaced_force_vjp_matches_finite_differences(order, dec, g):
    # the interlaced VJP against central differences of the interlaced
    # force; its two parts add up to the whole
    cfg = PMConfig(8, 16, 40.0, order=order, deconvolve=dec, grad_order=g, lap_order=0, interlace=True)
    rng = np.random.default_rng(50 + order)
    psi = rng.normal(0, 1.0, (3, cfg.N))
    u = rng.normal(size=(3, cfg.N))
    v = rng.normal(size=(3, cfg.N))
    jt = adjoint.force_vjp(cfg, psi, 2.0, u)
    eps = 1e-6
    fd = (np.sum(u * force.pm_force(cfg, psi + eps * v, 2.0))
          - np.sum(u * force.pm_force(cfg, psi - eps * v, 2.0))) / (2 * eps)
    assert abs(np.sum(jt * v) - fd) < 1e-6 * abs(fd)
    split = adjoint.force_vjp(cfg, psi, 2.0, u, parts=1) + adjoint.force_vjp(cfg, psi, 2.0, u, parts=2)
    assert np.allclose(split, jt, rtol=0, atol=1e-12 * np.abs(jt).max())
    # the single-grid VJP differs (the second grid's terms are in it)
    plain = adjoint.force_vjp(PMConfig(8, 16, 40.0, order=order, deconvolve=dec, grad_order=g), psi, 2.0, u)
    assert np.linalg.norm(plain - jt) > 1e-3 * np.linalg.norm(jt)


def test_interlaced_gradient_matches_finite_differences():
    cfg = PMConfig(8, 16, 40.0, order=3, deconvolve=True, grad_order=4, lap_order=0, interlace=True)
    prob = nbody.Problem(cfg, omega_m=0.31, a_start=0.02, a_end=1.0, n_steps=3, sigma8=0.9)
    n = cfg.n_p
    rng = np.random.default_rng(8)
    w = nbody.white_noise(prob, 4).astype(np.float64)
    target = rng.normal(size=cfg.n_g ** 3)

    def loss_of(w_):
        psi0, v0, _ = nbody.initial_state(prob, w_.reshape(n, n, n))
        psi, _ = nbody.run_from(prob, psi0, v0)
        return np.sum((adjoint.final_density(prob, psi) - target) ** 2)

    wbar, _, _ = adjoint.gradient(prob, w, lambda d: 2 * (d - target))
    for _ in range(2):
        dirn = rng.normal(size=n ** 3)
        dirn /= np.linalg.norm(dirn)
        eps = 1e-6
        fd = (loss_of(w.reshape(-1) + eps * dirn) - loss_of(w.reshape(-1) - eps * dirn)) / (2 * eps)
        assert abs(np.dot(wbar, dirn) - fd) < 1e-5 * abs(fd) + 1e-9


def test_ic_vjp_is_the_transpose():
    prob = _small_problem()
    n = prob.pm.n_p
    rng = np.random.default_rng(6)
    w = rng.normal(size=(n, n, n))
    pb = rng.normal(size=(3, n ** 3))
    psi = ics.zeldovich_psi(w, prob.pm.box, prob.spectrum_fn(), prob.D_ref())
    lhs = np.sum(psi * pb)
    rhs = np.sum(w.reshape(-1) * adjoint.ic_vjp(prob, pb).reshape(-1))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_full_gradient_matches_finite_differences():
    prob = _small_problem()
    n = prob.pm.n_p
    rng = np.random.default_rng(7)
    w = nbody.white_noise(prob, 3).astype(np.float64)
    target = rng.normal(size=prob.pm.n_g ** 3)

    def loss_of(w_, prob_=prob):
        psi0, v0, _ = nbody.initial_state(prob_, w_.reshape(n, n, n))
        psi, _ = nbody.run_from(prob_, psi0, v0)
        return np.sum((adjoint.final_density(prob_, psi) - target) ** 2)

    wbar, dsig, _ = adjoint.gradient(prob, w, lambda d: 2 * (d - target))
    for k in range(3):
        dirn = rng.normal(size=n ** 3)
        dirn /= np.linalg.norm(dirn)
        eps = 1e-6
        fd = (loss_of(w.reshape(-1) + eps * dirn) - loss_of(w.reshape(-1) - eps * dirn)) / (2 * eps)
        assert abs(np.dot(wbar, dirn) - fd) < 1e-5 * abs(fd) + 1e-9
    p2 = nbody.Problem(prob.pm, omega_m=0.31, a_start=0.02, a_end=1.0, n_steps=3, sigma8=0.9 + 1e-6)
    p3 = nbody.Problem(prob.pm, omega_m=0.31, a_start=0.02, a_end=1.0, n_steps=3, sigma8=0.9 - 1e-6)
    fd = (loss_of(w.reshape(-1), p2) - loss_of(w.reshape(-1), p3)) / 2e-6
    assert abs(dsig - fd) < 1e-5 * abs(fd)


def test_powerlaw_spectrum_gradient_has_no_sigma8_term():
    # the power-law configuration is normalised by its rms displacement, so
    # its forward run does not change with sigma8 and dL/dsigma8 is 0
    cfg = PMConfig(8, 16, 25.0, order=2, deconvolve=False, grad_order=4, lap_order=0)
    kw = dict(omega_m=1.0, spectrum="powerlaw", a_start=0.02, a_end=1.0, n_steps=2)
    p1 = nbody.Problem(cfg, sigma8=0.8, **kw)
    p2 = nbody.Problem(cfg, sigma8=1.1, **kw)
    w = nbody.white_noise(p1, 9).astype(np.float64)
    x1, _ = nbody.run(p1, w=w)
    x2, _ = nbody.run(p2, w=w)
    assert np.array_equal(x1, x2)
    _, dsig, _ = adjoint.gradient(p1, w, lambda d: 2 * d)
    assert dsig == 0.0


@pytest.mark.parametrize("stepper", ["bullfrog", "fastpm", "leapfrog"])
def test_temporal_adjoints_match_finite_differences(stepper):
    # tab. adjoint_dkd: the adjoints of each step's tau1, tau2, alpha, beta
    # against central differences of the forward map with that one scalar moved
    import dataclasses
    prob = _small_problem()
    prob.stepper = stepper
    prob._cache.clear()
    n = prob.pm.n_p
    rng = np.random.default_rng(11)
    w = nbody.white_noise(prob, 5).astype(np.float64)
    target = rng.normal(size=prob.pm.n_g ** 3)
    temporal = []
    adjoint.gradient(prob, w, lambda d: 2 * (d - target), temporal=temporal)
    steps = prob.steps()
    assert len(temporal) == len(steps)
    psi0, v0, _ = nbody.initial_state(prob, w)

    def loss_with(k, field, value):
        st = list(steps)
        st[k] = dataclasses.replace(st[k], **{field: value})
        psi, _ = nbody.run_from(prob, psi0, v0, steps=st)
        return np.sum((adjoint.final_density(prob, psi) - target) ** 2)

    for k in range(len(steps)):
        for j, field in enumerate(("tau1", "tau2", "alpha", "beta")):
            x = getattr(steps[k], field)
            eps = 1e-7 * max(abs(x), 1e-3)
            fd = (loss_with(k, field, x + eps) - loss_with(k, field, x - eps)) / (2 * eps)
            assert abs(temporal[k][j] - fd) < 1e-5 * abs(fd) + 1e-6, (k, field, temporal[k][j], fd)


def test_leapfrog_gradient_matches_finite_differences():
    # the store-all gradient with the canonical momentum (V = zeta(a_start)
    # times the growth-time velocity at the start), steps uniform in
    # superconformal time, against central differences of the run
    cfg = PMConfig(8, 16, 40.0, order=3, deconvolve=False, grad_order=4, lap_order=0)
    prob = nbody.Problem(cfg, omega_m=0.31, a_start=0.02, a_end=1.0, n_steps=4, sigma8=0.9,
                         stepper="leapfrog", time_var="superconft")
    n = cfg.n_p
    rng = np.random.default_rng(17)
    w = nbody.white_noise(prob, 8).astype(np.float64)
    target = rng.normal(size=cfg.n_g ** 3)

    def loss_of(wv, s8=0.9):
        p = nbody.Problem(cfg, omega_m=0.31, a_start=0.02, a_end=1.0, n_steps=4, sigma8=s8,
                          stepper="leapfrog", time_var="superconft")
        x, _ = nbody.run(p, w=wv.reshape(n, n, n))
        return np.sum((adjoint.final_density(p, x) - target) ** 2)

    wbar, dsig, _ = adjoint.gradient(prob, w, lambda d: 2 * (d - target))
    dirn = rng.normal(size=n ** 3)
    eps = 1e-6
    fd = (loss_of(w.reshape(-1) + eps * dirn) - loss_of(w.reshape(-1) - eps * dirn)) / (2 * eps)
    assert abs(np.dot(wbar, dirn) - fd) < 1e-6 * abs(fd)
    fd = (loss_of(w.reshape(-1), 0.9 + eps) - loss_of(w.reshape(-1), 0.9 - eps)) / (2 * eps)
    assert abs(dsig - fd) < 1e-6 * abs(fd)
