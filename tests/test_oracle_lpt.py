"""Pins of the oracle's second-order LPT displacement (oracle.ics).

Sec. "Lagrangian perturbation theory" (eq. LPT, eq. helmholtz, eq. LPT_L_and_T,
eq. LPT_kernels) and Sec. "Time stepping" (BullFrog aligns the N-body
trajectory with 2LPT after every step).  Three independent checks:
* a closed form: for phi = A cos(k1 x) + B cos(k2 y) the only second-order
  source is phi_xx phi_yy, so psi^(2) is one product term, written out;
* brute force: the de-aliased product evaluated with explicit DFT matrices on
  a grid twice as fine (no FFT, a different padding than the 3/2 rule);
* dynamics: BullFrog with the exact band-limited force (direct NUDFT sums)
  started on the 2LPT trajectory in EdS at a = 0.5 stays on it for 1, 2 and
  4 steps up to third-order terms, while the Zel'dovich start at the same
  time misses a large part of the second-order term (started early, BullFrog
  builds the 2LPT term itself, so the start must be late to tell them apart).
"""
import numpy as np
import pytest

from oracle import cosmo, ics, nbody, nufft
from oracle.force import PMConfig


def lattice(n):
    return np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij")).reshape(3, -1).astype(np.float64)


def band_limited_psi1(n, mmax, seed, rms):
    """psi^(1) = -grad phi with phi a random field of the modes |m_a| <= mmax."""
    rng = np.random.default_rng(seed)
    m = np.fft.fftfreq(n, 1.0 / n)
    band = np.abs(m) <= mmax
    phik = np.fft.fftn(rng.standard_normal((n, n, n))) * (band[:, None, None] & band[None, :, None] & band[None, None, :])
    k = 2 * np.pi * m / n
    kk = [k[:, None, None], k[None, :, None], k[None, None, :]]
    psi = np.stack([np.fft.ifftn(-1j * kk[c] * phik).real.reshape(-1) for c in range(3)])
    return psi * rms / np.sqrt((psi ** 2).sum(0).mean())


def test_second_order_two_plane_waves_closed_form():
    n = 16
    q = lattice(n)
    m1, m2, A, B = 3, 5, 0.3, -0.2
    k1, k2 = 2 * np.pi * m1 / n, 2 * np.pi * m2 / n
    # phi = A cos(k1 x) + B cos(k2 y), psi1 = -grad phi
    psi1 = np.stack([A * k1 * np.sin(k1 * q[0]), B * k2 * np.sin(k2 * q[1]), 0 * q[0]])
    # mu_2L = phi_xx phi_yy = A B k1^2 k2^2 cos cos, Delta^-1 cos cos = -cos cos / (k1^2 + k2^2),
    # psi2 = -(3/7) grad Delta^-1 mu
    c = 3.0 / 7.0 * A * B * k1 ** 2 * k2 ** 2 / (k1 ** 2 + k2 ** 2)
    ref = c * np.stack([-k1 * np.sin(k1 * q[0]) * np.cos(k2 * q[1]),
                        -k2 * np.cos(k1 * q[0]) * np.sin(k2 * q[1]), 0 * q[0]])
    got = ics.second_order_psi(psi1, n)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    # a single plane wave has no second-order displacement
    assert np.abs(ics.second_order_psi(np.stack([psi1[0], 0 * q[0], 0 * q[0]]), n)).max() < 1e-15


def _dft_matrix(n_out, n_in, sign, scale_in):
    """E[a, b] = exp(sign 2 pi i a b' / n) with b' = b * scale_in (grid points
    of spacing scale_in lattice units), a, b' as signed modes / positions."""
    a = np.fft.fftfreq(n_out, 1.0 / n_out)[:, None]
    b = np.arange(n_in)[None, :] * scale_in
    return a, b


def test_second_order_dealiasing_by_direct_sums():
    n = 8
    psi1 = band_limited_psi1(n, n // 2 - 1, 11, 0.3)
    # spectra of psi1 by explicit sums: F[m] = sum_j psi(j) exp(-2 pi i m.j / n)
    m = np.fft.fftfreq(n, 1.0 / n)
    j = np.arange(n)
    E = np.exp(-2j * np.pi * np.outer(m, j) / n)               # (m, j)
    spec = [np.einsum("ax,by,cz,xyz->abc", E, E, E, psi1[c].reshape(n, n, n)) for c in range(3)]
    band = np.abs(m) < n // 2
    k = 2 * np.pi * m / n
    # gradients on the twice finer grid x = j / 2 by explicit sums over the band
    xf = np.arange(2 * n) / 2.0
    Ef = np.exp(2j * np.pi * np.outer(xf, m[band]) / n) / n     # (x, m)
    def fine(s):
        return np.einsum("xa,yb,zc,abc->xyz", Ef, Ef, Ef, s[np.ix_(band, band, band)]).real
    kk = [k[:, None, None], k[None, :, None], k[None, None, :]]
    g = [[fine(1j * kk[jj] * spec[i]) for jj in range(3)] for i in range(3)]
    mu = sum(0.5 * (g[i][i] * g[jj][jj] - g[i][jj] * g[jj][i]) for i in range(3) for jj in range(3))
    # coefficients of the (degree < n) product on the band, then psi2 on the lattice
    Eb = np.exp(-2j * np.pi * np.outer(m[band], xf) / n) / (2 * n)
    mu_b = np.einsum("ax,by,cz,xyz->abc", Eb, Eb, Eb, mu) * n ** 3
    kb = [k[band][:, None, None], k[band][None, :, None], k[band][None, None, :]]
    k2 = kb[0] ** 2 + kb[1] ** 2 + kb[2] ** 2
    inv = np.where(k2 > 0, -1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    Ei = np.exp(2j * np.pi * np.outer(j, m[band]) / n) / n
    ref = np.stack([np.einsum("xa,yb,zc,abc->xyz", Ei, Ei, Ei, 1j * kb[c] * inv * (-3.0 / 7.0) * mu_b).real.reshape(-1)
                    for c in range(3)])
    got = ics.second_order_psi(psi1, n)
    assert np.linalg.norm(got - ref) < 1e-12 * np.linalg.norm(ref)
    # the same product taken on the lattice itself (aliased) is measurably different
    gl = [[np.fft.ifftn(1j * kk[jj] * spec[i] * (band[:, None, None] & band[None, :, None] & band[None, None, :])).real
           for jj in range(3)] for i in range(3)]
    mu_l = sum(0.5 * (gl[i][i] * gl[jj][jj] - gl[i][jj] * gl[jj][i]) for i in range(3) for jj in range(3))
    muk = np.fft.fftn(mu_l)
    K2 = kk[0] ** 2 + kk[1] ** 2 + kk[2] ** 2
    INV = np.where(K2 > 0, -1.0 / np.where(K2 > 0, K2, 1.0), 0.0)
    aliased = np.stack([np.fft.ifftn(1j * kk[c] * INV * (-3.0 / 7.0) * muk).real.reshape(-1) for c in range(3)])
    assert np.linalg.norm(aliased - ref) > 1e-3 * np.linalg.norm(ref)


def _bullfrog_direct(psi, vel, n, steps, a_start):
    for st in cosmo.bullfrog_steps(1.0, a_start, 1.0, steps):
        psi = psi + st.tau1 * vel
        vel = st.alpha * vel + st.beta * nufft.nudft_force_direct(n, 2 * n, psi, st.s)
        psi = psi + st.tau2 * vel
    return psi, vel


@pytest.mark.parametrize("steps", [1, 2, 4])
def test_bullfrog_stays_on_2lpt_in_eds(steps):
    n = 8
    psi1 = band_limited_psi1(n, 1, 5, 0.005)     # rms displacement 0.005 dq at D = 1
    psi2 = ics.second_order_psi(psi1, n)
    X1, V1 = ics.lpt_state(psi1, psi2, 1.0)
    a0 = 0.5                                     # EdS: D = a
    X, V = _bullfrog_direct(*ics.lpt_state(psi1, psi2, a0), n, steps, a0)
    # residual relative to the 2LPT term: third order only (~ the amplitude)
    assert np.linalg.norm(X - X1) < 1e-2 * np.linalg.norm(psi2)
    assert np.linalg.norm(V - V1) < 1e-2 * np.linalg.norm(2 * psi2)
    # started on Zel'dovich, the run misses the second-order term
    Xz, _ = _bullfrog_direct(*ics.lpt_state(psi1, None, a0), n, steps, a0)
    assert np.linalg.norm(Xz - X1) > 0.3 * np.linalg.norm(psi2)


def test_second_order_vjp_and_jvp_match_differences():
    # the transposed and tangent maps of psi2(psi1) against central
    # differences of second_order_psi (a quadratic map: the differences are
    # exact up to rounding), their duality and Euler's identity for a
    # homogeneous quadratic, <VJP(b), psi1> = 2 <b, psi2>
    from oracle import ics
    rng = np.random.default_rng(11)
    n = 8
    psi1 = rng.normal(size=(3, n ** 3))
    b = rng.normal(size=(3, n ** 3))
    d = rng.normal(size=(3, n ** 3))
    eps = 1e-5
    fd = (ics.second_order_psi(psi1 + eps * d, n) - ics.second_order_psi(psi1 - eps * d, n)) / (2 * eps)
    jv = ics.second_order_psi_jvp(psi1, n, d)
    assert np.linalg.norm(jv - fd) < 1e-9 * np.linalg.norm(fd)
    vj = ics.second_order_psi_vjp(psi1, n, b)
    assert abs(np.sum(vj * d) - np.sum(b * jv)) < 1e-12 * abs(np.sum(b * jv))
    assert abs(np.sum(vj * psi1) - 2 * np.sum(b * ics.second_order_psi(psi1, n))) < 1e-12 * np.sum(np.abs(vj * psi1))


def test_second_order_gradient_and_tangent_match_differences():
    from oracle import adjoint, jvp
    cfg = PMConfig(8, 16, 40.0, order=3, deconvolve=False, grad_order=4)
    prob = nbody.Problem(cfg, omega_m=0.31, a_start=0.02, a_end=1.0, n_steps=3, sigma8=0.9, lpt_order=2)
    n = cfg.n_p
    rng = np.random.default_rng(12)
    w = nbody.white_noise(prob, 6).astype(np.float64)
    target = rng.normal(size=cfg.n_g ** 3)

    def final(wv, s8):
        p = nbody.Problem(cfg, omega_m=0.31, a_start=0.02, a_end=1.0, n_steps=3, sigma8=s8, lpt_order=2)
        x, _ = nbody.run(p, w=wv.reshape(n, n, n))
        return adjoint.final_density(p, x)

    wbar, dsig, _ = adjoint.gradient(prob, w, lambda d: 2 * (d - target))
    dirn = rng.normal(size=n ** 3)
    eps = 1e-6
    loss = lambda wv, s8: np.sum((final(wv, s8) - target) ** 2)
    fd = (loss(w.reshape(-1) + eps * dirn, 0.9) - loss(w.reshape(-1) - eps * dirn, 0.9)) / (2 * eps)
    assert abs(np.dot(wbar, dirn) - fd) < 1e-6 * abs(fd)
    fd = (loss(w.reshape(-1), 0.9 + eps) - loss(w.reshape(-1), 0.9 - eps)) / (2 * eps)
    assert abs(dsig - fd) < 1e-6 * abs(fd)
    _, _, _, dd = jvp.run_jvp(prob, w, dirn, 0.2)
    fd = (final(w.reshape(-1) + eps * dirn, 0.9 + 0.2 * eps) - final(w.reshape(-1) - eps * dirn, 0.9 - 0.2 * eps)) / (2 * eps)
    assert np.linalg.norm(dd - fd) < 1e-7 * np.linalg.norm(fd)
