"""Pins of the oracle's FFT convention and PM force: stencils vs Fourier
kernels, convergence order, symmetry invariants, Ewald pair force and a plane
wave (CPU only)."""
import math

import numpy as np
import pytest
from scipy.special import erfc

from oracle import force, mesh
from oracle.force import PMConfig

# real-space stencils printed in tab. derivative_kernels (offsets -h..h)
GRAD_STENCILS = {
    2: np.array([-1, 0, 1]) / 2.0,
    4: np.array([1, -8, 0, 8, -1]) / 12.0,
    6: np.array([-1, 9, -45, 0, 45, -9, 1]) / 60.0,
}
LAP_STENCILS = {
    2: np.array([1, -2, 1]) / 1.0,
    4: np.array([-1, 16, -30, 16, -1]) / 12.0,
    6: np.array([2, -27, 270, -490, 270, -27, 2]) / 180.0,
}


def test_fft_matches_naive_dft_8cubed():
    n = 8
    f = np.random.default_rng(0).normal(size=(n, n, n))
    j = np.arange(n)
    E = np.exp(-2j * np.pi * np.outer(j, j) / n)
    naive = np.einsum("ax,by,cz,xyz->abc", E, E, E, f)
    assert np.abs(np.fft.rfftn(f) - naive[:, :, : n // 2 + 1]).max() < 1e-12
    assert np.abs(np.fft.irfftn(np.fft.rfftn(f), s=(n, n, n), axes=(0, 1, 2)) - f).max() < 1e-14


def _stencil_multiplier(stencil, n):
    """Apply sum_s c_s f(x + s) by rolls and read off the Fourier multiplier."""
    f = np.random.default_rng(1).normal(size=n)
    h = len(stencil) // 2
    g = sum(c * np.roll(f, -s) for s, c in zip(range(-h, h + 1), stencil))
    return np.fft.fft(g) / np.fft.fft(f), 2 * np.pi * np.fft.fftfreq(n)


@pytest.mark.parametrize("order", [2, 4, 6])
def test_fourier_kernels_equal_printed_stencils(order):
    mg, th = _stencil_multiplier(GRAD_STENCILS[order], 32)
    assert np.allclose(force.grad_kernel(th, order), mg, atol=1e-12)
    ml, th = _stencil_multiplier(LAP_STENCILS[order], 32)
    assert np.allclose(force.lap_kernel_1d(th, order), ml, atol=1e-12)


@pytest.mark.parametrize("order", [2, 4, 6])
def test_fd_kernels_converge_at_their_order(order):
    errs = []
    for th in (0.2, 0.1):
        eg = abs(force.grad_kernel(th, order) / (1j * th) - 1)
        el = abs(force.lap_kernel_1d(th, order) / (-th * th) - 1)
        errs.append((eg, el))
    assert abs(math.log2(errs[0][0] / errs[1][0]) - order) < 0.1
    assert abs(math.log2(errs[0][1] / errs[1][1]) - order) < 0.1


CONFIGS = [
    PMConfig(8, 16, 20.0, order=2, deconvolve=False, grad_order=4, lap_order=0),
    PMConfig(8, 16, 20.0, order=3, deconvolve=True, grad_order=4, lap_order=0),
    PMConfig(8, 16, 20.0, order=2, deconvolve=False, grad_order=0, lap_order=0),
    PMConfig(8, 16, 20.0, order=3, deconvolve=False, grad_order=2, lap_order=2),
]


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: f"o{c.order}d{int(c.deconvolve)}g{c.grad_order}l{c.lap_order}")
def test_lone_particle_feels_no_self_force(cfg):
    rng = np.random.default_rng(3)
    for _ in range(5):
        u = rng.uniform(0, cfg.n_g, (3, 1))
        a = force.pm_force_u(cfg, u, 1.0)
        # reference scale: the force between two particles one cell apart
        pair = force.pm_force_u(cfg, np.concatenate([u, u + np.array([[1.0], [0], [0]])], 1), 1.0)
        assert np.abs(a).max() < 1e-12 * np.abs(pair).max()


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: f"o{c.order}d{int(c.deconvolve)}g{c.grad_order}l{c.lap_order}")
def test_net_force_vanishes(cfg):
    psi = np.random.default_rng(4).normal(0, 2.0, (3, cfg.N))
    A = force.pm_force(cfg, psi, 1.0)
    assert np.abs(A.sum(axis=1)).max() < 1e-12 * np.abs(A).sum()


def test_unperturbed_lattice_feels_no_force():
    cfg = CONFIGS[1]
    A = force.pm_force(cfg, np.zeros((3, cfg.N)), 1.0)
    assert np.abs(A).max() < 1e-13


def ewald_field(r, box, alpha=None, nmax=3, kmax=8):
    """E = -grad sum_n 1/|r + nL| with a neutralising background (Ewald)."""
    alpha = alpha or 5.0 / box
    E = np.zeros(3)
    rng_ = range(-nmax, nmax + 1)
    for nx in rng_:
        for ny in rng_:
            for nz in rng_:
                rn = r + box * np.array([nx, ny, nz])
                d = np.linalg.norm(rn)
                E += rn / d ** 3 * (erfc(alpha * d) + 2 * alpha * d / math.sqrt(math.pi) * math.exp(-(alpha * d) ** 2))
    kr = range(-kmax, kmax + 1)
    for mx in kr:
        for my in kr:
            for mz in kr:
                if mx == my == mz == 0:
                    continue
                k = 2 * math.pi / box * np.array([mx, my, mz])
                k2 = k @ k
                E += 4 * math.pi / box ** 3 * k / k2 * math.exp(-k2 / (4 * alpha ** 2)) * math.sin(k @ r)
    return E


def test_pair_force_matches_ewald_beyond_a_few_cells():
    # a particle of mass L^3/N (contrast units) at distance r: the periodic
    # point-mass force -(M / 4 pi) E_ewald, in mesh units and converted to dq
    cfg = PMConfig(16, 32, 32.0, order=2, deconvolve=False, grad_order=4, lap_order=0)
    rng = np.random.default_rng(5)
    M = cfg.n_g ** 3 / cfg.N
    rel = {}
    for r in (4.0, 6.0, 8.0):
        errs = []
        for _ in range(16):
            d = rng.normal(size=3)
            d *= r / np.linalg.norm(d)
            u1 = rng.uniform(0, cfg.n_g, 3)
            u = np.stack([u1, u1 + d], axis=1)
            a = force.pm_force_u(cfg, u, 1.0)[:, 0]
            ref = -(M / (4 * math.pi)) * ewald_field(-d, float(cfg.n_g)) / cfg.r
            errs.append(np.linalg.norm(a - ref) / np.linalg.norm(ref))
        rel[r] = math.sqrt(np.mean(np.square(errs)))
    assert rel[4.0] < 0.03 and rel[6.0] < 0.015 and rel[8.0] < 0.01, rel


def test_plane_wave_force_converges_at_fourth_order():
    # delta = eps cos(theta x) on the mesh: exact A = -eps sin(theta x)/theta
    # (mesh units) times s / r; the FD4 gradient errs by O(theta^4)
    errs = []
    for n in (16, 32):
        cfg = PMConfig(n // 2, n, 10.0, order=2, deconvolve=False, grad_order=4, lap_order=0)
        th = 2 * math.pi * 2 / n
        x = np.indices((n, n, n))[0].reshape(-1)
        delta = 0.01 * np.cos(th * x)
        g = force.force_meshes(cfg, delta, 1.0)
        exact = -0.01 * np.sin(th * x) / th / cfg.r
        assert np.abs(g[1]).max() < 1e-15 and np.abs(g[2]).max() < 1e-15
        errs.append(np.abs(g[0] - exact).max() / np.abs(exact).max())
    assert 14 < errs[0] / errs[1] < 18


@pytest.mark.parametrize("order", [2, 3, 4])
def test_window_is_single_particle_aliased_spectrum(order):
    # tab. interpolation_kernels, Fourier column: the DFT of one particle's
    # real-space deposit is, by Poisson summation, the aliased sum over images
    # of the kernel's continuous transform, sum_a W(theta + 2 pi a)
    # exp(-i (theta + 2 pi a) u), and the 3D deposit factorises over axes
    n = 16
    rng = np.random.default_rng(11)
    theta = 2 * np.pi * np.fft.fftfreq(n)
    a = np.arange(-20000, 20001)[:, None]
    for _ in range(3):
        u = rng.uniform(0, n, 3)
        rho = mesh.deposit_u(u[:, None], n, order).reshape(n, n, n)
        got = np.fft.fftn(rho)
        axes = []
        for c in range(3):
            th = theta[None, :] + 2 * np.pi * a
            axes.append(np.sum(force.window_1d(th, order) * np.exp(-1j * th * u[c]), axis=0))
        ref = axes[0][:, None, None] * axes[1][None, :, None] * axes[2][None, None, :]
        assert np.abs(got - ref).max() < 1e-8


@pytest.mark.parametrize("order", [2, 3, 4])
def test_deconvolution_divides_by_the_squared_window(order):
    # a plane wave on the mesh: the deconvolved multiplier is the plain one
    # divided by W(theta_x)^2 W(theta_y)^2 W(theta_z)^2 with the kernel's own
    # order p (window_1d pinned by the aliased-sum test above)
    n = 16
    m0 = np.array([2, 1, 3])
    j = np.indices((n, n, n)).reshape(3, -1)
    delta = 0.01 * np.cos(2 * np.pi * (m0 @ j) / n)
    plain = PMConfig(n // 2, n, 10.0, order=order, deconvolve=False, grad_order=4, lap_order=0)
    dec = PMConfig(n // 2, n, 10.0, order=order, deconvolve=True, grad_order=4, lap_order=0)
    g0 = force.force_meshes(plain, delta, 1.0)
    g1 = force.force_meshes(dec, delta, 1.0)
    th = 2 * np.pi * m0 / n
    W = np.prod(force.window_1d(th, order))
    assert np.abs(g1 - g0 / (W * W)).max() < 1e-13 * np.abs(g1).max()   # FP64 rounding (PCS divides by 0.48)


@pytest.mark.parametrize("order", [2, 3])
def test_interlaced_deposit_keeps_only_even_images(order):
    # one particle: the phase-averaged spectrum of the two grids equals the
    # sum of the aliased window images W(theta + 2 pi a) e^{-i(theta + 2 pi a).u}
    # over the images whose total order a_x + a_y + a_z is even (the odd ones
    # cancel), per mode, to the truncation of the image sums
    n = 8
    rng = np.random.default_rng(3 + order)
    u = rng.uniform(0, n, 3)
    r1 = mesh.deposit_u(u[:, None], n, order).reshape(n, n, n)
    r2 = mesh.deposit_u(np.mod(u + 0.5, n)[:, None], n, order).reshape(n, n, n)
    got = 0.5 * (np.fft.rfftn(r1) + force.interlace_phase(n) * np.fft.rfftn(r2))
    tx, ty, tz, _ = force.half_spectrum_theta(n)
    img = np.arange(-400, 401)
    even = np.zeros_like(got)
    odd_free = np.zeros_like(got)
    per_axis = []
    for c, th in enumerate((tx, ty, tz)):
        t = th[..., None] + 2 * np.pi * img
        e = force.window_1d(t, order) * np.exp(-1j * t * u[c])
        per_axis.append((np.sum(e, axis=-1), np.sum(e * (-1.0) ** img, axis=-1)))
    # product over axes of (S + S_alt)/2 combinations: even total parity
    # = (prod S + prod S_alt) / 2
    even = 0.5 * (per_axis[0][0] * per_axis[1][0] * per_axis[2][0]
                  + per_axis[0][1] * per_axis[1][1] * per_axis[2][1])
    tol = 3e-6 if order == 2 else 1e-8
    assert np.abs(got - even).max() < tol
    # and it differs from the plain deposit by the odd images
    assert np.abs(np.fft.rfftn(r1) - even).max() > 1e-3


def _band_force(n_p, n_g, psi, s):
    """The force of the exact particle density restricted to the mesh band
    |m_a| < n_g/2 (direct sums, exact i k and -k^2, no window): what a PM
    force without aliasing would give."""
    u = mesh.mesh_coords(psi, n_p, n_g)
    ms = np.arange(-(n_g // 2) + 1, n_g // 2)
    mx, my, mz = [a.reshape(-1) for a in np.meshgrid(ms, ms, ms, indexing="ij")]
    E = np.exp(-2j * np.pi / n_g * (np.outer(mx, u[0]) + np.outer(my, u[1]) + np.outer(mz, u[2])))
    d = E.sum(axis=1) * (n_g ** 3 / psi.shape[1])
    th = [2 * np.pi * m / n_g for m in (mx, my, mz)]
    t2 = th[0] ** 2 + th[1] ** 2 + th[2] ** 2
    z = t2 == 0
    K = [np.where(z, 0, 1j * th[c] * s / ((n_g // n_p) * np.where(z, 1, t2))) for c in range(3)]
    return np.stack([np.real((K[c] * d) @ np.conj(E)) / n_g ** 3 for c in range(3)])


def test_interlaced_force_symmetries_and_aliasing():
    # zero force on the lattice and zero net force; against the alias-free
    # band-limited force of the same particles, interlacing (which cancels
    # the odd images) cuts the error of the deconvolved PM force about 3x
    n_p = 8
    for interlace in (False, True):
        cfg = PMConfig(n_p, 2 * n_p, 16.0, order=2, deconvolve=True, grad_order=0, lap_order=0, interlace=interlace)
        assert np.abs(force.pm_force(cfg, np.zeros((3, n_p ** 3)), 1.0)).max() < 1e-12
    rng = np.random.default_rng(9)
    psi = rng.normal(0, 0.6, (3, n_p ** 3))
    exact = _band_force(n_p, 2 * n_p, psi, 1.0)
    for order in (2, 3):
        errs = []
        for interlace in (False, True):
            cfg = PMConfig(n_p, 2 * n_p, 16.0, order=order, deconvolve=True, grad_order=0, lap_order=0,
                           interlace=interlace)
            a = force.pm_force(cfg, psi, 1.0)
            assert np.abs(a.sum(axis=1)).max() < 1e-10 * np.abs(a).sum()
            errs.append(np.linalg.norm(a - exact) / np.linalg.norm(exact))
        assert errs[1] < 0.5 * errs[0], errs
