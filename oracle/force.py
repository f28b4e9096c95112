"""Particle-mesh force in FP64 (test infrastructure only).

Follows Sec. "Force evaluation: particle-mesh and non-uniform FFT":
deposit -> density contrast -> real FFT -> Poisson solve with the gradient
and Laplacian kernels of tab. derivative_kernels -> optional deconvolution by
the squared window of tab. interpolation_kernels -> one inverse real FFT per
component -> gather with the same kernel.

Readings of the paper used here (listed with the others in the design notes):
* Order-2 Laplacian: the printed Fourier form has the wrong sign; the stencil
  [1 -2 1] transforms to -2 (1 - cos theta), which is what is used.
* The 3D gradient kernel along axis c is the 1D kernel along c alone, and the
  3D Laplacian is the sum of the 1D second-derivative kernels (the table
  caption's "product" holds only for the interpolation windows).
* The exact gradient i k is odd and undefined on the Nyquist plane of its own
  axis, where it is set to zero; all multipliers vanish at k = 0.
* Acceleration in growth-factor time: A = -grad Laplacian^-1 delta / D^2 at
  the kick's midpoint (s = 1/D_{n+1/2}^2), which keeps V = dX/dD equal to the
  Zel'dovich velocity (see the design notes for the derivation).
* Units: wavenumbers as theta = 2 pi m / n_g (mesh units); the result is
  converted from mesh cells to lattice units dq by 1/r, r = n_g / n_p.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import mesh


@dataclass
class PMConfig:
    n_p: int
    n_g: int
    box: float
    order: int = 2          # 2 CIC, 3 TSC, 4 PCS
    deconvolve: bool = False
    grad_order: int = 4     # 0 exact i k, else 2/4/6
    lap_order: int = 0      # 0 exact -k^2, else 2/4/6
    interlace: bool = False # antialias = 1: a second grid half a cell along the diagonal

    @property
    def N(self):
        return self.n_p ** 3

    @property
    def r(self):
        return self.n_g // self.n_p


def grad_kernel(theta, order):
    """Fourier multiplier of d/dx in mesh units (divided by nothing: i theta
    for the exact kernel; FD stencils of tab. derivative_kernels)."""
    if order == 0:
        return 1j * theta
    if order == 2:
        return 1j * np.sin(theta)
    if order == 4:
        return 1j * (8.0 * np.sin(theta) - np.sin(2 * theta)) / 6.0
    if order == 6:
        return 1j * (45.0 * np.sin(theta) - 9.0 * np.sin(2 * theta) + np.sin(3 * theta)) / 30.0
    raise ValueError(order)


def lap_kernel_1d(theta, order):
    """Fourier multiplier of d^2/dx^2 in mesh units."""
    if order == 0:
        return -theta * theta
    if order == 2:
        return -2.0 * (1.0 - np.cos(theta))
    if order == 4:
        return -(np.cos(2 * theta) - 16.0 * np.cos(theta) + 15.0) / 6.0
    if order == 6:
        return -(-2.0 * np.cos(3 * theta) + 27.0 * np.cos(2 * theta)
                 - 270.0 * np.cos(theta) + 245.0) / 90.0
    raise ValueError(order)


def window_1d(theta, p):
    """sinc^p(k/2) with k in Nyquist units, i.e. (sin(theta/2)/(theta/2))^p."""
    h = 0.5 * np.asarray(theta, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        s = np.where(h == 0, 1.0, np.sin(h) / np.where(h == 0, 1.0, h))
    return s ** p


def half_spectrum_theta(n):
    """theta_x, theta_y, theta_z on the [n][n][n/2+1] half spectrum, and the
    integer modes (numpy fftfreq order: index n/2 on x, y is m = -n/2)."""
    m = np.fft.fftfreq(n, 1.0 / n)
    mz = np.arange(n // 2 + 1, dtype=np.float64)
    mx, my, mzz = np.meshgrid(m, m, mz, indexing="ij")
    return 2 * np.pi * mx / n, 2 * np.pi * my / n, 2 * np.pi * mzz / n, (mx, my, mzz)


def force_multipliers(cfg: PMConfig, s: float):
    """K_c = -G_c s / (r Lap W^(2 dec)) on the half spectrum, shape
    (3, n, n, n/2+1)."""
    n = cfg.n_g
    tx, ty, tz, (mx, my, mz) = half_spectrum_theta(n)
    lap = (lap_kernel_1d(tx, cfg.lap_order) + lap_kernel_1d(ty, cfg.lap_order)
           + lap_kernel_1d(tz, cfg.lap_order))
    zero = (mx == 0) & (my == 0) & (mz == 0)
    lap_safe = np.where(zero, 1.0, lap)
    H = -s / (cfg.r * lap_safe)
    if cfg.deconvolve:
        W = window_1d(tx, cfg.order) * window_1d(ty, cfg.order) * window_1d(tz, cfg.order)
        H = H / (W * W)
    H = np.where(zero, 0.0, H)
    K = np.empty((3,) + H.shape, dtype=np.complex128)
    for c, (t, m) in enumerate(((tx, mx), (ty, my), (tz, mz))):
        G = grad_kernel(t, cfg.grad_order)
        if cfg.grad_order == 0:
            G = np.where(np.abs(m) == n // 2, 0.0, G)
        K[c] = G * H
    return K


def density_contrast(cfg: PMConfig, psi):
    m = mesh.deposit(psi, cfg.n_p, cfg.n_g, cfg.order)
    return mesh.contrast(m, cfg.N, cfg.n_g)


def force_meshes(cfg: PMConfig, delta, s):
    """g_c = IDFT(K_c DFT(delta)) on the mesh, shape (3, n_g^3)."""
    n = cfg.n_g
    dk = np.fft.rfftn(np.asarray(delta, dtype=np.float64).reshape(n, n, n))
    K = force_multipliers(cfg, s)
    return np.stack([np.fft.irfftn(K[c] * dk, s=(n, n, n), axes=(0, 1, 2)).reshape(-1) for c in range(3)])


def interlace_phase(n):
    """exp(i (theta_x + theta_y + theta_z) / 2) on the half spectrum: the
    transform of a mesh sampled half a cell down the diagonal, times this,
    is the transform of the same density on the original nodes."""
    tx, ty, tz, _ = half_spectrum_theta(n)
    return np.exp(0.5j * (tx + ty + tz))


def pm_force_u(cfg: PMConfig, u, s):
    """A in dq units per unit D at mesh coordinates u (3, M) of M particles of
    mass 1 (the contrast is normalised by cfg.N; the k = 0 mode is removed,
    which is the uniform neutralising background).

    Interlaced grids (Sec. "Discreteness suppression", antialias = 1 of
    tab. default_parameters; the paper cites Chen 1974, Hockney & Eastwood
    and Sefusatti et al. 2016 for the scheme): the particles are deposited
    a second time at u + (1/2, 1/2, 1/2), i.e. onto nodes half a cell down
    the diagonal; the two transforms are averaged with the shift's phase,
    delta = (delta_1 + e^{i phi} delta_2) / 2, phi = (theta_x + theta_y +
    theta_z) / 2, which cancels the aliases of odd total image order; the
    force meshes are evaluated on both grids (the second with e^{-i phi})
    and the two gathers averaged."""
    n = cfg.n_g
    if not cfg.interlace:
        m = mesh.deposit_u(u, cfg.n_g, cfg.order)
        g = force_meshes(cfg, mesh.contrast(m, cfg.N, cfg.n_g), s)
        return np.stack([mesh.gather_u(g[c], u, cfg.n_g, cfg.order) for c in range(3)])
    u2 = np.mod(np.asarray(u, dtype=np.float64) + 0.5, n)
    d1 = np.fft.rfftn(mesh.contrast(mesh.deposit_u(u, n, cfg.order), cfg.N, n).reshape(n, n, n))
    d2 = np.fft.rfftn(mesh.contrast(mesh.deposit_u(u2, n, cfg.order), cfg.N, n).reshape(n, n, n))
    ph = interlace_phase(n)
    dk = 0.5 * (d1 + ph * d2)
    K = force_multipliers(cfg, s)
    A = np.zeros((3, np.asarray(u).shape[1]))
    for c in range(3):
        g1 = np.fft.irfftn(K[c] * dk, s=(n, n, n), axes=(0, 1, 2)).reshape(-1)
        g2 = np.fft.irfftn(K[c] * dk * np.conj(ph), s=(n, n, n), axes=(0, 1, 2)).reshape(-1)
        A[c] = 0.5 * (mesh.gather_u(g1, u, n, cfg.order) + mesh.gather_u(g2, u2, n, cfg.order))
    return A


def pm_force(cfg: PMConfig, psi, s):
    """A(X) in dq units per unit D, shape (3, N)."""
    return pm_force_u(cfg, mesh.mesh_coords(psi, cfg.n_p, cfg.n_g), s)
