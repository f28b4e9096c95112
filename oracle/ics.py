"""Zel'dovich initial conditions in FP64 (test infrastructure only).

Follows Sec. "Lagrangian perturbation theory" (first order: psi = -D grad_q
phi_ini, applied in Fourier space with the exact kernels i k and -k^2) and
Sec. "Time stepping" (V = dX/dD, so the Zel'dovich state at D is X = q + D psi,
V = psi).  Corner modes above the particle Nyquist wavenumber are zeroed
(default in the validation section's settings).

Conventions (the paper is silent on them; readings):
* forward DFT sum_j f_j exp(-2 pi i m.j / n), inverse with 1/n^3;
* delta_hat_m = w_hat_m sqrt(P(k_m) n^3 / L^3) with k_m = 2 pi m / L, so
  <|delta_hat|^2> L^3 / n^6 = P(k);
* psi_hat_c = i k_c delta_hat / (k^2 D_ref), D_ref = D(a=1) in D ~ a units, so
  that D(a) psi has the linear density of P at a = 1 scaled by D(a)/D_ref;
* zeroed: m = 0, the Nyquist plane of component c (the operator i k_c is odd
  and undefined there), and |m| > n/2;
* psi returned in lattice units dq = L / n_p.
"""
from __future__ import annotations

import math

import numpy as np


def ic_multipliers(n_p, box, spectrum, D_ref):
    """h_c on the [n][n][n/2+1] half spectrum, shape (3, n, n, n/2+1)."""
    n = n_p
    m = np.fft.fftfreq(n, 1.0 / n)
    mz = np.arange(n // 2 + 1, dtype=np.float64)
    mx, my, mzz = np.meshgrid(m, m, mz, indexing="ij")
    m2 = mx ** 2 + my ** 2 + mzz ** 2
    keep = (m2 > 0) & (4 * m2 <= n * n)
    kf = 2.0 * math.pi / box
    k2 = kf * kf * np.where(keep, m2, 1.0)
    k = np.sqrt(k2)
    amp = np.sqrt(spectrum(k) * n ** 3 / box ** 3)
    dq = box / n
    h = np.zeros((3,) + m2.shape, dtype=np.complex128)
    for c, mc in enumerate((mx, my, mzz)):
        ok = keep & (np.abs(mc) != n // 2)
        h[c] = np.where(ok, 1j * kf * mc / (k2 * D_ref) * amp / dq, 0.0)
    return h


def zeldovich_psi(w, box, spectrum, D_ref):
    """psi (3, N) in dq units from the real-space white noise w (n^3)."""
    w = np.asarray(w, dtype=np.float64)
    n = w.shape[0]
    wk = np.fft.rfftn(w)
    h = ic_multipliers(n, box, spectrum, D_ref)
    return np.stack([np.fft.irfftn(h[c] * wk, s=(n, n, n), axes=(0, 1, 2)).reshape(-1) for c in range(3)])
