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


def second_order_psi(psi1, n):
    """Second-order LPT displacement psi^(2) (3, N) in lattice units from the
    first-order field psi^(1) (3, N) on the n^3 lattice.

    Sec. "Lagrangian perturbation theory", eq. LPT_L at n = 2 (the only term
    is s = 1, with coefficient ((3-2)/2 - 1 - 1) / ((2 + 3/2)(2 - 1)) = -3/7;
    the mu_3 sum is empty), eq. LPT_T at n = 2 (its factor n - 2s vanishes, so
    T^(2) = 0), eq. LPT_kernels and eq. helmholtz:
      L2 = -(3/7) mu_2L^(1,1),  mu_2L = (1/2)(psi_i,i psi_j,j - psi_i,j psi_j,i),
      psi^(2) = Delta^-1 grad L2.
    Derivatives are the exact i k (k = 2 pi m / n per lattice spacing) and
    Delta^-1 is -1/k^2 (zero at k = 0).  The product mu is formed in real space
    on a grid of 3n/2 points per axis (Orszag's 3/2 rule) from the
    zero-padded spectra and cropped back to the modes |m_a| < n/2.
    Reading: the source field has every Nyquist plane zeroed (with the
    default corner-mode cut psi^(1) has none), and psi^(2) has none either.
    """
    psi1 = np.asarray(psi1, dtype=np.float64)
    assert n % 2 == 0
    P = np.stack([np.fft.fftn(psi1[c].reshape(n, n, n)) for c in range(3)])
    m = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    band = np.abs(m) < n // 2
    keep = band[:, None, None] & band[None, :, None] & band[None, None, :]
    P = P * keep
    k = 2.0 * np.pi * m / n
    kk = [k[:, None, None], k[None, :, None], k[None, None, :]]
    npad = 3 * n // 2
    idx = m[band] % npad

    def padded_real(spec):
        big = np.zeros((npad, npad, npad), dtype=np.complex128)
        big[np.ix_(idx, idx, idx)] = spec[np.ix_(band, band, band)]
        return np.fft.ifftn(big).real * (npad / n) ** 3

    g = [[padded_real(1j * kk[j] * P[i]) for j in range(3)] for i in range(3)]
    mu = np.zeros((npad, npad, npad))
    for i in range(3):
        for j in range(3):
            mu += 0.5 * (g[i][i] * g[j][j] - g[i][j] * g[j][i])
    mu_big = np.fft.fftn(mu) * (n / npad) ** 3
    mu_hat = np.zeros((n, n, n), dtype=np.complex128)
    mu_hat[np.ix_(band, band, band)] = mu_big[np.ix_(idx, idx, idx)]
    L2 = -3.0 / 7.0 * mu_hat
    k2 = kk[0] ** 2 + kk[1] ** 2 + kk[2] ** 2
    inv = np.where(k2 > 0, -1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    return np.stack([np.fft.ifftn(1j * kk[c] * inv * L2).real.reshape(-1) for c in range(3)])


def _second_order_parts(psi1, n):
    """The band-limited spectra of psi^(1), the derivative fields g_ij =
    d psi_i / d q_j on the padded grid, and the helpers of second_order_psi."""
    psi1 = np.asarray(psi1, dtype=np.float64)
    P = np.stack([np.fft.fftn(psi1[c].reshape(n, n, n)) for c in range(3)])
    m = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    band = np.abs(m) < n // 2
    keep = band[:, None, None] & band[None, :, None] & band[None, None, :]
    P = P * keep
    k = 2.0 * np.pi * m / n
    kk = [k[:, None, None], k[None, :, None], k[None, None, :]]
    npad = 3 * n // 2
    idx = m[band] % npad

    def padded_real(spec):
        big = np.zeros((npad, npad, npad), dtype=np.complex128)
        big[np.ix_(idx, idx, idx)] = spec[np.ix_(band, band, band)]
        return np.fft.ifftn(big).real * (npad / n) ** 3

    def crop(big):
        out = np.zeros((n, n, n), dtype=np.complex128)
        out[np.ix_(band, band, band)] = big[np.ix_(idx, idx, idx)]
        return out

    g = [[padded_real(1j * kk[j] * P[i]) for j in range(3)] for i in range(3)]
    k2 = kk[0] ** 2 + kk[1] ** 2 + kk[2] ** 2
    inv = np.where(k2 > 0, -1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    return g, kk, inv, band, idx, npad, crop


def second_order_psi_vjp(psi1, n, psi2_bar):
    """(d psi^(2) / d psi^(1))^T psi2_bar, shape (3, N): the transposes of
    second_order_psi's steps in reverse order.  With M_c = -(3/7) i k_c / -k^2
    the multiplier from mu to psi^(2)_c (odd and imaginary),
      mu_bar = ifft_pad(pad(sum_c conj(M_c) fft(psi2_bar_c))) (real),
    d mu / d g_ab = S delta_ab - g_ba (S the trace g_ii), and the transpose of
    psi1_i -> g_ij = padded_real(i k_j fft(psi1_i)) maps g_bar to
    ifft(-i k_j crop(fft_pad(g_bar))) (the (npad/n)^3 of padded_real and the
    1/npad^3 of its inverse transform cancel against the crop's unnormalised
    forward transform)."""
    g, kk, inv, band, idx, npad, crop = _second_order_parts(psi1, n)
    pb = np.asarray(psi2_bar, dtype=np.float64)
    keep = band[:, None, None] & band[None, :, None] & band[None, None, :]
    mbar = np.zeros((n, n, n), dtype=np.complex128)
    for c in range(3):
        Mc = 1j * kk[c] * inv * (-3.0 / 7.0)
        mbar += np.conj(Mc) * np.fft.fftn(pb[c].reshape(n, n, n))
    mbar *= keep
    big = np.zeros((npad, npad, npad), dtype=np.complex128)
    big[np.ix_(idx, idx, idx)] = mbar[np.ix_(band, band, band)]
    mu_bar = np.fft.ifftn(big).real
    S = g[0][0] + g[1][1] + g[2][2]
    out = np.zeros((3, n ** 3))
    for i in range(3):
        for j in range(3):
            gbar = mu_bar * ((S if i == j else 0.0) - g[j][i])
            out[i] += np.fft.ifftn(-1j * kk[j] * crop(np.fft.fftn(gbar))).real.reshape(-1)
    return out


def second_order_psi_jvp(psi1, n, psi1_dot):
    """d psi^(2) along psi1_dot: mu_dot = sum_ab (S delta_ab - g_ba) g_dot_ab
    through the same crop and multiplier as second_order_psi."""
    g, kk, inv, band, idx, npad, crop = _second_order_parts(psi1, n)
    gd, _, _, _, _, _, _ = _second_order_parts(psi1_dot, n)
    S = g[0][0] + g[1][1] + g[2][2]
    mu_dot = np.zeros((npad, npad, npad))
    for a in range(3):
        for b in range(3):
            mu_dot += ((S if a == b else 0.0) - g[b][a]) * gd[a][b]
    L2 = -3.0 / 7.0 * crop(np.fft.fftn(mu_dot)) * (n / npad) ** 3
    return np.stack([np.fft.ifftn(1j * kk[c] * inv * L2).real.reshape(-1) for c in range(3)])


def lpt_state(psi1, psi2, D):
    """Displacement and D-time velocity of the LPT series truncated at second
    order (eq. LPT, D^n approximation): Psi = D psi1 + D^2 psi2, V = dPsi/dD."""
    if psi2 is None:
        return D * psi1, psi1.copy()
    return D * psi1 + D * D * psi2, psi1 + 2.0 * D * psi2
