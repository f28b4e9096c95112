"""Binned power spectrum of a density-contrast mesh in FP64 (test
infrastructure only).

The paper names a (cross-)power-spectrum routine (Sec. "Miscellaneous
features") and measures final densities with deconvolved CIC (Sec. "Force
computation") without printing the estimator.  Reading:
  P(k_b) = (L^3 / n^6) sum_{m in b} w_m |delta_hat_m|^2 / W_CIC(m)^2 / sum w_m
with the half-spectrum multiplicity w_m (1 on the m_z = 0 and m_z = n/2
planes, 2 elsewhere), bin b >= 1 holding the modes with
(2b-1)^2 <= 4|m|^2 < (2b+1)^2 (an integer test without ties), m = 0
excluded; k_b = sum w |k| / sum w; no shot-noise subtraction.
"""
from __future__ import annotations

import math

import numpy as np

from .force import half_spectrum_theta, window_1d


def bin_index(m2):
    """b = ceil(isqrt(4 m^2) / 2) for integer |m|^2 (see module docstring)."""
    t = 4 * np.asarray(m2, dtype=np.int64)
    r = np.floor(np.sqrt(t.astype(np.float64))).astype(np.int64)
    r -= (r * r > t)                       # exact integer square root
    r += ((r + 1) * (r + 1) <= t)
    return (r + 1) // 2


def power_spectrum(delta, box, n_bins, deconvolve_cic=True):
    delta = np.asarray(delta, dtype=np.float64)
    n = round(delta.size ** (1 / 3))
    dk = np.fft.rfftn(delta.reshape(n, n, n))
    tx, ty, tz, (mx, my, mz) = half_spectrum_theta(n)
    p = np.abs(dk) ** 2
    if deconvolve_cic:
        W = window_1d(tx, 2) * window_1d(ty, 2) * window_1d(tz, 2)
        p = p / (W * W)
    wm = np.where((mz == 0) | (mz == n // 2), 1.0, 2.0)
    m2 = (mx ** 2 + my ** 2 + mz ** 2).astype(np.int64)
    b = bin_index(m2)
    kmag = 2 * math.pi / box * np.sqrt(m2)
    sel = (m2 > 0) & (b <= n_bins)
    bb = b[sel] - 1
    cnt = np.bincount(bb, weights=wm[sel], minlength=n_bins)
    ps = np.bincount(bb, weights=(wm * p)[sel], minlength=n_bins)
    ks = np.bincount(bb, weights=(wm * kmag)[sel], minlength=n_bins)
    with np.errstate(invalid="ignore", divide="ignore"):
        pk = box ** 3 / float(n) ** 6 * ps / cnt
        kb = ks / cnt
    return kb, pk, cnt.astype(np.int64)
