"""Pins of the oracle's RNG and Zel'dovich initial conditions (CPU only)."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import cosmo, ics, philox


@pytest.mark.parametrize("ctr,key,expect", [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
])
def test_philox_known_answers(ctr, key, expect):
    # known-answer vectors published with Philox-4x32-10 (Salmon et al. 2011)
    out = philox.philox4x32_10(tuple([c] for c in ctr), key)
    assert tuple(int(o[0]) for o in out) == expect


def test_white_noise_statistics():
    w = philox.white_noise(54321, 100).astype(np.float64).ravel()  # 1e6 draws
    assert abs(w.mean()) < 5 / math.sqrt(w.size)
    assert abs(w.var() - 1) < 5 * math.sqrt(2 / w.size)
    assert stats.kstest(w, "norm").pvalue > 1e-3
    w2 = philox.white_noise(54322, 100).ravel()
    assert abs(np.corrcoef(w, w2)[0, 1]) < 5 / math.sqrt(w.size)


def test_single_mode_ic_is_analytic_plane_wave():
    n, box = 16, 100.0
    sp = cosmo.Spectrum("powerlaw", 3.0, k_c=1.0)
    m0 = np.array([1, 2, 3])
    q = np.indices((n, n, n)).reshape(3, -1)
    phase = 2 * np.pi * (m0 @ q) / n
    w = np.cos(phase).reshape(n, n, n)
    psi = ics.zeldovich_psi(w, box, sp, D_ref=0.8)
    kf = 2 * np.pi / box
    k = kf * np.linalg.norm(m0)
    a = math.sqrt(float(sp(k)) * n ** 3 / box ** 3) / (box / n)
    for c in range(3):
        expect = -kf * m0[c] * a / (k * k * 0.8) * np.sin(phase)
        assert np.allclose(psi[c], expect, atol=1e-12 * a)


def test_ic_is_real_and_linear_in_amplitude():
    n, box = 16, 64.0
    w = philox.white_noise(7, n)
    sp = cosmo.bbks_spectrum(0.31, 0.68, 0.965, 0.81)
    sp2 = cosmo.bbks_spectrum(0.31, 0.68, 0.965, 0.405)
    p1 = ics.zeldovich_psi(w, box, sp, 1.0)
    p2 = ics.zeldovich_psi(w, box, sp2, 1.0)
    assert np.allclose(p2, 0.5 * p1, rtol=1e-12, atol=1e-15)
    # zero-mean displacement (k = 0 removed)
    assert np.abs(p1.mean(axis=1)).max() < 1e-12


def test_powerlaw_normalisation_via_impulse_response():
    # E|D psi(q)|^2 over white noise = sum_q |psi_impulse(q)|^2 (translation
    # invariance): an FFT route independent of the mode sum in cosmo
    n_p, n_g, box, a0 = 16, 32, 50.0, 0.02
    sp = cosmo.powerlaw_spectrum(n_p, n_g, box, a0, 0.2)
    e0 = np.zeros((n_p,) * 3)
    e0[0, 0, 0] = 1.0
    psi = ics.zeldovich_psi(e0, box, sp, 1.0) * (box / n_p)   # Mpc/h
    rms = a0 * math.sqrt(np.sum(psi ** 2))
    assert abs(rms / (0.2 * box / n_g) - 1) < 1e-10


def test_kept_modes_exclude_nyquist_and_corners():
    n, box = 8, 10.0
    sp = cosmo.Spectrum("powerlaw", 1.0, k_c=100.0)
    h = ics.ic_multipliers(n, box, sp, 1.0)
    m = np.fft.fftfreq(n, 1.0 / n)
    assert np.all(h[0][n // 2] == 0) and np.all(h[1][:, n // 2] == 0) and np.all(h[2][:, :, n // 2] == 0)
    mx, my, mz = np.meshgrid(m, m, np.arange(n // 2 + 1), indexing="ij")
    corner = 4 * (mx ** 2 + my ** 2 + mz ** 2) > n * n
    assert np.all(h[:, corner] == 0)
    assert np.all(h[:, 0, 0, 0] == 0)
