"""Pins of the oracle's NUFFT force VJP (App. "Custom VJP and JVP" applied to
the spreading NUFFT of Sec. "Force evaluation"): central finite differences
of the oracle's own forward force, of the brute-force NUDFT sums, and of the
whole loss through a BullFrog run."""
import numpy as np
import pytest

import synth
from oracle import adjoint, nufft, philox
from oracle.nbody import initial_state, run_from


def test_es_kernel_derivative_is_the_slope_of_the_kernel():
    x = np.linspace(-2.95, 2.95, 119)
    h = 1e-6
    fd = (nufft.es_kernel(x + h, 6, 13.8) - nufft.es_kernel(x - h, 6, 13.8)) / (2 * h)
    assert np.max(np.abs(fd - nufft.es_kernel_deriv(x, 6, 13.8))) < 1e-8
    # even kernel, odd slope; zero outside the support
    assert np.allclose(nufft.es_kernel_deriv(-x, 6, 13.8), -nufft.es_kernel_deriv(x, 6, 13.8))
    assert np.all(nufft.es_kernel_deriv(np.array([3.0, 3.5, -4.0]), 6, 13.8) == 0)


@pytest.mark.parametrize("seed", [4, 5])
def test_nufft_vjp_matches_fd_of_the_spreading_force(seed):
    rng = np.random.default_rng(seed)
    n_p, n_f = 4, 8
    N = n_p ** 3
    psi = rng.normal(0, 0.7, (3, N))
    v, d = rng.normal(size=(3, N)), rng.normal(size=(3, N))
    xb = nufft.nufft_force_vjp(n_p, n_f, psi, 0.8, v)
    eps = 1e-5
    fd = np.sum(v * (nufft.nufft_force(n_p, n_f, psi + eps * d, 0.8)
                     - nufft.nufft_force(n_p, n_f, psi - eps * d, 0.8))) / (2 * eps)
    assert abs(fd / np.sum(xb * d) - 1) < 1e-6


def test_nufft_vjp_matches_fd_of_the_direct_nudft():
    """The spreading NUFFT approximates the direct sums of eq. NUDFTII to the
    ES kernel's accuracy; so do their derivatives."""
    rng = np.random.default_rng(6)
    n_p, n_f = 4, 8
    N = n_p ** 3
    psi = rng.normal(0, 0.7, (3, N))
    v, d = rng.normal(size=(3, N)), rng.normal(size=(3, N))
    xb = nufft.nufft_force_vjp(n_p, n_f, psi, 0.8, v)
    eps = 1e-5
    fd = np.sum(v * (nufft.nudft_force_direct(n_p, n_f, psi + eps * d, 0.8)
                     - nufft.nudft_force_direct(n_p, n_f, psi - eps * d, 0.8))) / (2 * eps)
    assert abs(fd / np.sum(xb * d) - 1) < 1e-4


def test_nufft_vjp_is_linear_in_the_cotangent():
    rng = np.random.default_rng(7)
    n_p, n_f = 4, 8
    psi = rng.normal(0, 0.5, (3, 64))
    v1, v2 = rng.normal(size=(3, 64)), rng.normal(size=(3, 64))
    a = nufft.nufft_force_vjp(n_p, n_f, psi, 1.3, 2 * v1 - 3 * v2)
    b = 2 * nufft.nufft_force_vjp(n_p, n_f, psi, 1.3, v1) - 3 * nufft.nufft_force_vjp(n_p, n_f, psi, 1.3, v2)
    assert np.allclose(a, b, rtol=1e-10, atol=1e-12)


def test_nufft_gradient_matches_fd_of_the_loss():
    """dL/dw of the L2 loss on the final CIC density through 2 BullFrog steps
    with the NUFFT force, against a central difference of the loss."""
    rng = np.random.default_rng(4)
    prob = synth.oracle_problem(dict(synth.C3_SMALL, n_p=4, n_g=8, box=7.8125, n_steps=2))
    w = philox.white_noise(synth.SEED_W, 4).astype(np.float64)
    target = rng.normal(size=8 ** 3)
    wb, _, _ = adjoint.gradient(prob, w, lambda dl: 2 * (dl - target))
    dw = rng.normal(size=w.shape)

    def loss(ww):
        p0, v0, _ = initial_state(prob, ww)
        pN, _ = run_from(prob, p0, v0)
        return float(np.sum((adjoint.final_density(prob, pN) - target) ** 2))

    eps = 1e-5
    fd = (loss(w + eps * dw) - loss(w - eps * dw)) / (2 * eps)
    assert abs(fd / np.dot(wb.reshape(-1), dw.reshape(-1)) - 1) < 1e-7


def test_vjp_parts_add_up():
    """The direct and mesh terms of both force VJPs sum to the whole VJP."""
    from oracle import adjoint as oadj
    from oracle.force import PMConfig
    rng = np.random.default_rng(8)
    psi, v = rng.normal(0, 0.6, (3, 64)), rng.normal(size=(3, 64))
    whole = nufft.nufft_force_vjp(4, 8, psi, 1.1, v)
    split = nufft.nufft_force_vjp(4, 8, psi, 1.1, v, parts=1) + nufft.nufft_force_vjp(4, 8, psi, 1.1, v, parts=2)
    assert np.allclose(whole, split, rtol=1e-12, atol=1e-14)
    cfg = PMConfig(4, 8, 10.0, order=3, deconvolve=True, grad_order=4, lap_order=0)
    whole = oadj.force_vjp(cfg, psi, 1.1, v)
    split = oadj.force_vjp(cfg, psi, 1.1, v, parts=1) + oadj.force_vjp(cfg, psi, 1.1, v, parts=2)
    assert np.allclose(whole, split, rtol=1e-12, atol=1e-14)
