"""Pins of the oracle's mass assignment, gather and fixed-point deposit
(CPU only)."""
import numpy as np
import pytest

from oracle import mesh


def _rand_psi(n_p, seed, scale=1.5):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, (3, n_p ** 3))


@pytest.mark.parametrize("order", [2, 3, 4])
def test_bspline_moments(order):
    # partition of unity, first moment = position, and the sampled second
    # moment of the B-spline (TSC: 1/4 for every position; CIC: f (1 - f))
    u = np.random.default_rng(0).uniform(0, 64, 2000)
    idx, w, _ = mesh.weights_1d(u, order)
    d = idx - u
    assert np.allclose(w.sum(0), 1.0, atol=1e-14)
    assert np.allclose((w * d).sum(0), 0.0, atol=1e-13)
    m2 = (w * d * d).sum(0)
    if order >= 3:
        # B-splines of order >= 3 sample their variance p/12 exactly
        assert np.allclose(m2, order / 12.0, atol=1e-13)
        if order == 4:
            assert np.allclose((w * d ** 3).sum(0), 0.0, atol=1e-12)
    else:
        f = u - np.floor(u)
        assert np.allclose(m2, f * (1 - f), atol=1e-13)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_scatter_gather_adjoint(order):
    # App. "Custom VJP and JVP": <scatter(w), rho> = <w, gather(rho)>
    n_p, n_g = 8, 16
    psi = _rand_psi(n_p, 1)
    rng = np.random.default_rng(2)
    wts = rng.normal(size=n_p ** 3)
    rho = rng.normal(size=n_g ** 3)
    lhs = np.dot(mesh.deposit(psi, n_p, n_g, order, weights=wts), rho)
    rhs = np.dot(wts, mesh.gather(rho, psi, n_p, n_g, order))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_gather_reproduces_linear_field(order):
    n_p, n_g = 8, 16
    psi = _rand_psi(n_p, 3, 0.3)
    u = mesh.mesh_coords(psi, n_p, n_g)
    # keep particles away from the periodic seam
    ok = np.all((u > 3) & (u < n_g - 3), axis=0)
    g = np.indices((n_g,) * 3).reshape(3, -1).astype(float)
    field = 0.3 * g[0] - 1.2 * g[1] + 0.7 * g[2] + 2.0
    v = mesh.gather(field, psi, n_p, n_g, order)
    exp = 0.3 * u[0] - 1.2 * u[1] + 0.7 * u[2] + 2.0
    assert np.allclose(v[ok], exp[ok], atol=1e-12)
    assert np.allclose(mesh.gather(np.full(n_g ** 3, 3.5), psi, n_p, n_g, order), 3.5)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_grad_gather_matches_finite_differences(order):
    n_p, n_g = 4, 8
    psi = _rand_psi(n_p, 4)
    field = np.random.default_rng(5).normal(size=n_g ** 3)
    g = mesh.grad_gather(field, psi, n_p, n_g, order)
    eps = 1e-7
    for a in range(3):
        dp = psi.copy()
        dp[a] += eps
        dm = psi.copy()
        dm[a] -= eps
        fd = (mesh.gather(field, dp, n_p, n_g, order) - mesh.gather(field, dm, n_p, n_g, order)) / (2 * eps)
        assert np.allclose(g[a], fd, atol=1e-6)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_fixedpoint_mass_and_float_agreement(order):
    n_p, n_g = 16, 32
    psi = _rand_psi(n_p, 6, 3.0).astype(np.float32)
    fx = mesh.deposit_fixedpoint(psi, n_p, n_g, order)
    assert fx.dtype == np.int64
    assert int(fx.sum()) == n_p ** 3 << 32           # every particle is 2^32
    fl = mesh.deposit(psi.astype(np.float64), n_p, n_g, order)
    # positions and 1D weights are quantised at 2^-20 of a mesh cell, so the
    # integer mesh matches the exact one to ~1e-6 relative
    assert np.abs(fx / 2.0 ** 32 - fl).max() < 1e-5
    assert np.linalg.norm(fx / 2.0 ** 32 - fl) / np.linalg.norm(fl) < 4e-6


@pytest.mark.parametrize("order", [2, 3, 4])
def test_fixedpoint_per_particle_weights_sum_exactly(order):
    n_p, n_g = 8, 16
    psi = _rand_psi(n_p, 7, 2.0).astype(np.float32)
    U = mesh.fixed_coords(psi, n_p, n_g)
    _, W3 = mesh.fixed_stencil_weights(U, order)
    assert np.all(W3.sum(axis=0) == 1 << 32)
    assert np.all(W3 >= 0)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_fixedpoint_boundary_cases(order):
    # exactly on mesh nodes, on CIC faces / TSC midpoints, and wrapping the box
    n_p, n_g = 4, 8
    N = n_p ** 3
    psi = np.zeros((3, N), np.float32)
    psi[0, 1] = 0.25          # half a mesh cell (r = 2): TSC midpoint
    psi[1, 2] = -0.5          # exactly one mesh node back
    psi[2, 3] = 4.0           # a full box length: wraps onto itself
    psi[0, 4] = -7.75         # wraps through 0
    psi[:, 5] = 0.499999970198  # just below a half cell in FP32
    fx = mesh.deposit_fixedpoint(psi, n_p, n_g, order)
    assert int(fx.sum()) == N << 32
    fl = mesh.deposit(psi.astype(np.float64), n_p, n_g, order)
    assert np.abs(fx / 2.0 ** 32 - fl).max() < 1e-6
    # a particle on a node deposits everything (CIC) on that node
    if order == 2:
        one = mesh.deposit_fixedpoint(np.zeros((3, N), np.float32), n_p, n_g, 2)
        lat = mesh.lattice(n_p) * 2
        lin = (lat[0] * n_g + lat[1]) * n_g + lat[2]
        assert np.all(one[lin] == 1 << 32) and one.sum() == N << 32


def test_fixedpoint_whole_cell_shift_permutes_mesh():
    n_p, n_g = 8, 16
    # displacements on a 2^-12 grid, so adding half a lattice unit (one mesh
    # cell, r = 2) is exact in FP32 and shifts U by exactly 2^B
    psi = (np.round(_rand_psi(n_p, 8, 1.0) * 4096) / 4096).astype(np.float32)
    a = mesh.deposit_fixedpoint(psi, n_p, n_g, 3).reshape(n_g, n_g, n_g)
    psi2 = psi.copy()
    psi2[1] += np.float32(0.5)
    b = mesh.deposit_fixedpoint(psi2, n_p, n_g, 3).reshape(n_g, n_g, n_g)
    assert np.array_equal(np.roll(a, 1, axis=1), b)
