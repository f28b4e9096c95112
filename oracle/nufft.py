"""Non-uniform FFT force in FP64 (test infrastructure only).

Follows Sec. "Force evaluation" (paragraphs on the NUFFT density, the
deconvolution and the NUFFT interpolation) and eq. NUDFTII:
  F_m     = sum_i exp(-2 pi i m.X_i / L)                 (type 1, unit masses)
  delta_m = (n_p^3 / N) F_m for m != 0, 0 at m = 0
  g_c,m   = i k_c / k^2 s delta_m                         (exact i k gradient)
  A_i,c   = (1/n_p^3) sum_m g_c,m exp(+2 pi i m.X_i / L)  (type 2)
with m restricted to the particle reciprocal lattice strictly below the
particle Nyquist mode, |m_a| < n_p/2 per axis.

Readings (the paper prints no kernel formula and writes the sums over
{0..N_d-1}^3, which is read as the centred set above):
* "exponential of semicircle" kernel phi(z) = exp(beta (sqrt(1 - z^2) - 1)) for
  |z| < 1, 0 otherwise, with z = x / (w/2) for a fine-grid offset x in cells
  (Barnett, Magland & af Klinteberg 2019); width w = 6, beta = 2.3 w, upsampling
  sigma = n_f / n_p = 2;
* phi_hat(theta) = int phi(x) cos(theta x) dx by Gauss-Legendre quadrature;
* spreading: b_j = sum_i phi(j - u_i) on the periodic n_f^3 grid with
  u = (q + Psi) sigma in fine cells, F_m ~ DFT(b)_m / phi_hat(theta_m);
  interpolation: A_i = (1/n_p^3) sum_j c_j phi(u_i - j) with
  c = n_f^3 IDFT(zero-padded g / phi_hat).

Fixed-point ES spreading (the bit pattern the GPU reproduces): the 1D weight
of a node at fixed-point distance d (B = 20 fraction bits) is integer linear
interpolation in a table T[t] = rne(phi(t / 4096) 2^20), t = 0 .. 3*4096,
  w = T[i] + floor(((T[i+1] - T[i]) f + 128) / 256),  i = d >> 8, f = d & 255,
and the 3D weight of node (x, y, z) is formed in two truncating steps,
  A_xy = floor(w_x w_y / 2^17),  m_xyz = floor(A_xy w_z / 2^12),
so that A_xy < 2^24 and m_xyz <= 2^31: the unit is 2^31 at the kernel's peak
phi(0)^3, and each node costs two 24-bit products.  There is no remainder
step (the ES kernel is not a partition of unity); the truncations bias each
node by less than 2^-23 of the peak, far below FP32 resolution of the sums.
"""
from __future__ import annotations

import math

import numpy as np

from . import mesh

TAB_PER_CELL = 4096
K_ES = 20
ES_UNIT = 2.0 ** 31        # fixed-point value of phi(0)^3


def es_phi(z, beta):
    z = np.asarray(z, dtype=np.float64)
    inside = np.abs(z) < 1.0
    return np.where(inside, np.exp(beta * (np.sqrt(np.clip(1.0 - z * z, 0.0, None)) - 1.0)), 0.0)


def es_kernel(x, width, beta):
    """phi at a fine-grid offset x (cells)."""
    return es_phi(np.asarray(x, dtype=np.float64) / (width / 2.0), beta)


def es_phihat(theta, width, beta, n_quad=400):
    """int_{-w/2}^{w/2} phi(x) cos(theta x) dx."""
    t, wq = np.polynomial.legendre.leggauss(n_quad)
    half = width / 2.0
    x = half * t
    fx = es_kernel(x, width, beta) * wq * half
    theta = np.asarray(theta, dtype=np.float64)
    return np.cos(np.multiply.outer(theta, x)) @ fx


def kept_modes(n_p):
    """Centred modes strictly below the particle Nyquist mode."""
    return np.arange(-(n_p // 2) + 1, n_p // 2)


def fine_coords(psi, n_p, n_f):
    return mesh.mesh_coords(psi, n_p, n_f)


def _force_multiplier(mx, my, mz, n_p, s):
    """i k_c s / k^2 in lattice units (k = 2 pi m / n_p), zero at m = 0."""
    k = [2 * np.pi * m / n_p for m in (mx, my, mz)]
    k2 = k[0] ** 2 + k[1] ** 2 + k[2] ** 2
    zero = k2 == 0
    k2s = np.where(zero, 1.0, k2)
    return [np.where(zero, 0.0, 1j * kc * s / k2s) for kc in k]


def nudft_force_direct(n_p, n_f, psi, s):
    """Brute-force type-1 and type-2 sums, O(N n_p^3); tiny inputs only."""
    u = fine_coords(psi, n_p, n_f)
    ms = kept_modes(n_p)
    mx, my, mz = np.meshgrid(ms, ms, ms, indexing="ij")
    mx, my, mz = mx.reshape(-1), my.reshape(-1), mz.reshape(-1)
    phase = 2 * np.pi / n_f * (np.outer(mx, u[0]) + np.outer(my, u[1]) + np.outer(mz, u[2]))
    E = np.exp(-1j * phase)                   # (M, N)
    F = E.sum(axis=1)
    N = psi.shape[1]
    delta = F * (n_p ** 3 / N)
    K = _force_multiplier(mx, my, mz, n_p, s)
    A = np.stack([np.real((K[c] * delta) @ np.conj(E)) for c in range(3)]) / n_p ** 3
    return A


def es_kernel_deriv(x, width, beta):
    """d phi / dx at a fine-grid offset x (cells), inside the support; the
    jump of phi at |z| = 1 (of size exp(-beta)) carries no derivative."""
    half = width / 2.0
    z = np.asarray(x, dtype=np.float64) / half
    inside = np.abs(z) < 1.0
    root = np.sqrt(np.clip(1.0 - z * z, 1e-300, None))
    return np.where(inside, es_phi(z, beta) * beta * (-z / root) / half, 0.0)


def _es_axis_weights(u, width, beta):
    """First node floor(u) - w/2 + 1 and the w kernel values per axis."""
    base = np.floor(u).astype(np.int64) - (width // 2 - 1)
    wts = [np.stack([es_kernel(base[a] + o - u[a], width, beta) for o in range(width)])
           for a in range(3)]
    return base, wts


def _spread_float(u, n_f, width, beta, weights=None):
    """b_j = sum_i w_i phi(j - u_i) on the periodic n_f^3 grid (FP64); the
    stencil is the w nodes floor(u) - w/2 + 1 .. floor(u) + w/2 (even w)."""
    assert width % 2 == 0
    N = u.shape[1]
    w_i = np.ones(N) if weights is None else weights
    base, wts = _es_axis_weights(u, width, beta)
    out = np.zeros(n_f ** 3)
    for a in range(width):
        ix = (base[0] + a) % n_f
        idx, val = [], []
        for b in range(width):
            iy = (base[1] + b) % n_f
            wab = wts[0][a] * wts[1][b] * w_i
            for c in range(width):
                iz = (base[2] + c) % n_f
                idx.append((ix * n_f + iy) * n_f + iz)
                val.append(wab * wts[2][c])
        # one accumulation per x offset (same sum, fewer passes over the grid)
        out += np.bincount(np.concatenate(idx), weights=np.concatenate(val), minlength=n_f ** 3)
    return out


def _interp_float(field, u, n_f, width, beta):
    """v_i = sum_j field_j phi(u_i - j); field may carry trailing components."""
    f = field.reshape(n_f ** 3, -1)
    base, wts = _es_axis_weights(u, width, beta)
    v = np.zeros((u.shape[1], f.shape[1]))
    for a in range(width):
        ix = (base[0] + a) % n_f
        for b in range(width):
            iy = (base[1] + b) % n_f
            wab = wts[0][a] * wts[1][b]
            for c in range(width):
                iz = (base[2] + c) % n_f
                v += f[(ix * n_f + iy) * n_f + iz] * (wab * wts[2][c])[:, None]
    return v


def _interp_grad(field, u, n_f, width, beta):
    """d/du_i of sum_j field_j phi(u_i - j): shape (N, components, 3)."""
    f = field.reshape(n_f ** 3, -1)
    base = np.floor(u).astype(np.int64) - (width // 2 - 1)
    w = [np.stack([es_kernel(base[a] + o - u[a], width, beta) for o in range(width)]) for a in range(3)]
    # d/du phi(u - j) = phi'(u - j): offsets are u - node
    d = [np.stack([es_kernel_deriv(u[a] - (base[a] + o), width, beta) for o in range(width)])
         for a in range(3)]
    g = np.zeros((u.shape[1], f.shape[1], 3))
    for a in range(width):
        ix = (base[0] + a) % n_f
        for b in range(width):
            iy = (base[1] + b) % n_f
            for c in range(width):
                iz = (base[2] + c) % n_f
                fv = f[(ix * n_f + iy) * n_f + iz]
                g[:, :, 0] += fv * (d[0][a] * w[1][b] * w[2][c])[:, None]
                g[:, :, 1] += fv * (w[0][a] * d[1][b] * w[2][c])[:, None]
                g[:, :, 2] += fv * (w[0][a] * w[1][b] * d[2][c])[:, None]
    return g


def _nufft_pieces(n_p, n_f, N, s, width, beta):
    """Kept-mode index sets and the multipliers of the map b -> c_c:
    c_c = n_f^3 IDFT(pad(D_c restrict(DFT(b)))), D_c = K_c (n_p^3/N) / Phi^2,
    Phi = phi_hat(mx) phi_hat(my) phi_hat(mz)."""
    ms = kept_modes(n_p)
    mz = np.arange(0, n_p // 2)
    ix = ms % n_f
    ph = lambda m: es_phihat(2 * np.pi * m / n_f, width, beta)
    Phi = ph(ms)[:, None, None] * ph(ms)[None, :, None] * ph(mz)[None, None, :]
    MX, MY, MZ = np.meshgrid(ms, ms, mz, indexing="ij")
    K = _force_multiplier(MX, MY, MZ, n_p, s)
    D = [K[c] * (n_p ** 3 / N) / Phi ** 2 for c in range(3)]
    return ix, mz, D


def nufft_force_vjp(n_p, n_f, psi, s, v, width=6, beta=13.8, parts=3):
    """J_A(Psi)^T v for the spreading NUFFT force of ``nufft_force``; v (3, N).

    A_c(u_i) = (1/n_p^3) sum_j c_c,j phi(u_i - j), c_c = G_c b, b = spread(u),
    u = (q + Psi) sigma.  Two parts (App. "Custom VJP and JVP"): the
    interpolation differentiated w.r.t. the positions, and the transposed mesh
    path G_c^T = n_f^3 IDFT(pad(conj(D_c) restrict(DFT(.)))) applied to the
    spread of v_c / n_p^3, whose result is gathered with grad phi (the
    spreading differentiated w.r.t. the positions).  parts: 1 the first
    term only, 2 the second only, 3 both."""
    u = fine_coords(psi, n_p, n_f)
    N = u.shape[1]
    sig = n_f / n_p
    b = _spread_float(u, n_f, width, beta).reshape(n_f, n_f, n_f)
    bk = np.fft.rfftn(b)
    ix, mz, D = _nufft_pieces(n_p, n_f, N, s, width, beta)
    sub = bk[np.ix_(ix, ix, mz)]
    meshes = []
    for c in range(3):
        full = np.zeros((n_f, n_f, n_f // 2 + 1), dtype=np.complex128)
        full[np.ix_(ix, ix, mz)] = D[c] * sub
        meshes.append(np.fft.irfftn(full, s=(n_f, n_f, n_f), axes=(0, 1, 2)).reshape(-1) * n_f ** 3)
    # direct part
    g = _interp_grad(np.stack(meshes, axis=1), u, n_f, width, beta) / n_p ** 3   # (N, 3, 3)
    xbar = np.einsum("ci,icd->di", v, g) if parts & 1 else np.zeros((3, N))
    if not parts & 2:
        return xbar * sig
    # mesh part
    acc = np.zeros((len(ix), len(ix), len(mz)), dtype=np.complex128)
    for c in range(3):
        cbar = _spread_float(u, n_f, width, beta, weights=v[c] / n_p ** 3).reshape(n_f, n_f, n_f)
        acc += np.conj(D[c]) * np.fft.rfftn(cbar)[np.ix_(ix, ix, mz)]
    full = np.zeros((n_f, n_f, n_f // 2 + 1), dtype=np.complex128)
    full[np.ix_(ix, ix, mz)] = acc
    bbar = np.fft.irfftn(full, s=(n_f, n_f, n_f), axes=(0, 1, 2)).reshape(-1) * n_f ** 3
    xbar += _interp_grad(bbar[:, None], u, n_f, width, beta)[:, 0, :].T
    return xbar * sig


def _spread_grad(u, n_f, width, beta, t):
    """b_dot_j = sum_i t_i . d/du_i phi(j - u_i) = sum_i t_i . grad phi(u_i - j):
    the spread's tangent when the positions u (3, M) move along t (3, M)."""
    base = np.floor(u).astype(np.int64) - (width // 2 - 1)
    w = [np.stack([es_kernel(base[a] + o - u[a], width, beta) for o in range(width)]) for a in range(3)]
    d = [np.stack([es_kernel_deriv(u[a] - (base[a] + o), width, beta) for o in range(width)])
         for a in range(3)]
    out = np.zeros(n_f ** 3)
    for a in range(width):
        ix = (base[0] + a) % n_f
        for b in range(width):
            iy = (base[1] + b) % n_f
            for c in range(width):
                iz = (base[2] + c) % n_f
                v = (t[0] * d[0][a] * w[1][b] * w[2][c] + t[1] * w[0][a] * d[1][b] * w[2][c]
                     + t[2] * w[0][a] * w[1][b] * d[2][c])
                out += np.bincount((ix * n_f + iy) * n_f + iz, weights=v, minlength=n_f ** 3)
    return out


def nufft_force_jvp(n_p, n_f, psi, s, xdot, width=6, beta=13.8):
    """J_A(Psi) xdot for the spreading NUFFT force of ``nufft_force``; xdot
    (3, N) in dq units.  The JVP rules of App. "Custom VJP and JVP": the
    spread's tangent is a spread with grad phi dotted with the tangent
    positions, carried through the same linear map to tangent meshes and
    interpolated; the interpolation's own tangent is its gradient dotted
    with the tangent positions."""
    u = fine_coords(psi, n_p, n_f)
    N = u.shape[1]
    t = (n_f / n_p) * np.asarray(xdot, dtype=np.float64)
    ix, mz, D = _nufft_pieces(n_p, n_f, N, s, width, beta)

    def meshes_of(b):
        sub = np.fft.rfftn(b.reshape(n_f, n_f, n_f))[np.ix_(ix, ix, mz)]
        out = []
        for c in range(3):
            full = np.zeros((n_f, n_f, n_f // 2 + 1), dtype=np.complex128)
            full[np.ix_(ix, ix, mz)] = D[c] * sub
            out.append(np.fft.irfftn(full, s=(n_f, n_f, n_f), axes=(0, 1, 2)).reshape(-1) * n_f ** 3)
        return np.stack(out, axis=1)

    g = _interp_grad(meshes_of(_spread_float(u, n_f, width, beta)), u, n_f, width, beta)   # (N, 3, 3)
    direct = np.einsum("icd,di->ci", g, t)
    through = _interp_float(meshes_of(_spread_grad(u, n_f, width, beta, t)), u, n_f, width, beta).T
    return (direct + through) / n_p ** 3


def nufft_force(n_p, n_f, psi, s, width=6, beta=13.8):
    """Spreading-based NUFFT force A(X) (3, N) in dq units per unit D."""
    u = fine_coords(psi, n_p, n_f)
    N = u.shape[1]
    b = _spread_float(u, n_f, width, beta).reshape(n_f, n_f, n_f)
    bk = np.fft.rfftn(b)
    ms = kept_modes(n_p)
    mz = np.arange(0, n_p // 2)
    ix = ms % n_f
    ph = lambda m: es_phihat(2 * np.pi * m / n_f, width, beta)
    sub = bk[np.ix_(ix, ix, mz)] / (ph(ms)[:, None, None] * ph(ms)[None, :, None]
                                    * ph(mz)[None, None, :])
    delta = sub * (n_p ** 3 / N)
    MX, MY, MZ = np.meshgrid(ms, ms, mz, indexing="ij")
    K = _force_multiplier(MX, MY, MZ, n_p, s)
    meshes = []
    for c in range(3):
        g = K[c] * delta / (ph(ms)[:, None, None] * ph(ms)[None, :, None] * ph(mz)[None, None, :])
        full = np.zeros((n_f, n_f, n_f // 2 + 1), dtype=np.complex128)
        full[np.ix_(ix, ix, mz)] = g
        meshes.append(np.fft.irfftn(full, s=(n_f, n_f, n_f), axes=(0, 1, 2)).reshape(-1) * n_f ** 3)
    # interpolate the three components together
    return _interp_float(np.stack(meshes, axis=1), u, n_f, width, beta).T / n_p ** 3


# --------------------------------------------------------------------------
# Fixed-point specification of the ES spreading
# --------------------------------------------------------------------------

def es_table(width=6, beta=13.8):
    t = np.arange((width // 2) * TAB_PER_CELL + 2, dtype=np.float64) / TAB_PER_CELL
    return np.rint(es_kernel(t, width, beta) * 2.0 ** K_ES).astype(np.int64)


def es_fixed_weight(dist_fixed, table):
    """Integer 1D weight for a non-negative fixed-point distance (B = 20)."""
    shift = mesh.B_FRAC - int(math.log2(TAB_PER_CELL))       # 8
    i = dist_fixed >> shift
    f = dist_fixed & ((1 << shift) - 1)
    ok = i < table.size - 1
    ic = np.where(ok, i, 0)
    t0, t1 = table[ic], table[ic + 1]
    w = t0 + (((t1 - t0) * f + (1 << (shift - 1))) >> shift)
    return np.where(ok, w, 0)


def es_fixed_stencil(U, n_f, width=6, beta=13.8):
    """Nodes and integer 3D weights (2^31 at the kernel's peak, two
    truncating steps) of the fixed-point ES spreading for fixed-point
    coordinates U (3, n): yields (flat node index, weight) per stencil point,
    width^3 of them."""
    table = es_table(width, beta)
    one = 1 << mesh.B_FRAC
    base = (U >> mesh.B_FRAC) - (width // 2 - 1)
    W = []
    for a in range(3):
        rows = []
        for o in range(width):
            d = np.abs(((base[a] + o) << mesh.B_FRAC) - U[a])
            # strictly inside the support: |z| < 1
            rows.append(np.where(d < (width // 2) * one, es_fixed_weight(d, table), 0))
        W.append(np.stack(rows))
    for a in range(width):
        ix = (base[0] + a) % n_f
        for b in range(width):
            iy = (base[1] + b) % n_f
            A = (W[0][a] * W[1][b]) >> 17
            for c in range(width):
                iz = (base[2] + c) % n_f
                yield (ix * n_f + iy) * n_f + iz, (A * W[2][c]) >> 12


def deposit_fixedpoint_es(psi_f32, n_p, n_f, width=6, beta=13.8):
    """Integer ES spreading onto n_f^3 (flat int64) from FP32 Psi."""
    U = mesh.fixed_coords(psi_f32, n_p, n_f)
    out = np.zeros(n_f ** 3, dtype=np.int64)
    for lin, w3 in es_fixed_stencil(U, n_f, width, beta):
        hi = w3 >> 17
        lo = w3 - (hi << 17)
        out += np.rint(np.bincount(lin, weights=hi, minlength=n_f ** 3)).astype(np.int64) << 17
        out += np.rint(np.bincount(lin, weights=lo, minlength=n_f ** 3)).astype(np.int64)
    return out
