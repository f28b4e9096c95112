"""Mass assignment (scatter), interpolation (gather) and their position
derivatives, in FP64, plus the integer fixed-point deposit specification.

Test infrastructure only.  Follows tab. interpolation_kernels (CIC, TSC and
PCS 1D kernels, 3D kernel = product over axes) and App. "Custom VJP and JVP" (scatter
rho_j = sum_i w_i W_j(X_i); gather v_i = sum_j rho_j W_j(X_i); position
derivatives through grad W).

Geometry (the paper leaves it open; this is the reading used throughout):
particle i has lattice index (jx, jy, jz) (row-major, z fastest) on an n_p^3
lattice of spacing dq = L/n_p, and displacement Psi in units of dq.  The mesh
has n_g^3 nodes at integer mesh coordinates; with r = n_g/n_p the particle
sits at mesh coordinate u = (j + Psi) r, periodic in n_g.

Fixed-point deposit (the bit pattern the GPU must reproduce from identical
FP32 inputs): B = 20 fraction bits of position, 1D weights at K = 20 bits
(summing to 2^K exactly per axis), 3D product rounded half-to-even to a mass
unit of 2^M = 2^32 per particle, and the rounding remainder added to the
stencil point with the largest exact product (first in stencil order on
ties).  Every particle therefore deposits exactly 2^32.
"""
from __future__ import annotations

import numpy as np

B_FRAC = 20
K_W = 20
M_MASS = 32


def lattice(n_p):
    j = np.arange(n_p ** 3, dtype=np.int64)
    return np.stack([j // (n_p * n_p), (j // n_p) % n_p, j % n_p])


def mesh_coords(psi, n_p, n_g):
    """u = (j + Psi) r mod n_g, FP64, shape (3, N)."""
    r = n_g // n_p
    return np.mod((lattice(n_p) + np.asarray(psi, dtype=np.float64)) * r, n_g)


def weights_1d(u, order):
    """1D kernel nodes, weights and dW/du for mesh coordinate u.

    CIC (order 2): nodes floor(u), floor(u)+1 with weights 1-f, f.
    TSC (order 3): n = floor(u + 1/2), x = u - n, nodes n-1, n, n+1 with
    weights (1/2)(1/2 - x)^2, 3/4 - x^2, (1/2)(1/2 + x)^2.
    PCS (order 4): nodes floor(u)-1 .. floor(u)+2 with the cubic B-spline.
    """
    if order == 2:
        i0 = np.floor(u)
        f = u - i0
        i0 = i0.astype(np.int64)
        return (np.stack([i0, i0 + 1]), np.stack([1.0 - f, f]),
                np.stack([-np.ones_like(f), np.ones_like(f)]))
    if order == 3:
        n = np.floor(u + 0.5)
        x = u - n
        n = n.astype(np.int64)
        return (np.stack([n - 1, n, n + 1]),
                np.stack([0.5 * (0.5 - x) ** 2, 0.75 - x * x, 0.5 * (0.5 + x) ** 2]),
                np.stack([-(0.5 - x), -2.0 * x, 0.5 + x]))
    if order == 4:
        i0 = np.floor(u)
        f = u - i0
        g = 1.0 - f
        i0 = i0.astype(np.int64)
        # PCS: W(x) = (4 - 6x^2 + 3|x|^3)/6 for |x| <= 1, (2 - |x|)^3/6 for
        # 1 <= |x| <= 2, at node distances 1+f, f, 1-f, 2-f
        return (np.stack([i0 - 1, i0, i0 + 1, i0 + 2]),
                np.stack([g ** 3 / 6.0, (4.0 - 6.0 * f * f + 3.0 * f ** 3) / 6.0,
                          (4.0 - 6.0 * g * g + 3.0 * g ** 3) / 6.0, f ** 3 / 6.0]),
                np.stack([-0.5 * g * g, -2.0 * f + 1.5 * f * f, 2.0 * g - 1.5 * g * g, 0.5 * f * f]))
    raise ValueError("order must be 2 (CIC), 3 (TSC) or 4 (PCS)")


def _stencil(psi, n_p, n_g, order):
    u = mesh_coords(psi, n_p, n_g)
    return [weights_1d(u[a], order) for a in range(3)]


def _loop(st, n_g, order):
    """Yield (flat mesh index, (wx, wy, wz), (dx, dy, dz)) per stencil point."""
    for a in range(order):
        for b in range(order):
            for c in range(order):
                idx = ((st[0][0][a] % n_g) * n_g + st[1][0][b] % n_g) * n_g + st[2][0][c] % n_g
                yield (idx, (st[0][1][a], st[1][1][b], st[2][1][c]),
                       (st[0][2][a], st[1][2][b], st[2][2][c]))


def deposit_u(u, n_g, order, weights=None):
    """rho_j = sum_i w_i W_j(u_i) for mesh coordinates u (3, M)."""
    st = [weights_1d(np.asarray(u[a], dtype=np.float64), order) for a in range(3)]
    M = np.asarray(u).shape[1]
    w_i = np.ones(M) if weights is None else np.asarray(weights, dtype=np.float64)
    out = np.zeros(n_g ** 3)
    for idx, (wx, wy, wz), _ in _loop(st, n_g, order):
        out += np.bincount(idx, weights=wx * wy * wz * w_i, minlength=n_g ** 3)
    return out


def gather_u(field, u, n_g, order):
    """v_i = sum_j field_j W_j(u_i)."""
    st = [weights_1d(np.asarray(u[a], dtype=np.float64), order) for a in range(3)]
    f = np.asarray(field, dtype=np.float64).reshape(-1)
    v = np.zeros(np.asarray(u).shape[1])
    for idx, (wx, wy, wz), _ in _loop(st, n_g, order):
        v += f[idx] * wx * wy * wz
    return v


def grad_gather_u(field, u, n_g, order):
    """d/du_i of sum_j field_j W_j(u_i) in mesh units, shape (3, M)."""
    st = [weights_1d(np.asarray(u[a], dtype=np.float64), order) for a in range(3)]
    f = np.asarray(field, dtype=np.float64).reshape(-1)
    g = np.zeros((3, np.asarray(u).shape[1]))
    for idx, (wx, wy, wz), (dx, dy, dz) in _loop(st, n_g, order):
        fv = f[idx]
        g[0] += fv * dx * wy * wz
        g[1] += fv * wx * dy * wz
        g[2] += fv * wx * wy * dz
    return g


def deposit(psi, n_p, n_g, order, weights=None):
    """rho_j = sum_i w_i W_j(X_i) on the n_g^3 mesh (flat, FP64)."""
    return deposit_u(mesh_coords(psi, n_p, n_g), n_g, order, weights)


def gather(field, psi, n_p, n_g, order):
    """v_i = sum_j field_j W_j(X_i)."""
    return gather_u(field, mesh_coords(psi, n_p, n_g), n_g, order)


def grad_gather(field, psi, n_p, n_g, order):
    """d/dPsi_i of sum_j field_j W_j(X_i), shape (3, N), Psi in dq units
    (so the chain rule brings a factor r = n_g / n_p)."""
    st = _stencil(psi, n_p, n_g, order)
    r = n_g // n_p
    f = np.asarray(field, dtype=np.float64).reshape(-1)
    g = np.zeros((3, n_p ** 3))
    for idx, (wx, wy, wz), (dx, dy, dz) in _loop(st, n_g, order):
        fv = f[idx]
        g[0] += fv * dx * wy * wz
        g[1] += fv * wx * dy * wz
        g[2] += fv * wx * wy * dz
    return g * r


def contrast(mass, N, n_g):
    """delta_j = m_j n_g^3 / N - 1 (unit particle masses; its mean is zero)."""
    return np.asarray(mass, dtype=np.float64) * (n_g ** 3 / N) - 1.0


# --------------------------------------------------------------------------
# Fixed-point specification
# --------------------------------------------------------------------------

def _rne_shift(p, s):
    """Round-half-to-even of p / 2^s for non-negative int64 p."""
    p = np.asarray(p, dtype=np.int64)
    q = p >> s
    rem = p & ((1 << s) - 1)
    half = 1 << (s - 1)
    up = (rem > half) | ((rem == half) & ((q & 1) == 1))
    return q + up.astype(np.int64)


def fixed_coords(psi_f32, n_p, n_g):
    """U = j r 2^B + rne(Psi r 2^B) mod n_g 2^B, int64, from FP32 Psi.
    Psi r 2^B is exact in FP64 (r is a power of two)."""
    r = n_g // n_p
    assert r & (r - 1) == 0 and r >= 1
    psi = np.asarray(psi_f32, dtype=np.float32).astype(np.float64)
    frac = np.rint(psi * (r * 2.0 ** B_FRAC)).astype(np.int64)
    U = lattice(n_p) * (r << B_FRAC) + frac
    return np.mod(U, n_g << B_FRAC)


def fixed_weights_1d(U, order):
    """Integer nodes and K-bit weights summing to 2^K for fixed coordinate U."""
    one = 1 << B_FRAC
    if order == 2:
        i0 = U >> B_FRAC
        f = U & (one - 1)
        return np.stack([i0, i0 + 1]), np.stack([(1 << K_W) - f, f])
    if order == 3:
        n = (U + (one >> 1)) >> B_FRAC
        X = U - (n << B_FRAC)                 # in [-2^(B-1), 2^(B-1))
        s = 2 * B_FRAC + 1 - K_W
        wl = _rne_shift(((one >> 1) - X) ** 2, s)
        wr = _rne_shift(((one >> 1) + X) ** 2, s)
        wc = (1 << K_W) - wl - wr
        return np.stack([n - 1, n, n + 1]), np.stack([wl, wc, wr])
    if order == 4:
        # PCS with F = frac(u) 2^B, G = 2^B - F (B = K = 20): the outer
        # weights G^3/6 and F^3/6 and the node-below weight (4 - 6f^2 + 3f^3)/6
        # rounded half-even from exact integers, the last one the remainder
        i0 = U >> B_FRAC
        F = U & (one - 1)
        G = one - F
        D = 6 << (2 * B_FRAC)
        wa = _rne_div(G ** 3, D)
        wd = _rne_div(F ** 3, D)
        wb = _rne_div((4 << (3 * B_FRAC)) + 3 * F ** 3 - 6 * F * F * one, D)
        wc = (1 << K_W) - wa - wb - wd
        return np.stack([i0 - 1, i0, i0 + 1, i0 + 2]), np.stack([wa, wb, wc, wd])
    raise ValueError("order must be 2, 3 or 4")


def _rne_div(p, d):
    """Round-half-to-even of p / d for non-negative int64 p and d > 0."""
    p = np.asarray(p, dtype=np.int64)
    q = p // d
    rem = p - q * d
    up = (2 * rem > d) | ((2 * rem == d) & ((q & 1) == 1))
    return q + up.astype(np.int64)


def fixed_stencil_weights(U, order):
    """Per-particle integer 3D weights (order^3, N) in stencil order
    (x offset slowest), each particle summing to exactly 2^M, with the
    mesh indices (order^3, N)."""
    n_st = [fixed_weights_1d(U[a], order) for a in range(3)]
    shift = 3 * K_W - M_MASS
    prods, idxs = [], []
    for a in range(order):
        for b in range(order):
            for c in range(order):
                prods.append(n_st[0][1][a] * n_st[1][1][b] * n_st[2][1][c])
                idxs.append((n_st[0][0][a], n_st[1][0][b], n_st[2][0][c]))
    P = np.stack(prods)                   # exact, < 2^63
    W3 = _rne_shift(P, shift)
    home = np.argmax(P, axis=0)           # first maximum on ties
    rem = (1 << M_MASS) - W3.sum(axis=0)
    W3[home, np.arange(W3.shape[1])] += rem
    return idxs, W3


def deposit_fixedpoint(psi_f32, n_p, n_g, order):
    """Integer mesh of 2^-32 particle-mass units (flat int64, n_g^3)."""
    U = fixed_coords(psi_f32, n_p, n_g)
    idxs, W3 = fixed_stencil_weights(U, order)
    out = np.zeros(n_g ** 3, dtype=np.int64)
    for s, (ix, iy, iz) in enumerate(idxs):
        lin = ((ix % n_g) * n_g + iy % n_g) * n_g + iz % n_g
        # exact integer accumulation: split each weight (< 2^34, may be
        # negative by a few units after the remainder) into 17-bit halves so
        # every float64 partial sum of bincount stays an exact integer
        # (< 2^53 for any N < 2^36)
        w = W3[s]
        hi = w >> 17
        lo = w - (hi << 17)
        out += np.rint(np.bincount(lin, weights=hi, minlength=n_g ** 3)).astype(np.int64) << 17
        out += np.rint(np.bincount(lin, weights=lo, minlength=n_g ** 3)).astype(np.int64)
    return out
