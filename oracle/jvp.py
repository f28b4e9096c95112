"""Forward-mode tangents (JVPs) through the PM run, in FP64 (test
infrastructure only).

Forward mode (Sec. "Automatic differentiation") carries one tangent per
input direction from the initial conditions to the output.  The rules for
the interpolation operators are those of App. "Custom VJP and JVP"
(subsection "VJP and JVP derivations"): the JVP of a scatter w.r.t. the
positions is a scatter with the gradient kernel dotted with the tangent
positions; the JVP of a gather w.r.t. the mesh is a gather of the tangent
mesh, and w.r.t. the positions a gather with the gradient kernel dotted with
the tangent positions.  Through a drift-kick-drift step the tangents follow
the linearised updates,
  Xdot += tau1 Vdot,  Vdot = alpha Vdot + beta J_A(X^{n+1/2}) Xdot,
  Xdot += tau2 Vdot,
and at the start psi is linear in w and, with the BBKS spectrum, proportional
to sigma8, so psi_dot = T w_dot + (sigma8_dot / sigma8) psi.
"""
from __future__ import annotations

import numpy as np

from . import ics, mesh
from .force import PMConfig, force_multipliers, interlace_phase
from .pk import bin_index, power_spectrum
from .force import half_spectrum_theta, window_1d


def scatter_jvp_u(u, n_g, order, t):
    """sum_i t_i . grad_u W_j(u_i) on the mesh: the tangent of the deposit
    when the mesh coordinates u (3, M) move along t (3, M)."""
    st = [mesh.weights_1d(np.asarray(u[a], dtype=np.float64), order) for a in range(3)]
    out = np.zeros(n_g ** 3)
    for idx, (wx, wy, wz), (dx, dy, dz) in mesh._loop(st, n_g, order):
        v = t[0] * dx * wy * wz + t[1] * wx * dy * wz + t[2] * wx * wy * dz
        out += np.bincount(idx, weights=v, minlength=n_g ** 3)
    return out


def force_jvp(cfg: PMConfig, psi, s, xdot):
    """J_A(Psi) xdot for the PM force of ``force.pm_force`` (single or
    interlaced grids); xdot (3, N) in dq units."""
    n, N, r = cfg.n_g, cfg.N, cfg.r
    u1 = mesh.mesh_coords(psi, cfg.n_p, n)
    grids = [u1] if not cfg.interlace else [u1, np.mod(u1 + 0.5, n)]
    t = r * np.asarray(xdot, dtype=np.float64)
    f = n ** 3 / N
    d = [np.fft.rfftn(mesh.contrast(mesh.deposit_u(ug, n, cfg.order), N, n).reshape(n, n, n)) for ug in grids]
    dd = [np.fft.rfftn((f * scatter_jvp_u(ug, n, cfg.order, t)).reshape(n, n, n)) for ug in grids]
    if cfg.interlace:
        ph = interlace_phase(n)
        dk = 0.5 * (d[0] + ph * d[1])
        ddk = 0.5 * (dd[0] + ph * dd[1])
        phases = [1.0, np.conj(ph)]
    else:
        dk, ddk, phases = d[0], dd[0], [1.0]
    K = force_multipliers(cfg, s)
    out = np.zeros((3, N))
    for c in range(3):
        for ug, p in zip(grids, phases):
            g = np.fft.irfftn(K[c] * dk * p, s=(n, n, n), axes=(0, 1, 2)).reshape(-1)
            gd = np.fft.irfftn(K[c] * ddk * p, s=(n, n, n), axes=(0, 1, 2)).reshape(-1)
            gg = mesh.grad_gather_u(g, ug, n, cfg.order)
            out[c] += (np.sum(gg * t, axis=0) + mesh.gather_u(gd, ug, n, cfg.order)) / len(grids)
    return out


def problem_force_jvp(prob, psi, s, xdot):
    """JVP of the force the problem uses (PM or NUFFT)."""
    if prob.force == "pm":
        return force_jvp(prob.pm, psi, s, xdot)
    from . import nufft
    return nufft.nufft_force_jvp(prob.pm.n_p, prob.pm.n_g, psi, s, xdot, prob.es_width, prob.es_beta)


def density_jvp(psi, n_p, n_g, xdot):
    """Tangent of the final CIC contrast when Psi moves along xdot."""
    r = n_g // n_p
    u = mesh.mesh_coords(psi, n_p, n_g)
    return (n_g ** 3 / n_p ** 3) * scatter_jvp_u(u, n_g, 2, r * np.asarray(xdot, dtype=np.float64))


def initial_tangent(prob, w_dot, psi_lin, sigma8_dot=0.0):
    """(Psi_dot, V_dot) at a_start for the state Psi = D psi (+ D^2 psi2),
    V = psi (+ 2 D psi2)."""
    n = prob.pm.n_p
    psi_dot = ics.zeldovich_psi(np.asarray(w_dot, dtype=np.float64).reshape(n, n, n), prob.pm.box,
                                prob.spectrum_fn(), prob.D_ref())
    if prob.spectrum == "bbks":  # the power-law amplitude is set by its rms displacement
        psi_dot = psi_dot + (sigma8_dot / prob.sigma8) * psi_lin
    from .nbody import velocity_factor
    D, vf = prob.D_start(), velocity_factor(prob)
    if prob.lpt_order == 2:
        psi2_dot = ics.second_order_psi_jvp(psi_lin, n, psi_dot)
        return D * psi_dot + D * D * psi2_dot, vf * (psi_dot + 2.0 * D * psi2_dot)
    return D * psi_dot, vf * psi_dot


def run_jvp(prob, w, w_dot, sigma8_dot=0.0):
    """Primal and tangent of the run: returns (Psi, Psi_dot, delta,
    delta_dot) at a_end for the direction (w_dot, sigma8_dot)."""
    from .nbody import initial_state
    X, V, psi_lin = initial_state(prob, w)
    Xd, Vd = initial_tangent(prob, w_dot, psi_lin, sigma8_dot)
    X = np.array(X, dtype=np.float64)
    V = np.array(V, dtype=np.float64)
    force = prob.force_fn()
    for st in prob.steps():
        X += st.tau1 * V
        Xd = Xd + st.tau1 * Vd
        acc = force(X, st.s)
        jd = problem_force_jvp(prob, X, st.s, Xd)
        V = st.alpha * V + st.beta * acc
        Vd = st.alpha * Vd + st.beta * jd
        X += st.tau2 * V
        Xd = Xd + st.tau2 * Vd
    n_p, n_g = prob.pm.n_p, prob.pm.n_g
    delta = mesh.contrast(mesh.deposit(X, n_p, n_g, 2), n_p ** 3, n_g)
    return X, Xd, delta, density_jvp(X, n_p, n_g, Xd)


def power_spectrum_jvp(delta, delta_dot, box, n_bins, deconvolve_cic=True):
    """(k, P, P_dot, counts) with P_dot the tangent of ``pk.power_spectrum``
    when delta moves along delta_dot: the same bins of 2 Re(conj(d) d_dot)."""
    kb, pk, cnt = power_spectrum(delta, box, n_bins, deconvolve_cic)
    delta = np.asarray(delta, dtype=np.float64)
    n = round(delta.size ** (1 / 3))
    dk = np.fft.rfftn(delta.reshape(n, n, n))
    ddk = np.fft.rfftn(np.asarray(delta_dot, dtype=np.float64).reshape(n, n, n))
    tx, ty, tz, (mx, my, mz) = half_spectrum_theta(n)
    p = 2.0 * np.real(np.conj(dk) * ddk)
    if deconvolve_cic:
        W = window_1d(tx, 2) * window_1d(ty, 2) * window_1d(tz, 2)
        p = p / (W * W)
    wm = np.where((mz == 0) | (mz == n // 2), 1.0, 2.0)
    m2 = (mx ** 2 + my ** 2 + mz ** 2).astype(np.int64)
    b = bin_index(m2)
    sel = (m2 > 0) & (b <= n_bins)
    bb = b[sel] - 1
    ps = np.bincount(bb, weights=(wm * p)[sel], minlength=n_bins)
    with np.errstate(invalid="ignore", divide="ignore"):
        pdot = box ** 3 / float(n) ** 6 * ps / cnt
    return kb, pk, pdot, cnt
