"""Store-all reverse mode through the BullFrog PM run, in FP64 (test
infrastructure only).

This is the "discretise-then-optimise" gradient of Sec. "Adjoint method":
every midpoint state X^{n+1/2} of the forward run is kept and the exact VJPs
of each drift and kick are applied backwards.  It never integrates the primal
state backwards, so it is independent of the reverse-trajectory trick of the
adjoint method that the GPU uses; the recurrences for the cotangents are
those of tab. adjoint_dkd, and the VJP of the force is assembled from the
scatter/gather rules of App. "Custom VJP and JVP":

* gather w.r.t. positions (a gather with grad W, weighted by the cotangent),
* gather w.r.t. the mesh (a scatter of the cotangent with W),
* the transposed Fourier multiplier (conj K_c),
* scatter w.r.t. positions (a gather of the mesh cotangent with grad W).

The initial-condition VJP uses Psi^0 = D_start psi, V^0 = psi (plus
D^2 psi2 and 2 D psi2 at second order, psi2 quadratic in psi) and the
transposed IC multiplier; with the BBKS spectrum psi is proportional to
sigma8 (psi2 to its square) and the BullFrog coefficients do not depend on
it, so dL/dsigma8 = <psi_bar, psi> / sigma8 with psi_bar the total cotangent
of psi (Euler's theorem for the quadratic term; 0 for the power-law
spectrum, whose amplitude is set by its rms displacement).
"""
from __future__ import annotations

import numpy as np

from . import ics, mesh, nbody
from .force import force_multipliers, interlace_phase, PMConfig


def force_vjp(cfg: PMConfig, psi, s, u, parts=3):
    """J_A(Psi)^T u for the PM force A(Psi) of ``force.pm_force``; u (3, N).
    parts: 1 the direct term (gather w.r.t. positions) only, 2 the terms
    through the mesh only, 3 both."""
    if cfg.interlace:
        return force_vjp_interlaced(cfg, psi, s, u, parts)
    n, N = cfg.n_g, cfg.N
    delta = mesh.contrast(mesh.deposit(psi, cfg.n_p, n, cfg.order), N, n)
    dk = np.fft.rfftn(delta.reshape(n, n, n))
    K = force_multipliers(cfg, s)
    xbar = np.zeros((3, N))
    dbar_k = np.zeros_like(dk)
    for c in range(3):
        g_c = np.fft.irfftn(K[c] * dk, s=(n, n, n), axes=(0, 1, 2)).reshape(-1)
        # direct part: d/dX_i of gather(g_c)(X_i), weighted by u_c
        if parts & 1:
            xbar += mesh.grad_gather(g_c, psi, cfg.n_p, n, cfg.order) * u[c]
        # mesh part: gather^T = scatter of u_c, then the transposed multiplier
        gbar = mesh.deposit(psi, cfg.n_p, n, cfg.order, weights=u[c])
        dbar_k += np.conj(K[c]) * np.fft.rfftn(gbar.reshape(n, n, n))
    dbar = np.fft.irfftn(dbar_k, s=(n, n, n), axes=(0, 1, 2)).reshape(-1)
    # delta = (n^3/N) m - 1, and m = scatter(1): scatter^T w.r.t. positions
    if parts & 2:
        xbar += mesh.grad_gather(dbar * (n ** 3 / N), psi, cfg.n_p, n, cfg.order)
    return xbar


def force_vjp_interlaced(cfg: PMConfig, psi, s, u, parts=3):
    """J_A^T u for the interlaced force of ``force.pm_force_u``: with u1 the
    mesh coordinates and u2 = u1 + 1/2, A_c = (gather(g1_c, u1) +
    gather(g2_c, u2)) / 2, g1_c = IDFT(K_c dk), g2_c = IDFT(K_c e^{-i phi}
    dk), dk = (DFT(delta1) + e^{i phi} DFT(delta2)) / 2.  The same rules as
    the single grid apply per grid; the transposed multipliers carry the
    conjugate phase, so the mesh cotangents are
    delta1_bar = IDFT(B1 + e^{i phi} B2) / 2 and
    delta2_bar = IDFT(e^{-i phi} B1 + B2) / 2, with Bg = sum_c conj(K_c)
    DFT(scatter of u_c / 2 at ug)."""
    n, N, r = cfg.n_g, cfg.N, cfg.r
    x1 = mesh.mesh_coords(psi, cfg.n_p, n)
    x2 = np.mod(x1 + 0.5, n)
    d1 = np.fft.rfftn(mesh.contrast(mesh.deposit_u(x1, n, cfg.order), N, n).reshape(n, n, n))
    d2 = np.fft.rfftn(mesh.contrast(mesh.deposit_u(x2, n, cfg.order), N, n).reshape(n, n, n))
    ph = interlace_phase(n)
    dk = 0.5 * (d1 + ph * d2)
    K = force_multipliers(cfg, s)
    xbar = np.zeros((3, N))
    B1 = np.zeros_like(dk)
    B2 = np.zeros_like(dk)
    for c in range(3):
        if parts & 1:
            g1 = np.fft.irfftn(K[c] * dk, s=(n, n, n), axes=(0, 1, 2)).reshape(-1)
            g2 = np.fft.irfftn(K[c] * dk * np.conj(ph), s=(n, n, n), axes=(0, 1, 2)).reshape(-1)
            xbar += 0.5 * r * u[c] * (mesh.grad_gather_u(g1, x1, n, cfg.order)
                                      + mesh.grad_gather_u(g2, x2, n, cfg.order))
        B1 += np.conj(K[c]) * np.fft.rfftn(mesh.deposit_u(x1, n, cfg.order, weights=0.5 * u[c]).reshape(n, n, n))
        B2 += np.conj(K[c]) * np.fft.rfftn(mesh.deposit_u(x2, n, cfg.order, weights=0.5 * u[c]).reshape(n, n, n))
    if parts & 2:
        db1 = 0.5 * np.fft.irfftn(B1 + ph * B2, s=(n, n, n), axes=(0, 1, 2)).reshape(-1)
        db2 = 0.5 * np.fft.irfftn(np.conj(ph) * B1 + B2, s=(n, n, n), axes=(0, 1, 2)).reshape(-1)
        f = n ** 3 / N
        xbar += r * (mesh.grad_gather_u(db1 * f, x1, n, cfg.order) + mesh.grad_gather_u(db2 * f, x2, n, cfg.order))
    return xbar


def problem_force_vjp(prob, psi, s, u):
    """VJP of the force the problem uses (PM or NUFFT)."""
    if prob.force == "pm":
        return force_vjp(prob.pm, psi, s, u)
    from . import nufft
    return nufft.nufft_force_vjp(prob.pm.n_p, prob.pm.n_g, psi, s, u, prob.es_width, prob.es_beta)


def density_vjp(psi, n_p, n_g, dbar):
    """VJP of the final CIC contrast delta(Psi) w.r.t. Psi."""
    return mesh.grad_gather(np.asarray(dbar, dtype=np.float64) * (n_g ** 3 / n_p ** 3),
                            psi, n_p, n_g, 2)


def final_density(prob, psi):
    n_p, n_g = prob.pm.n_p, prob.pm.n_g
    return mesh.contrast(mesh.deposit(psi, n_p, n_g, 2), n_p ** 3, n_g)


def ic_vjp(prob, psibar):
    """w_bar = sum_c T_c^T psibar_c with psi_c = T_c w = IDFT(h_c DFT(w))."""
    n = prob.pm.n_p
    h = ics.ic_multipliers(n, prob.pm.box, prob.spectrum_fn(), prob.D_ref())
    acc = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
    for c in range(3):
        acc += np.conj(h[c]) * np.fft.rfftn(np.asarray(psibar[c]).reshape(n, n, n))
    return np.fft.irfftn(acc, s=(n, n, n), axes=(0, 1, 2))


def gradient(prob, w, dL_ddelta, progress=None, temporal=None):
    """Reverse-mode gradient of L(delta_final) w.r.t. the white noise w and
    sigma8, given a function dL_ddelta(delta) -> cotangent mesh.
    Returns (w_bar (n_p^3,), dL/dsigma8, delta_final).  ``progress``, if
    given, is called with a short message after each forward and reverse step;
    ``temporal`` (a list), if given, receives the per-step adjoints of
    (tau1, tau2, alpha, beta) (see reverse_cotangents)."""
    from .nbody import initial_state, run_from
    psi0, vel0, psi_lin = initial_state(prob, w)
    record = []
    psiN, _ = run_from(prob, psi0, vel0, record=record, progress=progress)
    delta = final_density(prob, psiN)
    xbar = density_vjp(psiN, prob.pm.n_p, prob.pm.n_g, dL_ddelta(delta))
    vbar = np.zeros_like(xbar)
    xbar, vbar = reverse_cotangents(prob, record, xbar, vbar, progress, temporal)
    D = prob.D_start()
    vf = nbody.velocity_factor(prob)
    psibar = D * xbar + vf * vbar
    if prob.lpt_order == 2:
        # Psi = D psi1 + D^2 psi2(psi1), V = vf (psi1 + 2 D psi2(psi1))
        psibar = psibar + ics.second_order_psi_vjp(psi_lin, prob.pm.n_p, D * D * xbar + 2.0 * D * vf * vbar)
    wbar = ic_vjp(prob, psibar)
    # the power-law spectrum is normalised by its rms displacement, not by
    # sigma8, so there the initial conditions do not depend on sigma8
    dsig = float(np.sum(psibar * psi_lin)) / prob.sigma8 if prob.spectrum == "bbks" else 0.0
    return wbar.reshape(-1), dsig, delta


def reverse_cotangents(prob, record, xbar, vbar, progress=None, temporal=None):
    """Apply the cotangent recurrences of tab. adjoint_dkd over the stored
    midpoints, last step first.  ``temporal`` (a list), if given, receives
    per step, first step first, the adjoints of its scalars (tau1, tau2,
    alpha, beta): for V^{n+1} = alpha V^n + beta A, X^{n+1} = X^{n+1/2} +
    tau2 V^{n+1}, X^{n+1/2} = X^n + tau1 V^n,
      tau2_bar = X_bar^{n+1} . V^{n+1},  alpha_bar = V_bar^{n+1/2} . V^n,
      beta_bar = V_bar^{n+1/2} . A^{n+1/2},  tau1_bar = X_bar^{n+1/2} . V^n,
    with V_bar^{n+1/2} the cotangent of the kick's output and X_bar^{n+1/2}
    that of the midpoint position (the table prints V^n for the velocity in
    the alpha row, read as the kick's input, the only factor the kick
    multiplies by alpha)."""
    out = []
    for i, (st, (psi_half, acc, v_n, v_np1)) in enumerate(zip(reversed(prob.steps()), reversed(record))):
        tau2_bar = float(np.sum(xbar * v_np1))
        vbar = vbar + st.tau2 * xbar                    # adjoint of drift 2
        alpha_bar = float(np.sum(vbar * v_n))
        beta_bar = float(np.sum(vbar * acc))
        xbar = xbar + problem_force_vjp(prob, psi_half, st.s, st.beta * vbar)  # adjoint kick
        vbar = st.alpha * vbar                          # velocity rescale
        tau1_bar = float(np.sum(xbar * v_n))
        vbar = vbar + st.tau1 * xbar                    # adjoint of drift 1
        out.append((tau1_bar, tau2_bar, alpha_bar, beta_bar))
        if progress is not None:
            progress(f"oracle reverse step {i} done")
    if temporal is not None:
        temporal.extend(reversed(out))
    return xbar, vbar
