"""BullFrog drift-kick-drift N-body run in FP64 (test infrastructure only).

Follows eq. dkd (Sec. "Time stepping"):
  X^{n+1/2} = X^n + tau1 V^n
  V^{n+1}   = alpha V^n + beta A(X^{n+1/2})
  X^{n+1}   = X^{n+1/2} + tau2 V^{n+1}
with V = dX/dD, BullFrog alpha/beta, uniform steps in D, and the Zel'dovich
initial state X = q + D(a_start) psi, V = psi (or its second-order LPT
extension, Sec. "Lagrangian perturbation theory").  Positions are carried as the
displacement Psi from the lattice point, in dq units.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import cosmo, ics, philox
from .force import PMConfig, pm_force


@dataclass
class Problem:
    pm: PMConfig
    omega_m: float = 0.31
    h: float = 0.68
    n_s: float = 0.965
    sigma8: float = 0.81
    spectrum: str = "bbks"          # "bbks" or "powerlaw"
    rms_cells: float = 0.2          # powerlaw normalisation
    a_start: float = 0.02
    a_end: float = 1.0
    n_steps: int = 6
    force: str = "pm"               # "pm" or "nufft"
    lpt_order: int = 1              # 1 Zel'dovich, 2 second-order LPT initial state
    stepper: str = "bullfrog"       # "bullfrog", "fastpm" or "leapfrog" (canonical momentum)
    time_var: str = "D"             # steps uniform in "D", "a", "lna" or "superconft"
    es_width: int = 6
    es_beta: float = 13.8
    _cache: dict = field(default_factory=dict, repr=False)

    def D_ref(self):
        return cosmo.D_of_a(self.omega_m, 1.0)

    def D_start(self):
        return cosmo.D_of_a(self.omega_m, self.a_start)

    def spectrum_fn(self):
        if "spec" not in self._cache:
            if self.spectrum == "bbks":
                sp = cosmo.bbks_spectrum(self.omega_m, self.h, self.n_s, self.sigma8)
            else:
                sp = cosmo.powerlaw_spectrum(self.pm.n_p, self.pm.n_g, self.pm.box,
                                             self.a_start, self.rms_cells,
                                             D_ref=self.D_ref(), D_start=self.D_start())
            self._cache["spec"] = sp
        return self._cache["spec"]

    def steps(self):
        if "steps" not in self._cache:
            self._cache["steps"] = cosmo.step_table(self.omega_m, self.a_start, self.a_end,
                                                    self.n_steps, self.stepper, self.time_var)
        return self._cache["steps"]

    def force_fn(self):
        if self.force == "pm":
            return lambda psi, s: pm_force(self.pm, psi, s)
        from . import nufft
        return lambda psi, s: nufft.nufft_force(self.pm.n_p, self.pm.n_g, psi, s,
                                                self.es_width, self.es_beta)


def velocity_factor(prob: Problem):
    """V per unit dX/dD at a_start: 1 for the growth-time velocity, and
    a^2 dX/dt = a^3 H dD/da dX/dD = zeta(a_start) for the canonical momentum."""
    return cosmo.zeta(prob.omega_m, prob.a_start) if prob.stepper == "leapfrog" else 1.0


def initial_state(prob: Problem, w):
    """(Psi, V, psi1) at a_start: the LPT series of eq. LPT truncated at
    prob.lpt_order (1: Zel'dovich; 2: plus the second-order term), V in the
    stepper's velocity variable."""
    psi = ics.zeldovich_psi(w, prob.pm.box, prob.spectrum_fn(), prob.D_ref())
    psi2 = ics.second_order_psi(psi, prob.pm.n_p) if prob.lpt_order == 2 else None
    X, V = ics.lpt_state(psi, psi2, prob.D_start())
    return X, velocity_factor(prob) * V, psi


def white_noise(prob: Problem, seed):
    return philox.white_noise(seed, prob.pm.n_p)


def run_from(prob: Problem, psi, vel, steps=None, record=None, progress=None):
    """Integrate (Psi, V) through the BullFrog steps; ``record`` (a list), if
    given, receives (Psi^{n+1/2}, A^{n+1/2}, V^n, V^{n+1}) per step;
    ``progress``, if given, is called with a short message after each step."""
    force = prob.force_fn()
    psi = np.array(psi, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    for i, st in enumerate(prob.steps() if steps is None else steps):
        psi += st.tau1 * vel
        acc = force(psi, st.s)
        v_before = vel
        vel = st.alpha * vel + st.beta * acc
        if record is not None:
            record.append((psi.copy(), acc, v_before.copy(), vel.copy()))
        psi += st.tau2 * vel
        if progress is not None:
            progress(f"oracle forward step {i} done")
    return psi, vel


def run(prob: Problem, seed=None, w=None, progress=None):
    if w is None:
        w = white_noise(prob, seed)
    psi0, vel0, _ = initial_state(prob, w)
    return run_from(prob, psi0, vel0, progress=progress)
