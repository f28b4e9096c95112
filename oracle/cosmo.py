"""Background cosmology, growth functions, linear spectra and BullFrog
coefficients in FP64 (test infrastructure only; see ``oracle/__init__``).

Paper passages followed
-----------------------
* App. "Exact vs approximate growth in LCDM", eq. growth_odes and the
  definition of gamma: second-order growth system for D and E, integrated in
  ln a.  The friction coefficient printed there is read as (2 - 3 gamma),
  the flat-LCDM value (the printed (1 - gamma) agrees with it only in EdS and
  contradicts the E series of Sec. "Time stepping"); this reading is pinned by
  the closed-form integral for D and by that series.
* Sec. "Time stepping": BullFrog alpha, beta, xi; uniform steps in D with the
  midpoint centred in D; D normalised so that D ~ a at early times (footnote
  of that section).
* Linear spectrum: the paper uses its Einstein-Boltzmann module; here the
  BBKS fitting formula (Bardeen, Bond, Kaiser & Szalay 1986) with shape
  Gamma = Omega_m h, normalised to sigma8 with a top-hat of 8 Mpc/h, and a
  power law A k^-2 exp(-(k/k_c)^2) normalised by an rms displacement.
  BBKS itself is "parity unpinned" against the paper (the paper never uses
  it); it is pinned only by its published formula's limits.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import integrate, optimize

A_INIT = 1e-5  # where the EdS growing mode is imposed


def hubble(a, omega_m):
    """H(a)/H0 for flat LCDM without radiation."""
    a = np.asarray(a, dtype=np.float64)
    return np.sqrt(omega_m * a ** -3 + (1.0 - omega_m))


def gamma(a, omega_m):
    """gamma = Omega_m H0^2 / (2 a^3 H^2)  (App. growth, definition of gamma)."""
    return omega_m / (2.0 * np.asarray(a, dtype=np.float64) ** 3 * hubble(a, omega_m) ** 2)


@dataclass
class Growth:
    """Dense solution of the D/E growth system in ln a (D ~ a normalisation)."""

    omega_m: float

    def __post_init__(self):
        om = self.omega_m
        self.eds = om == 1.0

        def rhs(lna, y):
            a = math.exp(lna)
            g = om / (2.0 * a ** 3 * (om * a ** -3 + 1.0 - om))
            D, dD, E, dE = y
            fr = 2.0 - 3.0 * g
            return [dD, -fr * dD + 3.0 * g * D, dE, -fr * dE + 3.0 * g * (E - D * D)]

        a0 = A_INIT
        y0 = [a0, a0, -3.0 / 7.0 * a0 ** 2, -6.0 / 7.0 * a0 ** 2]
        self.sol = integrate.solve_ivp(rhs, (math.log(a0), math.log(1.5)), y0,
                                       method="DOP853", rtol=1e-13, atol=1e-30,
                                       dense_output=True)
        assert self.sol.success

    # --- functions of a -------------------------------------------------
    def _y(self, a):
        return self.sol.sol(np.log(np.asarray(a, dtype=np.float64)))

    def D(self, a):
        return self._y(a)[0]

    def E(self, a):
        return self._y(a)[2]

    def dDdlna(self, a):
        return self._y(a)[1]

    def dEdlna(self, a):
        return self._y(a)[3]

    # --- functions of D -------------------------------------------------
    def a_of_D(self, D):
        f = lambda lna: self.sol.sol(lna)[0] - D
        lna = optimize.brentq(f, math.log(A_INIT), math.log(1.5), xtol=1e-15, rtol=1e-15)
        return math.exp(lna)

    def E_of_D(self, D):
        return float(self.E(self.a_of_D(D)))

    def dEdD(self, D):
        """E' = dE/dD (the derivative the BullFrog coefficients use)."""
        y = self._y(self.a_of_D(D))
        return float(y[3] / y[1])


def growth_closed_form(a, omega_m):
    """D(a) = (5/2) Omega_m H(a)/H0 int_0^a da' / (a' H(a')/H0)^3, which is the
    flat-LCDM growing mode with D ~ a at early times (an independent closed
    form used to pin the ODE)."""
    integrand = lambda x: 1.0 / (x * hubble(x, omega_m)) ** 3
    val, _ = integrate.quad(integrand, 0.0, a, epsabs=0.0, epsrel=1e-13, limit=200)
    return 2.5 * omega_m * float(hubble(a, omega_m)) * val


@dataclass
class StepCoeffs:
    D_n: float
    D_half: float
    D_np1: float
    alpha: float
    beta: float
    tau1: float
    tau2: float
    s: float  # 1 / D_{n+1/2}^2: D-time normalisation of the acceleration


def zeta(omega_m, a):
    """H(a) a^3 dD/da (EdS: a^(3/2)); D normalised as D ~ a at early times."""
    if omega_m == 1.0:
        return float(a) ** 1.5
    g = Growth(omega_m)
    return float(hubble(a, omega_m)) * a * a * float(g.dDdlna(a))


def superconformal(omega_m, a0, a):
    """Superconformal time from a0 to a, int da / (a^3 H) (dt_sc = dt / a^2,
    H0 = 1)."""
    return integrate.quad(lambda x: 1.0 / (x ** 3 * float(hubble(x, omega_m))), a0, a,
                          epsabs=0.0, epsrel=1e-13, limit=200)[0]


def step_table(omega_m, a_start, a_end, n_steps, stepper="bullfrog", time_var="D"):
    """Drift-kick-drift coefficients of eq. dkd (Sec. "Time stepping").

    Nodes uniform in the time variable t (D, a, ln a or superconformal time
    int da / (a^3 H)), the midpoint centred in t: D_n = D(t_n),
    D_{n+1/2} = D(t_0 + (n + 1/2) dt).  With the growth-time velocity
    V = dX/dD: tau1 = D_{n+1/2} - D_n, tau2 = D_{n+1} - D_{n+1/2},
    beta = (1 - alpha) D_{n+1/2} (Zel'dovich consistency), force scale
    s = 1 / D_{n+1/2}^2, and
      BullFrog: xi    = (E_n + E'(D_n) (D_{n+1} - D_n) / 2) / D_{n+1/2} - D_{n+1/2}
                alpha = (E'(D_{n+1}) - xi) / (E'(D_n) - xi)
      FastPM:   alpha = zeta(a_n) / zeta(a_{n+1}),  zeta(a) = H(a) a^3 dD/da.
    With the canonical momentum V = a^2 dX/dt (leapfrog, symplectic):
    alpha = 1, beta = int_{a_n}^{a_{n+1}} da / (H a^2), tau1 and tau2 the
    integrals of da / (H a^3) over the two halves, and the force of the
    comoving Poisson equation, s = (3/2) Omega_m (H0 = 1, lengths in dq).
    """
    if omega_m == 1.0:  # EdS closed forms: D = a, E = -(3/7) D^2, zeta = a^(3/2)
        Dfun = lambda a: a
        afun = lambda D: D
        Efun = lambda D: -3.0 / 7.0 * D * D
        dEfun = lambda D: -6.0 / 7.0 * D
        zeta = lambda a: a ** 1.5
    else:
        g = Growth(omega_m)
        Dfun = lambda a: float(g.D(a))
        afun = g.a_of_D
        Efun = g.E_of_D
        dEfun = g.dEdD
        # H a^3 dD/da = H a^2 dD/dln a
        zeta = lambda a: float(hubble(a, omega_m)) * a * a * float(g.dDdlna(a))
    if time_var == "D":
        t0, t1, D_of_t = Dfun(a_start), Dfun(a_end), (lambda t: t)
    elif time_var == "a":
        t0, t1, D_of_t = a_start, a_end, Dfun
    elif time_var == "lna":
        t0, t1, D_of_t = math.log(a_start), math.log(a_end), (lambda t: Dfun(math.exp(t)))
    elif time_var == "superconft":
        def a_of_sc(t):
            if t <= 0.0:
                return a_start
            return optimize.brentq(lambda a: superconformal(omega_m, a_start, a) - t, a_start, a_end * 1.5,
                                   xtol=1e-15, rtol=1e-15)
        t0, t1 = 0.0, superconformal(omega_m, a_start, a_end)
        D_of_t = lambda t: Dfun(a_of_sc(t))
    else:
        raise ValueError(time_var)
    dt = (t1 - t0) / n_steps
    out = []
    for n in range(n_steps):
        Dn = D_of_t(t0 + n * dt)
        Dp = D_of_t(t0 + (n + 1) * dt) if n + 1 < n_steps else D_of_t(t1)
        Dh = D_of_t(t0 + (n + 0.5) * dt)
        if stepper == "bullfrog":
            En, Epn, Epp = Efun(Dn), dEfun(Dn), dEfun(Dp)
            xi = (En + Epn * (Dp - Dn) / 2.0) / Dh - Dh
            alpha = (Epp - xi) / (Epn - xi)
        elif stepper == "fastpm":
            alpha = zeta(afun(Dn)) / zeta(afun(Dp))
        elif stepper == "leapfrog":
            an, ah, ap = afun(Dn), afun(Dh), afun(Dp)
            h = lambda x: float(hubble(x, omega_m))
            q = lambda f, lo, hi: integrate.quad(f, lo, hi, epsabs=0.0, epsrel=1e-13, limit=200)[0]
            kick = q(lambda x: 1.0 / (h(x) * x * x), an, ap)
            t1_ = q(lambda x: 1.0 / (h(x) * x ** 3), an, ah)
            t2_ = q(lambda x: 1.0 / (h(x) * x ** 3), ah, ap)
            out.append(StepCoeffs(Dn, Dh, Dp, 1.0, kick, t1_, t2_, 1.5 * omega_m))
            continue
        else:
            raise ValueError(stepper)
        beta = (1.0 - alpha) * Dh
        out.append(StepCoeffs(Dn, Dh, Dp, alpha, beta, Dh - Dn, Dp - Dh, 1.0 / (Dh * Dh)))
    return out


def bullfrog_steps(omega_m, a_start, a_end, n_steps):
    """BullFrog coefficients for uniform steps in D (Sec. "Time stepping")."""
    return step_table(omega_m, a_start, a_end, n_steps, "bullfrog", "D")


def D_of_a(omega_m, a):
    if omega_m == 1.0:
        return float(a)
    return float(Growth(omega_m).D(a))


# --------------------------------------------------------------------------
# Linear spectra
# --------------------------------------------------------------------------

def bbks_transfer(k, omega_m, h):
    """BBKS transfer function, q = k / (Omega_m h), k in h/Mpc, no baryon
    correction.  Parity unpinned against the paper (not used there)."""
    k = np.asarray(k, dtype=np.float64)
    q = k / (omega_m * h)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = (np.log1p(2.34 * q) / (2.34 * q)) * (
            1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4) ** -0.25
    return np.where(q > 0, t, 1.0)


def tophat_window(x):
    x = np.asarray(x, dtype=np.float64)
    small = np.abs(x) < 1e-3
    xs = np.where(small, 1.0, x)
    w = 3.0 * (np.sin(xs) - xs * np.cos(xs)) / xs ** 3
    return np.where(small, 1.0 - x * x / 10.0, w)


def sigma_R(pk_fun, R=8.0):
    """sigma(R)^2 = 1/(2 pi^2) int k^2 P(k) W^2(kR) dk, integrated in ln k over
    [1e-6, 1e3] h/Mpc by composite 32-point Gauss-Legendre on 720 panels."""
    x, wq = np.polynomial.legendre.leggauss(32)
    edges = np.linspace(math.log(1e-6), math.log(1e3), 721)
    lo, hi = edges[:-1, None], edges[1:, None]
    lnk = 0.5 * (hi - lo) * x[None, :] + 0.5 * (hi + lo)
    k = np.exp(lnk)
    f = k ** 3 * pk_fun(k) * tophat_window(k * R) ** 2
    total = float(np.sum(0.5 * (hi - lo) * wq[None, :] * f))
    return math.sqrt(total / (2.0 * math.pi ** 2))


@dataclass
class Spectrum:
    """Linear P(k) at a = 1 in (Mpc/h)^3 with k in h/Mpc."""

    kind: str              # "bbks" or "powerlaw"
    amp: float
    omega_m: float = 1.0
    h: float = 0.7
    n_s: float = 1.0
    k_c: float = 1.0

    def __call__(self, k):
        k = np.asarray(k, dtype=np.float64)
        if self.kind == "bbks":
            return self.amp * k ** self.n_s * bbks_transfer(k, self.omega_m, self.h) ** 2
        with np.errstate(divide="ignore"):
            return self.amp * k ** -2.0 * np.exp(-(k / self.k_c) ** 2)


def bbks_spectrum(omega_m, h, n_s, sigma8):
    unit = Spectrum("bbks", 1.0, omega_m, h, n_s)
    s = sigma_R(unit)
    return Spectrum("bbks", (sigma8 / s) ** 2, omega_m, h, n_s)


def kept_mode_mask(n):
    """Modes of an n^3 grid (index order of numpy's fftfreq) kept by the IC
    generator: m != 0 and |m| <= n/2 (corner modes with k above the particle
    Nyquist wavenumber zeroed, the default of tab. default_parameters)."""
    m = np.fft.fftfreq(n, 1.0 / n)
    mx, my, mz = np.meshgrid(m, m, m, indexing="ij")
    m2 = mx ** 2 + my ** 2 + mz ** 2
    return mx, my, mz, (m2 > 0) & (4 * m2 <= n * n)


def powerlaw_spectrum(n_p, n_g, box, a_start, rms_cells=0.2, D_ref=1.0, D_start=None):
    """P = A k^-2 exp(-(k/k_c)^2), k_c = half the particle Nyquist wavenumber;
    A such that the expected 3D rms Zel'dovich displacement D(a_start) psi at
    a_start is rms_cells PM-mesh cells (EdS: D = a).  The expectation is the
    exact discrete mode sum over the modes the IC generator keeps."""
    k_c = 0.5 * math.pi * n_p / box
    if D_start is None:
        D_start = a_start
    mx, my, mz, keep = kept_mode_mask(n_p)
    kf = 2.0 * math.pi / box
    ssum = 0.0
    for mc in (mx, my, mz):
        kc_ = kf * mc
        ok = keep & (mc != -n_p // 2)  # the c-th Nyquist plane is zeroed in psi_c
        k2 = kf ** 2 * (mx ** 2 + my ** 2 + mz ** 2)
        k = np.sqrt(k2[ok])
        ssum += np.sum(kc_[ok] ** 2 / k2[ok] ** 2 * k ** -2.0 * np.exp(-(k / k_c) ** 2))
    var_unit = D_start ** 2 * ssum / box ** 3 / D_ref ** 2
    target = rms_cells * box / n_g
    return Spectrum("powerlaw", target ** 2 / var_unit, k_c=k_c)
