// Host-side FP64 tables: growth functions, BullFrog coefficients and linear
// spectra.  Everything here runs once per context on the host; the device
// receives only the resulting scalars and small tables.
//
// Growth: App. "Exact vs approximate growth in LCDM", eq. growth_odes, with the
// friction coefficient read as (2 - 3 gamma) (flat LCDM; the printed (1 - gamma)
// disagrees with the E series of Sec. "Time stepping" outside EdS).  Solved
// with fixed-step RK4 uniform in ln a, as the appendix describes, and cubic
// Hermite interpolation between the steps.
// Steppers: Sec. "Time stepping" (BullFrog alpha, beta, xi; FastPM alpha from
// zeta = H a^3 dD/da; steps uniform in D, a or ln a).
// Spectra: BBKS fitting formula with Gamma = Omega_m h normalised to sigma8
// (top-hat of 8 Mpc/h, composite Simpson in ln k), or a Gaussian-truncated
// k^-2 power law normalised by an rms displacement.
#include <cmath>
#include <cstdio>

#include "pm_internal.h"

namespace pm {

namespace {

void growth_rhs(double om, double x, const double* y, double* f) {
  double a3 = std::exp(3.0 * x);
  double g = om / (2.0 * (om + (1.0 - om) * a3));  // Om H0^2 / (2 a^3 H^2)
  double fr = 2.0 - 3.0 * g;
  f[0] = y[1];
  f[1] = -fr * y[1] + 3.0 * g * y[0];
  f[2] = y[3];
  f[3] = -fr * y[3] + 3.0 * g * (y[2] - y[0] * y[0]);
}

// cubic Hermite on [x0, x0 + h] from values and derivatives at the ends
double hermite(double t, double h, double y0, double d0, double y1, double d1) {
  double t2 = t * t, t3 = t2 * t;
  return (2 * t3 - 3 * t2 + 1) * y0 + (t3 - 2 * t2 + t) * h * d0 + (-2 * t3 + 3 * t2) * y1 +
         (t3 - t2) * h * d1;
}

}  // namespace

static constexpr double kAInit = 1e-5, kAMax = 1.5;
static constexpr int kGrowthSteps = 40000;

void Growth::solve(double om) {
  omega_m = om;
  eds = (om == 1.0);
  lna.clear(); D.clear(); dD.clear(); E.clear(); dE.clear();
  if (eds) return;
  double x0 = std::log(kAInit), x1 = std::log(kAMax);
  double h = (x1 - x0) / kGrowthSteps;
  double y[4] = {kAInit, kAInit, -3.0 / 7.0 * kAInit * kAInit, -6.0 / 7.0 * kAInit * kAInit};
  for (int i = 0; i <= kGrowthSteps; ++i) {
    double x = x0 + i * h;
    lna.push_back(x); D.push_back(y[0]); dD.push_back(y[1]); E.push_back(y[2]); dE.push_back(y[3]);
    if (i == kGrowthSteps) break;
    double k1[4], k2[4], k3[4], k4[4], t[4];
    growth_rhs(om, x, y, k1);
    for (int j = 0; j < 4; ++j) t[j] = y[j] + 0.5 * h * k1[j];
    growth_rhs(om, x + 0.5 * h, t, k2);
    for (int j = 0; j < 4; ++j) t[j] = y[j] + 0.5 * h * k2[j];
    growth_rhs(om, x + 0.5 * h, t, k3);
    for (int j = 0; j < 4; ++j) t[j] = y[j] + h * k3[j];
    growth_rhs(om, x + h, t, k4);
    for (int j = 0; j < 4; ++j) y[j] += h / 6.0 * (k1[j] + 2 * k2[j] + 2 * k3[j] + k4[j]);
  }
}

// interpolate (D, D', E, E') at ln a = x (primes: d/dln a)
static void growth_at(const Growth& g, double x, double out[4]) {
  double x0 = g.lna.front(), h = g.lna[1] - g.lna[0];
  int i = (int)std::floor((x - x0) / h);
  if (i < 0) i = 0;
  if (i > (int)g.lna.size() - 2) i = (int)g.lna.size() - 2;
  double t = (x - g.lna[i]) / h;
  double ya[4] = {g.D[i], g.dD[i], g.E[i], g.dE[i]};
  double yb[4] = {g.D[i + 1], g.dD[i + 1], g.E[i + 1], g.dE[i + 1]};
  double fa[4], fb[4];
  growth_rhs(g.omega_m, g.lna[i], ya, fa);
  growth_rhs(g.omega_m, g.lna[i + 1], yb, fb);
  for (int j = 0; j < 4; ++j) out[j] = hermite(t, h, ya[j], fa[j], yb[j], fb[j]);
}

double Growth::D_of_a(double a) const {
  if (eds) return a;
  double y[4];
  growth_at(*this, std::log(a), y);
  return y[0];
}

double Growth::a_of_D(double Dv) const {
  if (eds) return Dv;
  double lo = lna.front(), hi = lna.back();
  for (int it = 0; it < 200 && hi - lo > 1e-15; ++it) {
    double mid = 0.5 * (lo + hi), y[4];
    growth_at(*this, mid, y);
    if (y[0] < Dv) lo = mid; else hi = mid;
  }
  return std::exp(0.5 * (lo + hi));
}

void Growth::at_D(double Dv, double* Ev, double* dEdD) const {
  if (eds) {
    *Ev = -3.0 / 7.0 * Dv * Dv;
    *dEdD = -6.0 / 7.0 * Dv;
    return;
  }
  double y[4];
  growth_at(*this, std::log(a_of_D(Dv)), y);
  *Ev = y[2];
  *dEdD = y[3] / y[1];
}

// FastPM's zeta(a) = H(a) a^3 dD/da = H a^2 dD/dln a (EdS: a^(3/2))
double Growth::zeta(double a) const {
  if (eds) return a * std::sqrt(a);
  double y[4];
  growth_at(*this, std::log(a), y);
  return std::sqrt(omega_m / (a * a * a) + 1.0 - omega_m) * a * a * y[1];
}

// eq. dkd coefficients (Sec. "Time stepping"): nodes uniform in the time
// variable t (D, a or ln a) with the midpoint centred in t; Zel'dovich
// consistency beta = (1 - alpha) D_{n+1/2}; BullFrog
//   xi = (E_n + E'(D_n) (D_{n+1} - D_n) / 2) / D_{n+1/2} - D_{n+1/2},
//   alpha = (E'(D_{n+1}) - xi) / (E'(D_n) - xi),
// or FastPM alpha = zeta(a_n) / zeta(a_{n+1}).
// int_a^b f(x) dx by 8 panels of 16-point Gauss-Legendre in ln x (the
// integrands here are powers of x times 1/H, smooth in ln x)
template <class F>
static double integrate_lnx(F f, double a, double b) {
  static const double xg[8] = {0.0950125098376374, 0.2816035507792589, 0.4580167776572274, 0.6178762444026438,
                               0.7554044083550030, 0.8656312023878318, 0.9445750230732326, 0.9894009349916499};
  static const double wg[8] = {0.1894506104550685, 0.1826034150449236, 0.1691565193950025, 0.1495959888165767,
                               0.1246289712555339, 0.0951585116824928, 0.0622535239386479, 0.0271524594117541};
  const double l0 = std::log(a), l1 = std::log(b), h = (l1 - l0) / 8.0;
  double sum = 0.0;
  for (int p = 0; p < 8; ++p) {
    const double c = l0 + (p + 0.5) * h, r = 0.5 * h;
    for (int k = 0; k < 8; ++k)
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        const double x = std::exp(c + sgn * r * xg[k]);
        sum += wg[k] * r * f(x) * x;
      }
  }
  return sum;
}

static double hubble(double a, double om) { return std::sqrt(om / (a * a * a) + (1.0 - om)); }

std::vector<StepCoef> step_table(const Growth& g, double a_start, double a_end, int n_steps, int stepper,
                                 int time_var) {
  std::vector<StepCoef> out;
  const double om = g.omega_m;
  // superconformal time from a_start (dt_sc = dt / a^2 = da / (a^3 H)) and its inverse by bisection
  auto sconf = [&](double a) { return integrate_lnx([&](double x) { return 1.0 / (x * x * x * hubble(x, om)); }, a_start, a); };
  auto a_of_sc = [&](double t) {
    if (t <= 0.0) return a_start;
    double lo = a_start, hi = a_end * 1.5;
    for (int it = 0; it < 200 && hi - lo > 1e-16 * hi; ++it) {
      const double mid = 0.5 * (lo + hi);
      (sconf(mid) < t ? lo : hi) = mid;
    }
    return 0.5 * (lo + hi);
  };
  auto D_of_t = [&](double t) {
    return time_var == 1 ? g.D_of_a(t)
                         : (time_var == 2 ? g.D_of_a(std::exp(t)) : (time_var == 3 ? g.D_of_a(a_of_sc(t)) : t));
  };
  double t0, t1;
  if (time_var == 3) {
    t0 = 0.0;
    t1 = sconf(a_end);
  } else if (time_var == 1) {
    t0 = a_start;
    t1 = a_end;
  } else if (time_var == 2) {
    t0 = std::log(a_start);
    t1 = std::log(a_end);
  } else {
    t0 = g.D_of_a(a_start);
    t1 = g.D_of_a(a_end);
  }
  const double dt = (t1 - t0) / n_steps;
  for (int n = 0; n < n_steps; ++n) {
    double Dn = D_of_t(t0 + n * dt), Dh = D_of_t(t0 + (n + 0.5) * dt);
    double Dp = D_of_t(n + 1 < n_steps ? t0 + (n + 1) * dt : t1);
    double alpha;
    if (stepper == 2) {
      // canonical momentum V = a^2 dX/dt: the symplectic leapfrog of the
      // comoving equations (H0 = 1): alpha = 1, kick int da / (H a^2), the two
      // drifts int da / (H a^3), force of the Poisson equation s = 3/2 Omega_m
      const double an = g.a_of_D(Dn), ah = g.a_of_D(Dh), ap = g.a_of_D(Dp);
      auto drift = [&](double x) { return 1.0 / (hubble(x, om) * x * x * x); };
      auto kick = [&](double x) { return 1.0 / (hubble(x, om) * x * x); };
      out.push_back({Dn, Dh, Dp, 1.0, integrate_lnx(kick, an, ap), integrate_lnx(drift, an, ah),
                     integrate_lnx(drift, ah, ap), 1.5 * om});
      continue;
    }
    if (stepper == 1) {
      alpha = g.zeta(g.a_of_D(Dn)) / g.zeta(g.a_of_D(Dp));
    } else {
      double En, Epn, Ep1, tmp;
      g.at_D(Dn, &En, &Epn);
      g.at_D(Dp, &tmp, &Ep1);
      double xi = (En + Epn * (Dp - Dn) / 2.0) / Dh - Dh;
      alpha = (Ep1 - xi) / (Epn - xi);
    }
    double beta = (1.0 - alpha) * Dh;
    out.push_back({Dn, Dh, Dp, alpha, beta, Dh - Dn, Dp - Dh, 1.0 / (Dh * Dh)});
  }
  return out;
}

static double bbks_T(double k, double omega_m, double h) {
  double q = k / (omega_m * h);
  if (q <= 0) return 1.0;
  double p = 1.0 + 3.89 * q + std::pow(16.1 * q, 2) + std::pow(5.46 * q, 3) + std::pow(6.71 * q, 4);
  return std::log1p(2.34 * q) / (2.34 * q) * std::pow(p, -0.25);
}

static double tophat(double x) {
  if (std::fabs(x) < 1e-3) return 1.0 - x * x / 10.0;
  return 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
}

double bbks_amplitude(double omega_m, double h, double n_s, double sigma8) {
  // sigma8^2 = A / (2 pi^2) int k^3 k^n_s T^2 W^2(8k) dln k, composite Simpson
  const int n = 40000;  // even
  double x0 = std::log(1e-6), x1 = std::log(1e3), dx = (x1 - x0) / n, sum = 0.0;
  for (int i = 0; i <= n; ++i) {
    double k = std::exp(x0 + i * dx);
    double T = bbks_T(k, omega_m, h), W = tophat(8.0 * k);
    double f = k * k * k * std::pow(k, n_s) * T * T * W * W;
    double c = (i == 0 || i == n) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
    sum += c * f;
  }
  double s2unit = sum * dx / 3.0 / (2.0 * M_PI * M_PI);
  return sigma8 * sigma8 / s2unit;
}

double spectrum_eval(const pm_config& c, double amp, double k) {
  if (k <= 0) return 0.0;
  if (c.spectrum == PM_SPEC_BBKS) {
    double T = bbks_T(k, c.omega_m, c.h);
    return amp * std::pow(k, c.n_s) * T * T;
  }
  double kc = 0.5 * M_PI * c.n_p / c.box;
  return amp * std::exp(-(k / kc) * (k / kc)) / (k * k);
}

double powerlaw_amplitude(const pm_config& c, double D_start, double D_ref) {
  // expected 3D rms of D_start psi over the kept modes equals pl_rms_cells
  // PM cells: sum_c sum_m k_c^2 / k^4 P(k) / L^3 (D_start / D_ref)^2
  int n = c.n_p;
  double kf = 2.0 * M_PI / c.box, sum = 0.0;
  pm_config unit = c;
  for (int ix = 0; ix < n; ++ix)
    for (int iy = 0; iy < n; ++iy)
      for (int iz = 0; iz < n; ++iz) {
        int m[3] = {ix < n / 2 ? ix : ix - n, iy < n / 2 ? iy : iy - n, iz < n / 2 ? iz : iz - n};
        long long m2 = (long long)m[0] * m[0] + (long long)m[1] * m[1] + (long long)m[2] * m[2];
        if (m2 == 0 || 4 * m2 > (long long)n * n) continue;
        double k2 = kf * kf * m2, p = spectrum_eval(unit, 1.0, std::sqrt(k2));
        for (int a = 0; a < 3; ++a) {
          if (m[a] == -n / 2) continue;  // Nyquist plane of component a
          sum += (kf * m[a]) * (kf * m[a]) / (k2 * k2) * p;
        }
      }
  double var = D_start * D_start * sum / (c.box * c.box * c.box) / (D_ref * D_ref);
  double target = c.pl_rms_cells * c.box / c.n_g;
  return target * target / var;
}

double es_phihat(double theta, int width, double beta) {
  // int_{-w/2}^{w/2} phi(x) cos(theta x) dx with phi(x) = exp(beta (sqrt(1 - z^2) - 1)),
  // z = 2x/w: even integrand, composite Simpson on [0, w/2]
  const int n = 16384;
  double half = 0.5 * width, dx = half / n, sum = 0.0;
  for (int i = 0; i <= n; ++i) {
    double x = i * dx, z = x / half;
    double p = (z < 1.0) ? std::exp(beta * (std::sqrt(1.0 - z * z) - 1.0)) : 0.0;
    double c = (i == 0 || i == n) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
    sum += c * p * std::cos(theta * x);
  }
  return 2.0 * sum * dx / 3.0;
}

}  // namespace pm
