/*
 * Oracle (test infrastructure only): Van-der-Waals thermodynamics of Sec. 2.1
 * (free energy density, pressure as rho W' - W, reduced constants a = 3,
 * b = 1/3, R = 8/3), the Maxwell (binodal) and spinodal densities, the
 * gradient-theory surface-tension integral and the Young-Laplace initial
 * densities of the head-on collision set-up (Sec. 4.3.1).
 */
#include <math.h>
#include "oracle.h"

static const double A_VDW = 3.0;
static const double B_VDW = 1.0 / 3.0;
static const double R_VDW = 8.0 / 3.0;

/* W(rho) = rho R T ln(rho / (1 - b rho)) - a rho^2 */
double or_W(double T, double rho) {
  return rho * R_VDW * T * log(rho / (1.0 - B_VDW * rho)) - A_VDW * rho * rho;
}

/* W'(rho) = R T [ln(rho / (1 - b rho)) + 1 / (1 - b rho)] - 2 a rho */
double or_dW(double T, double rho) {
  return R_VDW * T * (log(rho / (1.0 - B_VDW * rho)) + 1.0 / (1.0 - B_VDW * rho)) -
         2.0 * A_VDW * rho;
}

/* W''(rho) = R T / (rho (1 - b rho)^2) - 2 a */
double or_d2W(double T, double rho) {
  double q = 1.0 - B_VDW * rho;
  return R_VDW * T / (rho * q * q) - 2.0 * A_VDW;
}

/* p = rho W' - W, which simplifies to rho R T / (1 - b rho) - a rho^2 */
double or_p(double T, double rho) {
  return rho * R_VDW * T / (1.0 - B_VDW * rho) - A_VDW * rho * rho;
}

/* p'(rho) = rho W''(rho) = R T / (1 - b rho)^2 - 2 a rho */
double or_dp(double T, double rho) {
  double q = 1.0 - B_VDW * rho;
  return R_VDW * T / (q * q) - 2.0 * A_VDW * rho;
}

/* Bisection for a root of f on [a, b] with a sign change. */
static double bisect(double (*f)(double, double), double T, double target, double a, double b) {
  double fa = f(T, a) - target;
  for (int it = 0; it < 200; ++it) {
    double m = 0.5 * (a + b);
    double fm = f(T, m) - target;
    if ((fm < 0) == (fa < 0)) { a = m; fa = fm; } else { b = m; }
  }
  return 0.5 * (a + b);
}

int or_spinodal(double T, double* rho_sv, double* rho_sl) {
  /* p'(rho) > 0 near 0, < 0 at the critical density 1 for T < 1, > 0 near 3 */
  if (!(T > 0.0 && T < 1.0)) return -1;
  *rho_sv = bisect(or_dp, T, 0.0, 1e-6, 1.0);
  *rho_sl = bisect(or_dp, T, 0.0, 1.0, 3.0 - 1e-9);
  return 0;
}

/* Maxwell construction: p(rho_v) = p(rho_l) and W'(rho_v) = W'(rho_l).
 * Newton iteration in the two unknowns from the spinodal-bracketed guesses. */
int or_maxwell(double T, double* rho_v, double* rho_l, double* p_sat, double* mu_sat) {
  double sv, sl;
  if (or_spinodal(T, &sv, &sl)) return -1;
  double v = 0.5 * sv, l = 0.5 * (sl + 3.0);
  for (int it = 0; it < 200; ++it) {
    double f1 = or_p(T, l) - or_p(T, v);
    double f2 = or_dW(T, l) - or_dW(T, v);
    /* Jacobian wrt (v, l): dp/drho = p', dmu/drho = W'' */
    double a11 = -or_dp(T, v), a12 = or_dp(T, l);
    double a21 = -or_d2W(T, v), a22 = or_d2W(T, l);
    double det = a11 * a22 - a12 * a21;
    double dv = (f1 * a22 - a12 * f2) / det;
    double dl = (a11 * f2 - a21 * f1) / det;
    /* damped step that keeps the iterates on their branches */
    double s = 1.0;
    while ((v - s * dv <= 0.0 || v - s * dv >= sv || l - s * dl <= sl || l - s * dl >= 3.0) && s > 1e-6)
      s *= 0.5;
    v -= s * dv;
    l -= s * dl;
    if (fabs(dv) + fabs(dl) < 1e-15) break;
  }
  *rho_v = v;
  *rho_l = l;
  if (p_sat) *p_sat = or_p(T, v);
  if (mu_sat) *mu_sat = or_dW(T, v);
  return 0;
}

/* Integral over [rho_v, rho_l] of sqrt(2 (W(rho) - mu_sat rho + p_sat)), by a
 * composite 8-point Gauss-Legendre rule on 4000 panels.  The integrand is the
 * planar equilibrium profile's kappa*rho_x (up to sqrt(kappa)) expressed as a
 * function of rho, so sigma = integral of kappa rho_x^2 dx = sqrt(kappa) I. */
double or_surface_integral(double T) {
  double v, l, ps, mus;
  if (or_maxwell(T, &v, &l, &ps, &mus)) return NAN;
  or_basis b;
  or_make_basis(7, &b);
  const int panels = 4000;
  double h = (l - v) / panels, sum = 0.0;
  for (int k = 0; k < panels; ++k) {
    double a = v + k * h;
    for (int q = 0; q < 8; ++q) {
      double rho = a + 0.5 * h * (b.xi[q] + 1.0);
      double g = or_W(T, rho) - mus * rho + ps;
      if (g < 0.0) g = 0.0;
      sum += 0.5 * h * b.w[q] * sqrt(2.0 * g);
    }
  }
  return sum;
}

/* Young-Laplace adjusted phase pressures of a droplet of radius r with surface
 * tension sigma, then the densities on the liquid and vapour branches of the
 * isotherm that carry these pressures. */
int or_young_laplace(double T, double sigma, double r, double* rho_l, double* rho_v) {
  double v, l, ps, mus, sv, sl;
  if (or_maxwell(T, &v, &l, &ps, &mus)) return -1;
  if (or_spinodal(T, &sv, &sl)) return -1;
  double pl = ps + l / (l - v) * 2.0 * sigma / r;
  double pv = ps + v / (l - v) * 2.0 * sigma / r;
  *rho_l = bisect(or_p, T, pl, sl, 3.0 - 1e-12);
  *rho_v = bisect(or_p, T, pv, 1e-9, sv);
  return 0;
}
