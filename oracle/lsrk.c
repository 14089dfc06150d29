/*
 * Oracle (test infrastructure only): explicit low-storage Runge-Kutta time
 * integration (Sec. 3.1: fourth order, five stages, low storage).  The paper
 * names the family but prints no coefficients; the scheme used is the
 * published Carpenter-Kennedy (1994) 2N-storage RK4(5):
 *     dU <- A_s dU + dt R(U, t + C_s dt);   U <- U + B_s dU,   s = 1..5.
 */
#include <math.h>
#include "oracle.h"

void or_lsrk45(double A[5], double B[5], double C[5]) {
  A[0] = 0.0;
  A[1] = -567301805773.0 / 1357537059087.0;
  A[2] = -2404267990393.0 / 2016746695238.0;
  A[3] = -3550918686646.0 / 2091501179385.0;
  A[4] = -1275806237668.0 / 842570457699.0;
  B[0] = 1432997174477.0 / 9575080441755.0;
  B[1] = 5161836677717.0 / 13612068292357.0;
  B[2] = 1720146321549.0 / 2090206949498.0;
  B[3] = 3134564353537.0 / 4481467310338.0;
  B[4] = 2277821191437.0 / 14882151754819.0;
  C[0] = 0.0;
  C[1] = 1432997174477.0 / 9575080441755.0;
  C[2] = 2526269341429.0 / 6820363962896.0;
  C[3] = 2006345519317.0 / 3224310063776.0;
  C[4] = 2802321613138.0 / 2924317926251.0;
}

/* Apply one step to y' = z y with polynomial coefficients in z: the state and
 * the register are polynomials of degree <= 5. */
void or_lsrk_stability_poly(double g[6]) {
  double A[5], B[5], C[5];
  or_lsrk45(A, B, C);
  double u[7] = {1, 0, 0, 0, 0, 0, 0};
  double du[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int s = 0; s < 5; ++s) {
    /* dt R(U) = z u  -> shift coefficients by one power of z */
    double zu[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < 6; ++k) zu[k + 1] = u[k];
    for (int k = 0; k < 7; ++k) du[k] = A[s] * du[k] + zu[k];
    for (int k = 0; k < 7; ++k) u[k] += B[s] * du[k];
  }
  for (int k = 0; k < 6; ++k) g[k] = u[k];
}

static double stab_abs(const double g[6], double x) {
  double z = -x, r = 0.0, zp = 1.0;
  for (int k = 0; k < 6; ++k) { r += g[k] * zp; zp *= z; }
  return fabs(r);
}

double or_lsrk_real_limit(void) {
  double g[6];
  or_lsrk_stability_poly(g);
  /* march outward to the first x with |R(-x)| > 1, then bisect */
  double x = 0.0, step = 1e-3;
  while (stab_abs(g, x + step) <= 1.0 && x < 100.0) x += step;
  double a = x, b = x + step;
  for (int it = 0; it < 200; ++it) {
    double m = 0.5 * (a + b);
    if (stab_abs(g, m) <= 1.0) a = m; else b = m;
  }
  return a;
}
