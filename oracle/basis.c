/*
 * Oracle (test infrastructure only): one-dimensional nodal basis of the DGSEM
 * (Sec. 3.1, the tensor-product Lagrange basis on Gauss-Legendre nodes and the
 * collocated Gauss quadrature of the weak form).
 *
 * Everything is computed in long double and rounded once at the end.
 */
#include <math.h>
#include <string.h>
#include "oracle.h"

/* Legendre polynomial P_n(x) and its derivative by the three-term recurrence. */
static void legendre(int n, long double x, long double* P, long double* dP) {
  long double p0 = 1.0L, p1 = x;
  if (n == 0) { *P = 1.0L; *dP = 0.0L; return; }
  for (int k = 2; k <= n; ++k) {
    long double p2 = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *P = p1;
  /* derivative from (1 - x^2) P_n' = n (P_{n-1} - x P_n) */
  *dP = n * (p0 - x * p1) / (1.0L - x * x);
}

int or_make_basis(int N, or_basis* b) {
  if (N < 0 || N > OR_NMAX) return -1;
  memset(b, 0, sizeof(*b));
  b->N = N;
  const int n = N + 1;
  long double x[OR_NMAX + 1], w[OR_NMAX + 1];

  /* Gauss-Legendre nodes: the n roots of P_n, by Newton from Chebyshev guesses. */
  if (n == 1) {
    x[0] = 0.0L;
    w[0] = 2.0L;
  } else {
    for (int i = 0; i < n; ++i) {
      long double z = -cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
      for (int it = 0; it < 100; ++it) {
        long double P, dP;
        legendre(n, z, &P, &dP);
        long double dz = P / dP;
        z -= dz;
        if (fabsl(dz) < 1e-19L) break;
      }
      long double P, dP;
      legendre(n, z, &P, &dP);
      x[i] = z;
      w[i] = 2.0L / ((1.0L - z * z) * dP * dP);
    }
  }

  /* Barycentric weights lambda_j = 1 / prod_{k != j} (x_j - x_k). */
  long double lam[OR_NMAX + 1];
  for (int j = 0; j < n; ++j) {
    long double prod = 1.0L;
    for (int k = 0; k < n; ++k)
      if (k != j) prod *= (x[j] - x[k]);
    lam[j] = 1.0L / prod;
  }

  /* Differentiation matrix D_ij = l_j'(x_i); the diagonal is the negative row
   * sum so that the derivative of a constant is exactly zero. */
  long double D[OR_NMAX + 1][OR_NMAX + 1];
  for (int i = 0; i < n; ++i) {
    long double s = 0.0L;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      D[i][j] = (lam[j] / lam[i]) / (x[i] - x[j]);
      s += D[i][j];
    }
    D[i][i] = -s;
  }

  /* Values of the Lagrange polynomials at the element ends, l_j(+-1). */
  for (int j = 0; j < n; ++j) {
    long double lm = 1.0L, lp = 1.0L;
    for (int k = 0; k < n; ++k) {
      if (k == j) continue;
      lm *= (-1.0L - x[k]) / (x[j] - x[k]);
      lp *= (1.0L - x[k]) / (x[j] - x[k]);
    }
    b->Lm[j] = (double)lm;
    b->Lp[j] = (double)lp;
  }

  for (int i = 0; i < n; ++i) {
    b->xi[i] = (double)x[i];
    b->w[i] = (double)w[i];
    for (int j = 0; j < n; ++j) {
      b->D[i][j] = (double)D[i][j];
      /* weak-form volume operator: integration by parts moves the derivative
       * onto the test function l_i, sum_j w_j l_i'(x_j) F_j / w_i */
      b->Dhat[i][j] = (double)(w[j] / w[i] * D[j][i]);
    }
  }
  return 0;
}
