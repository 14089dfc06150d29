/*
 * Oracle (test infrastructure only): a second, independently written DGSEM
 * operator for relaxation model II, in strong form.  For Gauss-Legendre
 * collocation the summation-by-parts identity
 *     omega_i D_ij + omega_j D_ji = l_i(1) l_j(1) - l_i(-1) l_j(-1)
 * makes it algebraically equal to the weak form of Sec. 3.1, so the two agree
 * to rounding; the comparison pins the assembly (signs, transposes, face
 * indexing) of the weak-form operator.
 *
 *   Q_i = (2/h) [ (D w)_i + (L+_i (w*_+ - w_+) - L-_i (w*_- - w_-)) / omega_i ]
 *   R_i = -(2/h) [ (D F)_i + (L+_i (F*_+ - F_+) - L-_i (F*_- - F_-)) / omega_i ] + S_i
 *
 * with w_+-, F_+- the element's own traces of the nodal polynomials.
 * Indexing is written out with explicit (i, j, k) loops and shares nothing
 * with the weak-form file.
 */
#include <math.h>
#include <stdlib.h>
#include "oracle.h"

typedef struct {
  int dim, np, n[3], nel[3];
  long E;
  int nn;
  double* h[3]; /* widths per element index per direction */
  or_basis b;
} sgeo;

static long eidx(const sgeo* g, int ex, int ey, int ez) { return ex + (long)g->nel[0] * (ey + (long)g->nel[1] * ez); }
static int nidx(const sgeo* g, int i, int j, int k) { return i + g->np * (j + g->np * k); }

/* value of array a (one variable, [E][nn]) at element (ex,ey,ez), node whose
 * index in direction d is replaced by l */
static double at_line(const sgeo* g, const double* a, const int E3[3], const int I3[3], int d, int l) {
  int I[3] = {I3[0], I3[1], I3[2]};
  I[d] = l;
  return a[eidx(g, E3[0], E3[1], E3[2]) * g->nn + nidx(g, I[0], I[1], I[2])];
}

/* trace on side s (0: -1, 1: +1) in direction d of the element shifted by
 * sh in direction d, on the line through node I3 */
static double line_trace(const sgeo* g, const double* a, const int E3[3], const int I3[3], int d, int sh, int s) {
  int E[3] = {E3[0], E3[1], E3[2]};
  E[d] = (E[d] + sh + g->nel[d]) % g->nel[d];
  const double* L = s ? g->b.Lp : g->b.Lm;
  double t = 0.0;
  for (int l = 0; l < g->np; ++l) t += L[l] * at_line(g, a, E, I3, d, l);
  return t;
}

static double pressure_alpha(const or_prob* P, double r) {
  /* reduced Van-der-Waals: p = 8 T r / (3 - r) - 3 r^2, plus alpha r^2 / 2 */
  return 8.0 * P->T * r / (3.0 - r) - 3.0 * r * r + 0.5 * P->alpha * r * r;
}
static double sound(const or_prob* P, double r) {
  double dp = 24.0 * P->T / ((3.0 - r) * (3.0 - r)) - 6.0 * r;
  return sqrt(dp + P->alpha * r);
}

/* Convective numerical flux (fL, fR: physical fluxes of the two states).
 * Rusanov: central flux minus lam (uR - uL)/2.  HLLC, written with the
 * star states of the barotropic system: with the Davis speeds SL, SR and the
 * HLL averages rho_hll, m_hll (normal momentum) and c_hll, the star state on
 * side K is (rho_hll, m_hll, rho_hll v_t,K, c_hll); the contact moves with
 * S* = F_hll[rho] / rho_hll and the flux is F_K + S_K (U*_K - U_K) with K the
 * side of the contact that holds the face (K = L if S* >= 0). */
static void convective_numflux(const or_prob* P, int dim, int d, const double* uL, const double* uR,
                               const double* fL, const double* fR, double* Fc) {
  const int nv = dim + 2;
  if (P->flux == 0) {
    double sL = fabs(uL[1 + d] / uL[0]) + sound(P, uL[0]);
    double sR = fabs(uR[1 + d] / uR[0]) + sound(P, uR[0]);
    double lam = sL > sR ? sL : sR;
    for (int q = 0; q < nv; ++q) {
      double diss = (q == dim + 1 && !P->diss_c) ? 0.0 : lam * (uR[q] - uL[q]);
      Fc[q] = 0.5 * (fL[q] + fR[q]) - 0.5 * diss;
    }
    return;
  }
  double unL = uL[1 + d] / uL[0], unR = uR[1 + d] / uR[0];
  double SL = unL - sound(P, uL[0]), SR = unR + sound(P, uR[0]);
  if (unR - sound(P, uR[0]) < SL) SL = unR - sound(P, uR[0]);
  if (unL + sound(P, uL[0]) > SR) SR = unL + sound(P, uL[0]);
  if (SL >= 0.0 || SR <= 0.0) {
    const double* f = SL >= 0.0 ? fL : fR;
    for (int q = 0; q < nv; ++q) Fc[q] = f[q];
    return;
  }
  /* HLL averages: (SR uR - SL uL - (fR - fL)) / (SR - SL) */
  double hll[5];
  for (int q = 0; q < nv; ++q) hll[q] = (SR * uR[q] - SL * uL[q] - (fR[q] - fL[q])) / (SR - SL);
  /* HLL mass flux and contact speed */
  double Fmass = fL[0] + SL * (hll[0] - uL[0]);
  double Sstar = Fmass / hll[0];
  const double* uK = Sstar >= 0.0 ? uL : uR;
  const double* fK = Sstar >= 0.0 ? fL : fR;
  double SK = Sstar >= 0.0 ? SL : SR;
  double star[5];
  star[0] = hll[0];
  for (int j = 0; j < dim; ++j) star[1 + j] = j == d ? hll[1 + d] : hll[0] * uK[1 + j] / uK[0];
  star[dim + 1] = hll[dim + 1];
  for (int q = 0; q < nv; ++q) Fc[q] = fK[q] + SK * (star[q] - uK[q]);
  if (!P->diss_c) Fc[dim + 1] = 0.0;
}

int or_rhs_strong(const or_prob* P, const double* U, double* R) {
  sgeo g;
  g.dim = P->dim;
  g.np = P->N + 1;
  if (or_make_basis(P->N, &g.b)) return -1;
  g.E = 1;
  g.nn = 1;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = d < g.dim ? g.np : 1;
    g.nel[d] = d < g.dim ? P->nel[d] : 1;
    g.E *= g.nel[d];
    g.nn *= g.n[d];
    g.h[d] = malloc(sizeof(double) * g.nel[d]);
    for (int q = 0; q < g.nel[d]; ++q) g.h[d][q] = d < g.dim ? P->xb[d][q + 1] - P->xb[d][q] : 1.0;
  }
  const int dim = g.dim, nv = dim + 2, nl = dim + 1;
  const size_t S = (size_t)g.E * g.nn;
  double* w = malloc(sizeof(double) * nl * S);
  double* Q = malloc(sizeof(double) * dim * nl * S);  /* Q[d][k] */
  double* F = malloc(sizeof(double) * dim * nv * S);  /* total flux Fc - Fv */
  double* Fv = malloc(sizeof(double) * dim * nv * S); /* viscous flux      */

  for (size_t o = 0; o < S; ++o) {
    for (int d = 0; d < dim; ++d) w[d * S + o] = U[(1 + d) * S + o] / U[o];
    w[dim * S + o] = U[(dim + 1) * S + o];
  }

  /* strong-form BR1 lifting */
#pragma omp parallel for collapse(3)
  for (int ez = 0; ez < g.nel[2]; ++ez)
    for (int ey = 0; ey < g.nel[1]; ++ey)
      for (int ex = 0; ex < g.nel[0]; ++ex) {
        int E3[3] = {ex, ey, ez};
        long e = eidx(&g, ex, ey, ez);
        for (int k = 0; k < g.n[2]; ++k)
          for (int j = 0; j < g.n[1]; ++j)
            for (int i = 0; i < g.n[0]; ++i) {
              int I3[3] = {i, j, k};
              int node = nidx(&g, i, j, k);
              for (int d = 0; d < dim; ++d) {
                int id = I3[d];
                double fac = 2.0 / g.h[d][E3[d]];
                for (int q = 0; q < nl; ++q) {
                  const double* a = w + q * S;
                  double Dw = 0.0;
                  for (int l = 0; l < g.np; ++l) Dw += g.b.D[id][l] * at_line(&g, a, E3, I3, d, l);
                  double own_p = line_trace(&g, a, E3, I3, d, 0, 1);
                  double own_m = line_trace(&g, a, E3, I3, d, 0, 0);
                  double nb_p = line_trace(&g, a, E3, I3, d, +1, 0);
                  double nb_m = line_trace(&g, a, E3, I3, d, -1, 1);
                  double star_p = 0.5 * (own_p + nb_p), star_m = 0.5 * (own_m + nb_m);
                  Q[((size_t)d * nl + q) * S + e * g.nn + node] =
                      fac * (Dw + (g.b.Lp[id] * (star_p - own_p) - g.b.Lm[id] * (star_m - own_m)) / g.b.w[id]);
                }
              }
            }
      }

  /* nodal fluxes */
  for (size_t o = 0; o < S; ++o) {
    double r = U[o];
    double pa = pressure_alpha(P, r);
    double div = 0.0;
    for (int d = 0; d < dim; ++d) div += Q[((size_t)d * nl + d) * S + o];
    for (int d = 0; d < dim; ++d) {
      double md = U[(1 + d) * S + o];
      /* rho row */
      F[((size_t)d * nv + 0) * S + o] = md;
      Fv[((size_t)d * nv + 0) * S + o] = 0.0;
      /* momentum rows j: m_d m_j / rho + delta p_alpha - tau_jd */
      for (int j = 0; j < dim; ++j) {
        double tau = P->eps * (Q[((size_t)d * nl + j) * S + o] + Q[((size_t)j * nl + d) * S + o]);
        if (j == d) tau -= P->eps * 2.0 / 3.0 * div;
        double conv = md * U[(1 + j) * S + o] / r + (j == d ? pa : 0.0);
        F[((size_t)d * nv + 1 + j) * S + o] = conv - tau;
        Fv[((size_t)d * nv + 1 + j) * S + o] = tau;
      }
      /* c row: convective 0, viscous (kappa/beta) dc/dx_d */
      double fc = P->kappa / P->beta * Q[((size_t)d * nl + dim) * S + o];
      F[((size_t)d * nv + dim + 1) * S + o] = -fc;
      Fv[((size_t)d * nv + dim + 1) * S + o] = fc;
    }
  }

  /* numerical flux at the face between left element EL and right element ER
   * along direction d, line through I3; result for all nv variables */
#pragma omp parallel for collapse(3)
  for (int ez = 0; ez < g.nel[2]; ++ez)
    for (int ey = 0; ey < g.nel[1]; ++ey)
      for (int ex = 0; ex < g.nel[0]; ++ex) {
        int E3[3] = {ex, ey, ez};
        long e = eidx(&g, ex, ey, ez);
        for (int k = 0; k < g.n[2]; ++k)
          for (int j = 0; j < g.n[1]; ++j)
            for (int i = 0; i < g.n[0]; ++i) {
              int I3[3] = {i, j, k};
              int node = nidx(&g, i, j, k);
              double acc[5] = {0, 0, 0, 0, 0};
              for (int d = 0; d < dim; ++d) {
                int id = I3[d];
                double fac = 2.0 / g.h[d][E3[d]];
                /* faces: side +1 (own right, neighbour +1 left) and side -1 */
                double Fstar[2][5];
                for (int side = 0; side < 2; ++side) {
                  int shL = side ? 0 : -1, shR = side ? +1 : 0;
                  double uL[5], uR[5], vL[5], vR[5];
                  for (int q = 0; q < nv; ++q) {
                    uL[q] = line_trace(&g, U + q * S, E3, I3, d, shL, 1);
                    uR[q] = line_trace(&g, U + q * S, E3, I3, d, shR, 0);
                    vL[q] = line_trace(&g, Fv + ((size_t)d * nv + q) * S, E3, I3, d, shL, 1);
                    vR[q] = line_trace(&g, Fv + ((size_t)d * nv + q) * S, E3, I3, d, shR, 0);
                  }
                  double fL[5], fR[5];
                  fL[0] = uL[1 + d];
                  fR[0] = uR[1 + d];
                  for (int jj = 0; jj < dim; ++jj) {
                    fL[1 + jj] = uL[1 + d] * uL[1 + jj] / uL[0] + (jj == d ? pressure_alpha(P, uL[0]) : 0.0);
                    fR[1 + jj] = uR[1 + d] * uR[1 + jj] / uR[0] + (jj == d ? pressure_alpha(P, uR[0]) : 0.0);
                  }
                  fL[dim + 1] = fR[dim + 1] = 0.0;
                  double Fc[5];
                  convective_numflux(P, dim, d, uL, uR, fL, fR, Fc);
                  for (int q = 0; q < nv; ++q) Fstar[side][q] = Fc[q] - 0.5 * (vL[q] + vR[q]);
                }
                for (int q = 0; q < nv; ++q) {
                  const double* a = F + ((size_t)d * nv + q) * S;
                  double DF = 0.0;
                  for (int l = 0; l < g.np; ++l) DF += g.b.D[id][l] * at_line(&g, a, E3, I3, d, l);
                  double own_p = line_trace(&g, a, E3, I3, d, 0, 1);
                  double own_m = line_trace(&g, a, E3, I3, d, 0, 0);
                  acc[q] -= fac * (DF + (g.b.Lp[id] * (Fstar[1][q] - own_p) - g.b.Lm[id] * (Fstar[0][q] - own_m)) / g.b.w[id]);
                }
              }
              size_t o = (size_t)e * g.nn + node;
              double r = U[o], c = U[(dim + 1) * S + o];
              for (int q = 0; q < nv; ++q) R[q * S + o] = acc[q];
              for (int d = 0; d < dim; ++d) R[(1 + d) * S + o] += P->alpha * r * Q[((size_t)d * nl + dim) * S + o];
              R[(dim + 1) * S + o] += P->alpha / P->beta * (r - c);
            }
      }
  free(w); free(Q); free(F); free(Fv);
  for (int d = 0; d < 3; ++d) free(g.h[d]);
  return 0;
}
