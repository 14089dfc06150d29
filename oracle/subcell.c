/*
 * Oracle (test infrastructure only): finite-volume sub-cell shock capturing
 * for relaxation model II (Sec. 3.2), on top of the weak-form DGSEM of
 * dg_weak.c.
 *
 * Troubled elements: the Persson-Peraire indicator of rho, log10 of the
 * share of the modal energy in the highest modes (orthonormal Legendre
 * expansion, modes whose largest one-direction degree is N), above a
 * threshold.  A troubled element is treated on (N+1)^dim equidistant
 * sub-cells:
 *   - sub-cell means u_bar = M u per direction, M[k][j] = mean of l_j over
 *     sub-cell k (exact Gauss integration), and back u = M^{-1} u_bar;
 *   - d u_bar/dt = sum_d (F*_{d,-} - F*_{d,+}) / dx_d + S(u_bar), dx_d = h_d/(N+1);
 *   - inside the element and on faces shared with another troubled element:
 *     second-order reconstruction of the primitives (rho, v, c) with the
 *     MinMod limiter, the Rusanov flux, and the viscous flux from face
 *     gradients, each the mean of the two adjacent sub-cell gradients, which
 *     are central differences of sub-cell means (the Green-Gauss gradient
 *     with face values the means of the two adjacent cells);
 *   - on faces shared with a DG element: the mean over each sub-face of the
 *     DG face-flux polynomial, the one through the Gauss-point fluxes the DG
 *     element itself uses, so the two sides exchange the same mass;
 *   - the source (0, alpha rho grad c, (alpha/beta)(rho - c)) at the
 *     sub-cell means with the sub-cell gradient of c.
 * The element's right-hand side is M^{-1} applied to the sub-cell rates, so
 * that a Runge-Kutta stage on the nodal values advances the means exactly.
 * Neighbouring sub-cells across the element boundary (reconstruction and
 * gradient stencils) are the neighbour element's sub-cell means.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "geom.h"

/* Orthonormal Legendre polynomial of degree k at x (three-term recurrence). */
static double legendre_on(int k, double x) {
  double p0 = 1.0, p1 = x;
  if (k == 0) return sqrt(0.5);
  for (int n = 2; n <= k; ++n) {
    double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
    p0 = p1;
    p1 = p2;
  }
  return sqrt(k + 0.5) * p1;
}

/* M[k][j]: mean of the Lagrange polynomial l_j over sub-cell k of [-1, 1]
 * (N+1 equal sub-cells), by (N+1)-point Gauss quadrature on the sub-cell;
 * Minv its inverse (Gauss-Jordan with partial pivoting). */
int or_subcell_matrices(int N, double* M, double* Minv) {
  or_basis b;
  if (or_make_basis(N, &b)) return -1;
  const int np = N + 1;
  const double dxi = 2.0 / np;
  for (int k = 0; k < np; ++k)
    for (int j = 0; j < np; ++j) {
      double s = 0.0;
      for (int q = 0; q < np; ++q) {
        double x = -1.0 + dxi * (k + 0.5 * (b.xi[q] + 1.0));
        /* l_j(x) by the Lagrange product formula */
        double l = 1.0;
        for (int m = 0; m < np; ++m)
          if (m != j) l *= (x - b.xi[m]) / (b.xi[j] - b.xi[m]);
        s += 0.5 * b.w[q] * l;
      }
      M[k * np + j] = s;
    }
  double A[OR_NMAX + 1][2 * (OR_NMAX + 1)];
  for (int i = 0; i < np; ++i)
    for (int j = 0; j < 2 * np; ++j) A[i][j] = j < np ? M[i * np + j] : (j - np == i ? 1.0 : 0.0);
  for (int c = 0; c < np; ++c) {
    int p = c;
    for (int r = c + 1; r < np; ++r)
      if (fabs(A[r][c]) > fabs(A[p][c])) p = r;
    for (int j = 0; j < 2 * np; ++j) {
      double t = A[c][j];
      A[c][j] = A[p][j];
      A[p][j] = t;
    }
    double piv = A[c][c];
    if (fabs(piv) < 1e-300) return -1;
    for (int j = 0; j < 2 * np; ++j) A[c][j] /= piv;
    for (int r = 0; r < np; ++r)
      if (r != c) {
        double f = A[r][c];
        for (int j = 0; j < 2 * np; ++j) A[r][j] -= f * A[c][j];
      }
  }
  for (int i = 0; i < np; ++i)
    for (int j = 0; j < np; ++j) Minv[i * np + j] = A[i][np + j];
  return 0;
}

/* Persson-Peraire indicator of rho per element: log10 of
 * sum_{modes with max index N} c^2 / sum_{all modes} c^2 (-99 for zero). */
int or_persson(const or_prob* P, const double* U, double* ind) {
  or_geom g;
  if (or_geom_init(&g, P)) return -1;
  const int np = g.np, nn = g.nnode, dim = g.dim;
  double V[OR_NMAX + 1][OR_NMAX + 1]; /* V[k][i] = w_i P_k(xi_i) */
  for (int k = 0; k < np; ++k)
    for (int i = 0; i < np; ++i) V[k][i] = g.b.w[i] * legendre_on(k, g.b.xi[i]);
  for (long e = 0; e < g.E; ++e) {
    const double* u = U + (size_t)e * nn;
    double tot = 0.0, top = 0.0;
    for (int mode = 0; mode < nn; ++mode) {
      int km[3] = {0, 0, 0}, r = mode, kmax = 0;
      for (int d = 0; d < dim; ++d) { km[d] = r % np; r /= np; if (km[d] > kmax) kmax = km[d]; }
      double c = 0.0;
      for (int n = 0; n < nn; ++n) {
        int in[3] = {0, 0, 0}, q = n;
        double f = 1.0;
        for (int d = 0; d < dim; ++d) { in[d] = q % np; q /= np; f *= V[km[d]][in[d]]; }
        c += f * u[n];
      }
      tot += c * c;
      if (kmax == np - 1) top += c * c;
    }
    ind[e] = (top > 0.0 && tot > 0.0) ? log10(top / tot) : -99.0;
  }
  return 0;
}

static double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) < fabs(b) ? a : b;
}

/* primitives (rho, v_1..v_dim, c) from conserved values */
static void to_prim(int dim, const double* u, double* w) {
  w[0] = u[0];
  for (int d = 0; d < dim; ++d) w[1 + d] = u[1 + d] / u[0];
  w[dim + 1] = u[dim + 1];
}
static void to_cons(int dim, const double* w, double* u) {
  u[0] = w[0];
  for (int d = 0; d < dim; ++d) u[1 + d] = w[0] * w[1 + d];
  u[dim + 1] = w[dim + 1];
}

/* Sub-cell means of every element: Ub[v][e][sub-cell], sub-cells indexed
 * like nodes (x fastest). */
static void subcell_means(const or_geom* g, const double* M, const double* U, double* Ub) {
  const int np = g->np, nn = g->nnode, dim = g->dim, nv = g->nvar;
  const size_t S = (size_t)g->E * nn;
  for (int v = 0; v < nv; ++v)
    for (long e = 0; e < g->E; ++e)
      for (int k = 0; k < nn; ++k) {
        int kk[3] = {0, 0, 0}, r = k;
        for (int d = 0; d < dim; ++d) { kk[d] = r % np; r /= np; }
        double s = 0.0;
        for (int n = 0; n < nn; ++n) {
          int in[3] = {0, 0, 0}, q = n;
          double f = 1.0;
          for (int d = 0; d < dim; ++d) { in[d] = q % np; q /= np; f *= M[kk[d] * np + in[d]]; }
          s += f * U[v * S + (size_t)e * nn + n];
        }
        Ub[v * S + (size_t)e * nn + k] = s;
      }
}

/* index of the sub-cell next to sub-cell k of element e in direction d,
 * side s (-1/+1), possibly in the neighbouring element: (element, sub-cell) */
static void sub_neighbor(const or_geom* g, long e, int k, int d, int s, long* en, int* kn) {
  int kk[3] = {0, 0, 0}, r = k;
  for (int dd = 0; dd < g->dim; ++dd) { kk[dd] = r % g->np; r /= g->np; }
  kk[d] += s;
  long ee = e;
  if (kk[d] < 0) { kk[d] = g->np - 1; ee = or_neighbor(g, e, d, -1); }
  if (kk[d] >= g->np) { kk[d] = 0; ee = or_neighbor(g, e, d, +1); }
  *en = ee;
  *kn = kk[0] + g->np * (kk[1] + g->np * kk[2]);
}

/* central-difference gradient of the primitives (v, c) at sub-cell k of
 * element e: grad[dd][j], j over (v_1..v_dim, c) */
static void sub_gradient(const or_geom* g, const double* Ub, long e, int k, double grad[3][4]) {
  const int dim = g->dim;
  const size_t S = (size_t)g->E * g->nnode;
  for (int dd = 0; dd < dim; ++dd) {
    long em, ep;
    int km, kp;
    sub_neighbor(g, e, k, dd, -1, &em, &km);
    sub_neighbor(g, e, k, dd, +1, &ep, &kp);
    double um[5], up[5], wm[5], wp[5];
    for (int v = 0; v < g->nvar; ++v) {
      um[v] = Ub[v * S + (size_t)em * g->nnode + km];
      up[v] = Ub[v * S + (size_t)ep * g->nnode + kp];
    }
    to_prim(dim, um, wm);
    to_prim(dim, up, wp);
    double dx = or_width(g, e, dd) / g->np;
    for (int j = 0; j <= dim; ++j) grad[dd][j] = (wp[1 + j] - wm[1 + j]) / (2.0 * dx);
  }
}

/* viscous flux (0, tau_{.d}, (kappa/beta) dc/dx_d) from primitive gradients */
static void visc_flux(const or_prob* P, int dim, int d, double q[3][4], double* F) {
  double div = 0.0;
  for (int j = 0; j < dim; ++j) div += q[j][j];
  F[0] = 0.0;
  for (int j = 0; j < dim; ++j) F[1 + j] = P->eps * (q[d][j] + q[j][d] - (j == d ? 2.0 / 3.0 * div : 0.0));
  F[dim + 1] = P->kappa / P->beta * q[d][dim];
}

/* FV flux across the face between sub-cell a (left) and b (right) in
 * direction d; am/bp are the sub-cells beyond a and b. */
static void fv_flux(const or_prob* P, const or_geom* g, const double* Ub, long ea, int ka, long eb, int kb, int d,
                    double* F) {
  const int dim = g->dim, nv = g->nvar;
  const size_t S = (size_t)g->E * g->nnode;
  long eam, ebp;
  int kam, kbp;
  sub_neighbor(g, ea, ka, d, -1, &eam, &kam);
  sub_neighbor(g, eb, kb, d, +1, &ebp, &kbp);
  double u[4][5], w[4][5];
  const long es[4] = {eam, ea, eb, ebp};
  const int ks[4] = {kam, ka, kb, kbp};
  for (int t = 0; t < 4; ++t) {
    for (int v = 0; v < nv; ++v) u[t][v] = Ub[v * S + (size_t)es[t] * g->nnode + ks[t]];
    to_prim(dim, u[t], w[t]);
  }
  double wL[5], wR[5], uL[5], uR[5];
  for (int v = 0; v < nv; ++v) {
    wL[v] = w[1][v] + 0.5 * minmod(w[1][v] - w[0][v], w[2][v] - w[1][v]);
    wR[v] = w[2][v] - 0.5 * minmod(w[2][v] - w[1][v], w[3][v] - w[2][v]);
  }
  to_cons(dim, wL, uL);
  to_cons(dim, wR, uR);
  or_numflux(P, d, uL, uR, F);
  double ga[3][4], gb[3][4], q[3][4], fv[5];
  sub_gradient(g, Ub, ea, ka, ga);
  sub_gradient(g, Ub, eb, kb, gb);
  for (int i = 0; i < dim; ++i)
    for (int j = 0; j <= dim; ++j) q[i][j] = 0.5 * (ga[i][j] + gb[i][j]);
  visc_flux(P, dim, d, q, fv);
  for (int v = 0; v < nv; ++v) F[v] -= fv[v];
}

/* DG face flux at the Gauss point f of the face between element e (left)
 * and eR (right) in direction d: Rusanov/HLLC of the traces minus the mean
 * of the traced viscous fluxes, as in the weak-form operator. */
static void dg_face_flux(const or_prob* P, const or_geom* g, const double* U, const double* Fv, long e, long eR,
                         int d, int f, double* F) {
  const int nv = g->nvar, nn = g->nnode;
  const size_t S = (size_t)g->E * nn;
  double uL[5], uR[5], vL[5], vR[5];
  for (int v = 0; v < nv; ++v) {
    uL[v] = uR[v] = vL[v] = vR[v] = 0.0;
    for (int l = 0; l < g->np; ++l) {
      int nl = or_line_node(g, d, f, l);
      uL[v] += g->b.Lp[l] * U[v * S + (size_t)e * nn + nl];
      uR[v] += g->b.Lm[l] * U[v * S + (size_t)eR * nn + nl];
      vL[v] += g->b.Lp[l] * Fv[((size_t)d * nv + v) * S + (size_t)e * nn + nl];
      vR[v] += g->b.Lm[l] * Fv[((size_t)d * nv + v) * S + (size_t)eR * nn + nl];
    }
  }
  or_numflux(P, d, uL, uR, F);
  for (int v = 0; v < nv; ++v) F[v] -= 0.5 * (vL[v] + vR[v]);
}

int or_rhs_subcell(const or_prob* P, const double* U, double threshold, double* R, int* flags) {
  or_geom g;
  if (or_geom_init(&g, P)) return -1;
  const int dim = g.dim, nv = g.nvar, nl = g.nlift, nn = g.nnode, np = g.np, nf = g.nf;
  const size_t S = (size_t)g.E * nn;
  double M[(OR_NMAX + 1) * (OR_NMAX + 1)], Minv[(OR_NMAX + 1) * (OR_NMAX + 1)];
  if (or_subcell_matrices(P->N, M, Minv)) return -1;

  /* DG right-hand side of every element, with the lifted gradients */
  double* Q = malloc(sizeof(double) * dim * nl * S);
  if (or_rhs_weak(P, U, R, Q)) { free(Q); return -1; }
  double* ind = malloc(sizeof(double) * g.E);
  or_persson(P, U, ind);
  int* tr = malloc(sizeof(int) * g.E);
  for (long e = 0; e < g.E; ++e) tr[e] = ind[e] > threshold;
  if (flags) memcpy(flags, tr, sizeof(int) * g.E);

  /* nodal viscous fluxes of the DG operator (for the DG face fluxes) */
  double* Fv = malloc(sizeof(double) * dim * nv * S);
  for (size_t o = 0; o < S; ++o) {
    double q[3][4], fv[5];
    for (int dd = 0; dd < dim; ++dd)
      for (int k = 0; k < nl; ++k) q[dd][k] = Q[((size_t)dd * nl + k) * S + o];
    for (int d = 0; d < dim; ++d) {
      visc_flux(P, dim, d, q, fv);
      for (int v = 0; v < nv; ++v) Fv[((size_t)d * nv + v) * S + o] = fv[v];
    }
  }
  double* Ub = malloc(sizeof(double) * nv * S);
  subcell_means(&g, M, U, Ub);

  double* rs = malloc(sizeof(double) * nv * nn);  /* sub-cell rates of one element */
  double* fs = malloc(sizeof(double) * nv * nf);  /* DG face fluxes at Gauss points of one face */
  for (long e = 0; e < g.E; ++e) {
    if (!tr[e]) continue;
    for (int i = 0; i < nv * nn; ++i) rs[i] = 0.0;
    for (int d = 0; d < dim; ++d) {
      const double dx = or_width(&g, e, d) / np;
      for (int side = -1; side <= 1; side += 2) {
        /* element-boundary face on this side */
        long en = or_neighbor(&g, e, d, side);
        if (!tr[en]) {
          long eL = side > 0 ? e : en, eR = side > 0 ? en : e;
          for (int f = 0; f < nf; ++f) dg_face_flux(P, &g, U, Fv, eL, eR, d, f, fs + f * nv);
          /* sub-face means of the face-flux polynomial: M along the face's directions */
          for (int fk = 0; fk < nf; ++fk) {
            int kk[3] = {0, 0, 0}, r = fk;
            for (int dd = 0; dd < dim; ++dd) {
              if (dd == d) continue;
              kk[dd] = r % np;
              r /= np;
            }
            double Fm[5] = {0, 0, 0, 0, 0};
            for (int f = 0; f < nf; ++f) {
              int ii[3] = {0, 0, 0}, q = f;
              double wgt = 1.0;
              for (int dd = 0; dd < dim; ++dd) {
                if (dd == d) continue;
                ii[dd] = q % np;
                q /= np;
                wgt *= M[kk[dd] * np + ii[dd]];
              }
              for (int v = 0; v < nv; ++v) Fm[v] += wgt * fs[f * nv + v];
            }
            /* the sub-cell of this element on that face */
            kk[d] = side > 0 ? np - 1 : 0;
            int k = kk[0] + np * (kk[1] + np * kk[2]);
            for (int v = 0; v < nv; ++v) rs[v * nn + k] += (side > 0 ? -Fm[v] : Fm[v]) / dx;
          }
        }
      }
      /* FV faces: inside the element, and on boundaries shared with a troubled neighbour */
      for (int k = 0; k < nn; ++k) {
        int kk[3] = {0, 0, 0}, r = k;
        for (int dd = 0; dd < dim; ++dd) { kk[dd] = r % np; r /= np; }
        /* + face of sub-cell k */
        int at_boundary = kk[d] == np - 1;
        long en;
        int kn;
        sub_neighbor(&g, e, k, d, +1, &en, &kn);
        if (!at_boundary || tr[en]) {
          double F[5];
          fv_flux(P, &g, Ub, e, k, en, kn, d, F);
          for (int v = 0; v < nv; ++v) rs[v * nn + k] -= F[v] / dx;
          if (!at_boundary) for (int v = 0; v < nv; ++v) rs[v * nn + kn] += F[v] / dx;
        }
        /* - face of a boundary sub-cell shared with a troubled neighbour */
        if (kk[d] == 0) {
          long em;
          int km;
          sub_neighbor(&g, e, k, d, -1, &em, &km);
          if (tr[em]) {
            double F[5];
            fv_flux(P, &g, Ub, em, km, e, k, d, F);
            for (int v = 0; v < nv; ++v) rs[v * nn + k] += F[v] / dx;
          }
        }
      }
    }
    /* source at the sub-cell means */
    for (int k = 0; k < nn; ++k) {
      double grad[3][4];
      sub_gradient(&g, Ub, e, k, grad);
      double rho = Ub[(size_t)e * nn + k], c = Ub[(dim + 1) * S + (size_t)e * nn + k];
      for (int d = 0; d < dim; ++d) rs[(1 + d) * nn + k] += P->alpha * rho * grad[d][dim];
      rs[(dim + 1) * nn + k] += P->alpha / P->beta * (rho - c);
    }
    /* nodal right-hand side: M^{-1} per direction */
    for (int v = 0; v < nv; ++v)
      for (int n = 0; n < nn; ++n) {
        int in[3] = {0, 0, 0}, r = n;
        for (int dd = 0; dd < dim; ++dd) { in[dd] = r % np; r /= np; }
        double s = 0.0;
        for (int k = 0; k < nn; ++k) {
          int kk[3] = {0, 0, 0}, q = k;
          double f = 1.0;
          for (int dd = 0; dd < dim; ++dd) { kk[dd] = q % np; q /= np; f *= Minv[in[dd] * np + kk[dd]]; }
          s += f * rs[v * nn + k];
        }
        R[v * S + (size_t)e * nn + n] = s;
      }
  }
  free(Q); free(ind); free(tr); free(Fv); free(Ub); free(rs); free(fs);
  return 0;
}
