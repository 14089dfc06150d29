/*
 * Oracle (test infrastructure only): what the learned closure adds to the
 * relaxation model II right-hand side, and the nudging step that produces its
 * training pairs.  The paper defines no closure; these are the definitions
 * the GPU path implements, written out plainly.
 *
 * Features at a node (element-local, no lifting), from the collocation
 * derivative D of Sec. 3.1 applied along each direction inside the element:
 *   g_d  = (2/h_d) sum_j D_ij rho_j                    (gradient of rho)
 *   lap  = sum_d (2/h_d)^2 sum_l D_il sum_j D_lj rho_j (Laplacian proxy)
 *   x    = ((rho - s0) k0, (c - s1) k1, |g| k2, lap k3)
 *   n    = g / sqrt(|g|^2 + g0^2)
 * Closure source with y = MLP(x):
 *   S_m = out_m y_0 n,   S_c = out_c y_1,   nothing on rho.
 * norm[] packs (s0, k0, s1, k1, k2, k3, g0, out_m, out_c).
 *
 * Nudging step (training pairs): with the reference state mapped into the
 * frame of the cheaper model, U* = (rho_r, m_r, rho_r + cmap (c_r - rho_r)),
 * the step records x(U) and the targets ((m* - m).n / tau, (c* - c) / tau),
 * then moves m and c by (dt / tau)(U* - U).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "geom.h"

/* gradient and Laplacian proxy of rho at every node of element e */
static void rho_derivs(const or_geom* g, long e, const double* rho, double* grad /*[3][nn]*/, double* lap /*[nn]*/) {
  const int np = g->np, nn = g->nnode;
  int stride[3] = {1, np, np * np};
  double first[OR_NMAX + 1];
  for (int n = 0; n < nn; ++n) lap[n] = 0.0;
  for (int d = 0; d < g->dim; ++d) {
    const double s = 2.0 / or_width(g, e, d);
    for (int n = 0; n < nn; ++n) {
      const int i = (n / stride[d]) % np;
      const int base = n - i * stride[d];
      double t = 0.0;
      for (int j = 0; j < np; ++j) t += g->b.D[i][j] * rho[base + j * stride[d]];
      grad[d * nn + n] = s * t;
      /* second derivative along the same line: D applied to the D sweep */
      for (int l = 0; l < np; ++l) {
        double u = 0.0;
        for (int j = 0; j < np; ++j) u += g->b.D[l][j] * rho[base + j * stride[d]];
        first[l] = u;
      }
      double v = 0.0;
      for (int l = 0; l < np; ++l) v += g->b.D[i][l] * first[l];
      lap[n] += s * s * v;
    }
  }
}

int or_closure_features(const or_prob* P, const double* U, const double* norm, double* X, double* nvec) {
  or_geom g;
  if (or_geom_init(&g, P)) return -1;
  const size_t S = (size_t)g.E * g.nnode;
  const int nn = g.nnode;
  int rc = 0;
#pragma omp parallel
  {
    double* grad = malloc(sizeof(double) * 3 * nn);
    double* lap = malloc(sizeof(double) * nn);
    if (!grad || !lap) rc = -1;
#pragma omp for
    for (long e = 0; e < g.E; ++e) {
      if (!grad || !lap) continue;
      const double* rho = U + (size_t)e * nn;
      rho_derivs(&g, e, rho, grad, lap);
      for (int n = 0; n < nn; ++n) {
        const size_t o = (size_t)e * nn + n;
        double gg = 0.0;
        for (int d = 0; d < g.dim; ++d) gg += grad[d * nn + n] * grad[d * nn + n];
        const double c = U[(size_t)(g.dim + 1) * S + o];
        if (X) {
          X[o * 4 + 0] = (rho[n] - norm[0]) * norm[1];
          X[o * 4 + 1] = (c - norm[2]) * norm[3];
          X[o * 4 + 2] = sqrt(gg) * norm[4];
          X[o * 4 + 3] = lap[n] * norm[5];
        }
        if (nvec) {
          const double den = sqrt(gg + norm[6] * norm[6]);
          for (int d = 0; d < g.dim; ++d) nvec[d * S + o] = grad[d * nn + n] / den;
        }
      }
    }
    free(grad);
    free(lap);
  }
  return rc;
}

int or_closure_source(const or_prob* P, const double* U, const double* w, const double* norm, double* Sc) {
  or_geom g;
  if (or_geom_init(&g, P)) return -1;
  const size_t S = (size_t)g.E * g.nnode;
  double* X = malloc(sizeof(double) * 4 * S);
  double* nv = malloc(sizeof(double) * g.dim * S);
  double* Y = malloc(sizeof(double) * 2 * S);
  int rc = (X && nv && Y) ? 0 : -1;
  if (!rc) rc = or_closure_features(P, U, norm, X, nv);
  if (!rc) {
    or_mlp_forward(w, X, (long)S, Y);
    memset(Sc, 0, sizeof(double) * g.nvar * S);
    for (size_t o = 0; o < S; ++o) {
      for (int d = 0; d < g.dim; ++d) Sc[(1 + d) * S + o] = norm[7] * Y[o * 2 + 0] * nv[d * S + o];
      Sc[(g.dim + 1) * S + o] = norm[8] * Y[o * 2 + 1];
    }
  }
  free(X);
  free(nv);
  free(Y);
  return rc;
}

int or_closure_nudge(const or_prob* P, double* U, const double* Uref, double dt, double tau, double cmap,
                     const double* norm, double* X, double* Y) {
  or_geom g;
  if (or_geom_init(&g, P) || !(tau > 0.0)) return -1;
  const size_t S = (size_t)g.E * g.nnode;
  double* nv = malloc(sizeof(double) * g.dim * S);
  if (!nv) return -1;
  int rc = or_closure_features(P, U, norm, X, nv);
  if (!rc) {
    const int ic = g.dim + 1;
    for (size_t o = 0; o < S; ++o) {
      const double cstar = Uref[o] + cmap * (Uref[ic * S + o] - Uref[o]);
      double dm_n = 0.0;
      for (int d = 0; d < g.dim; ++d) dm_n += (Uref[(1 + d) * S + o] - U[(1 + d) * S + o]) * nv[d * S + o];
      const double dc = cstar - U[ic * S + o];
      if (Y) {
        Y[o * 2 + 0] = dm_n / tau;
        Y[o * 2 + 1] = dc / tau;
      }
      for (int d = 0; d < g.dim; ++d) U[(1 + d) * S + o] += dt / tau * (Uref[(1 + d) * S + o] - U[(1 + d) * S + o]);
      U[ic * S + o] += dt / tau * dc;
    }
  }
  free(nv);
  return rc;
}
