/*
 * Oracle (test infrastructure only): the DGSEM semi-discretisation of
 * relaxation model II (Sec. 2.3, the model II fluxes, source and modified
 * pressure p_alpha = p + alpha rho^2 / 2) on a periodic tensor-product grid of
 * affine box elements, in the weak form of Sec. 3.1:
 *
 *   J U_t - int F . grad_xi(phi) + surface int (F.n)* phi = J S,
 *
 * with Gauss-Legendre collocation, a local Lax-Friedrichs (Rusanov) or HLLC
 * flux for the convective part, BR1 lifting of the primitive variables (v, c) with the
 * central flux, the arithmetic mean of the viscous fluxes on faces, and the
 * non-conservative source evaluated pointwise from the lifted gradient of c
 * (end of Sec. 3.1).  It also holds the time loop, the time-step rule and the
 * diagnostics.
 *
 * Step order of one right-hand side evaluation:
 *   1. nodal primitives w = (v_1..v_d, c)
 *   2. BR1 lifting Q_d = dw/dx_d (volume part with Dhat, surface part with the
 *      central trace w* = (w- + w+)/2)
 *   3. nodal fluxes  F_d = Fc_d(U) - Fv_d(Q)
 *   4. face fluxes F*_d = Rusanov or HLLC(U-, U+) - (Fv_d(Q-) + Fv_d(Q+))/2
 *   5. R = sum_d (2/h_d) [Dhat F_d - (L+ F*_+ - L- F*_-)/w] + S
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "geom.h"

/* ------------------------------------------------------------------------ */
/* Step 1: primitives w = (v_1..v_dim, c) at every node.                    */
static void primitives(const or_geom* g, const double* U, double* w) {
  const size_t S = (size_t)g->E * g->nnode;
#pragma omp parallel for
  for (long e = 0; e < g->E; ++e)
    for (int n = 0; n < g->nnode; ++n) {
      size_t o = (size_t)e * g->nnode + n;
      double rho = U[o];
      for (int d = 0; d < g->dim; ++d) w[d * S + o] = U[(1 + d) * S + o] / rho;
      w[g->dim * S + o] = U[(g->dim + 1) * S + o];
    }
}

/* Trace of the nodal polynomial a[e][.] on face side s (0: xi_d = -1,
 * 1: xi_d = +1) at face node f: sum_l l_l(+-1) a(l). */
static double trace(const or_geom* g, const double* a, long e, int d, int s, int f) {
  const double* L = s ? g->b.Lp : g->b.Lm;
  double t = 0.0;
  for (int l = 0; l < g->np; ++l) t += L[l] * a[(size_t)e * g->nnode + or_line_node(g, d, f, l)];
  return t;
}

/* ------------------------------------------------------------------------ */
/* Step 2: BR1 lifting of w.  For each direction d and node i on its line:
 *   Q_d,i = (2/h_d) [ -sum_l Dhat_il w_l + (L+_i w*_+ - L-_i w*_-) / omega_i ] */
static void lift(const or_geom* g, const double* w, double* Q) {
  const size_t S = (size_t)g->E * g->nnode;
  for (int d = 0; d < g->dim; ++d)
    for (int k = 0; k < g->nlift; ++k) {
      const double* wk = w + k * S;
      double* Qdk = Q + ((size_t)d * g->nlift + k) * S;
#pragma omp parallel for
      for (long e = 0; e < g->E; ++e) {
        long eL = or_neighbor(g, e, d, -1), eR = or_neighbor(g, e, d, +1);
        double two_h = 2.0 / or_width(g, e, d);
        for (int n = 0; n < g->nnode; ++n) {
          int f, i;
          or_node_line(g, n, d, &f, &i);
          double wstar_p = 0.5 * (trace(g, wk, e, d, 1, f) + trace(g, wk, eR, d, 0, f));
          double wstar_m = 0.5 * (trace(g, wk, eL, d, 1, f) + trace(g, wk, e, d, 0, f));
          double vol = 0.0;
          for (int l = 0; l < g->np; ++l)
            vol += g->b.Dhat[i][l] * wk[(size_t)e * g->nnode + or_line_node(g, d, f, l)];
          Qdk[(size_t)e * g->nnode + n] =
              two_h * (-vol + (g->b.Lp[i] * wstar_p - g->b.Lm[i] * wstar_m) / g->b.w[i]);
        }
      }
    }
}

/* ------------------------------------------------------------------------ */
/* Model II physical fluxes in direction d at one point.                     */
/* Convective: (m_d, m_d v_j + delta_jd p_alpha, 0).                          */
static void flux_conv(const or_prob* P, int dim, int d, const double* u, double* F) {
  double rho = u[0];
  double pa = or_p(P->T, rho) + 0.5 * P->alpha * rho * rho;
  F[0] = u[1 + d];
  for (int j = 0; j < dim; ++j) F[1 + j] = u[1 + d] * u[1 + j] / rho + (j == d ? pa : 0.0);
  F[dim + 1] = 0.0;
}

/* Viscous: (0, tau_jd, (kappa/beta) dc/dx_d), tau = eps (grad v + grad v^T
 * - 2/3 div v I).  q[dd][k] = d w_k / d x_dd. */
static void flux_visc(const or_prob* P, int dim, int d, double q[3][4], double* F) {
  double div = 0.0;
  for (int j = 0; j < dim; ++j) div += q[j][j];
  F[0] = 0.0;
  for (int j = 0; j < dim; ++j)
    F[1 + j] = P->eps * (q[d][j] + q[j][d] - (j == d ? 2.0 / 3.0 * div : 0.0));
  F[dim + 1] = P->kappa / P->beta * q[d][dim];
}

/* Largest model II wave speed |v.n| + sqrt(p_alpha'(rho)) of a state. */
static double wave_speed(const or_prob* P, int d, const double* u) {
  double rho = u[0];
  double a = sqrt(or_dp(P->T, rho) + P->alpha * rho);
  return fabs(u[1 + d] / rho) + a;
}

/* Convective numerical flux in direction d.
 * flux 0, Rusanov: (F(uL) + F(uR))/2 - lam (uR - uL)/2, lam the larger wave
 *   speed of the two states (on c only if diss_c).
 * flux 1, HLLC for the barotropic convective part (Toro's HLLC with the
 *   contact speed taken from the HLL mass flux): Davis speeds
 *   SL = min(vL - aL, vR - aR), SR = max(vL + aL, vR + aR) (v normal
 *   velocity, a = sqrt(p_alpha'));  F = F(uL) if SL >= 0, F(uR) if SR <= 0;
 *   otherwise the HLL flux (SR F(uL) - SL F(uR) + SL SR (uR - uL))/(SR - SL)
 *   for mass and normal momentum, the mass flux times the tangential
 *   velocity of the upwind side of the contact S* = F_hll[rho] / rho_hll for
 *   the tangential momenta, and SL SR (cR - cL)/(SR - SL) for c (0 if not
 *   diss_c). */
static void numflux_conv(const or_prob* P, int dim, int d, const double* uL, const double* uR, double* Fs) {
  const int nvar = dim + 2;
  double fL[5], fR[5];
  flux_conv(P, dim, d, uL, fL);
  flux_conv(P, dim, d, uR, fR);
  if (P->flux == 0) {
    double lam = fmax(wave_speed(P, d, uL), wave_speed(P, d, uR));
    for (int v = 0; v < nvar; ++v) {
      double diss = (v == nvar - 1 && !P->diss_c) ? 0.0 : lam * (uR[v] - uL[v]);
      Fs[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * diss;
    }
    return;
  }
  const double vL = uL[1 + d] / uL[0], vR = uR[1 + d] / uR[0];
  const double aL = sqrt(or_dp(P->T, uL[0]) + P->alpha * uL[0]);
  const double aR = sqrt(or_dp(P->T, uR[0]) + P->alpha * uR[0]);
  const double SL = fmin(vL - aL, vR - aR), SR = fmax(vL + aL, vR + aR);
  if (SL >= 0.0) {
    for (int v = 0; v < nvar; ++v) Fs[v] = fL[v];
    return;
  }
  if (SR <= 0.0) {
    for (int v = 0; v < nvar; ++v) Fs[v] = fR[v];
    return;
  }
  const double w = 1.0 / (SR - SL);
  const double Fm = (SR * fL[0] - SL * fR[0] + SL * SR * (uR[0] - uL[0])) * w;
  const double rho_hll = (SR * uR[0] - SL * uL[0] - (fR[0] - fL[0])) * w;
  const double Sstar = Fm / rho_hll;
  Fs[0] = Fm;
  for (int j = 0; j < dim; ++j) {
    if (j == d)
      Fs[1 + j] = (SR * fL[1 + j] - SL * fR[1 + j] + SL * SR * (uR[1 + j] - uL[1 + j])) * w;
    else
      Fs[1 + j] = Fm * (Sstar >= 0.0 ? uL[1 + j] / uL[0] : uR[1 + j] / uR[0]);
  }
  Fs[dim + 1] = P->diss_c ? SL * SR * (uR[dim + 1] - uL[dim + 1]) * w : 0.0;
}

int or_numflux(const or_prob* P, int d, const double* uL, const double* uR, double* F) {
  if (!P || P->dim < 1 || P->dim > 3 || d < 0 || d >= P->dim) return -1;
  numflux_conv(P, P->dim, d, uL, uR, F);
  return 0;
}

int or_rhs_weak(const or_prob* P, const double* U, double* R, double* Qout) {
  or_geom g;
  if (or_geom_init(&g, P)) return -1;
  const int dim = g.dim, nvar = g.nvar, nlift = g.nlift, nn = g.nnode;
  const size_t S = (size_t)g.E * nn;

  /* Step 1 and step 2 */
  double* w = malloc(sizeof(double) * nlift * S);
  double* Q = malloc(sizeof(double) * dim * nlift * S);
  primitives(&g, U, w);
  lift(&g, w, Q);

  /* Step 3: nodal total flux F_d = Fc_d - Fv_d and the viscous part alone */
  double* F = malloc(sizeof(double) * dim * nvar * S);
  double* Fv = malloc(sizeof(double) * dim * nvar * S);
#pragma omp parallel for
  for (long e = 0; e < g.E; ++e)
    for (int n = 0; n < nn; ++n) {
      size_t o = (size_t)e * nn + n;
      double u[5], q[3][4], fc[5], fv[5];
      for (int v = 0; v < nvar; ++v) u[v] = U[v * S + o];
      for (int dd = 0; dd < dim; ++dd)
        for (int k = 0; k < nlift; ++k) q[dd][k] = Q[((size_t)dd * nlift + k) * S + o];
      for (int d = 0; d < dim; ++d) {
        flux_conv(P, dim, d, u, fc);
        flux_visc(P, dim, d, q, fv);
        for (int v = 0; v < nvar; ++v) {
          F[((size_t)d * nvar + v) * S + o] = fc[v] - fv[v];
          Fv[((size_t)d * nvar + v) * S + o] = fv[v];
        }
      }
    }

  /* Step 4: numerical flux on the face on the +xi_d side of every element.
   * Fs[d][v][e][f]; left state from e, right state from its +d neighbour. */
  double* Fs = malloc(sizeof(double) * dim * nvar * g.E * g.nf);
  for (int d = 0; d < dim; ++d) {
#pragma omp parallel for
    for (long e = 0; e < g.E; ++e) {
      long eR = or_neighbor(&g, e, d, +1);
      for (int f = 0; f < g.nf; ++f) {
        double uL[5], uR[5], fL[5], vL[5], vR[5];
        for (int v = 0; v < nvar; ++v) {
          uL[v] = trace(&g, U + v * S, e, d, 1, f);
          uR[v] = trace(&g, U + v * S, eR, d, 0, f);
          vL[v] = trace(&g, Fv + ((size_t)d * nvar + v) * S, e, d, 1, f);
          vR[v] = trace(&g, Fv + ((size_t)d * nvar + v) * S, eR, d, 0, f);
        }
        numflux_conv(P, dim, d, uL, uR, fL);
        for (int v = 0; v < nvar; ++v)
          Fs[(((size_t)d * nvar + v) * g.E + e) * g.nf + f] = fL[v] - 0.5 * (vL[v] + vR[v]);
      }
    }
  }

  /* Step 5: volume integral, surface integral and source */
#pragma omp parallel for
  for (long e = 0; e < g.E; ++e)
    for (int n = 0; n < nn; ++n) {
      size_t o = (size_t)e * nn + n;
      for (int v = 0; v < nvar; ++v) {
        double r = 0.0;
        for (int d = 0; d < dim; ++d) {
          int f, i;
          or_node_line(&g, n, d, &f, &i);
          long eL = or_neighbor(&g, e, d, -1);
          const double* Fdv = F + ((size_t)d * nvar + v) * S;
          double vol = 0.0;
          for (int l = 0; l < g.np; ++l) vol += g.b.Dhat[i][l] * Fdv[(size_t)e * nn + or_line_node(&g, d, f, l)];
          double Fp = Fs[(((size_t)d * nvar + v) * g.E + e) * g.nf + f];
          double Fm = Fs[(((size_t)d * nvar + v) * g.E + eL) * g.nf + f];
          r += 2.0 / or_width(&g, e, d) * (vol - (g.b.Lp[i] * Fp - g.b.Lm[i] * Fm) / g.b.w[i]);
        }
        R[v * S + o] = r;
      }
      /* source S = (0, alpha rho dc/dx_d, (alpha/beta)(rho - c)) */
      double rho = U[o], c = U[(dim + 1) * S + o];
      for (int d = 0; d < dim; ++d) R[(1 + d) * S + o] += P->alpha * rho * Q[((size_t)d * nlift + dim) * S + o];
      R[(dim + 1) * S + o] += P->alpha / P->beta * (rho - c);
    }

  if (Qout) memcpy(Qout, Q, sizeof(double) * dim * nlift * S);
  free(w); free(Q); free(F); free(Fv); free(Fs);
  or_geom_free(&g);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Time integration with the low-storage scheme, fixed step dt.             */
int or_run(const or_prob* P, double* U, double dt, int nsteps, double t0, or_forcing_fn fn, void* user) {
  or_geom g;
  if (or_geom_init(&g, P)) return -1;
  const size_t M = (size_t)g.nvar * g.E * g.nnode;
  or_geom_free(&g);
  double A[5], B[5], C[5];
  or_lsrk45(A, B, C);
  double* dU = calloc(M, sizeof(double));
  double* R = malloc(sizeof(double) * M);
  double* Fx = fn ? malloc(sizeof(double) * M) : NULL;
  for (int step = 0; step < nsteps; ++step) {
    double t = t0 + step * dt;
    for (int s = 0; s < 5; ++s) {
      if (or_rhs_weak(P, U, R, NULL)) { free(dU); free(R); free(Fx); return -1; }
      if (fn) {
        fn(t + C[s] * dt, Fx, user);
        for (size_t q = 0; q < M; ++q) R[q] += Fx[q];
      }
      for (size_t q = 0; q < M; ++q) {
        dU[q] = A[s] * dU[q] + dt * R[q];
        U[q] += B[s] * dU[q];
      }
    }
  }
  free(dU); free(R); free(Fx);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Time-step rule (parabolic bound of Sec. 3.1, with the relaxation source of
 * Sec. 2.3 acting on the same equation for c):
 *   dt = CFL * min(dt_conv, dt_mom, dt_c)
 *   dt_conv = 1 / ((2N+1) max_e sum_d max_nodes(|v_d| + a) / h_d)
 *   dt_mom  = 1 / ((2N+1)^2 (4/3) (eps / rho_min) max_e sum_d 1 / h_d^2)
 *             (viscous momentum: the stress eps (grad v + grad v^T - (2/3) div v I)
 *             diffuses v = m / rho, fastest in the longitudinal mode and where
 *             the density is smallest; NaN if rho_min <= 0)
 *   dt_c    = 1 / ((2N+1)^2 max_e sum_d (kappa/beta) / h_d^2 + alpha / (beta |z_R|))
 * The screened heat equation beta c_t = kappa lap c + alpha (rho - c) has real
 * negative eigenvalues: the diffusion's and the source's, which add.  Both
 * must fit together inside the real-axis stability limit |z_R| of the
 * Runge-Kutta scheme, so their rates are summed rather than bounded apart
 * (bounded apart, the step leaves the stability region where the two are
 * about equal). */
double or_dt(const or_prob* P, const double* U, double cfl) {
  or_geom g;
  if (or_geom_init(&g, P)) return NAN;
  const size_t S = (size_t)g.E * g.nnode;
  /* the momentum diffuses v = m / rho: its largest rate is that of the
     longitudinal mode, (4/3) eps / rho, taken at the smallest density */
  double rmin = INFINITY;
  for (size_t o = 0; o < S; ++o) rmin = fmin(rmin, U[o]);
  if (!(rmin > 0.0)) {
    or_geom_free(&g);
    return NAN;
  }
  const double nu = (4.0 / 3.0) * P->eps / rmin;
  double lam_c = 0.0, lam_m = 0.0, lam_k = 0.0;
  for (long e = 0; e < g.E; ++e) {
    double sc = 0.0, sm = 0.0, sk = 0.0;
    for (int d = 0; d < g.dim; ++d) {
      double h = or_width(&g, e, d), mx = 0.0;
      for (int n = 0; n < g.nnode; ++n) {
        double u[5];
        for (int v = 0; v < g.nvar; ++v) u[v] = U[v * S + (size_t)e * g.nnode + n];
        mx = fmax(mx, wave_speed(P, d, u));
      }
      sc += mx / h;
      sm += nu / (h * h);
      sk += (P->kappa / P->beta) / (h * h);
    }
    lam_c = fmax(lam_c, sc);
    lam_m = fmax(lam_m, sm);
    lam_k = fmax(lam_k, sk);
  }
  const double N2 = 2.0 * P->N + 1.0;
  const double dtc = 1.0 / (N2 * lam_c);
  const double dtm = 1.0 / (N2 * N2 * lam_m);
  const double dtk = 1.0 / (N2 * N2 * lam_k + P->alpha / (P->beta * or_lsrk_real_limit()));
  or_geom_free(&g);
  return cfl * fmin(dtc, fmin(dtm, dtk));
}

/* ------------------------------------------------------------------------ */
/* Diagnostics by the collocated quadrature sum_e J_e sum_n omega_n (.)       */
int or_diagnostics(const or_prob* P, const double* U, double* out) {
  or_geom g;
  if (or_geom_init(&g, P)) return -1;
  const int dim = g.dim, nn = g.nnode;
  const size_t S = (size_t)g.E * nn;
  for (int k = 0; k < 16; ++k) out[k] = 0.0;
  double* w = malloc(sizeof(double) * g.nlift * S);
  double* Q = malloc(sizeof(double) * dim * g.nlift * S);
  primitives(&g, U, w);
  lift(&g, w, Q);
  double rmin = INFINITY, rmax = -INFINITY, amax = 0.0, bad = 0.0;
  for (long e = 0; e < g.E; ++e)
    for (int n = 0; n < nn; ++n) {
      size_t o = (size_t)e * nn + n;
      double wq = or_quad_weight(&g, e, n);
      double u[5];
      for (int v = 0; v < g.nvar; ++v) {
        u[v] = U[v * S + o];
        out[v] += wq * u[v];
        if (!isfinite(u[v])) bad += 1.0;
      }
      double rho = u[0], c = u[dim + 1], ek = 0.0, gc2 = 0.0;
      for (int d = 0; d < dim; ++d) ek += 0.5 * u[1 + d] * u[1 + d] / rho;
      for (int d = 0; d < dim; ++d) {
        double gc = Q[((size_t)d * g.nlift + dim) * S + o];
        gc2 += gc * gc;
        amax = fmax(amax, wave_speed(P, d, u));
      }
      out[7] += wq * ek;
      out[8] += wq * (ek + or_W(P->T, rho) + 0.5 * P->alpha * (rho - c) * (rho - c) + 0.5 * P->kappa * gc2);
      out[9] += wq * (rho - c) * (rho - c);
      rmin = fmin(rmin, rho);
      rmax = fmax(rmax, rho);
    }
  out[9] = sqrt(out[9]);
  out[10] = rmin;
  out[11] = rmax;
  out[12] = amax;
  out[13] = bad;
  free(w); free(Q);
  or_geom_free(&g);
  return 0;
}

int or_node_coords(const or_prob* P, double* X) {
  or_geom g;
  if (or_geom_init(&g, P)) return -1;
  const size_t S = (size_t)g.E * g.nnode;
  for (long e = 0; e < g.E; ++e)
    for (int n = 0; n < g.nnode; ++n)
      for (int d = 0; d < g.dim; ++d) {
        int f, i;
        or_node_line(&g, n, d, &f, &i);
        int ed = or_elem_index(&g, e, d);
        double h = P->xb[d][ed + 1] - P->xb[d][ed];
        X[d * S + (size_t)e * g.nnode + n] = P->xb[d][ed] + 0.5 * (g.b.xi[i] + 1.0) * h;
      }
  or_geom_free(&g);
  return 0;
}

long or_nelem(const or_prob* P) {
  long E = 1;
  for (int d = 0; d < P->dim; ++d) E *= P->nel[d];
  return E;
}

int or_nnode(const or_prob* P) {
  int n = 1;
  for (int d = 0; d < P->dim; ++d) n *= P->N + 1;
  return n;
}
