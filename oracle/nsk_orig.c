/*
 * Oracle (test infrastructure only): the DGSEM semi-discretisation of the
 * original isothermal Navier-Stokes-Korteweg equations (Sec. 2.2, scaled
 * form: 1/Re = eps, 1/We = eps^2 gamma = kappa) on the periodic box grid of
 * the model II oracle, state U = (rho, rho v), with
 *
 *   F^c_d = (m_d, m_d v + p e_d)              (Van-der-Waals p, no alpha)
 *   F^v_d = (0, Sigma_{.d}),  Sigma = eps (grad v + grad v^T - 2/3 div v I)
 *           + kappa ((rho lap rho + |grad rho|^2 / 2) I - grad rho (x) grad rho)
 *
 * (the Korteweg stress of Sec. 2.2 in its conservative form, whose divergence
 * is kappa rho grad lap rho).  Gradients come from a BR1 lifting of the
 * primitives (v, rho) with the central flux; the Laplacian of rho from a
 * second BR1 lifting of the lifted density gradient, lap rho = div(grad rho)
 * (end of Sec. 3.1).  The convective face flux is the global Lax-Friedrichs
 * flux (Sec. 2.2 and 4.1.2), whose dissipation speed is one number for the
 * whole grid: the maximum over all nodes and directions of
 * |v_d| + sqrt(max(p'(rho), 0)) (the flux Jacobian has real eigenvalues
 * v.n +- sqrt(p') only outside the spinodal interval).  The second-order face
 * flux is the mean of the two traces of the nodal F^v, the trace of the flux
 * polynomial of Sec. 3.1.
 *
 * Step order of one right-hand side evaluation:
 *   1. nodal primitives w = (v_1..v_d, rho)
 *   2. BR1 lifting Q_d = dw/dx_d
 *   3. second BR1 lifting lap rho = sum_d d(Q_d[rho])/dx_d
 *   4. nodal fluxes F_d = Fc_d(U) - Fv_d(U, Q, lap rho)
 *   5. face fluxes F*_d = LF(U-, U+; lambda) - (Fv_d- + Fv_d+)/2
 *   6. R = sum_d (2/h_d) [Dhat F_d - (L+ F*_+ - L- F*_-)/w]
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "geom.h"

static int nsk_geom(or_geom* g, const or_prob* P) {
  if (or_geom_init(g, P)) return -1;
  g->nvar = g->dim + 1;   /* rho, m_1..m_dim */
  g->nlift = g->dim + 1;  /* v_1..v_dim, rho */
  return 0;
}

static double trace(const or_geom* g, const double* a, long e, int d, int s, int f) {
  const double* L = s ? g->b.Lp : g->b.Lm;
  double t = 0.0;
  for (int l = 0; l < g->np; ++l) t += L[l] * a[(size_t)e * g->nnode + or_line_node(g, d, f, l)];
  return t;
}

/* BR1 derivative of the nodal field a along direction d at node n of element
 * e: (2/h_d) [ -sum_l Dhat_il a_l + (L+_i a*_+ - L-_i a*_-) / omega_i ] with
 * the central face values a* = (a- + a+)/2. */
static double br1_derivative(const or_geom* g, const double* a, long e, int n, int d) {
  int f, i;
  or_node_line(g, n, d, &f, &i);
  long eL = or_neighbor(g, e, d, -1), eR = or_neighbor(g, e, d, +1);
  double ap = 0.5 * (trace(g, a, e, d, 1, f) + trace(g, a, eR, d, 0, f));
  double am = 0.5 * (trace(g, a, eL, d, 1, f) + trace(g, a, e, d, 0, f));
  double vol = 0.0;
  for (int l = 0; l < g->np; ++l) vol += g->b.Dhat[i][l] * a[(size_t)e * g->nnode + or_line_node(g, d, f, l)];
  return 2.0 / or_width(g, e, d) * (-vol + (g->b.Lp[i] * ap - g->b.Lm[i] * am) / g->b.w[i]);
}

/* Steps 1-3: Q[d][k][elem][node] = d w_k / dx_d with w = (v, rho), and
 * lap[elem][node] = sum_d d Q[d][rho] / dx_d. */
static void gradients(const or_geom* g, const double* U, double* Q, double* lap) {
  const int dim = g->dim, nl = g->nlift;
  const size_t S = (size_t)g->E * g->nnode;
  double* w = malloc(sizeof(double) * nl * S);
  for (size_t o = 0; o < S; ++o) {
    for (int d = 0; d < dim; ++d) w[d * S + o] = U[(1 + d) * S + o] / U[o];
    w[dim * S + o] = U[o];
  }
  for (int d = 0; d < dim; ++d)
    for (int k = 0; k < nl; ++k)
#pragma omp parallel for
      for (long e = 0; e < g->E; ++e)
        for (int n = 0; n < g->nnode; ++n)
          Q[((size_t)d * nl + k) * S + (size_t)e * g->nnode + n] = br1_derivative(g, w + k * S, e, n, d);
#pragma omp parallel for
  for (long e = 0; e < g->E; ++e)
    for (int n = 0; n < g->nnode; ++n) {
      double s = 0.0;
      for (int d = 0; d < dim; ++d) s += br1_derivative(g, Q + ((size_t)d * nl + dim) * S, e, n, d);
      lap[(size_t)e * g->nnode + n] = s;
    }
  free(w);
}

/* Convective flux (m_d, m_d v_j + delta_jd p) at one point. */
static void flux_conv(const or_prob* P, int dim, int d, const double* u, double* F) {
  double rho = u[0], p = or_p(P->T, rho);
  F[0] = u[1 + d];
  for (int j = 0; j < dim; ++j) F[1 + j] = u[1 + d] * u[1 + j] / rho + (j == d ? p : 0.0);
}

/* Second-order flux (0, Sigma_{jd}) at one point; q[dd][k] = d w_k/dx_dd,
 * q[dd][dim] = d rho/dx_dd, lap = Laplacian of rho. */
static void flux_visc(const or_prob* P, int dim, int d, double rho, double q[3][4], double lap, double* F) {
  double div = 0.0, g2 = 0.0;
  for (int j = 0; j < dim; ++j) {
    div += q[j][j];
    g2 += q[j][dim] * q[j][dim];
  }
  F[0] = 0.0;
  for (int j = 0; j < dim; ++j) {
    double tau = P->eps * (q[d][j] + q[j][d] - (j == d ? 2.0 / 3.0 * div : 0.0));
    double kor = P->kappa * ((j == d ? rho * lap + 0.5 * g2 : 0.0) - q[j][dim] * q[d][dim]);
    F[1 + j] = tau + kor;
  }
}

/* Global Lax-Friedrichs speed: max over nodes and directions of
 * |v_d| + sqrt(max(p'(rho), 0)). */
double or_nsk_lf_speed(const or_prob* P, const double* U) {
  or_geom g;
  if (nsk_geom(&g, P)) return NAN;
  const size_t S = (size_t)g.E * g.nnode;
  double lam = 0.0;
  for (size_t o = 0; o < S; ++o) {
    double rho = U[o], a = sqrt(fmax(or_dp(P->T, rho), 0.0));
    for (int d = 0; d < g.dim; ++d) lam = fmax(lam, fabs(U[(1 + d) * S + o] / rho) + a);
  }
  return lam;
}

/* The right-hand side with the global LF speed lam given (the speed of a
 * larger grid of which U is a part); or_nsk_rhs uses the speed of U. */
int or_nsk_rhs_lam(const or_prob* P, const double* U, double lam, double* R, double* Qout, double* lapout) {
  or_geom g;
  if (nsk_geom(&g, P)) return -1;
  const int dim = g.dim, nvar = g.nvar, nl = g.nlift, nn = g.nnode;
  const size_t S = (size_t)g.E * nn;

  double* Q = malloc(sizeof(double) * dim * nl * S);
  double* lap = malloc(sizeof(double) * S);
  gradients(&g, U, Q, lap);

  /* Step 4: nodal total flux and its second-order part */
  double* F = malloc(sizeof(double) * dim * nvar * S);
  double* Fv = malloc(sizeof(double) * dim * nvar * S);
#pragma omp parallel for
  for (long e = 0; e < g.E; ++e)
    for (int n = 0; n < nn; ++n) {
      size_t o = (size_t)e * nn + n;
      double u[4], q[3][4], fc[4], fv[4];
      for (int v = 0; v < nvar; ++v) u[v] = U[v * S + o];
      for (int dd = 0; dd < dim; ++dd)
        for (int k = 0; k < nl; ++k) q[dd][k] = Q[((size_t)dd * nl + k) * S + o];
      for (int d = 0; d < dim; ++d) {
        flux_conv(P, dim, d, u, fc);
        flux_visc(P, dim, d, u[0], q, lap[o], fv);
        for (int v = 0; v < nvar; ++v) {
          F[((size_t)d * nvar + v) * S + o] = fc[v] - fv[v];
          Fv[((size_t)d * nvar + v) * S + o] = fv[v];
        }
      }
    }

  /* Step 5: face flux on the +xi_d face of every element */
  double* Fs = malloc(sizeof(double) * dim * nvar * g.E * g.nf);
  for (int d = 0; d < dim; ++d) {
#pragma omp parallel for
    for (long e = 0; e < g.E; ++e) {
      long eR = or_neighbor(&g, e, d, +1);
      for (int f = 0; f < g.nf; ++f) {
        double uL[4], uR[4], fL[4], fR[4], vL[4], vR[4];
        for (int v = 0; v < nvar; ++v) {
          uL[v] = trace(&g, U + v * S, e, d, 1, f);
          uR[v] = trace(&g, U + v * S, eR, d, 0, f);
          vL[v] = trace(&g, Fv + ((size_t)d * nvar + v) * S, e, d, 1, f);
          vR[v] = trace(&g, Fv + ((size_t)d * nvar + v) * S, eR, d, 0, f);
        }
        flux_conv(P, dim, d, uL, fL);
        flux_conv(P, dim, d, uR, fR);
        for (int v = 0; v < nvar; ++v)
          Fs[(((size_t)d * nvar + v) * g.E + e) * g.nf + f] =
              0.5 * (fL[v] + fR[v]) - 0.5 * lam * (uR[v] - uL[v]) - 0.5 * (vL[v] + vR[v]);
      }
    }
  }

  /* Step 6: volume and surface integrals (no source) */
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
    }

  if (Qout) memcpy(Qout, Q, sizeof(double) * dim * nl * S);
  if (lapout) memcpy(lapout, lap, sizeof(double) * S);
  free(Q); free(lap); free(F); free(Fv); free(Fs);
  return 0;
}

int or_nsk_rhs(const or_prob* P, const double* U, double* R, double* Qout, double* lapout) {
  return or_nsk_rhs_lam(P, U, or_nsk_lf_speed(P, U), R, Qout, lapout);
}

int or_nsk_run(const or_prob* P, double* U, double dt, int nsteps, double t0, or_forcing_fn fn, void* user) {
  or_geom g;
  if (nsk_geom(&g, P)) return -1;
  const size_t M = (size_t)g.nvar * g.E * g.nnode;
  double A[5], B[5], C[5];
  or_lsrk45(A, B, C);
  double* dU = calloc(M, sizeof(double));
  double* R = malloc(sizeof(double) * M);
  double* Fx = fn ? malloc(sizeof(double) * M) : NULL;
  for (int step = 0; step < nsteps; ++step) {
    double t = t0 + step * dt;
    for (int s = 0; s < 5; ++s) {
      if (or_nsk_rhs(P, U, R, NULL, NULL)) { free(dU); free(R); free(Fx); return -1; }
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

/* Time-step rule: CFL * min(dt_conv, dt_visc, dt_disp) with
 *   dt_conv = 1 / ((2N+1) lambda max_e sum_d 1/h_d), lambda the global LF speed
 *   dt_visc = 1 / ((2N+1)^2 (4/3) (eps / rho_min) max_e sum_d 1/h_d^2)
 *             (the stress diffuses v = m / rho; NaN if rho_min <= 0)
 *   dt_disp = C_disp / ((2N+1)^2 sqrt(kappa rho_max) max_e sum_d 1/h_d^2).
 * The linearised system about a state at rest has the frequencies
 * w^2 = p' k^2 + kappa rho k^4, so the capillary modes behave like a
 * parabolic term of coefficient sqrt(kappa rho) on the imaginary axis.
 * C_disp = 1/4 is a reading (the paper gives no explicit bound for the
 * third-order system): with it, at CFL 1, the spectrum of the linearised
 * discrete operator stays inside the scheme's stability region for states at
 * rest in both phases (N = 1..6, 1D and 2D) and for interface states. */
#define OR_NSK_CDISP 0.25
double or_nsk_dt(const or_prob* P, const double* U, double cfl) {
  or_geom g;
  if (nsk_geom(&g, P)) return NAN;
  const size_t S = (size_t)g.E * g.nnode;
  double s1 = 0.0, s2 = 0.0, rmax = 0.0;
  for (long e = 0; e < g.E; ++e) {
    double a = 0.0, b = 0.0;
    for (int d = 0; d < g.dim; ++d) {
      double h = or_width(&g, e, d);
      a += 1.0 / h;
      b += 1.0 / (h * h);
    }
    s1 = fmax(s1, a);
    s2 = fmax(s2, b);
  }
  double rmin = INFINITY;
  for (size_t o = 0; o < S; ++o) {
    rmax = fmax(rmax, U[o]);
    rmin = fmin(rmin, U[o]);
  }
  if (!(rmin > 0.0)) return NAN;
  const double N2 = 2.0 * P->N + 1.0;
  const double lam = or_nsk_lf_speed(P, U);
  double dt = INFINITY;
  if (lam > 0.0) dt = fmin(dt, 1.0 / (N2 * lam * s1));
  /* viscous: the longitudinal mode of v = m / rho, rate (4/3) eps / rho */
  if (P->eps > 0.0) dt = fmin(dt, 1.0 / (N2 * N2 * (4.0 / 3.0) * (P->eps / rmin) * s2));
  if (P->kappa > 0.0) dt = fmin(dt, OR_NSK_CDISP / (N2 * N2 * sqrt(P->kappa * rmax) * s2));
  return cfl * dt;
}

/* Diagnostics in the layout of or_diagnostics: out[0..dim] integrals of rho
 * and m, out[7] kinetic energy, out[8] the NSK energy
 * int (rho |v|^2/2 + W(rho) + kappa |grad rho|^2 / 2) (Sec. 2.2) with the
 * lifted gradient, out[9] = 0, out[10] rho min, out[11] rho max, out[12] the
 * global LF speed, out[13] number of non-finite values. */
int or_nsk_diagnostics(const or_prob* P, const double* U, double* out) {
  or_geom g;
  if (nsk_geom(&g, P)) return -1;
  const int dim = g.dim, nn = g.nnode, nl = g.nlift;
  const size_t S = (size_t)g.E * nn;
  for (int k = 0; k < 16; ++k) out[k] = 0.0;
  double* Q = malloc(sizeof(double) * dim * nl * S);
  double* lap = malloc(sizeof(double) * S);
  gradients(&g, U, Q, lap);
  double rmin = INFINITY, rmax = -INFINITY, bad = 0.0;
  for (long e = 0; e < g.E; ++e)
    for (int n = 0; n < nn; ++n) {
      size_t o = (size_t)e * nn + n;
      double wq = or_quad_weight(&g, e, n);
      double u[4];
      for (int v = 0; v < g.nvar; ++v) {
        u[v] = U[v * S + o];
        out[v] += wq * u[v];
        if (!isfinite(u[v])) bad += 1.0;
      }
      double rho = u[0], ek = 0.0, g2 = 0.0;
      for (int d = 0; d < dim; ++d) {
        ek += 0.5 * u[1 + d] * u[1 + d] / rho;
        double gr = Q[((size_t)d * nl + dim) * S + o];
        g2 += gr * gr;
      }
      out[7] += wq * ek;
      out[8] += wq * (ek + or_W(P->T, rho) + 0.5 * P->kappa * g2);
      rmin = fmin(rmin, rho);
      rmax = fmax(rmax, rho);
    }
  out[10] = rmin;
  out[11] = rmax;
  out[12] = or_nsk_lf_speed(P, U);
  out[13] = bad;
  free(Q); free(lap);
  return 0;
}
