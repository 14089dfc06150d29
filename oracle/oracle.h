/*
 * Plain FP64 CPU oracle for the parabolic relaxation model II of the
 * isothermal Navier-Stokes-Korteweg equations (Hitz, Keim, Munz, Rohde,
 * "A Parabolic Relaxation Model for the Navier-Stokes-Korteweg Equations").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the checker that the GPU path is
 * compared against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * generator with the HIP library; the two are written independently.
 *
 * Every function follows a passage of the paper (cited by section and
 * equation) and is written for a reader who checks it against the paper by
 * eye: straight loops, no blocking, no fusion.
 *
 * State layout shared with the caller (not with the GPU code): U[var][elem][node]
 *   var  = 0 rho, 1..dim momentum rho*v_d, dim+1 relaxation variable c
 *   elem = ex + nel0*(ey + nel1*ez)       (x fastest)
 *   node = i + (N+1)*(j + (N+1)*k)        (xi_1 fastest)
 */
#ifndef NSK_ORACLE_H
#define NSK_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------- 1D basis on Gauss-Legendre nodes (Sec. 3.1) -------------- */
#define OR_NMAX 12
typedef struct {
  int N;                         /* polynomial degree                            */
  double xi[OR_NMAX + 1];        /* Gauss-Legendre nodes on [-1,1], ascending   */
  double w[OR_NMAX + 1];         /* quadrature weights                           */
  double D[OR_NMAX + 1][OR_NMAX + 1];    /* D[i][j] = l_j'(xi_i)                 */
  double Dhat[OR_NMAX + 1][OR_NMAX + 1]; /* weak-form operator w_j/w_i * D[j][i] */
  double Lm[OR_NMAX + 1];        /* l_j(-1)                                      */
  double Lp[OR_NMAX + 1];        /* l_j(+1)                                      */
} or_basis;

int or_make_basis(int N, or_basis* b);

/* ---------------- Van-der-Waals thermodynamics (Sec. 2.1) ------------------ */
double or_W(double T, double rho);      /* Helmholtz free energy density         */
double or_dW(double T, double rho);     /* chemical potential W'(rho)            */
double or_p(double T, double rho);      /* pressure rho W' - W                   */
double or_dp(double T, double rho);     /* p'(rho) = rho W''(rho)                */
double or_d2W(double T, double rho);    /* W''(rho)                              */
/* Maxwell construction: equal pressure and equal chemical potential. */
int or_maxwell(double T, double* rho_v, double* rho_l, double* p_sat, double* mu_sat);
/* Spinodal densities: the two zeros of p'(rho). */
int or_spinodal(double T, double* rho_sv, double* rho_sl);
/* Integral of sqrt(2 (W - mu_sat rho + p_sat)) over [rho_v, rho_l]; the planar
 * gradient-theory surface tension is sqrt(kappa) times this number. */
double or_surface_integral(double T);
/* Young-Laplace initial densities for a spherical droplet (Sec. 4.3.1). */
int or_young_laplace(double T, double sigma, double r, double* rho_l, double* rho_v);

/* ---------------- low-storage Runge-Kutta (Sec. 3.1) ----------------------- */
/* Carpenter-Kennedy five-stage fourth-order 2N-storage scheme. */
void or_lsrk45(double A[5], double B[5], double C[5]);
/* Stability polynomial R(z) = sum_k g[k] z^k of the scheme (k = 0..5). */
void or_lsrk_stability_poly(double g[6]);
/* Largest x such that |R(-y)| <= 1 for all y in [0, x] (bisection). */
double or_lsrk_real_limit(void);

/* ---------------- DGSEM operator for relaxation model II ------------------- */
typedef struct {
  int dim;                 /* 1, 2 or 3                                       */
  int N;                   /* polynomial degree                               */
  int nel[3];              /* elements per direction (unused dims: 1)         */
  const double* xb[3];     /* breakpoints per direction, nel[d]+1 values      */
  double T;                /* temperature                                     */
  double eps;              /* viscosity 1/Re                                  */
  double kappa;            /* eps^2 gamma: coefficient of the Laplacian of c  */
  double alpha, beta;      /* relaxation parameters                           */
  int diss_c;              /* 1: dissipation of the numerical flux also on c  */
  int flux;                /* 0: Rusanov, 1: HLLC (barotropic form)           */
} or_prob;

/* Optional forcing added to the right-hand side at time t (manufactured
 * solutions).  F has the layout of U. */
typedef void (*or_forcing_fn)(double t, double* F, void* user);

long or_nelem(const or_prob* P);
int or_nnode(const or_prob* P);

/* Weak-form DGSEM right-hand side R = dU/dt (eqs. for the weak form and the
 * semi-discrete scheme of Sec. 3.1, BR1 lifting of the primitives).
 * Q (optional, may be NULL) receives the lifted gradients, layout
 * Q[d][k][elem][node] with k over (v_1..v_dim, c).  Returns 0 on success. */
int or_rhs_weak(const or_prob* P, const double* U, double* R, double* Q);
/* Convective numerical flux of the weak form between the point states uL, uR
 * (nvar values each) in direction d (for tests). */
int or_numflux(const or_prob* P, int d, const double* uL, const double* uR, double* F);
/* The same semi-discretisation written in strong form (independent code). */
int or_rhs_strong(const or_prob* P, const double* U, double* R);

/* LSRK4(5) integration in place: nsteps steps of size dt, from time t0. */
int or_run(const or_prob* P, double* U, double dt, int nsteps, double t0,
           or_forcing_fn f, void* user);

/* Time step rule: CFL * min(convective, viscous, relaxation-source) bound. */
double or_dt(const or_prob* P, const double* U, double cfl);

/* Diagnostics: out[0..nvar-1] = integral of each conserved variable,
 * out[7] kinetic energy, out[8] total energy E^alpha, out[9] L2 norm of rho-c,
 * out[10] rho min, out[11] rho max, out[12] max wave speed, out[13] number of
 * non-finite values.  out must hold 16 doubles. */
int or_diagnostics(const or_prob* P, const double* U, double* out);

/* Nodal coordinates (for tests): X[d][elem][node]. */
int or_node_coords(const or_prob* P, double* X);

/* ---------------- original NSK equations (Sec. 2.2) ------------------------ */
/* State U = (rho, rho v): dim+1 variables, layout as above.  Uses dim, N, nel,
 * xb, T, eps and kappa of the problem (alpha, beta, diss_c, flux unused).
 * Right-hand side with the Korteweg stress, two BR1 liftings and the global
 * Lax-Friedrichs flux; Q (optional) receives the lifted gradients
 * Q[d][k][elem][node], k over (v_1..v_dim, rho), lap (optional) the lifted
 * Laplacian of rho. */
int or_nsk_rhs(const or_prob* P, const double* U, double* R, double* Q, double* lap);
/* The same with the global Lax-Friedrichs speed lam given by the caller. */
int or_nsk_rhs_lam(const or_prob* P, const double* U, double lam, double* R, double* Q, double* lap);
int or_nsk_run(const or_prob* P, double* U, double dt, int nsteps, double t0, or_forcing_fn f, void* user);
double or_nsk_lf_speed(const or_prob* P, const double* U);
double or_nsk_dt(const or_prob* P, const double* U, double cfl);
int or_nsk_diagnostics(const or_prob* P, const double* U, double* out);

/* ---------------- FV sub-cell shock capturing (Sec. 3.2), model II --------- */
/* Sub-cell averaging matrix M (row k: mean of each Lagrange polynomial over
 * sub-cell k of N+1 equal sub-cells) and its inverse, (N+1)^2 row-major. */
int or_subcell_matrices(int N, double* M, double* Minv);
/* Persson-Peraire indicator of rho per element (log10 of the share of the
 * modal energy in the highest modes). */
int or_persson(const or_prob* P, const double* U, double* ind);
/* Right-hand side with troubled elements (indicator > threshold) on FV
 * sub-cells; flags (optional) receives the troubled-element flags. */
int or_rhs_subcell(const or_prob* P, const double* U, double threshold, double* R, int* flags);

/* ---------------- learned closure (no counterpart in the paper) ------------ */
#define OR_MLP_IN 4
#define OR_MLP_HIDDEN 64
#define OR_MLP_OUT 2
#define OR_MLP_NPARAM 8770
double or_relu(double z);
double or_relu_d(double z);
long or_mlp_nparam(void);
/* Y[n][2] = network(X[n][4]) with parameters w (layout in mlp.c). */
void or_mlp_forward(const double* w, const double* X, long n, double* Y);
/* Returns L = 1/(2n) sum (y - t)^2 and writes dL/dw into grad[8770]. */
double or_mlp_loss_grad(const double* w, const double* X, const double* Yt, long n, double* grad);
/* One Adam step (step number t >= 1) on np parameters. */
void or_adam_step(double* w, double* m, double* v, const double* g, long np, double lr, double b1, double b2,
                  double eps, int t);
/* Features X[node][4] and unit gradient direction nvec[d][node] (either may
 * be NULL); norm = (s0, k0, s1, k1, k2, k3, g0, out_m, out_c). */
int or_closure_features(const or_prob* P, const double* U, const double* norm, double* X, double* nvec);
/* Closure source in the layout of U (zero on rho). */
int or_closure_source(const or_prob* P, const double* U, const double* w, const double* norm, double* Sc);
/* Nudging step toward a reference state; records features and targets. */
int or_closure_nudge(const or_prob* P, double* U, const double* Uref, double dt, double tau, double cmap,
                     const double* norm, double* X, double* Y);

#ifdef __cplusplus
}
#endif
#endif
