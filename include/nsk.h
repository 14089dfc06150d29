/*
 * libnsk: MI355X (gfx950) DGSEM right-hand side and low-storage Runge-Kutta
 * update for the parabolic relaxation model II of the isothermal
 * Navier-Stokes-Korteweg equations (Hitz, Keim, Munz, Rohde, "A Parabolic
 * Relaxation Model for the Navier-Stokes-Korteweg Equations").
 *
 * The model (Sec. 2.3): U = (rho, rho v, c) obeys U_t + div(Fc - Fv) = S with
 *   Fc_i = (rho v_i, rho v_i v + p_alpha e_i, 0),  p_alpha = p + alpha rho^2/2,
 *   Fv_i = (0, tau_{.i}, (kappa/beta) dc/dx_i),
 *   S    = (0, alpha rho grad c, (alpha/beta)(rho - c)),
 * with the reduced Van-der-Waals pressure p = 8 T rho/(3 - rho) - 3 rho^2
 * (Sec. 2.1), tau = eps (grad v + grad v^T - 2/3 div v I) and
 * kappa = eps^2 gamma (the coefficient of the Laplacian of c).
 * The discretisation (Sec. 3.1): DGSEM on Gauss-Legendre nodes, weak form,
 * Rusanov (local Lax-Friedrichs) or HLLC convective flux, BR1 lifting of the
 * primitive variables (v, c) with central fluxes, arithmetic mean of the
 * viscous face fluxes, pointwise non-conservative source from the lifted
 * gradient of c, and the five-stage fourth-order 2N-storage Runge-Kutta
 * scheme of Carpenter and Kennedy.
 *
 * The original NSK equations (Sec. 2.2, model = 1): U = (rho, rho v) with
 *   Fc_i = (rho v_i, rho v_i v + p e_i),  Fv_i = (0, Sigma_{.i}),
 *   Sigma = tau + kappa ((rho lap rho + |grad rho|^2/2) I - grad rho (x) grad rho)
 * (the Korteweg stress, whose divergence is kappa rho grad lap rho), no
 * source.  grad rho comes from the BR1 lifting of (v, rho), lap rho from a
 * second BR1 lifting of the lifted gradient (end of Sec. 3.1); the
 * convective face flux is the global Lax-Friedrichs flux with one speed for
 * the whole grid, max over nodes and directions of |v_d| + sqrt(max(p', 0)),
 * recomputed at every evaluation; the second-order face flux is the mean of
 * the traces of the nodal Sigma.
 *
 * FV sub-cell shock capturing (Sec. 3.2, subcell = 1, model II): at every
 * right-hand side, elements whose Persson-Peraire indicator of rho (log10 of
 * the share of the orthonormal-Legendre modal energy in the modes whose
 * largest one-direction degree is N) exceeds subcell_threshold are treated
 * on (N+1)^dim equidistant sub-cells: sub-cell means by exact integration,
 * MinMod-limited reconstruction of (rho, v, c), the Rusanov or HLLC flux
 * (flux 0 or 1), viscous flux
 * from the means of the adjacent central-difference sub-cell gradients, the
 * source at the sub-cell means; on faces shared with DG elements the
 * sub-face means of the DG face-flux polynomial (mass is conserved exactly);
 * the element's nodal rate is the inverse sub-cell averaging of its
 * sub-cell rates, so a Runge-Kutta stage advances the sub-cell means.
 *
 * Mesh: periodic tensor-product grid of axis-aligned box elements.
 *
 * Data layout of every state array (device memory, double):
 *   U[var][elem][node], var = 0 rho, 1..dim rho v_d, dim+1 c (model 0 only);
 *   elem = ex + nel0 (ey + nel1 ez); node = i + (N+1)(j + (N+1) k)
 *   with i, j, k the Gauss-node indices along x, y, z.
 *
 * Ownership: the caller allocates all device memory (state, register and a
 * workspace of nsk_workspace_bytes()); the library never allocates device
 * memory.  The context itself is a small host object.
 *
 * Streams: every call is enqueued on the stream given to nsk_bind and returns
 * without waiting, except nsk_create, nsk_destroy, nsk_dt_estimate and
 * nsk_diagnostics, which wait for the stream.
 *
 * Errors: functions return 0 on success and a negative NSK_E* code otherwise;
 * nsk_strerror names the code.  A context is not reentrant; distinct contexts
 * are independent.
 */
#ifndef NSK_H
#define NSK_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NSK_OK 0
#define NSK_EINVAL (-1)    /* invalid mesh, parameters or argument           */
#define NSK_ENONPHYS (-2)  /* non-finite values or rho outside (0, 3)        */
#define NSK_EHIP (-3)      /* HIP runtime error                              */
#define NSK_EUNBOUND (-4)  /* device memory not bound yet                    */
#define NSK_EUNSUPPORTED (-5) /* degree/dimension combination not built      */
#define NSK_ENOCONV (-6)   /* implicit stage equations did not converge      */
#define NSK_ESCRATCH (-7)  /* problem too large for the static scratch of nsk_rhs_noalloc */

typedef struct nsk_ctx nsk_ctx;

typedef struct {
  int dim;              /* 1, 2 or 3                                        */
  int N;                /* polynomial degree, 1..6 (1..5 when dim = 3)      */
  int nel[3];           /* elements per direction (entries >= dim ignored)  */
  double lo[3], hi[3];  /* box [lo, hi] per direction (uniform spacing)     */
  const double* xbreaks[3]; /* optional host arrays of nel[d]+1 increasing
                               breakpoints per direction; NULL = uniform    */
} nsk_mesh;

typedef struct {
  double T;       /* temperature of the isotherm (reduced units), 0 < T < 1 */
  double eps;     /* viscosity eps = 1/Re                                   */
  double kappa;   /* eps^2 gamma, coefficient of the Laplacian of c         */
  double alpha;   /* relaxation parameter, > 6 (1 - T) (hyperbolicity)     */
  double beta;    /* parabolic relaxation parameter (> 0)                   */
  int flux;       /* 0 = Rusanov, 1 = HLLC (barotropic form), 2 = global
                     Lax-Friedrichs (model 1 only)                          */
  int diss_c;     /* 1 = numerical-flux dissipation also on c, 0 = not on c */
  int precision;  /* 0 = FP64 throughout; 1 = mixed (FP32 volume/surface)   */
  int closure;    /* 1: add the learned closure source (nsk_closure_set)   */
  int model;      /* 0 = relaxation model II (Sec. 2.3); 1 = the original
                     NSK equations (Sec. 2.2): flux must be 2, precision 0,
                     closure 0; alpha, beta and diss_c are not used          */
  int subcell;    /* 1: FV sub-cell shock capturing (Sec. 3.2) in elements
                     whose Persson-Peraire indicator exceeds
                     subcell_threshold (model 0, precision 0, closure 0
                     only; the FV faces use the Rusanov or HLLC flux of
                     the flux field)                                          */
  double subcell_threshold; /* log10 of the share of the modal energy of rho
                     in the highest modes above which an element is troubled */
} nsk_params;

typedef struct {
  double mass[5];        /* integral of each conserved variable             */
  double e_kin;          /* integral of rho |v|^2 / 2                        */
  double e_total;        /* relaxation energy E^alpha (Sec. 2.3)             */
  double l2_rho_minus_c; /* L2 norm of rho - c                               */
  double rho_min, rho_max;   /* nodal extremes of rho                        */
  double max_wavespeed;  /* max over nodes and directions of |v_d| + a        */
  long long nonfinite;   /* number of non-finite state values               */
  int status;            /* NSK_OK or NSK_ENONPHYS                           */
} nsk_diag;

/* Creates a context for a mesh and parameter set (host only; no device
 * memory is touched).  Rejects dim outside 1..3, N outside 1..6, nel < 1,
 * (NSK_EUNSUPPORTED for dim = 3 with N = 6: not built, its 343-node element
 * exceeds the sub-cell workgroups and its rhs tile would take about 105 KB
 * of LDS),
 * non-increasing breakpoints, T outside (0,1), eps < 0, kappa < 0, model
 * outside 0..1, and for model 0 alpha <= 6 (1 - T), beta <= 0 or flux
 * outside 0..1; for model 1 flux != 2, precision != 0, closure != 0 or
 * subcell != 0; subcell = 1 with precision or closure not 0, or a
 * non-finite threshold.
 * *out is set on success. */
int nsk_create(const nsk_mesh* mesh, const nsk_params* params, nsk_ctx** out);

/* Frees the host context (waits for the bound stream first). */
void nsk_destroy(nsk_ctx* ctx);

/* Number of doubles in one state array: nvar * elements * (N+1)^dim with
 * nvar = dim+2 (model 0) or dim+1 (model 1). */
size_t nsk_state_size(const nsk_ctx* ctx);

/* Bytes of device workspace nsk_bind expects (second state buffer, lifted
 * gradients, geometry, reduction scratch). */
size_t nsk_workspace_bytes(const nsk_ctx* ctx);

/* Binds caller-owned device memory: d_U and d_dU hold nsk_state_size()
 * doubles each, d_work nsk_workspace_bytes() bytes (256-byte aligned);
 * hip_stream is a hipStream_t (NULL = default stream).  Uploads the geometry
 * into the workspace and clears the Runge-Kutta register. */
int nsk_bind(nsk_ctx* ctx, double* d_U, double* d_dU, void* d_work, void* hip_stream);

/* Copies a device state (layout above) into the bound state. */
int nsk_set_state(nsk_ctx* ctx, const double* d_src);

/* Copies the bound state into a device array. */
int nsk_get_state(nsk_ctx* ctx, double* d_dst);

/* Semi-discrete right-hand side R = dU/dt of the device state d_U (any
 * array with the state layout, not necessarily the bound one): the DGSEM
 * weak form of Sec. 3.1 on Gauss-Legendre nodes with BR1 lifting of (v, c),
 * applied to relaxation model II of Sec. 2.3 (convective flux with the
 * modified pressure p + alpha rho^2/2, viscous flux (tau, (kappa/beta) grad c),
 * source (0, alpha rho grad c, (alpha/beta)(rho - c))), or to the original
 * NSK equations of Sec. 2.2 when model = 1.  d_R must not alias d_U.  The
 * scheme is autonomous, t is unused. */
int nsk_rhs(nsk_ctx* ctx, const double* d_U, double* d_R, double t);

/* nsk_rhs for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * right-hand side of d_U into d_R, computed by the same kernels, with the
 * lifted gradients, the geometry and the element order in a file-scope
 * static device array of NSK_NOALLOC_SCRATCH_BYTES (128 MiB, held by every
 * GPU the library runs on until the process ends) instead of the bound
 * workspace.  The context need not be bound; hip_stream is a hipStream_t
 * (NULL = default stream) on the current device.  Allocates nothing (no
 * hipMalloc, hipFree or host-to-device copy; the geometry is written by a
 * kernel).  Needs about 8 (FP64) or 4 (mixed) bytes times
 * (dim(dim+1)/2 + dim) per node plus the geometry: NSK_ESCRATCH if that
 * exceeds the array (checked before any device call); NSK_EUNSUPPORTED for
 * non-uniform meshes (breakpoints), the learned closure, FV sub-cells and
 * the original NSK path (model 1).  All calls on one GPU share its array:
 * calls that overlap on one GPU (other streams, other threads) race. */
#define NSK_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int nsk_rhs_noalloc(nsk_ctx* ctx, const double* d_U, double* d_R, void* hip_stream);

/* Time-step estimate for the bound state, after the parabolic bound of
 * Sec. 3.1 with the relaxation source of Sec. 2.3 on the same equation:
 *   dt = cfl * min(1/((2N+1) max_e sum_d max(|v_d|+a)/h_d),
 *                  1/((2N+1)^2 nu max_e sum_d 1/h_d^2),
 *                  1/((2N+1)^2 (kappa/beta) max_e sum_d 1/h_d^2 + alpha/(beta z_R)))
 * with a = sqrt(p'(rho) + alpha rho), nu = (4/3) eps / rho_min (the viscous
 * stress diffuses v = m / rho, fastest in the longitudinal mode and at the
 * smallest density) and z_R the negative-real-axis stability limit of the
 * Runge-Kutta scheme.  The last bound is that of the equation for c: its
 * diffusion and relaxation-source rates are both real and negative, so they
 * add.  Model 1:
 *   dt = cfl * min(1/((2N+1) lam max_e sum_d 1/h_d),
 *                  1/((2N+1)^2 nu max_e sum_d 1/h_d^2),
 *                  (1/4)/((2N+1)^2 sqrt(kappa rho_max) max_e sum_d 1/h_d^2))
 * with lam the global Lax-Friedrichs speed (the last bound is that of the
 * capillary modes, frequencies sqrt(kappa rho) k^2).  Waits for the stream.
 * NSK_ENONPHYS if the state holds non-finite values or a density <= 0. */
int nsk_dt_estimate(nsk_ctx* ctx, double cfl, double* dt_out);

/* Advances the bound state by nsteps steps of size dt of the five-stage,
 * fourth-order low-storage Runge-Kutta scheme of Sec. 3.1 (Carpenter-Kennedy
 * 2N-storage coefficients): per stage dU <- A_s dU + dt R(U), U <- U + B_s dU,
 * fused into the right-hand-side kernel.  Asynchronous.  On return of the
 * enqueued work the state is in d_U.  Launch forms (all give the same bits):
 * a 1D model II mesh that one workgroup holds (no closure, sub-cells or
 * stage timing) runs all nsteps in one launch; otherwise, on a non-null
 * stream, pairs of steps replay one captured graph, and the rest is launched
 * stage by stage. */
int nsk_rk_step(nsk_ctx* ctx, double dt, int nsteps);

/* Diagnostics of the bound state (quadrature over all elements, with the
 * lifted gradient of c in the capillary energy).  Model 1: e_total is the
 * NSK energy int (rho |v|^2/2 + W + kappa |grad rho|^2/2) with the lifted
 * gradient of rho, l2_rho_minus_c is 0 and max_wavespeed is the global
 * Lax-Friedrichs speed.  Waits for the stream.
 * host_out->status is NSK_ENONPHYS, and so is the return value, if any value
 * is non-finite or rho leaves (0, 3). */
int nsk_diagnostics(nsk_ctx* ctx, nsk_diag* host_out);

/* Launch shape (performance only; results are bitwise identical for every
 * choice).  variant 0: as many elements per workgroup as fit about 256
 * threads within 40 KB of LDS; variant 1: half as many.  order selects the
 * element work order: 0 natural order in the hardware's round-robin over
 * XCDs; 1 natural order cut into one contiguous range per XCD; 2..5 x-y
 * tiles of 4, 6, 8, 12 elements marched along z in 3D (x-strips of 16, 24,
 * 32, 48 elements marched along y in 2D), one contiguous range per XCD.
 * With a bound context a new order is uploaded at once (waits for the
 * stream).  Defaults: variant 0, order 4 in 3D, order 0 otherwise. */
int nsk_set_tile(nsk_ctx* ctx, int variant, int order);

/* Autotuner over the launch shapes of nsk_set_tile: times `reps`
 * right-hand-side evaluations of the bound state for each (variant, order)
 * pair with HIP events, keeps in the context the first pair (in index
 * order) within 1% of the fastest, and returns it: near-equal timings are
 * noise, and among the tiled orders the first is the smallest tile, which
 * re-reads the fewest neighbour elements.  ms_out (12 doubles, may be NULL)
 * receives the mean ms per evaluation at index variant * 6 + order (-1 for
 * pairs skipped because they coincide with another: tiled orders in 1D, and
 * variant 1 where both variants put the same number of elements in a
 * workgroup).  Uses the workspace's second state buffer as scratch, so it
 * must be called between steps, and waits for the stream. */
int nsk_autotune(nsk_ctx* ctx, int reps, int* variant_out, int* order_out, double* ms_out);

/* Changes alpha, beta, eps, kappa of an existing context (same mesh). */
int nsk_set_params(nsk_ctx* ctx, const nsk_params* params);

/* Troubled-element flags (0/1 per element, element order) of the last
 * right-hand side evaluated with subcell = 1, copied to the device array
 * d_flags (nelem ints).  Asynchronous.  NSK_EINVAL for contexts without
 * subcell. */
int nsk_subcell_flags(nsk_ctx* ctx, int* d_flags);

/* Kernel timing with HIP events on the bound stream (measurement only).
 * nsk_timing_enable(ctx, 1) makes every stage enqueued by nsk_rk_step record
 * events before the lifting kernel, after it, after the closure kernel (if
 * any) and after the right-hand-side/update kernel (at most 4096 stages
 * until the next read).  nsk_timing_read waits for the stream and returns
 * out[0] = summed ms of the lifting kernel, out[1] = summed ms of the
 * right-hand-side/update kernel, out[2] = number of stages timed, out[3] =
 * summed ms of the closure kernel (model 0) or of the speed reduction and
 * second lifting (model 1), then clears the record.
 * nsk_timing_enable(ctx, 0) stops recording and releases the events. */
int nsk_timing_enable(nsk_ctx* ctx, int enable);
int nsk_timing_read(nsk_ctx* ctx, double out[4]);

/* ------------------------------------------------------------------------
 * Implicit time stepping (Sec. 3.1: the implicit runs use a six-stage,
 * fourth-order ESDIRK scheme): Kennedy and Carpenter's ARK4(3)6L[2]SA
 * implicit tableau, gamma = 1/4, explicit first stage, stiffly accurate.
 * For stage i = 2..6 the equation X - dt gamma R(X) = B_i,
 * B_i = U_n + dt sum_{j<i} a_ij K_j, is solved by Newton's method (initial
 * guess B_i + dt gamma K_{i-1}); each Newton correction comes from one cycle
 * of right-preconditioned GMRES (at most gmres_m Krylov vectors, classical
 * Gram-Schmidt, repeated as reorth_tol says) with the Jacobian-vector product
 * (R(X + s z) - R(X))/s, s = sqrt(eps_machine)(1 + |X|_2).  K_i = (X - B_i)/
 * (dt gamma); U_{n+1} is the last stage.  Works on FP64 contexts of either
 * model without the closure.
 * ------------------------------------------------------------------------ */
#define NSK_GMRES_MAX 64
typedef struct {
  double newton_tol; /* stage converged when |B + dt gamma R(X) - X|_2 <= newton_tol |B|_2 */
  int newton_max;    /* Newton corrections per stage, 1..1000                  */
  double gmres_rtol; /* GMRES stops when the residual falls by this factor, (0,1) */
  int gmres_m;       /* Krylov vectors per GMRES cycle, 1..NSK_GMRES_MAX         */
  int precond;       /* 1: node-local inverse of the stiff relaxation source
                        (model II only): c -> (c + a rho)/(1 + a),
                        a = dt gamma alpha/beta; 0: none                        */
  int basis_fp32;    /* 1: Krylov basis stored in FP32 (half the Gram-Schmidt
                        traffic; products, sums, the new vector and all
                        Newton quantities stay FP64); 0: FP64 basis          */
  double reorth_tol; /* the Gram-Schmidt projection is repeated when
                        |w - sum h_j V_j|^2 <= reorth_tol |w|^2, [0, 1):
                        1/2 is Kahan's criterion, 0 never repeats it        */
} nsk_implicit_opts;

typedef struct {
  long long steps;        /* steps completed                                  */
  long long rhs_evals;    /* right-hand-side evaluations                      */
  long long newton_iters; /* Newton corrections                               */
  long long gmres_iters;  /* Jacobian-vector products (GMRES iterations)      */
  long long reorth;       /* Arnoldi steps that needed a second projection    */
  double max_residual;    /* largest final relative stage residual            */
  int converged;          /* 1 if every stage met newton_tol                  */
} nsk_implicit_stats;

/* Bytes of the device workspace nsk_esdirk_step needs (in addition to the
 * bound workspace): 13 + gmres_m + 1 state vectors plus reduction scratch
 * (sized for an FP64 basis).
 * 0 for invalid arguments. */
size_t nsk_implicit_workspace_bytes(const nsk_ctx* ctx, int gmres_m);

/* Advances the bound state by nsteps ESDIRK4(6) steps of size dt.  d_iwork:
 * caller-owned device memory of nsk_implicit_workspace_bytes(ctx,
 * opts->gmres_m) bytes, 256-byte aligned.  Synchronises the stream after
 * every Arnoldi step (the host needs the dot products).  Returns
 * NSK_ENOCONV, with the state left at the last completed step, when a stage
 * misses newton_tol after newton_max corrections; NSK_EUNSUPPORTED for mixed
 * precision, closure or sub-cell contexts; NSK_EINVAL for invalid options or precond 1
 * on a model 1 context.  stats_out (may be NULL) receives the counts. */
int nsk_esdirk_step(nsk_ctx* ctx, void* d_iwork, double dt, int nsteps, const nsk_implicit_opts* opts,
                    nsk_implicit_stats* stats_out);

/* ------------------------------------------------------------------------
 * Learned closure (no counterpart in the paper; the paper's model II is the
 * closure-free method).  A per-node network
 *   x -> 64 -> 64 -> 64 -> y,  ReLU on the hidden layers,
 * with BF16 parameters and FP32 accumulation, adds to the right-hand side
 *   momentum: out_m y_0 n,   c: out_c y_1,   n = g / sqrt(|g|^2 + g0^2),
 * from element-local features of the state (g = grad rho and lap = the
 * Laplacian of rho, both from the collocation derivative applied inside the
 * element):
 *   x = ((rho - s0) k0, (c - s1) k1, |g| k2, lap k3).
 * Parameters are NSK_MLP_NPARAM BF16 values (IEEE binary32 truncated to the
 * upper 16 bits, rounded to nearest even), weights row-major [out][in]:
 *   W1[64][4] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[2][64] b4[2].
 * The closure is trained on nudged pairs of runs (nsk_closure_nudge) with
 * the training kernels below.
 * ------------------------------------------------------------------------ */
#define NSK_MLP_NPARAM 8770

typedef struct {
  float s0, k0;     /* rho feature: (rho - s0) k0                            */
  float s1, k1;     /* c feature: (c - s1) k1                                */
  float k2, k3;     /* |grad rho| k2, Laplacian of rho times k3              */
  float g0;         /* > 0: regularisation of the unit direction n           */
  float out_m;      /* scale of the momentum output                          */
  float out_c;      /* scale of the c output                                 */
} nsk_closure_norm;

/* Sets the network of a context created with params.closure = 1.  d_w_bf16
 * is a 16-byte aligned device pointer to NSK_MLP_NPARAM BF16 values that the
 * caller keeps valid and unchanged while the context steps (it is read, not
 * copied).
 * A closure kernel (features + network, FP32 result in the workspace) then
 * runs before the right-hand-side kernel, which adds the source in FP64:
 * in every stage (every_stage = 1), or in the first stage of each
 * nsk_rk_step step only, its source serving the step's five stages
 * (every_stage = 0; nsk_rhs always evaluates it).  NSK_EINVAL if the
 * context has closure = 0, an argument is NULL or d_w_bf16 misaligned,
 * every_stage is not 0 or 1, a scale is not finite or g0 <= 0.  nsk_rhs, nsk_rk_step and nsk_autotune
 * of a closure context return NSK_EINVAL until a network is set.  Host only. */
int nsk_closure_set(nsk_ctx* ctx, const uint16_t* d_w_bf16, const nsk_closure_norm* norm, int every_stage);

/* Why nsk_closure_run left the closure run (nsk_closure_report.reason). */
#define NSK_CLOSURE_KEPT 0      /* the closure run reached the end            */
#define NSK_CLOSURE_PARAMS 1    /* a network parameter is not finite          */
#define NSK_CLOSURE_NONPHYS 2   /* the state turned non-physical (diagnostics) */
#define NSK_CLOSURE_ENERGY 3    /* the energy grew beyond the tolerance       */

typedef struct {
  int fell_back;             /* 1: the run finished on the fallback context      */
  int reason;                /* NSK_CLOSURE_* above                              */
  long long closure_steps;   /* steps of size dt kept from the closure run       */
  long long fallback_steps;  /* steps of size dt / ratio on the fallback context */
  double e_start;            /* e_total of the initial state                     */
  double e_last;             /* e_total at the last check of the closure run     */
} nsk_closure_report;

/* The closure run with the plain large-alpha run as its fallback and as the
 * reference its error is measured against.
 * Advances the bound state of cl (params.closure = 1, network set, model
 * II at the moderate alpha) by nsteps steps of dt, checking its diagnostics
 * every check_every steps and copying every state that passes into the
 * bound state of ref (params.closure = 0, the plain run at the large alpha
 * whose relaxation limit the closure imitates (alpha -> infinity recovers
 * the NSK equations, Sec. 2.3), same mesh).  If a network parameter is not
 * finite (checked first), the state turns non-physical (NSK_ENONPHYS of the
 * diagnostics), or, with energy_tol >= 0, e_total exceeds its initial value
 * by more than energy_tol |e_start|, the remaining time is run on ref from
 * the last state that passed, in steps of dt / ratio (ratio >= 1: ref's step
 * is that fraction of cl's), and the result is copied back into cl.  Either
 * way the final state is cl's bound state; *report says which run produced
 * it.  Returns NSK_ENONPHYS if the initial state or the fallback run is
 * non-physical, NSK_EINVAL for mismatched contexts or arguments (checked
 * before any device call), NSK_EUNBOUND if either context is not bound.
 * Waits for both streams. */
int nsk_closure_run(nsk_ctx* cl, nsk_ctx* ref, double dt, int nsteps, int ratio, int check_every,
                    double energy_tol, nsk_closure_report* report);

/* One nudging step on the bound state of any context (training pairs):
 * with the reference state d_Uref (layout of the state, device) mapped into
 * this model's frame, U* = (rho_r, m_r, rho_r + cmap (c_r - rho_r)), and the
 * features x and direction n of the current state U under *norm (its
 * out_m, out_c are not used),
 *   d_X[node][4] = x(U),  d_Y[node][2] = ((m* - m).n / tau, (c* - c) / tau)
 * (either may be NULL; node = elem * (N+1)^dim + local node), then
 *   m += (dt / tau)(m* - m),  c += (dt / tau)(c* - c);  rho is unchanged.
 * tau > 0, dt >= 0, norm->g0 > 0.  Asynchronous on the bound stream. */
int nsk_closure_nudge(nsk_ctx* ctx, const nsk_closure_norm* norm, const double* d_Uref, double dt, double tau,
                      double cmap, float* d_X, float* d_Y);

/* Network outputs y (unscaled) of n feature vectors: d_X[n][4] -> d_Y[n][2],
 * with the inference kernel of the closure (BF16 MFMA).  d_w_bf16 and d_X
 * are 16-byte aligned (else NSK_EINVAL).  Device pointers; asynchronous on
 * hip_stream. */
int nsk_mlp_forward(const uint16_t* d_w_bf16, const float* d_X, long long n, float* d_Y, void* hip_stream);

/* Bytes of device workspace for nsk_mlp_loss_grad with n <= batch samples
 * and for nsk_mlp_moments. */
size_t nsk_mlp_workspace_bytes(long long batch);

/* Loss L = 1/(2n) sum_s sum_o (y_so - q_o t_so)^2 of n samples (targets t
 * scaled by q_0 = tscale0, q_1 = tscale1) and its gradient
 * with respect to the NSK_MLP_NPARAM parameters, in FP32 with the network's
 * rounding points (BF16 parameters, BF16 activations of the first two hidden
 * layers; the backward pass takes that rounding as the identity).  Sample s
 * is row d_idx[s] of d_X[.][4] and d_Y[.][2] (d_idx may be NULL: row s).
 * d_grad receives NSK_MLP_NPARAM floats, d_loss (may be NULL) one float.  The
 * per-workgroup partial sums are added in a fixed order (deterministic).
 * d_ws: nsk_mlp_workspace_bytes(n) bytes.  Asynchronous on hip_stream. */
int nsk_mlp_loss_grad(const uint16_t* d_w_bf16, const float* d_X, const float* d_Y, const int* d_idx, long long n,
                      float tscale0, float tscale1, void* d_ws, float* d_grad, float* d_loss, void* hip_stream);

/* Adam step t (>= 1) of Kingma and Ba on the FP32 master parameters
 * d_master, with first and second moments d_m, d_v (zero before step 1);
 * d_w_bf16 receives the master values rounded to BF16.  Asynchronous. */
int nsk_mlp_adam(float* d_master, uint16_t* d_w_bf16, float* d_m, float* d_v, const float* d_grad, int t,
                 double lr, double beta1, double beta2, double eps, void* hip_stream);

/* Column means and standard deviations of d_Y[n][ncol] (ncol <= 4):
 * d_out[0..ncol-1] = means, d_out[ncol..2 ncol-1] = standard deviations
 * (FP64, device).  d_ws: nsk_mlp_workspace_bytes(1) bytes.  Asynchronous. */
int nsk_mlp_moments(const float* d_Y, long long n, int ncol, void* d_ws, double* d_out, void* hip_stream);

/* ------------------------------------------------------------------------
 * Batched form: many 3D instances of uneven mesh size and degree advanced
 * together with one shared parameter set and one shared time step.  The
 * states of all instances are packed into one device buffer; instance i
 * starts nsk_batch_state_offset(i) doubles into it and has the layout of a
 * single context.  Instances of one degree form a group, split into chunks
 * of whole instances; each stage of a chunk runs one lifting and one
 * right-hand-side kernel over the chunk's (instance, element block) items,
 * either one workgroup per item or a persistent grid walking the list in
 * rounds.  Two full steps (ten stages of every chunk, chunk after chunk)
 * are captured into one HIP graph that nsk_batch_rk_step replays.
 * ------------------------------------------------------------------------ */
typedef struct nsk_batch nsk_batch;

/* meshes[0..ninst-1] must all be 3D, params->model 0, params->closure 0,
 * params->subcell 0 and params->flux 0 (Rusanov) (NSK_EUNSUPPORTED otherwise); the validation rules of
 * nsk_create apply per instance.  Host only. */
int nsk_batch_create(const nsk_mesh* meshes, int ninst, const nsk_params* params, nsk_batch** out);

/* Frees the batch and its instance contexts (waits for the bound stream). */
void nsk_batch_destroy(nsk_batch* b);

/* Doubles in the packed state buffer (each instance slice 256-byte aligned). */
size_t nsk_batch_state_size(const nsk_batch* b);

/* Offset in doubles of instance inst inside the packed state buffer. */
size_t nsk_batch_state_offset(const nsk_batch* b, int inst);

/* Bytes of device workspace nsk_batch_bind expects. */
size_t nsk_batch_workspace_bytes(const nsk_batch* b);

/* Binds caller-owned device memory: d_U and d_dU hold nsk_batch_state_size()
 * doubles each, d_work nsk_batch_workspace_bytes() bytes; all 256-byte
 * aligned.  hip_stream must be a created stream (not the null stream), since
 * the step graph is captured on it. */
int nsk_batch_bind(nsk_batch* b, double* d_U, double* d_dU, void* d_work, void* hip_stream);

/* Context of instance inst (owned by the batch, bound to its slices): use it
 * with nsk_set_state, nsk_get_state, nsk_rhs and nsk_diagnostics.  Do not
 * destroy it, rebind it or step it with nsk_rk_step. */
int nsk_batch_ctx(nsk_batch* b, int inst, nsk_ctx** out);

/* Smallest nsk_dt_estimate over the instances.  Waits for the stream. */
int nsk_batch_dt_estimate(nsk_batch* b, double cfl, double* dt_out);

/* Advances every instance by nsteps steps of size dt: nsteps/2 replays of
 * the captured two-step graph (re-captured when dt changes), then one
 * ordinary step if nsteps is odd.  Asynchronous. */
int nsk_batch_rk_step(nsk_batch* b, double dt, int nsteps);

/* Autotuner.  First every instance is tuned as by nsk_autotune (its
 * elements-per-workgroup variant and element order, used when it runs as a
 * chunk of its own).  Then per degree group, on the whole group as one
 * chunk, it times `reps` evaluations of the batch kernels (right-hand side
 * into scratch) for each variant (0, 1) and grid multiplier m in
 * {0, 2, 4, 8} (m = 0: one workgroup per item; otherwise a persistent grid
 * of m workgroups per CU), and last, with that shape, working-set budgets
 * of 0 (the whole group as one chunk), 128, 256 and 512 MiB over ten
 * consecutive stages: a group runs as chunks of whole instances whose
 * state, state copy, register and lifted gradients fit the budget, and a
 * graph replay runs the ten stages of one chunk back to back while its data
 * is still in the caches.  A chunk of one instance runs the single-mesh
 * kernels with the instance's own variant and order.  The fastest choices
 * are kept.  ms_out (may be NULL, 12 doubles per group) receives the means
 * per stage: at group*12 + variant*4 + multiplier index and at
 * group*12 + 8 + budget index.  Call between steps; waits for the stream. */
int nsk_batch_autotune(nsk_batch* b, int reps, double* ms_out);

/* Sets the launch of group `group` (the order of nsk_batch_groups) by hand:
 * elements-per-workgroup variant (0, 1) of the batch kernels and of every
 * instance, grid multiplier (0, 2, 4, 8), element order (0..5) of its
 * instances and working-set budget in MiB
 * (>= 0, 0: no chunking).  Results do not depend on these choices.  Call
 * between steps; waits for the stream. */
int nsk_batch_set_group(nsk_batch* b, int group, int variant, int gridmul, int order, int chunk_mib);

/* Describes up to max groups: polynomial degree, chosen variant, grid
 * multiplier (0: one workgroup per item), element order of the group's
 * first instance and working-set budget in MiB (0: no chunking).  Any output
 * pointer may be NULL.  Returns the number of groups. */
int nsk_batch_groups(const nsk_batch* b, int* N_out, int* variant_out, int* gridmul_out, int* order_out,
                     int* chunk_mib_out, int max);

/* Static text for an NSK_* code. */
const char* nsk_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
