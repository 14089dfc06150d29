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
 * Rusanov (local Lax-Friedrichs) convective flux, BR1 lifting of the
 * primitive variables (v, c) with central fluxes, arithmetic mean of the
 * viscous face fluxes, pointwise non-conservative source from the lifted
 * gradient of c, and the five-stage fourth-order 2N-storage Runge-Kutta
 * scheme of Carpenter and Kennedy.
 *
 * Mesh: periodic tensor-product grid of axis-aligned box elements.
 *
 * Data layout of every state array (device memory, double):
 *   U[var][elem][node], var = 0 rho, 1..dim rho v_d, dim+1 c;
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

#ifdef __cplusplus
extern "C" {
#endif

#define NSK_OK 0
#define NSK_EINVAL (-1)    /* invalid mesh, parameters or argument           */
#define NSK_ENONPHYS (-2)  /* non-finite values or rho outside (0, 3)        */
#define NSK_EHIP (-3)      /* HIP runtime error                              */
#define NSK_EUNBOUND (-4)  /* device memory not bound yet                    */
#define NSK_EUNSUPPORTED (-5) /* degree/dimension combination not built      */

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
  int flux;       /* 0 = Rusanov (the only flux built)                      */
  int diss_c;     /* 1 = Rusanov dissipation also on c, 0 = not on c        */
  int precision;  /* 0 = FP64 throughout; 1 = mixed (FP32 volume/surface)   */
  int closure;    /* reserved, must be 0                                    */
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
 * (NSK_EUNSUPPORTED for dim = 3 with N = 6, whose element tile exceeds 64 KB
 * of LDS),
 * non-increasing breakpoints, T outside (0,1), alpha <= 6 (1 - T), beta <= 0,
 * eps < 0, kappa < 0.  *out is set on success. */
int nsk_create(const nsk_mesh* mesh, const nsk_params* params, nsk_ctx** out);

/* Frees the host context (waits for the bound stream first). */
void nsk_destroy(nsk_ctx* ctx);

/* Number of doubles in one state array: (dim+2) * elements * (N+1)^dim. */
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

/* Semi-discrete right-hand side R = dU/dt of the device state d_U
 * (any array with the state layout, not necessarily the bound one), source
 * included.  d_R must not alias d_U.  The scheme is autonomous, t is unused. */
int nsk_rhs(nsk_ctx* ctx, const double* d_U, double* d_R, double t);

/* Time-step estimate for the bound state:
 *   dt = cfl * min(1/((2N+1) max_e sum_d max(|v_d|+a)/h_d),
 *                  1/((2N+1)^2 max_e sum_d max(eps, kappa/beta)/h_d^2),
 *                  z_R beta/alpha)
 * with a = sqrt(p'(rho) + alpha rho) and z_R the negative-real-axis
 * stability limit of the Runge-Kutta scheme.  Waits for the stream. */
int nsk_dt_estimate(nsk_ctx* ctx, double cfl, double* dt_out);

/* Advances the bound state by nsteps steps of size dt (five stages each).
 * Asynchronous.  On return of the enqueued work the state is in d_U. */
int nsk_rk_step(nsk_ctx* ctx, double dt, int nsteps);

/* Diagnostics of the bound state (quadrature over all elements, with the
 * lifted gradient of c in the capillary energy).  Waits for the stream.
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
 * pair with HIP events, keeps the fastest in the context and returns it;
 * ms_out (12 doubles, may be NULL) receives the mean ms per evaluation at
 * index variant * 6 + order (-1 for pairs skipped because they coincide with
 * another, e.g. tiled orders in 1D).  Uses the workspace's second state
 * buffer as scratch, so it must be called between steps, and waits for the
 * stream. */
int nsk_autotune(nsk_ctx* ctx, int reps, int* variant_out, int* order_out, double* ms_out);

/* Changes alpha, beta, eps, kappa of an existing context (same mesh). */
int nsk_set_params(nsk_ctx* ctx, const nsk_params* params);

/* Kernel timing with HIP events on the bound stream (measurement only).
 * nsk_timing_enable(ctx, 1) makes every stage enqueued by nsk_rk_step record
 * events before the lifting kernel, between the two kernels and after the
 * right-hand-side/update kernel (at most 4096 stages until the next read).
 * nsk_timing_read waits for the stream and returns out[0] = summed ms of the
 * lifting kernel, out[1] = summed ms of the right-hand-side/update kernel,
 * out[2] = number of stages timed, then clears the record.
 * nsk_timing_enable(ctx, 0) stops recording and releases the events. */
int nsk_timing_enable(nsk_ctx* ctx, int enable);
int nsk_timing_read(nsk_ctx* ctx, double out[3]);

/* ------------------------------------------------------------------------
 * Batched form: many 3D instances of uneven mesh size and degree advanced
 * together with one shared parameter set and one shared time step.  The
 * states of all instances are packed into one device buffer; instance i
 * starts nsk_batch_state_offset(i) doubles into it and has the layout of a
 * single context.  Instances of one degree form a group; each stage runs one
 * lifting and one right-hand-side kernel per group over the group's list of
 * (instance, element block) items, either one workgroup per item or a
 * persistent grid walking the list in rounds, and two full steps (ten
 * stages) are captured into one HIP graph that nsk_batch_rk_step replays.
 * ------------------------------------------------------------------------ */
typedef struct nsk_batch nsk_batch;

/* meshes[0..ninst-1] must all be 3D (NSK_EUNSUPPORTED otherwise); the
 * validation rules of nsk_create apply per instance.  Host only. */
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

/* Autotuner per degree group: times `reps` evaluations of the group's two
 * kernels (right-hand side into scratch), first for each element order
 * 0..5 of nsk_set_tile applied to every member instance, then, with the
 * fastest order, for each elements-per-workgroup variant (0, 1) and grid
 * multiplier m in {0, 2, 4, 8} (m = 0: one workgroup per item; otherwise a
 * persistent grid of m workgroups per CU), and keeps the fastest per group.
 * ms_out (may be NULL, 14 doubles per group) receives the means: at
 * group*14 + variant*4 + multiplier index, and at group*14 + 8 + order.
 * Call between steps; waits for the stream. */
int nsk_batch_autotune(nsk_batch* b, int reps, double* ms_out);

/* Describes up to max groups: polynomial degree, chosen variant, grid
 * multiplier (0: one workgroup per item) and element order of the member
 * instances.  Any output pointer may be NULL.  Returns the number of
 * groups. */
int nsk_batch_groups(const nsk_batch* b, int* N_out, int* variant_out, int* gridmul_out, int* order_out, int max);

/* Static text for an NSK_* code. */
const char* nsk_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
