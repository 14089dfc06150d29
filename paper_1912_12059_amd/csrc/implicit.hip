// libnsk: implicit time stepping with the six-stage fourth-order ESDIRK
// scheme named in Sec. 3.1 for the implicit runs (Kennedy and Carpenter's
// ARK4(3)6L[2]SA implicit tableau: gamma = 1/4, explicit first stage,
// stiffly accurate), with a Jacobian-free Newton-Krylov solver for the stage
// equations.
//
// One step from U_n:  K_1 = R(U_n); for stage i = 2..6 solve
//   G(X) = X - dt gamma R(X) - B_i = 0,   B_i = U_n + dt sum_{j<i} a_ij K_j,
// by Newton's method, each correction from one cycle of right-preconditioned
// GMRES with classical Gram-Schmidt (repeated when the projection cancels
// most of the vector) and the Jacobian-vector product (R(X + s z) - R(X))/s;
// then K_i = (X - B_i)/(dt gamma); U_{n+1} is the last stage's X.  Every
// right-hand side is nsk_rhs on the bound context; the vector work runs in
// the kernels below, with fixed-order reductions, so a run is bitwise
// reproducible.  The host reads back only the dot products of each Arnoldi
// step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

#include "../../include/nsk.h"
#include "host_common.hpp"

using namespace nsk;

namespace {

constexpr int kVecThreads = 256;
constexpr int kDotBlocks = 1024;  // partial sums per dot product
constexpr int kLinTerms = 8;      // vectors per linear-combination launch

struct LinArgs {
  const double* x[kLinTerms];
  double a[kLinTerms];
  int nk;
};

// Calls f(std::integral_constant<int, K>{}) for the runtime count k in
// [0, kLinTerms]: the vector kernels take their vector count as a template
// parameter, so that all of an entry's loads issue together instead of one
// branch and wait per vector.
template <typename F>
void with_count(int k, F&& f) {
  switch (k) {
    case 0: f(std::integral_constant<int, 0>{}); break;
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    default: f(std::integral_constant<int, 8>{}); break;
  }
}
static_assert(kLinTerms == 8, "with_count covers counts up to 8");

// y[i] = sum_{k < NK} a_k x_k[i] (y may be one of the x_k: each entry is read
// before it is written by the same thread)
template <int NK>
__global__ void __launch_bounds__(kVecThreads) lincomb_kernel(LinArgs L, double* y, long long n) {
  const long long stride = (long long)gridDim.x * kVecThreads;
  for (long long i = (long long)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NK; ++k) s += L.a[k] * L.x[k][i];
    y[i] = s;
  }
}

// part[b * ld + j] = sum over block b's contiguous chunk of w[i] * v_j[i],
// v_j = V + j * vstride, for j < NJ <= kLinTerms; with self, also
// part[b * ld + NJ] = the chunk's sum of w[i]^2.  V is the Krylov basis
// (FP64 or FP32); products and sums are FP64.
template <typename VT, int NJ>
__global__ void __launch_bounds__(kVecThreads) multidot_kernel(const double* __restrict__ w,
                                                               const VT* __restrict__ V, long long vstride,
                                                               int self, long long n, double* __restrict__ part,
                                                               int ld) {
  __shared__ double red[NJ + 1][kVecThreads / 64];
  const long long chunk = (n + gridDim.x - 1) / gridDim.x;
  const long long beg = (long long)blockIdx.x * chunk;
  const long long end = beg + chunk < n ? beg + chunk : n;
  double s[NJ + 1];
#pragma unroll
  for (int j = 0; j <= NJ; ++j) s[j] = 0.0;
  for (long long i = beg + threadIdx.x; i < end; i += kVecThreads) {
    const double wi = w[i];
#pragma unroll
    for (int j = 0; j < NJ; ++j) s[j] += wi * double(V[j * vstride + i]);
    s[NJ] += wi * wi;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j <= NJ; ++j) {
    double v = s[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[j][wv] = v;
  }
  __syncthreads();
  const int outs = NJ + (self ? 1 : 0);
  if (threadIdx.x < outs) {
    const int j = threadIdx.x;
    double t = 0.0;
    for (int k = 0; k < kVecThreads / 64; ++k) t += red[j][k];
    part[(long long)blockIdx.x * ld + threadIdx.x] = t;
  }
}

// y[i] = aw w[i] + sum_{j < NK} a_j v_j[i], v_j = V + j * vstride (NK <=
// kLinTerms; w may be null; y may be w)
struct BasisCoefs {
  double a[kLinTerms];
};
template <typename VT, typename OT, int NK>
__global__ void __launch_bounds__(kVecThreads) basis_comb_kernel(const double* w, double aw,
                                                                 const VT* __restrict__ V, long long vstride,
                                                                 BasisCoefs c, OT* y, long long n) {
  const long long stride = (long long)gridDim.x * kVecThreads;
  for (long long i = (long long)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride) {
    double t = w ? aw * w[i] : 0.0;
#pragma unroll
    for (int j = 0; j < NK; ++j) t += c.a[j] * double(V[j * vstride + i]);
    y[i] = OT(t);
  }
}

// out[j] = sum_b part[b * ld + j] in a fixed order; one workgroup per j
__global__ void __launch_bounds__(kVecThreads) dot_final_kernel(const double* __restrict__ part, int nb, int ld,
                                                                double* __restrict__ out) {
  __shared__ double red[kVecThreads];
  const int j = blockIdx.x;
  double t = 0.0;
  for (int b = threadIdx.x; b < nb; b += kVecThreads) t += part[(long long)b * ld + j];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int w = kVecThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

// Node-local preconditioner of the relaxation source (model II): with
// a = dt gamma alpha / beta the stiff part of I - dt gamma dR/dU at a node is
// identity except the c row, (1 + a) c - a rho; its inverse maps v to v with
// c replaced by (v_c + a v_rho) / (1 + a).
struct Precond {
  int on;
  int ci;      // index of the c variable
  double a;
  long long S; // entries per variable
};

template <typename VT>
__device__ __forceinline__ double pinv(const VT* __restrict__ v, long long i, const Precond& p) {
  const long long c0 = (long long)p.ci * p.S;  // first entry of the c variable
  if (p.on && i >= c0 && i - c0 < p.S) {
    const long long o = i - c0;
    return (double(v[i]) + p.a * double(v[o])) / (1.0 + p.a);
  }
  return double(v[i]);
}

// Xp = X + s P^{-1} v
template <typename VT>
__global__ void __launch_bounds__(kVecThreads) perturb_kernel(const double* __restrict__ X,
                                                              const VT* __restrict__ v, double s, Precond p,
                                                              double* __restrict__ Xp, long long n) {
  const long long stride = (long long)gridDim.x * kVecThreads;
  for (long long i = (long long)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride)
    Xp[i] = X[i] + s * pinv(v, i, p);
}

// w = (P^{-1} v - v) - c (Rp - RX), c = dt gamma / s: the product of v with
// B = A - I, where A = (I - dt gamma dR/dU) P^{-1} is the GMRES operator.
// A and B span the same Krylov spaces and A's Hessenberg matrix is B's plus
// the identity; A is close to the identity, so projecting A v onto the basis
// would cancel most of it, while B v keeps only the part that is not v.
template <typename VT>
__global__ void __launch_bounds__(kVecThreads) jvp_kernel(const VT* __restrict__ v,
                                                          const double* __restrict__ Rp,
                                                          const double* __restrict__ RX, double c, Precond p,
                                                          double* __restrict__ w, long long n) {
  const long long stride = (long long)gridDim.x * kVecThreads;
  for (long long i = (long long)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride)
    w[i] = (pinv(v, i, p) - double(v[i])) - c * (Rp[i] - RX[i]);
}

// X += P^{-1} Y
__global__ void __launch_bounds__(kVecThreads) correct_kernel(double* __restrict__ X, const double* __restrict__ Y,
                                                              Precond p, long long n) {
  const long long stride = (long long)gridDim.x * kVecThreads;
  for (long long i = (long long)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride)
    X[i] += pinv(Y, i, p);
}

// ESDIRK4(6) implicit tableau (lower triangle with the diagonal gamma), gamma = 1/4.
constexpr double kGamma = 0.25;
const double kA[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 4, 0.25, 0, 0, 0, 0},
    {8611.0 / 62500, -1743.0 / 31250, 0.25, 0, 0, 0},
    {5012029.0 / 34652500, -654441.0 / 2922500, 174375.0 / 388108, 0.25, 0, 0},
    {15267082809.0 / 155376265600, -71443401.0 / 120774400, 730878875.0 / 902184768, 2285395.0 / 8070912, 0.25,
     0},
    {82889.0 / 524892, 0.0, 15625.0 / 83664, 69875.0 / 102672, -2260.0 / 8211, 0.25},
};

// Workspace: FP64 vectors (each M doubles, padded to 256 bytes), then the
// Krylov basis V_0..V_m (FP64 or FP32), then the reduction scratch
enum { vK0 = 0, vB = 5, vX, vRX, vR, vXp, vRp, vY, vW, kNumVec };

struct Solver {
  nsk_ctx* c;
  char* base;
  long long M;       // doubles per state vector
  long long stride;  // doubles between workspace vectors
  int m;
  double* part;
  double* dots;
  hipStream_t st;
  Precond pre;
  nsk_implicit_stats* stats;

  int f32;            // Krylov basis in FP32
  double reorth_tol;  // second projection when |w'|^2 <= reorth_tol |w|^2
  long long vstride;  // elements between basis vectors
  double* vec(int k) const { return reinterpret_cast<double*>(base) + (long long)k * stride; }
  template <typename VT>
  VT* V(int k) const {
    return reinterpret_cast<VT*>(reinterpret_cast<double*>(base) + (long long)kNumVec * stride) + (long long)k * vstride;
  }
  unsigned grid() const {
    const long long b = (M + kVecThreads - 1) / kVecThreads;
    return (unsigned)(b < 8192 ? b : 8192);
  }

  int lin(double* y, int nk, const double* const* x, const double* a) {
    // chains of kLinTerms terms: y = sum; later chunks add onto y
    int k0 = 0;
    bool first = true;
    while (k0 < nk || first) {
      LinArgs L;
      std::memset(&L, 0, sizeof(L));
      int t = 0;
      if (!first) { L.x[t] = y; L.a[t] = 1.0; ++t; }
      while (t < kLinTerms && k0 < nk) { L.x[t] = x[k0]; L.a[t] = a[k0]; ++t; ++k0; }
      L.nk = t;
      with_count(t, [&](auto K) {
        hipLaunchKernelGGL(lincomb_kernel<decltype(K)::value>, dim3(grid()), dim3(kVecThreads), 0, st, L, y, M);
      });
      first = false;
    }
    return hipGetLastError() == hipSuccess ? NSK_OK : NSK_EHIP;
  }

  // h[j] = <w, V_j> for j < nj and h[nj] = <w, w> (synchronous)
  template <typename VT>
  int dot_basis(const double* w, int nj, double* h) {
    int j0 = 0;
    do {
      const int nn = nj - j0 < kLinTerms ? nj - j0 : kLinTerms;
      const bool last = j0 + nn >= nj;
      with_count(nn, [&](auto K) {
        hipLaunchKernelGGL((multidot_kernel<VT, decltype(K)::value>), dim3(kDotBlocks), dim3(kVecThreads), 0, st, w,
                           V<VT>(j0), vstride, last ? 1 : 0, M, part + j0, m + 3);
      });
      j0 += nn;
    } while (j0 < nj);
    return fetch_dots(nj + 1, h);
  }

  int fetch_dots(int nout, double* h) {
    hipLaunchKernelGGL(dot_final_kernel, dim3(nout), dim3(kVecThreads), 0, st, part, kDotBlocks, m + 3, dots);
    if (hipGetLastError() != hipSuccess) return NSK_EHIP;
    if (hipMemcpyAsync(h, dots, sizeof(double) * nout, hipMemcpyDeviceToHost, st) != hipSuccess) return NSK_EHIP;
    return hipStreamSynchronize(st) == hipSuccess ? NSK_OK : NSK_EHIP;
  }

  int norm(const double* w, double* out) {
    hipLaunchKernelGGL((multidot_kernel<double, 0>), dim3(kDotBlocks), dim3(kVecThreads), 0, st, w, w, 0LL, 1, M,
                       part, m + 3);
    int rc = fetch_dots(1, out);
    *out = std::sqrt(*out);
    return rc;
  }

  // y = aw w + sum_{j<nk} a_j V_j for any nk: launches of kLinTerms basis
  // vectors, the partial sums accumulated in the FP64 vector acc (which may
  // be w) when more than one launch is needed
  template <typename VT, typename OT>
  int comb(const double* w, double aw, int nk, const double* a, OT* y, double* acc) {
    int j0 = 0;
    const double* src = w;
    double asrc = aw;
    while (nk - j0 > kLinTerms) {
      BasisCoefs cf;
      for (int j = 0; j < kLinTerms; ++j) cf.a[j] = a[j0 + j];
      hipLaunchKernelGGL((basis_comb_kernel<VT, double, kLinTerms>), dim3(grid()), dim3(kVecThreads), 0, st, src,
                         asrc, V<VT>(j0), vstride, cf, acc, M);
      src = acc;
      asrc = 1.0;
      j0 += kLinTerms;
    }
    BasisCoefs cf;
    std::memset(&cf, 0, sizeof(cf));
    for (int j = j0; j < nk; ++j) cf.a[j - j0] = a[j];
    with_count(nk - j0, [&](auto K) {
      hipLaunchKernelGGL((basis_comb_kernel<VT, OT, decltype(K)::value>), dim3(grid()), dim3(kVecThreads), 0, st, src,
                         asrc, V<VT>(j0), vstride, cf, y, M);
    });
    return hipGetLastError() == hipSuccess ? NSK_OK : NSK_EHIP;
  }

  int rhs(const double* X, double* R) {
    ++stats->rhs_evals;
    return nsk_rhs(c, X, R, 0.0);
  }

  int gmres(double dtg, double xnorm, double rtol, int* iters) {
    return f32 ? gmres_t<float>(dtg, xnorm, rtol, iters) : gmres_t<double>(dtg, xnorm, rtol, iters);
  }

  // One GMRES cycle for (I - dtg J) P^{-1} y = r, r in vR; X += P^{-1} V y.
  template <typename VT>
  int gmres_t(double dtg, double xnorm, double rtol, int* iters) {
    double beta;
    int rc = norm(vec(vR), &beta);
    if (rc) return rc;
    *iters = 0;
    if (!(beta > 0.0)) return NSK_OK;
    if ((rc = comb<VT, VT>(vec(vR), 1.0 / beta, 0, nullptr, V<VT>(0), vec(vW)))) return rc;
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1, 0.0), h(m + 2), h2(m + 2);
    g[0] = beta;
    const double s = std::sqrt(2.2204460492503131e-16) * (1.0 + xnorm);
    int kd = 0;
    std::vector<double> cf(m + 1);
    for (int k = 0; k < m; ++k) {
      hipLaunchKernelGGL(perturb_kernel<VT>, dim3(grid()), dim3(kVecThreads), 0, st, vec(vX), V<VT>(k), s, pre,
                         vec(vXp), M);
      if ((rc = rhs(vec(vXp), vec(vRp)))) return rc;
      double* w = vec(vW);
      hipLaunchKernelGGL(jvp_kernel<VT>, dim3(grid()), dim3(kVecThreads), 0, st, V<VT>(k), vec(vRp), vec(vRX),
                         dtg / s, pre, w, M);
      // classical Gram-Schmidt: one multi-dot gives <w, V_0..V_k> and |w|^2
      // together; |w - sum h_j V_j|^2 then follows from Pythagoras, and the
      // subtraction and the normalisation into V_{k+1} are one combination.
      // When |w - sum h_j V_j|^2 <= reorth_tol |w|^2 (1/2: Kahan's criterion,
      // more than 1/sqrt(2) of |w| cancelled) the projection is repeated on
      // the FP64 w and the norm taken again.
      if ((rc = dot_basis<VT>(w, k + 1, h.data()))) return rc;
      const double ww = h[k + 1];
      double proj = 0.0;
      for (int j = 0; j <= k; ++j) proj += h[j] * h[j];
      double hk1 = ww - proj > 0.0 ? std::sqrt(ww - proj) : 0.0;
      const bool again = !(hk1 * hk1 > reorth_tol * ww) || !(hk1 > 0.0);
      for (int j = 0; j <= k; ++j) h2[j] = 0.0;
      if (!again) {
        for (int j = 0; j <= k; ++j) cf[j] = -h[j] / hk1;
        if ((rc = comb<VT, VT>(w, 1.0 / hk1, k + 1, cf.data(), V<VT>(k + 1), w))) return rc;
      } else {
        for (int j = 0; j <= k; ++j) cf[j] = -h[j];
        if ((rc = comb<VT, double>(w, 1.0, k + 1, cf.data(), w, w))) return rc;
        if ((rc = dot_basis<VT>(w, k + 1, h2.data()))) return rc;
        const double ww2 = h2[k + 1];
        double proj2 = 0.0;
        for (int j = 0; j <= k; ++j) proj2 += h2[j] * h2[j];
        hk1 = ww2 - proj2 > 0.0 ? std::sqrt(ww2 - proj2) : 0.0;
        const double sc = hk1 > 0.0 ? 1.0 / hk1 : 1.0;
        for (int j = 0; j <= k; ++j) cf[j] = -h2[j] * sc;
        if ((rc = comb<VT, VT>(w, sc, k + 1, cf.data(), V<VT>(k + 1), w))) return rc;
        ++stats->reorth;
      }
      for (int j = 0; j <= k; ++j) H[(size_t)j * m + k] = h[j] + h2[j];
      H[(size_t)k * m + k] += 1.0;  // A = I + B
      H[(size_t)(k + 1) * m + k] = hk1;
      // Givens rotations on the new column
      for (int j = 0; j < k; ++j) {
        const double t0 = H[(size_t)j * m + k], t1 = H[(size_t)(j + 1) * m + k];
        H[(size_t)j * m + k] = cs[j] * t0 + sn[j] * t1;
        H[(size_t)(j + 1) * m + k] = -sn[j] * t0 + cs[j] * t1;
      }
      const double a0 = H[(size_t)k * m + k], a1 = H[(size_t)(k + 1) * m + k];
      const double r = std::hypot(a0, a1);
      cs[k] = r > 0.0 ? a0 / r : 1.0;
      sn[k] = r > 0.0 ? a1 / r : 0.0;
      H[(size_t)k * m + k] = r;
      H[(size_t)(k + 1) * m + k] = 0.0;
      g[k + 1] = -sn[k] * g[k];
      g[k] = cs[k] * g[k];
      kd = k + 1;
      ++stats->gmres_iters;
      if (std::fabs(g[k + 1]) <= rtol * beta || !(hk1 > 0.0)) break;
    }
    // back substitution and the correction X += P^{-1} sum_j y_j V_j
    std::vector<double> y(kd);
    for (int i = kd - 1; i >= 0; --i) {
      double t = g[i];
      for (int j = i + 1; j < kd; ++j) t -= H[(size_t)i * m + j] * y[j];
      y[i] = t / H[(size_t)i * m + i];
    }
    if ((rc = comb<VT, double>(nullptr, 0.0, kd, y.data(), vec(vY), vec(vY)))) return rc;
    hipLaunchKernelGGL(correct_kernel, dim3(grid()), dim3(kVecThreads), 0, st, vec(vX), vec(vY), pre, M);
    *iters = kd;
    return hipGetLastError() == hipSuccess ? NSK_OK : NSK_EHIP;
  }
};

size_t vec_stride(const nsk_ctx* c) {
  const size_t M = (size_t)c->nvar * c->S;
  return (M + 31) / 32 * 32;
}

// doubles taken by the Krylov basis of gmres_m + 1 vectors (either precision)
size_t basis_doubles(const nsk_ctx* c, int gmres_m) { return (size_t)(gmres_m + 1) * vec_stride(c); }

int check_opts(const nsk_implicit_opts* o) {
  if (!o) return NSK_EINVAL;
  if (!(o->newton_tol > 0.0) || !std::isfinite(o->newton_tol) || o->newton_max < 1 || o->newton_max > 1000)
    return NSK_EINVAL;
  if (!(o->gmres_rtol > 0.0) || !(o->gmres_rtol < 1.0) || o->gmres_m < 1 || o->gmres_m > NSK_GMRES_MAX)
    return NSK_EINVAL;
  if (o->precond != 0 && o->precond != 1) return NSK_EINVAL;
  if (o->basis_fp32 != 0 && o->basis_fp32 != 1) return NSK_EINVAL;
  if (!(o->reorth_tol >= 0.0 && o->reorth_tol < 1.0)) return NSK_EINVAL;
  return NSK_OK;
}

}  // namespace

extern "C" {

size_t nsk_implicit_workspace_bytes(const nsk_ctx* c, int gmres_m) {
  if (!c || gmres_m < 1 || gmres_m > NSK_GMRES_MAX) return 0;
  return sizeof(double) * ((size_t)kNumVec * vec_stride(c) + basis_doubles(c, gmres_m) +
                           (size_t)kDotBlocks * (gmres_m + 3) + 256);
}

int nsk_esdirk_step(nsk_ctx* c, void* d_iwork, double dt, int nsteps, const nsk_implicit_opts* opts,
                    nsk_implicit_stats* stats_out) {
  if (!c || !d_iwork || nsteps < 0 || !(dt > 0.0) || !std::isfinite(dt)) return NSK_EINVAL;
  int rc = check_opts(opts);
  if (rc) return rc;
  if ((reinterpret_cast<uintptr_t>(d_iwork) & 255) != 0) return NSK_EINVAL;
  // finite-difference Jacobian products need FP64 right-hand sides
  // FV sub-cell right-hand sides switch elements and limit slopes: not differentiable
  if (c->par.precision != 0 || c->par.closure != 0 || c->par.subcell != 0) return NSK_EUNSUPPORTED;
  if (opts->precond == 1 && c->par.model != 0) return NSK_EINVAL;  // the relaxation source is model II's
  if (!c->bound) return NSK_EUNBOUND;
  if (c->cur != 0) return NSK_EINVAL;

  nsk_implicit_stats stats;
  std::memset(&stats, 0, sizeof(stats));
  stats.converged = 1;
  Solver S;
  S.c = c;
  S.base = static_cast<char*>(d_iwork);
  S.M = (long long)c->nvar * c->S;
  S.stride = (long long)vec_stride(c);
  S.m = opts->gmres_m;
  S.f32 = opts->basis_fp32;
  S.reorth_tol = opts->reorth_tol;
  S.vstride = S.stride;  // elements of either precision (an FP32 basis fills half its region)
  S.part = reinterpret_cast<double*>(S.base) + (long long)kNumVec * S.stride + (long long)basis_doubles(c, S.m);
  S.dots = S.part + (long long)kDotBlocks * (S.m + 3);
  S.st = c->stream;
  S.stats = &stats;
  const double dtg = dt * kGamma;
  S.pre.on = opts->precond;
  S.pre.ci = c->dim + 1;
  S.pre.a = dtg * c->par.alpha / c->par.beta;
  S.pre.S = c->S;

  double* U = c->U;
  for (int step = 0; step < nsteps && rc == NSK_OK; ++step) {
    if ((rc = S.rhs(U, S.vec(vK0)))) break;
    for (int i = 1; i < 6 && rc == NSK_OK; ++i) {
      // B = U + dt sum_{j<i} a_ij K_j
      std::vector<const double*> xs{U};
      std::vector<double> as{1.0};
      for (int j = 0; j < i; ++j)
        if (kA[i][j] != 0.0) { xs.push_back(S.vec(vK0 + j)); as.push_back(dt * kA[i][j]); }
      if ((rc = S.lin(S.vec(vB), (int)xs.size(), xs.data(), as.data()))) break;
      // predictor X = B + dt gamma K_{i-1}
      {
        const double* x[2] = {S.vec(vB), S.vec(vK0 + i - 1)};
        const double a[2] = {1.0, dtg};
        if ((rc = S.lin(S.vec(vX), 2, x, a))) break;
      }
      double bnorm;
      if ((rc = S.norm(S.vec(vB), &bnorm))) break;
      bool conv = false;
      double res = 0.0;
      for (int it = 0; it <= opts->newton_max; ++it) {
        if ((rc = S.rhs(S.vec(vX), S.vec(vRX)))) break;
        // r = B + dtg R(X) - X = -G(X)
        const double* x[3] = {S.vec(vB), S.vec(vRX), S.vec(vX)};
        const double a[3] = {1.0, dtg, -1.0};
        if ((rc = S.lin(S.vec(vR), 3, x, a))) break;
        double rn;
        if ((rc = S.norm(S.vec(vR), &rn))) break;
        res = rn / (bnorm > 0.0 ? bnorm : 1.0);
        if (!std::isfinite(rn)) { rc = NSK_ENONPHYS; break; }
        if (res <= opts->newton_tol) { conv = true; break; }
        if (it == opts->newton_max) break;
        double xnorm;
        if ((rc = S.norm(S.vec(vX), &xnorm))) break;
        int gi = 0;
        if ((rc = S.gmres(dtg, xnorm, opts->gmres_rtol, &gi))) break;
        ++stats.newton_iters;
      }
      if (rc) break;
      if (res > stats.max_residual) stats.max_residual = res;
      if (!conv) { stats.converged = 0; rc = NSK_ENOCONV; break; }
      if (i < 5) {
        // K_i = (X - B) / (dt gamma)
        const double* x[2] = {S.vec(vX), S.vec(vB)};
        const double a[2] = {1.0 / dtg, -1.0 / dtg};
        if ((rc = S.lin(S.vec(vK0 + i), 2, x, a))) break;
      }
    }
    if (rc) break;
    // stiffly accurate: U_{n+1} is the last stage
    if (hipMemcpyAsync(U, S.vec(vX), sizeof(double) * S.M, hipMemcpyDeviceToDevice, S.st) != hipSuccess) {
      rc = NSK_EHIP;
      break;
    }
    ++stats.steps;
  }
  if (hipStreamSynchronize(S.st) != hipSuccess && rc == NSK_OK) rc = NSK_EHIP;
  if (stats_out) *stats_out = stats;
  return rc;
}

}  // extern "C"
