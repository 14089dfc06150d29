// Host-side pieces shared by the single-mesh and the batched C ABI: the 1D
// basis, the Runge-Kutta coefficients, parameter checks, the context
// structure, work orders and the kernel-argument builders.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/nsk.h"
#include "dg_kernels.hpp"

using namespace nsk;

namespace {

// ---------------------------------------------------------------------------
// 1D basis (Sec. 3.1): nodes are the roots of P_{N+1}; for Gauss nodes the
// derivative matrix has the closed form
//   D_ij = P'(x_i) / (P'(x_j) (x_i - x_j))  (i != j),   D_ii = x_i / (1 - x_i^2)
// and the weights are 2 / ((1 - x_i^2) P'(x_i)^2).
// ---------------------------------------------------------------------------
struct Basis1D {
  int np;
  double x[kMaxNP], w[kMaxNP], D[kMaxNP][kMaxNP], Dhat[kMaxNP][kMaxNP], Lm[kMaxNP], Lp[kMaxNP];
};

void legendre_eval(int n, long double x, long double& P, long double& dP) {
  // upward recurrence for P_k and P_k' together
  long double pm = 1.0L, p = x, dpm = 0.0L, dp = 1.0L;
  if (n == 0) { P = 1.0L; dP = 0.0L; return; }
  for (int k = 1; k < n; ++k) {
    long double pn = ((2 * k + 1) * x * p - k * pm) / (k + 1);
    long double dpn = dpm + (2 * k + 1) * p;  // P'_{k+1} = P'_{k-1} + (2k+1) P_k
    pm = p; p = pn;
    dpm = dp; dp = dpn;
  }
  P = p;
  dP = dp;
}

void make_basis(int N, Basis1D& b) {
  const int n = N + 1;
  b.np = n;
  long double x[kMaxNP], dPx[kMaxNP];
  for (int i = 0; i < n; ++i) {
    // ascending roots; initial guess from the asymptotic formula
    long double z = std::cos(3.141592653589793238462643383279L * (n - i - 0.25L) / (n + 0.5L));
    for (int it = 0; it < 60; ++it) {
      long double P, dP;
      legendre_eval(n, z, P, dP);
      long double step = P / dP;
      z -= step;
      if (std::fabs((double)step) < 1e-20) break;
    }
    long double P, dP;
    legendre_eval(n, z, P, dP);
    x[i] = z;
    dPx[i] = dP;
  }
  for (int i = 0; i < n; ++i) {
    b.x[i] = (double)x[i];
    b.w[i] = (double)(2.0L / ((1.0L - x[i] * x[i]) * dPx[i] * dPx[i]));
  }
  long double D[kMaxNP][kMaxNP];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      D[i][j] = (i == j) ? x[i] / (1.0L - x[i] * x[i]) : dPx[i] / (dPx[j] * (x[i] - x[j]));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      b.D[i][j] = (double)D[i][j];
      long double wi = 2.0L / ((1.0L - x[i] * x[i]) * dPx[i] * dPx[i]);
      long double wj = 2.0L / ((1.0L - x[j] * x[j]) * dPx[j] * dPx[j]);
      b.Dhat[i][j] = (double)(wj / wi * D[j][i]);
    }
  // Lagrange polynomials at the ends: l_j(s) = P(s) / (P'(x_j) (s - x_j))
  for (int j = 0; j < n; ++j) {
    long double Pp, dPp, Pm, dPm;
    legendre_eval(n, 1.0L, Pp, dPp);
    legendre_eval(n, -1.0L, Pm, dPm);
    b.Lp[j] = (double)(Pp / (dPx[j] * (1.0L - x[j])));
    b.Lm[j] = (double)(Pm / (dPx[j] * (-1.0L - x[j])));
  }
}

// Carpenter-Kennedy 2N-storage RK4(5) (the five-stage fourth-order
// low-storage scheme of Sec. 3.1).
const double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
const double kRkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};

// Negative-real-axis stability limit: apply one step to y' = -x y and find
// the first x where the amplification exceeds one.
double rk_amplification(double x) {
  double y = 1.0, k = 0.0;
  for (int s = 0; s < 5; ++s) {
    k = kRkA[s] * k + (-x) * y;
    y += kRkB[s] * k;
  }
  return std::fabs(y);
}

double rk_real_limit() {
  double lo = 0.0;
  while (rk_amplification(lo + 0.01) <= 1.0) lo += 0.01;
  double hi = lo + 0.01;
  for (int it = 0; it < 100; ++it) {
    double m = 0.5 * (lo + hi);
    (rk_amplification(m) <= 1.0 ? lo : hi) = m;
  }
  return lo;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Launch shapes: elements-per-workgroup variants x element work orders.
constexpr int kTileVariants = 2;
constexpr int kOrders = 6;
// order 0: natural element order in hardware round-robin; 1: natural order,
// one contiguous range per XCD; 2..5: x-y tiles of kTileEdge[order] elements
// (3D) marched along z, or x-strips of 4x that width marched along y (2D),
// one contiguous range per XCD.
constexpr int kTileEdge[kOrders] = {0, 0, 4, 6, 8, 12};
constexpr int kXcds = 8;

}  // namespace

struct nsk_ctx {
  nsk_mesh mesh;
  nsk_params par;
  int dim = 0, N = 0, np = 0, nn = 0, nvar = 0, ng = 0;
  bool uniform = true;  // no breakpoints: equal elements along every direction
  int nel[3] = {1, 1, 1};
  long long E = 0, S = 0;
  std::vector<double> h2[3];  // 2/h per element index
  Basis1D basis;
  double zR = 0.0;
  double rho_lo64 = 0.0, rho_hi64 = 0.0;
  // workspace layout (byte offsets)
  size_t off_U2 = 0, off_G = 0, off_h2[3] = {0, 0, 0}, off_wq = 0, off_order = 0, off_part = 0, off_out = 0;
  size_t off_cl = 0;  // closure source [dim+1][elem][node], FP32 (closure contexts only)
  size_t off_lf = 0;  // original NSK path: global LF speed, then per-workgroup partial maxima
  // FV sub-cells: flags, the elements needing sub-cell means, the means
  size_t off_sc_flags = 0, off_sc_need = 0, off_sc_Ub = 0, off_sc_Gb = 0;
  double sc_M[kMaxNP][kMaxNP] = {}, sc_Minv[kMaxNP][kMaxNP] = {}, sc_V[kMaxNP][kMaxNP] = {};
  size_t ws_bytes = 0;
  int diag_blocks = 0;
  int tile = 0;      // elements-per-workgroup variant
  int order = 0;     // element work order
  std::vector<int> order_host;
  // bound memory
  bool bound = false;
  double* U = nullptr;
  double* dU = nullptr;
  char* work = nullptr;
  hipStream_t stream = nullptr;
  int cur = 0;  // 0: state in U, 1: state in the workspace copy
  // learned closure: caller-owned BF16 parameters and the feature/output scaling
  const uint16_t* cl_w = nullptr;
  float cl_norm[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  int cl_every_stage = 1;  // 0: the closure source of a step's first stage serves all five
  int cl_stage = 0;        // stage index within the step being enqueued (0..4), -1 outside a step
  // optional kernel timing
  std::vector<hipEvent_t> events;  // 4 per timed stage
  int timed = 0;                   // stages recorded since the last read
  // two Runge-Kutta steps captured on the bound stream, and what the
  // captured launches depend on (a different key re-captures)
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<unsigned char> graph_key;
};

namespace {

int check_params(const nsk_params* p) {
  if (!p) return NSK_EINVAL;
  if (!(p->T > 0.0 && p->T < 1.0)) return NSK_EINVAL;
  if (!(p->eps >= 0.0) || !(p->kappa >= 0.0) || !std::isfinite(p->eps) || !std::isfinite(p->kappa))
    return NSK_EINVAL;
  if (p->subcell != 0 && p->subcell != 1) return NSK_EINVAL;
  if (p->model == 1) {
    // original NSK equations: global Lax-Friedrichs flux, FP64, no closure
    if (p->flux != 2 || p->precision != 0 || p->closure != 0 || p->subcell != 0) return NSK_EINVAL;
    return NSK_OK;
  }
  if (p->subcell == 1 && (p->precision != 0 || p->closure != 0 || !std::isfinite(p->subcell_threshold)))
    return NSK_EINVAL;
  if (p->model != 0) return NSK_EINVAL;
  if (!(p->alpha > 0.0) || !(p->beta > 0.0)) return NSK_EINVAL;
  if (!std::isfinite(p->alpha) || !std::isfinite(p->beta)) return NSK_EINVAL;
  // model II is hyperbolic only for alpha > -min W''(rho) = 6 (1 - T), the
  // minimum of the reduced Van-der-Waals W'' being taken at rho = 1
  if (!(p->alpha > 6.0 * (1.0 - p->T))) return NSK_EINVAL;
  if ((p->flux != 0 && p->flux != 1) || (p->closure != 0 && p->closure != 1)) return NSK_EINVAL;
  if (p->precision != 0 && p->precision != 1) return NSK_EINVAL;
  if (p->diss_c != 0 && p->diss_c != 1) return NSK_EINVAL;
  return NSK_OK;
}

// spinodal band of the reduced Van-der-Waals isotherm, widened by 0.05:
// the mixed-precision path evaluates the EoS in FP64 inside it
void spinodal_band(double T, double& lo, double& hi) {
  auto dp = [T](double r) { return 24.0 * T / ((3.0 - r) * (3.0 - r)) - 6.0 * r; };
  auto root = [&](double a, double b) {
    bool sa = dp(a) < 0;
    for (int i = 0; i < 200; ++i) {
      double m = 0.5 * (a + b);
      ((dp(m) < 0) == sa ? a : b) = m;
    }
    return 0.5 * (a + b);
  };
  lo = root(1e-6, 1.0) - 0.05;
  hi = root(1.0, 3.0 - 1e-9) + 0.05;
}

// Element work order for one of the kOrders choices (see kTileEdge).
void build_order(const nsk_ctx* c, int order, std::vector<int>& out) {
  const int E = (int)c->E, nx = c->nel[0], ny = c->nel[1], nz = c->nel[2];
  out.clear();
  out.reserve(E);
  const int T = kTileEdge[order];
  if (T == 0 || c->dim == 1) {
    for (int e = 0; e < E; ++e) out.push_back(e);
    return;
  }
  if (c->dim == 2) {
    const int W = 4 * T;
    for (int x0 = 0; x0 < nx; x0 += W)
      for (int y = 0; y < ny; ++y)
        for (int x = x0; x < std::min(nx, x0 + W); ++x) out.push_back(x + nx * y);
    return;
  }
  for (int y0 = 0; y0 < ny; y0 += T)
    for (int x0 = 0; x0 < nx; x0 += T)
      for (int z = 0; z < nz; ++z)
        for (int y = y0; y < std::min(ny, y0 + T); ++y)
          for (int x = x0; x < std::min(nx, x0 + T); ++x) out.push_back(x + nx * (y + ny * z));
}

int upload_order(nsk_ctx* c, int order) {
  build_order(c, order, c->order_host);
  if (hipMemcpyAsync(c->work + c->off_order, c->order_host.data(), sizeof(int) * c->order_host.size(),
                     hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return NSK_EHIP;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return NSK_EHIP;
  c->order = order;
  return NSK_OK;
}

BasisArgs basis_args(const nsk_ctx* c) {
  BasisArgs b;
  std::memset(&b, 0, sizeof(b));
  for (int i = 0; i < c->np; ++i) {
    for (int j = 0; j < c->np; ++j) b.Dhat[i][j] = c->basis.Dhat[i][j];
    b.Lm[i] = c->basis.Lm[i];
    b.Lp[i] = c->basis.Lp[i];
    b.invw[i] = 1.0 / c->basis.w[i];
  }
  return b;
}

MeshArgs mesh_args(const nsk_ctx* c) {
  MeshArgs m;
  for (int d = 0; d < 3; ++d) {
    m.h2[d] = reinterpret_cast<const double*>(c->work + c->off_h2[d]);
    m.nel[d] = c->nel[d];
  }
  m.order = reinterpret_cast<const int*>(c->work + c->off_order);
  m.E = (int)c->E;
  m.S = c->S;
  m.nxcd = c->order == 0 ? 1 : kXcds;
  return m;
}

PhysArgs phys_args(const nsk_ctx* c) {
  PhysArgs p;
  p.T = c->par.T;
  p.eps = c->par.eps;
  p.kappa = c->par.kappa;
  // the original NSK path has the plain Van-der-Waals pressure (alpha = 0)
  // and no relaxation terms
  const bool nsk = c->par.model == 1;
  p.alpha = nsk ? 0.0 : c->par.alpha;
  p.beta = c->par.beta;
  p.kb = nsk ? 0.0 : c->par.kappa / c->par.beta;
  p.ab = nsk ? 0.0 : c->par.alpha / c->par.beta;
  p.diss_c = c->par.diss_c;
  p.flux = c->par.flux;
  p.rho_lo64 = c->rho_lo64;
  p.rho_hi64 = c->rho_hi64;
  return p;
}

// Elements per workgroup: variant 0 is the largest count up to about 256
// threads whose right-hand-side LDS (FP64) stays within 40 KB; variant 1 is
// half of it (at least one).
template <int DIM, int NP>
struct Epb {
  using Sh = Shape<DIM, NP>;
  static constexpr int NX = Sh::NVAR + DIM + 1;
  static constexpr int lds(int epb) {
    return 8 * epb * (3 * NX * Sh::NN + Sh::NVAR * Sh::NN + 2 * Sh::NVAR * Sh::NF) + 1024;
  }
  static constexpr int pick(int epb) { return (epb <= 1 || lds(epb) <= 40960) ? (epb < 1 ? 1 : epb) : pick(epb - 1); }
  static constexpr int V0 = pick(256 / Sh::NN);
  static constexpr int V1 = V0 / 2 < 1 ? 1 : V0 / 2;
};

}  // namespace

namespace {
// FV sub-cell matrices for degree N: M[k][j] the mean of the Lagrange
// polynomial l_j over sub-cell k of N+1 equal sub-cells of [-1, 1] (Gauss
// quadrature with N+1 points on the sub-cell, exact), Minv its inverse, and
// V[k][i] = w_i P_k(x_i) with P_k the orthonormal Legendre polynomial, which
// maps nodal values to modal coefficients.
void subcell_matrices(const Basis1D& b, double M[kMaxNP][kMaxNP], double Minv[kMaxNP][kMaxNP],
                      double V[kMaxNP][kMaxNP]) {
  const int n = b.np;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int q = 0; q < n; ++q) {
        const double x = -1.0 + (2.0 / n) * (k + 0.5 * (b.x[q] + 1.0));
        double l = 1.0;
        for (int m = 0; m < n; ++m)
          if (m != j) l *= (x - b.x[m]) / (b.x[j] - b.x[m]);
        acc += 0.5 * b.w[q] * l;
      }
      M[k][j] = acc;
    }
  double A[kMaxNP][2 * kMaxNP];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < 2 * n; ++j) A[i][j] = j < n ? M[i][j] : (j - n == i ? 1.0 : 0.0);
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
    for (int j = 0; j < 2 * n; ++j) std::swap(A[c][j], A[piv][j]);
    const double d = A[c][c];
    for (int j = 0; j < 2 * n; ++j) A[c][j] /= d;
    for (int r = 0; r < n; ++r)
      if (r != c) {
        const double f = A[r][c];
        for (int j = 0; j < 2 * n; ++j) A[r][j] -= f * A[c][j];
      }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Minv[i][j] = A[i][n + j];
  for (int k = 0; k < n; ++k)
    for (int i = 0; i < n; ++i) {
      long double P, dP;
      legendre_eval(k, (long double)b.x[i], P, dP);
      V[k][i] = b.w[i] * std::sqrt(k + 0.5) * (double)P;
    }
}
}  // namespace
