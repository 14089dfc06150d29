// Device kernels of the DGSEM right-hand side for relaxation model II
// (Hitz, Keim, Munz, Rohde, Sec. 2.3 for the model, Sec. 3.1 for the scheme),
// written for gfx950 (64-wide wavefronts, 160 KB LDS per CU, 8 XCDs with a
// private 4 MB L2 each).
//
// One stage of the explicit scheme is two launches:
//   lift_kernel : state U -> G, where G holds per node the viscous stress
//                 tau (symmetric, dim(dim+1)/2 entries) and grad c, both built
//                 from the BR1-lifted gradients of the primitives (v, c)
//   rhs_kernel  : U, G -> volume integral + Rusanov/BR1 surface integral +
//                 pointwise source, then either R (dU/dt) or the fused
//                 low-storage Runge-Kutta stage update of U and the register.
//
// Work layout.  A workgroup owns EPB elements, one thread per (element, node).
// Direction by direction, the two neighbour elements across the d-faces are
// loaded whole with coalesced loads (one thread per node) into LDS: with
// Gauss-Legendre nodes the element ends are not nodes, so a face trace needs
// every node of the neighbour's line.  Face traces, the numerical flux and
// the contraction with the derivative matrix then work from LDS.  Each face
// value is computed identically by both elements sharing it (same operands,
// same order), so the scheme stays conservative bit for bit.
//
// Element order.  Which elements a workgroup owns comes from a host-built
// table.  The hardware hands consecutive workgroups to the XCDs in turn;
// renumbering the workgroups so that each XCD walks one contiguous range of
// that table, and building the table so that each range is a set of x-y tiles
// marched along z, keeps the neighbour re-reads inside the XCD's L2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace nsk {

constexpr int kMaxNP = 7;  // N <= 6

template <int B, int E>
struct ipow { static constexpr int v = B * ipow<B, E - 1>::v; };
template <int B>
struct ipow<B, 0> { static constexpr int v = 1; };

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// f(std::integral_constant<int, 0>), ..., f(std::integral_constant<int, K-1>)
template <int K, int I = 0, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < K) {
    f(std::integral_constant<int, I>{});
    static_for<K, I + 1>(f);
  }
}
constexpr int round64(int x) { return ((x + 63) / 64) * 64; }

template <int DIM, int NP>
struct Shape {
  static constexpr int NN = ipow<NP, DIM>::v;          // nodes per element
  static constexpr int NF = ipow<NP, DIM - 1>::v;      // nodes per face
  static constexpr int NVAR = DIM + 2;                 // rho, m, c
  static constexpr int NLIFT = DIM + 1;                // v, c
  static constexpr int NTAU = DIM * (DIM + 1) / 2;     // symmetric stress
  static constexpr int NG = NTAU + DIM;                // tau + grad c
};

template <int DIM, int NP, int EPB>
struct Tile {
  using Sh = Shape<DIM, NP>;
  static constexpr int THREADS = round64(cmax(EPB * Sh::NN, EPB * 2 * Sh::NF));
};

// stride of Gauss index along direction d inside an element
template <int NP>
__host__ __device__ constexpr int dstride(int d) { return d == 0 ? 1 : (d == 1 ? NP : NP * NP); }

// Index of tau_{ij} (i, j < DIM) inside the packed symmetric storage:
// diagonal first, then (0,1), (0,2), (1,2).
template <int DIM>
__host__ __device__ constexpr int tau_index(int i, int j) {
  if (i == j) return i;
  int a = i < j ? i : j, b = i < j ? j : i;
  if (DIM == 2) return 2;
  return a == 0 ? (b == 1 ? 3 : 4) : 5;
}

// Constants of the 1D basis and the geometry, passed by value.
struct BasisArgs {
  double Dhat[kMaxNP][kMaxNP];  // weak-form derivative operator
  double Lm[kMaxNP], Lp[kMaxNP];  // Lagrange polynomials at xi = -1, +1
  double invw[kMaxNP];          // 1 / Gauss weight
};

struct MeshArgs {
  const double* h2[3];  // 2 / h per element index along each direction
  const int* order;     // element of each position of the work order
  int nel[3];
  int E;                // number of elements
  long long S;          // E * NN, stride between variables
  int nxcd;             // XCDs sharing the work order in contiguous ranges
};

struct PhysArgs {
  double T, eps, kappa, alpha, beta;
  double kb;         // kappa / beta
  double ab;         // alpha / beta
  int diss_c;        // numerical-flux dissipation on c
  int flux;          // 0: Rusanov, 1: HLLC, 2: global Lax-Friedrichs
  double rho_lo64, rho_hi64;  // mixed precision: FP64 EoS inside this band
};

struct StageArgs {
  double A, B, dt;   // low-storage coefficients of the stage and step size
  int mode;          // 0: write R; 1: Runge-Kutta stage update
  const float* closure = nullptr;  // learned closure source [dim+1][elem][node], or none
  const double* lf = nullptr;      // global Lax-Friedrichs speed (original NSK path)
  const int* skip = nullptr;       // elements left to the FV sub-cell kernel (flag per element)
};

// -------------------------------------------------------------------------
// Thermodynamics of the reduced Van-der-Waals fluid (Sec. 2.1)
//   p = 8 T rho / (3 - rho) - 3 rho^2,   p' = 24 T / (3 - rho)^2 - 6 rho
// Model II modified pressure p_alpha = p + alpha rho^2 / 2 and sound speed
// a = sqrt(p_alpha') = sqrt(p' + alpha rho) (Sec. 2.3).
// -------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R p_alpha(R rho, R T, R alpha) {
  const R q = R(1) / (R(3) - rho);
  return R(8) * T * rho * q - R(3) * rho * rho + R(0.5) * alpha * rho * rho;
}

template <typename R>
__device__ __forceinline__ R sound_speed(R rho, R T, R alpha) {
  const R q = R(1) / (R(3) - rho);
  return sqrt(R(24) * T * q * q - R(6) * rho + alpha * rho);
}

// p_alpha and a together, sharing the reciprocal 1/(3 - rho)
template <typename R>
__device__ __forceinline__ void p_alpha_sound(R rho, R T, R alpha, R& pa, R& a) {
  const R q = R(1) / (R(3) - rho);
  pa = R(8) * T * rho * q - R(3) * rho * rho + R(0.5) * alpha * rho * rho;
  a = sqrt(R(24) * T * q * q - R(6) * rho + alpha * rho);
}

// EoS in the working precision R, except inside the spinodal band where the
// Van-der-Waals pressure is evaluated in FP64 (mixed-precision rule).
template <typename R>
__device__ __forceinline__ bool eos_in_fp64(double rho64, const PhysArgs& ph) {
  return sizeof(R) == sizeof(double) || (rho64 > ph.rho_lo64 && rho64 < ph.rho_hi64);
}

template <typename R>
__device__ __forceinline__ R p_alpha_guarded(double rho64, const PhysArgs& ph) {
  if (eos_in_fp64<R>(rho64, ph)) return R(p_alpha<double>(rho64, ph.T, ph.alpha));
  return p_alpha<R>(R(rho64), R(ph.T), R(ph.alpha));
}

template <typename R>
__device__ __forceinline__ void p_alpha_sound_guarded(double rho64, const PhysArgs& ph, R& pa, R& a) {
  if (eos_in_fp64<R>(rho64, ph)) {
    double p64, a64;
    p_alpha_sound<double>(rho64, ph.T, ph.alpha, p64, a64);
    pa = R(p64);
    a = R(a64);
  } else {
    p_alpha_sound<R>(R(rho64), R(ph.T), R(ph.alpha), pa, a);
  }
}

// Hardware hands consecutive workgroups to the XCDs in turn; renumber them
// so that XCD x works through one contiguous range of the work order.
__device__ __forceinline__ int remap_block(int b, int G, int nx) {
  if (nx <= 1) return b;
  const int q = G / nx, r = G - (G / nx) * nx;
  const int x = b % nx, i = b / nx;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Per-workgroup element data: element ids (-1 past the end), neighbour ids
// and 2/h.
template <int DIM, int EPB>
struct ElemInfo {
  int e[EPB];
  int nb[EPB][DIM][2];
  double h2[EPB][DIM];
};

template <int DIM, int EPB>
__device__ __forceinline__ void elem_info(ElemInfo<DIM, EPB>& info, const MeshArgs& m, int L, int tid) {
  if (tid < EPB) {
    const int pos = L * EPB + tid;
    const int e = pos < m.E ? m.order[pos] : -1;
    info.e[tid] = e;
    if (e >= 0) {
      int idx[3];
      idx[0] = e % m.nel[0];
      const int r = e / m.nel[0];
      idx[1] = DIM > 1 ? r % m.nel[1] : 0;
      idx[2] = DIM > 2 ? r / m.nel[1] : 0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        info.h2[tid][d] = m.h2[d][idx[d]];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          int j[3] = {idx[0], idx[1], idx[2]};
          j[d] = j[d] + (s ? 1 : -1);
          if (j[d] < 0) j[d] += m.nel[d];
          if (j[d] >= m.nel[d]) j[d] -= m.nel[d];
          info.nb[tid][d][s] = j[0] + m.nel[0] * (j[1] + m.nel[1] * j[2]);
        }
      }
    }
  }
}

// node with Gauss index 0 along d on the line of face node f
template <int NP>
__device__ __forceinline__ int face_base(int d, int f) {
  const int sd = dstride<NP>(d);
  return (f % sd) + sd * NP * (f / sd);
}

// face node of node n for direction d
template <int NP>
__device__ __forceinline__ int face_of(int d, int n) {
  const int sd = dstride<NP>(d);
  return (n % sd) + sd * (n / (sd * NP));
}

// Convective flux in direction d; irho = 1/rho; NV = DIM + 2 (model II, c
// not convected) or DIM + 1 (original NSK).
template <int DIM, typename R, int NV = DIM + 2>
__device__ __forceinline__ void conv_flux(int d, const R* u, R irho, R pa, R* F) {
  const R vd = u[1 + d] * irho;
  F[0] = u[1 + d];
#pragma unroll
  for (int j = 0; j < DIM; ++j) F[1 + j] = vd * u[1 + j] + (j == d ? pa : R(0));
  if constexpr (NV == DIM + 2) F[DIM + 1] = R(0);
}

// Original NSK path: the speed of the global Lax-Friedrichs flux at a node,
// max_d |v_d| + sqrt(max(p', 0)) (the sound speed is imaginary inside the
// spinodal interval).
template <int DIM>
__device__ __forceinline__ double lf_node_speed(const double* u, double T) {
  const double rho = u[0], q = 1.0 / (3.0 - rho);
  const double dp = 24.0 * T * q * q - 6.0 * rho;
  const double a = dp > 0.0 ? sqrt(dp) : 0.0;
  double m = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) m = fmax(m, fabs(u[1 + d] / rho));
  return m + a;
}

// Maximum of v over the workgroup, written by thread 0 to *out (all threads
// call it).
template <int THREADS>
__device__ __forceinline__ void block_max_store(double v, double* red, double* out, int tid) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    double m = red[0];
    for (int w = 1; w < (THREADS + 63) / 64; ++w) m = fmax(m, red[w]);
    *out = m;
  }
}

// -------------------------------------------------------------------------
// Lifting: G = (tau, grad s) from the BR1 gradients of (v, s), s = c for
// model II (MODEL 0) and s = rho for the original NSK path (MODEL 1):
//   q_d,i = (2/h_d) [ (L+_i w*_+ - L-_i w*_-) / omega_i - sum_l Dhat_il w_l ]
// along each d-line, w* = (w_left + w_right) / 2 on the faces.
// -------------------------------------------------------------------------
template <int DIM, int NP, int EPB, typename R, typename GT, int MODEL = 0>
__device__ __forceinline__ void lift_block(int L, int tid, const double* __restrict__ U, GT* __restrict__ G,
                                           const BasisArgs& bas, const MeshArgs& msh, const PhysArgs& ph,
                                           double* __restrict__ lfpart = nullptr) {
  using Sh = Shape<DIM, NP>;
  constexpr int NN = Sh::NN, NF = Sh::NF, NL = Sh::NLIFT;
  constexpr int NV = MODEL == 1 ? DIM + 1 : DIM + 2;  // conserved variables
  constexpr int SI = MODEL == 1 ? 0 : DIM + 1;        // the lifted scalar: rho or c
  __shared__ R sW[EPB][NL][NN];             // nodal primitives (v, s)
  __shared__ R sNbW[EPB][2][NL][NN];        // primitives of the two neighbours in direction d
  __shared__ R sWs[EPB][DIM][2][NL][NF];    // central face values w*
  __shared__ R sD[NP][NP];
  __shared__ R sLm[NP], sLp[NP], sIw[NP];
  __shared__ ElemInfo<DIM, EPB> info;

  const long long S = msh.S;
  if (tid < NP * NP) sD[tid / NP][tid % NP] = R(bas.Dhat[tid / NP][tid % NP]);
  if (tid < NP) { sLm[tid] = R(bas.Lm[tid]); sLp[tid] = R(bas.Lp[tid]); sIw[tid] = R(bas.invw[tid]); }
  elem_info<DIM, EPB>(info, msh, L, tid);
  __syncthreads();

  const int el = tid / NN, n = tid - (tid / NN) * NN;
  const int e = el < EPB ? info.e[el] : -1;
  const bool active = e >= 0;

  double lfs = 0.0;  // global Lax-Friedrichs speed at this node (MODEL 1)
  if (active) {
    const long long o = (long long)e * NN + n;
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = U[v * S + o];
    const double irho = 1.0 / u[0];
#pragma unroll
    for (int d = 0; d < DIM; ++d) sW[el][d][n] = R(u[1 + d] * irho);
    sW[el][DIM][n] = R(u[SI]);
    if constexpr (MODEL == 1) lfs = lf_node_speed<DIM>(u, ph.T);
  }
  if constexpr (MODEL == 1) {
    __shared__ double sRed[(Tile<DIM, NP, EPB>::THREADS + 63) / 64];
    if (lfpart) block_max_store<Tile<DIM, NP, EPB>::THREADS>(lfs, sRed, lfpart + L, tid);
  }

  // the next direction's neighbour states are fetched into registers while
  // the current direction's face values are formed
  double nbu[2][NV];
  auto fetch_nb = [&](auto dc) {
    constexpr int dd = decltype(dc)::value;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const long long on = (long long)info.nb[el][dd][s] * NN + n;
#pragma unroll
      for (int v = 0; v < NV; ++v) nbu[s][v] = U[v * S + on];
    }
  };
  if (active) fetch_nb(std::integral_constant<int, 0>{});

  // Per direction: stage the neighbours' primitives, then the central face
  // values.  (Double-buffering the neighbours so that the face values of d
  // share a phase with the staging of d+1 costs occupancy and was slower.)
  auto stage = [&](auto dc) {
    constexpr int d = decltype(dc)::value;
    if (active) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const double irho = 1.0 / nbu[s][0];
#pragma unroll
        for (int k = 0; k < DIM; ++k) sNbW[el][s][k][n] = R(nbu[s][1 + k] * irho);
        sNbW[el][s][DIM][n] = R(nbu[s][SI]);
      }
      if constexpr (d + 1 < DIM) fetch_nb(std::integral_constant<int, d + 1>{});
    }
  };
  auto faces = [&](auto dc) {
    constexpr int d = decltype(dc)::value;
    if (tid < EPB * 2 * NF) {
      const int f = tid % NF;
      const int s = (tid / NF) & 1;
      const int le = tid / (2 * NF);
      if (info.e[le] >= 0) {
        const int base = face_base<NP>(d, f);
        const int sd = dstride<NP>(d);
        // on side + the element is the left state: the left trace takes the
        // weights of xi = +1, the right one those of xi = -1
        const R (*eL)[NN] = s ? sW[le] : sNbW[le][s];
        const R (*eR)[NN] = s ? sNbW[le][s] : sW[le];
        R wl[NL], wr[NL];
#pragma unroll
        for (int k = 0; k < NL; ++k) { wl[k] = R(0); wr[k] = R(0); }
#pragma unroll
        for (int l = 0; l < NP; ++l) {
          const R Lp = sLp[l], Lm = sLm[l];
          const int node = base + l * sd;
#pragma unroll
          for (int k = 0; k < NL; ++k) {
            wl[k] += Lp * eL[k][node];
            wr[k] += Lm * eR[k][node];
          }
        }
#pragma unroll
        for (int k = 0; k < NL; ++k) sWs[le][d][s][k][f] = R(0.5) * (wl[k] + wr[k]);
      }
    }
  };
  stage(std::integral_constant<int, 0>{});
  __syncthreads();
  static_for<DIM>([&](auto dc) {  // d-dependent index math is compile-time
    constexpr int d = decltype(dc)::value;
    faces(dc);
    __syncthreads();
    if constexpr (d + 1 < DIM) {
      stage(std::integral_constant<int, d + 1>{});
      __syncthreads();
    }
  });

  if (active) {
    R q[DIM][NL];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int sd = dstride<NP>(d);
      const int i = (n / sd) % NP;
      const int f = face_of<NP>(d, n);
      const R h2 = R(info.h2[el][d]);
#pragma unroll
      for (int k = 0; k < NL; ++k) {
        R vol = R(0);
#pragma unroll
        for (int l = 0; l < NP; ++l) vol += sD[i][l] * sW[el][k][n + (l - i) * sd];
        const R surf = (sLp[i] * sWs[el][d][1][k][f] - sLm[i] * sWs[el][d][0][k][f]) * sIw[i];
        q[d][k] = h2 * (surf - vol);
      }
    }
    R div = R(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) div += q[d][d];
    const long long o = (long long)e * NN + n;
    const R eps = R(ph.eps);
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int b = a; b < DIM; ++b) {
        R t = eps * (q[b][a] + q[a][b]);
        if (a == b) t -= eps * R(2.0 / 3.0) * div;
        G[(long long)tau_index<DIM>(a, b) * S + o] = GT(t);
      }
#pragma unroll
    for (int d = 0; d < DIM; ++d) G[(long long)(Sh::NTAU + d) * S + o] = GT(q[d][DIM]);
  }
}

// -------------------------------------------------------------------------
// Original NSK path, second BR1 lifting (end of Sec. 3.1): with g = grad rho
// from the first lifting (G slots NTAU..NTAU+DIM-1),
//   lap_i = sum_d (2/h_d) [ (L+_i g*_+ - L-_i g*_-) / omega_i - sum_l Dhat_il g_d,l ],
// g* = (g_left + g_right) / 2 the central face values of g_d on the d-faces;
// then the viscous stress in G's tau slots becomes the full second-order
// stress Sigma = eps tau + kappa ((rho lap + |g|^2/2) I - g g^T) (the
// Korteweg stress of Sec. 2.2 in conservative form).  The gradient slots are
// only read, so neighbouring workgroups see the first lifting's values.
// -------------------------------------------------------------------------
template <int DIM, int NP, int EPB>
__device__ __forceinline__ void lap_block(int L, int tid, const double* __restrict__ U, double* __restrict__ G,
                                          const BasisArgs& bas, const MeshArgs& msh, const PhysArgs& ph) {
  using Sh = Shape<DIM, NP>;
  constexpr int NN = Sh::NN, NF = Sh::NF, NT = Sh::NTAU;
  __shared__ double sg[EPB][NN];          // own g_d
  __shared__ double sNb[EPB][2][NN];      // g_d of the two neighbours in direction d
  __shared__ double sgs[EPB][2][NF];      // central face values on the two d-faces
  __shared__ double sD[NP][NP];
  __shared__ double sLm[NP], sLp[NP], sIw[NP];
  __shared__ ElemInfo<DIM, EPB> info;

  const long long S = msh.S;
  if (tid < NP * NP) sD[tid / NP][tid % NP] = bas.Dhat[tid / NP][tid % NP];
  if (tid < NP) { sLm[tid] = bas.Lm[tid]; sLp[tid] = bas.Lp[tid]; sIw[tid] = bas.invw[tid]; }
  elem_info<DIM, EPB>(info, msh, L, tid);
  __syncthreads();

  const int el = tid / NN, n = tid - (tid / NN) * NN;
  const int e = el < EPB ? info.e[el] : -1;
  const bool active = e >= 0;
  const long long o = (long long)(active ? e : 0) * NN + n;

  double g[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) g[d] = active ? G[(long long)(NT + d) * S + o] : 0.0;
  double lap = 0.0;

  static_for<DIM>([&](auto dc) {
    constexpr int d = decltype(dc)::value;
    if (active) {
      sg[el][n] = g[d];
#pragma unroll
      for (int s = 0; s < 2; ++s) sNb[el][s][n] = G[(long long)(NT + d) * S + (long long)info.nb[el][d][s] * NN + n];
    }
    __syncthreads();
    if (tid < EPB * 2 * NF) {
      const int f = tid % NF;
      const int s = (tid / NF) & 1;
      const int le = tid / (2 * NF);
      if (info.e[le] >= 0) {
        const int base = face_base<NP>(d, f);
        const int sd = dstride<NP>(d);
        double own = 0.0, oth = 0.0;
#pragma unroll
        for (int l = 0; l < NP; ++l) {
          const int node = base + l * sd;
          own += (s ? sLp[l] : sLm[l]) * sg[le][node];
          oth += (s ? sLm[l] : sLp[l]) * sNb[le][s][node];
        }
        sgs[le][s][f] = 0.5 * (own + oth);
      }
    }
    __syncthreads();
    if (active) {
      const int sd = dstride<NP>(d);
      const int i = (n / sd) % NP;
      const int f = face_of<NP>(d, n);
      double vol = 0.0;
#pragma unroll
      for (int l = 0; l < NP; ++l) vol += sD[i][l] * sg[el][n + (l - i) * sd];
      const double surf = (sLp[i] * sgs[el][1][f] - sLm[i] * sgs[el][0][f]) * sIw[i];
      lap += info.h2[el][d] * (surf - vol);
    }
    __syncthreads();  // LDS reused by the next direction
  });

  if (active) {
    const double rho = U[o];
    double g2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) g2 += g[d] * g[d];
    const double iso = ph.kappa * (rho * lap + 0.5 * g2);
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int b = a; b < DIM; ++b) {
        const long long ot = (long long)tau_index<DIM>(a, b) * S + o;
        double t = G[ot] - ph.kappa * g[a] * g[b];
        if (a == b) t += iso;
        G[ot] = t;
      }
  }
}

// -------------------------------------------------------------------------
// Right-hand side and fused Runge-Kutta stage:
//   R_i = sum_d (2/h_d) [ sum_l Dhat_il F_d,l - (L+_i F*_+ - L-_i F*_-) / omega_i ] + S_i
// with F_d = Fc_d(U) - Fv_d(G), F* = Rusanov, HLLC or global LF (U-, U+)
// - (Fv(G-) + Fv(G+)) / 2 and S = (0, alpha rho grad c, (alpha/beta)(rho - c))
// (model II); the original NSK path (MODEL 1) has U = (rho, m), the
// second-order stress Sigma in G's tau slots and no source; then
//   dU <- A dU + dt R,  U <- U + B dU.
// -------------------------------------------------------------------------
template <int DIM, int NP, int EPB, typename R, typename GT, int FLUX = 0, int MODEL = 0>
__device__ __forceinline__ void rhs_block(int L, int tid, const double* __restrict__ U, const GT* __restrict__ G,
                                          double* __restrict__ Uout, double* __restrict__ dU, const BasisArgs& bas,
                                          const MeshArgs& msh, const PhysArgs& ph, const StageArgs& st) {
  using Sh = Shape<DIM, NP>;
  constexpr int NN = Sh::NN, NF = Sh::NF, NT = Sh::NTAU;
  constexpr int NV = MODEL == 1 ? DIM + 1 : DIM + 2;   // conserved variables
  constexpr int NG = MODEL == 1 ? NT : Sh::NG;         // G slots read: Sigma, or (tau, grad c)
  constexpr int NVX = MODEL == 1 ? DIM : DIM + 1;      // viscous flux components of one direction
  constexpr int NX = NV + NVX;              // per node: U and the viscous flux components of direction d
  static_assert(MODEL == 0 || FLUX == 2, "the original NSK path uses the global Lax-Friedrichs flux");
  constexpr bool MIXED = sizeof(R) != sizeof(double);
  constexpr int R64E = MIXED ? EPB : 1, R64N = MIXED ? NN : 1;
  __shared__ R sOwn[EPB][NX][NN];           // own U and (tau_{.d}, dc/dx_d)
  __shared__ R sNb[EPB][2][NX][NN];         // the same for the two neighbours in direction d
  __shared__ double sRho64[R64E][3][R64N];  // FP64 densities (mixed precision only)
  // The nodal flux is double-buffered by direction (so that the
  // accumulation of d and the staging of d+1 share a phase) only where the
  // second buffer costs no workgroup per CU, or where at least 5 still fit
  // (measured: the original NSK kernel runs faster pipelined at 5 per CU than
  // with one buffer at 6); otherwise one buffer and one more barrier per
  // direction.
  constexpr int kLdsCu = 163840;
  constexpr int LDS_FIXED = int(sizeof(R)) * (EPB * 3 * NX * NN + EPB * 2 * NV * NF + NP * NP + 3 * NP) +
                            int(sizeof(double)) * R64E * 3 * R64N + int(sizeof(ElemInfo<DIM, EPB>));
  constexpr int LDS_F = int(sizeof(R)) * EPB * NV * NN;
  constexpr bool PIPE = kLdsCu / (LDS_FIXED + 2 * LDS_F) == kLdsCu / (LDS_FIXED + LDS_F) ||
                        kLdsCu / (LDS_FIXED + 2 * LDS_F) >= 5;
  __shared__ R sF[PIPE ? 2 : 1][EPB][NV][NN];  // total flux Fc_d - Fv_d
  __shared__ R sFs[EPB][2][NV][NF];         // numerical flux on the two d-faces
  __shared__ R sD[NP][NP];
  __shared__ R sLm[NP], sLp[NP], sIw[NP];
  __shared__ ElemInfo<DIM, EPB> info;

  const long long S = msh.S;
  if (tid < NP * NP) sD[tid / NP][tid % NP] = R(bas.Dhat[tid / NP][tid % NP]);
  if (tid < NP) { sLm[tid] = R(bas.Lm[tid]); sLp[tid] = R(bas.Lp[tid]); sIw[tid] = R(bas.invw[tid]); }
  elem_info<DIM, EPB>(info, msh, L, tid);
  // elements on FV sub-cells are updated by their own kernel: treat them as absent
  if (st.skip && tid < EPB && info.e[tid] >= 0 && st.skip[info.e[tid]]) info.e[tid] = -1;
  __syncthreads();

  const int el = tid / NN, n = tid - (tid / NN) * NN;
  const int e = el < EPB ? info.e[el] : -1;
  const bool active = e >= 0;
  const long long o = (long long)(active ? e : 0) * NN + n;
  const R kb = R(ph.kb);

  double rho64 = 0.0, c64 = 0.0;
  const R lam_g = FLUX == 2 ? R(*st.lf) : R(0);  // global Lax-Friedrichs speed
  double u64[NV], du_old[NV];
  R u[NV], g[NG];
#pragma unroll
  for (int v = 0; v < NV; ++v) { u64[v] = 0.0; du_old[v] = 0.0; u[v] = R(0); }
#pragma unroll
  for (int k = 0; k < NG; ++k) g[k] = R(0);
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) u64[v] = U[v * S + o];
#pragma unroll
    for (int k = 0; k < NG; ++k) g[k] = R(G[(long long)k * S + o]);
    // FP64: the register is read early (occupancy is held at 2 waves per
    // SIMD by the LDS anyway); mixed precision reads it at the update,
    // which keeps the kernel under 168 VGPRs (3 waves per SIMD)
    if (!MIXED && st.mode == 1 && st.A != 0.0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) du_old[v] = dU[v * S + o];
    }
    rho64 = u64[0];
    if constexpr (MODEL == 0) c64 = u64[DIM + 1];
#pragma unroll
    for (int v = 0; v < NV; ++v) { u[v] = R(u64[v]); sOwn[el][v][n] = u[v]; }
    if (MIXED) sRho64[MIXED ? el : 0][0][MIXED ? n : 0] = rho64;
  }
  R pa = R(0), irho = R(0);
  if (active) {
    pa = p_alpha_guarded<R>(rho64, ph);
    irho = R(1) / u[0];
  }
  R acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = R(0);

  // Neighbour values of one direction (U and the direction's viscous
  // components) in registers.  In FP64 model II the LDS holds the kernel at
  // 2 waves per SIMD whatever its register count, so the next direction's
  // values are fetched while the current one is computed.  The
  // mixed-precision kernel (3 waves per SIMD) and the original NSK path
  // (whose smaller LDS tile allows 5 elements per CU at 3 waves per SIMD,
  // which the prefetch's registers would forbid) fetch them when they stage
  // them; the HLLC face code needs the registers.
  constexpr bool PREFETCH = !MIXED && FLUX != 1 && MODEL == 0;
  double nbv[2][NX];
  auto fetch_nb = [&](auto dc) {
    constexpr int dd = decltype(dc)::value;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const long long on = (long long)info.nb[el][dd][s] * NN + n;
#pragma unroll
      for (int v = 0; v < NV; ++v) nbv[s][v] = U[v * S + on];
#pragma unroll
      for (int j = 0; j < DIM; ++j) nbv[s][NV + j] = double(G[(long long)tau_index<DIM>(j, dd) * S + on]);
      if constexpr (MODEL == 0) nbv[s][NV + DIM] = double(G[(long long)(NT + dd) * S + on]);
    }
  };
  if (PREFETCH && active) fetch_nb(std::integral_constant<int, 0>{});

  // Per direction: stage (own viscous components, nodal flux, neighbours),
  // faces (numerical fluxes), accumulate (volume and surface terms).  The
  // accumulation of direction d and the staging of d+1 share a phase: the
  // nodal flux alternates between two buffers, and everything else staging
  // writes is read only by the face phase before it.
  auto stage = [&](auto dc) {  // d-dependent index math is compile-time
    constexpr int d = decltype(dc)::value;
    if (active) {
      // own viscous components of direction d and the nodal total flux
#pragma unroll
      for (int j = 0; j < DIM; ++j) sOwn[el][NV + j][n] = g[tau_index<DIM>(j, d)];
      if constexpr (MODEL == 0) sOwn[el][NV + DIM][n] = g[NT + d];
      R F[NV];
      conv_flux<DIM, R, NV>(d, u, irho, pa, F);
#pragma unroll
      for (int j = 0; j < DIM; ++j) F[1 + j] -= g[tau_index<DIM>(j, d)];
      if constexpr (MODEL == 0) F[DIM + 1] -= kb * g[NT + d];
#pragma unroll
      for (int v = 0; v < NV; ++v) sF[PIPE ? (d & 1) : 0][el][v][n] = F[v];
      // the two neighbours, coalesced
      if (!PREFETCH) fetch_nb(dc);
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        if (MIXED) sRho64[MIXED ? el : 0][1 + s][MIXED ? n : 0] = nbv[s][0];
#pragma unroll
        for (int x = 0; x < NX; ++x) sNb[el][s][x][n] = R(nbv[s][x]);
      }
      if constexpr (PREFETCH && d + 1 < DIM) fetch_nb(std::integral_constant<int, d + 1>{});
    }
  };
  auto faces = [&](auto dc) {
    constexpr int d = decltype(dc)::value;
    if (tid < EPB * 2 * NF) {
      const int f = tid % NF;
      const int s = (tid / NF) & 1;
      const int le = tid / (2 * NF);
      if (info.e[le] >= 0) {
        const int base = face_base<NP>(d, f);
        const int sd = dstride<NP>(d);
        // left/right in direction d: on side + this element is the left
        // state.  The left trace takes the weights of xi = +1, the right one
        // those of xi = -1, so only the two source elements depend on s.
        const R (*eL)[NN] = s ? sOwn[le] : sNb[le][s];
        const R (*eR)[NN] = s ? sNb[le][s] : sOwn[le];
        const int qL = s ? 0 : 1, qR = s ? 2 : 0;  // FP64 density slots (mixed precision)
        double rL = 0.0, rR = 0.0;  // density traces in FP64 (EoS guard)
        R uL[NV], uR[NV], vL[NVX], vR[NVX];
#pragma unroll
        for (int v = 0; v < NV; ++v) { uL[v] = R(0); uR[v] = R(0); }
#pragma unroll
        for (int k = 0; k < NVX; ++k) { vL[k] = R(0); vR[k] = R(0); }
#pragma unroll
        for (int l = 0; l < NP; ++l) {
          const int node = base + l * sd;
          const R Lp = sLp[l], Lm = sLm[l];
          const double xl = MIXED ? sRho64[MIXED ? le : 0][MIXED ? qL : 0][MIXED ? node : 0] : double(eL[0][node]);
          const double xr = MIXED ? sRho64[MIXED ? le : 0][MIXED ? qR : 0][MIXED ? node : 0] : double(eR[0][node]);
          rL += bas.Lp[l] * xl;
          rR += bas.Lm[l] * xr;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            uL[v] += Lp * eL[v][node];
            uR[v] += Lm * eR[v][node];
          }
#pragma unroll
          for (int k = 0; k < NVX; ++k) {
            vL[k] += Lp * eL[NV + k][node];
            vR[k] += Lm * eR[NV + k][node];
          }
        }
        R paL, paR, aL = R(0), aR = R(0);
        if constexpr (FLUX == 2) {
          // the global Lax-Friedrichs flux needs no local sound speed
          paL = p_alpha_guarded<R>(rL, ph);
          paR = p_alpha_guarded<R>(rR, ph);
        } else {
          p_alpha_sound_guarded<R>(rL, ph, paL, aL);
          p_alpha_sound_guarded<R>(rR, ph, paR, aR);
        }
        const R irL = R(1) / uL[0], irR = R(1) / uR[0];
        R FL[NV], FR[NV], Fc[NV];
        conv_flux<DIM, R, NV>(d, uL, irL, paL, FL);
        conv_flux<DIM, R, NV>(d, uR, irR, paR, FR);
        if constexpr (FLUX == 2) {
          // global Lax-Friedrichs: one dissipation speed for the whole grid
#pragma unroll
          for (int v = 0; v < NV; ++v) Fc[v] = R(0.5) * (FL[v] + FR[v]) - R(0.5) * lam_g * (uR[v] - uL[v]);
        } else if constexpr (FLUX == 0) {
          // Rusanov: central flux minus the larger wave speed times the jump
          const R sL = fabs(uL[1 + d] * irL) + aL;
          const R sR = fabs(uR[1 + d] * irR) + aR;
          const R lam = sL > sR ? sL : sR;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const R diss = (v == NV - 1 && !ph.diss_c) ? R(0) : lam * (uR[v] - uL[v]);
            Fc[v] = R(0.5) * (FL[v] + FR[v]) - R(0.5) * diss;
          }
        } else {
          // HLLC of the barotropic convective part: Davis speeds; HLL flux for
          // mass and normal momentum; tangential momenta carried by the mass
          // flux with the velocity of the upwind side of the contact
          // S* = F_hll[rho] / rho_hll; HLL dissipation alone on c
          const R vnL = uL[1 + d] * irL, vnR = uR[1 + d] * irR;
          const R SL = fmin(vnL - aL, vnR - aR), SR = fmax(vnL + aL, vnR + aR);
          if (SL >= R(0)) {
#pragma unroll
            for (int v = 0; v < NV; ++v) Fc[v] = FL[v];
          } else if (SR <= R(0)) {
#pragma unroll
            for (int v = 0; v < NV; ++v) Fc[v] = FR[v];
          } else {
            const R w = R(1) / (SR - SL);
            const R Fm = (SR * FL[0] - SL * FR[0] + SL * SR * (uR[0] - uL[0])) * w;
            const R rh = (SR * uR[0] - SL * uL[0] - (FR[0] - FL[0])) * w;
            const bool left = Fm / rh >= R(0);
            Fc[0] = Fm;
#pragma unroll
            for (int j = 0; j < DIM; ++j) {
              if (j == d)
                Fc[1 + j] = (SR * FL[1 + j] - SL * FR[1 + j] + SL * SR * (uR[1 + j] - uL[1 + j])) * w;
              else
                Fc[1 + j] = Fm * (left ? uL[1 + j] * irL : uR[1 + j] * irR);
            }
            Fc[NV - 1] = ph.diss_c ? SL * SR * (uR[NV - 1] - uL[NV - 1]) * w : R(0);
          }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          R Fs = Fc[v];
          if (v >= 1 && v <= DIM) Fs -= R(0.5) * (vL[v - 1] + vR[v - 1]);
          if constexpr (MODEL == 0) {
            if (v == NV - 1) Fs -= R(0.5) * kb * (vL[DIM] + vR[DIM]);
          }
          sFs[le][s][v][f] = Fs;
        }
      }
    }
  };
  auto accum = [&](auto dc) {
    constexpr int d = decltype(dc)::value;
    if (active) {
      const int sd = dstride<NP>(d);
      const int i = (n / sd) % NP;
      const int f = face_of<NP>(d, n);
      const R h2 = R(info.h2[el][d]);
      R Drow[NP];
#pragma unroll
      for (int l = 0; l < NP; ++l) Drow[l] = sD[i][l];
      const R lp = sLp[i] * sIw[i], lm = sLm[i] * sIw[i];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        R vol = R(0);
#pragma unroll
        for (int l = 0; l < NP; ++l) vol += Drow[l] * sF[PIPE ? (d & 1) : 0][el][v][n + (l - i) * sd];
        acc[v] += h2 * (vol - (lp * sFs[el][1][v][f] - lm * sFs[el][0][v][f]));
      }
    }
  };
  stage(std::integral_constant<int, 0>{});
  __syncthreads();
  static_for<DIM>([&](auto dc) {
    constexpr int d = decltype(dc)::value;
    faces(dc);
    __syncthreads();
    accum(dc);
    if constexpr (d + 1 < DIM) {
      if constexpr (!PIPE) __syncthreads();  // the single nodal-flux buffer is reused
      stage(std::integral_constant<int, d + 1>{});
      __syncthreads();
    }
  });

  // source (FP64) and update
  if (active) {
    double Rv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Rv[v] = double(acc[v]);
    if constexpr (MODEL == 0) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) Rv[1 + d] += ph.alpha * rho64 * double(g[NT + d]);
      Rv[DIM + 1] += ph.ab * (rho64 - c64);
    }
    if constexpr (MODEL == 0) {
      if (st.closure) {
#pragma unroll
        for (int d = 0; d <= DIM; ++d) Rv[1 + d] += double(st.closure[d * S + o]);
      }
    }
    if (st.mode == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Uout[v * S + o] = Rv[v];
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if (MIXED) du_old[v] = st.A != 0.0 ? dU[v * S + o] : 0.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double du = st.A * du_old[v] + st.dt * Rv[v];
        dU[v * S + o] = du;
        Uout[v * S + o] = u64[v] + st.B * du;
      }
    }
  }
}

// -------------------------------------------------------------------------
// One launch per stage kernel over a single mesh.
// -------------------------------------------------------------------------
template <int DIM, int NP, int EPB, typename R, typename GT>
__global__ void __launch_bounds__((Tile<DIM, NP, EPB>::THREADS))
lift_kernel(const double* __restrict__ U, GT* __restrict__ G, BasisArgs bas, MeshArgs msh, PhysArgs ph) {
  lift_block<DIM, NP, EPB, R, GT>(remap_block(blockIdx.x, gridDim.x, msh.nxcd), threadIdx.x, U, G, bas, msh, ph);
}

// The original NSK path's kernel is held to 3 waves per SIMD (it fits in
// 168 VGPRs without its prefetch); the others keep the compiler's choice.
template <int DIM, int NP, int EPB, typename R, typename GT, int FLUX = 0, int MODEL = 0>
__global__ void __launch_bounds__((Tile<DIM, NP, EPB>::THREADS)) __attribute__((amdgpu_waves_per_eu(MODEL == 1 ? 3 : 2)))
rhs_kernel(const double* __restrict__ U, const GT* __restrict__ G, double* __restrict__ Uout,
           double* __restrict__ dU, BasisArgs bas, MeshArgs msh, PhysArgs ph, StageArgs st) {
  rhs_block<DIM, NP, EPB, R, GT, FLUX, MODEL>(remap_block(blockIdx.x, gridDim.x, msh.nxcd), threadIdx.x, U, G, Uout,
                                              dU, bas, msh, ph, st);
}

// Whole Runge-Kutta steps in one launch, for meshes that one workgroup tile
// holds (grid of one workgroup): each stage's lifting and right-hand side run
// back to back inside the workgroup, a barrier between them (the
// workgroup's own global writes are visible to it after a barrier), the
// state alternating between U0 and U1 from U_cur = (cur ? U1 : U0).  The
// same device code as the stage-by-stage kernels, so the same bits; what
// goes is the launch latency of two kernels per stage.
struct RkCoefs {
  double A[5], B[5];
};

template <int DIM, int NP, int EPB, typename R, typename GT, int FLUX>
__global__ void __launch_bounds__((Tile<DIM, NP, EPB>::THREADS))
steps_kernel(double* U0, double* U1, GT* G, double* dU, BasisArgs bas, MeshArgs msh, PhysArgs ph, RkCoefs rk,
             double dt, int nsteps, int cur) {
  for (int step = 0; step < nsteps; ++step) {
#pragma nounroll
    for (int s = 0; s < 5; ++s) {
      const double* Uin = cur ? U1 : U0;
      double* Uout = cur ? U0 : U1;
      lift_block<DIM, NP, EPB, R, GT>(0, threadIdx.x, Uin, G, bas, msh, ph);
      __syncthreads();
      StageArgs st{rk.A[s], rk.B[s], dt, 1};
      rhs_block<DIM, NP, EPB, R, GT, FLUX, 0>(0, threadIdx.x, Uin, G, Uout, dU, bas, msh, ph, st);
      __syncthreads();
      cur ^= 1;
    }
  }
}

// Original NSK path: the first lifting, which also writes the workgroup's
// maximum of the global Lax-Friedrichs speed to lfpart[logical block] (when
// lfpart is set) ...
template <int DIM, int NP, int EPB>
__global__ void __launch_bounds__((Tile<DIM, NP, EPB>::THREADS))
nsk_lift_kernel(const double* __restrict__ U, double* __restrict__ G, BasisArgs bas, MeshArgs msh, PhysArgs ph,
                double* __restrict__ lfpart) {
  lift_block<DIM, NP, EPB, double, double, 1>(remap_block(blockIdx.x, gridDim.x, msh.nxcd), threadIdx.x, U, G, bas,
                                              msh, ph, lfpart);
}

// ... the second lifting ...
template <int DIM, int NP, int EPB>
__global__ void __launch_bounds__((Tile<DIM, NP, EPB>::THREADS))
lap_kernel(const double* __restrict__ U, double* __restrict__ G, BasisArgs bas, MeshArgs msh, PhysArgs ph) {
  lap_block<DIM, NP, EPB>(remap_block(blockIdx.x, gridDim.x, msh.nxcd), threadIdx.x, U, G, bas, msh, ph);
}

// ... and the maximum of the partial speeds, in two launches: kMaxReduceBlocks
// workgroups each reduce a strided share into out[blockIdx.x], then one
// workgroup reduces those.
constexpr int kMaxReduceThreads = 256;
constexpr int kMaxReduceBlocks = 128;
template <int THREADS>
__global__ void __launch_bounds__(THREADS)
max_reduce_kernel(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double red[THREADS / 64];
  const int tid = threadIdx.x;
  double m = 0.0;
  for (int i = blockIdx.x * THREADS + tid; i < n; i += gridDim.x * THREADS) m = fmax(m, part[i]);
  block_max_store<THREADS>(m, red, out + blockIdx.x, tid);
}

// -------------------------------------------------------------------------
// Persistent kernels over a batch of instances with the same degree.  The
// work list holds (instance, logical block) items; workgroup w takes the
// contiguous item range [w * chunk, (w + 1) * chunk), so that consecutive
// blocks of one instance's tiled work order stay on one XCD.
// -------------------------------------------------------------------------
struct BatchInst {
  const double* U;     // stage input state
  double* Uout;        // stage output state (or R)
  double* dU;          // Runge-Kutta register
  void* G;             // lifted gradients (tau, grad c)
  MeshArgs msh;        // mesh of the instance (nxcd unused)
};

constexpr int kBatchXcds = 8;  // XCDs the batched kernels spread rounds over

struct BatchItem {
  int inst;            // instance index
  int L;               // logical block of that instance
};

// Batched kernels: a group of instances of one degree shares a list of
// (instance, element block) items.  The one-item form gives every item its
// own workgroup; the persistent form runs a fixed grid that takes the list
// in rounds of gridDim.x consecutive items.  In both, each XCD takes a
// contiguous slice of the items in flight, so neighbouring elements meet in
// the same L2.
template <int DIM, int NP, int EPB, typename R, typename GT>
__global__ void __launch_bounds__((Tile<DIM, NP, EPB>::THREADS))
lift_kernel_batch1(const BatchInst* __restrict__ inst, const BatchItem* __restrict__ items, BasisArgs bas,
                   PhysArgs ph) {
  const BatchItem w = items[remap_block(blockIdx.x, gridDim.x, kBatchXcds)];
  const BatchInst& I = inst[w.inst];
  lift_block<DIM, NP, EPB, R, GT>(w.L, threadIdx.x, I.U, reinterpret_cast<GT*>(I.G), bas, I.msh, ph);
}

template <int DIM, int NP, int EPB, typename R, typename GT>
__global__ void __launch_bounds__((Tile<DIM, NP, EPB>::THREADS)) __attribute__((amdgpu_waves_per_eu(2)))
rhs_kernel_batch1(const BatchInst* __restrict__ inst, const BatchItem* __restrict__ items, BasisArgs bas,
                  PhysArgs ph, StageArgs st) {
  const BatchItem w = items[remap_block(blockIdx.x, gridDim.x, kBatchXcds)];
  const BatchInst& I = inst[w.inst];
  rhs_block<DIM, NP, EPB, R, GT>(w.L, threadIdx.x, I.U, reinterpret_cast<const GT*>(I.G), I.Uout, I.dU, bas, I.msh,
                                 ph, st);
}

// The thread index handed to the block functions is made opaque in every
// round: otherwise the compiler hoists the per-thread basis and index work
// out of the loop and holds it in registers across items, which lowers
// occupancy.
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

template <int DIM, int NP, int EPB, typename R, typename GT>
__global__ void __launch_bounds__((Tile<DIM, NP, EPB>::THREADS))
lift_kernel_batch(const BatchInst* __restrict__ inst, const BatchItem* __restrict__ items, int nitems,
                  BasisArgs bas, PhysArgs ph) {
  const int slot = remap_block(blockIdx.x, gridDim.x, kBatchXcds);
  for (int base = 0; base < nitems; base += gridDim.x) {
    const int it = base + slot;
    if (it < nitems) {
      const BatchItem w = items[it];
      const BatchInst& I = inst[w.inst];
      lift_block<DIM, NP, EPB, R, GT>(w.L, opaque_tid(), I.U, reinterpret_cast<GT*>(I.G), bas, I.msh, ph);
    }
    __syncthreads();  // LDS is reused by the next item
  }
}

template <int DIM, int NP, int EPB, typename R, typename GT>
__global__ void __launch_bounds__((Tile<DIM, NP, EPB>::THREADS)) __attribute__((amdgpu_waves_per_eu(2)))
rhs_kernel_batch(const BatchInst* __restrict__ inst, const BatchItem* __restrict__ items, int nitems,
                 BasisArgs bas, PhysArgs ph, StageArgs st) {
  const int slot = remap_block(blockIdx.x, gridDim.x, kBatchXcds);
  for (int base = 0; base < nitems; base += gridDim.x) {
    const int it = base + slot;
    if (it < nitems) {
      const BatchItem w = items[it];
      const BatchInst& I = inst[w.inst];
      rhs_block<DIM, NP, EPB, R, GT>(w.L, opaque_tid(), I.U, reinterpret_cast<const GT*>(I.G), I.Uout, I.dU, bas,
                                     I.msh, ph, st);
    }
    __syncthreads();
  }
}

// -------------------------------------------------------------------------
// Diagnostics: per-block partial sums, then one block reduces in a fixed
// order (deterministic).  Slots: 0..4 conserved integrals, 5 kinetic energy,
// 6 E^alpha, 7 (rho-c)^2, 8 rho min, 9 rho max, 10 max wave speed,
// 11 non-finite count, 12 max_e sum_d max(|v_d|+a)/h_d.
// -------------------------------------------------------------------------
constexpr int kDiagSlots = 13;

__device__ __forceinline__ int elem_index_dir_diag(const MeshArgs& m, long long e, int d) {
  if (d == 0) return int(e % m.nel[0]);
  if (d == 1) return int((e / m.nel[0]) % m.nel[1]);
  return int(e / ((long long)m.nel[0] * m.nel[1]));
}
constexpr int kDiagThreads = 256;

__device__ __forceinline__ double vdw_W(double rho, double T) {
  // W = rho R T ln(rho/(1 - b rho)) - a rho^2 with a = 3, b = 1/3, R = 8/3
  return rho * (8.0 / 3.0) * T * log(3.0 * rho / (3.0 - rho)) - 3.0 * rho * rho;
}

__device__ __forceinline__ double diag_combine(int k, double a, double b) {
  return k == 8 ? fmin(a, b) : ((k == 9 || k == 10 || k == 12) ? fmax(a, b) : a + b);
}

template <int DIM, int NP, typename GT, int MODEL = 0>
__global__ void __launch_bounds__(kDiagThreads)
diag_partial_kernel(const double* __restrict__ U, const GT* __restrict__ G, double* __restrict__ part,
                    const double* __restrict__ wq1, MeshArgs msh, PhysArgs ph) {
  using Sh = Shape<DIM, NP>;
  constexpr int NN = Sh::NN, NT = Sh::NTAU;
  constexpr int NV = MODEL == 1 ? DIM + 1 : DIM + 2;
  constexpr int EPBD = (kDiagThreads / NN) > 0 ? kDiagThreads / NN : 1;  // whole elements per group
  constexpr int SLOTS = EPBD * NN;
  __shared__ double red[kDiagSlots][kDiagThreads];
  __shared__ double spd[DIM][kDiagThreads];  // per-node |v_d| + a
  const int tid = threadIdx.x;
  double acc[kDiagSlots];
  for (int k = 0; k < kDiagSlots; ++k) acc[k] = 0.0;
  acc[8] = INFINITY;
  acc[9] = -INFINITY;
  const long long S = msh.S;
  const int el = tid / NN, n = tid - (tid / NN) * NN;
  int r = n;
  double wn = 1.0;  // tensor-product quadrature weight of the node
#pragma unroll
  for (int d = 0; d < DIM; ++d) { wn *= wq1[r % NP]; r /= NP; }
  // groups of whole elements, one thread per node (coalesced loads); the
  // per-element directional maxima of the wave speed go through LDS
  const long long ngroups = (msh.E + EPBD - 1) / EPBD;
  for (long long grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const long long e = grp * EPBD + el;
    const bool active = tid < SLOTS && e < msh.E;
    double hinv[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) spd[d][tid] = 0.0;
    if (active) {
      const long long o = e * NN + n;
      double J = 1.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double h2 = msh.h2[d][elem_index_dir_diag(msh, e, d)];
        J *= 1.0 / h2;  // h/2
        hinv[d] = 0.5 * h2;
      }
      const double wgt = J * wn;
      double u[NV];
      bool finite = true;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        u[v] = U[v * S + o];
        if (!isfinite(u[v])) { acc[11] += 1.0; finite = false; }
        acc[v] += wgt * u[v];
      }
      // model II: c and its lifted gradient; original NSK: the lifted
      // gradient of rho in the same slots, no relaxation energy
      const double rho = u[0], c = MODEL == 0 ? u[NV - 1] : rho;
      double ek = 0.0, gc2 = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        ek += 0.5 * u[1 + d] * u[1 + d] / rho;
        const double gcd = double(G[(long long)(NT + d) * S + o]);
        gc2 += gcd * gcd;
      }
      acc[5] += wgt * ek;
      acc[6] += wgt * (ek + vdw_W(rho, ph.T) + 0.5 * ph.alpha * (rho - c) * (rho - c) + 0.5 * ph.kappa * gc2);
      acc[7] += wgt * (rho - c) * (rho - c);
      if (finite) {
        acc[8] = fmin(acc[8], rho);
        acc[9] = fmax(acc[9], rho);
        double a;
        if constexpr (MODEL == 1) {
          const double q = 1.0 / (3.0 - rho), dp = 24.0 * ph.T * q * q - 6.0 * rho;
          a = dp > 0.0 ? sqrt(dp) : 0.0;
        } else {
          a = sound_speed<double>(rho, ph.T, ph.alpha);
        }
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const double sp = fabs(u[1 + d] / rho) + a;
          acc[10] = fmax(acc[10], sp);
          spd[d][tid] = sp;
        }
      }
    }
    __syncthreads();
    if (active && n == 0) {
      double lam = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        double m = 0.0;
        for (int k = 0; k < NN; ++k) m = fmax(m, spd[d][el * NN + k]);
        lam += m * hinv[d];
      }
      acc[12] = fmax(acc[12], lam);
    }
    __syncthreads();
  }
  for (int k = 0; k < kDiagSlots; ++k) red[k][tid] = acc[k];
  __syncthreads();
  for (int w = kDiagThreads / 2; w > 0; w >>= 1) {
    if (tid < w)
      for (int k = 0; k < kDiagSlots; ++k) red[k][tid] = diag_combine(k, red[k][tid], red[k][tid + w]);
    __syncthreads();
  }
  if (tid < kDiagSlots) part[(long long)blockIdx.x * kDiagSlots + tid] = red[tid][0];
}

template <int SLOTS>
__global__ void __launch_bounds__(kDiagThreads) diag_final_kernel(const double* __restrict__ part, int nblocks,
                                                                  double* __restrict__ out) {
  __shared__ double red[kDiagSlots][kDiagThreads];
  const int tid = threadIdx.x;
  double acc[kDiagSlots];
  for (int k = 0; k < kDiagSlots; ++k) acc[k] = 0.0;
  acc[8] = INFINITY;
  acc[9] = -INFINITY;
  for (int b = tid; b < nblocks; b += kDiagThreads)
    for (int k = 0; k < kDiagSlots; ++k) acc[k] = diag_combine(k, acc[k], part[(long long)b * kDiagSlots + k]);
  for (int k = 0; k < kDiagSlots; ++k) red[k][tid] = acc[k];
  __syncthreads();
  for (int w = kDiagThreads / 2; w > 0; w >>= 1) {
    if (tid < w)
      for (int k = 0; k < kDiagSlots; ++k) red[k][tid] = diag_combine(k, red[k][tid], red[k][tid + w]);
    __syncthreads();
  }
  if (tid < kDiagSlots) out[tid] = red[tid][0];
}

}  // namespace nsk
