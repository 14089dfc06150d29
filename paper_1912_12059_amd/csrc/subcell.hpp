// Finite-volume sub-cell shock capturing for relaxation model II (Sec. 3.2).
//
// Per right-hand side evaluation, on top of the DG kernels:
//   persson_kernel  Persson-Peraire indicator of rho per element (log10 of the
//                   share of the orthonormal-Legendre modal energy in the
//                   modes whose largest one-direction degree is N) against a
//                   threshold -> flags[e];
//   dilate_kernel   need[e]: a troubled element within one element in every
//                   direction (the elements whose sub-cell means the FV
//                   stencils read);
//   means_kernel    sub-cell means Ub = (M x M x M) U of the needed elements,
//                   M[k][j] the mean of l_j over sub-cell k of N+1 equal ones;
//   grad_kernel     the central-difference sub-cell gradients of (v, c) of the
//                   troubled elements (all the FV fluxes and sources use);
//   (the DG right-hand-side kernel skips flagged elements)
//   fv_kernel       troubled elements on (N+1)^dim sub-cells:
//                   MinMod-limited reconstruction of (rho, v, c), Rusanov or
//                   HLLC flux (as the DG faces),
//                   viscous flux from face gradients (means of the two
//                   adjacent central-difference sub-cell gradients); on a face
//                   shared with a DG element, the sub-face means of the DG face
//                   flux polynomial through the Gauss-point fluxes the DG
//                   element uses; the source at the sub-cell means; the nodal
//                   rate (M^-1 x M^-1 x M^-1) of the sub-cell rates, and the
//                   Runge-Kutta stage update.
#pragma once

#include "dg_kernels.hpp"

namespace nsk {

struct SubcellArgs {
  double M[kMaxNP][kMaxNP];     // sub-cell averaging
  double Minv[kMaxNP][kMaxNP];  // its inverse
  double V[kMaxNP][kMaxNP];     // V[k][i] = w_i P_k(xi_i), orthonormal Legendre P_k
  double threshold;
  int* flags;
  int* need;
  double* Ub;                   // sub-cell means, layout of U
  double* Gb;                   // sub-cell gradients of (v, c) of troubled elements, [dd*(dim+1)+j][elem][sub-cell]
};

// element index of e shifted by (sx, sy, sz) with periodic wrap
__device__ __forceinline__ int shifted_elem(const MeshArgs& m, int e, int sx, int sy, int sz) {
  int ix = e % m.nel[0];
  const int r = e / m.nel[0];
  int iy = r % m.nel[1], iz = r / m.nel[1];
  ix = (ix + sx + m.nel[0]) % m.nel[0];
  iy = (iy + sy + m.nel[1]) % m.nel[1];
  iz = (iz + sz + m.nel[2]) % m.nel[2];
  return ix + m.nel[0] * (iy + m.nel[1] * iz);
}

__device__ __forceinline__ int elem_step(const MeshArgs& m, int e, int d, int s) {
  return shifted_elem(m, e, d == 0 ? s : 0, d == 1 ? s : 0, d == 2 ? s : 0);
}

// one sweep of an (NP x NP) matrix along direction d over the node values in
// a (in LDS), result in b: b[..k..] = sum_i A[k][i] a[..i..]
template <int DIM, int NP>
__device__ __forceinline__ void sweep(const double (*A)[kMaxNP], const double* a, double* b, int d, int t) {
  constexpr int NN = ipow<NP, DIM>::v;
  if (t < NN) {
    const int sd = dstride<NP>(d);
    const int k = (t / sd) % NP;
    const int base = t - k * sd;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) s += A[k][i] * a[base + i * sd];
    b[t] = s;
  }
}

constexpr int kSubThreads = 256;

// elements of the indicator kernel per workgroup (one thread per node)
template <int DIM, int NP>
struct PerssonTile {
  static constexpr int NN = ipow<NP, DIM>::v;
  static constexpr int EPG = kSubThreads / NN > 0 ? kSubThreads / NN : 1;
};

template <int DIM, int NP>
__global__ void __launch_bounds__(kSubThreads) persson_kernel(const double* __restrict__ U, SubcellArgs sa,
                                                              MeshArgs msh) {
  constexpr int NN = ipow<NP, DIM>::v, EPG = PerssonTile<DIM, NP>::EPG;
  __shared__ double a[EPG][NN], b[EPG][NN];
  __shared__ double tot_s[EPG][NN], top_s[EPG][NN];
  __shared__ double sV[kMaxNP][kMaxNP];
  const int t = threadIdx.x, le = t / NN, n = t - (t / NN) * NN;
  const int e = blockIdx.x * EPG + le;
  const bool active = le < EPG && e < msh.E;
  if (t < NP * NP) sV[t / NP][t % NP] = sa.V[t / NP][t % NP];
  if (active) a[le][n] = U[(long long)e * NN + n];
  __syncthreads();
  double* src = active ? a[le] : a[0];
  double* dst = active ? b[le] : b[0];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    if (active) sweep<DIM, NP>(sV, src, dst, d, n);
    __syncthreads();
    double* x = src;
    src = dst;
    dst = x;
  }
  if (active) {
    const double c = src[n];
    int r = n, kmax = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int k = r % NP;
      r /= NP;
      kmax = k > kmax ? k : kmax;
    }
    tot_s[le][n] = c * c;
    top_s[le][n] = kmax == NP - 1 ? c * c : 0.0;
  }
  __syncthreads();
  // Modal energy sums in a fixed two-level order: NN / NP threads per
  // element sum the NP modes along the slowest index (each thread reads only
  // its own column, and writes its first entry), then one thread per element
  // sums those partial sums.
  constexpr int NC = NN / NP;
  if (active && n < NC) {
    double T0 = 0.0, T1 = 0.0;
#pragma unroll
    for (int k = 0; k < NP; ++k) { T0 += tot_s[le][n + k * NC]; T1 += top_s[le][n + k * NC]; }
    tot_s[le][n] = T0;
    top_s[le][n] = T1;
  }
  __syncthreads();
  const int et = (int)blockIdx.x * EPG + t;  // element of thread t < EPG
  if (t < EPG && et < msh.E) {
    double T0 = 0.0, T1 = 0.0;
    for (int k = 0; k < NC; ++k) { T0 += tot_s[t][k]; T1 += top_s[t][k]; }
    const double ind = (T1 > 0.0 && T0 > 0.0) ? log10(T1 / T0) : -99.0;
    sa.flags[et] = ind > sa.threshold ? 1 : 0;
  }
}

template <int DIM>
__global__ void __launch_bounds__(kSubThreads) dilate_kernel(SubcellArgs sa, MeshArgs msh) {
  const int e = blockIdx.x * kSubThreads + threadIdx.x;
  if (e >= msh.E) return;
  int any = 0;
  for (int sz = (DIM > 2 ? -1 : 0); sz <= (DIM > 2 ? 1 : 0); ++sz)
    for (int sy = (DIM > 1 ? -1 : 0); sy <= (DIM > 1 ? 1 : 0); ++sy)
      for (int sx = -1; sx <= 1; ++sx) any |= sa.flags[shifted_elem(msh, e, sx, sy, sz)];
  sa.need[e] = any;
}

template <int DIM, int NP>
__global__ void __launch_bounds__(kSubThreads) means_kernel(const double* __restrict__ U, SubcellArgs sa,
                                                            MeshArgs msh) {
  constexpr int NN = ipow<NP, DIM>::v;
  constexpr int NV = DIM + 2;
  __shared__ double a[NV][NN], b[NV][NN];
  __shared__ double sM[kMaxNP][kMaxNP];
  const int e = blockIdx.x, t = threadIdx.x;
  if (!sa.need[e]) return;  // uniform over the workgroup
  // all variables at once: one load latency and DIM + 1 barriers per element
  if (t < NP * NP) sM[t / NP][t % NP] = sa.M[t / NP][t % NP];
  if (t < NN) {
#pragma unroll
    for (int v = 0; v < NV; ++v) a[v][t] = U[(long long)v * msh.S + (long long)e * NN + t];
  }
  __syncthreads();
  double (*src)[NN] = a;
  double (*dst)[NN] = b;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
#pragma unroll
    for (int v = 0; v < NV; ++v) sweep<DIM, NP>(sM, src[v], dst[v], d, t);
    __syncthreads();
    double (*x)[NN] = src;
    src = dst;
    dst = x;
  }
  if (t < NN) {
#pragma unroll
    for (int v = 0; v < NV; ++v) sa.Ub[(long long)v * msh.S + (long long)e * NN + t] = src[v][t];
  }
}

// ---- FV sub-cell operator ---------------------------------------------------
template <int DIM, int NP>
struct Sub {
  static constexpr int NN = ipow<NP, DIM>::v;
  static constexpr int NF = ipow<NP, DIM - 1>::v;
  static constexpr int NV = DIM + 2;
};

// the sub-cell next to (e, k) in direction d on side s: (element, sub-cell)
template <int DIM, int NP>
__device__ __forceinline__ void sub_nb(const MeshArgs& m, int e, int k, int d, int s, int& en, int& kn) {
  const int sd = dstride<NP>(d);
  const int i = (k / sd) % NP;
  int j = i + s;
  en = e;
  if (j < 0) { j = NP - 1; en = elem_step(m, e, d, -1); }
  if (j >= NP) { j = 0; en = elem_step(m, e, d, +1); }
  kn = k + (j - i) * sd;
}

template <int DIM, int NP>
__device__ __forceinline__ void prim_at(const double* Ub, long long S, int e, int k, double* w) {
  constexpr int NN = Sub<DIM, NP>::NN;
  const long long o = (long long)e * NN + k;
  const double rho = Ub[o];
  w[0] = rho;
#pragma unroll
  for (int d = 0; d < DIM; ++d) w[1 + d] = Ub[(1 + d) * S + o] / rho;
  w[DIM + 1] = Ub[(DIM + 1) * S + o];
}

// central-difference gradient of (v, c) at sub-cell (e, k): q[dd][j]
template <int DIM, int NP>
__global__ void __launch_bounds__(kSubThreads) grad_kernel(SubcellArgs sa, MeshArgs msh) {
  // Central-difference gradients of (v, c) on the sub-cells of a troubled
  // element: each sub-cell differences the primitives of its two
  // neighbours along each direction.  The primitives of the element's own
  // sub-cells and of the adjacent sub-cell layer of each neighbour element
  // are formed once in LDS.
  constexpr int NN = Sub<DIM, NP>::NN, NF = NN / NP, NW = DIM + 1;
  __shared__ double sw[NN][NW];            // own sub-cells: (v, c)
  __shared__ double sh[DIM][2][NF][NW];    // the neighbours' layers at the two d-faces
  const int e = blockIdx.x, t = threadIdx.x;
  if (!sa.flags[e]) return;  // uniform over the workgroup
  double w[DIM + 2];
  if (t < NN) {
    prim_at<DIM, NP>(sa.Ub, msh.S, e, t, w);
#pragma unroll
    for (int j = 0; j < NW; ++j) sw[t][j] = w[1 + j];
  }
  for (int i = t; i < DIM * 2 * NF; i += kSubThreads) {
    const int dd = i / (2 * NF), s = (i / NF) & 1, f = i % NF;
    const int en = elem_step(msh, e, dd, s ? +1 : -1);
    // the neighbour's sub-cell next to the face: last position before it, first after it
    const int k = face_base<NP>(dd, f) + (s ? 0 : NP - 1) * dstride<NP>(dd);
    prim_at<DIM, NP>(sa.Ub, msh.S, en, k, w);
#pragma unroll
    for (int j = 0; j < NW; ++j) sh[dd][s][f][j] = w[1 + j];
  }
  __syncthreads();
  if (t >= NN) return;
  const long long o = (long long)e * NN + t;
#pragma unroll
  for (int dd = 0; dd < DIM; ++dd) {
    const int sd = dstride<NP>(dd);
    const int i = (t / sd) % NP;
    const int f = face_of<NP>(dd, t);
    const double* wm = i > 0 ? sw[t - sd] : sh[dd][0][f];
    const double* wp = i < NP - 1 ? sw[t + sd] : sh[dd][1][f];
    // dx = h / NP along dd; h2 = 2/h
    const int ed = dd == 0 ? e % msh.nel[0] : (dd == 1 ? (e / msh.nel[0]) % msh.nel[1] : e / (msh.nel[0] * msh.nel[1]));
    const double inv_dx = 0.5 * msh.h2[dd][ed] * NP;
#pragma unroll
    for (int j = 0; j < NW; ++j) sa.Gb[(long long)(dd * NW + j) * msh.S + o] = (wp[j] - wm[j]) * 0.5 * inv_dx;
  }
}

// the stored sub-cell gradient of a troubled element's sub-cell
template <int DIM, int NP>
__device__ __forceinline__ void load_grad(const double* Gb, long long S, int e, int k, double q[DIM][DIM + 1]) {
  const long long o = (long long)e * Sub<DIM, NP>::NN + k;
#pragma unroll
  for (int dd = 0; dd < DIM; ++dd)
#pragma unroll
    for (int j = 0; j <= DIM; ++j) q[dd][j] = Gb[(long long)(dd * (DIM + 1) + j) * S + o];
}

__device__ __forceinline__ double minmod_d(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) < fabs(b) ? a : b;
}

// Rusanov flux of model II between the point states uL, uR in direction d
// (dissipation on c as diss_c says), as the DG face flux computes it (flux = 0)
template <int DIM>
__device__ __forceinline__ void rusanov(int d, const double* uL, const double* uR, const PhysArgs& ph, double* Fc) {
  constexpr int NV = DIM + 2;
  double paL, paR, aL, aR;
  p_alpha_sound<double>(uL[0], ph.T, ph.alpha, paL, aL);
  p_alpha_sound<double>(uR[0], ph.T, ph.alpha, paR, aR);
  const double irL = 1.0 / uL[0], irR = 1.0 / uR[0];
  double FL[NV], FR[NV];
  conv_flux<DIM, double>(d, uL, irL, paL, FL);
  conv_flux<DIM, double>(d, uR, irR, paR, FR);
  const double sL = fabs(uL[1 + d] * irL) + aL, sR = fabs(uR[1 + d] * irR) + aR;
  const double lam = sL > sR ? sL : sR;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double diss = (v == NV - 1 && !ph.diss_c) ? 0.0 : lam * (uR[v] - uL[v]);
    Fc[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * diss;
  }
}

// HLLC flux of the barotropic model II convective part between uL and uR
// (flux = 1), the formula of the DG right-hand-side kernel: Davis speeds;
// HLL flux for mass and normal momentum; tangential momenta carried by the
// mass flux with the upwind tangential velocity of the contact
// S* = F_hll[rho] / rho_hll; HLL dissipation alone on c (if diss_c)
template <int DIM>
__device__ __forceinline__ void hllc(int d, const double* uL, const double* uR, const PhysArgs& ph, double* Fc) {
  constexpr int NV = DIM + 2;
  double paL, paR, aL, aR;
  p_alpha_sound<double>(uL[0], ph.T, ph.alpha, paL, aL);
  p_alpha_sound<double>(uR[0], ph.T, ph.alpha, paR, aR);
  const double irL = 1.0 / uL[0], irR = 1.0 / uR[0];
  double FL[NV], FR[NV];
  conv_flux<DIM, double>(d, uL, irL, paL, FL);
  conv_flux<DIM, double>(d, uR, irR, paR, FR);
  const double vnL = uL[1 + d] * irL, vnR = uR[1 + d] * irR;
  const double SL = fmin(vnL - aL, vnR - aR), SR = fmax(vnL + aL, vnR + aR);
  if (SL >= 0.0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Fc[v] = FL[v];
  } else if (SR <= 0.0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Fc[v] = FR[v];
  } else {
    const double w = 1.0 / (SR - SL);
    const double Fm = (SR * FL[0] - SL * FR[0] + SL * SR * (uR[0] - uL[0])) * w;
    const double rh = (SR * uR[0] - SL * uL[0] - (FR[0] - FL[0])) * w;
    const bool left = Fm / rh >= 0.0;
    Fc[0] = Fm;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      if (j == d)
        Fc[1 + j] = (SR * FL[1 + j] - SL * FR[1 + j] + SL * SR * (uR[1 + j] - uL[1 + j])) * w;
      else
        Fc[1 + j] = Fm * (left ? uL[1 + j] * irL : uR[1 + j] * irR);
    }
    Fc[NV - 1] = ph.diss_c ? SL * SR * (uR[NV - 1] - uL[NV - 1]) * w : 0.0;
  }
}

// the numerical flux is a compile-time choice, so that a kernel holds only
// the registers of the one it uses
template <int DIM, int FLUX>
__device__ __forceinline__ void conv_numflux(int d, const double* uL, const double* uR, const PhysArgs& ph,
                                             double* F) {
  if constexpr (FLUX == 1)
    hllc<DIM>(d, uL, uR, ph, F);
  else
    rusanov<DIM>(d, uL, uR, ph, F);
}

// FV flux across the face between sub-cell a = (ea, ka) (left) and
// b = (eb, kb) (right) in direction d
template <int DIM, int NP, int FLUX>
__device__ __forceinline__ void fv_face(const double* w0, const double* w1, const double* w2, const double* w3,
                                        const double* Gb, const MeshArgs& m, const PhysArgs& ph, int ea, int ka,
                                        int eb, int kb, int d, double* F) {
  constexpr int NV = DIM + 2;
  double uL[NV], uR[NV];
  {
    double wL[NV], wR[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      wL[v] = w1[v] + 0.5 * minmod_d(w1[v] - w0[v], w2[v] - w1[v]);
      wR[v] = w2[v] - 0.5 * minmod_d(w2[v] - w1[v], w3[v] - w2[v]);
    }
    uL[0] = wL[0];
    uR[0] = wR[0];
#pragma unroll
    for (int j = 0; j < DIM; ++j) { uL[1 + j] = wL[0] * wL[1 + j]; uR[1 + j] = wR[0] * wR[1 + j]; }
    uL[NV - 1] = wL[NV - 1];
    uR[NV - 1] = wR[NV - 1];
  }
  conv_numflux<DIM, FLUX>(d, uL, uR, ph, F);
  double ga[DIM][DIM + 1], gb[DIM][DIM + 1], q[DIM][DIM + 1];
  load_grad<DIM, NP>(Gb, m.S, ea, ka, ga);
  load_grad<DIM, NP>(Gb, m.S, eb, kb, gb);
  double div = 0.0;
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j <= DIM; ++j) q[i][j] = 0.5 * (ga[i][j] + gb[i][j]);
#pragma unroll
  for (int j = 0; j < DIM; ++j) div += q[j][j];
#pragma unroll
  for (int j = 0; j < DIM; ++j) F[1 + j] -= ph.eps * (q[d][j] + q[j][d] - (j == d ? 2.0 / 3.0 * div : 0.0));
  F[NV - 1] -= ph.kb * q[d][DIM];
}

// DG face flux at Gauss point f of the face between eL (left) and eR
// (right) in direction d: Rusanov of the traces minus the mean of the traced
// viscous fluxes, from the same operands as the DG right-hand-side kernel
template <int DIM, int NP, int FLUX>
__device__ __forceinline__ void dg_face(const double* U, const double* G, const BasisArgs& bas, const MeshArgs& m,
                                        const PhysArgs& ph, int eL, int eR, int d, int f, double* F) {
  constexpr int NN = Sub<DIM, NP>::NN, NV = DIM + 2, NT = Shape<DIM, NP>::NTAU;
  const int base = face_base<NP>(d, f), sd = dstride<NP>(d);
  double uL[NV], uR[NV], vL[DIM + 1], vR[DIM + 1];
#pragma unroll
  for (int v = 0; v < NV; ++v) { uL[v] = 0.0; uR[v] = 0.0; }
#pragma unroll
  for (int k = 0; k <= DIM; ++k) { vL[k] = 0.0; vR[k] = 0.0; }
  const long long oL = (long long)eL * NN, oR = (long long)eR * NN;
#pragma unroll
  for (int l = 0; l < NP; ++l) {
    const int node = base + l * sd;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      uL[v] += bas.Lp[l] * U[v * m.S + oL + node];
      uR[v] += bas.Lm[l] * U[v * m.S + oR + node];
    }
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      vL[j] += bas.Lp[l] * G[(long long)tau_index<DIM>(j, d) * m.S + oL + node];
      vR[j] += bas.Lm[l] * G[(long long)tau_index<DIM>(j, d) * m.S + oR + node];
    }
    vL[DIM] += bas.Lp[l] * G[(long long)(NT + d) * m.S + oL + node];
    vR[DIM] += bas.Lm[l] * G[(long long)(NT + d) * m.S + oR + node];
  }
  conv_numflux<DIM, FLUX>(d, uL, uR, ph, F);
#pragma unroll
  for (int j = 0; j < DIM; ++j) F[1 + j] -= 0.5 * (vL[j] + vR[j]);
  F[NV - 1] -= 0.5 * ph.kb * (vL[DIM] + vR[DIM]);
}

template <int DIM, int NP, int FLUX>
__global__ void __launch_bounds__(kSubThreads) fv_kernel(const double* __restrict__ U, const double* __restrict__ G,
                                                         double* __restrict__ Uout, double* __restrict__ dU,
                                                         BasisArgs bas, MeshArgs msh, PhysArgs ph, StageArgs st,
                                                         SubcellArgs sa) {
  using SB = Sub<DIM, NP>;
  constexpr int NN = SB::NN, NF = SB::NF, NV = SB::NV, NT = Shape<DIM, NP>::NTAU;
  __shared__ double rs[NV][NN];                 // sub-cell rates
  __shared__ double Ff[NP + 1][NF][NV];         // face fluxes of one direction, by position along the lines
  __shared__ double Fg[2][NF][NV];              // DG face fluxes at the Gauss points of the two boundary faces
  __shared__ double tb[NV][NN];                 // second buffer of the inverse averaging
  __shared__ double sMinv[kMaxNP][kMaxNP];
  __shared__ double sW[NF][NP + 4][NV];         // primitives along the lines of one direction, two beyond each end
  const int e = blockIdx.x, t = threadIdx.x;
  if (!sa.flags[e]) return;  // uniform over the workgroup
  const double* Ub = sa.Ub;
  for (int i = t; i < NV * NN; i += kSubThreads) rs[i / NN][i % NN] = 0.0;
  if (t < NP * NP) sMinv[t / NP][t % NP] = sa.Minv[t / NP][t % NP];
  __syncthreads();

#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int sd = dstride<NP>(d);
    const int en[2] = {elem_step(msh, e, d, -1), elem_step(msh, e, d, +1)};
    const int trn[2] = {sa.flags[en[0]], sa.flags[en[1]]};
    // DG fluxes at the Gauss points of boundary faces shared with DG elements
    for (int i = t; i < 2 * NF; i += kSubThreads) {
      const int s = i / NF, f = i % NF;
      if (!trn[s]) {
        double F[NV];
        if (s == 0) dg_face<DIM, NP, FLUX>(U, G, bas, msh, ph, en[0], e, d, f, F);
        else dg_face<DIM, NP, FLUX>(U, G, bas, msh, ph, e, en[1], d, f, F);
#pragma unroll
        for (int v = 0; v < NV; ++v) Fg[s][f][v] = F[v];
      }
    }
    // primitives of the sub-cells of every line of direction d, from
    // position -2 (in the element before) to NP + 1 (in the element after):
    // the four cells the MUSCL reconstruction of each face reads
    for (int i = t; i < NF * (NP + 4); i += kSubThreads) {
      const int line = i / (NP + 4), p = i % (NP + 4) - 2;
      const int k0 = face_base<NP>(d, line);
      int ec = e, kc = k0 + p * sd;
      if (p < 0) { ec = en[0]; kc = k0 + (NP + p) * sd; }
      if (p >= NP) { ec = en[1]; kc = k0 + (p - NP) * sd; }
      prim_at<DIM, NP>(Ub, msh.S, ec, kc, sW[line][p + 2]);
    }
    __syncthreads();
    // face fluxes at every position 0..NP of every line of direction d
    for (int i = t; i < (NP + 1) * NF; i += kSubThreads) {
      const int pos = i / NF, line = i % NF;
      const int k0 = face_base<NP>(d, line);  // sub-cell at position 0 of the line
      double F[NV];
      if ((pos == 0 && !trn[0]) || (pos == NP && !trn[1])) {
        // sub-face mean of the DG face-flux polynomial: M along the face directions
        const int s = pos == 0 ? 0 : 1;
#pragma unroll
        for (int v = 0; v < NV; ++v) F[v] = 0.0;
        for (int f = 0; f < NF; ++f) {
          double wgt = 1.0;
          int rl = line, rf = f;
#pragma unroll
          for (int dd = 0; dd < DIM; ++dd) {
            if (dd == d) continue;
            // face index: the directions other than d, in increasing order, x fastest
            wgt *= sa.M[rl % NP][rf % NP];
            rl /= NP;
            rf /= NP;
          }
#pragma unroll
          for (int v = 0; v < NV; ++v) F[v] += wgt * Fg[s][f][v];
        }
      } else {
        int ea, ka, eb, kb;
        if (pos == 0) {
          sub_nb<DIM, NP>(msh, e, k0, d, -1, ea, ka);
          eb = e;
          kb = k0;
        } else {
          ea = e;
          ka = k0 + (pos - 1) * sd;
          sub_nb<DIM, NP>(msh, e, ka, d, +1, eb, kb);
        }
        fv_face<DIM, NP, FLUX>(sW[line][pos], sW[line][pos + 1], sW[line][pos + 2], sW[line][pos + 3], sa.Gb, msh, ph,
                               ea, ka, eb, kb, d, F);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) Ff[pos][line][v] = F[v];
    }
    __syncthreads();
    if (t < NN) {
      const int i = (t / sd) % NP;
      const int line = face_of<NP>(d, t);
      const int ed = d == 0 ? e % msh.nel[0] : (d == 1 ? (e / msh.nel[0]) % msh.nel[1] : e / (msh.nel[0] * msh.nel[1]));
      const double inv_dx = 0.5 * msh.h2[d][ed] * NP;
#pragma unroll
      for (int v = 0; v < NV; ++v) rs[v][t] += (Ff[i][line][v] - Ff[i + 1][line][v]) * inv_dx;
    }
    __syncthreads();
  }
  // source at the sub-cell means
  if (t < NN) {
    const long long o = (long long)e * NN + t;
    double q[DIM][DIM + 1];
    load_grad<DIM, NP>(sa.Gb, msh.S, e, t, q);
    const double rho = Ub[o], c = Ub[(DIM + 1) * msh.S + o];
#pragma unroll
    for (int d = 0; d < DIM; ++d) rs[1 + d][t] += ph.alpha * rho * q[d][DIM];
    rs[NV - 1][t] += ph.ab * (rho - c);
  }
  __syncthreads();
  // nodal rates (the inverse averaging, all variables at once) and the
  // stage update
  double (*src)[NN] = rs;
  double (*dst)[NN] = tb;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
#pragma unroll
    for (int v = 0; v < NV; ++v) sweep<DIM, NP>(sMinv, src[v], dst[v], d, t);
    __syncthreads();
    double (*x)[NN] = src;
    src = dst;
    dst = x;
  }
  if (t < NN) {
#pragma unroll 1
    for (int v = 0; v < NV; ++v) {
      const long long o = (long long)v * msh.S + (long long)e * NN + t;
      const double R = src[v][t];
      if (st.mode == 0) {
        Uout[o] = R;
      } else {
        const double du = (st.A != 0.0 ? st.A * dU[o] : 0.0) + st.dt * R;
        dU[o] = du;
        Uout[o] = U[o] + st.B * du;
      }
    }
  }
  (void)NT;
}

}  // namespace nsk
