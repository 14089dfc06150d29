// Device kernels of the DGSEM right-hand side for relaxation model II
// (Hitz, Keim, Munz, Rohde, Sec. 2.3 for the model, Sec. 3.1 for the scheme),
// written for gfx950 (64-wide wavefronts, 160 KB LDS per CU, 8 XCDs).
//
// One stage of the explicit scheme is two launches:
//   lift_kernel : state U -> G, where G holds per node the viscous stress
//                 tau (symmetric, dim(dim+1)/2 entries) and grad c, both built
//                 from the BR1-lifted gradients of the primitives (v, c)
//   rhs_kernel  : U, G -> volume integral + Rusanov/BR1 surface integral +
//                 pointwise source, then either R (dU/dt) or the fused
//                 low-storage Runge-Kutta stage update of U and the register.
//
// Work layout: a workgroup owns EPB consecutive elements; one thread per
// (element, node) for nodal work and one thread per (element, direction,
// side, face node) for face work, in a single pass.  The element's own data
// is staged in LDS, so its own face traces come from LDS; the neighbour's
// trace needs the whole Gauss line of the neighbour element (Gauss nodes do
// not contain the element ends), which is read from global memory where the
// neighbour's own workgroup has pulled it into cache.  Workgroups are
// renumbered so that each XCD sweeps one contiguous range of elements (its L2
// then holds the x- and y-neighbours).  Each face value is computed
// identically by both elements that share it, so the scheme stays
// conservative bit for bit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nsk {

constexpr int kMaxNP = 7;  // N <= 6

template <int B, int E>
struct ipow { static constexpr int v = B * ipow<B, E - 1>::v; };
template <int B>
struct ipow<B, 0> { static constexpr int v = 1; };

constexpr int cmax(int a, int b) { return a > b ? a : b; }
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
  static constexpr int NITEMS = EPB * DIM * 2 * Sh::NF;  // face work items
  static constexpr int THREADS = round64(cmax(EPB * Sh::NN, NITEMS));
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
  int nel[3];
  int E;                // number of elements
  long long S;          // E * NN, stride between variables
  int nxcd;             // XCDs to spread contiguous element ranges over
};

struct PhysArgs {
  double T, eps, kappa, alpha, beta;
  double kb;         // kappa / beta
  double ab;         // alpha / beta
  int diss_c;        // Rusanov dissipation on c
  double rho_lo64, rho_hi64;  // mixed precision: FP64 EoS inside this band
};

struct StageArgs {
  double A, B, dt;   // low-storage coefficients of the stage and step size
  int mode;          // 0: write R; 1: Runge-Kutta stage update
};

// -------------------------------------------------------------------------
// Thermodynamics of the reduced Van-der-Waals fluid (Sec. 2.1)
//   p = 8 T rho / (3 - rho) - 3 rho^2,   p' = 24 T / (3 - rho)^2 - 6 rho
// Model II modified pressure p_alpha = p + alpha rho^2 / 2 and sound speed
// a = sqrt(p_alpha') = sqrt(p' + alpha rho) (Sec. 2.3).
// -------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R p_alpha(R rho, R T, R alpha) {
  return R(8) * T * rho / (R(3) - rho) - R(3) * rho * rho + R(0.5) * alpha * rho * rho;
}

template <typename R>
__device__ __forceinline__ R sound_speed(R rho, R T, R alpha) {
  R q = R(3) - rho;
  return sqrt(R(24) * T / (q * q) - R(6) * rho + alpha * rho);
}

// EoS in the working precision R, except inside the spinodal band where the
// Van-der-Waals pressure is evaluated in FP64 (mixed-precision rule).
template <typename R>
__device__ __forceinline__ R p_alpha_guarded(double rho64, const PhysArgs& ph) {
  if (sizeof(R) == sizeof(double) || (rho64 > ph.rho_lo64 && rho64 < ph.rho_hi64))
    return R(p_alpha<double>(rho64, ph.T, ph.alpha));
  return p_alpha<R>(R(rho64), R(ph.T), R(ph.alpha));
}

template <typename R>
__device__ __forceinline__ R sound_guarded(double rho64, const PhysArgs& ph) {
  if (sizeof(R) == sizeof(double) || (rho64 > ph.rho_lo64 && rho64 < ph.rho_hi64))
    return R(sound_speed<double>(rho64, ph.T, ph.alpha));
  return sound_speed<R>(R(rho64), R(ph.T), R(ph.alpha));
}

// Hardware hands consecutive workgroups to the XCDs in turn; renumber them
// so that XCD x works through one contiguous range of tiles.
__device__ __forceinline__ int remap_block(int b, int G, int nx) {
  if (nx <= 1) return b;
  const int q = G / nx, r = G - (G / nx) * nx;
  const int x = b % nx, i = b / nx;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Per-element geometry for the workgroup: neighbour ids and 2/h.
template <int DIM, int EPB>
struct ElemInfo {
  int nb[EPB][DIM][2];
  double h2[EPB][DIM];
};

template <int DIM, int EPB>
__device__ __forceinline__ void elem_info(ElemInfo<DIM, EPB>& info, int e0, const MeshArgs& m, int tid) {
  if (tid < EPB) {
    const int e = e0 + tid;
    if (e < m.E) {
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

// -------------------------------------------------------------------------
// Lifting: G = (tau, grad c) from the BR1 gradients of (v, c).
// -------------------------------------------------------------------------
template <int DIM, int NP, int EPB, typename R, typename GT>
__global__ void __launch_bounds__((Tile<DIM, NP, EPB>::THREADS))
lift_kernel(const double* __restrict__ U, GT* __restrict__ G, BasisArgs bas, MeshArgs msh, PhysArgs ph) {
  using Sh = Shape<DIM, NP>;
  using Tl = Tile<DIM, NP, EPB>;
  constexpr int NN = Sh::NN, NF = Sh::NF, NL = Sh::NLIFT;
  __shared__ R sW[EPB][NL][NN];             // nodal primitives (v, c)
  __shared__ R sWs[EPB][DIM][2][NL][NF];    // central face values w*
  __shared__ R sD[NP][NP];
  __shared__ R sLm[NP], sLp[NP], sIw[NP];
  __shared__ ElemInfo<DIM, EPB> info;

  const int tid = threadIdx.x;
  const int blk = remap_block(blockIdx.x, gridDim.x, msh.nxcd);
  const int e0 = blk * EPB;
  const long long S = msh.S;
  if (tid < NP * NP) sD[tid / NP][tid % NP] = R(bas.Dhat[tid / NP][tid % NP]);
  if (tid < NP) { sLm[tid] = R(bas.Lm[tid]); sLp[tid] = R(bas.Lp[tid]); sIw[tid] = R(bas.invw[tid]); }
  elem_info<DIM, EPB>(info, e0, msh, tid);

  const int el = tid / NN, n = tid - (tid / NN) * NN;
  const int e = e0 + el;
  const bool active = el < EPB && e < msh.E;

  // step 1: nodal primitives
  if (active) {
    const long long o = (long long)e * NN + n;
    const double rho = U[o];
#pragma unroll
    for (int d = 0; d < DIM; ++d) sW[el][d][n] = R(U[(1 + d) * S + o] / rho);
    sW[el][DIM][n] = R(U[(DIM + 1) * S + o]);
  }
  __syncthreads();

  // step 2: central traces w* = (w_left + w_right) / 2 on every face
  if (tid < Tl::NITEMS) {
    const int f = tid % NF;
    const int s = (tid / NF) & 1;
    const int d = (tid / (2 * NF)) % DIM;
    const int le = tid / (2 * NF * DIM);
    if (e0 + le < msh.E) {
      const int nb = info.nb[le][d][s];
      const int base = face_base<NP>(d, f);
      const int sd = dstride<NP>(d);
      R own[NL], oth[NL];
#pragma unroll
      for (int k = 0; k < NL; ++k) { own[k] = R(0); oth[k] = R(0); }
#pragma unroll
      for (int l = 0; l < NP; ++l) {
        const R Lo = s ? sLp[l] : sLm[l];
        const R Ln = s ? sLm[l] : sLp[l];
        const int node = base + l * sd;
        const long long on = (long long)nb * NN + node;
        const double rho = U[on];
#pragma unroll
        for (int k = 0; k < NL; ++k) own[k] += Lo * sW[le][k][node];
#pragma unroll
        for (int k = 0; k < DIM; ++k) oth[k] += Ln * R(U[(1 + k) * S + on] / rho);
        oth[DIM] += Ln * R(U[(DIM + 1) * S + on]);
      }
#pragma unroll
      for (int k = 0; k < NL; ++k) {
        // left state first: on side + the element is left, on side - it is right
        const R wl = s ? own[k] : oth[k];
        const R wr = s ? oth[k] : own[k];
        sWs[le][d][s][k][f] = R(0.5) * (wl + wr);
      }
    }
  }
  __syncthreads();

  // step 3: lifted gradients q[d][k] = d w_k / d x_d, then tau and grad c
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
// Right-hand side and fused Runge-Kutta stage.
// -------------------------------------------------------------------------
// Convective flux of model II in direction d.
template <int DIM, typename R>
__device__ __forceinline__ void conv_flux(int d, const R* u, R pa, R* F) {
  const R vd = u[1 + d] / u[0];
  F[0] = u[1 + d];
#pragma unroll
  for (int j = 0; j < DIM; ++j) F[1 + j] = vd * u[1 + j] + (j == d ? pa : R(0));
  F[DIM + 1] = R(0);
}

template <int DIM, int NP, int EPB, typename R, typename GT>
__global__ void __launch_bounds__((Tile<DIM, NP, EPB>::THREADS))
rhs_kernel(const double* __restrict__ U, const GT* __restrict__ G, double* __restrict__ Uout,
           double* __restrict__ dU, BasisArgs bas, MeshArgs msh, PhysArgs ph, StageArgs st) {
  using Sh = Shape<DIM, NP>;
  using Tl = Tile<DIM, NP, EPB>;
  constexpr int NN = Sh::NN, NF = Sh::NF, NV = Sh::NVAR, NT = Sh::NTAU, NG = Sh::NG;
  constexpr bool MIXED = sizeof(R) != sizeof(double);
  constexpr int R64E = MIXED ? EPB : 1, R64N = MIXED ? NN : 1;
  __shared__ R sUG[EPB][NV + NG][NN];       // own state and G (own face traces)
  __shared__ double sRho64[R64E][R64N];     // FP64 density (mixed precision only)
  __shared__ R sF[EPB][NV][NN];             // total flux Fc - Fv in one direction
  __shared__ R sFs[EPB][DIM][2][NV][NF];    // numerical flux on the faces
  __shared__ R sD[NP][NP];
  __shared__ R sLm[NP], sLp[NP], sIw[NP];
  __shared__ ElemInfo<DIM, EPB> info;

  const int tid = threadIdx.x;
  const int blk = remap_block(blockIdx.x, gridDim.x, msh.nxcd);
  const int e0 = blk * EPB;
  const long long S = msh.S;
  if (tid < NP * NP) sD[tid / NP][tid % NP] = R(bas.Dhat[tid / NP][tid % NP]);
  if (tid < NP) { sLm[tid] = R(bas.Lm[tid]); sLp[tid] = R(bas.Lp[tid]); sIw[tid] = R(bas.invw[tid]); }
  elem_info<DIM, EPB>(info, e0, msh, tid);

  const int el = tid / NN, n = tid - (tid / NN) * NN;
  const int e = e0 + el;
  const bool active = el < EPB && e < msh.E;
  const long long o = (long long)e * NN + n;
  const R kb = R(ph.kb);

  // step 1: own state and G into registers and LDS; prefetch the register dU
  double rho64 = 0.0, c64 = 0.0;
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
    if (st.mode == 1 && st.A != 0.0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) du_old[v] = dU[v * S + o];
    }
    rho64 = u64[0];
    c64 = u64[DIM + 1];
#pragma unroll
    for (int v = 0; v < NV; ++v) { u[v] = R(u64[v]); sUG[el][v][n] = u[v]; }
#pragma unroll
    for (int k = 0; k < NG; ++k) sUG[el][NV + k][n] = g[k];
    if (MIXED) sRho64[MIXED ? el : 0][MIXED ? n : 0] = rho64;
  }
  __syncthreads();

  // step 2: face fluxes F* = Rusanov(uL, uR) - (Fv(gL) + Fv(gR)) / 2, one
  // thread per (element, direction, side, face node); own side from LDS
  if (tid < Tl::NITEMS) {
    const int f = tid % NF;
    const int s = (tid / NF) & 1;
    const int d = (tid / (2 * NF)) % DIM;
    const int le = tid / (2 * NF * DIM);
    if (e0 + le < msh.E) {
      const int nb = info.nb[le][d][s];
      const int base = face_base<NP>(d, f);
      const int sd = dstride<NP>(d);
      double ro64 = 0.0, rn64 = 0.0;   // density traces in FP64 (EoS guard)
      R uo[NV], un[NV], vo[DIM + 1], vn[DIM + 1];
#pragma unroll
      for (int v = 0; v < NV; ++v) { uo[v] = R(0); un[v] = R(0); }
#pragma unroll
      for (int k = 0; k <= DIM; ++k) { vo[k] = R(0); vn[k] = R(0); }
#pragma unroll
      for (int l = 0; l < NP; ++l) {
        const int node = base + l * sd;
        const long long on = (long long)nb * NN + node;
        const R Lo = s ? sLp[l] : sLm[l];   // own trace on side s
        const R Ln = s ? sLm[l] : sLp[l];   // neighbour trace on the opposite side
        const double Lo64 = s ? bas.Lp[l] : bas.Lm[l];
        const double Ln64 = s ? bas.Lm[l] : bas.Lp[l];
        const double rn = U[on];
        const double ro = MIXED ? sRho64[MIXED ? le : 0][MIXED ? node : 0] : double(sUG[le][0][node]);
        ro64 += Lo64 * ro;
        rn64 += Ln64 * rn;
        uo[0] += Lo * sUG[le][0][node];
        un[0] += Ln * R(rn);
#pragma unroll
        for (int v = 1; v < NV; ++v) {
          uo[v] += Lo * sUG[le][v][node];
          un[v] += Ln * R(U[v * S + on]);
        }
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
          const int gi = tau_index<DIM>(j, d);
          vo[j] += Lo * sUG[le][NV + gi][node];
          vn[j] += Ln * R(G[(long long)gi * S + on]);
        }
        vo[DIM] += Lo * sUG[le][NV + NT + d][node];
        vn[DIM] += Ln * R(G[(long long)(NT + d) * S + on]);
      }
      // left/right in direction d: on side + this element is the left state
      R uL[NV], uR[NV], vL[DIM + 1], vR[DIM + 1];
#pragma unroll
      for (int v = 0; v < NV; ++v) { uL[v] = s ? uo[v] : un[v]; uR[v] = s ? un[v] : uo[v]; }
#pragma unroll
      for (int k = 0; k <= DIM; ++k) { vL[k] = s ? vo[k] : vn[k]; vR[k] = s ? vn[k] : vo[k]; }
      const double rL = s ? ro64 : rn64, rR = s ? rn64 : ro64;
      const R paL = p_alpha_guarded<R>(rL, ph), paR = p_alpha_guarded<R>(rR, ph);
      const R aL = sound_guarded<R>(rL, ph), aR = sound_guarded<R>(rR, ph);
      const R sL = fabs(uL[1 + d] / uL[0]) + aL;
      const R sR = fabs(uR[1 + d] / uR[0]) + aR;
      const R lam = sL > sR ? sL : sR;
      R FL[NV], FR[NV];
      conv_flux<DIM, R>(d, uL, paL, FL);
      conv_flux<DIM, R>(d, uR, paR, FR);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const R diss = (v == NV - 1 && !ph.diss_c) ? R(0) : lam * (uR[v] - uL[v]);
        R Fs = R(0.5) * (FL[v] + FR[v]) - R(0.5) * diss;
        if (v >= 1 && v <= DIM) Fs -= R(0.5) * (vL[v - 1] + vR[v - 1]);
        if (v == NV - 1) Fs -= R(0.5) * kb * (vL[DIM] + vR[DIM]);
        sFs[le][d][s][v][f] = Fs;
      }
    }
  }

  // step 3: per direction, stage the nodal flux F_d in LDS and contract
  R acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = R(0);
  R pa = R(0);
  if (active) pa = p_alpha_guarded<R>(rho64, ph);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    if (d > 0) __syncthreads();  // previous direction's contraction is done
    if (active) {
      R F[NV];
      conv_flux<DIM, R>(d, u, pa, F);
#pragma unroll
      for (int j = 0; j < DIM; ++j) F[1 + j] -= g[tau_index<DIM>(j, d)];
      F[DIM + 1] -= kb * g[NT + d];
#pragma unroll
      for (int v = 0; v < NV; ++v) sF[el][v][n] = F[v];
    }
    __syncthreads();
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
        for (int l = 0; l < NP; ++l) vol += Drow[l] * sF[el][v][n + (l - i) * sd];
        acc[v] += h2 * (vol - (lp * sFs[el][d][1][v][f] - lm * sFs[el][d][0][v][f]));
      }
    }
  }

  // step 4: source (FP64) and update
  if (active) {
    double Rv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Rv[v] = double(acc[v]);
#pragma unroll
    for (int d = 0; d < DIM; ++d) Rv[1 + d] += ph.alpha * rho64 * double(g[NT + d]);
    Rv[DIM + 1] += ph.ab * (rho64 - c64);

    if (st.mode == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Uout[v * S + o] = Rv[v];
    } else {
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
// Diagnostics: per-block partial sums, then one block reduces in a fixed
// order (deterministic).  Slots: 0..4 conserved integrals, 5 kinetic energy,
// 6 E^alpha, 7 (rho-c)^2, 8 rho min, 9 rho max, 10 max wave speed,
// 11 non-finite count, 12 max_e sum_d max(|v_d|+a)/h_d.
// -------------------------------------------------------------------------
constexpr int kDiagSlots = 13;
constexpr int kDiagThreads = 256;

__device__ __forceinline__ double vdw_W(double rho, double T) {
  // W = rho R T ln(rho/(1 - b rho)) - a rho^2 with a = 3, b = 1/3, R = 8/3
  return rho * (8.0 / 3.0) * T * log(3.0 * rho / (3.0 - rho)) - 3.0 * rho * rho;
}

__device__ __forceinline__ double diag_combine(int k, double a, double b) {
  return k == 8 ? fmin(a, b) : ((k == 9 || k == 10 || k == 12) ? fmax(a, b) : a + b);
}

template <int DIM, int NP, typename GT>
__global__ void __launch_bounds__(kDiagThreads)
diag_partial_kernel(const double* __restrict__ U, const GT* __restrict__ G, double* __restrict__ part,
                    const double* __restrict__ wq1, MeshArgs msh, PhysArgs ph) {
  using Sh = Shape<DIM, NP>;
  constexpr int NN = Sh::NN, NV = Sh::NVAR, NT = Sh::NTAU;
  __shared__ double red[kDiagSlots][kDiagThreads];
  const int tid = threadIdx.x;
  double acc[kDiagSlots];
  for (int k = 0; k < kDiagSlots; ++k) acc[k] = 0.0;
  acc[8] = INFINITY;
  acc[9] = -INFINITY;
  const long long S = msh.S;
  // each thread walks whole elements so that the per-element wave-speed sum
  // can be formed locally
  for (int e = blockIdx.x * kDiagThreads + tid; e < msh.E; e += gridDim.x * kDiagThreads) {
    int idx[3];
    idx[0] = e % msh.nel[0];
    idx[1] = (e / msh.nel[0]) % msh.nel[1];
    idx[2] = e / (msh.nel[0] * msh.nel[1]);
    double J = 1.0, hinv[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double h2 = msh.h2[d][idx[d]];
      J *= 1.0 / h2;  // h/2
      hinv[d] = 0.5 * h2;
    }
    double smax[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) smax[d] = 0.0;
    for (int n = 0; n < NN; ++n) {
      const long long o = (long long)e * NN + n;
      double wgt = J;
      int r = n;
#pragma unroll
      for (int d = 0; d < DIM; ++d) { wgt *= wq1[r % NP]; r /= NP; }
      double u[NV];
      bool finite = true;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        u[v] = U[v * S + o];
        if (!isfinite(u[v])) { acc[11] += 1.0; finite = false; }
        acc[v] += wgt * u[v];
      }
      const double rho = u[0], c = u[DIM + 1];
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
        const double a = sound_speed<double>(rho, ph.T, ph.alpha);
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const double sp = fabs(u[1 + d] / rho) + a;
          acc[10] = fmax(acc[10], sp);
          smax[d] = fmax(smax[d], sp);
        }
      }
    }
    double lam = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) lam += smax[d] * hinv[d];
    acc[12] = fmax(acc[12], lam);
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
