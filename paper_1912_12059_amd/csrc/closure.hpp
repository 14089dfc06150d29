// Device code of the learned closure: a per-node network
//   x (4 features) -> 64 -> 64 -> 64 -> y (2), ReLU on the hidden layers,
// with BF16 parameters and FP32 accumulation, whose outputs add
//   S_m = out_m y_0 n,  S_c = out_c y_1,   n = grad rho / sqrt(|grad rho|^2 + g0^2)
// to the momentum and c equations of relaxation model II.  The paper defines
// no closure; it is trained on nudged pairs of runs at a moderate and a large
// relaxation parameter.
//
// Features are element-local (no lifting): with the collocation derivative D
// of the Gauss-Legendre basis applied along each direction inside an element,
//   g_d = (2/h_d) D rho,   lap = sum_d (2/h_d)^2 D (D rho),
//   x = ((rho - s0) k0, (c - s1) k1, |g| k2, lap k3).
//
// Inference (closure_kernel) on gfx950: a workgroup of 256 threads takes
// whole elements (up to 256 nodes).  Features are formed per node from the
// densities staged in LDS; the network runs per wavefront on 64 nodes with
// the nodes as the MFMA columns: layer 1 (4 -> 64) as FP32 MFMA
// (v_mfma_f32_32x32x2f32), layers 2 and 3 as BF16 MFMA
// (v_mfma_f32_32x32x16_bf16, the full-rate BF16 form of gfx950; the
// accumulator layout of one layer is the B-operand layout of the next), and
// layer 4 as an FP32 dot product finished across the two half-waves.
//
// Training runs in FP32 vector arithmetic with the same rounding points
// (BF16 parameters; BF16 activations where inference feeds a BF16 MFMA), so the
// trained network is the one inference evaluates up to summation order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "dg_kernels.hpp"

namespace nsk {

constexpr int kMlpIn = 4, kMlpHid = 64, kMlpOut = 2;
// parameter blocks, row-major [out][in]
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpHid * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpHid;
constexpr int kOffB2 = kOffW2 + kMlpHid * kMlpHid;
constexpr int kOffW3 = kOffB2 + kMlpHid;
constexpr int kOffB3 = kOffW3 + kMlpHid * kMlpHid;
constexpr int kOffW4 = kOffB3 + kMlpHid;
constexpr int kOffB4 = kOffW4 + kMlpOut * kMlpHid;
constexpr int kMlpParams = kOffB4 + kMlpOut;  // 8770

constexpr int kClosureThreads = 256;
// the small parameter blocks kept in LDS as FP32 by the inference kernels
constexpr int kCW1 = 0, kCB1 = kCW1 + kMlpHid * kMlpIn, kCB2 = kCB1 + kMlpHid, kCB3 = kCB2 + kMlpHid,
              kCW4 = kCB3 + kMlpHid, kCB4 = kCW4 + kMlpOut * kMlpHid, kCSmall = kCB4 + kMlpOut;

struct ClosureArgs {
  const uint16_t* w;       // BF16 parameters
  double D[kMaxNP][kMaxNP];  // collocation derivative D_ij = l_j'(xi_i)
  float s0, k0, s1, k1, k2, k3, g0, out_m, out_c;
};

// ---- BF16 -----------------------------------------------------------------
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

// round to nearest even (the conversion lowers to v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f32_to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__device__ __forceinline__ float bf16_round(float f) { return bf16_to_f32(f32_to_bf16(f)); }

// ---- activation ---------------------------------------------------------------
// ReLU, g(z) = max(z, 0), with derivative 1 for z > 0 and 0 otherwise.  On
// the bit pattern of an IEEE value it is the signed-integer maximum with 0
// (negative values, -0 included, have the sign bit set and become +0): one
// v_max_i32, without the quieting of signalling NaNs that fmaxf adds for
// operands the compiler cannot prove canonical, such as MFMA results.
__device__ __forceinline__ float act_f(float z) { return __int_as_float(max(__float_as_int(z), 0)); }

__device__ __forceinline__ float act_df(float z) { return z > 0.f ? 1.f : 0.f; }

// ---- element-local features ---------------------------------------------------
template <int DIM, int NP>
struct ClosureShape {
  static constexpr int NN = ipow<NP, DIM>::v;
  static constexpr int EPB = (kClosureThreads / NN) > 0 ? kClosureThreads / NN : 1;
  static constexpr int SLOTS = EPB * NN;
  static_assert(SLOTS <= kClosureThreads, "a workgroup takes whole elements, one thread per node");
};

// Element coordinates (x fastest).  A context holds at most 2^30 elements,
// so 32-bit unsigned division suffices: two divisions for all directions.
template <int DIM>
__device__ __forceinline__ void elem_coords(const MeshArgs& m, long long e, int ic[DIM]) {
  const unsigned eu = unsigned(e), n0 = unsigned(m.nel[0]);
  const unsigned q0 = eu / n0;
  ic[0] = int(eu - q0 * n0);
  if constexpr (DIM > 1) {
    const unsigned n1 = unsigned(m.nel[1]);
    const unsigned q1 = q0 / n1;
    ic[1] = int(q0 - q1 * n1);
    if constexpr (DIM > 2) ic[2] = int(q1);
  }
}

// Per node thread t < SLOTS: gradient, unit direction and features of the
// node.  sRho and sDer are LDS scratch of the workgroup; every thread of the
// workgroup must call (it synchronises).
template <int DIM, int NP>
__device__ __forceinline__ void closure_features(int t, long long e, bool active, double rho, double c,
                                                 const MeshArgs& msh, const ClosureArgs& ca,
                                                 double* sRho, double (*sDer)[ClosureShape<DIM, NP>::SLOTS],
                                                 float x[4], double nvec[DIM]) {
  constexpr int NN = ClosureShape<DIM, NP>::NN;
  const int el = t / NN, n = t - (t / NN) * NN;
  if (t < ClosureShape<DIM, NP>::SLOTS) sRho[t] = active ? rho : 0.0;
  __syncthreads();
  double g[DIM], h2[DIM];
  double gg = 0.0;
  int ic[DIM];
  elem_coords<DIM>(msh, active ? e : 0, ic);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    g[d] = 0.0;
    h2[d] = 0.0;
    if (active) {
      const int sd = dstride<NP>(d);
      const int i = (n / sd) % NP;
      const int base = el * NN + n - i * sd;
      h2[d] = msh.h2[d][ic[d]];
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < NP; ++j) s += ca.D[i][j] * sRho[base + j * sd];
      g[d] = h2[d] * s;
      sDer[d][t] = g[d];
      gg += g[d] * g[d];
    }
  }
  __syncthreads();
  double lap = 0.0;
  if (active) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int sd = dstride<NP>(d);
      const int i = (n / sd) % NP;
      const int base = el * NN + n - i * sd;
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < NP; ++l) s += ca.D[i][l] * sDer[d][base + l * sd];
      lap += h2[d] * s;
    }
  }
  // the direction and |g| feed FP32 values only: FP32 square roots (the
  // differences and sums above stay FP64, which keeps small gradients of a
  // near-constant density resolved)
  const float ggf = float(gg);
  const float inv = rsqrtf(fmaf(ca.g0, ca.g0, ggf));
#pragma unroll
  for (int d = 0; d < DIM; ++d) nvec[d] = active ? double(float(g[d]) * inv) : 0.0;
  x[0] = active ? float((rho - double(ca.s0)) * double(ca.k0)) : 0.f;
  x[1] = active ? float((c - double(ca.s1)) * double(ca.k1)) : 0.f;
  x[2] = active ? sqrtf(ggf) * ca.k2 : 0.f;
  x[3] = active ? float(lap * double(ca.k3)) : 0.f;
}

// ---- network on one wavefront: 64 nodes, features from LDS ------------------
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ short bf16_bits(float f) { return short(f32_to_bf16(f)); }

// four FP32 values rounded to BF16 (nearest even), two per v_cvt_pk_bf16_f32
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ bf16x4 bf16_pack4(float a, float b, float c, float d) {
  const bf16x2_t lo = __builtin_convertvector((f32x2_t){a, b}, bf16x2_t);
  const bf16x2_t hi = __builtin_convertvector((f32x2_t){c, d}, bf16x2_t);
  typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
  const u32x2_t w = {__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi)};
  return __builtin_bit_cast(bf16x4, w);
}

// ReLU of four BF16 values (two v_pk_max_i16).  BF16 rounding keeps the
// sign, so this equals rounding the FP32 ReLU.
__device__ __forceinline__ bf16x4 act_bf16x4(bf16x4 v) { return __builtin_elementwise_max(v, (bf16x4){0, 0, 0, 0}); }

// eight BF16 values as the operand of v_mfma_f32_32x32x16_bf16
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ bf16x8 bf16_cat8(bf16x4 lo, bf16x4 hi) {
  typedef short s16x8 __attribute__((ext_vector_type(8)));
  const s16x8 v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_bit_cast(bf16x8, v);
}

// Row of output unit of accumulator register r in lane l of a 32x32 block.
__device__ __forceinline__ int mfma_row(int r, int half) { return (r >> 2) * 8 + half * 4 + (r & 3); }

// sX: features of the workgroup's slots; sW: W2 and W3 as BF16, rows padded
// to kWPad; slot0: first slot of this wave.  Returns y for slot slot0 + lane.
constexpr int kWPad = kMlpHid + 4;

__device__ __forceinline__ void mlp_wave(const float4* sX, const uint16_t* sW, const float* sP, int slot0, float y[2]) {
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5, col = lane & 31;
  y[0] = y[1] = 0.f;
  // one 32-node column block at a time keeps the live accumulators and
  // operands to 2 x 16 + 8 x 2 registers
#pragma nounroll
  for (int jb = 0; jb < 2; ++jb) {
    // the parameters are re-read from LDS in each block rather than held in
    // registers across blocks
    asm volatile("" ::: "memory");
    // layer 1 on the FP32 matrix cores (v_mfma_f32_32x32x2f32, K = 4 inputs
    // in two k-steps of 2: half-wave h supplies inputs h and 2 + h of node
    // col), accumulators starting from the bias.  FP32 operands keep c - rho
    // resolved.  Accumulator rows 8(r/4) + 4 half + r%4 of block ib are the
    // units of k-step 4 ib + r/4 of layer 2's B operand.
    const float4 x = sX[slot0 + jb * 32 + col];
    const float xk0 = half ? x.y : x.x, xk1 = half ? x.w : x.z;
    f32x16 acc[2];
    bf16x4 bop[8];
#pragma unroll
    for (int ib = 0; ib < 2; ++ib) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const float4 b = *reinterpret_cast<const float4*>(sP + kCB1 + ib * 32 + 8 * g + 4 * half);
        acc[ib][4 * g + 0] = b.x;
        acc[ib][4 * g + 1] = b.y;
        acc[ib][4 * g + 2] = b.z;
        acc[ib][4 * g + 3] = b.w;
      }
      const float* w1 = sP + kCW1 + (ib * 32 + col) * kMlpIn + half;
      acc[ib] = __builtin_amdgcn_mfma_f32_32x32x2f32(w1[0], xk0, acc[ib], 0, 0, 0);
      acc[ib] = __builtin_amdgcn_mfma_f32_32x32x2f32(w1[2], xk1, acc[ib], 0, 0, 0);
#pragma unroll
      for (int s = 0; s < 4; ++s)
        bop[4 * ib + s] =
            act_bf16x4(bf16_pack4(acc[ib][4 * s], acc[ib][4 * s + 1], acc[ib][4 * s + 2], acc[ib][4 * s + 3]));
    }
    // layers 2 and 3
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
      const uint16_t* W = sW + layer * kMlpHid * kWPad;
      // the accumulators start from the bias: registers 4g..4g+3 of block ib
      // hold rows ib 32 + 8g + 4 half + (0..3), four consecutive units
      const float* bias = sP + (layer == 0 ? kCB2 : kCB3);
#pragma unroll
      for (int ib = 0; ib < 2; ++ib)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const float4 b = *reinterpret_cast<const float4*>(bias + ib * 32 + 8 * g + 4 * half);
          acc[ib][4 * g + 0] = b.x;
          acc[ib][4 * g + 1] = b.y;
          acc[ib][4 * g + 2] = b.z;
          acc[ib][4 * g + 3] = b.w;
        }
      // k-step S of 16 units pairs the B registers bop[2S], bop[2S+1] (units
      // 16S + 4 half + (0..3) and 16S + 8 + 4 half + (0..3)) with the same
      // units of each weight row
#pragma unroll
      for (int S = 0; S < 4; ++S) {
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) {
          const uint16_t* wr = W + (ib * 32 + col) * kWPad + 16 * S + 4 * half;
          const bf16x8 a = bf16_cat8(*reinterpret_cast<const bf16x4*>(wr), *reinterpret_cast<const bf16x4*>(wr + 8));
          acc[ib] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bf16_cat8(bop[2 * S], bop[2 * S + 1]), acc[ib], 0, 0, 0);
        }
      }
      if (layer == 0) {
        // accumulator rows 8(r/4) + 4 half + r%4 of block ib are exactly the
        // units of k-step 4 ib + r/4 of the next layer's B operand
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
          for (int s = 0; s < 4; ++s)
            bop[4 * ib + s] = act_bf16x4(
                bf16_pack4(acc[ib][4 * s], acc[ib][4 * s + 1], acc[ib][4 * s + 2], acc[ib][4 * s + 3]));
      } else {
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[ib][r] = act_f(acc[ib][r]);
      }
    }
    // layer 4: FP32 dot over this lane's 32 units, then across the half-waves
    float part[2];
#pragma unroll
    for (int o = 0; o < 2; ++o) {
      float sum = 0.f;
#pragma unroll
      for (int ib = 0; ib < 2; ++ib)
#pragma unroll
        for (int r = 0; r < 16; ++r) sum += sP[kCW4 + o * kMlpHid + ib * 32 + mfma_row(r, half)] * acc[ib][r];
      part[o] = sum + __shfl_xor(sum, 32, 64);
    }
    // lane = half * 32 + col takes node slot0 + lane, i.e. column block half
    if (half == jb) {
      y[0] = sP[kCB4 + 0] + part[0];
      y[1] = sP[kCB4 + 1] + part[1];
    }
  }
}

// Stage the parameters the network reads from LDS: W2, W3 as BF16 with
// padded rows, and W1, b1, b2, b3, W4, b4 as FP32 in the compact block.
// W2 and W3 move 8 values (16 bytes) per load; w is 16-byte aligned and both
// blocks start at multiples of 8 values.
__device__ __forceinline__ void mlp_stage_params(const uint16_t* __restrict__ w, uint16_t* sW, float* sP) {
  static_assert(kOffW2 % 8 == 0 && kOffW3 % 8 == 0 && kMlpHid % 8 == 0 && kWPad % 4 == 0, "staging layout");
  constexpr int CH = kMlpHid / 8;  // 16-byte chunks per row
  for (int k = threadIdx.x; k < 2 * kMlpHid * CH; k += blockDim.x) {
    const int l = k / (kMlpHid * CH), r = (k / CH) % kMlpHid, cc = k % CH;
    const uint4 v = *reinterpret_cast<const uint4*>(w + (l ? kOffW3 : kOffW2) + r * kMlpHid + 8 * cc);
    uint2* dst = reinterpret_cast<uint2*>(sW + l * kMlpHid * kWPad + r * kWPad + 8 * cc);
    dst[0] = make_uint2(v.x, v.y);
    dst[1] = make_uint2(v.z, v.w);
  }
  // the compact block is three contiguous runs of the parameter array:
  // W1 b1 | b2 | b3 W4 b4
  static_assert(kCW1 == kOffW1 && kCB1 == kOffB1 && kOffB4 == kOffW4 + kMlpOut * kMlpHid &&
                    kOffW4 == kOffB3 + kMlpHid && kCW4 == kCB3 + kMlpHid,
                "compact block layout");
  for (int k = threadIdx.x; k < kCSmall; k += blockDim.x) {
    const int src = k < kCB2 ? k : (k < kCB3 ? kOffB2 + (k - kCB2) : kOffB3 + (k - kCB3));
    sP[k] = bf16_to_f32(w[src]);
  }
}

// ---- inference kernels -----------------------------------------------------------
// Closure source of every node of the mesh: Sc[d] = out_m y0 n_d (d < DIM),
// Sc[DIM] = out_c y1, FP32, layout [comp][elem][node].
//
// Persistent: a grid of (at most) as many workgroups as fit on the device at
// once, each staging the parameters into LDS once and then taking blocks of
// EPB elements gridDim.x apart.  Every block passes three barriers (two in
// the features, one before the network), so a block's LDS writes cannot
// overtake the previous block's reads: the writes of sRho come after the
// previous block's network, and those of sDer, sX and sN after this block's
// first barrier, which every thread reaches only when done with the
// previous block.
template <int DIM, int NP>
__global__ void __launch_bounds__(kClosureThreads)
closure_kernel(const double* __restrict__ U, float* __restrict__ Sc, MeshArgs msh, ClosureArgs ca) {
  using CS = ClosureShape<DIM, NP>;
  constexpr int NN = CS::NN, SLOTS = CS::SLOTS;
  __shared__ double sRho[SLOTS];
  __shared__ double sDer[DIM][SLOTS];
  __shared__ float4 sX[kClosureThreads];
  __shared__ float sN[DIM][kClosureThreads];
  __shared__ __attribute__((aligned(16))) uint16_t sW[2 * kMlpHid * kWPad];
  __shared__ __attribute__((aligned(16))) float sP[kCSmall];
  mlp_stage_params(ca.w, sW, sP);
  const int t = threadIdx.x;
  const long long S = msh.S;
  const long long nblk = (msh.E + CS::EPB - 1) / CS::EPB;
  for (long long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const long long e = blk * CS::EPB + t / NN;
    const bool active = t < SLOTS && e < msh.E;
    const long long o = active ? e * NN + (t - (t / NN) * NN) : 0;
    const double rho = active ? U[o] : 0.0;
    const double c = active ? U[(DIM + 1) * S + o] : 0.0;
    float x[4];
    double nv[DIM];
    closure_features<DIM, NP>(t, e, active, rho, c, msh, ca, sRho, sDer, x, nv);
    sX[t] = make_float4(x[0], x[1], x[2], x[3]);
#pragma unroll
    for (int d = 0; d < DIM; ++d) sN[d][t] = float(nv[d]);
    __syncthreads();
    // every wave runs the network on its 64 slots (inactive slots compute on
    // zero features and are not written)
    float y[2];
    mlp_wave(sX, sW, sP, (t >> 6) << 6, y);
    if (active) {
      const float sm = ca.out_m * y[0];
#pragma unroll
      for (int d = 0; d < DIM; ++d) Sc[d * S + o] = sm * sN[d][t];
      Sc[DIM * S + o] = ca.out_c * y[1];
    }
  }
}

// Grid of closure_kernel for nblk blocks: the workgroups that fit on the
// current device at once (occupancy query, cached per instantiation; every
// device of the library is a gfx950), at most nblk.
template <int DIM, int NP>
inline unsigned closure_grid(long long nblk) {
  static std::atomic<int> cached{0};
  int per_cu = cached.load(std::memory_order_relaxed);
  if (per_cu <= 0) {
    // a failed query gives one workgroup per CU for this launch (still
    // correct: the blocks are walked in a loop) and is asked again next time
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, closure_kernel<DIM, NP>, kClosureThreads, 0) ==
            hipSuccess &&
        per_cu > 0)
      cached.store(per_cu, std::memory_order_relaxed);
    else
      per_cu = 1;
  }
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                               hipSuccess || cus <= 0)
    cus = 1;
  const long long g = (long long)per_cu * cus;
  return (unsigned)(nblk < g ? nblk : g);
}

// ---- nudging step: training pairs -------------------------------------------------
// U* = (rho_r, m_r, rho_r + cmap (c_r - rho_r)); records X = features(U) and
// Y = ((m* - m).n / tau, (c* - c) / tau); then m, c += (dt/tau)(U* - U).
template <int DIM, int NP>
__global__ void __launch_bounds__(kClosureThreads)
nudge_kernel(double* __restrict__ U, const double* __restrict__ Ur, MeshArgs msh, ClosureArgs ca, double relax,
             double inv_tau, double cmap, float* __restrict__ X, float* __restrict__ Y) {
  using CS = ClosureShape<DIM, NP>;
  constexpr int NN = CS::NN, SLOTS = CS::SLOTS;
  __shared__ double sRho[SLOTS];
  __shared__ double sDer[DIM][SLOTS];
  const int t = threadIdx.x;
  const long long S = msh.S;
  const long long e = (long long)blockIdx.x * CS::EPB + t / NN;
  const bool active = t < SLOTS && e < msh.E;
  const long long o = active ? e * NN + (t - (t / NN) * NN) : 0;
  const double rho = active ? U[o] : 0.0;
  const double c = active ? U[(DIM + 1) * S + o] : 0.0;
  float x[4];
  double nv[DIM];
  closure_features<DIM, NP>(t, e, active, rho, c, msh, ca, sRho, sDer, x, nv);
  if (!active) return;
  const double rr = Ur[o];
  const double cstar = rr + cmap * (Ur[(DIM + 1) * S + o] - rr);
  double dmn = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double m = U[(1 + d) * S + o], dm = Ur[(1 + d) * S + o] - m;
    dmn += dm * nv[d];
    U[(1 + d) * S + o] = m + relax * dm;
  }
  const double dc = cstar - c;
  U[(DIM + 1) * S + o] = c + relax * dc;
  if (X) reinterpret_cast<float4*>(X)[o] = make_float4(x[0], x[1], x[2], x[3]);
  if (Y) {
    Y[2 * o] = float(dmn * inv_tau);
    Y[2 * o + 1] = float(dc * inv_tau);
  }
}

}  // namespace nsk
