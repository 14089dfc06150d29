// libnsk: the learned closure's C ABI (include/nsk.h): setting the network
// of a context, the nudging step that produces training pairs, and the
// training kernels (loss and gradient, Adam, target moments).  Device code of
// the network and the features is in closure.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/nsk.h"
#include "closure.hpp"
#include "dg_kernels.hpp"
#include "host_common.hpp"

namespace nsk {
namespace {

// Network outputs on a list of feature vectors X[n][4] -> Y[n][2] (no output
// scaling).  256 nodes per workgroup.
__global__ void __launch_bounds__(kClosureThreads)
mlp_forward_kernel(const uint16_t* __restrict__ w, const float* __restrict__ X, long long n, float* __restrict__ Y) {
  __shared__ float4 sX[kClosureThreads];
  __shared__ __attribute__((aligned(16))) uint16_t sW[2 * kMlpHid * kWPad];
  __shared__ __attribute__((aligned(16))) float sP[kCSmall];
  mlp_stage_params(w, sW, sP);
  const int t = threadIdx.x;
  const long long s = (long long)blockIdx.x * kClosureThreads + t;
  sX[t] = s < n ? reinterpret_cast<const float4*>(X)[s] : make_float4(0.f, 0.f, 0.f, 0.f);
  __syncthreads();
  float y[2];
  mlp_wave(sX, sW, sP, (t >> 6) << 6, y);
  if (s < n) {
    Y[2 * s] = y[0];
    Y[2 * s + 1] = y[1];
  }
}


// ---- training: loss and gradient --------------------------------------------------
// One workgroup takes 32 samples (optionally gathered through idx) and
// writes its partial gradient (kMlpParams values) and partial loss to
// part[blockIdx.x][0 .. kMlpParams].  Backward treats the BF16 rounding of
// the activations as the identity.
constexpr int kTrainTile = 32;
constexpr int kTrainThreads = 256;

__global__ void __launch_bounds__(kTrainThreads)
mlp_train_kernel(const uint16_t* __restrict__ w, const float* __restrict__ X, const float* __restrict__ Yt,
                 const int* __restrict__ idx, long long n, float inv_n, float tscale0, float tscale1,
                 float* __restrict__ part) {
  constexpr int T = kTrainTile, Hd = kMlpHid;
  __shared__ float sX[T][kMlpIn];
  __shared__ float sZ1[T][Hd], sZ2[T][Hd], sZ3[T][Hd];
  __shared__ float sH1[T][Hd], sH2[T][Hd], sH3[T][Hd];
  __shared__ float sD[T][Hd];
  __shared__ float sDy[T][kMlpOut], sRes[T][kMlpOut];
  const int t = threadIdx.x;
  const long long base = (long long)blockIdx.x * T;
  float* out = part + (long long)blockIdx.x * (kMlpParams + 1);
  auto W = [&](int k) { return bf16_to_f32(w[k]); };
  if (t < T * kMlpIn) {
    const int s = t / kMlpIn, i = t - s * kMlpIn;
    const long long g = base + s;
    const long long src = g < n ? (idx ? (long long)idx[g] : g) : 0;
    sX[s][i] = g < n ? X[src * kMlpIn + i] : 0.f;
  }
  __syncthreads();
  // forward
  for (int p = t; p < T * Hd; p += kTrainThreads) {
    const int s = p / Hd, u = p - s * Hd;
    float z = W(kOffB1 + u);
    for (int i = 0; i < kMlpIn; ++i) z += W(kOffW1 + u * kMlpIn + i) * sX[s][i];
    sZ1[s][u] = z;
    sH1[s][u] = bf16_round(act_f(z));
  }
  __syncthreads();
  for (int p = t; p < T * Hd; p += kTrainThreads) {
    const int s = p / Hd, u = p - s * Hd;
    float z = W(kOffB2 + u);
    for (int k = 0; k < Hd; ++k) z += W(kOffW2 + u * Hd + k) * sH1[s][k];
    sZ2[s][u] = z;
    sH2[s][u] = bf16_round(act_f(z));
  }
  __syncthreads();
  for (int p = t; p < T * Hd; p += kTrainThreads) {
    const int s = p / Hd, u = p - s * Hd;
    float z = W(kOffB3 + u);
    for (int k = 0; k < Hd; ++k) z += W(kOffW3 + u * Hd + k) * sH2[s][k];
    sZ3[s][u] = z;
    sH3[s][u] = act_f(z);
  }
  __syncthreads();
  if (t < T * kMlpOut) {
    const int s = t / kMlpOut, oo = t - s * kMlpOut;
    const long long g = base + s;
    float y = W(kOffB4 + oo);
    for (int k = 0; k < Hd; ++k) y += W(kOffW4 + oo * Hd + k) * sH3[s][k];
    const long long src = g < n ? (idx ? (long long)idx[g] : g) : 0;
    const float r = g < n ? y - (oo == 0 ? tscale0 : tscale1) * Yt[src * kMlpOut + oo] : 0.f;
    sDy[s][oo] = r * inv_n;
    sRes[s][oo] = r;
  }
  __syncthreads();
  // output layer gradients
  for (int k = t; k < kMlpOut * Hd + kMlpOut; k += kTrainThreads) {
    float acc = 0.f;
    if (k < kMlpOut * Hd) {
      const int oo = k / Hd, u = k - oo * Hd;
      for (int s = 0; s < T; ++s) acc += sDy[s][oo] * sH3[s][u];
      out[kOffW4 + k] = acc;
    } else {
      const int oo = k - kMlpOut * Hd;
      for (int s = 0; s < T; ++s) acc += sDy[s][oo];
      out[kOffB4 + oo] = acc;
    }
  }
  // dz3 = (W4^T dy) g'(z3)
  for (int p = t; p < T * Hd; p += kTrainThreads) {
    const int s = p / Hd, u = p - s * Hd;
    float dh = 0.f;
    for (int oo = 0; oo < kMlpOut; ++oo) dh += W(kOffW4 + oo * Hd + u) * sDy[s][oo];
    sD[s][u] = dh * act_df(sZ3[s][u]);
  }
  __syncthreads();
  // gradients of layer 3; dz2 = (W3^T dz3) g'(z2) into sZ3 (no longer needed)
  for (int k = t; k < Hd * Hd + Hd; k += kTrainThreads) {
    float acc = 0.f;
    if (k < Hd * Hd) {
      const int u = k / Hd, j = k - u * Hd;
      for (int s = 0; s < T; ++s) acc += sD[s][u] * sH2[s][j];
      out[kOffW3 + k] = acc;
    } else {
      const int u = k - Hd * Hd;
      for (int s = 0; s < T; ++s) acc += sD[s][u];
      out[kOffB3 + u] = acc;
    }
  }
  for (int p = t; p < T * Hd; p += kTrainThreads) {
    const int s = p / Hd, j = p - s * Hd;
    float dh = 0.f;
    for (int u = 0; u < Hd; ++u) dh += W(kOffW3 + u * Hd + j) * sD[s][u];
    sZ3[s][j] = dh * act_df(sZ2[s][j]);
  }
  __syncthreads();
  // gradients of layer 2; dz1 = (W2^T dz2) g'(z1) into sD
  for (int k = t; k < Hd * Hd + Hd; k += kTrainThreads) {
    float acc = 0.f;
    if (k < Hd * Hd) {
      const int u = k / Hd, j = k - u * Hd;
      for (int s = 0; s < T; ++s) acc += sZ3[s][u] * sH1[s][j];
      out[kOffW2 + k] = acc;
    } else {
      const int u = k - Hd * Hd;
      for (int s = 0; s < T; ++s) acc += sZ3[s][u];
      out[kOffB2 + u] = acc;
    }
  }
  __syncthreads();
  for (int p = t; p < T * Hd; p += kTrainThreads) {
    const int s = p / Hd, j = p - s * Hd;
    float dh = 0.f;
    for (int u = 0; u < Hd; ++u) dh += W(kOffW2 + u * Hd + j) * sZ3[s][u];
    sD[s][j] = dh * act_df(sZ1[s][j]);
  }
  __syncthreads();
  // gradients of layer 1
  for (int k = t; k < Hd * kMlpIn + Hd; k += kTrainThreads) {
    float acc = 0.f;
    if (k < Hd * kMlpIn) {
      const int u = k / kMlpIn, i = k - u * kMlpIn;
      for (int s = 0; s < T; ++s) acc += sD[s][u] * sX[s][i];
      out[kOffW1 + k] = acc;
    } else {
      const int u = k - Hd * kMlpIn;
      for (int s = 0; s < T; ++s) acc += sD[s][u];
      out[kOffB1 + u] = acc;
    }
  }
  if (t == 0) {
    float l = 0.f;
    for (int s = 0; s < T; ++s)
      for (int oo = 0; oo < kMlpOut; ++oo) l += 0.5f * sRes[s][oo] * sRes[s][oo];
    out[kMlpParams] = l * inv_n;
  }
}

// Sum of the partial gradients (and loss) over the training workgroups, in
// a fixed order. A workgroup owns 64 consecutive parameters (one per lane, so
// each partial row is read 256 bytes at a time); each of its waves sums one
// contiguous range of the partials, and the wave sums are added in wave order.
constexpr int kRedCols = 64, kRedWaves = 8;
__global__ void __launch_bounds__(kRedCols * kRedWaves)
mlp_reduce_kernel(const float* __restrict__ part, int nparts, float* __restrict__ grad, float* __restrict__ loss) {
  __shared__ double sp[kRedWaves][kRedCols];
  const int lane = (int)threadIdx.x % kRedCols, wv = (int)threadIdx.x / kRedCols;
  const int k = (int)blockIdx.x * kRedCols + lane;
  const int q = (nparts + kRedWaves - 1) / kRedWaves;
  const int p0 = min(nparts, wv * q), p1 = min(nparts, p0 + q);
  double s = 0.0;
  if (k <= kMlpParams)
    for (int p = p0; p < p1; ++p) s += part[(long long)p * (kMlpParams + 1) + k];
  sp[wv][lane] = s;
  __syncthreads();
  if (wv != 0 || k > kMlpParams) return;
  double t = 0.0;
  for (int w = 0; w < kRedWaves; ++w) t += sp[w][lane];
  if (k < kMlpParams) grad[k] = float(t);
  else if (loss) *loss = float(t);
}

// Adam (Kingma and Ba) on the FP32 master copy; the BF16 parameters the
// network reads are the master values rounded to nearest even.
__global__ void mlp_adam_kernel(float* __restrict__ master, uint16_t* __restrict__ w, float* __restrict__ m,
                                float* __restrict__ v, const float* __restrict__ g, float lr, float b1, float b2,
                                float eps, float c1, float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kMlpParams) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  const float wk = master[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
  master[k] = wk;
  w[k] = f32_to_bf16(wk);
}

// Column means and standard deviations of Y[n][ncol] (ncol <= 4): partial
// sums per workgroup, then a fixed-order final sum.
constexpr int kMomThreads = 256;
__global__ void __launch_bounds__(kMomThreads)
moments_partial_kernel(const float* __restrict__ Y, long long n, int ncol, double* __restrict__ part) {
  __shared__ double s1[kMomThreads][4], s2[kMomThreads][4];
  const int t = threadIdx.x;
  double a[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0};
  for (long long i = (long long)blockIdx.x * kMomThreads + t; i < n; i += (long long)gridDim.x * kMomThreads)
    for (int cc = 0; cc < ncol; ++cc) {
      const double y = Y[i * ncol + cc];
      a[cc] += y;
      b[cc] += y * y;
    }
  for (int cc = 0; cc < 4; ++cc) { s1[t][cc] = a[cc]; s2[t][cc] = b[cc]; }
  __syncthreads();
  for (int h = kMomThreads / 2; h > 0; h >>= 1) {
    if (t < h)
      for (int cc = 0; cc < 4; ++cc) { s1[t][cc] += s1[t + h][cc]; s2[t][cc] += s2[t + h][cc]; }
    __syncthreads();
  }
  if (t == 0)
    for (int cc = 0; cc < 4; ++cc) {
      part[blockIdx.x * 8 + cc] = s1[0][cc];
      part[blockIdx.x * 8 + 4 + cc] = s2[0][cc];
    }
}

__global__ void moments_final_kernel(const double* __restrict__ part, int nparts, long long n, int ncol,
                                     double* __restrict__ out) {
  const int cc = threadIdx.x;
  if (cc >= ncol) return;
  double a = 0.0, b = 0.0;
  for (int p = 0; p < nparts; ++p) { a += part[p * 8 + cc]; b += part[p * 8 + 4 + cc]; }
  const double mean = a / double(n);
  out[cc] = mean;
  out[ncol + cc] = sqrt(fmax(b / double(n) - mean * mean, 0.0));
}


}  // namespace
}  // namespace nsk

using namespace nsk;

namespace {

constexpr int kMomParts = 1024;

ClosureArgs nudge_args(const nsk_ctx* c, const nsk_closure_norm& q) {
  ClosureArgs a;
  std::memset(&a, 0, sizeof(a));
  for (int i = 0; i < c->np; ++i)
    for (int j = 0; j < c->np; ++j) a.D[i][j] = c->basis.D[i][j];
  a.s0 = q.s0; a.k0 = q.k0; a.s1 = q.s1; a.k1 = q.k1; a.k2 = q.k2; a.k3 = q.k3; a.g0 = q.g0;
  a.out_m = q.out_m; a.out_c = q.out_c;
  return a;
}

bool norm_ok(const nsk_closure_norm* q) {
  const float v[9] = {q->s0, q->k0, q->s1, q->k1, q->k2, q->k3, q->g0, q->out_m, q->out_c};
  for (float x : v)
    if (!std::isfinite(x)) return false;
  return q->g0 > 0.f;
}

template <int DIM, int NP>
int launch_nudge_t(nsk_ctx* c, const ClosureArgs& ca, const double* Ur, double relax, double inv_tau, double cmap,
                   float* X, float* Y) {
  using CS = ClosureShape<DIM, NP>;
  const unsigned blocks = (unsigned)((c->E + CS::EPB - 1) / CS::EPB);
  double* U = c->cur == 0 ? c->U : reinterpret_cast<double*>(c->work + c->off_U2);
  hipLaunchKernelGGL((nudge_kernel<DIM, NP>), dim3(blocks), dim3(kClosureThreads), 0, c->stream, U, Ur, mesh_args(c),
                     ca, relax, inv_tau, cmap, X, Y);
  return hipGetLastError() == hipSuccess ? NSK_OK : NSK_EHIP;
}

template <int DIM>
int launch_nudge_np(nsk_ctx* c, const ClosureArgs& ca, const double* Ur, double relax, double inv_tau, double cmap,
                    float* X, float* Y) {
  switch (c->np) {
    case 2: return launch_nudge_t<DIM, 2>(c, ca, Ur, relax, inv_tau, cmap, X, Y);
    case 3: return launch_nudge_t<DIM, 3>(c, ca, Ur, relax, inv_tau, cmap, X, Y);
    case 4: return launch_nudge_t<DIM, 4>(c, ca, Ur, relax, inv_tau, cmap, X, Y);
    case 5: return launch_nudge_t<DIM, 5>(c, ca, Ur, relax, inv_tau, cmap, X, Y);
    case 6: return launch_nudge_t<DIM, 6>(c, ca, Ur, relax, inv_tau, cmap, X, Y);
    case 7:
      if constexpr (DIM < 3) return launch_nudge_t<DIM, 7>(c, ca, Ur, relax, inv_tau, cmap, X, Y);
      break;
  }
  return NSK_EUNSUPPORTED;
}

// number of parameters whose BF16 exponent is all ones (infinite or NaN),
// as a double in *out; one workgroup
constexpr int kParamCheckThreads = 256;
__global__ void __launch_bounds__(kParamCheckThreads)
param_nonfinite_kernel(const uint16_t* __restrict__ w, int n, double* __restrict__ out) {
  __shared__ int red[kParamCheckThreads / 64];
  int cnt = 0;
  for (int i = threadIdx.x; i < n; i += kParamCheckThreads) cnt += (w[i] & 0x7F80u) == 0x7F80u ? 1 : 0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int k = 0; k < kParamCheckThreads / 64; ++k) t += red[k];
    *out = (double)t;
  }
}

bool same_mesh(const nsk_ctx* a, const nsk_ctx* b) {
  if (a->dim != b->dim || a->N != b->N || a->E != b->E || a->nvar != b->nvar) return false;
  for (int d = 0; d < 3; ++d)
    if (a->nel[d] != b->nel[d] || a->h2[d] != b->h2[d]) return false;
  return true;
}

// D2D copy of one context's state into another's, finished before return
// (the two contexts may be bound to different streams)
int copy_state(nsk_ctx* dst, nsk_ctx* src) {
  if (hipStreamSynchronize(src->stream) != hipSuccess) return NSK_EHIP;
  int rc = nsk_set_state(dst, src->U);
  if (rc) return rc;
  return hipStreamSynchronize(dst->stream) == hipSuccess ? NSK_OK : NSK_EHIP;
}

}  // namespace

extern "C" {

int nsk_closure_run(nsk_ctx* cl, nsk_ctx* ref, double dt, int nsteps, int ratio, int check_every,
                    double energy_tol, nsk_closure_report* report) {
  if (!cl || !ref || cl == ref || !report) return NSK_EINVAL;
  if (cl->par.closure != 1 || !cl->cl_w || ref->par.closure != 0) return NSK_EINVAL;
  if (cl->par.model != 0 || ref->par.model != 0 || !same_mesh(cl, ref)) return NSK_EINVAL;
  if (!(dt > 0.0) || !std::isfinite(dt) || nsteps < 0 || ratio < 1 || check_every < 1) return NSK_EINVAL;
  if (!std::isfinite(energy_tol)) return NSK_EINVAL;
  if (!cl->bound || !ref->bound) return NSK_EUNBOUND;
  std::memset(report, 0, sizeof(*report));
  // the parameters, counted on the device
  double* out = reinterpret_cast<double*>(cl->work + cl->off_out) + kDiagSlots;
  hipLaunchKernelGGL(param_nonfinite_kernel, dim3(1), dim3(kParamCheckThreads), 0, cl->stream, cl->cl_w,
                     kMlpParams, out);
  double bad = 0.0;
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&bad, out, sizeof(double), hipMemcpyDeviceToHost, cl->stream) != hipSuccess ||
      hipStreamSynchronize(cl->stream) != hipSuccess)
    return NSK_EHIP;
  nsk_diag d;
  int rc = nsk_diagnostics(cl, &d);
  if (rc) return rc;  // NSK_ENONPHYS: no state to start either run from
  report->e_start = report->e_last = d.e_total;
  rc = copy_state(ref, cl);
  if (rc) return rc;
  long long done = 0;
  int reason = bad > 0.0 ? NSK_CLOSURE_PARAMS : NSK_CLOSURE_KEPT;
  while (reason == NSK_CLOSURE_KEPT && done < nsteps) {
    const int n = (int)std::min<long long>(check_every, nsteps - done);
    rc = nsk_rk_step(cl, dt, n);
    if (rc) return rc;
    rc = nsk_diagnostics(cl, &d);  // waits for cl's stream
    if (rc == NSK_ENONPHYS) {
      reason = NSK_CLOSURE_NONPHYS;
    } else if (rc) {
      return rc;
    } else if (energy_tol >= 0.0 && d.e_total > report->e_start + energy_tol * std::fabs(report->e_start)) {
      reason = NSK_CLOSURE_ENERGY;
    } else {
      done += n;
      report->e_last = d.e_total;
      rc = copy_state(ref, cl);  // the last state that passed
      if (rc) return rc;
    }
  }
  report->closure_steps = done;
  report->reason = reason;
  if (reason == NSK_CLOSURE_KEPT) return NSK_OK;
  // the rest of the time on the large-alpha run, from the last state that passed
  report->fell_back = 1;
  long long left = (nsteps - done) * (long long)ratio;
  report->fallback_steps = left;
  const double dtr = dt / ratio;
  while (left > 0) {
    const int n = (int)std::min<long long>(left, 1 << 30);
    rc = nsk_rk_step(ref, dtr, n);
    if (rc) return rc;
    left -= n;
  }
  rc = nsk_diagnostics(ref, &d);
  if (rc) return rc;
  return copy_state(cl, ref);
}


int nsk_closure_set(nsk_ctx* c, const uint16_t* d_w_bf16, const nsk_closure_norm* norm, int every_stage) {
  if (!c || !d_w_bf16 || !norm || (every_stage != 0 && every_stage != 1)) return NSK_EINVAL;
  if ((reinterpret_cast<uintptr_t>(d_w_bf16) & 15) != 0) return NSK_EINVAL;  // staged 8 values at a time
  if (c->par.closure != 1 || !norm_ok(norm)) return NSK_EINVAL;
  c->cl_every_stage = every_stage;
  const float q[9] = {norm->s0, norm->k0, norm->s1, norm->k1, norm->k2, norm->k3, norm->g0, norm->out_m, norm->out_c};
  std::memcpy(c->cl_norm, q, sizeof(q));
  c->cl_w = d_w_bf16;
  return NSK_OK;
}

int nsk_closure_nudge(nsk_ctx* c, const nsk_closure_norm* norm, const double* d_Uref, double dt, double tau,
                      double cmap, float* d_X, float* d_Y) {
  if (!c || !norm || !d_Uref || !(tau > 0.0) || !(dt >= 0.0) || !std::isfinite(cmap)) return NSK_EINVAL;
  if (!norm_ok(norm)) return NSK_EINVAL;
  if (!c->bound) return NSK_EUNBOUND;
  const ClosureArgs ca = nudge_args(c, *norm);
  switch (c->dim) {
    case 1: return launch_nudge_np<1>(c, ca, d_Uref, dt / tau, 1.0 / tau, cmap, d_X, d_Y);
    case 2: return launch_nudge_np<2>(c, ca, d_Uref, dt / tau, 1.0 / tau, cmap, d_X, d_Y);
    case 3: return launch_nudge_np<3>(c, ca, d_Uref, dt / tau, 1.0 / tau, cmap, d_X, d_Y);
  }
  return NSK_EUNSUPPORTED;
}

int nsk_mlp_forward(const uint16_t* d_w, const float* d_X, long long n, float* d_Y, void* hip_stream) {
  if (!d_w || n < 0 || (n > 0 && (!d_X || !d_Y))) return NSK_EINVAL;
  if (((reinterpret_cast<uintptr_t>(d_X) | reinterpret_cast<uintptr_t>(d_w)) & 15) != 0) return NSK_EINVAL;
  if (n == 0) return NSK_OK;
  const long long blocks = (n + kClosureThreads - 1) / kClosureThreads;
  if (blocks > (1LL << 31) - 1) return NSK_EINVAL;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)blocks), dim3(kClosureThreads), 0,
                     static_cast<hipStream_t>(hip_stream), d_w, d_X, n, d_Y);
  return hipGetLastError() == hipSuccess ? NSK_OK : NSK_EHIP;
}

size_t nsk_mlp_workspace_bytes(long long batch) {
  if (batch < 1) batch = 1;
  const size_t tiles = (size_t)((batch + kTrainTile - 1) / kTrainTile);
  const size_t grad = tiles * (size_t)(kMlpParams + 1) * sizeof(float);
  const size_t mom = (size_t)kMomParts * 8 * sizeof(double);
  return grad > mom ? grad : mom;
}

int nsk_mlp_loss_grad(const uint16_t* d_w, const float* d_X, const float* d_Y, const int* d_idx, long long n,
                      float tscale0, float tscale1, void* d_ws, float* d_grad, float* d_loss, void* hip_stream) {
  if (!d_w || !d_X || !d_Y || !d_ws || !d_grad || n < 1) return NSK_EINVAL;
  if (!std::isfinite(tscale0) || !std::isfinite(tscale1)) return NSK_EINVAL;
  const long long tiles = (n + kTrainTile - 1) / kTrainTile;
  if (tiles > (1LL << 30)) return NSK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  float* part = static_cast<float*>(d_ws);
  hipLaunchKernelGGL(mlp_train_kernel, dim3((unsigned)tiles), dim3(kTrainThreads), 0, s, d_w, d_X, d_Y, d_idx, n,
                     float(1.0 / double(n)), tscale0, tscale1, part);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kMlpParams + 1 + kRedCols - 1) / kRedCols), dim3(kRedCols * kRedWaves), 0,
                     s, part, (int)tiles, d_grad, d_loss);
  return hipGetLastError() == hipSuccess ? NSK_OK : NSK_EHIP;
}

int nsk_mlp_adam(float* d_master, uint16_t* d_w, float* d_m, float* d_v, const float* d_grad, int t, double lr,
                 double beta1, double beta2, double eps, void* hip_stream) {
  if (!d_master || !d_w || !d_m || !d_v || !d_grad || t < 1) return NSK_EINVAL;
  if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
    return NSK_EINVAL;
  const double c1 = 1.0 - std::pow(beta1, t), c2 = 1.0 - std::pow(beta2, t);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0,
                     static_cast<hipStream_t>(hip_stream), d_master, d_w, d_m, d_v, d_grad, float(lr), float(beta1),
                     float(beta2), float(eps), float(c1), float(c2));
  return hipGetLastError() == hipSuccess ? NSK_OK : NSK_EHIP;
}

int nsk_mlp_moments(const float* d_Y, long long n, int ncol, void* d_ws, double* d_out, void* hip_stream) {
  if (!d_Y || n < 1 || ncol < 1 || ncol > 4 || !d_ws || !d_out) return NSK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  long long blocks = (n + kMomThreads - 1) / kMomThreads;
  if (blocks > kMomParts) blocks = kMomParts;
  double* part = static_cast<double*>(d_ws);
  hipLaunchKernelGGL(moments_partial_kernel, dim3((unsigned)blocks), dim3(kMomThreads), 0, s, d_Y, n, ncol, part);
  hipLaunchKernelGGL(moments_final_kernel, dim3(1), dim3(64), 0, s, part, (int)blocks, n, ncol, d_out);
  return hipGetLastError() == hipSuccess ? NSK_OK : NSK_EHIP;
}

}  // extern "C"
