// libnsk host side: the C ABI declared in include/nsk.h.
//
// Builds the 1D Gauss-Legendre basis and the geometry on the host, lays out
// the caller-provided workspace, builds the element work order, and enqueues
// the kernels of dg_kernels.hpp on the bound stream.  No device memory is
// allocated here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/nsk.h"
#include "closure.hpp"
#include "dg_kernels.hpp"
#include "host_common.hpp"
#include "subcell.hpp"

using namespace nsk;

namespace {

// ---------------------------------------------------------------------------
// Launch dispatch over (dim, N, precision, elements per workgroup)
// ---------------------------------------------------------------------------
// events of the next timed stage, or nullptr when timing is off or full
hipEvent_t* stage_events(nsk_ctx* c, const StageArgs& st) {
  if (st.mode != 1 || c->events.empty() || 4 * (size_t)(c->timed + 1) > c->events.size()) return nullptr;
  return &c->events[4 * (size_t)c->timed++];
}

ClosureArgs closure_args_of(const nsk_ctx* c) {
  ClosureArgs a;
  std::memset(&a, 0, sizeof(a));
  a.w = c->cl_w;
  for (int i = 0; i < c->np; ++i)
    for (int j = 0; j < c->np; ++j) a.D[i][j] = c->basis.D[i][j];
  const float* q = c->cl_norm;
  a.s0 = q[0]; a.k0 = q[1]; a.s1 = q[2]; a.k1 = q[3]; a.k2 = q[4]; a.k3 = q[5]; a.g0 = q[6];
  a.out_m = q[7]; a.out_c = q[8];
  return a;
}

// Original NSK path: first lifting (with the per-workgroup maxima of the
// global Lax-Friedrichs speed), their reduction, the second lifting, then the
// right-hand side with the global Lax-Friedrichs flux.
template <int DIM, int NP, int EPB>
int launch_stage_nsk(nsk_ctx* c, const double* Uin, double* Uout, double* dU, const StageArgs& st) {
  using Tl = Tile<DIM, NP, EPB>;
  const BasisArgs b = basis_args(c);
  const MeshArgs m = mesh_args(c);
  const PhysArgs p = phys_args(c);
  double* G = reinterpret_cast<double*>(c->work + c->off_G);
  // lf[0]: the speed; lf[1..kMaxReduceBlocks]: second-level maxima; then one
  // partial maximum per lifting workgroup
  double* lf = reinterpret_cast<double*>(c->work + c->off_lf);
  double* lf2 = lf + 1;
  double* lfpart = lf + 1 + kMaxReduceBlocks;
  const unsigned blocks = (unsigned)((c->E + EPB - 1) / EPB);
  hipEvent_t* ev = stage_events(c, st);
  if (ev) (void)hipEventRecord(ev[0], c->stream);
  hipLaunchKernelGGL((nsk_lift_kernel<DIM, NP, EPB>), dim3(blocks), dim3(Tl::THREADS), 0, c->stream, Uin, G, b, m, p,
                     lfpart);
  if (ev) (void)hipEventRecord(ev[1], c->stream);
  hipLaunchKernelGGL(max_reduce_kernel<kMaxReduceThreads>, dim3(kMaxReduceBlocks), dim3(kMaxReduceThreads), 0,
                     c->stream, lfpart, (int)blocks, lf2);
  hipLaunchKernelGGL(max_reduce_kernel<kMaxReduceThreads>, dim3(1), dim3(kMaxReduceThreads), 0, c->stream, lf2,
                     kMaxReduceBlocks, lf);
  hipLaunchKernelGGL((lap_kernel<DIM, NP, EPB>), dim3(blocks), dim3(Tl::THREADS), 0, c->stream, Uin, G, b, m, p);
  if (ev) (void)hipEventRecord(ev[2], c->stream);
  StageArgs sta = st;
  sta.lf = lf;
  hipLaunchKernelGGL((rhs_kernel<DIM, NP, EPB, double, double, 2, 1>), dim3(blocks), dim3(Tl::THREADS), 0, c->stream,
                     Uin, G, Uout, dU, b, m, p, sta);
  if (ev) (void)hipEventRecord(ev[3], c->stream);
  return hipGetLastError() == hipSuccess ? NSK_OK : NSK_EHIP;
}

SubcellArgs subcell_args(const nsk_ctx* c) {
  SubcellArgs a;
  std::memset(&a, 0, sizeof(a));
  std::memcpy(a.M, c->sc_M, sizeof(a.M));
  std::memcpy(a.Minv, c->sc_Minv, sizeof(a.Minv));
  std::memcpy(a.V, c->sc_V, sizeof(a.V));
  a.threshold = c->par.subcell_threshold;
  a.flags = reinterpret_cast<int*>(c->work + c->off_sc_flags);
  a.need = reinterpret_cast<int*>(c->work + c->off_sc_need);
  a.Ub = reinterpret_cast<double*>(c->work + c->off_sc_Ub);
  a.Gb = reinterpret_cast<double*>(c->work + c->off_sc_Gb);
  return a;
}

// Model II with FV sub-cells: indicator, the elements needing sub-cell means,
// the means, the lifting, the DG right-hand side of the untroubled
// elements, then the FV sub-cell update of the troubled ones.
template <int DIM, int NP, int EPB>
int launch_stage_subcell(nsk_ctx* c, const double* Uin, double* Uout, double* dU, const StageArgs& st) {
  using Tl = Tile<DIM, NP, EPB>;
  const BasisArgs b = basis_args(c);
  const MeshArgs m = mesh_args(c);
  const PhysArgs p = phys_args(c);
  const SubcellArgs sa = subcell_args(c);
  double* G = reinterpret_cast<double*>(c->work + c->off_G);
  const unsigned blocks = (unsigned)((c->E + EPB - 1) / EPB);
  const unsigned E = (unsigned)c->E;
  hipEvent_t* ev = stage_events(c, st);
  if (ev) (void)hipEventRecord(ev[0], c->stream);
  hipLaunchKernelGGL((lift_kernel<DIM, NP, EPB, double, double>), dim3(blocks), dim3(Tl::THREADS), 0, c->stream, Uin,
                     G, b, m, p);
  if (ev) (void)hipEventRecord(ev[1], c->stream);
  constexpr int EPG = PerssonTile<DIM, NP>::EPG;
  hipLaunchKernelGGL((persson_kernel<DIM, NP>), dim3((E + EPG - 1) / EPG), dim3(kSubThreads), 0, c->stream, Uin, sa,
                     m);
  hipLaunchKernelGGL((dilate_kernel<DIM>), dim3((E + kSubThreads - 1) / kSubThreads), dim3(kSubThreads), 0,
                     c->stream, sa, m);
  hipLaunchKernelGGL((means_kernel<DIM, NP>), dim3(E), dim3(kSubThreads), 0, c->stream, Uin, sa, m);
  hipLaunchKernelGGL((grad_kernel<DIM, NP>), dim3(E), dim3(kSubThreads), 0, c->stream, sa, m);
  if (ev) (void)hipEventRecord(ev[2], c->stream);
  StageArgs sta = st;
  sta.skip = sa.flags;
  if (c->par.flux == 1) {
    hipLaunchKernelGGL((rhs_kernel<DIM, NP, EPB, double, double, 1>), dim3(blocks), dim3(Tl::THREADS), 0, c->stream,
                       Uin, G, Uout, dU, b, m, p, sta);
    hipLaunchKernelGGL((fv_kernel<DIM, NP, 1>), dim3(E), dim3(kSubThreads), 0, c->stream, Uin, G, Uout, dU, b, m, p,
                       sta, sa);
  } else {
    hipLaunchKernelGGL((rhs_kernel<DIM, NP, EPB, double, double, 0>), dim3(blocks), dim3(Tl::THREADS), 0, c->stream,
                       Uin, G, Uout, dU, b, m, p, sta);
    hipLaunchKernelGGL((fv_kernel<DIM, NP, 0>), dim3(E), dim3(kSubThreads), 0, c->stream, Uin, G, Uout, dU, b, m, p,
                       sta, sa);
  }
  if (ev) (void)hipEventRecord(ev[3], c->stream);
  return hipGetLastError() == hipSuccess ? NSK_OK : NSK_EHIP;
}

template <int DIM, int NP, int EPB, typename R, typename GT>
int launch_stage_e(nsk_ctx* c, const double* Uin, double* Uout, double* dU, const StageArgs& st) {
  if constexpr (std::is_same<R, double>::value) {
    if (c->par.model == 1) return launch_stage_nsk<DIM, NP, EPB>(c, Uin, Uout, dU, st);
    if (c->par.subcell == 1) return launch_stage_subcell<DIM, NP, EPB>(c, Uin, Uout, dU, st);
  }
  using Tl = Tile<DIM, NP, EPB>;
  const BasisArgs b = basis_args(c);
  const MeshArgs m = mesh_args(c);
  const PhysArgs p = phys_args(c);
  GT* G = reinterpret_cast<GT*>(c->work + c->off_G);
  const unsigned blocks = (unsigned)((c->E + EPB - 1) / EPB);
  hipEvent_t* ev = stage_events(c, st);
  if (ev) (void)hipEventRecord(ev[0], c->stream);
  hipLaunchKernelGGL((lift_kernel<DIM, NP, EPB, R, GT>), dim3(blocks), dim3(Tl::THREADS), 0, c->stream, Uin, G, b, m,
                     p);
  if (ev) (void)hipEventRecord(ev[1], c->stream);
  StageArgs sta = st;
  if (c->par.closure == 1) {
    // the source of the step's first stage is reused in the later stages
    // when the context evaluates the closure once per step
    const bool fresh = c->cl_every_stage || c->cl_stage <= 0;
    using CS = ClosureShape<DIM, NP>;
    float* Sc = reinterpret_cast<float*>(c->work + c->off_cl);
    if (fresh)
      hipLaunchKernelGGL((closure_kernel<DIM, NP>), dim3(closure_grid<DIM, NP>((c->E + CS::EPB - 1) / CS::EPB)),
                         dim3(kClosureThreads), 0, c->stream, Uin, Sc, mesh_args(c), closure_args_of(c));
    sta.closure = Sc;
  }
  if (ev) (void)hipEventRecord(ev[2], c->stream);
  if (c->par.flux == 1)
    hipLaunchKernelGGL((rhs_kernel<DIM, NP, EPB, R, GT, 1>), dim3(blocks), dim3(Tl::THREADS), 0, c->stream, Uin, G,
                       Uout, dU, b, m, p, sta);
  else
    hipLaunchKernelGGL((rhs_kernel<DIM, NP, EPB, R, GT, 0>), dim3(blocks), dim3(Tl::THREADS), 0, c->stream, Uin, G,
                       Uout, dU, b, m, p, sta);
  if (ev) (void)hipEventRecord(ev[3], c->stream);
  return hipGetLastError() == hipSuccess ? NSK_OK : NSK_EHIP;
}

template <int DIM, int NP, typename R, typename GT>
int launch_stage_t(nsk_ctx* c, const double* Uin, double* Uout, double* dU, const StageArgs& st) {
  if (c->tile == 1 && Epb<DIM, NP>::V1 != Epb<DIM, NP>::V0)
    return launch_stage_e<DIM, NP, Epb<DIM, NP>::V1, R, GT>(c, Uin, Uout, dU, st);
  return launch_stage_e<DIM, NP, Epb<DIM, NP>::V0, R, GT>(c, Uin, Uout, dU, st);
}

template <int DIM, int NP, typename GT>
int launch_diag_t(nsk_ctx* c, const double* Uin) {
  constexpr int EPB = Epb<DIM, NP>::V0;
  using Tl = Tile<DIM, NP, EPB>;
  const BasisArgs b = basis_args(c);
  const MeshArgs m = mesh_args(c);
  const PhysArgs p = phys_args(c);
  GT* G = reinterpret_cast<GT*>(c->work + c->off_G);
  const unsigned blocks = (unsigned)((c->E + EPB - 1) / EPB);
  using R = GT;
  double* part = reinterpret_cast<double*>(c->work + c->off_part);
  double* out = reinterpret_cast<double*>(c->work + c->off_out);
  const double* wq = reinterpret_cast<const double*>(c->work + c->off_wq);
  bool done = false;
  if constexpr (std::is_same<GT, double>::value) {
    if (c->par.model == 1) {
      // the lifted gradient of rho for the capillary energy; the speed is
      // reduced by the diagnostics kernel itself
      hipLaunchKernelGGL((nsk_lift_kernel<DIM, NP, EPB>), dim3(blocks), dim3(Tl::THREADS), 0, c->stream, Uin, G, b, m,
                         p, nullptr);
      hipLaunchKernelGGL((diag_partial_kernel<DIM, NP, GT, 1>), dim3(c->diag_blocks), dim3(kDiagThreads), 0,
                         c->stream, Uin, G, part, wq, m, p);
      done = true;
    }
  }
  if (!done) {
    hipLaunchKernelGGL((lift_kernel<DIM, NP, EPB, R, GT>), dim3(blocks), dim3(Tl::THREADS), 0, c->stream, Uin, G, b,
                       m, p);
    hipLaunchKernelGGL((diag_partial_kernel<DIM, NP, GT>), dim3(c->diag_blocks), dim3(kDiagThreads), 0, c->stream,
                       Uin, G, part, wq, m, p);
  }
  hipLaunchKernelGGL(diag_final_kernel<kDiagSlots>, dim3(1), dim3(kDiagThreads), 0, c->stream, part, c->diag_blocks,
                     out);
  return hipGetLastError() == hipSuccess ? NSK_OK : NSK_EHIP;
}

template <int DIM, int NP>
int dispatch_prec(nsk_ctx* c, int what, const double* Uin, double* Uout, double* dU, const StageArgs& st) {
  if (c->par.precision == 0) {
    if (what == 0) return launch_stage_t<DIM, NP, double, double>(c, Uin, Uout, dU, st);
    return launch_diag_t<DIM, NP, double>(c, Uin);
  }
  if (what == 0) return launch_stage_t<DIM, NP, float, float>(c, Uin, Uout, dU, st);
  return launch_diag_t<DIM, NP, float>(c, Uin);
}

template <int DIM>
int dispatch_np(nsk_ctx* c, int what, const double* Uin, double* Uout, double* dU, const StageArgs& st) {
  switch (c->np) {
    case 2: return dispatch_prec<DIM, 2>(c, what, Uin, Uout, dU, st);
    case 3: return dispatch_prec<DIM, 3>(c, what, Uin, Uout, dU, st);
    case 4: return dispatch_prec<DIM, 4>(c, what, Uin, Uout, dU, st);
    case 5: return dispatch_prec<DIM, 5>(c, what, Uin, Uout, dU, st);
    case 6: return dispatch_prec<DIM, 6>(c, what, Uin, Uout, dU, st);
    case 7:
      if constexpr (DIM < 3) return dispatch_prec<DIM, 7>(c, what, Uin, Uout, dU, st);
      break;
  }
  return NSK_EUNSUPPORTED;
}

// what = 0: one stage (lift + rhs), what = 1: diagnostics
int dispatch(nsk_ctx* c, int what, const double* Uin, double* Uout, double* dU, const StageArgs& st) {
  switch (c->dim) {
    case 1: return dispatch_np<1>(c, what, Uin, Uout, dU, st);
    case 2: return dispatch_np<2>(c, what, Uin, Uout, dU, st);
    case 3: return dispatch_np<3>(c, what, Uin, Uout, dU, st);
  }
  return NSK_EUNSUPPORTED;
}

double* state_buf(nsk_ctx* c, int which) {
  return which == 0 ? c->U : reinterpret_cast<double*>(c->work + c->off_U2);
}

int run_diag(nsk_ctx* c, double* h) {
  StageArgs st{0.0, 0.0, 0.0, 0};
  int rc = dispatch(c, 1, state_buf(c, c->cur), nullptr, nullptr, st);
  if (rc) return rc;
  if (hipMemcpyAsync(h, c->work + c->off_out, sizeof(double) * kDiagSlots, hipMemcpyDeviceToHost, c->stream) !=
      hipSuccess)
    return NSK_EHIP;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return NSK_EHIP;
  return NSK_OK;
}

// whether the two tile variants launch the same elements per workgroup
template <int DIM, int NP>
constexpr bool same_variants() { return Epb<DIM, NP>::V0 == Epb<DIM, NP>::V1; }
template <int DIM>
bool variants_coincide_dim(int N) {
  switch (N) {
    case 1: return same_variants<DIM, 2>();
    case 2: return same_variants<DIM, 3>();
    case 3: return same_variants<DIM, 4>();
    case 4: return same_variants<DIM, 5>();
    case 5: return same_variants<DIM, 6>();
    default: return same_variants<DIM, 7>();
  }
}
bool variants_coincide(int dim, int N) {
  return dim == 1 ? variants_coincide_dim<1>(N) : dim == 2 ? variants_coincide_dim<2>(N) : variants_coincide_dim<3>(N);
}

// Whole steps in one launch of one workgroup: 1D model II meshes (FP64 or
// mixed, Rusanov or HLLC, no closure, no sub-cells) that the first tile
// variant holds in one workgroup, unless per-stage timing is on.
template <int NP, typename R, typename GT>
int launch_steps_t(nsk_ctx* c, double dt, int nsteps) {
  constexpr int EPB = Epb<1, NP>::V0;
  using Tl = Tile<1, NP, EPB>;
  RkCoefs rk;
  for (int s = 0; s < 5; ++s) {
    rk.A[s] = kRkA[s];
    rk.B[s] = kRkB[s];
  }
  GT* G = reinterpret_cast<GT*>(c->work + c->off_G);
  if (c->par.flux == 1)
    hipLaunchKernelGGL((steps_kernel<1, NP, EPB, R, GT, 1>), dim3(1), dim3(Tl::THREADS), 0, c->stream,
                       state_buf(c, 0), state_buf(c, 1), G, c->dU, basis_args(c), mesh_args(c), phys_args(c), rk, dt,
                       nsteps, c->cur);
  else
    hipLaunchKernelGGL((steps_kernel<1, NP, EPB, R, GT, 0>), dim3(1), dim3(Tl::THREADS), 0, c->stream,
                       state_buf(c, 0), state_buf(c, 1), G, c->dU, basis_args(c), mesh_args(c), phys_args(c), rk, dt,
                       nsteps, c->cur);
  if (hipGetLastError() != hipSuccess) return NSK_EHIP;
  if (nsteps & 1) c->cur = 1 - c->cur;  // five buffer swaps per step
  return NSK_OK;
}

template <int NP>
int launch_steps_np(nsk_ctx* c, double dt, int nsteps) {
  if (c->par.precision == 0) return launch_steps_t<NP, double, double>(c, dt, nsteps);
  return launch_steps_t<NP, float, float>(c, dt, nsteps);
}

int launch_steps(nsk_ctx* c, double dt, int nsteps) {
  switch (c->np) {
    case 2: return launch_steps_np<2>(c, dt, nsteps);
    case 3: return launch_steps_np<3>(c, dt, nsteps);
    case 4: return launch_steps_np<4>(c, dt, nsteps);
    case 5: return launch_steps_np<5>(c, dt, nsteps);
    case 6: return launch_steps_np<6>(c, dt, nsteps);
    case 7: return launch_steps_np<7>(c, dt, nsteps);
  }
  return NSK_EUNSUPPORTED;
}

int epb_v0_1d(int np) {
  switch (np) {
    case 2: return Epb<1, 2>::V0;
    case 3: return Epb<1, 3>::V0;
    case 4: return Epb<1, 4>::V0;
    case 5: return Epb<1, 5>::V0;
    case 6: return Epb<1, 6>::V0;
    case 7: return Epb<1, 7>::V0;
  }
  return 0;
}

bool steps_in_one_workgroup(const nsk_ctx* c) {
  if (c->dim != 1 || c->par.model != 0 || c->par.subcell != 0 || c->par.closure != 0 || !c->events.empty())
    return false;
  if (c->tile != 0 && !variants_coincide(1, c->N)) return false;
  return c->E <= epb_v0_1d(c->np);
}

// nsteps Runge-Kutta steps enqueued stage by stage on the bound stream
int enqueue_steps(nsk_ctx* c, double dt, int nsteps) {
  for (int step = 0; step < nsteps; ++step) {
    for (int s = 0; s < 5; ++s) {
      StageArgs st{kRkA[s], kRkB[s], dt, 1};
      c->cl_stage = s;
      int rc = dispatch(c, 0, state_buf(c, c->cur), state_buf(c, 1 - c->cur), c->dU, st);
      c->cl_stage = -1;
      if (rc) return rc;
      c->cur = 1 - c->cur;
    }
  }
  return NSK_OK;
}

void drop_step_graph(nsk_ctx* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
  c->graph_key.clear();
}

// Everything the launches of a step take from the context: the step size,
// the state buffer it starts from, the bound memory and stream, the launch
// shape, the parameters and the closure network.
std::vector<unsigned char> step_graph_key(const nsk_ctx* c, double dt) {
  std::vector<unsigned char> k;
  auto put = [&k](const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    k.insert(k.end(), b, b + n);
  };
  put(&dt, sizeof(dt));
  put(&c->cur, sizeof(c->cur));
  put(&c->U, sizeof(c->U));
  put(&c->dU, sizeof(c->dU));
  put(&c->work, sizeof(c->work));
  put(&c->stream, sizeof(c->stream));
  put(&c->tile, sizeof(c->tile));
  put(&c->order, sizeof(c->order));
  put(&c->par, sizeof(c->par));
  put(&c->cl_w, sizeof(c->cl_w));
  put(c->cl_norm, sizeof(c->cl_norm));
  put(&c->cl_every_stage, sizeof(c->cl_every_stage));
  return k;
}

int build_step_graph(nsk_ctx* c, double dt) {
  drop_step_graph(c);
  if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return NSK_EHIP;
  const int cur0 = c->cur;
  const int rc = enqueue_steps(c, dt, 2);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->stream, &g);
  c->cur = cur0;  // capturing ran nothing
  if (rc || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return rc ? rc : NSK_EHIP;
  }
  c->graph = g;
  if (hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
    drop_step_graph(c);
    return NSK_EHIP;
  }
  return NSK_OK;
}

// ---------------------------------------------------------------------------
// Scratch of nsk_rhs_noalloc: element widths, element order and lifted
// gradients, in a static device array instead of a caller's workspace.  Host
// code reaches it only through the per-device address hipGetSymbolAddress
// returns (the array's name is a host-side stand-in, not a device address).
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[NSK_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
unsigned char* g_scratch[kMaxDevices] = {};

// the array's address on the current device, looked up once per device
int scratch_address(unsigned char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return NSK_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NSK_EHIP;
    g_scratch[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch[dev];
  return NSK_OK;
}

struct NoallocLayout {
  size_t off_h2[3], off_order, off_G, bytes;
};

NoallocLayout noalloc_layout(const nsk_ctx* c) {
  NoallocLayout l;
  const size_t gsz = c->par.precision == 0 ? sizeof(double) : sizeof(float);
  size_t off = 0;
  for (int d = 0; d < 3; ++d) {
    l.off_h2[d] = off;
    off = align256(off + sizeof(double) * (size_t)c->nel[d]);
  }
  l.off_order = off;
  off = align256(off + sizeof(int) * (size_t)c->E);
  l.off_G = off;
  off = align256(off + gsz * (size_t)c->ng * (size_t)c->S);
  l.bytes = off;
  return l;
}

// 2/h per element index along each direction of a uniform mesh, with the
// host's arithmetic of nsk_create (the same bits), and the natural element
// order
__global__ void noalloc_geometry_kernel(double* __restrict__ h2x, double* __restrict__ h2y,
                                        double* __restrict__ h2z, int* __restrict__ order, int dim, int nx, int ny,
                                        int nz, double lo0, double hi0, double lo1, double hi1, double lo2,
                                        double hi2, int E) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < E) order[i] = i;
  const int nel[3] = {nx, ny, nz};
  const double lo[3] = {lo0, lo1, lo2}, hi[3] = {hi0, hi1, hi2};
  double* h2[3] = {h2x, h2y, h2z};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (i >= nel[d]) continue;
    if (d >= dim) {
      h2[d][i] = 1.0;
      continue;
    }
    const double L = hi[d] - lo[d];
    const double a = lo[d] + L * i / nel[d];
    const double b = lo[d] + L * (i + 1) / nel[d];
    h2[d][i] = 2.0 / (b - a);
  }
}

}  // namespace

extern "C" {

const char* nsk_strerror(int code) {
  switch (code) {
    case NSK_OK: return "ok";
    case NSK_EINVAL: return "invalid mesh, parameters or argument";
    case NSK_ENONPHYS: return "non-physical state (non-finite value or density outside (0,3))";
    case NSK_EHIP: return "HIP runtime error";
    case NSK_EUNBOUND: return "device memory not bound";
    case NSK_EUNSUPPORTED: return "unsupported dimension/degree";
    case NSK_ENOCONV: return "implicit stage equations did not converge";
    case NSK_ESCRATCH: return "problem too large for the static scratch of nsk_rhs_noalloc";
  }
  return "unknown error";
}

int nsk_create(const nsk_mesh* mesh, const nsk_params* params, nsk_ctx** out) {
  if (!mesh || !out) return NSK_EINVAL;
  *out = nullptr;
  if (mesh->dim < 1 || mesh->dim > 3 || mesh->N < 1 || mesh->N > kMaxNP - 1) return NSK_EINVAL;
  // not built: a 3D element of degree 6 has 343 nodes, more than the 256
  // threads of the sub-cell workgroups, and its rhs tile would take about
  // 105 KB of LDS (one workgroup per CU)
  if (mesh->dim == 3 && mesh->N > 5) return NSK_EUNSUPPORTED;
  int rc = check_params(params);
  if (rc) return rc;
  nsk_ctx* c = new (std::nothrow) nsk_ctx();
  if (!c) return NSK_EINVAL;
  c->mesh = *mesh;
  c->par = *params;
  c->dim = mesh->dim;
  c->N = mesh->N;
  c->np = mesh->N + 1;
  c->nn = 1;
  for (int d = 0; d < c->dim; ++d) c->nn *= c->np;
  c->nvar = c->dim + (c->par.model == 1 ? 1 : 2);
  c->ng = c->dim * (c->dim + 1) / 2 + c->dim;
  c->E = 1;
  for (int d = 0; d < 3; ++d) {
    if (d < c->dim && mesh->xbreaks[d]) c->uniform = false;
    c->mesh.xbreaks[d] = nullptr;  // not kept: copied into h2 below
    if (d >= c->dim) {
      c->nel[d] = 1;
      c->h2[d].assign(1, 1.0);
      continue;
    }
    if (mesh->nel[d] < 1 || mesh->nel[d] > (1 << 20)) { delete c; return NSK_EINVAL; }
    c->nel[d] = mesh->nel[d];
    c->E *= c->nel[d];
    c->h2[d].resize(c->nel[d]);
    for (int k = 0; k < c->nel[d]; ++k) {
      double a, b;
      if (mesh->xbreaks[d]) {
        a = mesh->xbreaks[d][k];
        b = mesh->xbreaks[d][k + 1];
      } else {
        const double L = mesh->hi[d] - mesh->lo[d];
        a = mesh->lo[d] + L * k / c->nel[d];
        b = mesh->lo[d] + L * (k + 1) / c->nel[d];
      }
      if (!(b > a) || !std::isfinite(a) || !std::isfinite(b)) { delete c; return NSK_EINVAL; }
      c->h2[d][k] = 2.0 / (b - a);
    }
  }
  c->S = c->E * c->nn;
  if (c->E > (1LL << 30) || c->S * (c->nvar > c->ng ? c->nvar : c->ng) > (1LL << 40)) { delete c; return NSK_EINVAL; }
  make_basis(c->N, c->basis);
  c->zR = rk_real_limit();
  spinodal_band(c->par.T, c->rho_lo64, c->rho_hi64);

  // workspace layout
  const size_t gsz = c->par.precision == 0 ? sizeof(double) : sizeof(float);
  size_t off = 0;
  c->off_U2 = off;
  off = align256(off + sizeof(double) * (size_t)c->nvar * c->S);
  c->off_G = off;
  off = align256(off + gsz * (size_t)c->ng * c->S);
  for (int d = 0; d < 3; ++d) {
    c->off_h2[d] = off;
    off = align256(off + sizeof(double) * c->h2[d].size());
  }
  c->off_wq = off;
  off = align256(off + sizeof(double) * kMaxNP);
  c->off_order = off;
  off = align256(off + sizeof(int) * (size_t)c->E);
  const int epbd = kDiagThreads / c->nn > 0 ? kDiagThreads / c->nn : 1;  // elements per diagnostics group
  long long blk = (c->E + epbd - 1) / epbd;
  c->diag_blocks = (int)(blk < 1024 ? blk : 1024);
  c->off_part = off;
  off = align256(off + sizeof(double) * kDiagSlots * (size_t)c->diag_blocks);
  c->off_out = off;
  off = align256(off + sizeof(double) * 16);
  if (c->par.closure == 1) {
    c->off_cl = off;
    off = align256(off + sizeof(float) * (size_t)(c->dim + 1) * c->S);
  }
  if (c->par.subcell == 1) {
    subcell_matrices(c->basis, c->sc_M, c->sc_Minv, c->sc_V);
    c->off_sc_flags = off;
    off = align256(off + sizeof(int) * (size_t)c->E);
    c->off_sc_need = off;
    off = align256(off + sizeof(int) * (size_t)c->E);
    c->off_sc_Ub = off;
    off = align256(off + sizeof(double) * (size_t)c->nvar * c->S);
    c->off_sc_Gb = off;
    off = align256(off + sizeof(double) * (size_t)c->dim * (c->dim + 1) * c->S);
  }
  if (c->par.model == 1) {
    // global LF speed, the second-level maxima and one partial maximum per
    // lifting workgroup (at most one workgroup per element)
    c->off_lf = off;
    off = align256(off + sizeof(double) * (size_t)(c->E + 1 + kMaxReduceBlocks));
  }
  c->ws_bytes = off;
  // default launch shape: tiled work order in 3D, natural order otherwise
  c->order = c->dim == 3 ? 4 : 0;
  *out = c;
  return NSK_OK;
}

void nsk_destroy(nsk_ctx* c) {
  if (!c) return;
  if (c->bound) (void)hipStreamSynchronize(c->stream);
  drop_step_graph(c);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  delete c;
}

int nsk_subcell_flags(nsk_ctx* c, int* d_flags) {
  if (!c || !d_flags || c->par.subcell != 1) return NSK_EINVAL;
  if (!c->bound) return NSK_EUNBOUND;
  return hipMemcpyAsync(d_flags, c->work + c->off_sc_flags, sizeof(int) * (size_t)c->E, hipMemcpyDeviceToDevice,
                        c->stream) == hipSuccess
             ? NSK_OK
             : NSK_EHIP;
}

int nsk_timing_enable(nsk_ctx* c, int enable) {
  if (!c) return NSK_EINVAL;
  if (c->bound) (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  c->events.clear();
  c->timed = 0;
  if (!enable) return NSK_OK;
  const int n = 4 * 4096;
  c->events.resize(n);
  for (int i = 0; i < n; ++i)
    if (hipEventCreate(&c->events[i]) != hipSuccess) {
      c->events.resize(i);
      nsk_timing_enable(c, 0);
      return NSK_EHIP;
    }
  return NSK_OK;
}

int nsk_timing_read(nsk_ctx* c, double out[4]) {
  if (!c || !out) return NSK_EINVAL;
  out[0] = out[1] = out[2] = out[3] = 0.0;
  if (c->timed == 0) return NSK_OK;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return NSK_EHIP;
  for (int k = 0; k < c->timed; ++k) {
    float a = 0.f, b = 0.f, q = 0.f;
    if (hipEventElapsedTime(&a, c->events[4 * k], c->events[4 * k + 1]) != hipSuccess) return NSK_EHIP;
    if (hipEventElapsedTime(&q, c->events[4 * k + 1], c->events[4 * k + 2]) != hipSuccess) return NSK_EHIP;
    if (hipEventElapsedTime(&b, c->events[4 * k + 2], c->events[4 * k + 3]) != hipSuccess) return NSK_EHIP;
    out[0] += a;
    out[1] += b;
    out[3] += q;
  }
  out[2] = c->timed;
  c->timed = 0;
  return NSK_OK;
}

size_t nsk_state_size(const nsk_ctx* c) { return c ? (size_t)c->nvar * c->S : 0; }

size_t nsk_workspace_bytes(const nsk_ctx* c) { return c ? c->ws_bytes : 0; }

int nsk_bind(nsk_ctx* c, double* d_U, double* d_dU, void* d_work, void* hip_stream) {
  if (!c || !d_U || !d_dU || !d_work) return NSK_EINVAL;
  if ((reinterpret_cast<uintptr_t>(d_work) & 255) != 0) return NSK_EINVAL;
  c->U = d_U;
  c->dU = d_dU;
  c->work = static_cast<char*>(d_work);
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->cur = 0;
  for (int d = 0; d < 3; ++d)
    if (hipMemcpyAsync(c->work + c->off_h2[d], c->h2[d].data(), sizeof(double) * c->h2[d].size(),
                       hipMemcpyHostToDevice, c->stream) != hipSuccess)
      return NSK_EHIP;
  double wq[kMaxNP] = {0};
  for (int i = 0; i < c->np; ++i) wq[i] = c->basis.w[i];
  if (hipMemcpyAsync(c->work + c->off_wq, wq, sizeof(wq), hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return NSK_EHIP;
  if (hipMemsetAsync(c->dU, 0, sizeof(double) * nsk_state_size(c), c->stream) != hipSuccess) return NSK_EHIP;
  // the host arrays above are stack/heap memory owned here: wait for the copies
  if (hipStreamSynchronize(c->stream) != hipSuccess) return NSK_EHIP;
  int rc = upload_order(c, c->order);
  if (rc) return rc;
  c->bound = true;
  return NSK_OK;
}

int nsk_set_state(nsk_ctx* c, const double* d_src) {
  if (!c || !d_src) return NSK_EINVAL;
  if (!c->bound) return NSK_EUNBOUND;
  c->cur = 0;
  if (d_src == c->U) return NSK_OK;
  return hipMemcpyAsync(c->U, d_src, sizeof(double) * nsk_state_size(c), hipMemcpyDeviceToDevice, c->stream) ==
                 hipSuccess
             ? NSK_OK
             : NSK_EHIP;
}

int nsk_get_state(nsk_ctx* c, double* d_dst) {
  if (!c || !d_dst) return NSK_EINVAL;
  if (!c->bound) return NSK_EUNBOUND;
  const double* src = state_buf(c, c->cur);
  if (src == d_dst) return NSK_OK;
  return hipMemcpyAsync(d_dst, src, sizeof(double) * nsk_state_size(c), hipMemcpyDeviceToDevice, c->stream) ==
                 hipSuccess
             ? NSK_OK
             : NSK_EHIP;
}

int nsk_rhs(nsk_ctx* c, const double* d_U, double* d_R, double t) {
  (void)t;
  if (!c || !d_U || !d_R || d_U == d_R) return NSK_EINVAL;
  if (!c->bound) return NSK_EUNBOUND;
  if (c->par.closure == 1 && !c->cl_w) return NSK_EINVAL;  // closure enabled, no network set
  StageArgs st{0.0, 0.0, 0.0, 0};
  return dispatch(c, 0, d_U, d_R, nullptr, st);
}

int nsk_rhs_noalloc(nsk_ctx* c, const double* d_U, double* d_R, void* hip_stream) {
  if (!c || !d_U || !d_R || d_U == d_R) return NSK_EINVAL;
  if (c->par.model != 0 || c->par.closure != 0 || c->par.subcell != 0 || !c->uniform) return NSK_EUNSUPPORTED;
  const NoallocLayout l = noalloc_layout(c);
  if (l.bytes > NSK_NOALLOC_SCRATCH_BYTES) return NSK_ESCRATCH;
  unsigned char* base = nullptr;
  int rc = scratch_address(&base);
  if (rc) return rc;
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  const int span = (int)std::max<long long>(c->E, std::max(c->nel[0], std::max(c->nel[1], c->nel[2])));
  hipLaunchKernelGGL(noalloc_geometry_kernel, dim3((span + 255) / 256), dim3(256), 0, stream,
                     reinterpret_cast<double*>(base + l.off_h2[0]), reinterpret_cast<double*>(base + l.off_h2[1]),
                     reinterpret_cast<double*>(base + l.off_h2[2]), reinterpret_cast<int*>(base + l.off_order),
                     c->dim, c->nel[0], c->nel[1], c->nel[2], c->mesh.lo[0], c->mesh.hi[0], c->mesh.lo[1],
                     c->mesh.hi[1], c->mesh.lo[2], c->mesh.hi[2], (int)c->E);
  if (hipGetLastError() != hipSuccess) return NSK_EHIP;
  // the stage launchers read the workspace, stream and order from the
  // context: point them at the scratch for this call (a context is not
  // reentrant), then restore them
  char* work = c->work;
  const size_t off_G = c->off_G, off_order = c->off_order;
  const size_t off_h2[3] = {c->off_h2[0], c->off_h2[1], c->off_h2[2]};
  hipStream_t bound_stream = c->stream;
  const int order = c->order;
  c->work = reinterpret_cast<char*>(base);
  c->off_G = l.off_G;
  c->off_order = l.off_order;
  for (int d = 0; d < 3; ++d) c->off_h2[d] = l.off_h2[d];
  c->stream = stream;
  c->order = 1;  // natural order, one contiguous range per XCD
  StageArgs st{0.0, 0.0, 0.0, 0};
  rc = dispatch(c, 0, d_U, d_R, nullptr, st);
  c->work = work;
  c->off_G = off_G;
  c->off_order = off_order;
  for (int d = 0; d < 3; ++d) c->off_h2[d] = off_h2[d];
  c->stream = bound_stream;
  c->order = order;
  return rc;
}

int nsk_rk_step(nsk_ctx* c, double dt, int nsteps) {
  if (!c || nsteps < 0 || !(dt > 0.0) || !std::isfinite(dt)) return NSK_EINVAL;
  if (!c->bound) return NSK_EUNBOUND;
  if (c->par.closure == 1 && !c->cl_w) return NSK_EINVAL;  // closure enabled, no network set
  // A mesh that one workgroup holds runs all its steps in one launch.
  // Otherwise pairs of steps replay one captured graph (ten stages bring the
  // state back to the buffer it started in); the null stream cannot be
  // captured, and timed stages record events between the launches.
  int left = nsteps;
  if (nsteps > 0 && steps_in_one_workgroup(c)) {
    // the whole mesh in one workgroup: all steps in one launch
    const int rc = launch_steps(c, dt, nsteps);
    if (rc) return rc;
    left = 0;
  } else if (nsteps >= 2 && c->stream != nullptr && c->events.empty()) {
    const std::vector<unsigned char> key = step_graph_key(c, dt);
    if (!c->graph_exec || key != c->graph_key) {
      int rc = build_step_graph(c, dt);
      if (rc) return rc;
      c->graph_key = key;
    }
    for (; left >= 2; left -= 2)
      if (hipGraphLaunch(c->graph_exec, c->stream) != hipSuccess) return NSK_EHIP;
  }
  int rc = enqueue_steps(c, dt, left);
  if (rc) return rc;
  if (c->cur == 1) {
    if (hipMemcpyAsync(c->U, state_buf(c, 1), sizeof(double) * nsk_state_size(c), hipMemcpyDeviceToDevice,
                       c->stream) != hipSuccess)
      return NSK_EHIP;
    c->cur = 0;
  }
  return NSK_OK;
}

int nsk_diagnostics(nsk_ctx* c, nsk_diag* o) {
  if (!c || !o) return NSK_EINVAL;
  if (!c->bound) return NSK_EUNBOUND;
  double h[kDiagSlots];
  int rc = run_diag(c, h);
  if (rc) return rc;
  std::memset(o, 0, sizeof(*o));
  for (int v = 0; v < c->nvar; ++v) o->mass[v] = h[v];
  o->e_kin = h[5];
  o->e_total = h[6];
  o->l2_rho_minus_c = std::sqrt(h[7]);
  o->rho_min = h[8];
  o->rho_max = h[9];
  o->max_wavespeed = h[10];
  o->nonfinite = (long long)h[11];
  const bool bad = o->nonfinite > 0 || !(o->rho_min > 0.0) || !(o->rho_max < 3.0);
  o->status = bad ? NSK_ENONPHYS : NSK_OK;
  return o->status;
}

int nsk_dt_estimate(nsk_ctx* c, double cfl, double* dt_out) {
  if (!c || !dt_out || !(cfl > 0.0)) return NSK_EINVAL;
  if (!c->bound) return NSK_EUNBOUND;
  double h[kDiagSlots];
  int rc = run_diag(c, h);
  if (rc) return rc;
  if (h[11] > 0.0 || !(h[8] > 0.0)) return NSK_ENONPHYS;
  const double N2 = 2.0 * c->N + 1.0;
  // the viscous stress diffuses v = m / rho: the longitudinal mode's rate,
  // (4/3) eps / rho, at the smallest density
  const double nu = (4.0 / 3.0) * c->par.eps / h[8];
  if (c->par.model == 1) {
    // original NSK: convective bound with the global LF speed, viscous bound,
    // and the bound of the capillary modes (frequencies sqrt(kappa rho) k^2)
    double s1 = 0.0, s2 = 0.0;  // max_e sum_d 1/h_d and 1/h_d^2
    for (int d = 0; d < c->dim; ++d) {
      double m = 0.0;
      for (double x : c->h2[d]) m = std::fmax(m, 0.5 * x);
      s1 += m;
      s2 += m * m;
    }
    const double lam = h[10], rmax = h[9];
    double dt = INFINITY;
    if (lam > 0.0) dt = std::fmin(dt, 1.0 / (N2 * lam * s1));
    if (c->par.eps > 0.0) dt = std::fmin(dt, 1.0 / (N2 * N2 * nu * s2));
    if (c->par.kappa > 0.0) dt = std::fmin(dt, 0.25 / (N2 * N2 * std::sqrt(c->par.kappa * rmax) * s2));
    *dt_out = cfl * dt;
    return NSK_OK;
  }
  // Sec. 3.1 bounds: convective, viscous momentum, and the equation for c,
  // whose diffusion rate (2N+1)^2 sum_d (kappa/beta)/h_d^2 and relaxation
  // source rate alpha/beta are both real and negative and so add against the
  // real-axis stability limit z_R of the Runge-Kutta scheme
  const double lam_c = h[12];
  double s2 = 0.0;  // max over elements of sum_d 1/h_d^2 (a tensor grid: the sum of per-direction maxima)
  for (int d = 0; d < c->dim; ++d) {
    double m = 0.0;
    for (double x : c->h2[d]) m = std::fmax(m, 0.25 * x * x);
    s2 += m;
  }
  double dt = INFINITY;
  if (lam_c > 0.0) dt = std::fmin(dt, 1.0 / (N2 * lam_c));
  if (c->par.eps > 0.0) dt = std::fmin(dt, 1.0 / (N2 * N2 * nu * s2));
  dt = std::fmin(dt, 1.0 / (N2 * N2 * (c->par.kappa / c->par.beta) * s2 + c->par.alpha / (c->par.beta * c->zR)));
  *dt_out = cfl * dt;
  return NSK_OK;
}

int nsk_set_tile(nsk_ctx* c, int variant, int order) {
  if (!c || variant < 0 || variant >= kTileVariants || order < 0 || order >= kOrders) return NSK_EINVAL;
  c->tile = variant;
  if (!c->bound) {
    c->order = order;
    return NSK_OK;
  }
  return order == c->order ? NSK_OK : upload_order(c, order);
}

int nsk_autotune(nsk_ctx* c, int reps, int* variant_out, int* order_out, double* ms_out) {
  if (!c || reps < 1) return NSK_EINVAL;
  if (!c->bound) return NSK_EUNBOUND;
  if (c->cur != 0) return NSK_EINVAL;  // the scratch state buffer must be free
  if (c->par.closure == 1 && !c->cl_w) return NSK_EINVAL;  // closure enabled, no network set
  const int keep_tile = c->tile, keep_order = c->order;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return NSK_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return NSK_EHIP; }
  StageArgs st{0.0, 0.0, 0.0, 0};
  double per_k[kTileVariants * kOrders];
  for (int k = 0; k < kTileVariants * kOrders; ++k) per_k[k] = INFINITY;
  int rc = NSK_OK;
  for (int k = 0; k < kTileVariants * kOrders && rc == NSK_OK; ++k) {
    const int v = k / kOrders, o = k % kOrders;
    if (ms_out) ms_out[k] = -1.0;
    // orders that coincide for this mesh (1D, or the same tiles) are skipped
    if (o >= 2 && c->dim == 1) continue;
    if (v == 1 && variants_coincide(c->dim, c->N)) continue;
    rc = nsk_set_tile(c, v, o);
    if (rc) break;
    // right-hand side of the bound state written into the scratch state buffer
    rc = dispatch(c, 0, c->U, state_buf(c, 1), nullptr, st);
    if (rc) break;
    if (hipEventRecord(e0, c->stream) != hipSuccess) { rc = NSK_EHIP; break; }
    for (int r = 0; r < reps && rc == NSK_OK; ++r) rc = dispatch(c, 0, c->U, state_buf(c, 1), nullptr, st);
    if (rc) break;
    float ms = 0.f;
    if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = NSK_EHIP;
      break;
    }
    const double per = ms / reps;
    if (ms_out) ms_out[k] = per;
    per_k[k] = per;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // the first shape within 1% of the fastest: timings of near-equal shapes
  // are noise, and among the tiled orders the first is the smallest tile,
  // which re-reads the fewest neighbour elements from HBM
  double best = INFINITY;
  for (int k = 0; k < kTileVariants * kOrders; ++k) best = per_k[k] < best ? per_k[k] : best;
  int bv = keep_tile, bo = keep_order;
  for (int k = 0; k < kTileVariants * kOrders; ++k)
    if (per_k[k] <= best * 1.01) {
      bv = k / kOrders;
      bo = k % kOrders;
      break;
    }
  int rc2 = nsk_set_tile(c, rc == NSK_OK ? bv : keep_tile, rc == NSK_OK ? bo : keep_order);
  if (rc == NSK_OK) rc = rc2;
  if (variant_out) *variant_out = c->tile;
  if (order_out) *order_out = c->order;
  return rc;
}

int nsk_set_params(nsk_ctx* c, const nsk_params* p) {
  if (!c) return NSK_EINVAL;
  int rc = check_params(p);
  if (rc) return rc;
  // the workspace layout depends on the model, the precision and the closure flag
  if (p->model != c->par.model || p->precision != c->par.precision || p->closure != c->par.closure ||
      p->subcell != c->par.subcell)
    return NSK_EINVAL;
  c->par = *p;
  spinodal_band(c->par.T, c->rho_lo64, c->rho_hi64);
  return NSK_OK;
}

}  // extern "C"
