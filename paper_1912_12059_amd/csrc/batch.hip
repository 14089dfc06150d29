// libnsk batched form: many 3D instances of uneven mesh size and degree
// advanced together.  Each instance is an ordinary context bound to a slice
// of one packed state buffer and of one workspace.  Instances are grouped by
// degree; per group and per stage one lifting kernel and one right-hand-side
// kernel walk a list of (instance, element block) items, one workgroup per
// item or a persistent grid taking the list in rounds.  Two full Runge-Kutta
// steps (ten stages, every group) are captured into one HIP graph that is
// replayed, so the whole batch advances with one graph launch per two steps.
// A built-in autotuner picks, per degree and precision, the elements per
// workgroup and the grid size.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/nsk.h"
#include "dg_kernels.hpp"
#include "host_common.hpp"

namespace {

// persistent grid = CUs * m; m = 0: one workgroup per item (no persistence)
constexpr int kGridMults[4] = {0, 2, 4, 8};
// working-set budget per chunk of instances (MiB; 0: the whole group at once)
constexpr int kChunkMiB[4] = {0, 128, 256, 512};
constexpr int kBatchTuneSlots = 8 + 4;  // timings per group in nsk_batch_autotune

struct BatchGroup {
  int np = 0;                 // N + 1
  std::vector<int> inst;      // member instances
  size_t off_items = 0;       // byte offset of the item list in the workspace
  size_t cap_items = 0;       // capacity in items (sum of element counts)
  int nitems = 0;             // items for the current variant
  int variant = 0;            // elements-per-workgroup variant
  int gridmul = 0;            // grid = CUs * gridmul, 0: one workgroup per item
  int chunk_mib = 0;          // working-set budget of a chunk of instances, 0: no chunking
  std::vector<int> chunks;    // item index boundaries of the chunks (first 0, last nitems)
  std::vector<int> chunk_inst;  // the instance of a one-instance chunk, else -1
};

}  // namespace

struct nsk_batch {
  int ninst = 0;
  nsk_params par;
  std::vector<nsk_ctx*> ctx;
  std::vector<size_t> state_off;   // doubles, 256-byte aligned
  size_t state_total = 0;
  std::vector<size_t> work_off;    // bytes
  size_t off_desc = 0;             // two BatchInst tables (stage parity 0 and 1)
  size_t ws_bytes = 0;
  std::vector<BatchGroup> groups;
  bool bound = false;
  double* U = nullptr;
  double* dU = nullptr;
  char* work = nullptr;
  hipStream_t stream = nullptr;
  int ncu = 256;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double graph_dt = -1.0;
};

namespace {

int epb_of(int np, int variant) {
  switch (np) {
    case 2: return variant ? Epb<3, 2>::V1 : Epb<3, 2>::V0;
    case 3: return variant ? Epb<3, 3>::V1 : Epb<3, 3>::V0;
    case 4: return variant ? Epb<3, 4>::V1 : Epb<3, 4>::V0;
    case 5: return variant ? Epb<3, 5>::V1 : Epb<3, 5>::V0;
    case 6: return variant ? Epb<3, 6>::V1 : Epb<3, 6>::V0;
  }
  return 1;
}

void drop_graph(nsk_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_dt = -1.0;
}

// descriptor of instance i for stage parity p: p = 0 reads U, writes the
// workspace copy; p = 1 the reverse
BatchInst make_desc(nsk_batch* b, int i, int p) {
  nsk_ctx* c = b->ctx[i];
  BatchInst d;
  double* U2 = reinterpret_cast<double*>(c->work + c->off_U2);
  d.U = p ? U2 : c->U;
  d.Uout = p ? c->U : U2;
  d.dU = c->dU;
  d.G = c->work + c->off_G;
  d.msh = mesh_args(c);
  d.msh.nxcd = 1;
  return d;
}

int upload_tables(nsk_batch* b) {
  std::vector<BatchInst> desc(2 * b->ninst);
  for (int p = 0; p < 2; ++p)
    for (int i = 0; i < b->ninst; ++i) desc[p * b->ninst + i] = make_desc(b, i, p);
  if (hipMemcpyAsync(b->work + b->off_desc, desc.data(), sizeof(BatchInst) * desc.size(), hipMemcpyHostToDevice,
                     b->stream) != hipSuccess)
    return NSK_EHIP;
  for (BatchGroup& g : b->groups) {
    const int epb = epb_of(g.np, g.variant);
    std::vector<BatchItem> items;
    for (int i : g.inst) {
      const int nblk = (int)((b->ctx[i]->E + epb - 1) / epb);
      for (int L = 0; L < nblk; ++L) items.push_back(BatchItem{i, L});
    }
    g.nitems = (int)items.size();
    if (items.size() > g.cap_items) return NSK_EINVAL;
    // chunks of whole instances whose working set (state, its copy, the
    // register and the lifted gradients) stays within the budget: a chunk
    // runs all the stages of a graph replay back to back while that data
    // is still in the caches
    g.chunks.assign(1, 0);
    g.chunk_inst.clear();
    const size_t budget = (size_t)g.chunk_mib << 20;
    size_t acc = 0;
    int pos = 0, first = -1, count = 0;
    for (int i : g.inst) {
      const nsk_ctx* c = b->ctx[i];
      const size_t gbytes = (size_t)c->S * (3 * sizeof(double) * (size_t)c->nvar +
                                            (size_t)c->ng * (c->par.precision == 0 ? sizeof(double) : sizeof(float)));
      const int nblk = (int)((c->E + epb - 1) / epb);
      if (budget && pos > g.chunks.back() && acc + gbytes > budget) {
        g.chunks.push_back(pos);
        g.chunk_inst.push_back(count == 1 ? first : -1);
        acc = 0;
        count = 0;
      }
      if (count == 0) first = i;
      ++count;
      acc += gbytes;
      pos += nblk;
    }
    if (g.chunks.back() != pos) {
      g.chunks.push_back(pos);
      g.chunk_inst.push_back(count == 1 ? first : -1);
    }
    if (hipMemcpyAsync(b->work + g.off_items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice,
                       b->stream) != hipSuccess)
      return NSK_EHIP;
  }
  if (hipStreamSynchronize(b->stream) != hipSuccess) return NSK_EHIP;
  drop_graph(b);
  return NSK_OK;
}

// one stage of chunk k of group g through the batch kernels (items of the
// group's elements-per-workgroup variant)
template <int NP, int EPB, typename R, typename GT>
int launch_chunk_e(nsk_batch* b, const BatchGroup& g, int k, int parity, const StageArgs& st) {
  using Tl = Tile<3, NP, EPB>;
  const BasisArgs bas = basis_args(b->ctx[g.inst[0]]);
  const PhysArgs ph = phys_args(b->ctx[g.inst[0]]);
  const BatchInst* desc = reinterpret_cast<const BatchInst*>(b->work + b->off_desc) + parity * b->ninst;
  const BatchItem* items = reinterpret_cast<const BatchItem*>(b->work + g.off_items) + g.chunks[k];
  const int n = g.chunks[k + 1] - g.chunks[k];
  if (n <= 0) return NSK_OK;
  if (g.gridmul == 0) {
    hipLaunchKernelGGL((lift_kernel_batch1<3, NP, EPB, R, GT>), dim3(n), dim3(Tl::THREADS), 0, b->stream, desc, items,
                       bas, ph);
    hipLaunchKernelGGL((rhs_kernel_batch1<3, NP, EPB, R, GT>), dim3(n), dim3(Tl::THREADS), 0, b->stream, desc, items,
                       bas, ph, st);
  } else {
    const int grid = std::min(n, b->ncu * g.gridmul);
    hipLaunchKernelGGL((lift_kernel_batch<3, NP, EPB, R, GT>), dim3(grid), dim3(Tl::THREADS), 0, b->stream, desc,
                       items, n, bas, ph);
    hipLaunchKernelGGL((rhs_kernel_batch<3, NP, EPB, R, GT>), dim3(grid), dim3(Tl::THREADS), 0, b->stream, desc,
                       items, n, bas, ph, st);
  }
  return hipGetLastError() == hipSuccess ? NSK_OK : NSK_EHIP;
}

// one stage of a one-instance chunk: the single-mesh kernels with the
// instance's own elements-per-workgroup variant, order and buffers as
// arguments (no descriptor loads)
template <int NP, int EPB, typename R, typename GT>
int launch_single_e(nsk_batch* b, nsk_ctx* c, int parity, const StageArgs& st) {
  using Tl = Tile<3, NP, EPB>;
  double* U2 = reinterpret_cast<double*>(c->work + c->off_U2);
  const double* Uin = parity ? U2 : c->U;
  double* Uout = parity ? c->U : U2;
  GT* G = reinterpret_cast<GT*>(c->work + c->off_G);
  const BasisArgs bas = basis_args(c);
  const MeshArgs m = mesh_args(c);
  const PhysArgs ph = phys_args(c);
  const unsigned blocks = (unsigned)((c->E + EPB - 1) / EPB);
  hipLaunchKernelGGL((lift_kernel<3, NP, EPB, R, GT>), dim3(blocks), dim3(Tl::THREADS), 0, b->stream, Uin, G, bas, m,
                     ph);
  hipLaunchKernelGGL((rhs_kernel<3, NP, EPB, R, GT>), dim3(blocks), dim3(Tl::THREADS), 0, b->stream, Uin, G, Uout,
                     c->dU, bas, m, ph, st);
  return hipGetLastError() == hipSuccess ? NSK_OK : NSK_EHIP;
}

template <int NP, typename R, typename GT>
int launch_group_t(nsk_batch* b, const BatchGroup& g, int chunk, int parity, const StageArgs& st) {
  constexpr bool TWO = Epb<3, NP>::V1 != Epb<3, NP>::V0;
  for (int k = 0; k + 1 < (int)g.chunks.size(); ++k) {
    if (chunk >= 0 && chunk != k) continue;
    int rc;
    if (g.gridmul == 0 && g.chunk_inst[k] >= 0) {
      nsk_ctx* c = b->ctx[g.chunk_inst[k]];
      rc = (TWO && c->tile == 1) ? launch_single_e<NP, Epb<3, NP>::V1, R, GT>(b, c, parity, st)
                                 : launch_single_e<NP, Epb<3, NP>::V0, R, GT>(b, c, parity, st);
    } else {
      rc = (TWO && g.variant == 1) ? launch_chunk_e<NP, Epb<3, NP>::V1, R, GT>(b, g, k, parity, st)
                                   : launch_chunk_e<NP, Epb<3, NP>::V0, R, GT>(b, g, k, parity, st);
    }
    if (rc) return rc;
  }
  return NSK_OK;
}

template <typename R, typename GT>
int launch_group_p(nsk_batch* b, const BatchGroup& g, int chunk, int parity, const StageArgs& st) {
  switch (g.np) {
    case 2: return launch_group_t<2, R, GT>(b, g, chunk, parity, st);
    case 3: return launch_group_t<3, R, GT>(b, g, chunk, parity, st);
    case 4: return launch_group_t<4, R, GT>(b, g, chunk, parity, st);
    case 5: return launch_group_t<5, R, GT>(b, g, chunk, parity, st);
    case 6: return launch_group_t<6, R, GT>(b, g, chunk, parity, st);
  }
  return NSK_EUNSUPPORTED;
}

// one stage of one chunk of group g (chunk < 0: every chunk of the group)
int launch_group(nsk_batch* b, const BatchGroup& g, int parity, const StageArgs& st, int chunk = -1) {
  if (b->par.precision == 0) return launch_group_p<double, double>(b, g, chunk, parity, st);
  return launch_group_p<float, float>(b, g, chunk, parity, st);
}

// two full steps, chunk by chunk: the ten stages (parity alternating, state
// back in U at the end) of one chunk of instances run back to back
int enqueue_two_steps(nsk_batch* b, double dt) {
  for (const BatchGroup& g : b->groups)
    for (int ch = 0; ch + 1 < (int)g.chunks.size(); ++ch)
      for (int k = 0; k < 10; ++k) {
        const StageArgs st{kRkA[k % 5], kRkB[k % 5], dt, 1};
        int rc = launch_group(b, g, k & 1, st, ch);
        if (rc) return rc;
      }
  return NSK_OK;
}

int build_graph(nsk_batch* b, double dt) {
  drop_graph(b);
  if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return NSK_EHIP;
  int rc = enqueue_two_steps(b, dt);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess || !g) return NSK_EHIP;
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    drop_graph(b);
    return NSK_EHIP;
  }
  b->graph_dt = dt;
  return NSK_OK;
}

}  // namespace

extern "C" {

int nsk_batch_create(const nsk_mesh* meshes, int ninst, const nsk_params* params, nsk_batch** out) {
  if (!meshes || !params || !out || ninst < 1) return NSK_EINVAL;
  *out = nullptr;
  for (int i = 0; i < ninst; ++i)
    if (meshes[i].dim != 3) return NSK_EUNSUPPORTED;
  if (params->model != 0 || params->closure != 0 || params->flux != 0 || params->subcell != 0) return NSK_EUNSUPPORTED;
  nsk_batch* b = new (std::nothrow) nsk_batch();
  if (!b) return NSK_EINVAL;
  b->ninst = ninst;
  b->par = *params;
  size_t soff = 0, woff = 0;
  for (int i = 0; i < ninst; ++i) {
    nsk_ctx* c = nullptr;
    int rc = nsk_create(&meshes[i], params, &c);
    if (rc) {
      for (nsk_ctx* x : b->ctx) nsk_destroy(x);
      delete b;
      return rc;
    }
    b->ctx.push_back(c);
    b->state_off.push_back(soff);
    soff += (nsk_state_size(c) + 31) / 32 * 32;  // 256-byte aligned slices
    b->work_off.push_back(woff);
    woff = align256(woff + nsk_workspace_bytes(c));
  }
  b->state_total = soff;
  b->off_desc = woff;
  woff = align256(woff + 2 * sizeof(BatchInst) * (size_t)ninst);
  // groups by degree
  for (int i = 0; i < ninst; ++i) {
    const int np = b->ctx[i]->np;
    BatchGroup* g = nullptr;
    for (BatchGroup& x : b->groups)
      if (x.np == np) g = &x;
    if (!g) {
      b->groups.push_back(BatchGroup());
      g = &b->groups.back();
      g->np = np;
    }
    g->inst.push_back(i);
    g->cap_items += (size_t)b->ctx[i]->E;
  }
  for (BatchGroup& g : b->groups) {
    g.off_items = woff;
    woff = align256(woff + sizeof(BatchItem) * g.cap_items);
  }
  b->ws_bytes = woff;
  *out = b;
  return NSK_OK;
}

void nsk_batch_destroy(nsk_batch* b) {
  if (!b) return;
  if (b->bound) (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  for (nsk_ctx* c : b->ctx) nsk_destroy(c);
  delete b;
}

size_t nsk_batch_state_size(const nsk_batch* b) { return b ? b->state_total : 0; }

size_t nsk_batch_state_offset(const nsk_batch* b, int inst) {
  return (b && inst >= 0 && inst < b->ninst) ? b->state_off[inst] : 0;
}

size_t nsk_batch_workspace_bytes(const nsk_batch* b) { return b ? b->ws_bytes : 0; }

int nsk_batch_bind(nsk_batch* b, double* d_U, double* d_dU, void* d_work, void* hip_stream) {
  if (!b || !d_U || !d_dU || !d_work || !hip_stream) return NSK_EINVAL;
  if ((reinterpret_cast<uintptr_t>(d_work) & 255) != 0 || (reinterpret_cast<uintptr_t>(d_U) & 255) != 0 ||
      (reinterpret_cast<uintptr_t>(d_dU) & 255) != 0)
    return NSK_EINVAL;
  b->U = d_U;
  b->dU = d_dU;
  b->work = static_cast<char*>(d_work);
  b->stream = static_cast<hipStream_t>(hip_stream);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return NSK_EHIP;
  for (int i = 0; i < b->ninst; ++i) {
    int rc = nsk_bind(b->ctx[i], d_U + b->state_off[i], d_dU + b->state_off[i], b->work + b->work_off[i], hip_stream);
    if (rc) return rc;
  }
  int rc = upload_tables(b);
  if (rc) return rc;
  b->bound = true;
  return NSK_OK;
}

int nsk_batch_ctx(nsk_batch* b, int inst, nsk_ctx** out) {
  if (!b || !out || inst < 0 || inst >= b->ninst) return NSK_EINVAL;
  *out = b->ctx[inst];
  return NSK_OK;
}

int nsk_batch_dt_estimate(nsk_batch* b, double cfl, double* dt_out) {
  if (!b || !dt_out) return NSK_EINVAL;
  if (!b->bound) return NSK_EUNBOUND;
  double dt = INFINITY;
  for (nsk_ctx* c : b->ctx) {
    double x;
    int rc = nsk_dt_estimate(c, cfl, &x);
    if (rc) return rc;
    dt = std::min(dt, x);
  }
  *dt_out = dt;
  return NSK_OK;
}

int nsk_batch_rk_step(nsk_batch* b, double dt, int nsteps) {
  if (!b || nsteps < 0 || !(dt > 0.0) || !std::isfinite(dt)) return NSK_EINVAL;
  if (!b->bound) return NSK_EUNBOUND;
  for (nsk_ctx* c : b->ctx)
    if (c->cur != 0) return NSK_EINVAL;
  const int pairs = nsteps / 2;
  if (pairs > 0) {
    if (!b->exec || b->graph_dt != dt) {
      int rc = build_graph(b, dt);
      if (rc) return rc;
    }
    for (int k = 0; k < pairs; ++k)
      if (hipGraphLaunch(b->exec, b->stream) != hipSuccess) return NSK_EHIP;
  }
  if (nsteps & 1)
    for (nsk_ctx* c : b->ctx) {
      int rc = nsk_rk_step(c, dt, 1);
      if (rc) return rc;
    }
  return NSK_OK;
}

int nsk_batch_autotune(nsk_batch* b, int reps, double* ms_out) {
  if (!b || reps < 1) return NSK_EINVAL;
  if (!b->bound) return NSK_EUNBOUND;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return NSK_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return NSK_EHIP; }
  const StageArgs st{0.0, 0.0, 0.0, 0};  // right-hand side into the scratch state buffers
  int rc = NSK_OK;
  // each instance's own variant and element order (used when it runs as a
  // chunk of its own)
  for (nsk_ctx* c : b->ctx) {
    int v = 0, o = 0;
    if ((rc = nsk_autotune(c, reps, &v, &o, nullptr)) != NSK_OK) break;
  }
  if (rc == NSK_OK) rc = upload_tables(b);
  for (size_t gi = 0; gi < b->groups.size() && rc == NSK_OK; ++gi) {
    BatchGroup& g = b->groups[gi];
    double best = INFINITY;
    // elements per workgroup and grid of the batch kernels, timed on the
    // whole group as one chunk
    g.chunk_mib = 0;
    int bv = g.variant, bm = g.gridmul;
    for (int v = 0; v < kTileVariants && rc == NSK_OK; ++v) {
      g.variant = v;
      if ((rc = upload_tables(b)) != NSK_OK) break;
      for (int mi = 0; mi < 4 && rc == NSK_OK; ++mi) {
        g.gridmul = kGridMults[mi];
        rc = launch_group(b, g, 0, st);
        if (rc) break;
        if (hipEventRecord(e0, b->stream) != hipSuccess) { rc = NSK_EHIP; break; }
        for (int r = 0; r < reps && rc == NSK_OK; ++r) rc = launch_group(b, g, 0, st);
        float ms = 0.f;
        if (rc || hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          if (!rc) rc = NSK_EHIP;
          break;
        }
        const double per = ms / reps;
        if (ms_out) ms_out[gi * kBatchTuneSlots + v * 4 + mi] = per;
        if (per < best) { best = per; bv = v; bm = kGridMults[mi]; }
      }
    }
    g.variant = bv;
    g.gridmul = bm;
    if (rc) break;
    // chunk budget, with the chosen order and launch shape
    best = INFINITY;
    int bc = g.chunk_mib;
    for (int ci = 0; ci < 4 && rc == NSK_OK; ++ci) {
      g.chunk_mib = kChunkMiB[ci];
      if ((rc = upload_tables(b)) != NSK_OK) break;
      // ten consecutive stages per chunk, as a graph replay runs them
      auto sweep = [&]() {
        int r2 = NSK_OK;
        for (int ch = 0; ch + 1 < (int)g.chunks.size() && r2 == NSK_OK; ++ch)
          for (int k = 0; k < 10 && r2 == NSK_OK; ++k) r2 = launch_group(b, g, 0, st, ch);
        return r2;
      };
      if ((rc = sweep()) != NSK_OK) break;
      if (hipEventRecord(e0, b->stream) != hipSuccess) { rc = NSK_EHIP; break; }
      for (int r = 0; r < reps && rc == NSK_OK; ++r) rc = sweep();
      float ms = 0.f;
      if (rc || hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        if (!rc) rc = NSK_EHIP;
        break;
      }
      const double per = ms / (10.0 * reps);  // per stage
      if (ms_out) ms_out[gi * kBatchTuneSlots + 8 + ci] = per;
      if (per < best) { best = per; bc = kChunkMiB[ci]; }
    }
    g.chunk_mib = bc;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  int rc2 = upload_tables(b);
  return rc ? rc : rc2;
}

int nsk_batch_set_group(nsk_batch* b, int group, int variant, int gridmul, int order, int chunk_mib) {
  if (!b || group < 0 || group >= (int)b->groups.size()) return NSK_EINVAL;
  if (variant < 0 || variant >= kTileVariants || order < 0 || order >= kOrders) return NSK_EINVAL;
  if (gridmul != 0 && gridmul != 2 && gridmul != 4 && gridmul != 8) return NSK_EINVAL;
  if (chunk_mib < 0) return NSK_EINVAL;
  if (!b->bound) return NSK_EUNBOUND;
  BatchGroup& g = b->groups[group];
  g.variant = variant;
  g.gridmul = gridmul;
  g.chunk_mib = chunk_mib;
  for (int i : g.inst) {
    b->ctx[i]->tile = variant;
    int rc = upload_order(b->ctx[i], order);
    if (rc) return rc;
  }
  return upload_tables(b);
}

int nsk_batch_groups(const nsk_batch* b, int* np_out, int* variant_out, int* gridmul_out, int* order_out,
                     int* chunk_mib_out, int max) {
  if (!b) return NSK_EINVAL;
  const int n = (int)b->groups.size();
  for (int i = 0; i < n && i < max; ++i) {
    if (np_out) np_out[i] = b->groups[i].np - 1;
    if (variant_out) variant_out[i] = b->groups[i].variant;
    if (gridmul_out) gridmul_out[i] = b->groups[i].gridmul;
    if (order_out) order_out[i] = b->ctx[b->groups[i].inst[0]]->order;
    if (chunk_mib_out) chunk_mib_out[i] = b->groups[i].chunk_mib;
  }
  return n;
}

}  // extern "C"
