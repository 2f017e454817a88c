// C ABI of the batched solver (jl_batch_*): problem table, largest-first
// ordering, workspace carve-up and the captured hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "internal.h"

using namespace jl;

struct jl_batch_s {
  jl_ctx ctx = nullptr;
  int count = 0, nev = 0;
  jl_batch_shape shape{};    // the launch shape in use (defaults resolved)
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ready = nullptr;
  double* h_out = nullptr;   // pinned: evals, res, status, stats
  double tick_s = 0.0;       // seconds per tick of the device wall clock
};

namespace {

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct BLayout {
  size_t table, order, queue, evals, res, status, stats, slots, total;
  size_t slot_bytes;
  jl_batch_shape shape;
  int64_t hmax;
};

jl_status batch_layout(jl_ctx ctx, int count, const int64_t* n, jl_dtype dtype, const jl_params* p,
                       const jl_batch_shape* shp, BLayout* L) {
  if (count < 1 || !n || !p) return set_err(ctx, JL_EINVAL, "count >= 1, n and params are required");
  if (dtype != JL_C64 && dtype != JL_C128) return set_err(ctx, JL_EINVAL, "dtype must be JL_C64 or JL_C128");
  jl_batch_shape sh = shp ? *shp : jl_batch_shape{};
  if (sh.threads == 0) sh.threads = 256;
  if (sh.rows_per_wave == 0) sh.rows_per_wave = 1;
  if (sh.unroll == 0) sh.unroll = 4;
  if (sh.threads != 128 && sh.threads != 256 && sh.threads != 512)
    return set_err(ctx, JL_EINVAL, "threads must be 128, 256 or 512");
  if (sh.rows_per_wave != 1 && sh.rows_per_wave != 2)
    return set_err(ctx, JL_EINVAL, "rows_per_wave must be 1 or 2");
  if (sh.unroll != 4 && sh.unroll != 8) return set_err(ctx, JL_EINVAL, "unroll must be 4 or 8");
  if (sh.lds_matrix_bytes < 0 || sh.lds_matrix_bytes % 16)
    return set_err(ctx, JL_EINVAL, "lds_matrix_bytes must be a non-negative multiple of 16");
  if (p->nev < 1 || p->mwin < p->nev || p->m <= p->mwin)
    return set_err(ctx, JL_EINVAL, "need 1 <= nev <= mwin < m");
  if (p->m + (p->m & 1) > 60) return set_err(ctx, JL_EINVAL, "batched solver supports m <= 59 (got %d)", p->m);
  if (!(p->tol > 0.0)) return set_err(ctx, JL_EINVAL, "tol must be positive");
  if (p->which != JL_LOWEST && p->which != JL_LARGEST) return set_err(ctx, JL_EINVAL, "invalid which");
  if (p->standard) return set_err(ctx, JL_EUNSUPPORTED, "the batched solver is J-restricted only");
  if (p->invert) return set_err(ctx, JL_EUNSUPPORTED, "the batched solver has no invert mode");
  int64_t hmax = 0;
  for (int i = 0; i < count; ++i) {
    if (n[i] < 2 || n[i] % 2) return set_err(ctx, JL_EINVAL, "n[%d] = %lld must be even and >= 2", i, (long long)n[i]);
    if ((int64_t)p->m > n[i] / 2) return set_err(ctx, JL_EINVAL, "m exceeds n[%d]/2", i);
    hmax = std::max(hmax, n[i] / 2);
  }
  const int es = dtype == JL_C64 ? 8 : 16;
  int dev = 0, ncu = 0, lds_max = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    ncu = 256;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
      lds_max <= 0)
    lds_max = 64 * 1024;
  if (batched_lds_bytes(hmax, p->m, es) + (size_t)sh.lds_matrix_bytes > (size_t)lds_max)
    return set_err(ctx, JL_EINVAL,
                   "largest problem (n = %lld) with %d bytes for a resident matrix exceeds the %d bytes "
                   "of LDS a workgroup may use", (long long)(2 * hmax), sh.lds_matrix_bytes, lds_max);
  if (sh.blocks <= 0) sh.blocks = std::min(count, 2 * ncu);
  L->shape = sh;
  L->hmax = hmax;
  L->slot_bytes = batched_slot_bytes(hmax, p->m, es);
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off = align_up(off + b); return o; };
  L->table = take(sizeof(BatchProblem) * count);
  L->order = take(sizeof(int) * count);
  L->queue = take(sizeof(int) * 64);
  L->evals = take(sizeof(double) * (size_t)count * p->nev);
  L->res = take(sizeof(double) * (size_t)count * p->nev);
  L->status = take(sizeof(int) * count);
  L->stats = take(sizeof(int) * kBatchStats * (size_t)count);
  L->slots = take(L->slot_bytes * (size_t)sh.blocks);
  L->total = off;
  return JL_OK;
}

}  // namespace

extern "C" {

jl_status jl_batch_workspace_bytes(int32_t count, const int64_t* n, jl_dtype dtype,
                                   const jl_params* p, const jl_batch_shape* shape, size_t* bytes) {
  if (!bytes) return set_err(nullptr, JL_EINVAL, "bytes is NULL");
  BLayout L;
  jl_status s = batch_layout(nullptr, count, n, dtype, p, shape, &L);
  if (s != JL_OK) return s;
  *bytes = L.total;
  return JL_OK;
}

jl_status jl_batch_create(jl_ctx ctx, int32_t count, const int64_t* n, const void* const* A11,
                          const void* const* A12, jl_dtype dtype, const jl_params* p,
                          void* const* X, void* ws, size_t ws_bytes, const jl_batch_shape* shape,
                          jl_batch* out) {
  if (!ctx || !out) return set_err(ctx, JL_EINVAL, "ctx and out are required");
  if (!A11 || !A12 || !X) return set_err(ctx, JL_EINVAL, "A11, A12 and X arrays are required");
  DeviceGuard g(ctx->device);
  BLayout L;
  jl_status s = batch_layout(ctx, count, n, dtype, p, shape, &L);
  if (s != JL_OK) return s;
  if (!ws || ws_bytes < L.total)
    return set_err(ctx, JL_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, L.total);
  std::vector<BatchProblem> table(count);
  for (int i = 0; i < count; ++i) {
    if (!A11[i] || !A12[i] || !X[i]) return set_err(ctx, JL_EINVAL, "NULL pointer for problem %d", i);
    table[i] = BatchProblem{n[i] / 2, A11[i], A12[i], n[i] / 2, X[i], n[i]};
  }
  // largest first (longest-processing-time order for the shared queue)
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n[a] > n[b]; });
  char* base = static_cast<char*>(ws);
  auto* d_table = reinterpret_cast<BatchProblem*>(base + L.table);
  auto* d_order = reinterpret_cast<int*>(base + L.order);
  auto* d_queue = reinterpret_cast<int*>(base + L.queue);
  BatchOut o;
  o.evals = reinterpret_cast<double*>(base + L.evals);
  o.res = reinterpret_cast<double*>(base + L.res);
  o.status = reinterpret_cast<int*>(base + L.status);
  o.stats = reinterpret_cast<int*>(base + L.stats);
  char* slots = base + L.slots;
  BatchParams P;
  P.nev = p->nev;
  P.m = p->m;
  P.mwin = p->mwin;
  P.which = p->which;
  P.max_cycles = p->max_cycles > 0 ? p->max_cycles : 10000;
  P.max_passes = p->max_passes > 0 ? p->max_passes : 16;
  P.min_passes = std::min(p->min_passes > 0 ? p->min_passes : 1, P.max_passes);
  P.tol_relative = p->tol_relative;
  P.lds_mat = L.shape.lds_matrix_bytes;
  P.tol = p->tol;

  jl_batch b = new jl_batch_s();
  b->ctx = ctx;
  b->count = count;
  b->nev = p->nev;
  b->shape = L.shape;
  auto fail = [&](jl_status code) {
    jl_batch_destroy(b);
    return code;
  };
  hipError_t e;
#define BCHK(expr)                                                                           \
  if ((e = (expr)) != hipSuccess)                                                            \
    return fail(set_err(ctx, JL_EHIP, "%s failed: %s", #expr, hipGetErrorString(e)));
  BCHK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
  BCHK(hipEventCreateWithFlags(&b->ready, hipEventDisableTiming));
  {
    int dev = 0, khz = 0;
    BCHK(hipGetDevice(&dev));
    BCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    b->tick_s = khz > 0 ? 1e-3 / khz : 0.0;
  }
  // doubles: evals, res, then the ints status [count] and stats [count][kBatchStats]
  const size_t nout = 2 * (size_t)count * p->nev + ((size_t)(1 + kBatchStats) * count + 1) / 2;
  BCHK(hipHostMalloc((void**)&b->h_out, sizeof(double) * nout, hipHostMallocDefault));
  // table and order are uploaded once (synchronously: the host vectors die here)
  BCHK(hipMemcpyAsync(d_table, table.data(), sizeof(BatchProblem) * count, hipMemcpyHostToDevice, b->stream));
  BCHK(hipMemcpyAsync(d_order, order.data(), sizeof(int) * count, hipMemcpyHostToDevice, b->stream));
  BCHK(hipStreamSynchronize(b->stream));
  // capture: queue reset, persistent launch, result copies
  double* h_evals = b->h_out;
  double* h_res = h_evals + (size_t)count * p->nev;
  int* h_status = reinterpret_cast<int*>(h_res + (size_t)count * p->nev);
  int* h_stats = h_status + count;
  BCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  hipError_t ce = launch_batched_init(d_queue, b->stream);
  if (ce == hipSuccess)
    ce = dtype == JL_C64
             ? launch_batched<float>(d_table, d_order, count, P, d_queue, slots, L.slot_bytes, L.hmax, o,
                                     L.shape.threads, L.shape.rows_per_wave, L.shape.unroll,
                                     L.shape.blocks, b->stream)
             : launch_batched<double>(d_table, d_order, count, P, d_queue, slots, L.slot_bytes, L.hmax, o,
                                      L.shape.threads, L.shape.rows_per_wave, L.shape.unroll,
                                      L.shape.blocks, b->stream);
  if (ce == hipSuccess)
    ce = hipMemcpyAsync(h_evals, o.evals, sizeof(double) * (size_t)count * p->nev, hipMemcpyDeviceToHost, b->stream);
  if (ce == hipSuccess)
    ce = hipMemcpyAsync(h_res, o.res, sizeof(double) * (size_t)count * p->nev, hipMemcpyDeviceToHost, b->stream);
  if (ce == hipSuccess)
    ce = hipMemcpyAsync(h_status, o.status, sizeof(int) * count, hipMemcpyDeviceToHost, b->stream);
  if (ce == hipSuccess)
    ce = hipMemcpyAsync(h_stats, o.stats, sizeof(int) * kBatchStats * (size_t)count, hipMemcpyDeviceToHost,
                        b->stream);
  hipError_t ee = hipStreamEndCapture(b->stream, &b->graph);
  if (ce != hipSuccess) return fail(set_err(ctx, JL_EHIP, "batched capture failed: %s", hipGetErrorString(ce)));
  if (ee != hipSuccess) return fail(set_err(ctx, JL_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(ee)));
  BCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
#undef BCHK
  *out = b;
  return JL_OK;
}

jl_status jl_batch_shape_used(jl_batch b, jl_batch_shape* shape) {
  if (!b || !shape) return set_err(b ? b->ctx : nullptr, JL_EINVAL, "batch and shape are required");
  *shape = b->shape;
  return JL_OK;
}

jl_status jl_batch_run(jl_batch b, double* evals, double* res, int32_t* status,
                       jl_batch_stats* stats) {
  if (!b) return set_err(nullptr, JL_EINVAL, "batch is NULL");
  jl_ctx ctx = b->ctx;
  if (!evals || !res || !status) return set_err(ctx, JL_EINVAL, "evals, res and status are required");
  DeviceGuard g(ctx->device);
  // order after the caller's work on the context stream
  JL_HIP(ctx, hipEventRecord(b->ready, ctx->stream));
  JL_HIP(ctx, hipStreamWaitEvent(b->stream, b->ready, 0));
  JL_HIP(ctx, hipGraphLaunch(b->exec, b->stream));
  JL_HIP(ctx, hipStreamSynchronize(b->stream));
  const size_t ne = (size_t)b->count * b->nev;
  const double* h_evals = b->h_out;
  const double* h_res = h_evals + ne;
  const int* h_status = reinterpret_cast<const int*>(h_res + ne);
  const int* h_stats = h_status + b->count;
  std::copy(h_evals, h_evals + ne, evals);
  std::copy(h_res, h_res + ne, res);
  bool all = true;
  for (int i = 0; i < b->count; ++i) {
    status[i] = h_status[i] == 0 ? JL_OK : (h_status[i] == 2 ? JL_BREAKDOWN : JL_NOT_CONVERGED);
    all = all && h_status[i] == 0;
    if (stats) {
      stats[i].cycles = h_stats[kBatchStats * i];
      stats[i].n_mv = h_stats[kBatchStats * i + 1];
      stats[i].gs_passes = h_stats[kBatchStats * i + 2];
      stats[i].icnv = h_stats[kBatchStats * i + 3];
      stats[i].n_resid = h_stats[kBatchStats * i + 4];
      double* t[kBatchPhases] = {&stats[i].t_apply, &stats[i].t_gs, &stats[i].t_ritz, &stats[i].t_restart,
                                 &stats[i].t_resid};
      for (int ph = 0; ph < kBatchPhases; ++ph) *t[ph] = b->tick_s * h_stats[kBatchStats * i + 5 + ph];
    }
  }
  return all ? JL_OK : JL_NOT_CONVERGED;
}

jl_status jl_batch_destroy(jl_batch b) {
  if (!b) return JL_OK;
  if (b->stream) hipStreamSynchronize(b->stream);
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->ready) hipEventDestroy(b->ready);
  if (b->stream) hipStreamDestroy(b->stream);
  if (b->h_out) hipHostFree(b->h_out);
  delete b;
  return JL_OK;
}

}  // extern "C"
