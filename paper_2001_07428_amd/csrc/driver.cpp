// Host driver and C ABI of the J-symmetric thick-restart Lanczos solver.
//
// The control flow is Algorithm 1 (outer thick-restart loop) with Algorithm 2
// (the J-restricted Lanczos steps) as its inner loop; every vector operation
// is a kernel on the context's stream and the host only handles the m x m
// projected matrix bookkeeping and a few scalars per step:
//   - per Lanczos step: t_jj (accumulated in the operator apply), the norm
//     b0 after the local three-term step and the norm b1 after each
//     reorthogonalisation pass (the sqrt(2) test of Alg. 2 is taken on the
//     host), fetched in one copy; the normalisation of v_{j+1} (its factor
//     read on the device) and the next operator apply are queued before the
//     host waits for that copy, and are redone in the rare step that needs
//     another pass;
//   - once per cycle the sorted Ritz values, the last row of Z and the true
//     residuals of the candidates.
// In invert mode each step's u = A^-1 v_j comes from conjugate gradients
// run entirely on the device (k_cg.hip); the host queues batches of
// iterations and looks at the device's done flag between batches.  The
// operators are the dense blocks, the 4D stencil and the Case B operator
// (k_tek.hip), all in the layout where J is the canonical [[0, -I], [I, 0]].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <complex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"

using namespace jl;

namespace {

thread_local std::string g_thread_err;

enum OpKind { OP_DENSE = 1, OP_STENCIL = 2, OP_TEK = 3 };

}  // namespace

struct jl_op_s {
  jl_ctx ctx = nullptr;
  OpKind kind = OP_DENSE;
  jl_dtype dtype = JL_C128;
  int64_t n = 0;
  StencilArgs<float> sf{};
  StencilArgs<double> sd{};
  DenseArgs<float> df{};
  DenseArgs<double> dd{};
  TekArgs<float> tf{};
  TekArgs<double> td{};
  void* links = nullptr;   // owned device memory: stencil links, or the TEK links and scratch
  ~jl_op_s() {
    if (links) (void)hipFree(links);
  }
};

namespace jl {

hipError_t work_stream(jl_ctx ctx, hipStream_t* out) {
  hipError_t e;
  if (!ctx->work && (e = hipStreamCreateWithFlags(&ctx->work, hipStreamNonBlocking)) != hipSuccess) {
    ctx->work = nullptr;
    return e;
  }
  if (!ctx->order && (e = hipEventCreateWithFlags(&ctx->order, hipEventDisableTiming)) != hipSuccess) {
    ctx->order = nullptr;
    return e;
  }
  if ((e = hipEventRecord(ctx->order, ctx->stream)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(ctx->work, ctx->order, 0)) != hipSuccess) return e;
  *out = ctx->work;
  return hipSuccess;
}

jl_status set_err(jl_ctx ctx, jl_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  g_thread_err = buf;
  return code;
}

size_t ritz_scratch_doubles(int m) {
  const size_t jac = eig_work_doubles(m) + (size_t)m + (size_t)m * m + (size_t)m;   // eig, lam, Z, perm
  const size_t dc = m <= dc_max_m() ? 3 * (size_t)m + dc_work_doubles(m) : 0;      // struct, perm, D&C
  return std::max(jac, dc);
}

template <typename S>
hipError_t ritz_arrow_device(int m, int k, const double* hstruct, int descending, int kcols,
                             double* scratch, double* lam_s, double* Zs, S* Zc, double* zlast,
                             hipStream_t st) {
  if (m > dc_max_m() || k < 0 || k >= m) return hipErrorInvalidValue;
  double* ds = scratch;                                    // 2m packed structure
  int* perm = reinterpret_cast<int*>(scratch + 2 * (size_t)m);
  double* work = scratch + 3 * (size_t)m;
  const size_t nstruct = 2 * (size_t)k + (size_t)(m - k) + (size_t)(m - k - 1);
  hipError_t e;
  if ((e = hipMemcpyAsync(ds, hstruct, sizeof(double) * nstruct, hipMemcpyHostToDevice, st)) != hipSuccess)
    return e;
  const double* lam = nullptr;
  const double* Z = nullptr;
  int ldz = 0;
  if ((e = ritz_dc(m, k, hstruct, ds, work, &lam, &Z, &ldz, st)) != hipSuccess) return e;
  return launch_ritz_sort<S>(m, lam, 1, Z, ldz, descending, kcols, perm, lam_s, Zs, Zc, zlast, st);
}

template hipError_t ritz_arrow_device<float>(int, int, const double*, int, int, double*, double*,
                                             double*, float*, double*, hipStream_t);
template hipError_t ritz_arrow_device<double>(int, int, const double*, int, int, double*, double*,
                                              double*, double*, double*, hipStream_t);

template <typename S>
hipError_t ritz_device(int m, const double* Tdev, double fro2, int descending, int kcols,
                       double* scratch, double* lam_s, double* Zs, S* Zc, double* zlast,
                       double* hs, hipStream_t st) {
  double* eigw = scratch;
  double* lam_raw = eigw + eig_work_doubles(m);
  double* Z_raw = lam_raw + m;
  int* perm = reinterpret_cast<int*>(Z_raw + (size_t)m * m);
  const double* lam_ptr;
  int64_t lstride;
  const double* Zptr;
  int ldz;
  const int mp = m + (m & 1);
  hipError_t e;
  if (mp <= eig_small_max()) {
    if ((e = launch_eig_small(Tdev, m, m, lam_raw, Z_raw, m, 60, st)) != hipSuccess) return e;
    lam_ptr = lam_raw;
    lstride = 1;
    Zptr = Z_raw;
    ldz = m;
  } else {
    EigWork w;
    w.A[0] = eigw;
    w.A[1] = eigw + (size_t)mp * mp;
    w.Z = eigw + 2 * (size_t)mp * mp;
    w.off = eigw + 3 * (size_t)mp * mp;
    if ((e = launch_eig_init(Tdev, m, m, w, st)) != hipSuccess) return e;
    int c = 0;
    for (int sweep = 0; sweep < 60; ++sweep) {
      for (int r = 0; r < mp - 1; ++r) {
        if ((e = launch_eig_round(m, w, c, r, st)) != hipSuccess) return e;
        c ^= 1;
      }
      if ((e = launch_eig_offnorm(m, w, c, st)) != hipSuccess) return e;
      if ((e = hipMemcpyAsync(hs, w.off, sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
      if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
      if (hs[0] <= 1e-30 * fro2) break;
    }
    lam_ptr = w.A[c];
    lstride = mp + 1;
    Zptr = w.Z;
    ldz = mp;
  }
  return launch_ritz_sort<S>(m, lam_ptr, lstride, Zptr, ldz, descending, kcols, perm, lam_s, Zs, Zc,
                             zlast, st);
}

template hipError_t ritz_device<float>(int, const double*, double, int, int, double*, double*,
                                       double*, float*, double*, double*, hipStream_t);
template hipError_t ritz_device<double>(int, const double*, double, int, int, double*, double*,
                                        double*, double*, double*, double*, hipStream_t);

}  // namespace jl

namespace {

// Operator dispatch over storage type.
template <typename S> struct OpView;
template <> struct OpView<float> {
  static const StencilArgs<float>& st(const jl_op_s* o) { return o->sf; }
  static const DenseArgs<float>& de(const jl_op_s* o) { return o->df; }
  static const TekArgs<float>& tk(const jl_op_s* o) { return o->tf; }
};
template <> struct OpView<double> {
  static const StencilArgs<double>& st(const jl_op_s* o) { return o->sd; }
  static const DenseArgs<double>& de(const jl_op_s* o) { return o->dd; }
  static const TekArgs<double>& tk(const jl_op_s* o) { return o->td; }
};

template <typename S>
hipError_t op_apply(const jl_op_s* op, const cplx<S>* x, cplx<S>* y, int64_t ld, int nrhs,
                    double* apart, hipStream_t st) {
  if (op->kind == OP_STENCIL)
    return launch_stencil_apply<S>(OpView<S>::st(op), x, y, ld, nrhs, apart, st);
  if (op->kind == OP_TEK) {   // one column at a time (the products are batched inside)
    if (apart && nrhs != 1) return hipErrorInvalidValue;
    for (int r = 0; r < nrhs; ++r) {
      const hipError_t e = launch_tek_apply<S>(OpView<S>::tk(op), x + (int64_t)r * ld,
                                               y + (int64_t)r * ld, apart, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  return launch_dense_apply<S>(OpView<S>::de(op), x, y, ld, nrhs, apart, st);
}

// One CG apply: p = r + beta p_old formed on the fly and stored to pnew,
// q = A p with the partials of p^H q; returns at once while *skip != 0 (CG
// launches queued past convergence).
template <typename S>
hipError_t op_apply_cg(const jl_op_s* op, const double* skip, const cplx<S>* r,
                       const cplx<S>* pold, const double* beta, cplx<S>* pnew, cplx<S>* q,
                       double* apart, hipStream_t st) {
  if (op->kind == OP_STENCIL) {
    StencilArgs<S> a = OpView<S>::st(op);
    a.skip = skip;
    return launch_stencil_apply_dir<S>(a, r, pold, beta, pnew, q, apart, st);
  }
  if (op->kind == OP_TEK) {
    TekArgs<S> a = OpView<S>::tk(op);
    a.skip = skip;
    return launch_tek_apply_dir<S>(a, r, pold, beta, pnew, q, apart, st);
  }
  DenseArgs<S> a = OpView<S>::de(op);
  a.skip = skip;
  return launch_dense_apply_dir<S>(a, r, pold, beta, pnew, q, apart, st);
}

template <typename S>
hipError_t op_resid(const jl_op_s* op, const cplx<S>* X, int64_t ldx, const int* cols,
                    const int* hcols, const double* lam, int ncols, double* partial, int* nblk,
                    hipStream_t st) {
  if (op->kind == OP_TEK)
    return launch_tek_resid<S>(OpView<S>::tk(op), X, ldx, hcols, lam, ncols, partial, nblk, st);
  if (op->kind == OP_STENCIL)
    return launch_stencil_resid<S>(OpView<S>::st(op), X, ldx, cols, lam, ncols, partial, nblk, st);
  return launch_dense_resid<S>(OpView<S>::de(op), X, ldx, cols, lam, ncols, partial, nblk, st);
}

int op_apply_blocks(const jl_op_s* op) {
  if (op->kind == OP_TEK) return tek_apply_blocks(op->tf.N);
  return op->kind == OP_STENCIL ? stencil_apply_blocks(op->n / 8)
                                 : dense_apply_blocks(op->n / 2);
}

int op_resid_blocks(const jl_op_s* op) {
  if (op->kind == OP_TEK) return tek_apply_blocks(op->tf.N);
  return op->kind == OP_STENCIL ? stencil_resid_blocks(op->n / 8) : dense_resid_blocks(op->n / 2);
}

// Algorithmic bytes of one operator apply (storage element size es); for
// the TEK operator (bound by its matrix products) the vectors and links only.
double op_bytes(const jl_op_s* op, int es) {
  if (op->kind == OP_TEK) return es * (2.0 * (double)op->n + 4.0 * op->tf.N * (double)op->tf.N);
  if (op->kind == OP_STENCIL) {
    const double V = (double)(op->n / 8);
    const int bps = op->dtype == JL_C64 ? op->sf.b_per_site : op->sd.b_per_site;
    return V * es * (16.0 + 64.0 + (bps ? 64.0 : 0.0));
  }
  const double h = (double)(op->n / 2);
  return es * (h * (double)op->n + 2.0 * (double)op->n);
}

// ----------------------------------------------------------- workspace layout
struct Layout {
  size_t V[2], apart, dots_part, upd_part, coef, scal, Tdev, ritz, lam_s, Zs, Zg, gmap, zlast, res_part,
      res_out, res_lam, res_cols, cg_vec[5], cg_part, cg_s, rloc, rd, wide_scr, wide_cnt, total;
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

Layout make_layout(const jl_op_s* op, const jl_params* p) {
  const int es = op->dtype == JL_C64 ? 8 : 16;   // bytes per complex element
  const int64_t n = op->n, h = n / 2;
  const int m = p->m;
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.V[0] = take((size_t)n * (m + 1) * es);
  L.V[1] = take((size_t)n * (m + 1) * es);
  L.apart = take(sizeof(double) * 2 * (size_t)op_apply_blocks(op));
  L.dots_part = take(sizeof(double) * (size_t)reorth_dots_blocks(h, es) * (size_t)dots_stride(m + 1));
  L.upd_part = take(sizeof(double) * (size_t)std::max(reorth_update_blocks(h, es, p->standard == 0), 1));
  L.coef = take(sizeof(double) * (4 * (size_t)(m + 1) + 1));
  const int wcols = dots_stride(m + 1);   // the most inner products one pass reduces
  // the slice sums of the wide reductions: the inner products of a pass, and
  // the true residuals of up to nev candidates (fewer columns than wcols)
  L.wide_scr = take(sizeof(double) * std::max(reduce_wide_scratch_doubles(reorth_dots_blocks(h, es), wcols),
                                              reduce_wide_scratch_doubles(op_resid_blocks(op), p->nev)));
  L.wide_cnt = take(sizeof(unsigned) * ((size_t)reduce_wide_tiles(wcols) + 1));   // + update norm
  L.scal = take(sizeof(double) * 64);
  L.Tdev = take(sizeof(double) * (size_t)m * m);
  L.ritz = take(sizeof(double) * ritz_scratch_doubles(m));
  L.lam_s = take(sizeof(double) * m);
  L.Zs = take(sizeof(double) * (size_t)m * m);
  L.Zg = take(sizeof(double) * (size_t)m * m);          // gathered columns of Z for the basis update
  L.gmap = take(sizeof(int) * 3 * (size_t)m);           // its output columns, then copy pairs
  L.zlast = take(sizeof(double) * m);
  L.res_part = take(sizeof(double) * (size_t)op_resid_blocks(op) * p->nev);
  L.res_out = take(sizeof(double) * p->nev);
  L.res_lam = take(sizeof(double) * p->nev);
  L.res_cols = take(sizeof(int) * p->nev);
  const int gd = reorth_dots_groups(h, es), gu = reorth_update_groups(h, es);
  if (gd > 1) L.rloc = take((size_t)n * es);              // the locally updated u (column groups)
  if (gu > 1) L.rd = take((size_t)gu * n * es);           // per-group corrections
  if (p->invert) {   // CG: x, r, q, two directions; partial sums; device scalars
    for (int i = 0; i < 5; ++i) L.cg_vec[i] = take((size_t)n * es);
    L.cg_part = take(sizeof(double) * 2 * (size_t)cg_blocks(n));
    L.cg_s = take(sizeof(double) * CG_NSLOTS);
  }
  L.total = off;
  return L;
}

jl_status check_params(jl_ctx ctx, const jl_op_s* op, const jl_params* p) {
  if (!p) return set_err(ctx, JL_EINVAL, "params is NULL");
  const int64_t n = op->n;
  if (p->nev < 1) return set_err(ctx, JL_EINVAL, "nev must be >= 1 (got %d)", p->nev);
  if (p->mwin < p->nev)
    return set_err(ctx, JL_EINVAL, "mwin (%d) must be >= nev (%d)", p->mwin, p->nev);
  if (p->m <= p->mwin) return set_err(ctx, JL_EINVAL, "m (%d) must exceed mwin (%d)", p->m, p->mwin);
  if (!p->standard && (int64_t)p->m > n / 2)
    return set_err(ctx, JL_EINVAL, "m (%d) exceeds n/2 (%lld): the J-half Krylov space is exhausted",
                   p->m, (long long)(n / 2));
  if (p->standard && (int64_t)p->m > n)
    return set_err(ctx, JL_EINVAL, "m (%d) exceeds n (%lld)", p->m, (long long)n);
  if (p->m + 1 > kReorthMaxCols)
    return set_err(ctx, JL_EINVAL, "m (%d) exceeds the supported maximum %d", p->m,
                   kReorthMaxCols - 1);
  if (!(p->tol > 0.0)) return set_err(ctx, JL_EINVAL, "tol must be positive");
  if (p->which != JL_LOWEST && p->which != JL_LARGEST)
    return set_err(ctx, JL_EINVAL, "which must be JL_LOWEST or JL_LARGEST");
  if (p->trace_cap < 0 || (p->trace_cap > 0 && !p->trace_ab))
    return set_err(ctx, JL_EINVAL, "trace_cap > 0 needs trace_ab");
  if (p->invert && !(p->cg_tol < 1.0))
    return set_err(ctx, JL_EINVAL, "cg_tol must be below 1");
  return JL_OK;
}

// Accumulates GPU time of kernel classes from HIP event pairs; pairs are
// resolved at the driver's synchronisation points.  With stride > 1 the
// per-step classes (operator apply, inner products, update) are timed only
// while `sample` is set (every stride-th Lanczos step), and count()/tcnt/
// tbytes keep the launches and bytes of the timed launches.
struct Timer {
  enum { MATVEC, DOTS, UPDATE, GEMM, RITZ, RESID, CG, NCLS };
  bool on = false;
  int stride = 1;
  bool sample = true;
  int64_t tcnt[NCLS] = {};
  double tbytes[NCLS] = {};
  static bool per_step(int cls) { return cls == MATVEC || cls == DOTS || cls == UPDATE; }
  bool timed(int cls) const { return on && (sample || !per_step(cls)); }
  void count(int cls, double bytes) {
    if (timed(cls)) {
      tcnt[cls]++;
      tbytes[cls] += bytes;
    }
  }
  hipStream_t st = nullptr;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  double t[NCLS] = {};
  int cur = -1;
  hipEvent_t cur_start = nullptr;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void start(int cls) {
    if (!timed(cls)) {
      cur_start = nullptr;
      return;
    }
    cur = cls;
    cur_start = get();
    if (cur_start) hipEventRecord(cur_start, st);
  }
  void stop() {
    if (!on || !cur_start) return;
    hipEvent_t e = get();
    if (!e) return;
    hipEventRecord(e, st);
    pending.push_back({cur, {cur_start, e}});
    cur_start = nullptr;
  }
  // Adds the intervals that have completed; the others stay pending (work
  // queued behind a partial wait).
  void resolve() {
    size_t keep = 0;
    for (auto& pr : pending) {
      if (hipEventQuery(pr.second.second) != hipSuccess) {
        pending[keep++] = pr;
        continue;
      }
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, pr.second.first, pr.second.second) == hipSuccess)
        t[pr.first] += 1e-3 * ms;
      pool.push_back(pr.second.first);
      pool.push_back(pr.second.second);
    }
    pending.resize(keep);
  }
  ~Timer() {
    for (auto e : pool) hipEventDestroy(e);
    for (auto& pr : pending) {
      hipEventDestroy(pr.second.first);
      hipEventDestroy(pr.second.second);
    }
  }
};

// Pinned host staging for the few values read back each step.
struct Pinned {
  double* p = nullptr;
  ~Pinned() {
    if (p) hipHostFree(p);
  }
};

template <typename S>
jl_status solve_impl(jl_op_s* op, const jl_params* prm, const void* v1, void* ws, size_t ws_bytes,
                     double* evals, void* Xout, int64_t ldx, double* res_out, jl_stats* stats) {
  jl_ctx ctx = op->ctx;
  hipStream_t st = nullptr;
  JL_HIP(ctx, work_stream(ctx, &st));
  const auto t_begin = std::chrono::steady_clock::now();
  jl_stats S_{};
  const int64_t n = op->n, h = n / 2;
  const int m = prm->m, nev = prm->nev, mwin = prm->mwin;
  const int kmax = std::min(nev + mwin, m - 1);
  const int max_cycles = prm->max_cycles > 0 ? prm->max_cycles : 10000;
  const int max_passes = prm->max_passes > 0 ? prm->max_passes : 16;
  const int min_passes = std::min(prm->min_passes > 0 ? prm->min_passes : 1, max_passes);
  const int es = (int)sizeof(cplx<S>);
  const double uround = sizeof(S) == 4 ? 5.9604644775390625e-08 : 1.1102230246251565e-16;
  const double bd_factor = 64.0;
  const bool jsym = prm->standard == 0;   // J-restricted (Alg. 2) or standard Gram-Schmidt
  const bool invert = prm->invert != 0;   // Lanczos on A^-1 (Alg. 1 and 2, invert mode)
  // sort order of theta: the wanted end of A's spectrum, reversed under inversion
  const int descending = ((prm->which == JL_LOWEST) == invert) ? 1 : 0;
  const int cg_maxit = prm->cg_maxit > 0 ? prm->cg_maxit : 10000;
  const double cg_tol = prm->cg_tol > 0.0 ? prm->cg_tol : prm->tol;
  constexpr int kCgChunk = 8;   // CG iterations queued between two looks at the done flag

  const Layout L = make_layout(op, prm);
  if (!ws || ws_bytes < L.total)
    return set_err(ctx, JL_ENOMEM, "workspace of %zu bytes is smaller than the %zu required",
                   ws_bytes, L.total);
  if (!evals || !Xout || !res_out) return set_err(ctx, JL_EINVAL, "evals, X and res are required");
  if (ldx < n) return set_err(ctx, JL_EINVAL, "ldx (%lld) < n (%lld)", (long long)ldx, (long long)n);

  char* base = static_cast<char*>(ws);
  cplx<S>* Vb[2] = {reinterpret_cast<cplx<S>*>(base + L.V[0]),
                    reinterpret_cast<cplx<S>*>(base + L.V[1])};
  double* apart = reinterpret_cast<double*>(base + L.apart);
  double* dots_part = reinterpret_cast<double*>(base + L.dots_part);
  double* upd_part = reinterpret_cast<double*>(base + L.upd_part);
  double* coef = reinterpret_cast<double*>(base + L.coef);
  double* wide_scr = reinterpret_cast<double*>(base + L.wide_scr);
  unsigned* wide_cnt = reinterpret_cast<unsigned*>(base + L.wide_cnt);
  double* scal = reinterpret_cast<double*>(base + L.scal);
  double* Tdev = reinterpret_cast<double*>(base + L.Tdev);
  double* ritz_scr = reinterpret_cast<double*>(base + L.ritz);
  double* lam_s = reinterpret_cast<double*>(base + L.lam_s);
  double* Zs = reinterpret_cast<double*>(base + L.Zs);
  double* Zg = reinterpret_cast<double*>(base + L.Zg);
  int* gmap = reinterpret_cast<int*>(base + L.gmap);
  double* zlast = reinterpret_cast<double*>(base + L.zlast);
  double* res_part = reinterpret_cast<double*>(base + L.res_part);
  double* res_dev = reinterpret_cast<double*>(base + L.res_out);
  double* res_lam = reinterpret_cast<double*>(base + L.res_lam);
  int* res_cols = reinterpret_cast<int*>(base + L.res_cols);
  cplx<S>* cgv[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // x, r, q, p (two)
  double* cg_part = nullptr;
  double* cgs = nullptr;
  if (invert) {
    for (int i = 0; i < 5; ++i) cgv[i] = reinterpret_cast<cplx<S>*>(base + L.cg_vec[i]);
    cg_part = reinterpret_cast<double*>(base + L.cg_part);
    cgs = reinterpret_cast<double*>(base + L.cg_s);
  }
  const int ncgb = cg_blocks(n);
  // column groups of the reorthogonalisation kernels for short vectors
  const int gd = reorth_dots_groups(h, es), gu = reorth_update_groups(h, es);
  cplx<S>* uloc = gd > 1 ? reinterpret_cast<cplx<S>*>(base + L.rloc) : nullptr;
  cplx<S>* dscr = gu > 1 ? reinterpret_cast<cplx<S>*>(base + L.rd) : nullptr;

  const int ndots = reorth_dots_blocks(h, es);
  const int wtiles = reduce_wide_tiles(dots_stride(m + 1));
  unsigned* upd_cnt = wide_cnt + wtiles;
  JL_HIP(ctx, hipMemsetAsync(wide_cnt, 0, sizeof(unsigned) * ((size_t)wtiles + 1), st));
  const int napply = op_apply_blocks(op);
  const int nupd = reorth_update_blocks(h, es, jsym);
  const int64_t ldv = n;

  struct Ev {
    hipEvent_t e = nullptr;
    ~Ev() {
      if (e) hipEventDestroy(e);
    }
  } ev_copy[2];   // the scalar copies of two consecutive steps
  for (auto& ev : ev_copy) JL_HIP(ctx, hipEventCreateWithFlags(&ev.e, hipEventDisableTiming));
  Pinned pin;
  const size_t pin_doubles = 16 + CG_NSLOTS + 3 * (size_t)m + 3 * (size_t)nev + 2 * (size_t)m * m +
                             2 * (size_t)m;
  JL_HIP(ctx, hipHostMalloc((void**)&pin.p, sizeof(double) * pin_doubles, hipHostMallocDefault));
  // Every return waits for the stream first (an error can leave queued work,
  // such as the next step's speculative apply); declared after `pin`, so the
  // wait comes before the pinned scalars are freed.
  struct StreamWait {
    hipStream_t s;
    ~StreamWait() { (void)hipStreamSynchronize(s); }
  } stream_wait{st};
  double* hs = pin.p;                    // [16] scalars
  double* hslot[2] = {pin.p, pin.p + 8};   // a step's scalars: slot 0 = hs[0..4], slot 1 = hs[8..12]
  int64_t n_queued = 0;                    // Lanczos steps queued (for the timing sample)
  double* h_cg = pin.p + 16;             // [CG_NSLOTS] CG scalars
  double* h_lam = h_cg + CG_NSLOTS;      // [m]
  double* h_zl = h_lam + m;              // [m]
  double* h_res = h_zl + m;              // [nev]
  double* h_rlam = h_res + nev;          // [nev]
  int* h_rcols = reinterpret_cast<int*>(h_rlam + nev);   // [nev] ints (fits in nev doubles)
  double* h_Z = h_rlam + 2 * (size_t)nev;                 // [m * m] the sorted Z of the cycle
  double* h_Zg = h_Z + (size_t)m * m;                     // [m * m] its gathered columns
  int* h_gmap = reinterpret_cast<int*>(h_Zg + (size_t)m * m);   // [3 m] ints

  Timer tm;
  tm.on = prm->timing != 0;
  tm.stride = prm->timing > 1 ? prm->timing : 1;
  tm.st = st;

  // ---- start vector (Alg. 1: v_1 = ones / ||ones||, or the caller's)
  int cur = 0;
  if (!v1) {
    JL_HIP(ctx, launch_fill<S>(Vb[cur], n, 1.0 / std::sqrt((double)n), st));
  } else {
    JL_HIP(ctx, hipMemcpyAsync(Vb[cur], v1, (size_t)n * es, hipMemcpyDeviceToDevice, st));
    JL_HIP(ctx, launch_reorth_dots<S>(Vb[cur], ldv, 0, Vb[cur], h, dots_part, ndots, st));
    JL_HIP(ctx, launch_reduce_cols(dots_part, ndots, dots_stride(0), 1, scal, st));
    JL_HIP(ctx, hipMemcpyAsync(hs, scal, sizeof(double), hipMemcpyDeviceToHost, st));
    JL_HIP(ctx, hipStreamSynchronize(st));
    if (!(hs[0] > 0.0) || !std::isfinite(hs[0]))
      return set_err(ctx, JL_EINVAL, "start vector has zero or non-finite norm");
    JL_HIP(ctx, launch_scale<S>(Vb[cur], n, 1.0 / std::sqrt(hs[0]), st));
  }

  // Tbar: (m+1) x m, column-major on the host (row i, column j at i + j*(m+1)).
  std::vector<double> T((size_t)(m + 1) * m, 0.0);
  auto Tat = [&](int i, int j) -> double& { return T[(size_t)i + (size_t)j * (m + 1)]; };
  double maxT = 0.0;
  std::vector<double> Tm((size_t)m * m);
  std::vector<double> lam_sorted(m), svec(m), evv(m), est(m);   // theta, t_{m+1,i}, ev, res_est
  double tol_scale = 0.0;   // running max |theta| for tol_relative
  std::vector<char> conv(nev);
  std::vector<double> resv(nev);
  int k = 0;
  int trace_n = 0;
  const double sqrt2 = std::sqrt(2.0);
  jl_status status = JL_NOT_CONVERGED;
  int icnv = 0;
  int64_t n_locked = 0;   // Ritz vectors copied rather than formed by the GEMM
  std::vector<int> out_order;

  // Invert mode: u = A^-1 b by CG on the device, then t_jj = b^H u into
  // scal[0..1] (where the normal mode's apply leaves it).
  int cg_prev = 0;   // iterations of the previous solve: queued before the first look
  auto cg_solve = [&](const cplx<S>* b, cplx<S>* u) -> jl_status {
    cplx<S>* const x = cgv[0];
    cplx<S>* const r = cgv[1];
    cplx<S>* const q = cgv[2];
    cplx<S>* const pb[2] = {cgv[3], cgv[4]};   // iteration c reads pb[c % 2], writes the other
    tm.start(Timer::CG);
    JL_HIP(ctx, launch_cg_init<S>(b, x, r, pb[0], n, cg_part, cgs, cg_tol, cg_maxit, st));
    int issued = 0;
    // batches are multiples of kCgChunk (even), so iteration c of a batch
    // has the parity of its global index
    int batch = std::max(kCgChunk, cg_prev - cg_prev % kCgChunk);
    for (;;) {
      for (int c = 0; c < batch; ++c) {
        cplx<S>* const pold = pb[c & 1];
        cplx<S>* const pnew = pb[(c + 1) & 1];
        JL_HIP(ctx, op_apply_cg<S>(op, cgs + CG_DONE, r, pold, cgs + CG_BETA, pnew, q, apart, st));
        JL_HIP(ctx, launch_cg_step<S>(x, r, pnew, q, n, apart, napply, cg_part, cgs, st));
      }
      issued += batch;
      JL_HIP(ctx, hipMemcpyAsync(h_cg, cgs, sizeof(double) * CG_NSLOTS, hipMemcpyDeviceToHost, st));
      JL_HIP(ctx, hipStreamSynchronize(st));
      if (h_cg[CG_DONE] != 0.0) break;
      if (issued > cg_maxit + kCgChunk)   // the stop test fires at cg_maxit at the latest
        return set_err(ctx, JL_EHIP, "CG did not report its stop after %d iterations", issued);
      batch = kCgChunk;
    }
    if (h_cg[CG_DONE] == 2.0)
      return set_err(ctx, JL_EINVAL,
                     "invert mode: CG met p^H A p <= 0 (the operator is not positive definite)");
    const int it = (int)h_cg[CG_ITERS];
    S_.cg_iters += it;
    S_.cg_max_iters = std::max(S_.cg_max_iters, it);
    if (!(h_cg[CG_RR] <= h_cg[CG_THR])) S_.cg_unconverged++;
    S_.n_matvec_launch += it;
    S_.bytes_matvec += it * op_bytes(op, es);
    S_.bytes_cg += it * (op_bytes(op, es) + 8.0 * (double)n * es);
    cg_prev = it;
    JL_HIP(ctx, launch_cg_finish<S>(x, u, b, n, cg_part, st));
    JL_HIP(ctx, launch_reduce_cols(cg_part, ncgb, 2, 2, scal, st));
    tm.stop();
    return JL_OK;
  };

  for (int cycle = 0; cycle < max_cycles; ++cycle) {
    S_.cycles++;
    cplx<S>* V = Vb[cur];
    cplx<S>* Vn = Vb[1 - cur];
    int meff = m;
    bool broke = false;
    // Normal mode queues the whole next step (its normalisation, factor read
    // on the device; the operator apply; the local step, with beta read on the
    // device; the inner products, the update and the copy of its scalars)
    // before it waits for this step's scalars, so the device always has a
    // step of work queued over the host's round trip.  A step that needs
    // another Gram-Schmidt pass (or breaks down) discards the queued step,
    // which is then queued again.
    bool queued = false;   // step j's work (apply, reorthogonalisation, scalar copy) is queued
    auto queue_apply = [&](const cplx<S>* x, cplx<S>* y) -> hipError_t {
      tm.start(Timer::MATVEC);
      hipError_t e = op_apply<S>(op, x, y, ldv, 1, apart, st);
      tm.stop();
      if (e == hipSuccess) e = launch_reduce_cols(apart, napply, 2, 2, scal, st);
      S_.n_matvec_launch++;
      S_.bytes_matvec += op_bytes(op, es);
      tm.count(Timer::MATVEC, op_bytes(op, es));
      return e;
    };
    // Step jj: [u = A v_jj, t_jj partials to scal[0..1]], local three-term
    // step u -= t_jj v_jj + beta_{jj-1} v_{jj-1} fused into the first inner
    // products against [V_jj, W_jj] (beta from the host, or with beta2 from
    // the device norm^2), the first update pass, and the copy of scal[0..4]
    // to the step's pinned slot, recorded by its event.
    auto queue_step = [&](int jj, bool with_apply, const double* beta2) -> jl_status {
      cplx<S>* vjj = V + (int64_t)jj * ldv;
      cplx<S>* uu = V + (int64_t)(jj + 1) * ldv;
      const int nc = jj + 1;
      const int sd = dots_stride(nc);
      tm.sample = n_queued++ % tm.stride == 0;   // this step's events
      if (with_apply) JL_HIP(ctx, queue_apply(vjj, uu));
      const double beta_host = (!beta2 && jj > k) ? Tat(jj, jj - 1) : 0.0;
      tm.start(Timer::DOTS);
      JL_HIP(ctx, launch_reorth_dots<S>(V, ldv, nc, uu, h, dots_part, ndots, st, scal, beta_host, jj,
                                        uloc, gd, beta2));
      tm.stop();
      // the norms entering the loop (the last two reduced columns: after the
      // local step, after t_jj v_jj alone) also to scal[3], scal[4]
      JL_HIP(ctx, launch_reduce_wide(dots_part, ndots, sd, sd, coef, wide_scr, wide_cnt, st, scal + 3));
      S_.n_dots_launch++;
      S_.bytes_dots += (double)(nc + 1) * n * es;
      tm.count(Timer::DOTS, (double)(nc + 1) * n * es);
      tm.start(Timer::UPDATE);
      JL_HIP(ctx, launch_reorth_update<S>(V, ldv, nc, uu, h, coef, upd_part, nupd, st, jsym,
                                          uloc ? uloc : uu, gu, dscr, scal + 2, upd_cnt));
      tm.stop();
      S_.n_update_launch++;
      S_.bytes_update += (double)(nc + 2) * n * es;
      tm.count(Timer::UPDATE, (double)(nc + 2) * n * es);
      JL_HIP(ctx, hipMemcpyAsync(hslot[jj & 1], scal, 5 * sizeof(double), hipMemcpyDeviceToHost, st));
      JL_HIP(ctx, hipEventRecord(ev_copy[jj & 1].e, st));
      return JL_OK;
    };
    // ================= Algorithm 2: Lanczos steps j = k .. m-1
    for (int j = k; j < m; ++j) {
      cplx<S>* u = V + (int64_t)(j + 1) * ldv;
      const int ncol = j + 1;
      const int stride = dots_stride(ncol);
      if (invert) {   // u = A^-1 v_j by CG, t_jj = v_j^H u into scal
        const jl_status cs = cg_solve(V + (int64_t)j * ldv, u);
        if (cs != JL_OK) return cs;
        const jl_status qs = queue_step(j, false, nullptr);
        if (qs != JL_OK) return qs;
      } else if (!queued) {
        const jl_status qs = queue_step(j, true, nullptr);
        if (qs != JL_OK) return qs;
      }
      queued = false;
      S_.n_mv++;
      S_.sum_ncol += ncol;
      double* hs = hslot[j & 1];
      // speculative: the whole of step j + 1 on v_{j+1} = u / ||u||, behind
      // this step's scalar copy
      const bool spec = !invert && j + 1 < m;
      if (spec) {
        JL_HIP(ctx, launch_scale_dev<S>(u, n, scal + 2, st));
        const jl_status qs = queue_step(j + 1, true, scal + 2);   // beta_j = ||u|| on the device
        if (qs != JL_OK) return qs;
      }
      JL_HIP(ctx, hipEventSynchronize(ev_copy[j & 1].e));
      tm.resolve();
      const double alpha = hs[0];
      Tat(j, j) = alpha;
      maxT = std::max(maxT, std::fabs(alpha));
      // norm entering the Gram-Schmidt loop: after the local three-term step,
      // or (b0_rule 1) after subtracting t_jj v_j alone, as Alg. 2 prints it
      double b0 = std::sqrt(prm->b0_rule == 1 ? hs[4] : hs[3]);
      double b1 = std::sqrt(hs[2]);
      // u on the device holds (u / usc): usc = b1 after the speculative scaling
      const double usc = spec ? b1 : 1.0;
      const double btol = bd_factor * uround * std::max(maxT, 1e-300);
      int passes = 1;
      S_.gs_passes++;
      bool drained = false;   // the speculative step has run out (its results are discarded)
      while (!(passes >= min_passes && b1 * sqrt2 > b0) && b1 > btol && passes < max_passes) {
        if (!drained) {
          JL_HIP(ctx, hipStreamSynchronize(st));
          tm.resolve();
          drained = true;
        }
        b0 = b1;
        tm.start(Timer::DOTS);
        JL_HIP(ctx, launch_reorth_dots<S>(V, ldv, ncol, u, h, dots_part, ndots, st, nullptr, 0.0, 0,
                                          nullptr, gd));
        tm.stop();
        JL_HIP(ctx, launch_reduce_wide(dots_part, ndots, stride, stride, coef, wide_scr, wide_cnt, st));
        S_.n_dots_launch++;
        S_.bytes_dots += (double)(ncol + 1) * n * es;
        tm.count(Timer::DOTS, (double)(ncol + 1) * n * es);
        tm.start(Timer::UPDATE);
        JL_HIP(ctx, launch_reorth_update<S>(V, ldv, ncol, u, h, coef, upd_part, nupd, st, jsym,
                                            u, gu, dscr, scal + 2, upd_cnt));
        tm.stop();
        S_.n_update_launch++;
        S_.bytes_update += (double)(ncol + 2) * n * es;
        tm.count(Timer::UPDATE, (double)(ncol + 2) * n * es);
        JL_HIP(ctx, hipMemcpyAsync(hs + 2, scal + 2, sizeof(double), hipMemcpyDeviceToHost, st));
        JL_HIP(ctx, hipStreamSynchronize(st));
        tm.resolve();
        b1 = usc * std::sqrt(hs[2]);   // Gram-Schmidt is linear: back to the units of u
        passes++;
        S_.gs_passes++;
      }
      if (trace_n < prm->trace_cap) {
        prm->trace_ab[trace_n] = alpha;
        prm->trace_ab[prm->trace_cap + trace_n] = b1;
        trace_n++;
      }
      if (!std::isfinite(b1) || !std::isfinite(alpha))
        return set_err(ctx, JL_EHIP, "non-finite Lanczos coefficient at step %d", j);
      if (b1 <= btol) {   // invariant subspace: the cycle ends at dimension j+1
        Tat(j + 1, j) = 0.0;
        meff = j + 1;
        broke = true;
        break;
      }
      if (spec && passes == 1) {
        queued = true;   // the queued step j + 1 stands
      } else {
        JL_HIP(ctx, launch_scale<S>(u, n, usc / b1, st));
      }
      Tat(j + 1, j) = b1;
      maxT = std::max(maxT, b1);
    }
    if (meff < nev) {
      status = JL_BREAKDOWN;
      icnv = 0;
      out_order.clear();
      for (int i = 0; i < nev; ++i) {
        evals[i] = NAN;
        res_out[i] = INFINITY;
      }
      break;
    }
    if (prm->basis_cycle == cycle + 1) {   // export the decomposition of this iteration
      if (prm->basis_out)
        JL_HIP(ctx, launch_copy_cols<S>(V, ldv, static_cast<cplx<S>*>(prm->basis_out), n, n,
                                        broke ? meff : meff + 1, st));
      if (prm->T_out) std::copy(T.begin(), T.end(), prm->T_out);
    }
    // ================= Rayleigh-Ritz: T_m = Z Lambda Z^T, sort (Alg. 1)
    const int kcols = std::min(kmax, meff);
    // Ritz vectors [c0, c1) of V_m Z (real GEMM on the interleaved basis).  A
    // column of Z that is exactly a unit vector e_i (a converged pair locked by
    // its zero coupling, deflated exactly by the Ritz step) gives v_i itself:
    // it is copied (the product would produce the same bits).  The other
    // columns go through the GEMM, gathered when some are left out.
    auto basis_gemm = [&](int c0, int c1) -> jl_status {
      if (c1 <= c0) return JL_OK;
      int ng = 0, np = 0;
      int* pairs = h_gmap + m;
      for (int c = c0; c < c1; ++c) {
        const double* z = h_Z + (size_t)c * meff;
        int src = -1;
        for (int i = 0; i < meff && src != -2; ++i)
          if (z[i] != 0.0) src = (src == -1 && z[i] == 1.0) ? i : -2;
        if (src >= 0) {
          pairs[2 * np] = c;
          pairs[2 * np + 1] = src;
          ++np;
        } else {
          h_gmap[ng++] = c;
        }
      }
      tm.start(Timer::GEMM);
      if (ng == c1 - c0) {   // no locked column: the contiguous product
        JL_HIP(ctx, (launch_gemm_nn<S, double>)(reinterpret_cast<const S*>(V), 2 * ldv,
                                              Zs + (size_t)c0 * meff, meff, reinterpret_cast<S*>(Vn + (int64_t)c0 * ldv),
                                              2 * ldv, 2 * n, ng, meff, st));
      } else {
        const int goff = c0;   // the two calls of a cycle use disjoint parts of the scratch
        double* hz = h_Zg + (size_t)goff * meff;
        for (int j = 0; j < ng; ++j)
          std::copy(h_Z + (size_t)h_gmap[j] * meff, h_Z + (size_t)(h_gmap[j] + 1) * meff,
                    hz + (size_t)j * meff);
        if (ng > 0) {
          JL_HIP(ctx, hipMemcpyAsync(Zg + (size_t)goff * meff, hz, sizeof(double) * (size_t)ng * meff,
                                     hipMemcpyHostToDevice, st));
          JL_HIP(ctx, hipMemcpyAsync(gmap + goff, h_gmap, sizeof(int) * ng, hipMemcpyHostToDevice, st));
          JL_HIP(ctx, (launch_gemm_nn<S, double>)(reinterpret_cast<const S*>(V), 2 * ldv,
                                                Zg + (size_t)goff * meff, meff, reinterpret_cast<S*>(Vn),
                                                2 * ldv, 2 * n, ng, meff, st, gmap + goff));
        }
        JL_HIP(ctx, hipMemcpyAsync(gmap + m + 2 * goff, pairs, sizeof(int) * 2 * np,
                                   hipMemcpyHostToDevice, st));
        JL_HIP(ctx, launch_copy_pairs<S>(V, ldv, Vn, ldv, n, gmap + m + 2 * goff, np, st));
      }
      tm.stop();
      S_.n_gemm_launch++;
      S_.flops_gemm += 2.0 * (double)(2 * n) * ng * meff;
      n_locked += np;
      return JL_OK;
    };
    // the nev candidates of the convergence check first (rounded up to the
    // GEMM's column tile); the rest of the kept vectors once icnv is known
    const int kfirst = std::min(kcols, (nev + kGemmTileN - 1) / kGemmTileN * kGemmTileN);
    tm.start(Timer::RITZ);
    if (meff <= dc_max_m()) {
      // restart structure: kept Ritz values and couplings, then this cycle's
      // tridiagonal (divide and conquer)
      for (int i = 0; i < k; ++i) {
        Tm[i] = Tat(i, i);
        Tm[k + i] = Tat(k, i);
      }
      for (int j = k; j < meff; ++j) Tm[2 * k + (j - k)] = Tat(j, j);
      for (int j = k; j + 1 < meff; ++j) Tm[2 * k + (meff - k) + (j - k)] = Tat(j + 1, j);
      JL_HIP(ctx, ritz_arrow_device<S>(meff, k, Tm.data(), descending, 0, ritz_scr, lam_s,
                                       Zs, nullptr, zlast, st));
    } else {
      for (int jj = 0; jj < meff; ++jj)
        for (int ii = 0; ii < meff; ++ii) {
          const double v = ii >= jj ? Tat(ii, jj) : Tat(jj, ii);
          Tm[(size_t)ii + (size_t)jj * meff] = v;
        }
      double fro2 = 0.0;
      for (int i = 0; i < meff * meff; ++i) fro2 += Tm[i] * Tm[i];
      JL_HIP(ctx, hipMemcpyAsync(Tdev, Tm.data(), sizeof(double) * (size_t)meff * meff,
                                 hipMemcpyHostToDevice, st));
      JL_HIP(ctx, ritz_device<S>(meff, Tdev, fro2, descending, 0, ritz_scr, lam_s, Zs,
                                 nullptr, zlast, hs, st));
    }
    JL_HIP(ctx, hipMemcpyAsync(h_lam, lam_s, sizeof(double) * meff, hipMemcpyDeviceToHost, st));
    JL_HIP(ctx, hipMemcpyAsync(h_zl, zlast, sizeof(double) * meff, hipMemcpyDeviceToHost, st));
    tm.stop();
    // the kept columns of Z, to find the locked ones before the basis update
    JL_HIP(ctx, hipMemcpyAsync(h_Z, Zs, sizeof(double) * (size_t)meff * kcols, hipMemcpyDeviceToHost, st));
    JL_HIP(ctx, hipStreamSynchronize(st));
    // ================= V_k := V_m Z[:, 0:k] (Alg. 1), candidates first
    {
      const jl_status gs = basis_gemm(0, kfirst);
      if (gs != JL_OK) return gs;
    }
    JL_HIP(ctx, hipStreamSynchronize(st));
    tm.resolve();
    const double beta_m = Tat(meff, meff - 1);
    for (int i = 0; i < meff; ++i) {
      lam_sorted[i] = h_lam[i];
      svec[i] = beta_m * h_zl[i];   // t_{m+1,i} = t_{m+1,m} z_{m,i}
    }
    // ================= estimated residuals (Alg. 1): |t_{m+1,i}|, or in
    // invert mode c |t_{m+1,i} ev_i| with ev_i = 1/theta_i, c = ||A v_{m+1}||
    if (invert) {
      double c = 0.0;
      if (!broke) {   // after a breakdown there is no v_{m+1} (the couplings are zero)
        tm.start(Timer::RESID);
        JL_HIP(ctx, op_apply<S>(op, V + (int64_t)meff * ldv, cgv[2], ldv, 1, nullptr, st));
        JL_HIP(ctx, launch_norm2<S>(cgv[2], n, cg_part, st));
        JL_HIP(ctx, launch_reduce_cols(cg_part, ncgb, 1, 1, scal + 5, st));
        JL_HIP(ctx, hipMemcpyAsync(hs + 5, scal + 5, sizeof(double), hipMemcpyDeviceToHost, st));
        tm.stop();
        JL_HIP(ctx, hipStreamSynchronize(st));
        tm.resolve();
        S_.n_resid++;
        c = std::sqrt(hs[5]);
      }
      tol_scale = std::max(tol_scale, c);
      for (int i = 0; i < meff; ++i) {
        evv[i] = 1.0 / lam_sorted[i];
        est[i] = c * std::fabs(svec[i] * evv[i]);
      }
      for (int i = 0; i < nev; ++i) tol_scale = std::max(tol_scale, std::fabs(evv[i]));
    } else {
      for (int i = 0; i < meff; ++i) {
        evv[i] = lam_sorted[i];
        est[i] = std::fabs(svec[i]);
      }
      tol_scale = std::max(tol_scale, std::max(std::fabs(lam_sorted[0]), std::fabs(lam_sorted[meff - 1])));
    }
    // ================= convergence check on the true residuals (Alg. 1)
    const double tol_abs = prm->tol_relative ? prm->tol * tol_scale : prm->tol;
    int ncand = 0;
    for (int i = 0; i < nev; ++i) {
      conv[i] = 0;
      resv[i] = INFINITY;
      if (est[i] < tol_abs) {
        h_rcols[ncand] = i;
        h_rlam[ncand] = evv[i];
        ncand++;
      }
    }
    if (ncand > 0) {
      tm.start(Timer::RESID);
      JL_HIP(ctx, hipMemcpyAsync(res_cols, h_rcols, sizeof(int) * ncand, hipMemcpyHostToDevice, st));
      JL_HIP(ctx, hipMemcpyAsync(res_lam, h_rlam, sizeof(double) * ncand, hipMemcpyHostToDevice, st));
      int nrb = 0;
      JL_HIP(ctx, op_resid<S>(op, Vn, ldv, res_cols, h_rcols, res_lam, ncand, res_part, &nrb, st));
      JL_HIP(ctx, launch_reduce_wide(res_part, nrb, ncand, ncand, res_dev, wide_scr, wide_cnt, st));
      JL_HIP(ctx, hipMemcpyAsync(h_res, res_dev, sizeof(double) * ncand, hipMemcpyDeviceToHost, st));
      tm.stop();
      JL_HIP(ctx, hipStreamSynchronize(st));
      tm.resolve();
      S_.n_resid += ncand;
      for (int c = 0; c < ncand; ++c) {
        const int i = h_rcols[c];
        resv[i] = std::sqrt(h_res[c]);
        conv[i] = resv[i] < tol_abs;
      }
    }
    icnv = 0;
    out_order.clear();
    for (int i = 0; i < nev; ++i)
      if (conv[i]) out_order.push_back(i), icnv++;
    for (int i = 0; i < nev; ++i)
      if (!conv[i]) out_order.push_back(i);
    if (prm->verbose) {
      double worst = 0.0;
      for (int i = 0; i < nev; ++i) worst = std::max(worst, est[i]);
      fprintf(stderr, "[jlanczos] cycle %d k %d m %d icnv %d/%d max res_est %.2e n_mv %d locked %lld t %.2fs\n",
              cycle + 1, k, meff, icnv, nev, worst, S_.n_mv, (long long)n_locked,
              std::chrono::duration<double>(std::chrono::steady_clock::now() - t_begin).count());
      fflush(stderr);
    }
    if (prm->cycle_times && cycle < prm->cycle_times_cap)   // the device is idle here
      prm->cycle_times[cycle] =
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t_begin).count();
    const bool last = (cycle + 1 == max_cycles);
    if (icnv == nev || broke || last) {
      status = icnv == nev ? JL_OK : (broke ? JL_BREAKDOWN : JL_NOT_CONVERGED);
      cur = 1 - cur;   // the Ritz vectors live in Vn
      break;
    }
    // ================= shrink to k + 1 (eq. dynamicwin) and continue
    k = std::min(icnv + mwin, m - 1);
    {
      const jl_status gs = basis_gemm(kfirst, k);   // the kept vectors past the candidates
      if (gs != JL_OK) return gs;
    }
    std::fill(T.begin(), T.end(), 0.0);
    maxT = 0.0;
    for (int i = 0; i < k; ++i) {
      Tat(i, i) = lam_sorted[i];
      const double si = (i < nev && conv[i]) ? 0.0 : svec[i];   // decouple converged
      Tat(k, i) = si;
      maxT = std::max(maxT, std::max(std::fabs(lam_sorted[i]), std::fabs(si)));
    }
    JL_HIP(ctx, launch_copy_cols<S>(V + (int64_t)meff * ldv, ldv, Vn + (int64_t)k * ldv, ldv, n, 1,
                                    st));
    cur = 1 - cur;
  }

  // ---- outputs: converged pairs first, desired order otherwise
  if (!out_order.empty()) {
    cplx<S>* Vf = Vb[cur];
    cplx<S>* X = static_cast<cplx<S>*>(Xout);
    for (int c = 0; c < nev; ++c) {
      const int i = out_order[c];
      evals[c] = evv[i];
      res_out[c] = resv[i];
      JL_HIP(ctx, launch_copy_cols<S>(Vf + (int64_t)i * ldv, ldv, X + (int64_t)c * ldx, ldx, n, 1,
                                      st));
    }
  }
  JL_HIP(ctx, hipStreamSynchronize(st));
  tm.resolve();
  S_.icnv = icnv;
  S_.status = status;
  if (tm.on && tm.stride > 1) {   // the per-step classes report their timed launches only
    S_.n_matvec_launch = tm.tcnt[Timer::MATVEC];
    S_.bytes_matvec = tm.tbytes[Timer::MATVEC];
    S_.n_dots_launch = tm.tcnt[Timer::DOTS];
    S_.bytes_dots = tm.tbytes[Timer::DOTS];
    S_.n_update_launch = tm.tcnt[Timer::UPDATE];
    S_.bytes_update = tm.tbytes[Timer::UPDATE];
  }
  S_.t_matvec = tm.t[Timer::MATVEC];
  S_.t_dots = tm.t[Timer::DOTS];
  S_.t_update = tm.t[Timer::UPDATE];
  S_.t_gemm = tm.t[Timer::GEMM];
  S_.t_ritz = tm.t[Timer::RITZ];
  S_.t_resid = tm.t[Timer::RESID];
  S_.t_cg = tm.t[Timer::CG];
  S_.t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_begin).count();
  if (stats) *stats = S_;
  return status;
}

}  // namespace

namespace {

// Memory of the TEK operator: [U 4 | X 4 | H 16 | T 16 | FB 16] matrices of
// Np x Np, the diagonal scratch, the projection tables, the product jobs.
template <typename S>
TekArgs<S> tek_layout(char* base, int N, int Np, double kappa, size_t* total) {
  const size_t M = (size_t)Np * Np * sizeof(cplx<S>);
  TekArgs<S> a{};
  a.N = N;
  a.Np = Np;
  a.na = (int64_t)N * N - 1;
  a.kappa = kappa;
  a.X = reinterpret_cast<cplx<S>*>(base + 4 * M);
  a.H = reinterpret_cast<cplx<S>*>(base + 8 * M);
  a.FB = reinterpret_cast<cplx<S>*>(base + 40 * M);
  a.zd = reinterpret_cast<double*>(base + 56 * M);
  const size_t proj_off = 56 * M + ((8 * (size_t)N * sizeof(double) + 255) & ~size_t(255));
  a.proj = reinterpret_cast<const double*>(base + proj_off);
  const size_t jobs_off = proj_off + 256 * sizeof(double);
  a.jobs1 = reinterpret_cast<const ZJob<S>*>(base + jobs_off);
  a.jobs2 = a.jobs1 + 16;
  *total = jobs_off + 32 * sizeof(ZJob<S>);
  return a;
}

// Host copies of the 32 product jobs (pointers into the device block):
// T = U h (q < 2) or U^H h (q >= 2), then FB = T U^H or T U.
template <typename S>
std::vector<ZJob<S>> tek_jobs(char* base, int Np) {
  const size_t M = (size_t)Np * Np;
  cplx<S>* U = reinterpret_cast<cplx<S>*>(base);
  cplx<S>* H = U + 8 * M;
  cplx<S>* T = U + 24 * M;
  cplx<S>* FB = U + 40 * M;
  std::vector<ZJob<S>> j(32);
  for (int mu = 0; mu < 4; ++mu)
    for (int q = 0; q < 4; ++q) {
      const int i = mu * 4 + q;
      const int dag = q >= 2 ? 1 : 0;
      j[i] = ZJob<S>{U + mu * M, H + i * M, T + i * M, dag, 0};
      j[16 + i] = ZJob<S>{T + i * M, U + mu * M, FB + i * M, 0, 1 - dag};
    }
  return j;
}

// Rank-2 factorisations I + s gamma_mu = A B (s = -1, +1; gamma_mu of the
// appendix), laid out as TekArgs::proj expects.  Returns false if a check of
// A B against I + s gamma_mu fails.
bool tek_projections(double* out) {
  using Z = std::complex<double>;
  const Z i1(0.0, 1.0);
  Z g[4][4][4] = {};
  g[0][0][3] = -i1; g[0][1][2] = -i1; g[0][2][1] = i1; g[0][3][0] = i1;
  g[1][0][3] = -1.0; g[1][1][2] = 1.0; g[1][2][1] = 1.0; g[1][3][0] = -1.0;
  g[2][0][2] = -i1; g[2][1][3] = i1; g[2][2][0] = i1; g[2][3][1] = -i1;
  g[3][0][0] = 1.0; g[3][1][1] = 1.0; g[3][2][2] = -1.0; g[3][3][3] = -1.0;
  for (int sg = 0; sg < 2; ++sg)
    for (int mu = 0; mu < 4; ++mu) {
      Z P[4][4];
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) P[r][c] = (r == c ? 1.0 : 0.0) + (sg ? 1.0 : -1.0) * g[mu][r][c];
      auto nrm = [&](int r) { double t = 0; for (int c = 0; c < 4; ++c) t += std::norm(P[r][c]); return t; };
      auto lead = [&](const Z* row) { int j = 0; for (int c = 1; c < 4; ++c) if (std::abs(row[c]) > std::abs(row[j])) j = c; return j; };
      auto ratio = [&](int r, const Z* brow, Z* c) {   // P[r] = c brow ?
        const int j = lead(brow);
        *c = P[r][j] / brow[j];
        double d = 0;
        for (int q = 0; q < 4; ++q) d += std::norm(P[r][q] - *c * brow[q]);
        return d < 1e-24;
      };
      Z B[2][4], A[4][2] = {};
      int nb = 0;
      for (int r = 0; r < 4 && nb < 2; ++r) {
        if (nrm(r) < 1e-24) continue;
        Z c;
        if (nb == 1 && ratio(r, B[0], &c)) continue;
        for (int q = 0; q < 4; ++q) B[nb][q] = P[r][q];
        ++nb;
      }
      if (nb != 2) return false;
      for (int r = 0; r < 4; ++r) {
        if (nrm(r) < 1e-24) continue;
        Z c;
        if (ratio(r, B[0], &c)) A[r][0] = c;
        else if (ratio(r, B[1], &c)) A[r][1] = c;
        else return false;
      }
      for (int r = 0; r < 4; ++r)   // check A B = P
        for (int q = 0; q < 4; ++q)
          if (std::abs(A[r][0] * B[0][q] + A[r][1] * B[1][q] - P[r][q]) > 1e-12) return false;
      for (int k = 0; k < 2; ++k)
        for (int b = 0; b < 4; ++b) {
          const int i = ((sg * 4 + mu) * 2 + k) * 4 + b;
          out[2 * i] = B[k][b].real();
          out[2 * i + 1] = B[k][b].imag();
        }
      for (int al = 0; al < 4; ++al)
        for (int k = 0; k < 2; ++k) {
          const int i = 64 + ((sg * 4 + mu) * 4 + al) * 2 + k;
          out[2 * i] = A[al][k].real();
          out[2 * i + 1] = A[al][k].imag();
        }
    }
  return true;
}

}  // namespace

// =============================================================== C ABI
extern "C" {

const char* jl_status_string(jl_status s) {
  switch (s) {
    case JL_OK: return "ok";
    case JL_EINVAL: return "invalid argument";
    case JL_EHIP: return "HIP runtime error";
    case JL_ENOMEM: return "workspace too small";
    case JL_EUNSUPPORTED: return "unsupported";
    case JL_NOT_CONVERGED: return "not converged";
    case JL_BREAKDOWN: return "breakdown (invariant subspace)";
    default: return "unknown status";
  }
}

const char* jl_last_error(jl_ctx ctx) { return ctx ? ctx->err.c_str() : g_thread_err.c_str(); }

jl_status jl_ctx_create(jl_ctx* out, int32_t device, void* hip_stream) {
  if (!out) return set_err(nullptr, JL_EINVAL, "out is NULL");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess)
    return set_err(nullptr, JL_EHIP, "hipGetDeviceCount failed: %s", hipGetErrorString(e));
  if (device < 0 || device >= ndev)
    return set_err(nullptr, JL_EINVAL, "device %d out of range (%d devices)", device, ndev);
  jl_ctx c = new jl_ctx_s();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  {   // the allocation-free entry points' scratch on this device (with it current)
    DeviceGuard g(device);
    const hipError_t se = noalloc_scratch_address(device, &c->na_scratch);
    if (se != hipSuccess) {
      c->na_scratch = nullptr;
      c->na_err = std::string("hipGetSymbolAddress of the static scratch: ") + hipGetErrorString(se);
    }
  }
  *out = c;
  return JL_OK;
}

jl_status jl_ctx_destroy(jl_ctx ctx) {
  delete ctx;
  return JL_OK;
}

jl_status jl_op_create_dense(jl_ctx ctx, int64_t n, const void* A11, const void* A12, int64_t ld,
                             jl_dtype dtype, jl_op* out) {
  if (!ctx || !out) return set_err(ctx, JL_EINVAL, "ctx and out are required");
  if (n <= 0 || n % 2) return set_err(ctx, JL_EINVAL, "n must be positive and even (got %lld)", (long long)n);
  if (ld < n / 2) return set_err(ctx, JL_EINVAL, "ld (%lld) < n/2", (long long)ld);
  if (!A11 || !A12) return set_err(ctx, JL_EINVAL, "A11 and A12 are required");
  if (dtype != JL_C64 && dtype != JL_C128) return set_err(ctx, JL_EINVAL, "dtype must be JL_C64 or JL_C128");
  jl_op o = new jl_op_s();
  o->ctx = ctx;
  o->kind = OP_DENSE;
  o->dtype = dtype;
  o->n = n;
  o->df = DenseArgs<float>{static_cast<const float2*>(A11), static_cast<const float2*>(A12), n / 2, ld};
  o->dd = DenseArgs<double>{static_cast<const double2*>(A11), static_cast<const double2*>(A12), n / 2, ld};
  *out = o;
  return JL_OK;
}

jl_status jl_op_create_stencil(jl_ctx ctx, const int32_t L[4], int32_t d, double diag,
                               double a12_scale, const void* U, const void* B, int32_t b_per_site,
                               jl_dtype dtype, jl_op* out) {
  if (!ctx || !out || !L) return set_err(ctx, JL_EINVAL, "ctx, L and out are required");
  if (d != 4) return set_err(ctx, JL_EUNSUPPORTED, "only internal dimension d = 4 is implemented (got %d)", d);
  for (int i = 0; i < 4; ++i)
    if (L[i] < 2) return set_err(ctx, JL_EINVAL, "L[%d] = %d must be >= 2", i, L[i]);
  if (!U || !B) return set_err(ctx, JL_EINVAL, "U and B are required");
  if (dtype != JL_C64 && dtype != JL_C128) return set_err(ctx, JL_EINVAL, "dtype must be JL_C64 or JL_C128");
  const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
  if (V >= ((int64_t)1 << 31))
    return set_err(ctx, JL_EINVAL, "the lattice must have fewer than 2^31 sites (got %lld)", (long long)V);
  const size_t es = dtype == JL_C64 ? sizeof(float2) : sizeof(double2);
  const size_t ubytes = (size_t)link_elems(V) * es;   // tiles of 64 sites (link_index)
  const size_t bbytes = b_per_site ? ubytes : 64 * es;
  DeviceGuard g(ctx->device);
  void* links = nullptr;
  hipError_t e = hipMalloc(&links, ubytes + bbytes);
  if (e != hipSuccess) {
    return set_err(ctx, JL_ENOMEM, "stencil link copy (%zu bytes): %s", ubytes + bbytes,
                   hipGetErrorString(e));
  }
  char* ub = static_cast<char*>(links);
  char* bb = ub + ubytes;
  if (dtype == JL_C64) {
    e = launch_links_tiled<float>(static_cast<const float2*>(U), reinterpret_cast<float2*>(ub), V,
                                         ctx->stream);
    if (e == hipSuccess)
      e = b_per_site ? launch_links_tiled<float>(static_cast<const float2*>(B),
                                                        reinterpret_cast<float2*>(bb), V, ctx->stream)
                     : hipMemcpyAsync(bb, B, bbytes, hipMemcpyDeviceToDevice, ctx->stream);
  } else {
    e = launch_links_tiled<double>(static_cast<const double2*>(U), reinterpret_cast<double2*>(ub),
                                          V, ctx->stream);
    if (e == hipSuccess)
      e = b_per_site ? launch_links_tiled<double>(static_cast<const double2*>(B),
                                                         reinterpret_cast<double2*>(bb), V, ctx->stream)
                     : hipMemcpyAsync(bb, B, bbytes, hipMemcpyDeviceToDevice, ctx->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    (void)hipFree(links);
    return set_err(ctx, JL_EHIP, "stencil link copy: %s", hipGetErrorString(e));
  }
  jl_op o = new jl_op_s();
  o->ctx = ctx;
  o->kind = OP_STENCIL;
  o->dtype = dtype;
  o->n = 2 * V * 4;
  o->links = links;
  StencilArgs<float> sf{};
  StencilArgs<double> sd{};
  for (int i = 0; i < 4; ++i) sf.L[i] = sd.L[i] = L[i];
  sf.V = sd.V = V;
  sf.b_per_site = sd.b_per_site = b_per_site ? 1 : 0;
  sf.diag = sd.diag = diag;
  sf.scale = sd.scale = a12_scale;
  sf.U = reinterpret_cast<const float2*>(ub);
  sf.B = reinterpret_cast<const float2*>(bb);
  sd.U = reinterpret_cast<const double2*>(ub);
  sd.B = reinterpret_cast<const double2*>(bb);
  o->sf = sf;
  o->sd = sd;
  *out = o;
  return JL_OK;
}

jl_status jl_op_create_tek(jl_ctx ctx, int32_t N, double kappa, const void* U, jl_dtype dtype,
                           jl_op* out) {
  if (!ctx || !out) return set_err(ctx, JL_EINVAL, "ctx and out are required");
  if (N < 2 || N > 1024) return set_err(ctx, JL_EINVAL, "N must be in 2..1024 (got %d)", N);
  if (!U) return set_err(ctx, JL_EINVAL, "U is required");
  if (dtype != JL_C64 && dtype != JL_C128) return set_err(ctx, JL_EINVAL, "dtype must be JL_C64 or JL_C128");
  double proj[256];
  if (!tek_projections(proj))
    return set_err(ctx, JL_EHIP, "TEK operator set-up: spin projection factorisation failed");
  const int Np = (N + 63) / 64 * 64;
  const size_t es = dtype == JL_C64 ? sizeof(float2) : sizeof(double2);
  size_t total = 0;
  if (dtype == JL_C64) (void)tek_layout<float>(nullptr, N, Np, kappa, &total);
  else (void)tek_layout<double>(nullptr, N, Np, kappa, &total);
  DeviceGuard g(ctx->device);
  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, total);
  if (e != hipSuccess)
    return set_err(ctx, JL_ENOMEM, "TEK operator memory (%zu bytes): %s", total, hipGetErrorString(e));
  char* base = static_cast<char*>(mem);
  // zero everything (the padding must stay zero), then the links into the padded rows
  e = hipMemsetAsync(mem, 0, total, ctx->stream);
  for (int mu = 0; mu < 4 && e == hipSuccess; ++mu)
    e = hipMemcpy2DAsync(base + (size_t)mu * Np * Np * es, (size_t)Np * es,
                         static_cast<const char*>(U) + (size_t)mu * N * N * es, (size_t)N * es,
                         (size_t)N * es, (size_t)N, hipMemcpyDeviceToDevice, ctx->stream);
  jl_op o = new jl_op_s();
  o->tf = tek_layout<float>(base, N, Np, kappa, &total);
  o->td = tek_layout<double>(base, N, Np, kappa, &total);
  const size_t jobs_bytes = 32 * (dtype == JL_C64 ? sizeof(ZJob<float>) : sizeof(ZJob<double>));
  const double* proj_dev = dtype == JL_C64 ? o->tf.proj : o->td.proj;
  if (e == hipSuccess)
    e = hipMemcpyAsync(const_cast<double*>(proj_dev), proj, sizeof(proj), hipMemcpyHostToDevice,
                       ctx->stream);
  std::vector<ZJob<float>> jf;
  std::vector<ZJob<double>> jd;
  const void* jobs_host = nullptr;
  if (dtype == JL_C64) {
    jf = tek_jobs<float>(base, Np);
    jobs_host = jf.data();
  } else {
    jd = tek_jobs<double>(base, Np);
    jobs_host = jd.data();
  }
  void* jobs_dev = dtype == JL_C64 ? (void*)o->tf.jobs1 : (void*)o->td.jobs1;
  if (e == hipSuccess) e = hipMemcpyAsync(jobs_dev, jobs_host, jobs_bytes, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    delete o;
    (void)hipFree(mem);
    return set_err(ctx, JL_EHIP, "TEK operator set-up: %s", hipGetErrorString(e));
  }
  o->ctx = ctx;
  o->kind = OP_TEK;
  o->dtype = dtype;
  o->n = 4 * ((int64_t)N * N - 1);
  o->links = mem;
  *out = o;
  return JL_OK;
}

jl_status jl_op_destroy(jl_op op) {
  delete op;
  return JL_OK;
}

jl_status jl_op_dim(jl_op op, int64_t* n) {
  if (!op || !n) return set_err(op ? op->ctx : nullptr, JL_EINVAL, "op and n are required");
  *n = op->n;
  return JL_OK;
}

jl_status jl_op_apply(jl_op op, const void* x, void* y, int32_t nrhs) {
  if (!op) return set_err(nullptr, JL_EINVAL, "op is NULL");
  jl_ctx ctx = op->ctx;
  if (!x || !y || nrhs < 0) return set_err(ctx, JL_EINVAL, "x, y required and nrhs >= 0");
  if (nrhs == 0) return JL_OK;
  if (op->kind == OP_STENCIL &&
      ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) % 16 != 0))
    return set_err(ctx, JL_EINVAL, "stencil vectors must be 16-byte aligned");
  DeviceGuard g(ctx->device);
  if (op->dtype == JL_C64)
    JL_HIP(ctx, op_apply<float>(op, static_cast<const float2*>(x), static_cast<float2*>(y), op->n, nrhs, nullptr, ctx->stream));
  else
    JL_HIP(ctx, op_apply<double>(op, static_cast<const double2*>(x), static_cast<double2*>(y), op->n, nrhs, nullptr, ctx->stream));
  return JL_OK;
}

jl_status jl_workspace_bytes(jl_op op, const jl_params* p, size_t* bytes) {
  if (!op || !bytes) return set_err(op ? op->ctx : nullptr, JL_EINVAL, "op and bytes are required");
  jl_status s = check_params(op->ctx, op, p);
  if (s != JL_OK) return s;
  *bytes = make_layout(op, p).total;
  return JL_OK;
}

jl_status jl_solve(jl_op op, const jl_params* p, const void* v1, void* ws, size_t ws_bytes,
                   double* evals, void* X, int64_t ldx, double* res, jl_stats* stats) {
  if (!op) return set_err(nullptr, JL_EINVAL, "op is NULL");
  jl_status s = check_params(op->ctx, op, p);
  if (s != JL_OK) return s;
  DeviceGuard g(op->ctx->device);
  if (op->dtype == JL_C64) return solve_impl<float>(op, p, v1, ws, ws_bytes, evals, X, ldx, res, stats);
  return solve_impl<double>(op, p, v1, ws, ws_bytes, evals, X, ldx, res, stats);
}

jl_status jl_pair_vectors(jl_ctx ctx, int64_t n, int32_t k, jl_dtype dtype, const void* X,
                          int64_t ldx, void* Y, int64_t ldy) {
  if (!ctx) return set_err(nullptr, JL_EINVAL, "ctx is NULL");
  if (n <= 0 || n % 2 || k < 0 || ldx < n || ldy < n || (k > 0 && (!X || !Y)))
    return set_err(ctx, JL_EINVAL, "invalid pair_vectors arguments");
  if (X == Y && ldx != ldy) return set_err(ctx, JL_EINVAL, "in-place pairing needs ldx == ldy");
  DeviceGuard g(ctx->device);
  if (dtype == JL_C64)
    JL_HIP(ctx, launch_pair<float>(static_cast<const float2*>(X), ldx, static_cast<float2*>(Y), ldy, n / 2, k, ctx->stream));
  else if (dtype == JL_C128)
    JL_HIP(ctx, launch_pair<double>(static_cast<const double2*>(X), ldx, static_cast<double2*>(Y), ldy, n / 2, k, ctx->stream));
  else
    return set_err(ctx, JL_EINVAL, "dtype must be JL_C64 or JL_C128");
  return JL_OK;
}

}  // extern "C"
