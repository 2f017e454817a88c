// C ABI of the individual iteration steps (include/jlanczos_kernels.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/jlanczos_kernels.h"
#include "internal.h"

using namespace jl;

namespace {

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// dots partials | update partials | wide-reduction slices | its tile counters
size_t reorth_ws_part(int64_t n, int ncol, int which) {
  const int64_t h = n / 2;
  const int nd = std::max(reorth_dots_blocks(h, 8), reorth_dots_blocks(h, 16)), stride = dots_stride(ncol);
  const size_t sz[4] = {
      align_up(sizeof(double) * (size_t)nd * (size_t)stride),
      align_up(sizeof(double) *
               (size_t)std::max({reorth_update_blocks(h, 8), reorth_update_blocks(h, 16), 1})),
      align_up(sizeof(double) * reduce_wide_scratch_doubles(nd, stride)),
      align_up(sizeof(unsigned) * (size_t)reduce_wide_tiles(stride))};
  size_t off = 0;
  for (int i = 0; i < which; ++i) off += sz[i];
  return off;
}
size_t reorth_ws(int64_t n, int ncol) { return reorth_ws_part(n, ncol, 4); }

// One pass with the scratch at dp (dots partials), up (update partials), scr
// (wide-reduction slices) and cnt (its tile counters, cleared here by a
// kernel, so the sequence holds no memset node when a caller captures it).
template <typename S>
hipError_t reorth_pass_on(int64_t n, int ncol, const cplx<S>* V, int64_t ldv, cplx<S>* u,
                          double* coef, double* dp, double* up, double* scr, unsigned* cnt,
                          hipStream_t st) {
  const int64_t h = n / 2;
  const int nd = reorth_dots_blocks(h, (int)sizeof(cplx<S>)),
            nu = reorth_update_blocks(h, (int)sizeof(cplx<S>));
  const int stride = dots_stride(ncol);   // coef[4 ncol + 1] is then overwritten by the norm after
  hipError_t e;
  if ((e = launch_zero_u32(cnt, reduce_wide_tiles(stride), st)) != hipSuccess) return e;
  if ((e = launch_reorth_dots<S>(V, ldv, ncol, u, h, dp, nd, st)) != hipSuccess) return e;
  if ((e = launch_reduce_wide(dp, nd, stride, stride, coef, scr, cnt, st)) != hipSuccess) return e;
  if ((e = launch_reorth_update<S>(V, ldv, ncol, u, h, coef, up, nu, st)) != hipSuccess) return e;
  return launch_reduce_cols(up, nu, 1, 1, coef + 4 * ncol + 1, st);
}

template <typename S>
hipError_t reorth_pass(int64_t n, int ncol, const cplx<S>* V, int64_t ldv, cplx<S>* u, double* coef,
                       char* ws, hipStream_t st) {
  return reorth_pass_on<S>(n, ncol, V, ldv, u, coef, reinterpret_cast<double*>(ws),
                           reinterpret_cast<double*>(ws + reorth_ws_part(n, ncol, 1)),
                           reinterpret_cast<double*>(ws + reorth_ws_part(n, ncol, 2)),
                           reinterpret_cast<unsigned*>(ws + reorth_ws_part(n, ncol, 3)), st);
}

// ---------------------------------------------------- allocation-free pass
// The scratch of jl_reorth_pass_noalloc lives in a static device array (one
// copy per GPU, held until the process ends), sized for at most
// kNaMaxCols basis columns and kNaMaxUpdBlocks update blocks: the dots
// partials of at most kNaMaxDotsBlocks blocks (short vectors take at most
// 2048 in any case; the LDS inner products of long ones take one block per
// 4096 FP32 or 2048 FP64 pairs, so n up to 16777216 in FP32, when n / 2 is
// even, and 8388608 in FP64), the update partials, the wide-reduction slices
// (at most 16) and the counters.
constexpr int kNaMaxCols = 256;
constexpr int kNaMaxDotsBlocks = 2048;
constexpr int kNaMaxUpdBlocks = 65536;
constexpr size_t na_up(size_t d) { return (d + 31) / 32 * 32; }   // 256-byte segments
constexpr size_t kNaDots = na_up((size_t)kNaMaxDotsBlocks * dots_stride(kNaMaxCols));
constexpr size_t kNaUpd = na_up(kNaMaxUpdBlocks);
constexpr size_t kNaWide = na_up((size_t)16 * dots_stride(kNaMaxCols));
constexpr size_t kNaCnt = na_up(((size_t)dots_stride(kNaMaxCols) + 63) / 64);   // unsigned fit in doubles
constexpr size_t kNaDoubles = kNaDots + kNaUpd + kNaWide + kNaCnt;   // 17.5 MB

}  // namespace

static __device__ __align__(256) double scratch[kNaDoubles];

namespace jl {

hipError_t noalloc_scratch_address(int device, void** out) {
  constexpr int kMaxDevices = 256;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *out = addr[device];
  return hipSuccess;
}

}  // namespace jl

extern "C" {

jl_status jl_reorth_pass_workspace_bytes(int64_t n, int32_t ncol, size_t* bytes) {
  if (!bytes || n <= 0 || n % 2 || ncol < 0 || ncol >= kReorthMaxCols)
    return set_err(nullptr, JL_EINVAL, "invalid reorth_pass sizes");
  *bytes = reorth_ws(n, ncol);
  return JL_OK;
}

jl_status jl_reorth_pass(jl_ctx ctx, jl_dtype dtype, int64_t n, int32_t ncol, const void* V,
                         int64_t ldv, void* u, double* coef, void* ws, size_t ws_bytes) {
  if (!ctx) return set_err(nullptr, JL_EINVAL, "ctx is NULL");
  if (n <= 0 || n % 2 || ncol < 0 || ncol >= kReorthMaxCols || ldv < n || !u || !coef ||
      (ncol > 0 && !V))
    return set_err(ctx, JL_EINVAL, "invalid reorth_pass arguments");
  if (!ws || ws_bytes < reorth_ws(n, ncol))
    return set_err(ctx, JL_ENOMEM, "workspace too small (%zu < %zu)", ws_bytes, reorth_ws(n, ncol));
  DeviceGuard g(ctx->device);
  if (dtype == JL_C64)
    JL_HIP(ctx, reorth_pass<float>(n, ncol, static_cast<const float2*>(V), ldv,
                                   static_cast<float2*>(u), coef, static_cast<char*>(ws), ctx->stream));
  else if (dtype == JL_C128)
    JL_HIP(ctx, reorth_pass<double>(n, ncol, static_cast<const double2*>(V), ldv,
                                    static_cast<double2*>(u), coef, static_cast<char*>(ws), ctx->stream));
  else
    return set_err(ctx, JL_EINVAL, "dtype must be JL_C64 or JL_C128");
  return JL_OK;
}

jl_status jl_reorth_pass_noalloc(jl_ctx ctx, jl_dtype dtype, int64_t n, int32_t ncol,
                                 const void* V, int64_t ldv, void* u, double* coef) {
  if (!ctx) return set_err(nullptr, JL_EINVAL, "ctx is NULL");
  if (n <= 0 || n % 2 || ncol < 0 || ldv < n || !u || !coef || (ncol > 0 && !V))
    return set_err(ctx, JL_EINVAL, "invalid reorth_pass_noalloc arguments");
  if (dtype != JL_C64 && dtype != JL_C128)
    return set_err(ctx, JL_EINVAL, "dtype must be JL_C64 or JL_C128");
  const int64_t h = n / 2;
  const int es = dtype == JL_C64 ? 8 : 16;
  if (ncol > kNaMaxCols)
    return set_err(ctx, JL_EINVAL, "reorth_pass_noalloc: ncol = %d exceeds the static scratch limit %d",
                   ncol, kNaMaxCols);
  if (reorth_update_blocks(h, es) > kNaMaxUpdBlocks || reorth_dots_blocks(h, es) > kNaMaxDotsBlocks)
    return set_err(ctx, JL_EINVAL,
                   "reorth_pass_noalloc: n = %lld exceeds the static scratch limit", (long long)n);
  if (!ctx->na_scratch)
    return set_err(ctx, JL_EHIP, "reorth_pass_noalloc: no static scratch on device %d (%s)",
                   ctx->device, ctx->na_err.c_str());
  double* base = static_cast<double*>(ctx->na_scratch);
  double* dp = base;
  double* up = dp + kNaDots;
  double* scr = up + kNaUpd;
  unsigned* cnt = reinterpret_cast<unsigned*>(scr + kNaWide);
  DeviceGuard g(ctx->device);
  if (dtype == JL_C64)
    JL_HIP(ctx, reorth_pass_on<float>(n, ncol, static_cast<const float2*>(V), ldv,
                                      static_cast<float2*>(u), coef, dp, up, scr, cnt, ctx->stream));
  else
    JL_HIP(ctx, reorth_pass_on<double>(n, ncol, static_cast<const double2*>(V), ldv,
                                       static_cast<double2*>(u), coef, dp, up, scr, cnt, ctx->stream));
  return JL_OK;
}

jl_status jl_ritz_workspace_bytes(int32_t m, size_t* bytes) {
  if (!bytes || m < 1) return set_err(nullptr, JL_EINVAL, "invalid ritz size");
  *bytes = sizeof(double) * (ritz_scratch_doubles(m) + (size_t)m);   // + zlast
  return JL_OK;
}

jl_status jl_ritz(jl_ctx ctx, int32_t m, const double* T, int32_t which, double* lam, double* Z,
                  void* ws, size_t ws_bytes) {
  if (!ctx) return set_err(nullptr, JL_EINVAL, "ctx is NULL");
  if (m < 1 || !T || !lam || !Z || (which != JL_LOWEST && which != JL_LARGEST))
    return set_err(ctx, JL_EINVAL, "invalid ritz arguments");
  const size_t need = sizeof(double) * (ritz_scratch_doubles(m) + (size_t)m);
  if (!ws || ws_bytes < need) return set_err(ctx, JL_ENOMEM, "workspace too small (%zu < %zu)", ws_bytes, need);
  DeviceGuard g(ctx->device);
  std::vector<double> hT((size_t)m * m);
  JL_HIP(ctx, hipMemcpyAsync(hT.data(), T, sizeof(double) * hT.size(), hipMemcpyDeviceToHost, ctx->stream));
  JL_HIP(ctx, hipStreamSynchronize(ctx->stream));
  double fro2 = 0.0;
  for (double v : hT) fro2 += v * v;
  double* scratch = static_cast<double*>(ws);
  double* zlast = scratch + ritz_scratch_doubles(m);
  double hs = 0.0;
  JL_HIP(ctx, ritz_device<double>(m, T, fro2, which == JL_LARGEST, 0, scratch, lam, Z, nullptr,
                                  zlast, &hs, ctx->stream));
  return JL_OK;
}

jl_status jl_ritz_restart_workspace_bytes(int32_t m, size_t* bytes) {
  if (!bytes || m < 1 || m > dc_max_m()) return set_err(nullptr, JL_EINVAL, "invalid ritz size");
  *bytes = sizeof(double) * (ritz_scratch_doubles(m) + (size_t)m);   // + zlast
  return JL_OK;
}

jl_status jl_ritz_restart(jl_ctx ctx, int32_t m, int32_t k, const double* packed, int32_t which,
                          double* lam, double* Z, void* ws, size_t ws_bytes) {
  if (!ctx) return set_err(nullptr, JL_EINVAL, "ctx is NULL");
  if (m < 1 || m > dc_max_m() || k < 0 || k >= m || !packed || !lam || !Z ||
      (which != JL_LOWEST && which != JL_LARGEST))
    return set_err(ctx, JL_EINVAL, "invalid ritz_restart arguments");
  const size_t need = sizeof(double) * (ritz_scratch_doubles(m) + (size_t)m);
  if (!ws || ws_bytes < need) return set_err(ctx, JL_ENOMEM, "workspace too small (%zu < %zu)", ws_bytes, need);
  DeviceGuard g(ctx->device);
  double* scratch = static_cast<double*>(ws);
  double* zlast = scratch + ritz_scratch_doubles(m);
  JL_HIP(ctx, ritz_arrow_device<double>(m, k, packed, which == JL_LARGEST, 0, scratch, lam, Z, nullptr,
                                        zlast, ctx->stream));
  JL_HIP(ctx, hipStreamSynchronize(ctx->stream));   // `packed` may be reused by the caller
  return JL_OK;
}

jl_status jl_basis_update(jl_ctx ctx, jl_dtype dtype, int64_t n, int32_t m, int32_t k,
                          const void* V, int64_t ldv, const void* Z, int64_t ldz, void* Y,
                          int64_t ldy) {
  if (!ctx) return set_err(nullptr, JL_EINVAL, "ctx is NULL");
  if (n <= 0 || n % 2 || m < 1 || k < 0 || ldv < n || ldy < n || ldz < m || (ldv % 2) ||
      (ldy % 2) || (k > 0 && (!V || !Z || !Y)))
    return set_err(ctx, JL_EINVAL, "invalid basis_update arguments");
  if (k == 0) return JL_OK;
  DeviceGuard g(ctx->device);
  if (dtype == JL_C64)
    JL_HIP(ctx, (launch_gemm_nn<float, double>)(static_cast<const float*>(V), 2 * ldv,
                                              static_cast<const double*>(Z), ldz,
                                              static_cast<float*>(Y), 2 * ldy, 2 * n, k, m, ctx->stream));
  else if (dtype == JL_C128)
    JL_HIP(ctx, (launch_gemm_nn<double, double>)(static_cast<const double*>(V), 2 * ldv,
                                       static_cast<const double*>(Z), ldz, static_cast<double*>(Y),
                                       2 * ldy, 2 * n, k, m, ctx->stream));
  else
    return set_err(ctx, JL_EINVAL, "dtype must be JL_C64 or JL_C128");
  return JL_OK;
}

}  // extern "C"
