// Internal host-side definitions shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/jlanczos.h"
#include "common.h"

struct jl_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;   // caller's stream (borrowed; NULL = legacy default stream)
  hipStream_t work = nullptr;     // owned non-blocking stream for jl_solve's launch sequence
  hipEvent_t order = nullptr;     // orders `work` after `stream`
  void* na_scratch = nullptr;     // device address of this device's allocation-free scratch
  std::string na_err;             // why na_scratch could not be set up (if it could not)
  std::string err;
  ~jl_ctx_s() {
    if (order) (void)hipEventDestroy(order);
    if (work) (void)hipStreamDestroy(work);
  }
};

namespace jl {

// The ctx's own non-blocking stream (created on first use, default
// priority), made to wait for the work already queued on the caller's
// stream.  A solve issues thousands of small launches; on the legacy default
// stream each one also synchronises with the other blocking streams.
hipError_t work_stream(jl_ctx ctx, hipStream_t* out);

// Device address of the library's static scratch array on `device` (the
// current device), looked up once per device and cached; used by the
// allocation-free entry points.
hipError_t noalloc_scratch_address(int device, void** out);

// Records the message for jl_last_error(ctx) (and the calling thread) and
// returns `code`.
jl_status set_err(jl_ctx ctx, jl_status code, const char* fmt, ...);

#define JL_HIP(ctx, expr)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return ::jl::set_err(ctx, JL_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                           __FILE__, __LINE__);                                                \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) hipSetDevice(prev);
  }
};

// Scratch doubles the Ritz step needs beyond its outputs for an m x m problem.
size_t ritz_scratch_doubles(int m);

// Rayleigh-Ritz on the device: eigen-decomposition of Tdev (m x m, ld m) by
// Jacobi (fro2 = ||T||_F^2 sets the stopping test), then the sort of
// launch_ritz_sort.  `scratch` holds ritz_scratch_doubles(m) doubles; `hs` is
// a host double used to read the off-diagonal norm back (stream synchronised).
template <typename S>
hipError_t ritz_device(int m, const double* Tdev, double fro2, int descending, int kcols,
                       double* scratch, double* lam_s, double* Zs, S* Zc, double* zlast,
                       double* hs, hipStream_t st);

// Rayleigh-Ritz for the restart structure of T_m (k kept Ritz values theta
// with couplings s, then the tridiagonal alpha/beta of the cycle, packed as
// theta[k], s[k], alpha[m - k], beta[m - k - 1] in host memory `hstruct`,
// which must stay unchanged until the stream is synchronised) by divide and
// conquer, then the sort of launch_ritz_sort.  m <= dc_max_m();
// `scratch` holds ritz_scratch_doubles(m) doubles.
template <typename S>
hipError_t ritz_arrow_device(int m, int k, const double* hstruct, int descending, int kcols,
                             double* scratch, double* lam_s, double* Zs, S* Zc, double* zlast,
                             hipStream_t st);

}  // namespace jl
