/*
 * jlanczos_kernels.h -- the individual steps of the J-restricted Lanczos
 * iteration as C-ABI calls, for callers that assemble their own iteration and
 * for step-by-step parity checks.  Conventions (status codes, dtypes, vector
 * layout, streams, device/host pointers, no device allocation) are those of
 * jlanczos.h.  Scratch space comes from the caller; its size from the
 * matching *_workspace_bytes call.
 */
#ifndef JLANCZOS_KERNELS_H
#define JLANCZOS_KERNELS_H

#include "jlanczos.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One pass of the J-restricted Gram-Schmidt of Alg. 2 in block form:
 *   c_v = V^H u,  c_w = W^H u  (W = J V^*, never stored),
 *   u  <- u - V c_v - W c_w,
 * against the ncol columns of V (device, n x ncol, leading dimension ldv,
 * dtype).  u (device, n) is updated in place.  coef (device, FP64 [4*ncol+2])
 * receives per column (Re c_v, Im c_v, Re c_w, Im c_w), then ||u||^2 before
 * the pass at [4*ncol] and ||u||^2 after it at [4*ncol+1].  Inner products
 * and norms are accumulated in FP64.  ncol may be 0 (norm only).
 * Errors: JL_EINVAL (odd n, ncol < 0 or > 2047, ldv < n, NULL), JL_ENOMEM. */
jl_status jl_reorth_pass_workspace_bytes(int64_t n, int32_t ncol, size_t* bytes);
jl_status jl_reorth_pass(jl_ctx ctx, jl_dtype dtype, int64_t n, int32_t ncol, const void* V,
                         int64_t ldv, void* u, double* coef, void* ws, size_t ws_bytes);

/* The same pass as jl_reorth_pass for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops): no workspace argument, no
 * device allocation, no memset.  Its scratch (partial sums and counters) is
 * a static device array of the library, 17.5 MB per GPU, held from the first
 * jl_ctx_create on that GPU until the process ends; every call on one GPU
 * shares it, so calls that overlap on one GPU (other streams, other
 * contexts, other threads) race and must be ordered by the caller.  Same
 * arguments and results as jl_reorth_pass.  Errors: JL_EINVAL as
 * jl_reorth_pass, and for ncol > 256 or n beyond the scratch (FP32 with an
 * even n / 2 and n above 16777216, or FP64 with n above 8388608, where the
 * inner products would write more than 2048 blocks of partial sums); JL_EHIP
 * if the scratch could not be located on the context's device. */
jl_status jl_reorth_pass_noalloc(jl_ctx ctx, jl_dtype dtype, int64_t n, int32_t ncol,
                                 const void* V, int64_t ldv, void* u, double* coef);

/* Rayleigh-Ritz step of Alg. 1: T = Z diag(lam) Z^T for a real symmetric
 * m x m FP64 matrix T (device, column-major, leading dimension m), with the
 * eigenpairs sorted ascending (which = JL_LOWEST) or descending
 * (JL_LARGEST).  lam (device, m) and Z (device, m x m column-major) are FP64.
 * Errors: JL_EINVAL (m < 1, NULL), JL_ENOMEM. */
jl_status jl_ritz_workspace_bytes(int32_t m, size_t* bytes);
jl_status jl_ritz(jl_ctx ctx, int32_t m, const double* T, int32_t which, double* lam, double* Z,
                  void* ws, size_t ws_bytes);

/* The same Rayleigh-Ritz step for the structure the thick restart of Alg. 1
 * gives T_m (the shrink to k + 1 and eq. dynamicwin): diagonal theta_0..k-1
 * (kept Ritz values), their couplings s_i = t_{k,i} in row and column k, and
 * from index k on the tridiagonal t_jj / t_{j+1,j} of the cycle's Lanczos
 * steps (k = 0: a plain tridiagonal matrix).  `packed` (host, FP64) holds
 * theta[k], s[k], alpha[m - k] (t_kk .. t_{m-1,m-1}), beta[m - k - 1]
 * (t_{k+1,k} .. t_{m-1,m-2}).  Solved by divide and conquer on the device
 * (tears at the tridiagonal couplings and at t_{k+1,k}; secular equations
 * with deflation; Gu-Eisenstat weights).  lam (device, m) and Z (device,
 * m x m column-major) as for jl_ritz.  Returns after the work is queued on
 * the ctx stream; `packed` is copied before the call returns.
 * Errors: JL_EINVAL (m < 1, m > 1024, k < 0, k >= m, NULL), JL_ENOMEM. */
jl_status jl_ritz_restart_workspace_bytes(int32_t m, size_t* bytes);
jl_status jl_ritz_restart(jl_ctx ctx, int32_t m, int32_t k, const double* packed, int32_t which,
                          double* lam, double* Z, void* ws, size_t ws_bytes);

/* Thick-restart basis update of Alg. 1 (V_m := V_m Z_m, first k columns):
 * Y = V Z with V (device, n x m complex, leading dimension ldv, dtype), Z
 * (device, m x k real FP64 column-major, leading dimension ldz) and Y
 * (device, n x k, leading dimension ldy, dtype).  Accumulation is FP64 for
 * both dtypes (FP32 inputs are widened, the result is rounded once).  Y must
 * not overlap V.  ldv and ldy must be even (16-byte aligned columns).
 * Errors: JL_EINVAL. */
jl_status jl_basis_update(jl_ctx ctx, jl_dtype dtype, int64_t n, int32_t m, int32_t k,
                          const void* V, int64_t ldv, const void* Z, int64_t ldz, void* Y,
                          int64_t ldy);

#ifdef __cplusplus
}
#endif

#endif /* JLANCZOS_KERNELS_H */
