// Column reductions of block partial sums and small vector kernels used
// around the Lanczos step (scaling, copies, the J-partner of vectors).
#include <algorithm>

#include "common.h"

namespace jl {
namespace {

// out[c] = sum over b of partial[b*stride + c].  A block of 256 threads
// covers C consecutive columns with 256/C threads per column, each summing
// every (256/C)-th row; the per-column partials are then combined in LDS in
// a fixed tree order (deterministic).
template <int C>
__global__ __launch_bounds__(256) void k_reduce_cols(const double* __restrict__ partial, int nblk,
                                                     int stride, int ncols,
                                                     double* __restrict__ out) {
  constexpr int G = 256 / C;
  __shared__ double sh[256];
  const int tx = threadIdx.x % C, ty = threadIdx.x / C;
  const int c = blockIdx.x * C + tx;
  // four independent running sums per thread (more loads in flight), added
  // in a fixed order
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (c < ncols) {
    int b = ty;
    for (; b + 3 * G < nblk; b += 4 * G) {
      s0 += partial[(int64_t)b * stride + c];
      s1 += partial[(int64_t)(b + G) * stride + c];
      s2 += partial[(int64_t)(b + 2 * G) * stride + c];
      s3 += partial[(int64_t)(b + 3 * G) * stride + c];
    }
    for (; b < nblk; b += G) s0 += partial[(int64_t)b * stride + c];
  }
  sh[threadIdx.x] = (s0 + s1) + (s2 + s3);
  __syncthreads();
#pragma unroll
  for (int g = G / 2; g > 0; g /= 2) {
    if (ty < g) sh[threadIdx.x] += sh[threadIdx.x + g * C];
    __syncthreads();
  }
  if (ty == 0 && c < ncols) out[c] = sh[tx];
}

// out[c] = sum over b of partial[b*stride + c] for many columns (the inner
// products of the reorthogonalisation, 4*ncol + 1 of them): grid (tiles of
// 64 columns, R row slices).  Block (t, r) sums its slice of rows for 64
// columns (four wavefronts over interleaved rows, combined in LDS) into
// scr[r * ncols + c]; the last slice of a tile to finish, found with the
// per-tile counter cnt[t], sums the R slice values in order r = 0 .. R-1 and
// resets the counter; last_out, if given, also receives out[ncols - 2] and
// out[ncols - 1] (at last_out[0], last_out[1]; ncols >= 2).
// The slice sums are agent-scope stores, complete before
// the counter moves, and are read back with agent-scope loads (the per-XCD
// L2s are not coherent with each other).  Deterministic for a given nblk.
__global__ __launch_bounds__(256) void k_reduce_wide(const double* __restrict__ partial, int nblk,
                                                     int stride, int ncols, double* __restrict__ out,
                                                     double* scr, unsigned* cnt, double* last_out) {
  __shared__ double sh[4][64];
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int c = blockIdx.x * 64 + lane;
  const int R = gridDim.y, r = blockIdx.y;
  const int per = (nblk + R - 1) / R;
  const int b1 = min(nblk, (r + 1) * per);
  double s = 0.0;
  if (c < ncols) {
    int b = r * per + w;
    for (; b + 12 < b1; b += 16) {   // four independent loads per pass
      const double x0 = partial[(int64_t)b * stride + c];
      const double x1 = partial[(int64_t)(b + 4) * stride + c];
      const double x2 = partial[(int64_t)(b + 8) * stride + c];
      const double x3 = partial[(int64_t)(b + 12) * stride + c];
      s += (x0 + x1) + (x2 + x3);
    }
    for (; b < b1; b += 4) s += partial[(int64_t)b * stride + c];
  }
  sh[w][lane] = s;
  __syncthreads();
  if (w != 0) return;
  const double t = (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
  if (R == 1) {
    if (c < ncols) out[c] = t;
    if (last_out && c >= ncols - 2 && c < ncols) last_out[c - (ncols - 2)] = t;
    return;
  }
  if (c < ncols)
    __hip_atomic_store(&scr[(int64_t)r * ncols + c], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __builtin_amdgcn_s_waitcnt(0);   // this wavefront's slice sums are complete
  unsigned done = 0;
  if (lane == 0) done = atomicAdd(&cnt[blockIdx.x], 1u);
  done = __shfl(done, 0);
  if (done != (unsigned)(R - 1)) return;   // uniform within the wavefront
  if (c < ncols) {
    double v = 0.0;
    for (int rr = 0; rr < R; ++rr)
      v += __hip_atomic_load(&scr[(int64_t)rr * ncols + c], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    out[c] = v;
    if (last_out && c >= ncols - 2) last_out[c - (ncols - 2)] = v;
  }
  if (lane == 0) cnt[blockIdx.x] = 0u;   // ready for the next launch
}

template <typename S>
__global__ void k_scale(cplx<S>* __restrict__ u, int64_t n, S s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    cplx<S> v = u[i];
    v.x *= s; v.y *= s;
    u[i] = v;
  }
}

// u *= 1 / sqrt(*nrm2), the factor formed on the device in FP64.
template <typename S>
__global__ void k_scale_dev(cplx<S>* __restrict__ u, int64_t n, const double* __restrict__ nrm2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const S s = (S)(1.0 / sqrt(*nrm2));
    cplx<S> v = u[i];
    v.x *= s; v.y *= s;
    u[i] = v;
  }
}

__global__ void k_zero_u32(unsigned* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

template <typename S>
__global__ void k_fill(cplx<S>* __restrict__ u, int64_t n, S val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    cplx<S> v;
    v.x = val; v.y = (S)0;
    u[i] = v;
  }
}

// Y = J X^* = [-conj(X_bot); conj(X_top)]; safe in place (each thread reads
// both halves of its pair before writing).
template <typename S>
__global__ void k_pair(const cplx<S>* X, int64_t ldx, cplx<S>* Y, int64_t ldy, int64_t h) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= h) return;
  const cplx<S>* x = X + (int64_t)blockIdx.y * ldx;
  cplx<S>* y = Y + (int64_t)blockIdx.y * ldy;
  const cplx<S> t = x[p], b = x[h + p];
  cplx<S> yt, yb;
  yt.x = -b.x; yt.y = b.y;
  yb.x = t.x; yb.y = -t.y;
  y[p] = yt;
  y[h + p] = yb;
}

template <typename S>
__global__ void k_copy_cols(const cplx<S>* __restrict__ X, int64_t ldx, cplx<S>* __restrict__ Y,
                            int64_t ldy, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) Y[(int64_t)blockIdx.y * ldy + i] = X[(int64_t)blockIdx.y * ldx + i];
}

template <typename S>
__global__ void k_copy_pairs(const cplx<S>* __restrict__ X, int64_t ldx, cplx<S>* __restrict__ Y,
                             int64_t ldy, int64_t n, const int* __restrict__ pairs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int dst = pairs[2 * blockIdx.y], src = pairs[2 * blockIdx.y + 1];
    Y[(int64_t)dst * ldy + i] = X[(int64_t)src * ldx + i];
  }
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_reduce_cols(const double* partial, int nblk, int stride, int ncols, double* out,
                              hipStream_t st) {
  if (ncols <= 1)
    hipLaunchKernelGGL(k_reduce_cols<1>, dim3(1), dim3(256), 0, st, partial, nblk, stride, ncols, out);
  else if (ncols <= 4)
    hipLaunchKernelGGL(k_reduce_cols<4>, dim3(1), dim3(256), 0, st, partial, nblk, stride, ncols, out);
  else
    hipLaunchKernelGGL(k_reduce_cols<16>, dim3(blocks_for(ncols, 16)), dim3(256), 0, st, partial,
                       nblk, stride, ncols, out);
  return hipGetLastError();
}

int reduce_wide_slices(int nblk) { return std::max(1, std::min(16, nblk / 64)); }
int reduce_wide_tiles(int ncols) { return (ncols + 63) / 64; }
size_t reduce_wide_scratch_doubles(int nblk, int ncols) {
  return (size_t)reduce_wide_slices(nblk) * (size_t)ncols;
}

hipError_t launch_reduce_wide(const double* partial, int nblk, int stride, int ncols, double* out,
                              double* scr, unsigned* cnt, hipStream_t st, double* last_out) {
  if (ncols <= 0 || nblk <= 0 || (last_out && ncols < 2)) return hipErrorInvalidValue;
  const int R = reduce_wide_slices(nblk);
  if (R > 1 && (!scr || !cnt)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce_wide, dim3((unsigned)reduce_wide_tiles(ncols), (unsigned)R), dim3(256),
                     0, st, partial, nblk, stride, ncols, out, scr, cnt, last_out);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_scale(cplx<S>* u, int64_t n, double scale, hipStream_t st) {
  hipLaunchKernelGGL(k_scale<S>, dim3(blocks_for(n, 256)), dim3(256), 0, st, u, n, (S)scale);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_scale_dev(cplx<S>* u, int64_t n, const double* nrm2, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_dev<S>, dim3(blocks_for(n, 256)), dim3(256), 0, st, u, n, nrm2);
  return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_fill(cplx<S>* u, int64_t n, double value, hipStream_t st) {
  hipLaunchKernelGGL(k_fill<S>, dim3(blocks_for(n, 256)), dim3(256), 0, st, u, n, (S)value);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_pair(const cplx<S>* X, int64_t ldx, cplx<S>* Y, int64_t ldy, int64_t h, int k,
                       hipStream_t st) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pair<S>, dim3(blocks_for(h, 256), (unsigned)k), dim3(256), 0, st, X, ldx, Y,
                     ldy, h);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_copy_cols(const cplx<S>* X, int64_t ldx, cplx<S>* Y, int64_t ldy, int64_t n,
                            int k, hipStream_t st) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_cols<S>, dim3(blocks_for(n, 256), (unsigned)k), dim3(256), 0, st, X,
                     ldx, Y, ldy, n);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_copy_pairs(const cplx<S>* X, int64_t ldx, cplx<S>* Y, int64_t ldy, int64_t n,
                             const int* pairs, int npairs, hipStream_t st) {
  if (npairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_pairs<S>, dim3(blocks_for(n, 256), (unsigned)npairs), dim3(256), 0, st, X,
                     ldx, Y, ldy, n, pairs);
  return hipGetLastError();
}

#define JL_INST(S)                                                                                \
  template hipError_t launch_scale<S>(cplx<S>*, int64_t, double, hipStream_t);                    \
  template hipError_t launch_scale_dev<S>(cplx<S>*, int64_t, const double*, hipStream_t);         \
  template hipError_t launch_fill<S>(cplx<S>*, int64_t, double, hipStream_t);                     \
  template hipError_t launch_pair<S>(const cplx<S>*, int64_t, cplx<S>*, int64_t, int64_t, int,    \
                                     hipStream_t);                                                \
  template hipError_t launch_copy_cols<S>(const cplx<S>*, int64_t, cplx<S>*, int64_t, int64_t,    \
                                          int, hipStream_t);                                      \
  template hipError_t launch_copy_pairs<S>(const cplx<S>*, int64_t, cplx<S>*, int64_t, int64_t,   \
                                           const int*, int, hipStream_t);
JL_INST(float)
JL_INST(double)
#undef JL_INST

}  // namespace jl
