// Conjugate gradients for the invert mode: u = A^-1 v with A Hermitian
// positive definite (the paper solves A^-1 v_j by CG, Sec. 4.2).  The
// iteration is the one of Hestenes and Stiefel with x_0 = 0:
//   alpha = r^H r / p^H A p,  x += alpha p,  r -= alpha A p,
//   beta = r'^H r' / r^H r,   p = r' + beta p,
// stopping when r^H r <= cg_tol^2 b^H b or after maxit iterations.
//
// Every scalar lives on the device (CgSlot), so a whole run of iterations
// is queued without host round trips.  One iteration is two launches: the
// operator apply, which forms the direction p = r + beta p_old on the fly,
// stores it (into the other of two direction buffers) and leaves the block
// partials of p^H A p; and the fused alpha / x, r update / beta step.  That
// step sets the done flag on convergence, after which every queued kernel
// (the operator applies too, through their skip pointer) returns at once.
//
// Vectors are n complex elements of storage type S, interleaved (re, im),
// 16-byte aligned; the vector kernels move 16 bytes per thread and step
// (two FP32 or one FP64 complex), arithmetic and partial sums in FP64.
#include <algorithm>

#include "common.h"

namespace jl {

namespace {

constexpr int kCgThreads = 256;
// At most 256 workgroups, one per CU, each thread with four chunks whose loads
// are in flight together (and 256 partial sums for the last workgroup): at
// 16^4 the fused step took 9 us less than with 1024 workgroups of one chunk
// per thread, whether those counted on one counter or on eight.
constexpr int kCgMaxBlocks = 256;
constexpr int kCgUnroll = 4;   // chunks per thread loaded together in the fused step

template <typename S> constexpr int kPerChunk = 16 / (int)sizeof(S);   // scalars per 16 bytes

template <typename S>
__device__ __forceinline__ void ld16(const S* p, S (&o)[kPerChunk<S>]) {
  using V = typename vec16_t<S>::type;
  const V v = *reinterpret_cast<const V*>(p);
  __builtin_memcpy(o, &v, 16);
}

template <typename S>
__device__ __forceinline__ void st16(S* p, const S (&o)[kPerChunk<S>]) {
  using V = typename vec16_t<S>::type;
  V v;
  __builtin_memcpy(&v, o, 16);
  *reinterpret_cast<V*>(p) = v;
}

__device__ __forceinline__ double cg_block_sum(double v, double* sh) {   // valid in thread 0
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kCgThreads / 64; ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

// Sum of part[b * stride] over b < nblk by one block (fixed order).
__device__ __forceinline__ double cg_reduce(const double* __restrict__ part, int nblk, int stride,
                                            double* sh) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kCgThreads) s += part[(int64_t)b * stride];
  return cg_block_sum(s, sh);
}

__device__ __forceinline__ bool cg_done(const double* cs) { return cs[CG_DONE] != 0.0; }

// x = 0, r = b, p = 0; part[blk] = block partial of b^H b.
template <typename S>
__global__ __launch_bounds__(kCgThreads) void k_cg_init(const S* __restrict__ b, S* __restrict__ x,
                                                        S* __restrict__ r, S* __restrict__ p,
                                                        int64_t nchunk, double* __restrict__ part) {
  __shared__ double sh[kCgThreads / 64];
  constexpr int K = kPerChunk<S>;
  double acc = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * kCgThreads + threadIdx.x; c < nchunk;
       c += (int64_t)gridDim.x * kCgThreads) {
    S v[K], z[K];
    ld16<S>(b + c * K, v);
#pragma unroll
    for (int e = 0; e < K; ++e) {
      acc += (double)v[e] * v[e];
      z[e] = (S)0;
    }
    st16<S>(x + c * K, z);
    st16<S>(r + c * K, v);
    st16<S>(p + c * K, z);
  }
  acc = cg_block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// b^H b from the init partials; sets rr, the stop threshold and the counters.
__global__ __launch_bounds__(kCgThreads) void k_cg_start(const double* __restrict__ part, int nblk,
                                                         double* __restrict__ cs, double tol2,
                                                         int maxit) {
  __shared__ double sh[kCgThreads / 64];
  const double bb = cg_reduce(part, nblk, 1, sh);
  if (threadIdx.x == 0) {
    *reinterpret_cast<unsigned*>(cs + CG_CNT) = 0u;
    cs[CG_RR] = bb;
    cs[CG_BB] = bb;
    cs[CG_THR] = tol2 * bb;
    cs[CG_ITERS] = 0.0;
    cs[CG_BETA] = 0.0;   // the first direction is r itself
    cs[CG_MAXIT] = (double)maxit;
    cs[CG_DONE] = (bb <= tol2 * bb || maxit <= 0) ? 1.0 : 0.0;   // b = 0 needs no iteration
  }
}

// alpha, x += alpha p, r -= alpha q, then beta and the stop test, in one
// launch: every block sums the apply partials of p^H q itself (the same
// order everywhere, so all blocks hold the same alpha), and the last block to
// finish (counted on cnt) sums the r^H r partials and updates the scalars.
// The partials are written and read with agent-scope accesses, which go past
// the caches that are not coherent across the chip.
template <typename S>
__global__ __launch_bounds__(kCgThreads) void k_cg_update_fused(
    S* __restrict__ x, S* __restrict__ r, const S* __restrict__ p, const S* __restrict__ q,
    int64_t nchunk, const double* __restrict__ apart, int napply, double* __restrict__ cs,
    double* __restrict__ part, unsigned* __restrict__ cnt) {
  __shared__ double sh[kCgThreads / 64];
  __shared__ double bcast;
  __shared__ bool last;
  if (cg_done(cs)) return;   // uniform
  constexpr int K = kPerChunk<S>;
  constexpr int U = kCgUnroll;
  const int64_t c0 = (int64_t)blockIdx.x * kCgThreads + threadIdx.x;
  const int64_t cstep = (int64_t)gridDim.x * kCgThreads;
  // The operands of the first U chunks do not depend on alpha: their loads go
  // out before the reduction of the apply partials, so the two waits overlap.
  S xv[U][K], rv[U][K], pv[U][K], qv[U][K];
  auto load = [&](int64_t cb) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t c = cb + u * cstep;
      if (c < nchunk) {
        ld16<S>(x + c * K, xv[u]);
        ld16<S>(r + c * K, rv[u]);
        ld16<S>(p + c * K, pv[u]);
        ld16<S>(q + c * K, qv[u]);
      }
    }
  };
  load(c0);
  const double rr_old = cs[CG_RR];
  const double pap = cg_reduce(apart, napply, 2, sh);
  if (threadIdx.x == 0) bcast = pap;
  __syncthreads();
  const double pq = bcast;
  if (!(pq > 0.0)) {   // not positive definite (or NaN): every block sees it
    if (blockIdx.x == 0 && threadIdx.x == 0) cs[CG_DONE] = 2.0;
    return;
  }
  const double al = rr_old / pq;
  double acc = 0.0;
  for (int64_t cb = c0; cb < nchunk; cb += U * cstep) {
    if (cb != c0) load(cb);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t c = cb + u * cstep;
      if (c >= nchunk) continue;
#pragma unroll
      for (int e = 0; e < K; ++e) {
        xv[u][e] = (S)((double)xv[u][e] + al * (double)pv[u][e]);
        rv[u][e] = (S)((double)rv[u][e] - al * (double)qv[u][e]);
        acc += (double)rv[u][e] * rv[u][e];
      }
      st16<S>(x + c * K, xv[u]);
      st16<S>(r + c * K, rv[u]);
    }
  }
  acc = cg_block_sum(acc, sh);
  if (threadIdx.x == 0) {
    // The partial is an agent-scope store, which bypasses the per-XCD L2
    // (not coherent across XCDs); waiting for it to complete before the
    // counter moves is all the last block needs to see it.  A release fence
    // here would write back every dirty line of this XCD's L2 (measured: the
    // kernel took 43 us instead of a few).
    __hip_atomic_store(&part[blockIdx.x], acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);
    const unsigned done_blocks = atomicAdd(cnt, 1u);
    last = done_blocks == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;   // uniform within the block
  double s = 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += kCgThreads)
    s += __hip_atomic_load(&part[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double rr = cg_block_sum(s, sh);
  if (threadIdx.x == 0) {
    const double it = cs[CG_ITERS] + 1.0;
    cs[CG_ALPHA] = al;
    cs[CG_BETA] = rr / cs[CG_RR];
    cs[CG_RR] = rr;
    cs[CG_ITERS] = it;
    if (rr <= cs[CG_THR] || it >= cs[CG_MAXIT] || !(rr == rr)) cs[CG_DONE] = 1.0;
    *cnt = 0u;   // ready for the next iteration's launch
  }
}

// u = x; part[2*blk], part[2*blk+1] = block partial of v^H u (Re, Im).
template <typename S>
__global__ __launch_bounds__(kCgThreads) void k_cg_finish(const S* __restrict__ x,
                                                          S* __restrict__ u,
                                                          const S* __restrict__ v, int64_t nchunk,
                                                          double* __restrict__ part) {
  __shared__ double sh[kCgThreads / 64];
  constexpr int K = kPerChunk<S>;
  double are = 0.0, aim = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * kCgThreads + threadIdx.x; c < nchunk;
       c += (int64_t)gridDim.x * kCgThreads) {
    S xv[K], vv[K];
    ld16<S>(x + c * K, xv);
    ld16<S>(v + c * K, vv);
    st16<S>(u + c * K, xv);
#pragma unroll
    for (int e = 0; e < K; e += 2) {   // (re, im) pairs: conj(v) u
      are += (double)vv[e] * xv[e] + (double)vv[e + 1] * xv[e + 1];
      aim += (double)vv[e] * xv[e + 1] - (double)vv[e + 1] * xv[e];
    }
  }
  are = cg_block_sum(are, sh);
  aim = cg_block_sum(aim, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = are;
    part[2 * blockIdx.x + 1] = aim;
  }
}

// part[blk] = block partial of x^H x.
template <typename S>
__global__ __launch_bounds__(kCgThreads) void k_norm2(const S* __restrict__ x, int64_t nchunk,
                                                      double* __restrict__ part) {
  __shared__ double sh[kCgThreads / 64];
  constexpr int K = kPerChunk<S>;
  double acc = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * kCgThreads + threadIdx.x; c < nchunk;
       c += (int64_t)gridDim.x * kCgThreads) {
    S v[K];
    ld16<S>(x + c * K, v);
#pragma unroll
    for (int e = 0; e < K; ++e) acc += (double)v[e] * v[e];
  }
  acc = cg_block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

template <typename S>
int64_t chunks(int64_t n) {   // 16-byte chunks in n complex elements (n even)
  return n * 2 * (int64_t)sizeof(S) / 16;
}

}  // namespace

int cg_blocks(int64_t n) {
  const int64_t nc = n / 2;   // FP32: two complex per chunk (FP64 grid-strides twice as far)
  const int64_t b = (nc + kCgThreads - 1) / kCgThreads;
  return (int)std::min<int64_t>(std::max<int64_t>(b, 1), kCgMaxBlocks);
}

template <typename S>
hipError_t launch_cg_init(const cplx<S>* b, cplx<S>* x, cplx<S>* r, cplx<S>* p, int64_t n,
                          double* part, double* cs, double tol, int maxit, hipStream_t st) {
  const int nb = cg_blocks(n);
  hipLaunchKernelGGL(k_cg_init<S>, dim3(nb), dim3(kCgThreads), 0, st,
                     reinterpret_cast<const S*>(b), reinterpret_cast<S*>(x),
                     reinterpret_cast<S*>(r), reinterpret_cast<S*>(p), chunks<S>(n), part);
  hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(kCgThreads), 0, st, part, nb, cs, tol * tol, maxit);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_cg_step(cplx<S>* x, cplx<S>* r, cplx<S>* p, const cplx<S>* q, int64_t n,
                          const double* apart, int napply, double* part, double* cs,
                          hipStream_t st) {
  const int nb = cg_blocks(n);
  hipLaunchKernelGGL(k_cg_update_fused<S>, dim3(nb), dim3(kCgThreads), 0, st,
                     reinterpret_cast<S*>(x), reinterpret_cast<S*>(r),
                     reinterpret_cast<const S*>(p), reinterpret_cast<const S*>(q), chunks<S>(n),
                     apart, napply, cs, part, reinterpret_cast<unsigned*>(cs + CG_CNT));
  return hipGetLastError();
}

template <typename S>
hipError_t launch_cg_finish(const cplx<S>* x, cplx<S>* u, const cplx<S>* v, int64_t n,
                            double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_finish<S>, dim3(cg_blocks(n)), dim3(kCgThreads), 0, st,
                     reinterpret_cast<const S*>(x), reinterpret_cast<S*>(u),
                     reinterpret_cast<const S*>(v), chunks<S>(n), part);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_norm2(const cplx<S>* x, int64_t n, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_norm2<S>, dim3(cg_blocks(n)), dim3(kCgThreads), 0, st,
                     reinterpret_cast<const S*>(x), chunks<S>(n), part);
  return hipGetLastError();
}

#define JL_INST(S)                                                                                 \
  template hipError_t launch_cg_init<S>(const cplx<S>*, cplx<S>*, cplx<S>*, cplx<S>*, int64_t,      \
                                        double*, double*, double, int, hipStream_t);               \
  template hipError_t launch_cg_step<S>(cplx<S>*, cplx<S>*, cplx<S>*, const cplx<S>*, int64_t,    \
                                        const double*, int, double*, double*, hipStream_t);        \
  template hipError_t launch_cg_finish<S>(const cplx<S>*, cplx<S>*, const cplx<S>*, int64_t,       \
                                          double*, hipStream_t);                                   \
  template hipError_t launch_norm2<S>(const cplx<S>*, int64_t, double*, hipStream_t);
JL_INST(float)
JL_INST(double)
#undef JL_INST

}  // namespace jl
