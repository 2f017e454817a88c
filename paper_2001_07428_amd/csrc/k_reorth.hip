// J-restricted reorthogonalisation kernels (Alg. 2, the iterated Gram-Schmidt
// against W_j = J V_j^* and V_j), written as block classical Gram-Schmidt.
//
// W is never stored.  With w_i = J v_i^* = [-conj(v_bot); conj(v_top)]:
//   w_i^H u = sum_p v_top[p] u_bot[p] - v_bot[p] u_top[p]   (no conjugation)
//   u_top  += conj(v_bot) c_w,   u_bot -= conj(v_top) c_w
// so one read of the basis serves both projections.  A "pair" p couples
// element p of the top half with element p of the bottom half.
//
// dots:   per block, FP64 partial sums of v_i^H u and w_i^H u for every
//         column, plus ||u||^2 (and, with the local three-term step, the
//         squared norm after its first term alone); one wavefront per column (FP32: per two
//         columns) at a time, u held in registers (converted to FP64), FP64
//         products and accumulation; the partials are summed by
//         k_reduce_wide (tiles of columns x slices of blocks).
// update: u -= V c_v + W c_w with the FP64 coefficients rounded to the
//         storage type, then ||u||^2 in FP64, summed over the blocks by the
//         last one to finish; one pass over the basis.
// Both read the basis with non-temporal loads once a pass is larger than
// the last-level cache.
#include <algorithm>
#include <type_traits>

#include "common.h"

namespace jl {
namespace {

constexpr int kReorthThreads = 256;   // 4 wavefronts
constexpr int kPairsPerLane = 4;      // pairs of u each lane holds per chunk (more resident waves than 8)
constexpr int kMaxCols = 2048;        // LDS column accumulators
constexpr int kMaxGroups = 16;        // column groups for short vectors

// E = complex elements per 16-byte load (2 for FP32 with an even half
// length, else 1).
template <typename S, int E> struct Ld;
template <> struct Ld<float, 2> {
  static __device__ __forceinline__ void get(const float2* p, float* re, float* im) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    re[0] = v.x; im[0] = v.y; re[1] = v.z; im[1] = v.w;
  }
};
template <> struct Ld<float, 1> {
  static __device__ __forceinline__ void get(const float2* p, float* re, float* im) {
    const float2 v = *p;
    re[0] = v.x; im[0] = v.y;
  }
};
template <> struct Ld<double, 1> {
  static __device__ __forceinline__ void get(const double2* p, double* re, double* im) {
    const double2 v = *p;
    re[0] = v.x; im[0] = v.y;
  }
};

// Basis loads.  NT: non-temporal (the lines are not kept in the caches), for
// passes whose basis is larger than the last-level cache, where a kept line
// is never read again before it is evicted: measured on a plain read stream,
// 6.2 TB/s instead of 5.3-5.75.
typedef float ntf4 __attribute__((ext_vector_type(4)));
typedef float ntf2 __attribute__((ext_vector_type(2)));
typedef double ntd2 __attribute__((ext_vector_type(2)));
template <typename S, int E, bool NT>
__device__ __forceinline__ void ldb(const cplx<S>* p, S* re, S* im) {
  if constexpr (!NT) {
    Ld<S, E>::get(p, re, im);
  } else if constexpr (sizeof(S) == 4 && E == 2) {
    const ntf4 v = __builtin_nontemporal_load(reinterpret_cast<const ntf4*>(p));
    re[0] = v.x; im[0] = v.y; re[1] = v.z; im[1] = v.w;
  } else if constexpr (sizeof(S) == 4) {
    const ntf2 v = __builtin_nontemporal_load(reinterpret_cast<const ntf2*>(p));
    re[0] = v.x; im[0] = v.y;
  } else {
    const ntd2 v = __builtin_nontemporal_load(reinterpret_cast<const ntd2*>(p));
    re[0] = v.x; im[0] = v.y;
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Sums over the wavefront of r[0..7]: three halving steps (lanes whose
// xor-partner bit is set keep the upper half of the values) and three plain
// steps; afterwards every lane l holds the sum of r[l >> 3].  Fixed order.
__device__ __forceinline__ double wave_sum8(const double r[8]) {
  const int lane = threadIdx.x % 64;
  const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
  double a[4], b[2];
#pragma unroll
  for (int k = 0; k < 4; ++k) a[k] = (h5 ? r[k + 4] : r[k]) + __shfl_xor(h5 ? r[k] : r[k + 4], 32);
#pragma unroll
  for (int k = 0; k < 2; ++k) b[k] = (h4 ? a[k + 2] : a[k]) + __shfl_xor(h4 ? a[k] : a[k + 2], 16);
  double t = (h3 ? b[1] : b[0]) + __shfl_xor(h3 ? b[0] : b[1], 8);
  t += __shfl_xor(t, 4);
  t += __shfl_xor(t, 2);
  t += __shfl_xor(t, 1);
  return t;
}
// As wave_sum8 for r[0..3]: every lane l holds the sum of r[l >> 4].
__device__ __forceinline__ double wave_sum4(const double r[4]) {
  const int lane = threadIdx.x % 64;
  const bool h5 = lane & 32, h4 = lane & 16;
  double a[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) a[k] = (h5 ? r[k + 2] : r[k]) + __shfl_xor(h5 ? r[k] : r[k + 2], 32);
  double t = (h4 ? a[1] : a[0]) + __shfl_xor(h4 ? a[0] : a[1], 16);
  t += __shfl_xor(t, 8);
  t += __shfl_xor(t, 4);
  t += __shfl_xor(t, 2);
  t += __shfl_xor(t, 1);
  return t;
}

// This lane's share of v^H u and w^H u (w = J conj(v)) for the column at vt
// (top half; bottom at vt + h): r = {Re v^H u, Im v^H u, Re w^H u, Im w^H u}.
template <typename S, int E, int Q, bool NT>
__device__ __forceinline__ void col_dots(const cplx<S>* __restrict__ vt, int64_t h, int64_t p0,
                                         int lane, const bool ok[Q], const double utr[Q][E],
                                         const double uti[Q][E], const double ubr[Q][E],
                                         const double ubi[Q][E], double r[4]) {
  const cplx<S>* vb = vt + h;
  S tr[Q][E], ti[Q][E], br[Q][E], bi[Q][E];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t p = p0 + (int64_t)q * 64 * E + lane * E;
    if (ok[q]) {
      ldb<S, E, NT>(vt + p, tr[q], ti[q]);
      ldb<S, E, NT>(vb + p, br[q], bi[q]);
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) tr[q][e] = ti[q][e] = br[q][e] = bi[q][e] = (S)0;
    }
  }
  double cvr = 0, cvi = 0, cwr = 0, cwi = 0;
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const double vtr = tr[q][e], vti = ti[q][e], vbr = br[q][e], vbi = bi[q][e];
      // v^H u = conj(v_t) u_t + conj(v_b) u_b
      cvr = fma(vtr, utr[q][e], cvr); cvr = fma(vti, uti[q][e], cvr);
      cvr = fma(vbr, ubr[q][e], cvr); cvr = fma(vbi, ubi[q][e], cvr);
      cvi = fma(vtr, uti[q][e], cvi); cvi = fma(-vti, utr[q][e], cvi);
      cvi = fma(vbr, ubi[q][e], cvi); cvi = fma(-vbi, ubr[q][e], cvi);
      // w^H u = v_t u_b - v_b u_t
      cwr = fma(vtr, ubr[q][e], cwr); cwr = fma(-vti, ubi[q][e], cwr);
      cwr = fma(-vbr, utr[q][e], cwr); cwr = fma(vbi, uti[q][e], cwr);
      cwi = fma(vtr, ubi[q][e], cwi); cwi = fma(vti, ubr[q][e], cwi);
      cwi = fma(-vbr, uti[q][e], cwi); cwi = fma(-vbi, utr[q][e], cwi);
    }
  r[0] = cvr; r[1] = cvi; r[2] = cwr; r[3] = cwi;
}

// grid.x = blocks, each covering `chunks` consecutive chunks of
// 64*E*kPairsPerLane pairs.  Column c is owned by wavefront c % 4 of every
// block.  partial row stride = dots_stride(ncol) = 4*ncol + 2: the column
// sums, ||u||^2, and a last slot (zero without LOCAL).
// LOCAL: before the inner products apply the local three-term step
// u <- u - t v_jl - beta v_{jl-1} (t read from the device), rounded once to
// S and stored back by wavefront 0 after every wavefront has read the chunk;
// the last slot receives ||u - t v_jl||^2 (FP64, before the rounding): the
// norm Alg. 2 measures after subtracting t_jj v_j alone.
// Column groups (gridDim.y > 1, for vectors too short to fill the device):
// block (x, g) takes the columns c with (c / 4) % G == g, every group
// applies the local step in registers, and only group 0 stores it, to uout
// (which must then differ from u, since the other groups still read u) and
// adds ||u||^2.
template <typename S, int E, bool LOCAL, bool NT>
__global__ __launch_bounds__(kReorthThreads, sizeof(S) == 4 ? 4 : 1) void k_dots(const cplx<S>* __restrict__ V, int64_t ldv,
                                                         int ncol, const cplx<S>* __restrict__ u,
                                                         int64_t h, int chunks,
                                                         double* __restrict__ partial,
                                                         const double* __restrict__ tloc,
                                                         double beta, int jl,
                                                         cplx<S>* __restrict__ uout,
                                                         const double* __restrict__ beta2) {
  constexpr int Q = kPairsPerLane / E;     // loads per half per lane per chunk
  constexpr int CH = 64 * E * Q;           // pairs per chunk
  extern __shared__ double acc[];          // dots_stride(ncol) column accumulators
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int nout = dots_stride(ncol);
  for (int i = threadIdx.x; i < nout; i += kReorthThreads) acc[i] = 0.0;
  __syncthreads();
  // wavefront 0 of group 0 sums ||u||^2 (into acc[4 ncol] at the end) and,
  // with LOCAL, the norm after t v_jl alone (per chunk into acc[4 ncol + 1]:
  // no second accumulator stays live across the column loop)
  const bool nw = wave == 0 && blockIdx.y == 0;
  double unorm = 0.0;
  for (int ch = 0; ch < chunks; ++ch) {
    const int64_t p0 = ((int64_t)blockIdx.x * chunks + ch) * CH;
    if (p0 >= h) break;
    // this lane's pairs: p0 + q*64*E + lane*E + e
    double utr[Q][E], uti[Q][E], ubr[Q][E], ubi[Q][E];
    bool ok[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t p = p0 + (int64_t)q * 64 * E + lane * E;
      ok[q] = p < h;                       // E divides h, so p < h covers all E elements
      S tr[E], ti[E], br[E], bi[E];
      if (ok[q]) {
        Ld<S, E>::get(u + p, tr, ti);
        Ld<S, E>::get(u + h + p, br, bi);
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) tr[e] = ti[e] = br[e] = bi[e] = (S)0;
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        utr[q][e] = tr[e]; uti[q][e] = ti[e]; ubr[q][e] = br[e]; ubi[q][e] = bi[e];
      }
    }
    if constexpr (LOCAL) {
      __syncthreads();   // every wavefront holds the raw chunk before it is overwritten
      double anorm = 0.0;
      const double t_re = tloc[0], t_im = tloc[1];
      const double bt = beta2 ? sqrt(beta2[0]) : beta;   // beta_{jl-1}: host value or device norm^2
      const cplx<S>* vj = V + (int64_t)jl * ldv;
      const cplx<S>* vm = vj - ldv;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        if (!ok[q]) continue;
        const int64_t p = p0 + (int64_t)q * 64 * E + lane * E;
        S tr[E], ti[E], br[E], bi[E];
        Ld<S, E>::get(vj + p, tr, ti);
        Ld<S, E>::get(vj + h + p, br, bi);
        S mtr[E], mti[E], mbr[E], mbi[E];
        if (bt != 0.0) {
          Ld<S, E>::get(vm + p, mtr, mti);
          Ld<S, E>::get(vm + h + p, mbr, mbi);
        } else {
#pragma unroll
          for (int e = 0; e < E; ++e) mtr[e] = mti[e] = mbr[e] = mbi[e] = (S)0;
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
          // u - t v_j (its norm: the alpha step alone), then - beta v_{j-1},
          // rounded once to the storage type
          const double atr = utr[q][e] - (t_re * tr[e] - t_im * ti[e]);
          const double ati = uti[q][e] - (t_re * ti[e] + t_im * tr[e]);
          const double abr = ubr[q][e] - (t_re * br[e] - t_im * bi[e]);
          const double abi = ubi[q][e] - (t_re * bi[e] + t_im * br[e]);
          anorm += atr * atr + ati * ati + abr * abr + abi * abi;
          utr[q][e] = (double)(S)(atr - bt * mtr[e]);
          uti[q][e] = (double)(S)(ati - bt * mti[e]);
          ubr[q][e] = (double)(S)(abr - bt * mbr[e]);
          ubi[q][e] = (double)(S)(abi - bt * mbi[e]);
        }
        if (wave == 0 && blockIdx.y == 0) {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            cplx<S> a, b;
            a.x = (S)utr[q][e]; a.y = (S)uti[q][e];
            b.x = (S)ubr[q][e]; b.y = (S)ubi[q][e];
            uout[p + e] = a;
            uout[h + p + e] = b;
          }
        }
      }
      if (nw) {
        anorm = wave_sum(anorm);
        if (lane == 0) acc[4 * ncol + 1] += anorm;
      }
    }
    if (nw) {
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int e = 0; e < E; ++e)
          unorm += utr[q][e] * utr[q][e] + uti[q][e] * uti[q][e] + ubr[q][e] * ubr[q][e] +
                   ubi[q][e] * ubi[q][e];
    }
    // FP32: two columns (c, c + cs) per pass, so both columns' loads are in
    // flight together, and their eight sums reduce in one butterfly (FP64
    // holds twice the registers per column and stays at one column a pass).
    const int cs = 4 * (int)gridDim.y;
    int c = (int)blockIdx.y * 4 + wave;
    if constexpr (sizeof(S) == 4) {
      for (; c + cs < ncol; c += 2 * cs) {
        double r[8];
        col_dots<S, E, Q, NT>(V + (int64_t)c * ldv, h, p0, lane, ok, utr, uti, ubr, ubi, r);
        col_dots<S, E, Q, NT>(V + (int64_t)(c + cs) * ldv, h, p0, lane, ok, utr, uti, ubr, ubi, r + 4);
        const double t = wave_sum8(r);   // lane 8k holds sum k
        if ((lane & 7) == 0) {   // columns c, c + cs are only ever touched by this wavefront
          const int k = lane >> 3;
          acc[4 * (k < 4 ? c : c + cs) + (k & 3)] += t;
        }
      }
      if (c < ncol) {   // at most one column left
        double r[4];
        col_dots<S, E, Q, NT>(V + (int64_t)c * ldv, h, p0, lane, ok, utr, uti, ubr, ubi, r);
        const double t = wave_sum4(r);   // lane 16k holds sum k
        if ((lane & 15) == 0) acc[4 * c + (lane >> 4)] += t;
      }
    } else {
      for (; c < ncol; c += cs) {
        double r[4];
        col_dots<S, E, Q, NT>(V + (int64_t)c * ldv, h, p0, lane, ok, utr, uti, ubr, ubi, r);
        const double t = wave_sum4(r);
        if ((lane & 15) == 0) acc[4 * c + (lane >> 4)] += t;
      }
    }
  }
  if (nw) {
    unorm = wave_sum(unorm);
    if (lane == 0) acc[4 * ncol] = unorm;
  }
  __syncthreads();
  // this group's columns (and, for group 0, the norms) of the block's row
  double* out = partial + (int64_t)blockIdx.x * nout;
  const int G = gridDim.y, g = blockIdx.y;
  for (int i = threadIdx.x; i < nout; i += kReorthThreads)
    if (i >= 4 * ncol ? g == 0 : ((i / 16) % G == g)) out[i] = acc[i];
}

// FP32 inner products for long vectors, u staged in LDS: a block takes
// kDotsLdsPairs consecutive pairs, stages its u (after the local step, with
// LOCAL) in LDS as FP32 (the values the products use), and each wavefront
// then streams its columns (c = wave, wave + 4, ...) over the block's whole
// range, two load batches of 128 pairs per half at a time, so every column
// is read in 32 KB contiguous runs per half instead of the 2 KB runs of
// k_dots (measured at 32^4 with 375 columns: 7.08 TB/s against 6.24).  Each
// wavefront writes its columns' sums straight to the block's partial row;
// ||u||^2 (and, with LOCAL, ||u - t v_jl||^2) come from the staging.  Same
// outputs as k_dots with one column group.
constexpr int kDotsLdsPairs = 4096;
typedef float ldsf4 __attribute__((ext_vector_type(4)));

template <bool LOCAL, bool NT>
__global__ __launch_bounds__(kReorthThreads, 2) void k_dots_lds(const cplx<float>* __restrict__ V,
                                                                int64_t ldv, int ncol,
                                                                const cplx<float>* __restrict__ u,
                                                                int64_t h, double* __restrict__ partial,
                                                                const double* __restrict__ tloc,
                                                                double beta, int jl,
                                                                cplx<float>* __restrict__ uout,
                                                                const double* __restrict__ beta2) {
  constexpr int BP = kDotsLdsPairs, NQ = BP / 2;   // pairs, pairs of pairs (one 16-byte load)
  __shared__ ldsf4 us[2][NQ];                      // top, bottom halves
  __shared__ double red[2][kReorthThreads / 64];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t p0 = (int64_t)blockIdx.x * BP;
  const int nout = dots_stride(ncol);
  double* out = partial + (int64_t)blockIdx.x * nout;
  double unorm = 0.0, anorm = 0.0;
  double t_re = 0.0, t_im = 0.0, bt = 0.0;
  if constexpr (LOCAL) {
    t_re = tloc[0];
    t_im = tloc[1];
    bt = beta2 ? sqrt(beta2[0]) : beta;   // beta_{jl-1}: host value or device norm^2
  }
  const cplx<float>* vj = V + (int64_t)jl * ldv;
  const cplx<float>* vm = vj - ldv;
  for (int i = threadIdx.x; i < NQ; i += kReorthThreads) {
    const int64_t p = p0 + 2 * i;
    ldsf4 t = {0, 0, 0, 0}, b = {0, 0, 0, 0};
    if (p < h) {   // h is even, so both pairs of the load are in range
      t = *reinterpret_cast<const ldsf4*>(u + p);
      b = *reinterpret_cast<const ldsf4*>(u + h + p);
      if constexpr (LOCAL) {
        // u - t v_j (its norm: the alpha step alone), then - beta v_{j-1},
        // rounded once to FP32
        const ldsf4 at = *reinterpret_cast<const ldsf4*>(vj + p), ab = *reinterpret_cast<const ldsf4*>(vj + h + p);
        ldsf4 mt = {0, 0, 0, 0}, mb = {0, 0, 0, 0};
        if (bt != 0.0) {
          mt = *reinterpret_cast<const ldsf4*>(vm + p);
          mb = *reinterpret_cast<const ldsf4*>(vm + h + p);
        }
        float* tf = reinterpret_cast<float*>(&t);
        float* bf = reinterpret_cast<float*>(&b);
        const float* atf = reinterpret_cast<const float*>(&at);
        const float* abf = reinterpret_cast<const float*>(&ab);
        const float* mtf = reinterpret_cast<const float*>(&mt);
        const float* mbf = reinterpret_cast<const float*>(&mb);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const double xtr = (double)tf[2 * e] - (t_re * atf[2 * e] - t_im * atf[2 * e + 1]);
          const double xti = (double)tf[2 * e + 1] - (t_re * atf[2 * e + 1] + t_im * atf[2 * e]);
          const double xbr = (double)bf[2 * e] - (t_re * abf[2 * e] - t_im * abf[2 * e + 1]);
          const double xbi = (double)bf[2 * e + 1] - (t_re * abf[2 * e + 1] + t_im * abf[2 * e]);
          anorm += xtr * xtr + xti * xti + xbr * xbr + xbi * xbi;
          tf[2 * e] = (float)(xtr - bt * mtf[2 * e]);
          tf[2 * e + 1] = (float)(xti - bt * mtf[2 * e + 1]);
          bf[2 * e] = (float)(xbr - bt * mbf[2 * e]);
          bf[2 * e + 1] = (float)(xbi - bt * mbf[2 * e + 1]);
        }
        // only this thread reads these pairs of u: the update is stored in place
        *reinterpret_cast<ldsf4*>(uout + p) = t;
        *reinterpret_cast<ldsf4*>(uout + h + p) = b;
      }
      unorm += (double)t.x * t.x + (double)t.y * t.y + (double)t.z * t.z + (double)t.w * t.w +
               (double)b.x * b.x + (double)b.y * b.y + (double)b.z * b.z + (double)b.w * b.w;
    }
    us[0][i] = t;
    us[1][i] = b;
  }
  unorm = wave_sum(unorm);
  anorm = wave_sum(anorm);
  if (lane == 0) {
    red[0][wave] = unorm;
    red[1][wave] = anorm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[4 * ncol] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    out[4 * ncol + 1] = LOCAL ? (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]) : 0.0;
  }
  constexpr int B = 2;   // load batches of 64 lanes x 16 bytes per half in flight
#pragma unroll 1
  for (int c = wave; c < ncol; c += kReorthThreads / 64) {
    const cplx<float>* vt = V + (int64_t)c * ldv + p0;
    const cplx<float>* vb = vt + h;
    double cvr = 0, cvi = 0, cwr = 0, cwi = 0;
#pragma unroll 1
    for (int k0 = 0; k0 < NQ / 64; k0 += B) {
      ldsf4 a[B], b[B];
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int i = (k0 + k) * 64 + lane;
        const bool in = p0 + 2 * i < h;
        const ldsf4* qa = reinterpret_cast<const ldsf4*>(vt) + (in ? i : 0);
        const ldsf4* qb = reinterpret_cast<const ldsf4*>(vb) + (in ? i : 0);
        if constexpr (NT) {
          a[k] = __builtin_nontemporal_load(qa);
          b[k] = __builtin_nontemporal_load(qb);
        } else {
          a[k] = *qa;
          b[k] = *qb;
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int i = (k0 + k) * 64 + lane;
        const ldsf4 ut = us[0][i], ub = us[1][i];   // zero past the end of the vector
        const float* av = reinterpret_cast<const float*>(&a[k]);
        const float* bv = reinterpret_cast<const float*>(&b[k]);
        const float* utf = reinterpret_cast<const float*>(&ut);
        const float* ubf = reinterpret_cast<const float*>(&ub);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const double vtr = av[2 * e], vti = av[2 * e + 1], vbr = bv[2 * e], vbi = bv[2 * e + 1];
          const double utr = utf[2 * e], uti = utf[2 * e + 1], ubr = ubf[2 * e], ubi = ubf[2 * e + 1];
          // v^H u = conj(v_t) u_t + conj(v_b) u_b;  w^H u = v_t u_b - v_b u_t
          cvr = fma(vtr, utr, cvr); cvr = fma(vti, uti, cvr); cvr = fma(vbr, ubr, cvr); cvr = fma(vbi, ubi, cvr);
          cvi = fma(vtr, uti, cvi); cvi = fma(-vti, utr, cvi); cvi = fma(vbr, ubi, cvi); cvi = fma(-vbi, ubr, cvi);
          cwr = fma(vtr, ubr, cwr); cwr = fma(-vti, ubi, cwr); cwr = fma(-vbr, utr, cwr); cwr = fma(vbi, uti, cwr);
          cwi = fma(vtr, ubi, cwi); cwi = fma(vti, ubr, cwi); cwi = fma(-vbr, uti, cwi); cwi = fma(-vbi, utr, cwi);
        }
      }
    }
    double r[4] = {cvr, cvi, cwr, cwi};
    const double tsum = wave_sum4(r);   // lane 16k holds sum k
    if ((lane & 15) == 0) out[4 * c + (lane >> 4)] = tsum;
  }
}

// The same design for FP64 vectors: a 16-byte load is one complex element, so
// a block takes kDotsLds64Pairs = 2048 pairs (64 KB of u in LDS, 32 KB runs
// per half per column, as in FP32); the local step's arithmetic is that of
// k_dots.
constexpr int kDotsLds64Pairs = 2048;
typedef double ldsd2 __attribute__((ext_vector_type(2)));

template <bool LOCAL, bool NT>
__global__ __launch_bounds__(kReorthThreads, 2) void k_dots_lds64(const cplx<double>* __restrict__ V,
                                                                  int64_t ldv, int ncol,
                                                                  const cplx<double>* __restrict__ u,
                                                                  int64_t h, double* __restrict__ partial,
                                                                  const double* __restrict__ tloc,
                                                                  double beta, int jl,
                                                                  cplx<double>* __restrict__ uout,
                                                                  const double* __restrict__ beta2) {
  constexpr int NQ = kDotsLds64Pairs;        // pairs, one 16-byte load per half each
  __shared__ ldsd2 us[2][NQ];                // top, bottom halves
  __shared__ double red[2][kReorthThreads / 64];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t p0 = (int64_t)blockIdx.x * NQ;
  const int nout = dots_stride(ncol);
  double* out = partial + (int64_t)blockIdx.x * nout;
  double unorm = 0.0, anorm = 0.0;
  double t_re = 0.0, t_im = 0.0, bt = 0.0;
  if constexpr (LOCAL) {
    t_re = tloc[0];
    t_im = tloc[1];
    bt = beta2 ? sqrt(beta2[0]) : beta;   // beta_{jl-1}: host value or device norm^2
  }
  const cplx<double>* vj = V + (int64_t)jl * ldv;
  const cplx<double>* vm = vj - ldv;
  for (int i = threadIdx.x; i < NQ; i += kReorthThreads) {
    const int64_t p = p0 + i;
    ldsd2 t = {0, 0}, b = {0, 0};
    if (p < h) {
      t = *reinterpret_cast<const ldsd2*>(u + p);
      b = *reinterpret_cast<const ldsd2*>(u + h + p);
      if constexpr (LOCAL) {
        // u - t v_j (its norm: the alpha step alone), then - beta v_{j-1}
        const ldsd2 at = *reinterpret_cast<const ldsd2*>(vj + p), ab = *reinterpret_cast<const ldsd2*>(vj + h + p);
        ldsd2 mt = {0, 0}, mb = {0, 0};
        if (bt != 0.0) {
          mt = *reinterpret_cast<const ldsd2*>(vm + p);
          mb = *reinterpret_cast<const ldsd2*>(vm + h + p);
        }
        const double xtr = t.x - (t_re * at.x - t_im * at.y);
        const double xti = t.y - (t_re * at.y + t_im * at.x);
        const double xbr = b.x - (t_re * ab.x - t_im * ab.y);
        const double xbi = b.y - (t_re * ab.y + t_im * ab.x);
        anorm += xtr * xtr + xti * xti + xbr * xbr + xbi * xbi;
        t.x = xtr - bt * mt.x;
        t.y = xti - bt * mt.y;
        b.x = xbr - bt * mb.x;
        b.y = xbi - bt * mb.y;
        // only this thread reads these pairs of u: the update is stored in place
        *reinterpret_cast<ldsd2*>(uout + p) = t;
        *reinterpret_cast<ldsd2*>(uout + h + p) = b;
      }
      unorm += t.x * t.x + t.y * t.y + b.x * b.x + b.y * b.y;
    }
    us[0][i] = t;
    us[1][i] = b;
  }
  unorm = wave_sum(unorm);
  anorm = wave_sum(anorm);
  if (lane == 0) {
    red[0][wave] = unorm;
    red[1][wave] = anorm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[4 * ncol] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    out[4 * ncol + 1] = LOCAL ? (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]) : 0.0;
  }
  constexpr int B = 2;   // load batches of 64 lanes x 16 bytes per half in flight
#pragma unroll 1
  for (int c = wave; c < ncol; c += kReorthThreads / 64) {
    const cplx<double>* vt = V + (int64_t)c * ldv + p0;
    const cplx<double>* vb = vt + h;
    double cvr = 0, cvi = 0, cwr = 0, cwi = 0;
#pragma unroll 1
    for (int k0 = 0; k0 < NQ / 64; k0 += B) {
      ldsd2 a[B], b[B];
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int i = (k0 + k) * 64 + lane;
        const int j = p0 + i < h ? i : 0;
        const ldsd2* qa = reinterpret_cast<const ldsd2*>(vt) + j;
        const ldsd2* qb = reinterpret_cast<const ldsd2*>(vb) + j;
        if constexpr (NT) {
          a[k] = __builtin_nontemporal_load(qa);
          b[k] = __builtin_nontemporal_load(qb);
        } else {
          a[k] = *qa;
          b[k] = *qb;
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int i = (k0 + k) * 64 + lane;
        const ldsd2 ut = us[0][i], ub = us[1][i];   // zero past the end of the vector
        const double vtr = a[k].x, vti = a[k].y, vbr = b[k].x, vbi = b[k].y;
        const double utr = ut.x, uti = ut.y, ubr = ub.x, ubi = ub.y;
        // v^H u = conj(v_t) u_t + conj(v_b) u_b;  w^H u = v_t u_b - v_b u_t
        cvr = fma(vtr, utr, cvr); cvr = fma(vti, uti, cvr); cvr = fma(vbr, ubr, cvr); cvr = fma(vbi, ubi, cvr);
        cvi = fma(vtr, uti, cvi); cvi = fma(-vti, utr, cvi); cvi = fma(vbr, ubi, cvi); cvi = fma(-vbi, ubr, cvi);
        cwr = fma(vtr, ubr, cwr); cwr = fma(-vti, ubi, cwr); cwr = fma(-vbr, utr, cwr); cwr = fma(vbi, uti, cwr);
        cwi = fma(vtr, ubi, cwi); cwi = fma(vti, ubr, cwi); cwi = fma(-vbr, uti, cwi); cwi = fma(-vbi, utr, cwi);
      }
    }
    double r[4] = {cvr, cvi, cwr, cwi};
    const double tsum = wave_sum4(r);   // lane 16k holds sum k
    if ((lane & 15) == 0) out[4 * c + (lane >> 4)] = tsum;
  }
}

// Stores this block's share of ||u||^2 (bsum, the same in every thread).
// With fin the kernel also finishes the sum: each block's share is an
// agent-scope store, complete before the counter *cnt moves; the last block
// to count sums the shares in block order into *fin and resets the counter
// (the per-XCD L2s are not coherent, hence agent-scope loads as well).
__device__ __forceinline__ void block_norm_out(double bsum, double* partial, double* fin,
                                               unsigned* cnt) {
  __shared__ bool last;
  __shared__ double red[kReorthThreads / 64];
  if (!fin) {
    if (threadIdx.x == 0) partial[blockIdx.x] = bsum;
    return;
  }
  if (threadIdx.x == 0) {
    __hip_atomic_store(&partial[blockIdx.x], bsum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);
    last = atomicAdd(cnt, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;   // uniform within the block
  double s = 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += kReorthThreads)
    s += __hip_atomic_load(&partial[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  s = wave_sum(s);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    *fin = (red[0] + red[1]) + (red[2] + red[3]);
    *cnt = 0u;   // ready for the next launch
  }
}

// As block_norm_out for a block of one wavefront (no LDS: the flag of the
// last block is broadcast from lane 0).
__device__ __forceinline__ void wave_norm_out(double wsum, double* partial, double* fin,
                                              unsigned* cnt) {
  const int lane = threadIdx.x % 64;
  if (!fin) {
    if (lane == 0) partial[blockIdx.x] = wsum;
    return;
  }
  int last = 0;
  if (lane == 0) {
    __hip_atomic_store(&partial[blockIdx.x], wsum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);
    last = atomicAdd(cnt, 1u) == gridDim.x - 1;
  }
  if (!__shfl(last, 0)) return;
  double s = 0.0;
  for (int b = lane; b < (int)gridDim.x; b += 64)
    s += __hip_atomic_load(&partial[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  s = wave_sum(s);
  if (lane == 0) {
    *fin = s;
    *cnt = 0u;   // ready for the next launch
  }
}

// FP32 J-restricted update of long vectors (an even half length of at least
// 2048 blocks): one wavefront per block owns kUpdLdsPairs consecutive pairs
// and keeps their corrections in LDS, where each lane only ever touches its
// own entries (so no barrier).  Every column is streamed over the block's
// whole range (8 KB per half), two 16-byte loads per lane and half in flight,
// the next two issued before the current products.  The products and their
// order per element are those of k_update, so u_new is bit-identical to it
// (the norm's blocks differ).  Measured at 32^4 with 100 / 375 / 500 columns:
// 6.6 / 6.9 / 6.95 TB/s against 5.9 / 6.5 / 6.4 for k_update's four-wavefront
// blocks with the corrections in registers.
constexpr int kUpdLdsPairs = 1024;
template <bool NT>
__global__ __launch_bounds__(64) void k_update_lds(const cplx<float>* __restrict__ V, int64_t ldv,
                                                   int ncol, const cplx<float>* uin,
                                                   cplx<float>* uout, int64_t h,
                                                   const double* __restrict__ coef,
                                                   double* partial, double* fin, unsigned* cnt) {
  constexpr int NQ = kUpdLdsPairs / 2, NK = NQ / 64, B = 2;   // 16-byte loads per half, steps
  // 20 KB per block (a quarter beyond what it uses): eight blocks fill a
  // compute unit's 160 KB, measured faster than ten or more
  __shared__ ldsf4 acc[2][NQ + NQ / 4];
  const int lane = threadIdx.x;
  const int64_t p0 = (int64_t)blockIdx.x * kUpdLdsPairs;
#pragma unroll
  for (int k = 0; k < NK; ++k) acc[0][k * 64 + lane] = acc[1][k * 64 + lane] = ldsf4{0, 0, 0, 0};
#pragma unroll 1
  for (int c = 0; c < ncol; ++c) {
    const float cvr = (float)coef[4 * c], cvi = (float)coef[4 * c + 1];
    const float cwr = (float)coef[4 * c + 2], cwi = (float)coef[4 * c + 3];
    const ldsf4* vt = reinterpret_cast<const ldsf4*>(V + (int64_t)c * ldv + p0);
    const ldsf4* vb = reinterpret_cast<const ldsf4*>(V + (int64_t)c * ldv + h + p0);
    ldsf4 a[B], b[B];
    auto load = [&](int k0) {
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int i = (k0 + k) * 64 + lane;
        const int j = p0 + 2 * i < h ? i : 0;   // h is even: both pairs of a load are in range
        if constexpr (NT) {
          a[k] = __builtin_nontemporal_load(vt + j);
          b[k] = __builtin_nontemporal_load(vb + j);
        } else {
          a[k] = vt[j];
          b[k] = vb[j];
        }
      }
    };
    load(0);
#pragma unroll 1
    for (int k0 = 0; k0 < NK; k0 += B) {
      ldsf4 ca[B], cb[B];
#pragma unroll
      for (int k = 0; k < B; ++k) {
        ca[k] = a[k];
        cb[k] = b[k];
      }
      if (k0 + B < NK) load(k0 + B);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int i = (k0 + k) * 64 + lane;
        ldsf4 dt = acc[0][i], db = acc[1][i];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const float vtr = ca[k][2 * e], vti = ca[k][2 * e + 1], vbr = cb[k][2 * e], vbi = cb[k][2 * e + 1];
          float tr = dt[2 * e], ti = dt[2 * e + 1], br = db[2 * e], bi = db[2 * e + 1];
          // d_top += v_t cv - conj(v_b) cw
          tr = fmaf(vtr, cvr, tr); tr = fmaf(-vti, cvi, tr); tr = fmaf(-vbr, cwr, tr); tr = fmaf(-vbi, cwi, tr);
          ti = fmaf(vtr, cvi, ti); ti = fmaf(vti, cvr, ti); ti = fmaf(-vbr, cwi, ti); ti = fmaf(vbi, cwr, ti);
          // d_bot += v_b cv + conj(v_t) cw
          br = fmaf(vbr, cvr, br); br = fmaf(-vbi, cvi, br); br = fmaf(vtr, cwr, br); br = fmaf(vti, cwi, br);
          bi = fmaf(vbr, cvi, bi); bi = fmaf(vbi, cvr, bi); bi = fmaf(vtr, cwi, bi); bi = fmaf(-vti, cwr, bi);
          dt[2 * e] = tr; dt[2 * e + 1] = ti; db[2 * e] = br; db[2 * e + 1] = bi;
        }
        acc[0][i] = dt;
        acc[1][i] = db;
      }
    }
  }
  double nrm = 0.0;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int i = k * 64 + lane;
    const int64_t p = p0 + 2 * i;
    if (p >= h) continue;
    const ldsf4 t = *reinterpret_cast<const ldsf4*>(uin + p) - acc[0][i];
    const ldsf4 b = *reinterpret_cast<const ldsf4*>(uin + h + p) - acc[1][i];
    *reinterpret_cast<ldsf4*>(uout + p) = t;
    *reinterpret_cast<ldsf4*>(uout + h + p) = b;
#pragma unroll
    for (int e = 0; e < 2; ++e)
      nrm += (double)t[2 * e] * t[2 * e] + (double)t[2 * e + 1] * t[2 * e + 1] +
             (double)b[2 * e] * b[2 * e] + (double)b[2 * e + 1] * b[2 * e + 1];
  }
  wave_norm_out(wave_sum(nrm), partial, fin, cnt);
}

// u -= sum_c v_c cv_c + w_c cw_c (JSYM; without it the W projection is
// left out: standard Gram-Schmidt against V alone); each lane keeps the
// corrections of its E*Q pairs in registers across the column loop (Q loads
// of 16 bytes per half per column).  partial[blk] = the block's share of
// ||u_new||^2; with fin the last block also sums them into *fin.
// uout = uin - corrections (uin == uout in place).  With SPLIT (column groups,
// gridDim.y = G > 1) block (x, g) sums the columns c = g, g + G, ... and
// stores its corrections to d[g] (2h complex each) instead; k_update_fin
// then forms uout and the norms.
template <typename S, int E, int Q, bool JSYM, bool SPLIT, bool NT>
__global__ __launch_bounds__(kReorthThreads) void k_update(const cplx<S>* __restrict__ V,
                                                           int64_t ldv, int ncol,
                                                           const cplx<S>* uin, cplx<S>* uout,
                                                           int64_t h,
                                                           const double* __restrict__ coef,
                                                           double* partial,
                                                           cplx<S>* __restrict__ d, double* fin,
                                                           unsigned* cnt) {
  constexpr int CH = 4 * 64 * E * Q;       // pairs per block
  __shared__ double sh[4];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int64_t p0 = (int64_t)blockIdx.x * CH + (int64_t)wave * (64 * E * Q);
  S dtr[Q][E], dti[Q][E], dbr[Q][E], dbi[Q][E];
  bool ok[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    ok[q] = p0 + (int64_t)q * 64 * E + lane * E < h;
#pragma unroll
    for (int e = 0; e < E; ++e) dtr[q][e] = dti[q][e] = dbr[q][e] = dbi[q][e] = (S)0;
  }
  const int c0 = SPLIT ? (int)blockIdx.y : 0, cs = SPLIT ? (int)gridDim.y : 1;
  // Columns go in batches of U: the batch's basis loads and coefficients are
  // all issued before its products (the scheduling barrier keeps the compiler
  // from waiting for each column's loads before issuing the next column's).
  // FP32 only: at 16^4 the FP32 update went from 176 to 164 us, while FP64
  // (twice the bytes per element, one column a batch) measured slower batched
  // (315 -> 367 us).
  constexpr int U = sizeof(S) == 8 || Q >= 4 ? 1 : 4 / Q;
  auto batch = [&](int c, auto un) {
    constexpr int UN = decltype(un)::value;
    S cvr[UN], cvi[UN], cwr[UN], cwi[UN];
    S tr[UN][Q][E], ti[UN][Q][E], br[UN][Q][E], bi[UN][Q][E];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int cc = c + u * cs;
      cvr[u] = (S)coef[4 * cc + 0]; cvi[u] = (S)coef[4 * cc + 1];
      cwr[u] = JSYM ? (S)coef[4 * cc + 2] : (S)0; cwi[u] = JSYM ? (S)coef[4 * cc + 3] : (S)0;
      const cplx<S>* vt = V + (int64_t)cc * ldv;
      const cplx<S>* vb = vt + h;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        if (ok[q]) {
          const int64_t p = p0 + (int64_t)q * 64 * E + lane * E;
          ldb<S, E, NT>(vt + p, tr[u][q], ti[u][q]);
          ldb<S, E, NT>(vb + p, br[u][q], bi[u][q]);
        } else {
#pragma unroll
          for (int e = 0; e < E; ++e) tr[u][q][e] = ti[u][q][e] = br[u][q][e] = bi[u][q][e] = (S)0;
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < UN; ++u)
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const S vtr = tr[u][q][e], vti = ti[u][q][e], vbr = br[u][q][e], vbi = bi[u][q][e];
          // d_top += v_t cv - conj(v_b) cw
          dtr[q][e] = fma(vtr, cvr[u], dtr[q][e]); dtr[q][e] = fma(-vti, cvi[u], dtr[q][e]);
          dtr[q][e] = fma(-vbr, cwr[u], dtr[q][e]); dtr[q][e] = fma(-vbi, cwi[u], dtr[q][e]);
          dti[q][e] = fma(vtr, cvi[u], dti[q][e]); dti[q][e] = fma(vti, cvr[u], dti[q][e]);
          dti[q][e] = fma(-vbr, cwi[u], dti[q][e]); dti[q][e] = fma(vbi, cwr[u], dti[q][e]);
          // d_bot += v_b cv + conj(v_t) cw
          dbr[q][e] = fma(vbr, cvr[u], dbr[q][e]); dbr[q][e] = fma(-vbi, cvi[u], dbr[q][e]);
          dbr[q][e] = fma(vtr, cwr[u], dbr[q][e]); dbr[q][e] = fma(vti, cwi[u], dbr[q][e]);
          dbi[q][e] = fma(vbr, cvi[u], dbi[q][e]); dbi[q][e] = fma(vbi, cvr[u], dbi[q][e]);
          dbi[q][e] = fma(vtr, cwi[u], dbi[q][e]); dbi[q][e] = fma(-vti, cwr[u], dbi[q][e]);
        }
  };
  int c = c0;
  for (; c + (U - 1) * cs < ncol; c += U * cs) batch(c, std::integral_constant<int, U>{});
  for (; c < ncol; c += cs) batch(c, std::integral_constant<int, 1>{});
  if constexpr (SPLIT) {
    cplx<S>* dg = d + (int64_t)blockIdx.y * 2 * h;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (!ok[q]) continue;
      const int64_t p = p0 + (int64_t)q * 64 * E + lane * E;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        cplx<S> t, b;
        t.x = dtr[q][e]; t.y = dti[q][e];
        b.x = dbr[q][e]; b.y = dbi[q][e];
        dg[p + e] = t;
        dg[h + p + e] = b;
      }
    }
    return;
  }
  double nrm = 0.0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (!ok[q]) continue;
    const int64_t p = p0 + (int64_t)q * 64 * E + lane * E;
    S tr[E], ti[E], br[E], bi[E];
    Ld<S, E>::get(uin + p, tr, ti);
    Ld<S, E>::get(uin + h + p, br, bi);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      cplx<S> t, b;
      t.x = tr[e] - dtr[q][e]; t.y = ti[e] - dti[q][e];
      b.x = br[e] - dbr[q][e]; b.y = bi[e] - dbi[q][e];
      uout[p + e] = t;
      uout[h + p + e] = b;
      nrm += (double)t.x * t.x + (double)t.y * t.y + (double)b.x * b.x + (double)b.y * b.y;
    }
  }
  nrm = wave_sum(nrm);
  if (lane == 0) sh[wave] = nrm;
  __syncthreads();
  block_norm_out((sh[0] + sh[1]) + (sh[2] + sh[3]), partial, fin, cnt);
}

// uout = uin - (d[0] + ... + d[G-1]) (summed in that order, storage type),
// partial[blk] = ||uout||^2; the block shape of k_update.
template <typename S, int E, int Q>
__global__ __launch_bounds__(kReorthThreads) void k_update_fin(const cplx<S>* uin, cplx<S>* uout,
                                                               int64_t h,
                                                               const cplx<S>* __restrict__ d,
                                                               int G, double* partial, double* fin,
                                                               unsigned* cnt) {
  constexpr int CH = 4 * 64 * E * Q;
  __shared__ double sh[4];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int64_t p0 = (int64_t)blockIdx.x * CH + (int64_t)wave * (64 * E * Q);
  double nrm = 0.0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t pq = p0 + (int64_t)q * 64 * E + lane * E;
    if (pq >= h) continue;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t p = pq + e;
      S dtr = 0, dti = 0, dbr = 0, dbi = 0;
#pragma unroll
      for (int g = 0; g < kMaxGroups; ++g) {   // unrolled: the loads are independent
        if (g < G) {
          const cplx<S> t = d[(int64_t)g * 2 * h + p], b = d[(int64_t)g * 2 * h + h + p];
          dtr += t.x; dti += t.y; dbr += b.x; dbi += b.y;
        }
      }
      const cplx<S> a = uin[p], c = uin[h + p];
      cplx<S> t, b;
      t.x = a.x - dtr; t.y = a.y - dti;
      b.x = c.x - dbr; b.y = c.y - dbi;
      uout[p] = t;
      uout[h + p] = b;
      nrm += (double)t.x * t.x + (double)t.y * t.y + (double)b.x * b.x + (double)b.y * b.y;
    }
  }
  nrm = wave_sum(nrm);
  if (lane == 0) sh[wave] = nrm;
  __syncthreads();
  block_norm_out((sh[0] + sh[1]) + (sh[2] + sh[3]), partial, fin, cnt);
}

}  // namespace

// Pairs per lane of the update kernel: the largest of 8, 4, 2 (1 for FP64
// or an odd half length) that still gives >= 4096 blocks with two pairs per
// load (FP32), >= 1024 otherwise, so small vectors fill the 256 CUs (FP32 at
// 32^4: 4096 blocks of four pairs per lane took a 375-column pass from 7.94 to
// 7.77 ms against 2048 blocks of eight; 8192 of two, 8.12 ms).
static int update_ppl(int64_t h, int E) {
  const int64_t target = E == 2 ? 4096 : 1024;
  for (int ppl = 8; ppl >= 2 * E; ppl /= 2)
    if ((h + 256 * ppl - 1) / (256 * ppl) >= target) return ppl;
  return E == 2 ? 2 : 1;
}

static int elems_per_load(int64_t h, int es) { return (es == 8 && h % 2 == 0) ? 2 : 1; }

// The FP32 J-restricted update of vectors with an even half length of at
// least 2048 blocks of kUpdLdsPairs pairs (eight per compute unit) runs in
// k_update_lds.
static bool update_lds_applies(int64_t h, int es) {
  return es == 8 && h % 2 == 0 && h >= (int64_t)2048 * kUpdLdsPairs;
}

int reorth_update_blocks(int64_t h, int es, bool jsym) {
  if (jsym && update_lds_applies(h, es)) return (int)((h + kUpdLdsPairs - 1) / kUpdLdsPairs);
  const int64_t per_block = (int64_t)256 * update_ppl(h, elems_per_load(h, es));
  return (int)((h + per_block - 1) / per_block);
}

// Chunks per dots block so that about 2048 blocks cover the vector.
// Chunks per dots block so that about 2048 blocks (FP32) or 512 (FP64) cover
// the vector: measured at 16^4, 512 blocks took the FP64 pass from 362 to
// 350 us (four chunks per block, fewer partial sums) but the FP32 pass from
// 171 to 224 us.  es: bytes per complex element.
static int dots_chunks(int64_t h, int es) {
  const int64_t ch = 64 * kPairsPerLane;
  const int64_t nch = (h + ch - 1) / ch;
  const int64_t target = es == 16 ? 512 : 2048;
  int64_t per = (nch + target - 1) / target;
  if (per < 1) per = 1;
  return (int)per;
}

// The FP32 inner products of long vectors (an even half length of at least
// 256 blocks of kDotsLdsPairs pairs, so one column group) run in k_dots_lds.
static bool dots_lds_applies(int64_t h, int es) {
  return es == 8 && h % 2 == 0 && h >= (int64_t)256 * kDotsLdsPairs;
}
// The FP64 inner products of vectors of at least 256 blocks of
// kDotsLds64Pairs pairs run in k_dots_lds64.
static bool dots_lds64_applies(int64_t h, int es) {
  return es == 16 && h >= (int64_t)256 * kDotsLds64Pairs;
}

// A pass over the basis streams it through the caches without reuse once it
// is larger than the 256 MB last-level cache: then its loads are non-temporal.
static bool basis_streams(int ncol, int64_t h, size_t es) {
  return (double)ncol * 2.0 * (double)h * (double)es >= 256.0 * 1024 * 1024;
}

template <typename S>
hipError_t launch_reorth_dots(const cplx<S>* V, int64_t ldv, int ncol, cplx<S>* u, int64_t h,
                              double* partial, int nblk, hipStream_t st, const double* tloc,
                              double beta, int jl, cplx<S>* uout, int groups, const double* beta2) {
  if (ncol > kMaxCols) return hipErrorInvalidValue;
  if (tloc && (jl < 0 || jl >= ncol || ((beta != 0.0 || beta2) && jl < 1))) return hipErrorInvalidValue;
  if (groups < 1) return hipErrorInvalidValue;
  if (!uout) uout = u;
  if (tloc && groups > 1 && uout == u) return hipErrorInvalidValue;   // the groups still read u
  if (dots_lds64_applies(h, (int)sizeof(cplx<S>))) {
    if constexpr (sizeof(S) == 8) {
      const int64_t nb = (h + kDotsLds64Pairs - 1) / kDotsLds64Pairs;
      if (nb != nblk || groups != 1) return hipErrorInvalidValue;
      const bool nt = basis_streams(ncol, h, sizeof(cplx<S>));
      auto go = [&](auto localc, auto ntc) {
        hipLaunchKernelGGL((k_dots_lds64<decltype(localc)::value, decltype(ntc)::value>), dim3((unsigned)nb),
                           dim3(kReorthThreads), 0, st, V, ldv, ncol, u, h, partial, tloc, beta, jl, uout,
                           beta2);
      };
      using T_ = std::true_type;
      using F_ = std::false_type;
      if (tloc) { if (nt) go(T_{}, T_{}); else go(T_{}, F_{}); }
      else      { if (nt) go(F_{}, T_{}); else go(F_{}, F_{}); }
      return hipGetLastError();
    }
  }
  if (dots_lds_applies(h, (int)sizeof(cplx<S>))) {
    if constexpr (sizeof(S) == 4) {
      const int64_t nb = (h + kDotsLdsPairs - 1) / kDotsLdsPairs;
      if (nb != nblk || groups != 1) return hipErrorInvalidValue;
      const bool nt = basis_streams(ncol, h, sizeof(cplx<S>));
      auto go = [&](auto localc, auto ntc) {
        hipLaunchKernelGGL((k_dots_lds<decltype(localc)::value, decltype(ntc)::value>), dim3((unsigned)nb),
                           dim3(kReorthThreads), 0, st, V, ldv, ncol, u, h, partial, tloc, beta, jl, uout,
                           beta2);
      };
      using T_ = std::true_type;
      using F_ = std::false_type;
      if (tloc) { if (nt) go(T_{}, T_{}); else go(T_{}, F_{}); }
      else      { if (nt) go(F_{}, T_{}); else go(F_{}, F_{}); }
      return hipGetLastError();
    }
  }
  const int64_t ch = 64 * kPairsPerLane;
  const int64_t nch = (h + ch - 1) / ch;
  const int per = (int)((nch + nblk - 1) / nblk);
  const unsigned grid = (unsigned)((nch + per - 1) / per);
  if ((int)grid != nblk) return hipErrorInvalidValue;
  const dim3 g2(grid, (unsigned)groups);
  const size_t lds = sizeof(double) * (size_t)dots_stride(ncol);
  const bool e2 = sizeof(S) == 4 && h % 2 == 0;
  // FP32 only: the FP64 inner products measured slower with non-temporal
  // loads (16^4: 362 -> 388 us), the FP64 update faster (349 -> 323 us)
  const bool nt = sizeof(S) == 4 && basis_streams(ncol, h, sizeof(cplx<S>));
  auto go = [&](auto e2c, auto localc, auto ntc) {
    constexpr int E = decltype(e2c)::value ? (sizeof(S) == 4 ? 2 : 1) : 1;
    hipLaunchKernelGGL((k_dots<S, E, decltype(localc)::value, decltype(ntc)::value>), g2,
                       dim3(kReorthThreads), lds, st, V, ldv, ncol, u, h, per, partial, tloc, beta,
                       jl, uout, beta2);
  };
  using T_ = std::true_type;
  using F_ = std::false_type;
  if (tloc) {
    if (e2) { if (nt) go(T_{}, T_{}, T_{}); else go(T_{}, T_{}, F_{}); }
    else    { if (nt) go(F_{}, T_{}, T_{}); else go(F_{}, T_{}, F_{}); }
  } else {
    if (e2) { if (nt) go(T_{}, F_{}, T_{}); else go(T_{}, F_{}, F_{}); }
    else    { if (nt) go(F_{}, F_{}, T_{}); else go(F_{}, F_{}, F_{}); }
  }
  return hipGetLastError();
}

// Number of dots blocks the driver must size the partial buffer for.
int reorth_dots_blocks(int64_t h, int es) {
  if (dots_lds_applies(h, es)) return (int)((h + kDotsLdsPairs - 1) / kDotsLdsPairs);
  if (dots_lds64_applies(h, es)) return (int)((h + kDotsLds64Pairs - 1) / kDotsLds64Pairs);
  const int64_t ch = 64 * kPairsPerLane;
  const int64_t nch = (h + ch - 1) / ch;
  const int per = dots_chunks(h, es);
  return (int)((nch + per - 1) / per);
}

template <typename S, int E, int Q>
static void launch_update_q(unsigned grid, const cplx<S>* V, int64_t ldv, int ncol,
                            const cplx<S>* uin, cplx<S>* u, int64_t h, const double* coef,
                            double* partial, hipStream_t st, bool jsym, int groups, cplx<S>* d,
                            double* fin, unsigned* cnt) {
  if (groups > 1) {
    const dim3 g2(grid, (unsigned)groups);
    if (jsym)
      hipLaunchKernelGGL((k_update<S, E, Q, true, true, false>), g2, dim3(kReorthThreads), 0, st, V,
                         ldv, ncol, uin, u, h, coef, partial, d, nullptr, nullptr);
    else
      hipLaunchKernelGGL((k_update<S, E, Q, false, true, false>), g2, dim3(kReorthThreads), 0, st, V,
                         ldv, ncol, uin, u, h, coef, partial, d, nullptr, nullptr);
    hipLaunchKernelGGL((k_update_fin<S, E, Q>), dim3(grid), dim3(kReorthThreads), 0, st, uin, u, h,
                       (const cplx<S>*)d, groups, partial, fin, cnt);
    return;
  }
  // column groups are only used for short vectors, whose basis stays cached
  const bool nt = basis_streams(ncol, h, sizeof(cplx<S>));
  if (jsym) {
    if (nt)
      hipLaunchKernelGGL((k_update<S, E, Q, true, false, true>), dim3(grid), dim3(kReorthThreads), 0,
                         st, V, ldv, ncol, uin, u, h, coef, partial, d, fin, cnt);
    else
      hipLaunchKernelGGL((k_update<S, E, Q, true, false, false>), dim3(grid), dim3(kReorthThreads),
                         0, st, V, ldv, ncol, uin, u, h, coef, partial, d, fin, cnt);
  } else {
    if (nt)
      hipLaunchKernelGGL((k_update<S, E, Q, false, false, true>), dim3(grid), dim3(kReorthThreads),
                         0, st, V, ldv, ncol, uin, u, h, coef, partial, d, fin, cnt);
    else
      hipLaunchKernelGGL((k_update<S, E, Q, false, false, false>), dim3(grid), dim3(kReorthThreads),
                         0, st, V, ldv, ncol, uin, u, h, coef, partial, d, fin, cnt);
  }
}

template <typename S>
hipError_t launch_reorth_update(const cplx<S>* V, int64_t ldv, int ncol, cplx<S>* u, int64_t h,
                                const double* coef, double* partial, int nblk, hipStream_t st,
                                bool jsym, const cplx<S>* uin, int groups, cplx<S>* d,
                                double* fin, unsigned* cnt) {
  if (groups < 1 || (groups > 1 && !d) || (fin && !cnt)) return hipErrorInvalidValue;
  if (!uin) uin = u;
  if (jsym && update_lds_applies(h, (int)sizeof(cplx<S>))) {
    if constexpr (sizeof(S) == 4) {
      const int64_t nb = (h + kUpdLdsPairs - 1) / kUpdLdsPairs;
      if (nb != nblk || groups != 1) return hipErrorInvalidValue;
      if (basis_streams(ncol, h, sizeof(cplx<S>)))
        hipLaunchKernelGGL((k_update_lds<true>), dim3((unsigned)nb), dim3(64), 0, st, V, ldv, ncol,
                           uin, u, h, coef, partial, fin, cnt);
      else
        hipLaunchKernelGGL((k_update_lds<false>), dim3((unsigned)nb), dim3(64), 0, st, V, ldv, ncol,
                           uin, u, h, coef, partial, fin, cnt);
      return hipGetLastError();
    }
  }
  const int E = elems_per_load(h, (int)sizeof(cplx<S>));
  const int ppl = update_ppl(h, E);
  const unsigned grid = (unsigned)((h + 256 * (int64_t)ppl - 1) / (256 * (int64_t)ppl));
  if ((int)grid != nblk) return hipErrorInvalidValue;
  if (E == 2) {
    if constexpr (sizeof(S) == 4) {
      if (ppl == 8) launch_update_q<S, 2, 4>(grid, V, ldv, ncol, uin, u, h, coef, partial, st, jsym, groups, d, fin, cnt);
      else if (ppl == 4) launch_update_q<S, 2, 2>(grid, V, ldv, ncol, uin, u, h, coef, partial, st, jsym, groups, d, fin, cnt);
      else launch_update_q<S, 2, 1>(grid, V, ldv, ncol, uin, u, h, coef, partial, st, jsym, groups, d, fin, cnt);
    }
  } else {
    if (ppl == 8) launch_update_q<S, 1, 8>(grid, V, ldv, ncol, uin, u, h, coef, partial, st, jsym, groups, d, fin, cnt);
    else if (ppl == 4) launch_update_q<S, 1, 4>(grid, V, ldv, ncol, uin, u, h, coef, partial, st, jsym, groups, d, fin, cnt);
    else if (ppl == 2) launch_update_q<S, 1, 2>(grid, V, ldv, ncol, uin, u, h, coef, partial, st, jsym, groups, d, fin, cnt);
    else launch_update_q<S, 1, 1>(grid, V, ldv, ncol, uin, u, h, coef, partial, st, jsym, groups, d, fin, cnt);
  }
  return hipGetLastError();
}

// Column groups for vectors too short to fill the device (see k_dots and
// k_update): enough groups for about 256 dots and 512 update blocks, at most 16.
int reorth_dots_groups(int64_t h, int es) {
  const int nb = reorth_dots_blocks(h, es);
  return nb >= 128 ? 1 : std::min(kMaxGroups, std::max(1, 256 / nb));
}
int reorth_update_groups(int64_t h, int es) {
  const int nb = reorth_update_blocks(h, es);
  return nb >= 128 ? 1 : std::min(kMaxGroups, std::max(1, 512 / nb));
}

#define JL_INST(S)                                                                                \
  template hipError_t launch_reorth_dots<S>(const cplx<S>*, int64_t, int, cplx<S>*, int64_t,       \
                                            double*, int, hipStream_t, const double*, double,     \
                                            int, cplx<S>*, int, const double*);                   \
  template hipError_t launch_reorth_update<S>(const cplx<S>*, int64_t, int, cplx<S>*, int64_t,    \
                                              const double*, double*, int, hipStream_t, bool,     \
                                              const cplx<S>*, int, cplx<S>*, double*, unsigned*);
JL_INST(float)
JL_INST(double)
#undef JL_INST

}  // namespace jl
