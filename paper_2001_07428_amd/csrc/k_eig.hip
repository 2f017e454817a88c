// Rayleigh-Ritz step of Alg. 1: T_m = Z Lambda Z^T for the real symmetric
// projected matrix (diagonal restart block, arrow row, tridiagonal tail), in
// FP64 on the GPU, then the sort that moves the desired Ritz pairs first.
//
// Parallel cyclic Jacobi with the round-robin ("circle") ordering: in round r
// of a sweep the mp/2 disjoint index pairs are
//   (mp-1, r) and ((r + I) mod (mp-1), (r - I) mod (mp-1)), I = 1..mp/2-1,
// so every pair meets once per sweep of mp-1 rounds.  For an odd m one
// padding index with a zero row and column is added; it never rotates.
// A round applies all mp/2 rotations at once: A' = R^T A R, Z' = Z R.  Each
// 2x2 block of A' depends only on the same 2x2 block of A and the two
// rotations of its row and column pairs, so large problems run one launch
// per round (A ping-ponged, Z updated in place) and small ones run all
// sweeps inside one workgroup in LDS.
#include "common.h"
#include "jacobi.h"

namespace jl {
namespace {

__global__ void k_eig_init(const double* __restrict__ T, int ldt, int m, int mp,
                           double* __restrict__ A, double* __restrict__ Z) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)mp * mp) return;
  const int i = (int)(idx % mp), j = (int)(idx / mp);
  A[idx] = (i < m && j < m) ? T[i + (int64_t)j * ldt] : 0.0;
  Z[idx] = (i == j) ? 1.0 : 0.0;
}

// One round: threads [0, P*P) handle A blocks (I <= J), threads
// [P*P, P*P + mp*P) handle Z row pairs.
__global__ void k_eig_round(int mp, int r, const double* __restrict__ A, double* __restrict__ An,
                            double* __restrict__ Z) {
  const int P = mp / 2;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nA = (int64_t)P * P;
  if (idx < nA) {
    const int I = (int)(idx % P), J = (int)(idx / P);
    if (I > J) return;
    int pi, qi, pj, qj;
    round_pair(mp, r, I, pi, qi);
    round_pair(mp, r, J, pj, qj);
    const Rot ri = jacobi_rot(A[pi + (int64_t)pi * mp], A[qi + (int64_t)qi * mp], A[pi + (int64_t)qi * mp]);
    if (I == J) {
      const double apq = A[pi + (int64_t)qi * mp];
      An[pi + (int64_t)pi * mp] = A[pi + (int64_t)pi * mp] - ri.t * apq;
      An[qi + (int64_t)qi * mp] = A[qi + (int64_t)qi * mp] + ri.t * apq;
      An[pi + (int64_t)qi * mp] = 0.0;
      An[qi + (int64_t)pi * mp] = 0.0;
      return;
    }
    const Rot rj = jacobi_rot(A[pj + (int64_t)pj * mp], A[qj + (int64_t)qj * mp], A[pj + (int64_t)qj * mp]);
    double o[4];
    rot_block(ri, rj, A[pi + (int64_t)pj * mp], A[pi + (int64_t)qj * mp], A[qi + (int64_t)pj * mp],
              A[qi + (int64_t)qj * mp], o);
    An[pi + (int64_t)pj * mp] = o[0]; An[pj + (int64_t)pi * mp] = o[0];
    An[pi + (int64_t)qj * mp] = o[1]; An[qj + (int64_t)pi * mp] = o[1];
    An[qi + (int64_t)pj * mp] = o[2]; An[pj + (int64_t)qi * mp] = o[2];
    An[qi + (int64_t)qj * mp] = o[3]; An[qj + (int64_t)qi * mp] = o[3];
    return;
  }
  const int64_t zi = idx - nA;
  if (zi >= (int64_t)mp * P) return;
  const int row = (int)(zi % mp), J = (int)(zi / mp);
  int pj, qj;
  round_pair(mp, r, J, pj, qj);
  const Rot rj = jacobi_rot(A[pj + (int64_t)pj * mp], A[qj + (int64_t)qj * mp], A[pj + (int64_t)qj * mp]);
  const double zp = Z[row + (int64_t)pj * mp], zq = Z[row + (int64_t)qj * mp];
  Z[row + (int64_t)pj * mp] = rj.c * zp - rj.s * zq;
  Z[row + (int64_t)qj * mp] = rj.s * zp + rj.c * zq;
}

__global__ __launch_bounds__(1024) void k_eig_offnorm(int mp, const double* __restrict__ A,
                                                      double* __restrict__ off) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int64_t idx = threadIdx.x; idx < (int64_t)mp * mp; idx += 1024) {
    const int i = (int)(idx % mp), j = (int)(idx / mp);
    if (i != j) s += A[idx] * A[idx];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += sh[w];
    off[0] = t;
  }
}

// All sweeps in one workgroup; A and Z (mp x mp) live in LDS.
constexpr int kSmallMp = kJacobiLdsMaxMp;
__global__ __launch_bounds__(256) void k_eig_small(const double* __restrict__ T, int ldt, int m,
                                                   double* __restrict__ lam, double* __restrict__ Zo,
                                                   int ldz, int max_sweeps) {
  __shared__ double A[kSmallMp * kSmallMp];
  __shared__ double Z[kSmallMp * kSmallMp];
  __shared__ double rc[kSmallMp / 2], rs[kSmallMp / 2], rt[kSmallMp / 2];
  __shared__ double red[4];
  __shared__ int pq[kSmallMp];
  const int mp = m + (m & 1), tid = threadIdx.x;
  for (int idx = tid; idx < mp * mp; idx += 256) {
    const int i = idx % mp, j = idx / mp;
    A[idx] = (i < m && j < m) ? T[i + (int64_t)j * ldt] : 0.0;
    Z[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi_lds<256>(A, Z, mp, rc, rs, rt, pq, red, max_sweeps);
  for (int i = tid; i < m; i += 256) lam[i] = A[i + i * mp];
  for (int idx = tid; idx < m * m; idx += 256) {
    const int i = idx % m, j = idx / m;
    Zo[i + (int64_t)j * ldz] = Z[i + j * mp];
  }
}

// perm[rank] = i with rank = #{j : lam_j before lam_i} (ties by index).
__global__ __launch_bounds__(1024) void k_ritz_rank(int m, const double* __restrict__ lam,
                                                    int64_t lstride, int descending,
                                                    int* __restrict__ perm) {
  for (int i = threadIdx.x; i < m; i += 1024) {
    const double li = lam[i * lstride];
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      const double lj = lam[j * lstride];
      // NaN compares as +inf so the ranks stay a permutation
      const double a = isnan(lj) ? INFINITY : lj, b = isnan(li) ? INFINITY : li;
      const bool before = descending ? (a > b || (a == b && j < i)) : (a < b || (a == b && j < i));
      rank += before ? 1 : 0;
    }
    perm[rank] = i;
  }
}

template <typename S>
__global__ void k_ritz_gather(int m, const double* __restrict__ lam, int64_t lstride,
                              const double* __restrict__ Z, int ldz, int kcols,
                              const int* __restrict__ perm, double* __restrict__ lam_s,
                              double* __restrict__ Zs, S* __restrict__ Zc,
                              double* __restrict__ zlast) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  const int i = (int)(idx % m), r = (int)(idx / m);
  int src = perm[r];
  src = src < 0 ? 0 : (src >= m ? m - 1 : src);   // stays in bounds even for NaN ranks
  const double z = Z[i + (int64_t)src * ldz];
  Zs[i + (int64_t)r * m] = z;
  if (r < kcols) Zc[i + (int64_t)r * m] = (S)z;
  if (i == 0) lam_s[r] = lam[src * lstride];
  if (i == m - 1) zlast[r] = z;
}

inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int eig_small_max() { return kSmallMp; }

size_t eig_work_doubles(int m) {
  const size_t mp = (size_t)(m + (m & 1));
  return 3 * mp * mp + 8;
}

hipError_t launch_eig_init(const double* T, int ldt, int m, EigWork w, hipStream_t st) {
  const int mp = m + (m & 1);
  hipLaunchKernelGGL(k_eig_init, dim3(nb((int64_t)mp * mp, 256)), dim3(256), 0, st, T, ldt, m, mp,
                     w.A[0], w.Z);
  return hipGetLastError();
}

hipError_t launch_eig_round(int m, EigWork w, int cur, int r, hipStream_t st) {
  const int mp = m + (m & 1), P = mp / 2;
  const int64_t n = (int64_t)P * P + (int64_t)mp * P;
  hipLaunchKernelGGL(k_eig_round, dim3(nb(n, 256)), dim3(256), 0, st, mp, r, w.A[cur],
                     w.A[1 - cur], w.Z);
  return hipGetLastError();
}

hipError_t launch_eig_offnorm(int m, EigWork w, int cur, hipStream_t st) {
  const int mp = m + (m & 1);
  hipLaunchKernelGGL(k_eig_offnorm, dim3(1), dim3(1024), 0, st, mp, w.A[cur], w.off);
  return hipGetLastError();
}

hipError_t launch_eig_small(const double* T, int ldt, int m, double* lam, double* Z, int ldz,
                            int max_sweeps, hipStream_t st) {
  if (m + (m & 1) > kSmallMp) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_eig_small, dim3(1), dim3(256), 0, st, T, ldt, m, lam, Z, ldz, max_sweeps);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_ritz_sort(int m, const double* lam, int64_t lstride, const double* Z, int ldz,
                            int descending, int kcols, int* perm, double* lam_s, double* Zs, S* Zc,
                            double* zlast, hipStream_t st) {
  hipLaunchKernelGGL(k_ritz_rank, dim3(1), dim3(1024), 0, st, m, lam, lstride, descending, perm);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ritz_gather<S>, dim3(nb((int64_t)m * m, 256)), dim3(256), 0, st, m, lam,
                     lstride, Z, ldz, kcols, perm, lam_s, Zs, Zc, zlast);
  return hipGetLastError();
}

template hipError_t launch_ritz_sort<float>(int, const double*, int64_t, const double*, int, int,
                                            int, int*, double*, double*, float*, double*,
                                            hipStream_t);
template hipError_t launch_ritz_sort<double>(int, const double*, int64_t, const double*, int, int,
                                             int, int*, double*, double*, double*, double*,
                                             hipStream_t);

}  // namespace jl
