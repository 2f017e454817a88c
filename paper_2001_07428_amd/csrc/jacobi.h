// Parallel cyclic Jacobi building blocks for the symmetric Ritz eigenproblem
// (Alg. 1: T_m = Z Lambda Z^T), shared by the stand-alone and the batched
// solvers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace jl {

struct Rot { double c, s, t; };


// Symmetric 2x2 Schur decomposition (Golub & Van Loan, Alg. 8.4.1):
// R = [[c, s], [-s, c]] makes R^T [[app, apq], [apq, aqq]] R diagonal,
// with new diagonal (app - t apq, aqq + t apq).
__device__ __forceinline__ Rot jacobi_rot(double app, double aqq, double apq) {
  Rot r{1.0, 0.0, 0.0};
  if (apq == 0.0) return r;
  const double tau = (aqq - app) / (2.0 * apq);
  double t;
  if (fabs(tau) > 1e150) t = 0.5 / tau;
  else t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  r.c = 1.0 / sqrt(1.0 + t * t);
  r.s = t * r.c;
  r.t = t;
  return r;
}

__device__ __forceinline__ void round_pair(int mp, int r, int I, int& p, int& q) {
  const int M1 = mp - 1;
  int a, b;
  if (I == 0) { a = M1; b = r; }
  else { a = (r + I) % M1; b = (r - I + M1) % M1; }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// X' = R_I^T X R_J for the 2x2 block X = A[{pi,qi},{pj,qj}].
__device__ __forceinline__ void rot_block(const Rot& ri, const Rot& rj, double x00, double x01,
                                          double x10, double x11, double out[4]) {
  const double y00 = rj.c * x00 - rj.s * x01, y01 = rj.s * x00 + rj.c * x01;
  const double y10 = rj.c * x10 - rj.s * x11, y11 = rj.s * x10 + rj.c * x11;
  out[0] = ri.c * y00 - ri.s * y10;
  out[1] = ri.c * y01 - ri.s * y11;
  out[2] = ri.s * y00 + ri.c * y10;
  out[3] = ri.s * y01 + ri.c * y11;
}


constexpr int kJacobiLdsMaxMp = 60;

// Sweeps of parallel cyclic Jacobi on A (mp x mp, symmetric, column-major)
// with eigenvector accumulation Z (mp x mp, column-major, on entry the
// identity or any orthogonal start), both in LDS, by one workgroup of NT
// threads.  rc/rs/rt hold mp/2 rotations, red NT/64 doubles.  Stops when the
// off-diagonal sum of squares is <= 1e-30 ||A||_F^2 or after max_sweeps.
// Must be called by every thread of the workgroup (it synchronises).
template <int NT>
__device__ void jacobi_lds(double* A, double* Z, int mp, double* rc, double* rs, double* rt,
                           double* red, int max_sweeps) {
  static_assert(NT % 64 == 0 && NT / 64 <= 16, "jacobi_lds reduces over at most 16 wavefronts");
  const int P = mp / 2, tid = threadIdx.x;
  double nrm = 0.0;
  for (int idx = tid; idx < mp * mp; idx += NT) nrm += A[idx] * A[idx];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) nrm += __shfl_xor(nrm, o);
  if (tid % 64 == 0) red[tid / 64] = nrm;
  __syncthreads();
  double fro2 = 0.0;
  for (int w = 0; w < NT / 64; ++w) fro2 += red[w];
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    for (int r = 0; r < mp - 1; ++r) {
      for (int I = tid; I < P; I += NT) {
        int p, q;
        round_pair(mp, r, I, p, q);
        const Rot ro = jacobi_rot(A[p + p * mp], A[q + q * mp], A[p + q * mp]);
        rc[I] = ro.c; rs[I] = ro.s; rt[I] = ro.t;
      }
      __syncthreads();
      for (int idx = tid; idx < P * P + mp * P; idx += NT) {
        if (idx < P * P) {
          const int I = idx % P, J = idx / P;
          if (I > J) continue;
          int pi, qi, pj, qj;
          round_pair(mp, r, I, pi, qi);
          round_pair(mp, r, J, pj, qj);
          const Rot ri{rc[I], rs[I], rt[I]};
          if (I == J) {
            const double apq = A[pi + qi * mp];
            A[pi + pi * mp] -= ri.t * apq;
            A[qi + qi * mp] += ri.t * apq;
            A[pi + qi * mp] = 0.0;
            A[qi + pi * mp] = 0.0;
            continue;
          }
          const Rot rj{rc[J], rs[J], rt[J]};
          double o[4];
          rot_block(ri, rj, A[pi + pj * mp], A[pi + qj * mp], A[qi + pj * mp], A[qi + qj * mp], o);
          A[pi + pj * mp] = o[0]; A[pj + pi * mp] = o[0];
          A[pi + qj * mp] = o[1]; A[qj + pi * mp] = o[1];
          A[qi + pj * mp] = o[2]; A[pj + qi * mp] = o[2];
          A[qi + qj * mp] = o[3]; A[qj + qi * mp] = o[3];
        } else {
          const int zi = idx - P * P;
          const int row = zi % mp, J = zi / mp;
          int pj, qj;
          round_pair(mp, r, J, pj, qj);
          const double zp = Z[row + pj * mp], zq = Z[row + qj * mp];
          Z[row + pj * mp] = rc[J] * zp - rs[J] * zq;
          Z[row + qj * mp] = rs[J] * zp + rc[J] * zq;
        }
      }
      __syncthreads();
    }
    double off = 0.0;
    for (int idx = tid; idx < mp * mp; idx += NT)
      if (idx % mp != idx / mp) off += A[idx] * A[idx];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) off += __shfl_xor(off, o);
    if (tid % 64 == 0) red[tid / 64] = off;
    __syncthreads();
    double offt = 0.0;
    for (int w = 0; w < NT / 64; ++w) offt += red[w];
    __syncthreads();
    if (offt <= 1e-30 * fro2) break;
  }
}

}  // namespace jl
