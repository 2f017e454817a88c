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
// threads.  rc/rs/rt hold mp/2 rotations, pq (ints) the mp indices of the
// round's pairs, red NT/64 doubles.  A pair is rotated only while
// |a_pq| > max(2 eps sqrt(|a_pp a_qq|), eps ||A||_F): smaller entries are
// left in place, a perturbation at the rounding level (the absolute floor
// keeps rounding noise around eigenvalues near zero from rotating forever);
// the sweeps stop after one without any rotation, or after max_sweeps.  Must be called by every thread of the
// workgroup (it synchronises).
template <int NT>
__device__ void jacobi_lds(double* A, double* Z, int mp, double* rc, double* rs, double* rt, int* pq,
                           double* red, int max_sweeps) {
  static_assert(NT % 64 == 0 && NT / 64 <= 16, "jacobi_lds reduces over at most 16 wavefronts");
  const int P = mp / 2, tid = threadIdx.x;
  constexpr double kSkip = 2.0 * 2.220446049250313e-16;
  // flat index -> (row, column) by a float reciprocal: exact for the index
  // ranges here (< 2^12), which keeps integer division out of the inner loops
  const float invP = 1.0f / (float)P, invM = 1.0f / (float)mp;
  double f2 = 0.0;
  for (int idx = tid; idx < mp * mp; idx += NT) f2 += A[idx] * A[idx];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) f2 += __shfl_xor(f2, o);
  if (tid % 64 == 0) red[tid / 64] = f2;
  __syncthreads();
  double fro2 = 0.0;
  for (int w = 0; w < NT / 64; ++w) fro2 += red[w];
  __syncthreads();
  const double floor_abs = 2.220446049250313e-16 * sqrt(fro2);
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) red[0] = 0.0;   // set to 1 by any rotation of this sweep
    __syncthreads();
    for (int r = 0; r < mp - 1; ++r) {
      for (int I = tid; I < P; I += NT) {
        int p, q;
        round_pair(mp, r, I, p, q);
        pq[2 * I] = p;
        pq[2 * I + 1] = q;
        const double app = A[p + p * mp], aqq = A[q + q * mp], apq = A[p + q * mp];
        Rot ro{1.0, 0.0, 0.0};
        if (fabs(apq) > fmax(kSkip * sqrt(fabs(app * aqq)), floor_abs) && apq != 0.0) {
          ro = jacobi_rot(app, aqq, apq);
          if (ro.s != 0.0) red[0] = 1.0;   // an underflowed rotation changes nothing
        }
        rc[I] = ro.c; rs[I] = ro.s; rt[I] = ro.t;
      }
      __syncthreads();
      for (int idx = tid; idx < P * P; idx += NT) {
        const int J = (int)(((float)idx + 0.5f) * invP);
        const int I = idx - J * P;
        if (I > J) continue;
        const int pi = pq[2 * I], qi = pq[2 * I + 1];
        const double si = rs[I];
        if (I == J) {
          if (si == 0.0) continue;   // not rotated: the block stays as it is
          const double apq = A[pi + qi * mp], t = rt[I];
          A[pi + pi * mp] -= t * apq;
          A[qi + qi * mp] += t * apq;
          A[pi + qi * mp] = 0.0;
          A[qi + pi * mp] = 0.0;
          continue;
        }
        const double sj = rs[J];
        if (si == 0.0 && sj == 0.0) continue;
        const int pj = pq[2 * J], qj = pq[2 * J + 1];
        const Rot ri{rc[I], si, 0.0}, rj{rc[J], sj, 0.0};
        double o[4];
        rot_block(ri, rj, A[pi + pj * mp], A[pi + qj * mp], A[qi + pj * mp], A[qi + qj * mp], o);
        A[pi + pj * mp] = o[0]; A[pj + pi * mp] = o[0];
        A[pi + qj * mp] = o[1]; A[qj + pi * mp] = o[1];
        A[qi + pj * mp] = o[2]; A[pj + qi * mp] = o[2];
        A[qi + qj * mp] = o[3]; A[qj + qi * mp] = o[3];
      }
      for (int zi = tid; zi < mp * P; zi += NT) {
        const int J = (int)(((float)zi + 0.5f) * invM);
        const int row = zi - J * mp;
        const double sj = rs[J];
        if (sj == 0.0) continue;
        const int pj = pq[2 * J], qj = pq[2 * J + 1];
        const double cj = rc[J];
        const double zp = Z[row + pj * mp], zq = Z[row + qj * mp];
        Z[row + pj * mp] = cj * zp - sj * zq;
        Z[row + qj * mp] = sj * zp + cj * zq;
      }
      __syncthreads();
    }
    const bool done = red[0] == 0.0;   // read by every thread after the last barrier
    __syncthreads();
    if (done) break;
  }
}

}  // namespace jl
