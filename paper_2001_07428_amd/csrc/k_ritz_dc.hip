// Rayleigh-Ritz step of Alg. 1 by divide and conquer, for the structure the
// thick restart gives T_m (eq. dynamicwin and the shrink of Alg. 1): an
// arrowhead block (the k kept Ritz values theta on the diagonal, their
// couplings s in row k, corner t_kk) joined by beta_k = t_{k+1,k} to the
// tridiagonal tail built by this cycle's Lanczos steps.  The first cycle
// (k = 0) is a plain tridiagonal matrix.
//
// T_m is torn at beta_k (Cuppen's tearing): T_m = diag(H, T2) + beta_k w w^T
// with w = e_k + e_{k+1}, H the arrowhead with corner t_kk - beta_k and T2 the
// tail with first diagonal entry t_{k+1,k+1} - beta_k.  The tail is torn the
// same way, recursively, into leaves of at most kDcLeaf rows that cyclic
// Jacobi solves in LDS; the arrowhead is solved through its bordered secular
// equation; each tear is undone by a rank-one merge (the secular equation of
// D + rho z z^T) followed by a GEMM with the children's eigenvectors.
//
// Both secular solves deflate zero weights (the converged pairs, whose
// couplings the restart sets to zero, arrive that way) and nearly equal
// poles (a plane rotation moves the weight onto one of them), find every
// root inside its pole interval in coordinates shifted to the nearer pole,
// and rebuild the weights from the computed roots (Gu and Eisenstat, SIAM J.
// Matrix Anal. Appl. 16 (1995) 172-191) so that the eigenvectors come out
// orthogonal to working precision.  One thread finds one root.
#include <algorithm>
#include <vector>

#include "common.h"
#include "jacobi.h"

namespace jl {
namespace {

constexpr double kEps = 2.220446049250313e-16;
constexpr int kDcLeaf = 32;     // largest tail block solved directly (cyclic Jacobi in LDS)
constexpr int kDcMaxM = 1024;   // LDS of one secular solve: about 100 bytes per pole
constexpr int kLeafThreads = 1024;   // about one update item per thread and Jacobi round
constexpr int kSecThreads = 512;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
// Workgroup sum / max; every thread gets the result.
template <int NT>
__device__ double wg_sum(double v, double* red) {
  v = wave_sum(v);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}
template <int NT>
__device__ double wg_max(double v, double* red) {
  v = wave_max(v);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) t = fmax(t, red[w]);
  __syncthreads();
  return t;
}

// Root of f(lam) = c0 + c1 lam + w sum_j z2_j / (D_j - lam) between the poles
// D[lo_pole] and D[hi_pole] (an index of -1 takes lo_bound / hi_bound
// instead); f increases there when w > 0 and decreases when w < 0.  The root
// is returned as lam = org + tau with org the nearer end, so that the
// differences D_j - lam = (D_j - org) - tau keep their relative accuracy.
// Each step takes, inside the current bracket, the root of the osculating
// model A + B / (pole - lam) at the origin pole, else a Newton step, else a
// bisection (geometric when the bracket spans orders of magnitude).  One
// wavefront finds one root: the lanes share the sums over the poles, and
// every lane takes the same (uniform) decisions.
struct Root { double org, tau; };

__device__ __forceinline__ void wave_sum2(double& a, double& b) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
}

__device__ Root secular_root_wave(double c0, double c1, double w, const double* __restrict__ D,
                                  const double* __restrict__ z2, int n, int lo_pole, int hi_pole,
                                  double lo_bound, double hi_bound) {
  const int lane = threadIdx.x % 64;
  const double a = lo_pole >= 0 ? D[lo_pole] : lo_bound;
  const double b = hi_pole >= 0 ? D[hi_pole] : hi_bound;
  const double mid = 0.5 * (a + b);
  double fm = 0.0, dummy = 0.0;
  for (int j = lane; j < n; j += 64) fm += z2[j] / (D[j] - mid);
  wave_sum2(fm, dummy);
  fm = c0 + c1 * mid + w * fm;
  const bool inc = w > 0.0;
  const bool left = inc ? (fm >= 0.0) : (fm <= 0.0);   // root in (a, mid]
  const int o = left ? lo_pole : hi_pole;
  const double org = left ? a : b;
  double lo = left ? 0.0 : (mid - b);
  double hi = left ? (mid - a) : 0.0;
  double tau = (o < 0) ? 0.5 * (lo + hi) : (left ? 0.5 * hi : 0.5 * lo);
  const double cc0 = c0 + c1 * org;
  for (int it = 0; it < 200; ++it) {
    double sf = 0.0, sp = 0.0;
    for (int j = lane; j < n; j += 64) {
      const double r = 1.0 / ((D[j] - org) - tau);
      const double t = z2[j] * r;
      sf += t;
      sp += t * r;
    }
    wave_sum2(sf, sp);
    const double f = cc0 + c1 * tau + w * sf, fp = c1 + w * sp;
    if (f == 0.0) break;
    if (inc ? (f < 0.0) : (f > 0.0)) lo = tau; else hi = tau;
    if (hi - lo <= 4.0 * kEps * fmax(fabs(lo), fabs(hi))) break;
    double step = 0.0;
    bool ok = false;
    if (o >= 0 && fp != 0.0) {
      const double B = fp * tau * tau;
      const double A = f + B / tau;
      if (A != 0.0) {
        const double c = B / A;
        if (c > lo && c < hi) { step = c; ok = true; }
      }
    }
    if (!ok && fp != 0.0) {
      const double c = tau - f / fp;
      if (c > lo && c < hi) { step = c; ok = true; }
    }
    if (!ok) {
      if (lo > 0.0 && hi > 4.0 * lo) step = sqrt(lo * hi);
      else if (hi < 0.0 && lo < 4.0 * hi) step = -sqrt(lo * hi);
      else step = 0.5 * (lo + hi);
      if (!(step > lo && step < hi)) break;
    }
    tau = step;
  }
  return Root{org, tau};
}

// LDS carve-up shared by the prepare and finish kernels, for at most `cap`
// poles.
struct SecLds {
  double *d, *z, *Dk, *z2, *org, *tau, *zh, *cn, *rc, *rs, *red;
  int *perm, *defl, *K, *ri, *rj, *misc;
};
__device__ SecLds carve_sec(char* raw, int cap) {
  SecLds L;
  double* p = reinterpret_cast<double*>(raw);
  L.d = p; p += cap;
  L.z = p; p += cap;
  L.Dk = p; p += cap;
  L.z2 = p; p += cap;
  L.org = p; p += cap + 1;
  L.tau = p; p += cap + 1;
  L.zh = p; p += cap;
  L.cn = p; p += cap + 1;
  L.rc = p; p += cap;
  L.rs = p; p += cap;
  L.red = p; p += 16;
  int* q = reinterpret_cast<int*>(p);
  L.perm = q; q += cap;
  L.defl = q; q += cap;
  L.K = q; q += cap;
  L.ri = q; q += cap;
  L.rj = q; q += cap;
  L.misc = q;   // [0] = number of non-deflated poles, [1] = number of rotations
  return L;
}
size_t sec_lds_bytes(int cap) {
  return sizeof(double) * (10 * (size_t)cap + 3 + 16) + sizeof(int) * (5 * (size_t)cap + 4);
}

// The state a secular solve keeps in device memory between its prepare,
// roots and finish kernels (one block per problem, `cap` poles):
// hdr = [n, nrot, sgn, w, c0, c1, lo_bound, hi_bound], then d, Dk, z2, zh,
// org, tau, rc, rs (doubles) and perm, defl, K, ri, rj (ints).
struct SecState {
  double *hdr, *d, *Dk, *z2, *zh, *org, *tau, *rc, *rs;
  int *perm, *defl, *K, *ri, *rj;
};
__host__ __device__ inline size_t sec_state_doubles(int cap) {
  return 16 + 8 * (size_t)cap + 2 + (5 * (size_t)cap + 1) / 2 + 2;
}
__device__ SecState state_view(double* g, int cap) {
  SecState S;
  S.hdr = g; g += 16;
  S.d = g; g += cap;
  S.Dk = g; g += cap;
  S.z2 = g; g += cap;
  S.zh = g; g += cap;
  S.org = g; g += cap + 1;
  S.tau = g; g += cap + 1;
  S.rc = g; g += cap;
  S.rs = g; g += cap;
  int* q = reinterpret_cast<int*>(g);
  S.perm = q; q += cap;
  S.defl = q; q += cap;
  S.K = q; q += cap;
  S.ri = q; q += cap;
  S.rj = q;
  return S;
}

// Sorts the N poles L.d (with weights L.z) ascending: afterwards L.d and L.z
// hold the sorted values and L.perm[r] the input index of sorted position r
// (ties keep input order).
template <int NT>
__device__ void sort_poles(const SecLds& L, int N) {
  for (int i = threadIdx.x; i < N; i += NT) {
    const double di = L.d[i];
    int rank = 0;
    for (int j = 0; j < N; ++j) {
      const double dj = L.d[j];
      rank += (dj < di || (dj == di && j < i)) ? 1 : 0;
    }
    L.perm[rank] = i;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < N; r += NT) {
    L.Dk[r] = L.d[L.perm[r]];
    L.z2[r] = L.z[L.perm[r]];
  }
  __syncthreads();
  for (int r = threadIdx.x; r < N; r += NT) {
    L.d[r] = L.Dk[r];
    L.z[r] = L.z2[r];
  }
  __syncthreads();
}

// Deflation on the sorted poles L.d with weights L.z (thread 0, in order):
// a weight with |wscale * z| <= tol deflates its pole; of two neighbouring
// live poles whose rotation (zeroing the first weight) leaves an off-diagonal
// |(d_j - d_i) c s| <= tol, the first deflates.  Rotations are recorded in
// order (L.ri, L.rj, L.rc, L.rs); the live poles (still ascending) go to
// L.K / L.Dk / L.z2 (squared weights) and keep their signed weight in L.zh.
// With all_deflate every pole deflates (no coupling).
template <int NT>
__device__ void deflate(const SecLds& L, int N, double wscale, double tol, bool all_deflate) {
  if (threadIdx.x == 0) {
    int nrot = 0, prev = -1;
    for (int j = 0; j < N; ++j) L.defl[j] = (all_deflate || fabs(wscale * L.z[j]) <= tol) ? 1 : 0;
    for (int j = 0; j < N; ++j) {
      if (L.defl[j]) continue;
      if (prev >= 0) {
        const int i = prev;
        const double rr = hypot(L.z[i], L.z[j]);
        const double c = L.z[j] / rr, s = L.z[i] / rr;
        if (fabs((L.d[j] - L.d[i]) * c * s) <= tol) {
          const double di = L.d[i], dj = L.d[j];
          L.d[i] = di * c * c + dj * s * s;
          L.d[j] = di * s * s + dj * c * c;
          L.z[i] = 0.0;
          L.z[j] = rr;
          L.defl[i] = 1;
          L.ri[nrot] = i; L.rj[nrot] = j; L.rc[nrot] = c; L.rs[nrot] = s;
          ++nrot;
        }
      }
      prev = j;
    }
    int n = 0;
    for (int j = 0; j < N; ++j) {
      if (L.defl[j]) continue;
      L.K[n] = j;
      L.Dk[n] = L.d[j];
      L.z2[n] = L.z[j] * L.z[j];
      L.zh[n] = L.z[j];
      ++n;
    }
    L.misc[0] = n;
    L.misc[1] = nrot;
  }
  __syncthreads();
}

// Saves the prepared problem (after sort_poles and deflate) to the state.
template <int NT>
__device__ void save_state(const SecLds& L, const SecState& S, int N, double sgn, double w, double c0,
                           double c1, double lo_b, double hi_b) {
  const int n = L.misc[0], nrot = L.misc[1];
  if (threadIdx.x == 0) {
    S.hdr[0] = n; S.hdr[1] = nrot; S.hdr[2] = sgn; S.hdr[3] = w;
    S.hdr[4] = c0; S.hdr[5] = c1; S.hdr[6] = lo_b; S.hdr[7] = hi_b;
  }
  for (int i = threadIdx.x; i < N; i += NT) {
    S.d[i] = L.d[i];
    S.perm[i] = L.perm[i];
    S.defl[i] = L.defl[i];
  }
  for (int i = threadIdx.x; i < n; i += NT) {
    S.Dk[i] = L.Dk[i];
    S.z2[i] = L.z2[i];
    S.zh[i] = L.zh[i];
    S.K[i] = L.K[i];
  }
  for (int i = threadIdx.x; i < nrot; i += NT) {
    S.ri[i] = L.ri[i]; S.rj[i] = L.rj[i]; S.rc[i] = L.rc[i]; S.rs[i] = L.rs[i];
  }
}

// Loads a solved problem (state plus roots) back into LDS for the finish.
template <int NT>
__device__ void load_state(const SecLds& L, const SecState& S, int N, int nroots) {
  const int n = (int)S.hdr[0], nrot = (int)S.hdr[1];
  if (threadIdx.x == 0) {
    L.misc[0] = n;
    L.misc[1] = nrot;
  }
  for (int i = threadIdx.x; i < N; i += NT) {
    L.d[i] = S.d[i];
    L.perm[i] = S.perm[i];
    L.defl[i] = S.defl[i];
  }
  for (int i = threadIdx.x; i < n; i += NT) {
    L.Dk[i] = S.Dk[i];
    L.zh[i] = S.zh[i];
    L.K[i] = S.K[i];
  }
  for (int i = threadIdx.x; i < nroots; i += NT) {
    L.org[i] = S.org[i];
    L.tau[i] = S.tau[i];
  }
  for (int i = threadIdx.x; i < nrot; i += NT) {
    L.ri[i] = S.ri[i]; L.rj[i] = S.rj[i]; L.rc[i] = S.rc[i]; L.rs[i] = S.rs[i];
  }
  __syncthreads();
}

// X (rows x cols, column-major, leading dimension ldx, in global memory) :=
// G X with G = R_1 ... R_nrot the recorded rotations, R_p replacing rows
// (i, j) by (c x_i + s x_j, -s x_i + c x_j); applied last to first.
template <int NT>
__device__ void rotate_rows(const SecLds& L, double* X, int ldx, int cols) {
  const int nrot = L.misc[1];
  for (int p = nrot - 1; p >= 0; --p) {
    const int i = L.ri[p], j = L.rj[p];
    const double c = L.rc[p], s = L.rs[p];
    for (int col = threadIdx.x; col < cols; col += NT) {
      const double xi = X[i + (int64_t)col * ldx], xj = X[j + (int64_t)col * ldx];
      X[i + (int64_t)col * ldx] = c * xi + s * xj;
      X[j + (int64_t)col * ldx] = -s * xi + c * xj;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ leaves
struct LeafJobs {
  int lo[64];
  int n[64];
};

// Each workgroup solves one leaf [lo, lo + n) of the torn tail: diagonal
// alpha with beta subtracted at torn ends (and rho0 at tail index 0),
// off-diagonals beta; eigenvalues to D[lo..], eigenvectors to the diagonal
// block of Q (t x t, column-major).
__global__ __launch_bounds__(kLeafThreads) void k_dc_leaves(LeafJobs jobs, const double* __restrict__ alpha,
                                                            const double* __restrict__ beta, double rho0,
                                                            int t, double* __restrict__ D,
                                                            double* __restrict__ Q) {
  __shared__ double A[kJacobiLdsMaxMp * kJacobiLdsMaxMp];
  __shared__ double Z[kJacobiLdsMaxMp * kJacobiLdsMaxMp];
  __shared__ double rc[kJacobiLdsMaxMp / 2], rs[kJacobiLdsMaxMp / 2], rt[kJacobiLdsMaxMp / 2];
  __shared__ double red[kLeafThreads / 64];
  __shared__ int pq[kJacobiLdsMaxMp];
  const int lo = jobs.lo[blockIdx.x], n = jobs.n[blockIdx.x];
  const int mp = n + (n & 1), tid = threadIdx.x;
  for (int idx = tid; idx < mp * mp; idx += kLeafThreads) {
    const int i = idx % mp, j = idx / mp;
    double v = 0.0;
    if (i < n && j < n) {
      if (i == j) {
        v = alpha[lo + i];
        if (i == 0 && lo > 0) v -= beta[lo - 1];
        if (i == 0 && lo == 0) v -= rho0;
        if (i == n - 1 && lo + n < t) v -= beta[lo + n - 1];
      } else if (i == j + 1) {
        v = beta[lo + j];
      } else if (j == i + 1) {
        v = beta[lo + i];
      }
    }
    A[idx] = v;
    Z[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi_lds<kLeafThreads>(A, Z, mp, rc, rs, rt, pq, red, 60);
  for (int c = tid; c < n; c += kLeafThreads) D[lo + c] = A[c + c * mp];
  for (int idx = tid; idx < n * n; idx += kLeafThreads) {
    const int r = idx % n, c = idx / n;
    Q[(int64_t)(lo + r) + (int64_t)(lo + c) * t] = Z[r + c * mp];
  }
}


// ------------------------------------------------------------ arrowhead
// eig([[diag(theta), s], [s^T, a]]) for k poles in three launches: prepare
// (sort, deflate; state of capacity k + 1), the roots, finish -> DA (k + 1),
// QA ((k + 1) x (k + 1), column-major, ld k + 1); X is a (k + 1)^2 scratch.
__global__ __launch_bounds__(kSecThreads) void k_dc_arrow_prep(const double* __restrict__ theta,
                                                               const double* __restrict__ s, double a,
                                                               int k, double* __restrict__ state) {
  extern __shared__ __align__(16) char lds_raw[];
  const SecLds L = carve_sec(lds_raw, k + 1);
  constexpr int NT = kSecThreads;
  const int tid = threadIdx.x;
  for (int i = tid; i < k; i += NT) {
    L.d[i] = theta[i];
    L.z[i] = s[i];
  }
  __syncthreads();
  sort_poles<NT>(L, k);
  double mx = 0.0, s2 = 0.0;
  for (int i = tid; i < k; i += NT) {
    mx = fmax(mx, fabs(L.d[i]));
    s2 += L.z[i] * L.z[i];
  }
  mx = wg_max<NT>(mx, L.red);
  s2 = wg_sum<NT>(s2, L.red);
  const double tol = 8.0 * kEps * fmax(fmax(mx, fabs(a)), sqrt(s2));
  deflate<NT>(L, k, 1.0, tol, false);
  const int n = L.misc[0];
  // the spectrum lies within ||s|| of the diagonal: bounds for the outer roots
  double R2 = 0.0;
  for (int j = tid; j < n; j += NT) R2 += L.z2[j];
  const double R = sqrt(wg_sum<NT>(R2, L.red));
  const double lo_b = (n ? fmin(L.Dk[0], a) : a) - R - kEps * (fabs(a) + mx);
  const double hi_b = (n ? fmax(L.Dk[n - 1], a) : a) + R + kEps * (fabs(a) + mx);
  save_state<NT>(L, state_view(state, k + 1), k, 1.0, -1.0, a, -1.0, lo_b, hi_b);
}

__global__ __launch_bounds__(kSecThreads) void k_dc_arrow_fin(int k, const double* __restrict__ state,
                                                              double* __restrict__ DA,
                                                              double* __restrict__ QA,
                                                              double* __restrict__ X) {
  extern __shared__ __align__(16) char lds_raw[];
  const SecLds L = carve_sec(lds_raw, k + 1);
  constexpr int NT = kSecThreads;
  const int tid = threadIdx.x, N = k + 1;
  const SecState S = state_view(const_cast<double*>(state), k + 1);
  const int n = (int)S.hdr[0];
  load_state<NT>(L, S, k, n + 1);
  // Rebuilt weights: s_j^2 = (d_j - lam_j)(lam_{j+1} - d_j) prod_{i != j}
  // (lam_{i or i+1} - d_j) / (d_i - d_j), from the interlacing.
  for (int j = tid; j < n; j += NT) {
    const double dj = L.Dk[j];
    double p = ((dj - L.org[j]) - L.tau[j]) * -((dj - L.org[j + 1]) - L.tau[j + 1]);
    for (int i = 0; i < n; ++i) {
      if (i == j) continue;
      const int li = i < j ? i : i + 1;
      p *= -((dj - L.org[li]) - L.tau[li]) / (L.Dk[i] - dj);
    }
    L.zh[j] = copysign(sqrt(fabs(p)), L.zh[j]);
  }
  __syncthreads();
  for (int i = tid; i <= n; i += NT) {   // norms of [s_j / (lam_i - d_j); 1]
    double q = 1.0;
    for (int j = 0; j < n; ++j) {
      const double v = L.zh[j] / ((L.Dk[j] - L.org[i]) - L.tau[i]);
      q += v * v;
    }
    L.cn[i] = 1.0 / sqrt(q);
  }
  __syncthreads();
  // X in sorted/rotated theta coordinates: columns [deflated poles | roots].
  const int nd = k - n;
  for (int idx = tid; idx < N * N; idx += NT) X[idx] = 0.0;
  __syncthreads();
  if (tid == 0) {
    int c = 0;
    for (int j = 0; j < k; ++j)
      if (L.defl[j]) {
        X[j + (int64_t)c * N] = 1.0;
        DA[c] = L.d[j];
        ++c;
      }
  }
  for (int i = tid; i <= n; i += NT) DA[nd + i] = L.org[i] + L.tau[i];
  for (int idx = tid; idx < (n + 1) * (n + 1); idx += NT) {
    const int jj = idx % (n + 1), i = idx / (n + 1);   // row jj (pole or corner), root i
    const int col = nd + i;
    double v;
    int row;
    if (jj < n) {
      v = -L.zh[jj] / ((L.Dk[jj] - L.org[i]) - L.tau[i]) * L.cn[i];
      row = L.K[jj];
    } else {
      v = L.cn[i];
      row = k;
    }
    X[row + (int64_t)col * N] = v;
  }
  __syncthreads();
  rotate_rows<NT>(L, X, N, N);
  // theta rows back to input order; the corner row stays last
  for (int idx = tid; idx < N * N; idx += NT) {
    const int r = idx % N, c = idx / N;
    QA[(r < k ? L.perm[r] : k) + (int64_t)c * N] = X[idx];
  }
}

// ------------------------------------------------------------ rank-one merge
struct MergeJob {
  const double* D1;
  const double* D2;
  const double* Q1;   // child eigenvectors (column-major blocks)
  const double* Q2;
  double* Dout;       // N eigenvalues
  double* W;          // N x N (ld N): parent vectors in the children's bases
  double* X;          // N x N scratch
  double* state;      // sec_state_doubles(N)
  double rho;
  int ld1, ld2, zrow1, zrow2, n1, n2;
};
constexpr int kMaxMergeJobs = 24;
struct MergeJobs {
  MergeJob j[kMaxMergeJobs];
};

// eig(diag(D1, D2) + rho z z^T), z = [row zrow1 of Q1; row zrow2 of Q2]: the
// merge of a tear, prepared (gather, scale, sort, deflate) by one workgroup
// per job.
__global__ __launch_bounds__(kSecThreads) void k_dc_merge_prep(MergeJobs jobs) {
  extern __shared__ __align__(16) char lds_raw[];
  constexpr int NT = kSecThreads;
  const MergeJob& J = jobs.j[blockIdx.x];
  const int N = J.n1 + J.n2, tid = threadIdx.x;
  const SecLds L = carve_sec(lds_raw, N);
  for (int i = tid; i < N; i += NT) {
    if (i < J.n1) {
      L.d[i] = J.D1[i];
      L.z[i] = J.Q1[J.zrow1 + (int64_t)i * J.ld1];
    } else {
      L.d[i] = J.D2[i - J.n1];
      L.z[i] = J.Q2[J.zrow2 + (int64_t)(i - J.n1) * J.ld2];
    }
  }
  __syncthreads();
  double zz = 0.0;
  for (int i = tid; i < N; i += NT) zz += L.z[i] * L.z[i];
  zz = wg_sum<NT>(zz, L.red);
  double r = J.rho * zz;
  const bool uncoupled = (r == 0.0 || zz == 0.0);   // the children's pairs as they are
  const double sgn = r < 0.0 ? -1.0 : 1.0;         // solve for -D + |r| z z^T when r < 0
  const double inv = uncoupled ? 1.0 : 1.0 / sqrt(zz);
  for (int i = tid; i < N; i += NT) {
    L.d[i] *= sgn;
    L.z[i] *= inv;
  }
  r = fabs(r);
  __syncthreads();
  sort_poles<NT>(L, N);
  double mx = 0.0;
  for (int i = tid; i < N; i += NT) mx = fmax(mx, fabs(L.d[i]));
  mx = wg_max<NT>(mx, L.red);
  const double tol = 8.0 * kEps * fmax(mx, r);
  deflate<NT>(L, N, r, tol, uncoupled);
  const int n = L.misc[0];
  double zs = 0.0;
  for (int j = tid; j < n; j += NT) zs += L.z2[j];
  zs = wg_sum<NT>(zs, L.red);
  const double hi_b = n ? L.Dk[n - 1] + r * zs : 0.0;
  save_state<NT>(L, state_view(J.state, N), N, sgn, r, 1.0, 0.0, 0.0, hi_b);
}

// Finish of a merge: weights from the roots, the vectors, the deflation
// rotations and the sort undone -> W and Dout.
__global__ __launch_bounds__(kSecThreads) void k_dc_merge_fin(MergeJobs jobs) {
  extern __shared__ __align__(16) char lds_raw[];
  constexpr int NT = kSecThreads;
  const MergeJob& J = jobs.j[blockIdx.x];
  const int N = J.n1 + J.n2, tid = threadIdx.x;
  const SecLds L = carve_sec(lds_raw, N);
  const SecState S = state_view(J.state, N);
  const int n = (int)S.hdr[0];
  const double sgn = S.hdr[2], r = S.hdr[3];
  load_state<NT>(L, S, N, n);
  // Rebuilt weights: z_j^2 = (lam_j - d_j) / r prod_{i != j} (lam_i - d_j) / (d_i - d_j).
  for (int j = tid; j < n; j += NT) {
    const double dj = L.Dk[j];
    double p = -((dj - L.org[j]) - L.tau[j]) / r;
    for (int i = 0; i < n; ++i) {
      if (i == j) continue;
      p *= -((dj - L.org[i]) - L.tau[i]) / (L.Dk[i] - dj);
    }
    L.zh[j] = copysign(sqrt(fabs(p)), L.zh[j]);
  }
  __syncthreads();
  for (int i = tid; i < n; i += NT) {
    double q = 0.0;
    for (int j = 0; j < n; ++j) {
      const double v = L.zh[j] / ((L.Dk[j] - L.org[i]) - L.tau[i]);
      q += v * v;
    }
    L.cn[i] = 1.0 / sqrt(q);
  }
  __syncthreads();
  // X in sorted/rotated coordinates, column c = slot c: a deflated pole keeps
  // e_c, a live pole K[i] carries root i.
  double* X = J.X;
  for (int idx = tid; idx < N * N; idx += NT) X[idx] = 0.0;
  __syncthreads();
  for (int c = tid; c < N; c += NT)
    if (L.defl[c]) {
      X[c + (int64_t)c * N] = 1.0;
      J.Dout[c] = sgn * L.d[c];
    }
  for (int i = tid; i < n; i += NT) J.Dout[L.K[i]] = sgn * (L.org[i] + L.tau[i]);
  for (int idx = tid; idx < n * n; idx += NT) {
    const int jj = idx % n, i = idx / n;
    X[L.K[jj] + (int64_t)L.K[i] * N] = L.zh[jj] / ((L.Dk[jj] - L.org[i]) - L.tau[i]) * L.cn[i];
  }
  __syncthreads();
  rotate_rows<NT>(L, X, N, N);
  for (int idx = tid; idx < N * N; idx += NT) {
    const int rr = idx % N, c = idx / N;
    J.W[L.perm[rr] + (int64_t)c * N] = X[idx];
  }
}

// ------------------------------------------------------------ secular roots
// One wavefront per root; jobs list the problems of a launch with the first
// wavefront of each (root0) and the upper bound of its roots (cap).
struct RootJob {
  double* state;
  int cap, root0, arrow;
};
constexpr int kMaxRootJobs = 48;
struct RootJobs {
  RootJob j[kMaxRootJobs];
  int njobs;
};

__global__ __launch_bounds__(256) void k_dc_roots(RootJobs jobs) {
  const int gw = blockIdx.x * 4 + threadIdx.x / 64;
  int jb = 0;
  while (jb + 1 < jobs.njobs && gw >= jobs.j[jb + 1].root0) ++jb;
  const RootJob& J = jobs.j[jb];
  const int i = gw - J.root0;
  const SecState S = state_view(J.state, J.cap);
  const int n = (int)S.hdr[0];
  const double w = S.hdr[3], c0 = S.hdr[4], c1 = S.hdr[5], lo_b = S.hdr[6], hi_b = S.hdr[7];
  Root r;
  if (J.arrow) {                      // n + 1 roots interlacing the n poles
    if (i > n) return;
    if (n == 0) r = Root{c0, 0.0};
    else r = secular_root_wave(c0, c1, w, S.Dk, S.z2, n, i - 1, i < n ? i : -1, lo_b, hi_b);
  } else {                            // n roots, root i above pole i
    if (i >= n) return;
    r = secular_root_wave(c0, c1, w, S.Dk, S.z2, n, i, i + 1 < n ? i + 1 : -1, lo_b, hi_b);
  }
  if (threadIdx.x % 64 == 0) {
    S.org[i] = r.org;
    S.tau[i] = r.tau;
  }
}

// ------------------------------------------------------------ GEMM jobs
// C (M x N) = A (M x K) B (K x N), all column-major FP64 with arbitrary
// leading dimensions and offsets: 64 x 64 tiles, 256 threads, 4 x 4 outputs
// per thread.
struct GemmJob {
  const double* A;
  const double* B;
  double* C;
  int lda, ldb, ldc, M, N, K, tile0;
};
constexpr int kMaxGemmJobs = 48;
struct GemmJobs {
  GemmJob j[kMaxGemmJobs];
  int njobs;
};

__global__ __launch_bounds__(256) void k_dc_gemm(GemmJobs jobs) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  int jb = 0;
  while (jb + 1 < jobs.njobs && (int)blockIdx.x >= jobs.j[jb + 1].tile0) ++jb;
  const GemmJob& G = jobs.j[jb];
  const int tile = blockIdx.x - G.tile0;
  const int tm = (G.M + 63) / 64;
  const int r0 = (tile % tm) * 64, c0 = (tile / tm) * 64;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < G.K; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int kk = e / 64, rr = e % 64;
      const int gr = r0 + rr, gk = k0 + kk;
      As[kk][rr] = (gr < G.M && gk < G.K) ? G.A[gr + (int64_t)gk * G.lda] : 0.0;
      const int gc = c0 + rr;
      Bs[kk][rr] = (gk < G.K && gc < G.N) ? G.B[gk + (int64_t)gc * G.ldb] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tx + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][ty + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gr = r0 + tx + 16 * i, gc = c0 + ty + 16 * j;
      if (gr < G.M && gc < G.N) G.C[gr + (int64_t)gc * G.ldc] = acc[i][j];
    }
}

// ------------------------------------------------------------ host plan
struct Node {
  int lo, n, h, c1, c2;   // children indices into the node list (-1 for a leaf)
};

int plan_tail(std::vector<Node>& nodes, int lo, int n) {
  if (n <= kDcLeaf) {
    nodes.push_back(Node{lo, n, 0, -1, -1});
    return (int)nodes.size() - 1;
  }
  const int h1 = n / 2;
  const int a = plan_tail(nodes, lo, h1);
  const int b = plan_tail(nodes, lo + h1, n - h1);
  nodes.push_back(Node{lo, n, 1 + std::max(nodes[a].h, nodes[b].h), a, b});
  return (int)nodes.size() - 1;
}

hipError_t launch_gemm_jobs(const std::vector<GemmJob>& all, hipStream_t st) {
  for (size_t b = 0; b < all.size(); b += kMaxGemmJobs) {
    GemmJobs J{};
    int tiles = 0;
    J.njobs = (int)std::min(all.size() - b, (size_t)kMaxGemmJobs);
    for (int i = 0; i < J.njobs; ++i) {
      J.j[i] = all[b + i];
      J.j[i].tile0 = tiles;
      tiles += ((J.j[i].M + 63) / 64) * ((J.j[i].N + 63) / 64);
    }
    if (tiles == 0) continue;
    hipLaunchKernelGGL(k_dc_gemm, dim3(tiles), dim3(256), 0, st, J);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_roots(const std::vector<RootJob>& all, hipStream_t st) {
  for (size_t b = 0; b < all.size(); b += kMaxRootJobs) {
    RootJobs J{};
    J.njobs = (int)std::min(all.size() - b, (size_t)kMaxRootJobs);
    int waves = 0;
    for (int i = 0; i < J.njobs; ++i) {
      J.j[i] = all[b + i];
      J.j[i].root0 = waves;
      waves += all[b + i].cap;
    }
    if (waves == 0) continue;
    hipLaunchKernelGGL(k_dc_roots, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, J);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Each merge: prepare (one workgroup per job), roots (one wavefront per
// possible root over the whole device), finish (one workgroup per job).
hipError_t launch_merges(const std::vector<MergeJob>& all, hipStream_t st) {
  for (size_t b = 0; b < all.size(); b += kMaxMergeJobs) {
    MergeJobs J{};
    const int nj = (int)std::min(all.size() - b, (size_t)kMaxMergeJobs);
    int cap = 0;
    std::vector<RootJob> rj;
    for (int i = 0; i < nj; ++i) {
      J.j[i] = all[b + i];
      const int N = J.j[i].n1 + J.j[i].n2;
      cap = std::max(cap, N);
      rj.push_back(RootJob{J.j[i].state, N, 0, 0});
    }
    hipLaunchKernelGGL(k_dc_merge_prep, dim3(nj), dim3(kSecThreads), sec_lds_bytes(cap), st, J);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_roots(rj, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_dc_merge_fin, dim3(nj), dim3(kSecThreads), sec_lds_bytes(cap), st, J);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

int dc_max_m() { return kDcMaxM; }

namespace {
size_t state_doubles(int m) { return 64 * 32 + 12 * (size_t)m; }   // >= 28 per node + 10.5 per pole
}  // namespace

size_t dc_work_doubles(int m) {
  int t = m, H = 0;
  while (t > kDcLeaf) {
    t = (t + 1) / 2;
    ++H;
  }
  const size_t mm = (size_t)m * m;
  // Q and D per tail height, then W, X, QA, Zfin (m x m), DA, Droot (m) and
  // the secular states of one level (at most 64 nodes)
  return (size_t)(H + 1) * (mm + (size_t)m) + 4 * mm + 2 * (size_t)m + state_doubles(m) + 64;
}

// T_m from its packed structure: theta[k], s[k], alpha[m - k], beta[m - k - 1]
// where, for k > 0, alpha[0] = t_kk and beta[0] = t_{k+1,k} and the rest is
// the tail; for k = 0, alpha and beta are the whole tridiagonal.  `hs` is the
// packed structure on the host, `ds` the same on the device.  Results: *lam
// (m, unsorted) and *Z (m x m, leading dimension *ldz), inside `work`
// (dc_work_doubles(m) doubles).
hipError_t ritz_dc(int m, int k, const double* hs, const double* ds, double* work, const double** lam,
                   const double** Z, int* ldz, hipStream_t st) {
  if (m > kDcMaxM || m < 1 || k < 0 || k >= m) return hipErrorInvalidValue;
  const int t = k > 0 ? m - k - 1 : m;                        // tail length
  const double* h_alpha = hs + 2 * k;
  const double* h_beta = h_alpha + (m - k);
  const double* h_tb = k > 0 ? h_beta + 1 : h_beta;          // tail off-diagonal (host)
  const double* d_theta = ds;
  const double* d_s = ds + k;
  const double* d_ta = ds + 2 * k + (k > 0 ? 1 : 0);          // tail diagonal (device)
  const double* d_tb = ds + 2 * k + (m - k) + (k > 0 ? 1 : 0); // tail off-diagonal (device)
  std::vector<Node> nodes;
  int root = -1, H = 0;
  if (t > 0) {
    root = plan_tail(nodes, 0, t);
    H = nodes[root].h;
  }
  const size_t mm = (size_t)m * m;
  double* p = work;
  std::vector<double*> Qh(H + 1), Dh(H + 1);
  for (int h = 0; h <= H; ++h) {
    Qh[h] = p; p += mm;
    Dh[h] = p; p += m;
  }
  double* W = p; p += mm;
  double* X = p; p += mm;
  double* QA = p; p += mm;
  double* Zf = p; p += mm;
  double* DA = p; p += m;
  double* Dr = p; p += m;
  double* SB = p;   // secular states, reused level by level
  hipError_t e;
  if (t > 0) {   // leaves of the tail
    std::vector<int> leaves;
    for (int i = 0; i < (int)nodes.size(); ++i)
      if (nodes[i].h == 0) leaves.push_back(i);
    for (size_t b = 0; b < leaves.size(); b += 64) {
      LeafJobs J{};
      const int nl = (int)std::min(leaves.size() - b, (size_t)64);
      for (int i = 0; i < nl; ++i) {
        J.lo[i] = nodes[leaves[b + i]].lo;
        J.n[i] = nodes[leaves[b + i]].n;
      }
      hipLaunchKernelGGL(k_dc_leaves, dim3(nl), dim3(kLeafThreads), 0, st, J, d_ta, d_tb,
                         k > 0 ? h_beta[0] : 0.0, t, Dh[0], Qh[0]);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  if (k > 0) {   // the arrowhead, corner torn from the tail
    const double a = h_alpha[0] - (t > 0 ? h_beta[0] : 0.0);
    hipLaunchKernelGGL(k_dc_arrow_prep, dim3(1), dim3(kSecThreads), sec_lds_bytes(k + 1), st, d_theta,
                       d_s, a, k, SB);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_roots(std::vector<RootJob>{RootJob{SB, k + 1, 0, 1}}, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_dc_arrow_fin, dim3(1), dim3(kSecThreads), sec_lds_bytes(k + 1), st, k, SB, DA, QA,
                       X);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  for (int h = 1; h <= H; ++h) {   // tail merges, one launch (plus its GEMMs) per height
    std::vector<MergeJob> mj;
    std::vector<GemmJob> gj;
    size_t woff = 0, soff = 0;
    for (const Node& nd : nodes) {
      if (nd.h != h) continue;
      const Node& a = nodes[nd.c1];
      const Node& b = nodes[nd.c2];
      const int N = nd.n;
      MergeJob J{};
      J.D1 = Dh[a.h] + a.lo;
      J.D2 = Dh[b.h] + b.lo;
      J.Q1 = Qh[a.h] + a.lo + (int64_t)a.lo * t;
      J.Q2 = Qh[b.h] + b.lo + (int64_t)b.lo * t;
      J.ld1 = t;
      J.ld2 = t;
      J.zrow1 = a.n - 1;
      J.zrow2 = 0;
      J.n1 = a.n;
      J.n2 = b.n;
      J.rho = h_tb[a.lo + a.n - 1];
      J.Dout = Dh[h] + nd.lo;
      J.W = W + woff;
      J.X = X + woff;
      J.state = SB + soff;
      woff += (size_t)N * N;
      soff += (sec_state_doubles(N) + 7) & ~size_t(7);
      mj.push_back(J);
      gj.push_back(GemmJob{J.Q1, J.W, Qh[h] + nd.lo + (int64_t)nd.lo * t, t, N, t, a.n, N, a.n, 0});
      gj.push_back(GemmJob{J.Q2, J.W + a.n, Qh[h] + b.lo + (int64_t)nd.lo * t, t, N, t, b.n, N, b.n, 0});
    }
    if ((e = launch_merges(mj, st)) != hipSuccess) return e;
    if ((e = launch_gemm_jobs(gj, st)) != hipSuccess) return e;
  }
  if (k == 0) {
    *lam = Dh[H];
    *Z = Qh[H];
    *ldz = t;
    return hipSuccess;
  }
  if (t == 0) {
    *lam = DA;
    *Z = QA;
    *ldz = k + 1;
    return hipSuccess;
  }
  // root: merge the arrowhead with the tail across beta_k
  MergeJob J{};
  J.D1 = DA;
  J.D2 = Dh[H];
  J.Q1 = QA;
  J.Q2 = Qh[H];
  J.ld1 = k + 1;
  J.ld2 = t;
  J.zrow1 = k;
  J.zrow2 = 0;
  J.n1 = k + 1;
  J.n2 = t;
  J.rho = h_beta[0];
  J.Dout = Dr;
  J.W = W;
  J.X = X;
  J.state = SB;
  if ((e = launch_merges(std::vector<MergeJob>{J}, st)) != hipSuccess) return e;
  std::vector<GemmJob> gj{GemmJob{QA, W, Zf, k + 1, m, m, k + 1, m, k + 1, 0},
                          GemmJob{Qh[H], W + (k + 1), Zf + (k + 1), t, m, m, t, m, t, 0}};
  if ((e = launch_gemm_jobs(gj, st)) != hipSuccess) return e;
  *lam = Dr;
  *Z = Zf;
  *ldz = m;
  return hipSuccess;
}

}  // namespace jl
