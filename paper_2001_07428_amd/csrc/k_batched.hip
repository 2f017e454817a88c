// Batched J-symmetric thick-restart Lanczos: many independent dense problems
// of uneven size in one persistent launch.
//
// Each workgroup pops problem ids from an atomic queue (the host orders them
// by decreasing size, so the longest problems start first) and runs the whole
// of Algorithm 1 with Algorithm 2 as its inner step for that problem:
//   operator apply  [A11 A12] row by row (one wavefront per row, the row read
//                   once for both halves), t_jj accumulated on the fly;
//   local step      u -= t_jj v_j + beta_{j-1} v_{j-1};
//   Gram-Schmidt    against [V_j, J V_j^*] (W implicit), FP64 inner products,
//                   sqrt(2) test on the norms, as in the stand-alone solver;
//   Rayleigh-Ritz   parallel cyclic Jacobi on T in LDS (FP64) and a rank sort;
//   restart         V Z[:, :k] with FP64 accumulation;
//   residuals       FP64-accumulated applies, two candidates per pass over A.
// The basis lives in a per-workgroup slot of the workspace; vectors being
// worked on, T, the Jacobi matrices and all scalars live in LDS.  Control
// decisions are taken by every thread from the same LDS values, so the
// workgroup stays converged.
#include "common.h"
#include "jacobi.h"

namespace jl {
namespace {

template <typename C> struct cx2 { C re, im; };

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Sum over the workgroup, returned to every thread (fixed order).
template <int NT>
__device__ __forceinline__ double wg_sum(double v, double* red) {
  v = wsum(v);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

// LDS carve-up for one problem of at most hmax pairs and basis size m.
template <typename S> struct Lds {
  cplx<S>* sv;      // staged operand of the apply [2 hmax]
  cplx<S>* su;      // staged Lanczos vector u [2 hmax]
  double* T;        // (m+1) x m, T[i + j (m+1)]
  double* JA;       // mp x mp
  double* JZ;       // mp x mp
  double* coef;     // 4 (m+1) + 2
  double* lam;      // mp sorted Ritz values
  double* svec;     // mp arrow coefficients t_{m+1,i}
  double* rc; double* rs; double* rt;   // mp/2 rotations
  double* red;      // 16
  double* resv;     // m
  double* misc;     // 32 scalars
  int* perm;        // mp
  int* pq;          // mp (pair table of a Jacobi round)
  int* conv;        // m
  int* order;       // m
  cplx<S>* mat;     // [A11 A12] of a problem that fits BatchParams::lds_mat bytes (h x h each)
};

template <typename S>
__host__ __device__ inline size_t lds_bytes(int64_t hmax, int m) {
  const int mp = m + (m & 1);
  size_t b = 0;
  b += 2 * 2 * (size_t)hmax * sizeof(cplx<S>);
  b += sizeof(double) * ((size_t)(m + 1) * m + 2 * (size_t)mp * mp + 4 * (m + 1) + 2 + 2 * mp +
                         3 * (mp / 2) + 16 + m + 32);
  b += sizeof(int) * (2 * (size_t)mp + 2 * m);
  return b + 64;
}

template <typename S>
__device__ inline Lds<S> carve(char* base, int64_t hmax, int m) {
  const int mp = m + (m & 1);
  Lds<S> L;
  L.sv = reinterpret_cast<cplx<S>*>(base);
  L.su = L.sv + 2 * hmax;
  double* d = reinterpret_cast<double*>(L.su + 2 * hmax);
  L.T = d; d += (size_t)(m + 1) * m;
  L.JA = d; d += (size_t)mp * mp;
  L.JZ = d; d += (size_t)mp * mp;
  L.coef = d; d += 4 * (m + 1) + 2;
  L.lam = d; d += mp;
  L.svec = d; d += mp;
  L.rc = d; d += mp / 2;
  L.rs = d; d += mp / 2;
  L.rt = d; d += mp / 2;
  L.red = d; d += 16;
  L.resv = d; d += m;
  L.misc = d; d += 32;
  int* ip = reinterpret_cast<int*>(d);
  L.perm = ip; ip += mp;
  L.pq = ip; ip += mp;
  L.conv = ip; ip += m;
  L.order = ip;
  L.mat = reinterpret_cast<cplx<S>*>(base + ((lds_bytes<S>(hmax, m) + 15) & ~size_t(15)));
  return L;
}

// y = A x; returns t = x^H y in *t_re, *t_im.  Each wavefront takes RPW
// rows at a time (they share the operand reads from LDS) and every lane
// issues the matrix loads of UNR column steps before their products (the
// tile knobs the autotuner picks per batch).
template <typename S, typename C, int NT, int RPW, int UNR>
__device__ void wg_apply(const BatchProblem& pb, const cplx<S>* __restrict__ x, cplx<S>* __restrict__ y,
                         const Lds<S>& L, double* t_re, double* t_im) {
  const int64_t h = pb.h;
  const cplx<S>* A11 = static_cast<const cplx<S>*>(pb.A11);
  const cplx<S>* A12 = static_cast<const cplx<S>*>(pb.A12);
  for (int64_t i = threadIdx.x; i < 2 * h; i += NT) L.sv[i] = x[i];
  __syncthreads();
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  double are = 0.0, aim = 0.0;
  for (int64_t r0 = (int64_t)w * RPW; r0 < h; r0 += (int64_t)(NT / 64) * RPW) {
    const cplx<S>* r11[RPW];
    const cplx<S>* r12[RPW];
#pragma unroll
    for (int k = 0; k < RPW; ++k) {   // rows past the end repeat the last row; not stored
      const int64_t r = r0 + k < h ? r0 + k : h - 1;
      r11[k] = A11 + r * pb.ld;
      r12[k] = A12 + r * pb.ld;
    }
    cx2<C> p[RPW], q[RPW];
#pragma unroll
    for (int k = 0; k < RPW; ++k) p[k] = q[k] = cx2<C>{0, 0};
    auto acc = [&](const cplx<S>& m11, const cplx<S>& m12, const cplx<S>& a, const cplx<S>& b,
                   cx2<C>& pp, cx2<C>& qq) {
      const C m11r = m11.x, m11i = m11.y, m12r = m12.x, m12i = m12.y;
      const C ar = a.x, ai = a.y, br = b.x, bi = b.y;
      // p += A11 a + A12 b
      pp.re += m11r * ar - m11i * ai + m12r * br - m12i * bi;
      pp.im += m11r * ai + m11i * ar + m12r * bi + m12i * br;
      // q += A11 conj(b) - A12 conj(a)
      qq.re += m11r * br + m11i * bi - m12r * ar - m12i * ai;
      qq.im += -m11r * bi + m11i * br + m12r * ai - m12i * ar;
    };
    // UNR column steps' loads in flight together, every step loaded: columns
    // past the row's end read the last column and multiply as zero, so no
    // lane leaves the batch for a one-load-at-a-time tail (each lane sums its
    // columns lane, lane + 64, ... in order, whatever UNR)
    for (int64_t cb = 0; cb < h; cb += UNR * 64) {
      cplx<S> m11[RPW][UNR], m12[RPW][UNR];
#pragma unroll
      for (int k = 0; k < RPW; ++k)
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int64_t c = cb + lane + 64 * u;
          const int64_t cc = c < h ? c : h - 1;
          m11[k][u] = r11[k][cc];
          m12[k][u] = r12[k][cc];
        }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int64_t c = cb + lane + 64 * u;
        const bool in = c < h;
        const int64_t cc = in ? c : 0;
        const cplx<S> a = L.sv[cc], b = L.sv[h + cc];
        const cplx<S> zero = {(S)0, (S)0};
#pragma unroll
        for (int k = 0; k < RPW; ++k)
          acc(in ? m11[k][u] : zero, in ? m12[k][u] : zero, a, b, p[k], q[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        p[k].re += __shfl_xor(p[k].re, o);
        p[k].im += __shfl_xor(p[k].im, o);
        q[k].re += __shfl_xor(q[k].re, o);
        q[k].im += __shfl_xor(q[k].im, o);
      }
    }
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < RPW; ++k) {
        const int64_t r = r0 + k;
        if (r >= h) break;
        const cplx<S> xt = L.sv[r], xb = L.sv[h + r];
        cplx<S> ut, ub;
        ut.x = (S)p[k].re; ut.y = (S)p[k].im;
        ub.x = (S)q[k].re; ub.y = (S)(-q[k].im);   // u_bot = conj(q)
        y[r] = ut;
        y[h + r] = ub;
        are += (double)xt.x * ut.x + (double)xt.y * ut.y + (double)xb.x * ub.x + (double)xb.y * ub.y;
        aim += (double)xt.x * ut.y - (double)xt.y * ut.x + (double)xb.x * ub.y - (double)xb.y * ub.x;
      }
    }
  }
  *t_re = wg_sum<NT>(are, L.red);
  *t_im = wg_sum<NT>(aim, L.red);
}

// Squared true residuals ||A x_k - lam_k x_k||^2 of nc <= kResRhs candidates
// x_k = X + idx[k] * n in one pass over [A11 A12] (the operator is read once
// per kResRhs candidates, not once per candidate): the lanes of a wavefront
// split as 4 rows x 16 column groups (128 contiguous bytes of a row per load
// in FP32), each lane applies its row's entries to every candidate (the
// candidates are read through the caches, the 4 row lanes of a column group at
// one address), FP64 products and accumulation; the column groups are summed
// by four butterfly steps.  r2[k] (LDS) receives the sums.  Two candidates
// per pass keep the solver's register count (and so its occupancy) where it
// was: four cost 50 more registers.  With UR > 1 every lane issues the loads
// of UR column steps (matrix entries and candidates) before their products,
// the last batch padded with zero-weight columns; 512-thread workgroups,
// whose register budget has room, take UR = 4.
constexpr int kResRhs = 2;
template <typename S, int NT, int UR = 1>
__device__ void wg_resid_multi(const BatchProblem& pb, const cplx<S>* __restrict__ X, int64_t n,
                               const int* idx, const double* lamv, int nc, const Lds<S>& L,
                               double* r2) {
  const int64_t h = pb.h;
  const cplx<S>* A11 = static_cast<const cplx<S>*>(pb.A11);
  const cplx<S>* A12 = static_cast<const cplx<S>*>(pb.A12);
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64, ri = lane >> 4, g = lane & 15;
  const cplx<S>* xk[kResRhs];
  double lk[kResRhs];
#pragma unroll
  for (int k = 0; k < kResRhs; ++k) {
    xk[k] = X + (int64_t)idx[k < nc ? k : 0] * n;
    lk[k] = k < nc ? lamv[k] : 0.0;
  }
  double acc[kResRhs];
#pragma unroll
  for (int k = 0; k < kResRhs; ++k) acc[k] = 0.0;
  for (int64_t rb = (int64_t)w * 4; rb < h; rb += (int64_t)(NT / 64) * 4) {
    const int64_t r = rb + ri;
    const bool rok = r < h;
    const cplx<S>* r11 = A11 + (rok ? r : h - 1) * pb.ld;
    const cplx<S>* r12 = A12 + (rok ? r : h - 1) * pb.ld;
    double pr[kResRhs], pi[kResRhs], qr[kResRhs], qi[kResRhs];
#pragma unroll
    for (int k = 0; k < kResRhs; ++k) pr[k] = pi[k] = qr[k] = qi[k] = 0.0;
    int64_t c0 = g;
    if constexpr (UR > 1) {
      // every column step and candidate slot is loaded: columns past the
      // row's end read the last column and multiply as zero, slots past nc
      // read candidate 0 and are never summed; no branch closes the batch
      for (int64_t cb = 0; cb < h; cb += UR * 16) {
        cplx<S> m11[UR], m12[UR], xa[UR][kResRhs], xb[UR][kResRhs];
#pragma unroll
        for (int u = 0; u < UR; ++u) {
          const int64_t c = cb + g + 16 * u;
          const int64_t cc = c < h ? c : h - 1;
          m11[u] = r11[cc];
          m12[u] = r12[cc];
#pragma unroll
          for (int k = 0; k < kResRhs; ++k) {
            xa[u][k] = xk[k][cc];
            xb[u][k] = xk[k][h + cc];
          }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < UR; ++u) {
          const bool in = cb + g + 16 * u < h;
          const double m11r = in ? (double)m11[u].x : 0.0, m11i = in ? (double)m11[u].y : 0.0;
          const double m12r = in ? (double)m12[u].x : 0.0, m12i = in ? (double)m12[u].y : 0.0;
#pragma unroll
          for (int k = 0; k < kResRhs; ++k) {
            const double ar = xa[u][k].x, ai = xa[u][k].y, br = xb[u][k].x, bi = xb[u][k].y;
            pr[k] += m11r * ar - m11i * ai + m12r * br - m12i * bi;
            pi[k] += m11r * ai + m11i * ar + m12r * bi + m12i * br;
            qr[k] += m11r * br + m11i * bi - m12r * ar - m12i * ai;
            qi[k] += -m11r * bi + m11i * br + m12r * ai - m12i * ar;
          }
        }
      }
      c0 = h;   // nothing left for the single-step loop
    }
    for (int64_t c = c0; c < h; c += 16) {
      const cplx<S> m11 = r11[c], m12 = r12[c];
      const double m11r = m11.x, m11i = m11.y, m12r = m12.x, m12i = m12.y;
#pragma unroll
      for (int k = 0; k < kResRhs; ++k) {
        if (k >= nc) break;   // uniform
        const cplx<S> a = xk[k][c], b = xk[k][h + c];
        const double ar = a.x, ai = a.y, br = b.x, bi = b.y;
        // p += A11 a + A12 b;  q += A11 conj(b) - A12 conj(a)
        pr[k] += m11r * ar - m11i * ai + m12r * br - m12i * bi;
        pi[k] += m11r * ai + m11i * ar + m12r * bi + m12i * br;
        qr[k] += m11r * br + m11i * bi - m12r * ar - m12i * ai;
        qi[k] += -m11r * bi + m11i * br + m12r * ai - m12i * ar;
      }
    }
#pragma unroll
    for (int k = 0; k < kResRhs; ++k) {
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        pr[k] += __shfl_xor(pr[k], o); pi[k] += __shfl_xor(pi[k], o);
        qr[k] += __shfl_xor(qr[k], o); qi[k] += __shfl_xor(qi[k], o);
      }
    }
    if (g == 0 && rok) {
#pragma unroll
      for (int k = 0; k < kResRhs; ++k) {
        if (k >= nc) break;
        const cplx<S> xt = xk[k][r], xb = xk[k][h + r];
        const double tr = pr[k] - lk[k] * xt.x, ti = pi[k] - lk[k] * xt.y;
        const double br = qr[k] - lk[k] * xb.x, bi = -qi[k] - lk[k] * xb.y;   // u_bot = conj(q)
        acc[k] += tr * tr + ti * ti + br * br + bi * bi;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kResRhs; ++k) {
    if (k < nc) {   // uniform
      const double t = wg_sum<NT>(acc[k], L.red);
      if (threadIdx.x == 0) r2[k] = t;
    }
  }
  __syncthreads();
}

// First half of a Gram-Schmidt pass: optional local step on u (stored back),
// then coef[4c..4c+3] = (v_c^H u, w_c^H u) for c < ncol and
// coef[4 ncol] = ||u||^2.  u is staged in L.su.
template <typename S, int NT>
__device__ void wg_dots(const cplx<S>* __restrict__ V, int64_t n, int ncol, cplx<S>* __restrict__ u,
                        int64_t h, const Lds<S>& L, bool local, double tre, double tim, double beta,
                        int jl) {
  double nrm = 0.0;
  const cplx<S>* vj = V + (int64_t)jl * n;
  const cplx<S>* vm = vj - n;
  for (int64_t p = threadIdx.x; p < 2 * h; p += NT) {
    cplx<S> x = u[p];
    if (local) {
      const cplx<S> a = vj[p];
      double xr = (double)x.x - (tre * a.x - tim * a.y);
      double xi = (double)x.y - (tre * a.y + tim * a.x);
      if (beta != 0.0) {
        const cplx<S> b = vm[p];
        xr -= beta * b.x;
        xi -= beta * b.y;
      }
      x.x = (S)xr;
      x.y = (S)xi;
      u[p] = x;
    }
    L.su[p] = x;
    nrm += (double)x.x * x.x + (double)x.y * x.y;
  }
  nrm = wg_sum<NT>(nrm, L.red);   // also orders the L.su writes before the reads below
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  for (int c = w; c < ncol; c += NT / 64) {
    const cplx<S>* vt = V + (int64_t)c * n;
    const cplx<S>* vb = vt + h;
    double cvr = 0, cvi = 0, cwr = 0, cwi = 0;
    auto acc = [&](const cplx<S>& a, const cplx<S>& b, int64_t p) {
      const cplx<S> ut = L.su[p], ub = L.su[h + p];
      const double vtr = a.x, vti = a.y, vbr = b.x, vbi = b.y;
      const double utr = ut.x, uti = ut.y, ubr = ub.x, ubi = ub.y;
      cvr += vtr * utr + vti * uti + vbr * ubr + vbi * ubi;
      cvi += vtr * uti - vti * utr + vbr * ubi - vbi * ubr;
      cwr += vtr * ubr - vti * ubi - vbr * utr + vbi * uti;
      cwi += vtr * ubi + vti * ubr - vbr * uti - vbi * utr;
    };
    // DS steps' loads in flight together, every step loaded: pairs past the
    // end read the last pair and are not summed (each lane sums its pairs
    // lane, lane + 64, ... in order)
    constexpr int DS = NT >= 512 ? 8 : 4;
    for (int64_t pb = 0; pb < h; pb += DS * 64) {
      cplx<S> a[DS], b[DS];
#pragma unroll
      for (int k = 0; k < DS; ++k) {
        const int64_t p = pb + lane + 64 * k;
        const int64_t pc = p < h ? p : h - 1;
        a[k] = vt[pc];
        b[k] = vb[pc];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < DS; ++k) {
        const int64_t p = pb + lane + 64 * k;
        if (p < h) acc(a[k], b[k], p);
      }
    }
    cvr = wsum(cvr); cvi = wsum(cvi); cwr = wsum(cwr); cwi = wsum(cwi);
    if (lane == 0) {
      L.coef[4 * c + 0] = cvr; L.coef[4 * c + 1] = cvi;
      L.coef[4 * c + 2] = cwr; L.coef[4 * c + 3] = cwi;
    }
  }
  if (threadIdx.x == 0) L.coef[4 * ncol] = nrm;
  __syncthreads();
}

// Second half of the pass: u -= V c_v + W c_w (u from L.su, written to both);
// returns ||u||^2.
template <typename S, int NT>
__device__ double wg_update(const cplx<S>* __restrict__ V, int64_t n, int ncol,
                            cplx<S>* __restrict__ u, int64_t h, const Lds<S>& L) {
  double nrm = 0.0;
  for (int64_t p = threadIdx.x; p < h; p += NT) {
    double dtr = 0, dti = 0, dbr = 0, dbi = 0;
    auto acc = [&](const cplx<S>& a, const cplx<S>& b, int c) {
      const double cvr = L.coef[4 * c], cvi = L.coef[4 * c + 1];
      const double cwr = L.coef[4 * c + 2], cwi = L.coef[4 * c + 3];
      const double tr = a.x, ti = a.y, br = b.x, bi = b.y;
      dtr += tr * cvr - ti * cvi - br * cwr - bi * cwi;
      dti += tr * cvi + ti * cvr - br * cwi + bi * cwr;
      dbr += br * cvr - bi * cvi + tr * cwr + ti * cwi;
      dbi += br * cvi + bi * cvr + tr * cwi - ti * cwr;
    };
    // UC columns' loads in flight together (the columns are summed in order)
    constexpr int UC = NT >= 512 ? 8 : 4;
    int c = 0;
    for (; c + UC - 1 < ncol; c += UC) {
      cplx<S> a[UC], b[UC];
#pragma unroll
      for (int k = 0; k < UC; ++k) {
        a[k] = V[(int64_t)(c + k) * n + p];
        b[k] = V[(int64_t)(c + k) * n + h + p];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < UC; ++k) acc(a[k], b[k], c + k);
    }
    for (; c < ncol; ++c) acc(V[(int64_t)c * n + p], V[(int64_t)c * n + h + p], c);
    cplx<S> t = L.su[p], b = L.su[h + p];
    t.x = (S)((double)t.x - dtr); t.y = (S)((double)t.y - dti);
    b.x = (S)((double)b.x - dbr); b.y = (S)((double)b.y - dbi);
    L.su[p] = t; L.su[h + p] = b;
    u[p] = t; u[h + p] = b;
    nrm += (double)t.x * t.x + (double)t.y * t.y + (double)b.x * b.x + (double)b.y * b.y;
  }
  return wg_sum<NT>(nrm, L.red);
}

template <typename S, int NT, int RPW, int UNR>
__device__ void solve_one(const BatchProblem& pg, int pid, const BatchParams& P, char* slot,
                          const Lds<S>& L, const BatchOut& out) {
  const int64_t h = pg.h, n = 2 * h;
  const int m = P.m, nev = P.nev, mwin = P.mwin, tid = threadIdx.x;
  // a matrix that fits the launch's LDS budget is read from LDS for the whole solve
  BatchProblem pb = pg;
  if ((size_t)2 * h * h * sizeof(cplx<S>) <= (size_t)P.lds_mat) {
    const cplx<S>* A11 = static_cast<const cplx<S>*>(pg.A11);
    const cplx<S>* A12 = static_cast<const cplx<S>*>(pg.A12);
    for (int64_t i = tid; i < h * h; i += NT) {
      const int64_t r = i / h, c = i - r * h;
      L.mat[i] = A11[r * pg.ld + c];
      L.mat[h * h + i] = A12[r * pg.ld + c];
    }
    pb.A11 = L.mat;
    pb.A12 = L.mat + h * h;
    pb.ld = h;
    __syncthreads();
  }
  const int kmax = min(nev + mwin, m - 1);
  const double uround = sizeof(S) == 4 ? 5.9604644775390625e-08 : 1.1102230246251565e-16;
  cplx<S>* Vb[2] = {reinterpret_cast<cplx<S>*>(slot), reinterpret_cast<cplx<S>*>(slot) + (size_t)(m + 1) * n};
  int cur = 0;
  {
    const S v0 = (S)(1.0 / sqrt((double)n));
    for (int64_t i = tid; i < n; i += NT) {
      cplx<S> z;
      z.x = v0; z.y = (S)0;
      Vb[0][i] = z;
    }
  }
  for (int i = tid; i < (m + 1) * m; i += NT) L.T[i] = 0.0;
  __syncthreads();
  auto Tat = [&](int i, int j) -> double& { return L.T[i + j * (m + 1)]; };
  int k = 0, icnv = 0, status = 1, n_mv = 0, passes_tot = 0, cycles = 0, n_resid = 0;
  // wall-clock ticks per phase (read at points where the workgroup is in step)
  long long ph[kBatchPhases] = {};
  long long t_mark = wall_clock64();
  auto phase = [&](int i) {
    const long long t = wall_clock64();
    ph[i] += t - t_mark;
    t_mark = t;
  };
  double maxT = 0.0, tol_scale = 0.0;
  const double sqrt2 = 1.4142135623730951;
  for (int cycle = 0; cycle < P.max_cycles; ++cycle) {
    ++cycles;
    cplx<S>* V = Vb[cur];
    cplx<S>* Vn = Vb[1 - cur];
    int meff = m;
    bool broke = false;
    for (int j = k; j < m; ++j) {
      cplx<S>* u = V + (int64_t)(j + 1) * n;
      double tre, tim;
      phase(1);   // the previous step's normalisation belongs to Gram-Schmidt
      wg_apply<S, S, NT, RPW, UNR>(pb, V + (int64_t)j * n, u, L, &tre, &tim);
      phase(0);
      ++n_mv;
      const double beta_prev = (j > k) ? Tat(j, j - 1) : 0.0;
      wg_dots<S, NT>(V, n, j + 1, u, h, L, true, tre, tim, beta_prev, j);
      double b0 = sqrt(L.coef[4 * (j + 1)]);
      double b1 = sqrt(wg_update<S, NT>(V, n, j + 1, u, h, L));
      if (tid == 0) Tat(j, j) = tre;
      maxT = fmax(maxT, fabs(tre));   // identical in every thread
      const double btol = 64.0 * uround * fmax(maxT, 1e-300);
      int passes = 1;
      while (!(passes >= P.min_passes && b1 * sqrt2 > b0) && b1 > btol && passes < P.max_passes) {
        b0 = b1;
        wg_dots<S, NT>(V, n, j + 1, u, h, L, false, 0.0, 0.0, 0.0, j);
        b1 = sqrt(wg_update<S, NT>(V, n, j + 1, u, h, L));
        ++passes;
      }
      passes_tot += passes;
      __syncthreads();
      if (b1 <= btol) {
        if (tid == 0) Tat(j + 1, j) = 0.0;
        meff = j + 1;
        broke = true;
        __syncthreads();
        break;
      }
      const double inv = 1.0 / b1;
      for (int64_t i = tid; i < n; i += NT) {
        cplx<S> z = u[i];
        z.x = (S)((double)z.x * inv);
        z.y = (S)((double)z.y * inv);
        u[i] = z;
      }
      if (tid == 0) Tat(j + 1, j) = b1;
      maxT = fmax(maxT, b1);
      __syncthreads();
    }
    phase(1);
    if (meff < nev) { status = 2; icnv = 0; break; }
    // ---- Rayleigh-Ritz in LDS
    const int mp = meff + (meff & 1);
    for (int idx = tid; idx < mp * mp; idx += NT) {
      const int i = idx % mp, jj = idx / mp;
      double v = 0.0;
      if (i < meff && jj < meff) v = i >= jj ? Tat(i, jj) : Tat(jj, i);
      L.JA[idx] = v;
      L.JZ[idx] = (i == jj) ? 1.0 : 0.0;
    }
    __syncthreads();
    jacobi_lds<NT>(L.JA, L.JZ, mp, L.rc, L.rs, L.rt, L.pq, L.red, 60);
    for (int i = tid; i < meff; i += NT) {
      const double li = L.JA[i + i * mp];
      int rank = 0;
      for (int jj = 0; jj < meff; ++jj) {
        const double lj = L.JA[jj + jj * mp];
        const double a = isnan(lj) ? INFINITY : lj, b = isnan(li) ? INFINITY : li;
        const bool before = P.which ? (a > b || (a == b && jj < i)) : (a < b || (a == b && jj < i));
        rank += before ? 1 : 0;
      }
      L.perm[rank < meff ? rank : meff - 1] = i;
    }
    __syncthreads();
    const double beta_m = Tat(meff, meff - 1);
    for (int r = tid; r < meff; r += NT) {
      const int src = L.perm[r];
      L.lam[r] = L.JA[src + src * mp];
      L.svec[r] = beta_m * L.JZ[(meff - 1) + src * mp];
    }
    __syncthreads();
    phase(2);
    // ---- V_k := V_m Z[:, perm[0:kcols]], FP64 accumulation, four output
    // columns per read of V
    const int kcols = min(kmax, meff);
    constexpr int CB = 4;
    for (int64_t e = tid; e < n; e += NT) {
      for (int c0 = 0; c0 < kcols; c0 += CB) {
        double ar[CB], ai[CB];
        int src[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          ar[c] = ai[c] = 0.0;
          src[c] = L.perm[c0 + c < kcols ? c0 + c : c0];
        }
        for (int i = 0; i < meff; ++i) {
          const cplx<S> v = V[(int64_t)i * n + e];
          const double vr = v.x, vi = v.y;
#pragma unroll
          for (int c = 0; c < CB; ++c) {
            const double z = L.JZ[i + src[c] * mp];
            ar[c] += vr * z;
            ai[c] += vi * z;
          }
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          if (c0 + c < kcols) {
            cplx<S> o;
            o.x = (S)ar[c]; o.y = (S)ai[c];
            Vn[(int64_t)(c0 + c) * n + e] = o;
          }
        }
      }
    }
    __syncthreads();
    phase(3);
    // ---- true residuals of the candidates
    tol_scale = fmax(tol_scale, fmax(fabs(L.lam[0]), fabs(L.lam[meff - 1])));
    const double tolc = P.tol_relative ? P.tol * tol_scale : P.tol;
    // candidates (est < tol) in chunks of kResRhs, each chunk one pass over A
    if (tid == 0) {
      int nc = 0;
      for (int i = 0; i < nev; ++i) {
        L.resv[i] = INFINITY;
        L.conv[i] = 0;
        if (fabs(L.svec[i]) < tolc) L.order[nc++] = i;   // L.order: candidate list for now
      }
      L.misc[0] = nc;
    }
    __syncthreads();
    const int ncand = (int)L.misc[0];
    n_resid += ncand;
    for (int c0 = 0; c0 < ncand; c0 += kResRhs) {
      const int nc = min(kResRhs, ncand - c0);
      double* r2 = L.misc + 16;   // kResRhs scalars
      if (tid < nc) L.misc[1 + tid] = L.lam[L.order[c0 + tid]];   // slots 1..kResRhs
      __syncthreads();
      wg_resid_multi<S, NT, (NT >= 512 ? 4 : 1)>(pb, Vn, n, L.order + c0, L.misc + 1, nc, L, r2);
      if (tid < nc) {
        const int i = L.order[c0 + tid];
        const double r = sqrt(r2[tid]);
        L.resv[i] = r;
        L.conv[i] = r < tolc ? 1 : 0;
      }
      __syncthreads();
    }
    phase(4);
    icnv = 0;
    for (int i = 0; i < nev; ++i) icnv += L.conv[i];
    if (tid == 0) {
      int o = 0;
      for (int i = 0; i < nev; ++i) if (L.conv[i]) L.order[o++] = i;
      for (int i = 0; i < nev; ++i) if (!L.conv[i]) L.order[o++] = i;
    }
    __syncthreads();
    const bool last = cycle + 1 == P.max_cycles;
    if (icnv == nev || broke || last) {
      status = icnv == nev ? 0 : (broke ? 2 : 1);
      cur = 1 - cur;
      break;
    }
    // ---- shrink (eq. dynamicwin)
    k = min(icnv + mwin, m - 1);
    for (int i = tid; i < (m + 1) * m; i += NT) L.T[i] = 0.0;
    __syncthreads();
    maxT = 0.0;
    for (int i = 0; i < k; ++i) {
      const double si = (i < nev && L.conv[i]) ? 0.0 : L.svec[i];
      maxT = fmax(maxT, fmax(fabs(L.lam[i]), fabs(si)));
    }
    if (tid == 0)
      for (int i = 0; i < k; ++i) {
        Tat(i, i) = L.lam[i];
        Tat(k, i) = (i < nev && L.conv[i]) ? 0.0 : L.svec[i];
      }
    for (int64_t e = tid; e < n; e += NT) Vn[(int64_t)k * n + e] = V[(int64_t)meff * n + e];
    __syncthreads();
    cur = 1 - cur;
  }
  // ---- outputs
  cplx<S>* X = static_cast<cplx<S>*>(pb.X);
  if (status != 2 || icnv > 0) {
    const cplx<S>* Vf = Vb[cur];
    for (int c = 0; c < nev; ++c) {
      const int i = L.order[c];
      for (int64_t e = tid; e < n; e += NT) X[(int64_t)c * pb.ldx + e] = Vf[(int64_t)i * n + e];
      if (tid == 0) {
        out.evals[(int64_t)pid * nev + c] = L.lam[i];
        out.res[(int64_t)pid * nev + c] = L.resv[i];
      }
    }
  } else if (tid == 0) {
    for (int c = 0; c < nev; ++c) {
      out.evals[(int64_t)pid * nev + c] = NAN;
      out.res[(int64_t)pid * nev + c] = INFINITY;
    }
  }
  if (tid == 0) {
    out.status[pid] = status == 0 ? 0 : (status == 2 ? 2 : 1);
    out.stats[kBatchStats * pid + 0] = cycles;
    out.stats[kBatchStats * pid + 1] = n_mv;
    out.stats[kBatchStats * pid + 2] = passes_tot;
    out.stats[kBatchStats * pid + 3] = icnv;
    out.stats[kBatchStats * pid + 4] = n_resid;
#pragma unroll
    for (int i = 0; i < kBatchPhases; ++i) out.stats[kBatchStats * pid + 5 + i] = (int)min(ph[i], 0x7fffffffLL);
  }
  __syncthreads();
}

// Launch bounds: with 256 threads and the smallest apply tile, three
// workgroups (three wavefronts per SIMD) per compute unit; the FP64 solver's
// register count sits just above that limit otherwise.  The larger tiles keep
// their registers.
template <int NT, int RPW, int UNR> constexpr int batched_min_blocks() {
  return (NT == 256 && RPW * UNR == 4) ? 3 : 1;
}

template <typename S, int NT, int RPW, int UNR>
__global__ __launch_bounds__(NT, (batched_min_blocks<NT, RPW, UNR>())) void k_batched(const BatchProblem* __restrict__ probs,
                                                const int* __restrict__ order, int count,
                                                BatchParams P, int* queue, char* slots,
                                                size_t slot_bytes, int64_t hmax, BatchOut out) {
  extern __shared__ __align__(16) char lds_raw[];
  __shared__ int next;
  const Lds<S> L = carve<S>(lds_raw, hmax, P.m);
  char* slot = slots + (size_t)blockIdx.x * slot_bytes;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(queue, 1);
    __syncthreads();
    const int q = next;
    __syncthreads();
    if (q >= count) break;
    const int pid = order[q];
    solve_one<S, NT, RPW, UNR>(probs[pid], pid, P, slot, L, out);
  }
}

__global__ void k_batched_init(int* queue) {
  if (threadIdx.x == 0) queue[0] = 0;
}

template <typename S, int NT, int RPW, int UNR>
hipError_t launch_nt(const BatchProblem* probs, const int* order, int count, const BatchParams& P,
                     int* queue, char* slots, size_t slot_bytes, int64_t hmax, const BatchOut& out,
                     int blocks, hipStream_t st) {
  const size_t lds = ((lds_bytes<S>(hmax, P.m) + 15) & ~size_t(15)) + (size_t)P.lds_mat;
  hipLaunchKernelGGL((k_batched<S, NT, RPW, UNR>), dim3(blocks), dim3(NT), lds, st, probs, order, count,
                     P, queue, slots, slot_bytes, hmax, out);
  return hipGetLastError();
}

template <typename S, int NT>
hipError_t launch_tile(const BatchProblem* probs, const int* order, int count, const BatchParams& P,
                       int* queue, char* slots, size_t slot_bytes, int64_t hmax, const BatchOut& out,
                       int rpw, int unr, int blocks, hipStream_t st) {
  if (rpw == 1 && unr == 4)
    return launch_nt<S, NT, 1, 4>(probs, order, count, P, queue, slots, slot_bytes, hmax, out, blocks, st);
  if (rpw == 1 && unr == 8)
    return launch_nt<S, NT, 1, 8>(probs, order, count, P, queue, slots, slot_bytes, hmax, out, blocks, st);
  if (rpw == 2 && unr == 4)
    return launch_nt<S, NT, 2, 4>(probs, order, count, P, queue, slots, slot_bytes, hmax, out, blocks, st);
  if (rpw == 2 && unr == 8)
    return launch_nt<S, NT, 2, 8>(probs, order, count, P, queue, slots, slot_bytes, hmax, out, blocks, st);
  return hipErrorInvalidValue;
}

}  // namespace

size_t batched_lds_bytes(int64_t hmax, int m, int es) {
  return ((es == 8 ? lds_bytes<float>(hmax, m) : lds_bytes<double>(hmax, m)) + 15) & ~size_t(15);
}

size_t batched_slot_bytes(int64_t hmax, int m, int es) {
  return ((size_t)2 * (m + 1) * 2 * hmax * es + 255) & ~size_t(255);
}

hipError_t launch_batched_init(int* queue, hipStream_t st) {
  hipLaunchKernelGGL(k_batched_init, dim3(1), dim3(64), 0, st, queue);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_batched(const BatchProblem* probs, const int* order, int count,
                          const BatchParams& P, int* queue, char* slots, size_t slot_bytes,
                          int64_t hmax, const BatchOut& out, int threads, int rpw, int unr,
                          int blocks, hipStream_t st) {
  if (P.m + (P.m & 1) > kJacobiLdsMaxMp) return hipErrorInvalidValue;
  switch (threads) {
    case 128: return launch_tile<S, 128>(probs, order, count, P, queue, slots, slot_bytes, hmax, out, rpw, unr, blocks, st);
    case 256: return launch_tile<S, 256>(probs, order, count, P, queue, slots, slot_bytes, hmax, out, rpw, unr, blocks, st);
    case 512: return launch_tile<S, 512>(probs, order, count, P, queue, slots, slot_bytes, hmax, out, rpw, unr, blocks, st);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_batched<float>(const BatchProblem*, const int*, int, const BatchParams&,
                                          int*, char*, size_t, int64_t, const BatchOut&, int, int,
                                          int, int, hipStream_t);
template hipError_t launch_batched<double>(const BatchProblem*, const int*, int,
                                           const BatchParams&, int*, char*, size_t, int64_t,
                                           const BatchOut&, int, int, int, int, hipStream_t);

}  // namespace jl
