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
//   residuals       FP64-accumulated apply of each candidate.
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
  double* misc;     // 16 scalars
  int* perm;        // mp
  int* pq;          // mp (pair table of a Jacobi round)
  int* conv;        // m
  int* order;       // m
};

template <typename S>
__host__ __device__ inline size_t lds_bytes(int64_t hmax, int m) {
  const int mp = m + (m & 1);
  size_t b = 0;
  b += 2 * 2 * (size_t)hmax * sizeof(cplx<S>);
  b += sizeof(double) * ((size_t)(m + 1) * m + 2 * (size_t)mp * mp + 4 * (m + 1) + 2 + 2 * mp +
                         3 * (mp / 2) + 16 + m + 16);
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
  L.misc = d; d += 16;
  int* ip = reinterpret_cast<int*>(d);
  L.perm = ip; ip += mp;
  L.pq = ip; ip += mp;
  L.conv = ip; ip += m;
  L.order = ip;
  return L;
}

// y = A x (RESID = false; returns t = x^H y in *t_re, *t_im) or the squared
// residual ||A x - lam x||^2 (RESID = true; C should be double).
template <typename S, typename C, int NT, bool RESID>
__device__ void wg_apply(const BatchProblem& pb, const cplx<S>* __restrict__ x, cplx<S>* __restrict__ y,
                         const Lds<S>& L, double lamv, double* t_re, double* t_im) {
  const int64_t h = pb.h;
  const cplx<S>* A11 = static_cast<const cplx<S>*>(pb.A11);
  const cplx<S>* A12 = static_cast<const cplx<S>*>(pb.A12);
  for (int64_t i = threadIdx.x; i < 2 * h; i += NT) L.sv[i] = x[i];
  __syncthreads();
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  double are = 0.0, aim = 0.0;
  for (int64_t r = w; r < h; r += NT / 64) {
    const cplx<S>* r11 = A11 + r * pb.ld;
    const cplx<S>* r12 = A12 + r * pb.ld;
    cx2<C> p{0, 0}, q{0, 0};
    auto acc = [&](const cplx<S>& m11, const cplx<S>& m12, int64_t c) {
      const cplx<S> a = L.sv[c], b = L.sv[h + c];
      const C m11r = m11.x, m11i = m11.y, m12r = m12.x, m12i = m12.y;
      const C ar = a.x, ai = a.y, br = b.x, bi = b.y;
      // p += A11 a + A12 b
      p.re += m11r * ar - m11i * ai + m12r * br - m12i * bi;
      p.im += m11r * ai + m11i * ar + m12r * bi + m12i * br;
      // q += A11 conj(b) - A12 conj(a)
      q.re += m11r * br + m11i * bi - m12r * ar - m12i * ai;
      q.im += -m11r * bi + m11i * br + m12r * ai - m12i * ar;
    };
    int64_t c = lane;
    for (; c + 3 * 64 < h; c += 4 * 64) {   // four steps' loads in flight together
      cplx<S> m11[4], m12[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        m11[k] = r11[c + 64 * k];
        m12[k] = r12[c + 64 * k];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < 4; ++k) acc(m11[k], m12[k], c + 64 * k);
    }
    for (; c < h; c += 64) acc(r11[c], r12[c], c);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      p.re += __shfl_xor(p.re, o);
      p.im += __shfl_xor(p.im, o);
      q.re += __shfl_xor(q.re, o);
      q.im += __shfl_xor(q.im, o);
    }
    if (lane == 0) {
      const cplx<S> xt = L.sv[r], xb = L.sv[h + r];
      if constexpr (RESID) {
        const double tr = (double)p.re - lamv * xt.x, ti = (double)p.im - lamv * xt.y;
        const double br2 = (double)q.re - lamv * xb.x, bi2 = -(double)q.im - lamv * xb.y;
        are += tr * tr + ti * ti + br2 * br2 + bi2 * bi2;
      } else {
        cplx<S> ut, ub;
        ut.x = (S)p.re; ut.y = (S)p.im;
        ub.x = (S)q.re; ub.y = (S)(-q.im);   // u_bot = conj(q)
        y[r] = ut;
        y[h + r] = ub;
        are += (double)xt.x * ut.x + (double)xt.y * ut.y + (double)xb.x * ub.x + (double)xb.y * ub.y;
        aim += (double)xt.x * ut.y - (double)xt.y * ut.x + (double)xb.x * ub.y - (double)xb.y * ub.x;
      }
    }
  }
  *t_re = wg_sum<NT>(are, L.red);
  if (!RESID) *t_im = wg_sum<NT>(aim, L.red);
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
    int64_t p = lane;
    for (; p + 3 * 64 < h; p += 4 * 64) {   // four steps' loads in flight together
      cplx<S> a[4], b[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        a[k] = vt[p + 64 * k];
        b[k] = vb[p + 64 * k];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < 4; ++k) acc(a[k], b[k], p + 64 * k);
    }
    for (; p < h; p += 64) acc(vt[p], vb[p], p);
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
    int c = 0;
    for (; c + 3 < ncol; c += 4) {   // four columns' loads in flight together
      cplx<S> a[4], b[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        a[k] = V[(int64_t)(c + k) * n + p];
        b[k] = V[(int64_t)(c + k) * n + h + p];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < 4; ++k) acc(a[k], b[k], c + k);
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

template <typename S, int NT>
__device__ void solve_one(const BatchProblem& pb, int pid, const BatchParams& P, char* slot,
                          const Lds<S>& L, const BatchOut& out) {
  const int64_t h = pb.h, n = 2 * h;
  const int m = P.m, nev = P.nev, mwin = P.mwin, tid = threadIdx.x;
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
  int k = 0, icnv = 0, status = 1, n_mv = 0, passes_tot = 0, cycles = 0;
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
      wg_apply<S, S, NT, false>(pb, V + (int64_t)j * n, u, L, 0.0, &tre, &tim);
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
    // ---- V_k := V_m Z[:, perm[0:kcols]], FP64 accumulation
    const int kcols = min(kmax, meff);
    for (int64_t e = tid; e < n; e += NT) {
      for (int c = 0; c < kcols; ++c) {
        const int src = L.perm[c];
        double ar = 0.0, ai = 0.0;
        for (int i = 0; i < meff; ++i) {
          const cplx<S> v = V[(int64_t)i * n + e];
          const double z = L.JZ[i + src * mp];
          ar += (double)v.x * z;
          ai += (double)v.y * z;
        }
        cplx<S> o;
        o.x = (S)ar; o.y = (S)ai;
        Vn[(int64_t)c * n + e] = o;
      }
    }
    __syncthreads();
    // ---- true residuals of the candidates
    tol_scale = fmax(tol_scale, fmax(fabs(L.lam[0]), fabs(L.lam[meff - 1])));
    const double tolc = P.tol_relative ? P.tol * tol_scale : P.tol;
    for (int i = 0; i < nev; ++i) {
      double r2 = INFINITY;
      if (fabs(L.svec[i]) < tolc) {
        double dummy;
        wg_apply<S, double, NT, true>(pb, Vn + (int64_t)i * n, nullptr, L, L.lam[i], &r2, &dummy);
        r2 = sqrt(r2);
      }
      if (tid == 0) {
        L.resv[i] = r2;
        L.conv[i] = r2 < tolc ? 1 : 0;
      }
    }
    __syncthreads();
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
    out.stats[4 * pid + 0] = cycles;
    out.stats[4 * pid + 1] = n_mv;
    out.stats[4 * pid + 2] = passes_tot;
    out.stats[4 * pid + 3] = icnv;
  }
  __syncthreads();
}

template <typename S, int NT>
__global__ __launch_bounds__(NT) void k_batched(const BatchProblem* __restrict__ probs,
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
    solve_one<S, NT>(probs[pid], pid, P, slot, L, out);
  }
}

__global__ void k_batched_init(int* queue) {
  if (threadIdx.x == 0) queue[0] = 0;
}

template <typename S, int NT>
hipError_t launch_nt(const BatchProblem* probs, const int* order, int count, const BatchParams& P,
                     int* queue, char* slots, size_t slot_bytes, int64_t hmax, const BatchOut& out,
                     int blocks, hipStream_t st) {
  const size_t lds = lds_bytes<S>(hmax, P.m);
  hipLaunchKernelGGL((k_batched<S, NT>), dim3(blocks), dim3(NT), lds, st, probs, order, count, P,
                     queue, slots, slot_bytes, hmax, out);
  return hipGetLastError();
}

}  // namespace

size_t batched_lds_bytes(int64_t hmax, int m, int es) {
  return es == 8 ? lds_bytes<float>(hmax, m) : lds_bytes<double>(hmax, m);
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
                          int64_t hmax, const BatchOut& out, int threads, int blocks,
                          hipStream_t st) {
  if (P.m + (P.m & 1) > kJacobiLdsMaxMp) return hipErrorInvalidValue;
  switch (threads) {
    case 128: return launch_nt<S, 128>(probs, order, count, P, queue, slots, slot_bytes, hmax, out, blocks, st);
    case 256: return launch_nt<S, 256>(probs, order, count, P, queue, slots, slot_bytes, hmax, out, blocks, st);
    case 512: return launch_nt<S, 512>(probs, order, count, P, queue, slots, slot_bytes, hmax, out, blocks, st);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_batched<float>(const BatchProblem*, const int*, int, const BatchParams&,
                                          int*, char*, size_t, int64_t, const BatchOut&, int, int,
                                          hipStream_t);
template hipError_t launch_batched<double>(const BatchProblem*, const int*, int,
                                           const BatchParams&, int*, char*, size_t, int64_t,
                                           const BatchOut&, int, int, hipStream_t);

}  // namespace jl
