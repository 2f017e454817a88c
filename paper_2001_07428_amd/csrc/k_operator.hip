// Operator applies for the J-symmetric eigensolver (gfx950).
//
// Both operators only need A11 and A12 (Sec. 1, eq. blockform):
//   u_top = A11 a + A12 b,   u_bot = A12^H a + A11^T b
// for v = [a; b].
//
// Stencil: one thread per lattice site computes all 4 internal components of
// both halves; the link U_mu(x) is read once for the forward hop of both
// halves and U_mu(x - mu) once for the backward hop, from the operator's
// tiled copy of the links (coalesced across the wavefront).  Each hop
// issues its 16 link loads and the neighbour's loads together before any
// product.
// Dense: one wavefront per row of [A11 A12]; the row is read once for both
// right-hand sides [a; b] and [conj(b); -conj(a)] (u_bot = conj(A11 conj(b) -
// A12 conj(a)) because A11^T = conj(A11) and A12^H = -conj(A12)).
// Every apply can take its operand as the conjugate-gradient direction
// p = r + beta p_old, formed on the fly and stored (Operand below), and can
// return at once on a device flag (StencilArgs::skip, DenseArgs::skip).
#include "common.h"

namespace jl {
namespace {

template <typename C> struct cx { C re, im; };

template <typename C>
__device__ __forceinline__ void mac(cx<C>& acc, C ar, C ai, C br, C bi) {  // acc += a*b
  acc.re = fma(ar, br, acc.re);
  acc.re = fma(-ai, bi, acc.re);
  acc.im = fma(ar, bi, acc.im);
  acc.im = fma(ai, br, acc.im);
}
template <typename C>
__device__ __forceinline__ void mac_conj_a(cx<C>& acc, C ar, C ai, C br, C bi) {  // acc += conj(a)*b
  acc.re = fma(ar, br, acc.re);
  acc.re = fma(ai, bi, acc.re);
  acc.im = fma(ar, bi, acc.im);
  acc.im = fma(-ai, br, acc.im);
}

// Site vectors: the 4 complex components of one site are contiguous (32 B
// in FP32, 64 B in FP64) and move as 16-byte vector loads and stores.
template <typename S, typename C>
__device__ __forceinline__ void load_site(const cplx<S>* __restrict__ p, C re[4], C im[4]) {
  if constexpr (sizeof(S) == 4) {
    const float4* q = reinterpret_cast<const float4*>(p);
    const float4 u = q[0], v = q[1];
    re[0] = (C)u.x; im[0] = (C)u.y; re[1] = (C)u.z; im[1] = (C)u.w;
    re[2] = (C)v.x; im[2] = (C)v.y; re[3] = (C)v.z; im[3] = (C)v.w;
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const cplx<S> v = p[c];
      re[c] = (C)v.x;
      im[c] = (C)v.y;
    }
  }
}
template <typename S, typename C>
__device__ __forceinline__ void store_site(cplx<S>* __restrict__ p, const cx<C> v[4]) {
  if constexpr (sizeof(S) == 4) {
    float4* q = reinterpret_cast<float4*>(p);
    q[0] = make_float4((float)v[0].re, (float)v[0].im, (float)v[1].re, (float)v[1].im);
    q[1] = make_float4((float)v[2].re, (float)v[2].im, (float)v[3].re, (float)v[3].im);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      cplx<S> o;
      o.x = (S)v[c].re;
      o.y = (S)v[c].im;
      p[c] = o;
    }
  }
}

// The operand of an apply: a plain vector x, or (in the conjugate-gradient
// loop) the new search direction p = r + beta p_old, formed on the fly from
// r and the previous direction so that the direction update needs no pass of
// its own.  Every element of p is formed by the same expression (an explicit
// fma) wherever it is used, so the copy of p that the kernel stores for the
// other CG kernels is bit-identical to the operand it applied A to.
template <typename S>
__device__ __forceinline__ S cg_dir(S r, S p, double beta) {
  return (S)fma(beta, (double)p, (double)r);
}
template <typename S, bool DIR> struct Operand;
template <typename S> struct Operand<S, false> {
  const cplx<S>* __restrict__ x;
  template <typename C>
  __device__ __forceinline__ void site(int64_t off, C re[4], C im[4]) const {
    load_site<S, C>(x + off, re, im);
  }
  __device__ __forceinline__ cplx<S> elem(int64_t off) const { return x[off]; }
};
template <typename S> struct Operand<S, true> {
  const cplx<S>* __restrict__ r;
  const cplx<S>* __restrict__ p;
  double beta;
  template <typename C>
  __device__ __forceinline__ void site(int64_t off, C re[4], C im[4]) const {
    S rr[4], ri[4], pr[4], pi[4];
    load_site<S, S>(r + off, rr, ri);
    load_site<S, S>(p + off, pr, pi);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      re[k] = (C)cg_dir<S>(rr[k], pr[k], beta);
      im[k] = (C)cg_dir<S>(ri[k], pi[k], beta);
    }
  }
  __device__ __forceinline__ cplx<S> elem(int64_t off) const {
    const cplx<S> a = r[off], b = p[off];
    cplx<S> o;
    o.x = cg_dir<S>(a.x, b.x, beta);
    o.y = cg_dir<S>(a.y, b.y, beta);
    return o;
  }
};

// The two hops of direction mu at a site, from the link entries lk already
// loaded and the neighbour's halves (ar, ai), (br, bi), for kernels that take
// operands from LDS (the same arithmetic as stencil_site's hops, which keep
// theirs inline: the helpers cost the FP64 search-direction apply 20
// registers and a wavefront per SIMD).  Forward (lk =
// U_mu(s), neighbour s + mu): U a, conj(U) b, B b, conj(B) a.  Backward (lk =
// U_mu(s - mu), neighbour s - mu = sl): U^H a, U^T b, B^T b, B^H a.  Without
// BSITE, B holds the 4 direction matrices B_mu (16 entries each), read at
// wavefront-uniform addresses (scalar loads); with BSITE it has the layout of U
// and the entries of site sl are used; Bm = B + 16 mu.
template <typename S, typename C, bool BSITE>
__device__ __forceinline__ void hop_fwd(const StencilArgs<S>& a, const cplx<S>* Bm, int64_t sl, int mu,
                                        const cplx<S> lk[16], C sc, const C ar[4], const C ai[4],
                                        const C br[4], const C bi[4], cx<C> top[4], cx<C> bot[4]) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    cx<C> t = {0, 0}, q = {0, 0}, tb = {0, 0}, qb = {0, 0};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const cplx<S> u = lk[4 * r + c];
      const cplx<S> w = BSITE ? a.B[link_index(sl, mu, 4 * r + c)] : Bm[4 * r + c];
      const C ur = (C)u.x, ui = (C)u.y, wr = (C)w.x, wi = (C)w.y;
      mac(t, ur, ui, ar[c], ai[c]);          // U a_f
      mac_conj_a(q, ur, ui, br[c], bi[c]);   // conj(U) b_f
      mac(tb, wr, wi, br[c], bi[c]);         // B b_f
      mac_conj_a(qb, wr, wi, ar[c], ai[c]);  // conj(B) a_f
    }
    top[r].re += sc * tb.re - t.re; top[r].im += sc * tb.im - t.im;
    bot[r].re -= q.re + sc * qb.re; bot[r].im -= q.im + sc * qb.im;
  }
}
template <typename S, typename C, bool BSITE>
__device__ __forceinline__ void hop_bwd(const StencilArgs<S>& a, const cplx<S>* Bm, int64_t sl, int mu,
                                        const cplx<S> lk[16], C sc, const C ar[4], const C ai[4],
                                        const C br[4], const C bi[4], cx<C> top[4], cx<C> bot[4]) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    cx<C> t = {0, 0}, q = {0, 0}, tb = {0, 0}, qb = {0, 0};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const cplx<S> u = lk[4 * c + r];
      const cplx<S> w = BSITE ? a.B[link_index(sl, mu, 4 * c + r)] : Bm[4 * c + r];
      const C ur = (C)u.x, ui = (C)u.y, wr = (C)w.x, wi = (C)w.y;
      mac_conj_a(t, ur, ui, ar[c], ai[c]);   // U^H a_b
      mac(q, ur, ui, br[c], bi[c]);          // U^T b_b
      mac(tb, wr, wi, br[c], bi[c]);         // B^T b_b
      mac_conj_a(qb, wr, wi, ar[c], ai[c]);  // B^H a_b
    }
    top[r].re -= t.re + sc * tb.re; top[r].im -= t.im + sc * tb.im;
    bot[r].re += sc * qb.re - q.re; bot[r].im += sc * qb.im - q.im;
  }
}

// Computes (A v)(s) for one site: top[4], bot[4] in compute type C.  Links are
// tiled: entry e (row-major index in the 4x4 link) of U_mu(s) is
// U[link_index(s, mu, e)], so the 64 lanes of a wavefront read 512
// contiguous bytes (FP32) per entry and the 64 entries of a tile sit in one
// 32 KB block (measured at 32^4: 209 -> 183 us per apply against the layout
// with each entry's sites spread over the whole lattice).  Without
// BSITE, B holds the 4 direction matrices B_mu (16 entries each), read at
// wavefront-uniform addresses (scalar loads); with BSITE it has the layout of
// U.  One direction and one hop are live at a time.  Directions MU0 .. MU1-1;
// with MU0 > 0 the caller has set (top, bot) and does the other directions.
template <typename S, typename C, bool BSITE, typename X, int MU0 = 0, int MU1 = 4>
__device__ __forceinline__ void stencil_site(const StencilArgs<S>& a, const X& xo, int64_t h,
                                             int64_t s, cx<C> top[4], cx<C> bot[4]) {
  // site coordinates in 32 bits (the lattice has fewer than 2^31 sites)
  const unsigned Ls[4] = {(unsigned)a.L[0], (unsigned)a.L[1], (unsigned)a.L[2], (unsigned)a.L[3]};
  const unsigned st[4] = {Ls[1] * Ls[2] * Ls[3], Ls[2] * Ls[3], Ls[3], 1u};
  unsigned x[4];
  {
    unsigned r = (unsigned)s;
    x[0] = r / st[0]; r -= x[0] * st[0];
    x[1] = r / st[1]; r -= x[1] * st[1];
    x[2] = r / st[2]; r -= x[2] * st[2];
    x[3] = r;
  }
  const C dg = (C)a.diag;
  const C sc = (C)a.scale;
  if (MU0 == 0) {
    C ar[4], ai[4], br[4], bi[4];
    xo.template site<C>(s * 4, ar, ai);
    xo.template site<C>(h + s * 4, br, bi);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      top[r].re = dg * ar[r]; top[r].im = dg * ai[r];
      bot[r].re = dg * br[r]; bot[r].im = dg * bi[r];
    }
  }
  const int64_t V = a.V;
#pragma unroll 1
  for (int mu = MU0; mu < MU1; ++mu) {
    const int64_t sf = (x[mu] == Ls[mu] - 1) ? s - (int64_t)((Ls[mu] - 1) * st[mu]) : s + st[mu];
    const int64_t sb = (x[mu] == 0) ? s + (int64_t)((Ls[mu] - 1) * st[mu]) : s - st[mu];
    const cplx<S>* Bm = a.B + mu * 16;   // site-independent B
    // ---- forward hop: U(x) a(x+mu), conj(U(x)) b(x+mu), B(x) b(x+mu), conj(B(x)) a(x+mu)
    // Each hop issues all of its loads before any product (the scheduling
    // barrier keeps the compiler from waiting for each link entry in turn).
    {
      C ar[4], ai[4], br[4], bi[4];
      cplx<S> lk[16];
      xo.template site<C>(sf * 4, ar, ai);
      xo.template site<C>(h + sf * 4, br, bi);
#pragma unroll
      for (int e = 0; e < 16; ++e) lk[e] = a.U[link_index(s, mu, e)];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        cx<C> t = {0, 0}, q = {0, 0}, tb = {0, 0}, qb = {0, 0};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const cplx<S> u = lk[4 * r + c];
          const cplx<S> w = BSITE ? a.B[link_index(s, mu, 4 * r + c)] : Bm[4 * r + c];
          const C ur = (C)u.x, ui = (C)u.y, wr = (C)w.x, wi = (C)w.y;
          mac(t, ur, ui, ar[c], ai[c]);          // U a_f
          mac_conj_a(q, ur, ui, br[c], bi[c]);   // conj(U) b_f
          mac(tb, wr, wi, br[c], bi[c]);         // B b_f
          mac_conj_a(qb, wr, wi, ar[c], ai[c]);  // conj(B) a_f
        }
        top[r].re += sc * tb.re - t.re; top[r].im += sc * tb.im - t.im;
        bot[r].re -= q.re + sc * qb.re; bot[r].im -= q.im + sc * qb.im;
      }
    }
    // ---- backward hop: U(x-mu)^H a, U(x-mu)^T b, B(x-mu)^T b, B(x-mu)^H a at x-mu
    {
      C ar[4], ai[4], br[4], bi[4];
      cplx<S> lk[16];
      xo.template site<C>(sb * 4, ar, ai);
      xo.template site<C>(h + sb * 4, br, bi);
#pragma unroll
      for (int e = 0; e < 16; ++e) lk[e] = a.U[link_index(sb, mu, e)];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        cx<C> t = {0, 0}, q = {0, 0}, tb = {0, 0}, qb = {0, 0};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const cplx<S> u = lk[4 * c + r];
          const cplx<S> w = BSITE ? a.B[link_index(sb, mu, 4 * c + r)] : Bm[4 * c + r];
          const C ur = (C)u.x, ui = (C)u.y, wr = (C)w.x, wi = (C)w.y;
          mac_conj_a(t, ur, ui, ar[c], ai[c]);   // U^H a_b
          mac(q, ur, ui, br[c], bi[c]);          // U^T b_b
          mac(tb, wr, wi, br[c], bi[c]);         // B^T b_b
          mac_conj_a(qb, wr, wi, ar[c], ai[c]);  // B^H a_b
        }
        top[r].re -= t.re + sc * tb.re; top[r].im -= t.im + sc * tb.im;
        bot[r].re += sc * qb.re - q.re; bot[r].im += sc * qb.im - q.im;
      }
    }
  }
}

constexpr int kStencilThreads = 256;

// Site block of this workgroup.  Workgroups are dealt to the eight XCDs in
// turn (workgroup b runs on XCD b mod 8).  When every x0-plane is a whole
// number of 8 blocks, workgroup b takes the block that gives each XCD one
// eighth of every plane, planes in increasing order: the operand one plane
// back or ahead, and the link of the backward hop in x0, were then read a
// short while before by the same XCD and come from its L2 (measured at 32^4:
// 1.25 -> 1.05 GB fetched per FP32 apply, 183 -> 175 us).  Otherwise the
// identity.
__device__ __forceinline__ int64_t stencil_site_block(const int32_t L[4]) {
  const int64_t P = (int64_t)L[1] * L[2] * L[3];
  if (P % (8 * kStencilThreads) != 0) return blockIdx.x;
  const int64_t bx = P / (8 * kStencilThreads), b = blockIdx.x, k = b >> 3;
  return (k / bx) * (8 * bx) + (b & 7) * bx + k % bx;
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh);

// y = A x per site; with apart != nullptr (single column) the block also
// writes its FP64 partial of x^H y (the alpha_j of Alg. 2) to apart[2*blk].
// With DIR (single column, CG) the operand is p = r + beta p_old with
// p_old = x, and p is stored to pnew as well.
template <typename S, bool BSITE, bool DIR>
__global__ __launch_bounds__(kStencilThreads) void k_stencil_apply(StencilArgs<S> a,
                                                                   const cplx<S>* __restrict__ x,
                                                                   cplx<S>* __restrict__ y,
                                                                   int64_t ld,
                                                                   double* __restrict__ apart,
                                                                   const cplx<S>* __restrict__ dr,
                                                                   const double* __restrict__ dbeta,
                                                                   cplx<S>* __restrict__ pnew) {
  if (a.skip && *a.skip != 0.0) return;   // uniform over the grid
  __shared__ double sh[kStencilThreads / 64];
  const int64_t s = stencil_site_block(a.L) * kStencilThreads + threadIdx.x;
  const int64_t h = a.V * 4;
  Operand<S, DIR> xo;
  if constexpr (DIR) xo = Operand<S, true>{dr, x, *dbeta};
  else xo = Operand<S, false>{x + (int64_t)blockIdx.y * ld};
  cplx<S>* yc = y + (int64_t)blockIdx.y * ld;
  double are = 0.0, aim = 0.0;
  if (s < a.V) {
    cx<S> top[4], bot[4];
    stencil_site<S, S, BSITE>(a, xo, h, s, top, bot);
    store_site<S, S>(yc + s * 4, top);
    store_site<S, S>(yc + h + s * 4, bot);
    if (apart || DIR) {   // the site's own operand components again (cache hit)
      S a0r[4], a0i[4], b0r[4], b0i[4];
      xo.template site<S>(s * 4, a0r, a0i);
      xo.template site<S>(h + s * 4, b0r, b0i);
      if constexpr (DIR) {
        cx<S> pt[4], pb[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          pt[r] = cx<S>{a0r[r], a0i[r]};
          pb[r] = cx<S>{b0r[r], b0i[r]};
        }
        store_site<S, S>(pnew + s * 4, pt);
        store_site<S, S>(pnew + h + s * 4, pb);
      }
      if (apart) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          are += (double)a0r[r] * top[r].re + (double)a0i[r] * top[r].im +
                 (double)b0r[r] * bot[r].re + (double)b0i[r] * bot[r].im;
          aim += (double)a0r[r] * top[r].im - (double)a0i[r] * top[r].re +
                 (double)b0r[r] * bot[r].im - (double)b0i[r] * bot[r].re;
        }
      }
    }
  }
  if (apart) {   // uniform over the grid
    are = block_sum<kStencilThreads>(are, sh);
    aim = block_sum<kStencilThreads>(aim, sh);
    if (threadIdx.x == 0) {
      apart[2 * blockIdx.x] = are;
      apart[2 * blockIdx.x + 1] = aim;
    }
  }
}

// Plane-pair bricks for the FP32 apply: a workgroup takes kBrickS in-plane
// sites of two consecutive x0-planes, and workgroup b takes the brick that
// gives XCD b mod 8 one eighth of every plane pair, pairs in increasing order.
// Each thread stages its site's operand, and in the first plane its x0 link,
// in LDS, so the x0 hops between the two planes of the brick take both from
// LDS instead of fetching them again; in directions 2 and 3 the neighbours
// inside the brick take their operand from LDS too (links from memory).
// Measured at 32^4: 168 -> 155 us in the solve for the x0 sharing (in a
// standalone harness 0.94 against 1.05 GB fetched; four planes per brick
// saved no more), 153.7 -> 151.0 us for the in-plane operands.
constexpr int kBrickZ = 2, kBrickS = kStencilThreads / kBrickZ;

template <typename S, bool DIR>
__global__ __launch_bounds__(kStencilThreads) void k_stencil_brick(StencilArgs<S> a,
                                                                   const cplx<S>* __restrict__ x,
                                                                   cplx<S>* __restrict__ y,
                                                                   int64_t ld,
                                                                   double* __restrict__ apart,
                                                                   const cplx<S>* __restrict__ dr,
                                                                   const double* __restrict__ dbeta,
                                                                   cplx<S>* __restrict__ pnew) {
  if (a.skip && *a.skip != 0.0) return;   // uniform over the grid
  __shared__ double sh[kStencilThreads / 64];
  // the 4 + 4 operand components of each thread's site, component-major so
  // that consecutive threads touch consecutive words
  __shared__ cplx<S> xs[8][kStencilThreads];
  __shared__ cplx<S> us[16][kBrickS];          // U_0 of the first plane's sites
  const int64_t P = (int64_t)a.L[1] * a.L[2] * a.L[3];
  const int64_t bx = P / (8 * kBrickS), b = blockIdx.x, k = b >> 3;
  const int64_t g = k / bx, c = (b & 7) * bx + k % bx;   // plane pair, in-plane brick
  const int t = threadIdx.x, zl = t / kBrickS, tq = t % kBrickS;
  const int64_t q = c * kBrickS + tq;
  const unsigned L0 = (unsigned)a.L[0];
  const unsigned z = (unsigned)(g * kBrickZ + zl);
  const int64_t s = (int64_t)z * P + q;
  const int64_t h = a.V * 4;
  Operand<S, DIR> xo;
  if constexpr (DIR) xo = Operand<S, true>{dr, x, *dbeta};
  else xo = Operand<S, false>{x + (int64_t)blockIdx.y * ld};
  cplx<S>* yc = y + (int64_t)blockIdx.y * ld;
  const S dg = (S)a.diag, sc = (S)a.scale;
  cx<S> top[4], bot[4];
  {
    S ar[4], ai[4], br[4], bi[4];
    xo.template site<S>(s * 4, ar, ai);
    xo.template site<S>(h + s * 4, br, bi);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      xs[r][t].x = ar[r]; xs[r][t].y = ai[r];
      xs[4 + r][t].x = br[r]; xs[4 + r][t].y = bi[r];
      top[r].re = dg * ar[r]; top[r].im = dg * ai[r];
      bot[r].re = dg * br[r]; bot[r].im = dg * bi[r];
    }
  }
  cplx<S> lk[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) lk[e] = a.U[link_index(s, 0, e)];
  if (zl == 0) {
#pragma unroll
    for (int e = 0; e < 16; ++e) us[e][tq] = lk[e];
  }
  __syncthreads();
  auto from_lds = [&](int i, S ar[4], S ai[4], S br[4], S bi[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      ar[r] = xs[r][i].x; ai[r] = xs[r][i].y;
      br[r] = xs[4 + r][i].x; bi[r] = xs[4 + r][i].y;
    }
  };
  {   // x0 forward: the second plane's operand from LDS
    S ar[4], ai[4], br[4], bi[4];
    if (zl == 0) {
      from_lds(t + kBrickS, ar, ai, br, bi);
    } else {
      const int64_t sf = (int64_t)(z + 1 == L0 ? 0 : z + 1) * P + q;
      xo.template site<S>(sf * 4, ar, ai);
      xo.template site<S>(h + sf * 4, br, bi);
    }
    hop_fwd<S, S, false>(a, a.B, s, 0, lk, sc, ar, ai, br, bi, top, bot);
  }
  {   // x0 backward: the first plane's operand and link from LDS
    S ar[4], ai[4], br[4], bi[4];
    cplx<S> lb[16];
    if (zl == 1) {
      from_lds(t - kBrickS, ar, ai, br, bi);
#pragma unroll
      for (int e = 0; e < 16; ++e) lb[e] = us[e][tq];
    } else {
      const int64_t sb = (int64_t)(z == 0 ? L0 - 1 : z - 1) * P + q;
      xo.template site<S>(sb * 4, ar, ai);
      xo.template site<S>(h + sb * 4, br, bi);
#pragma unroll
      for (int e = 0; e < 16; ++e) lb[e] = a.U[link_index(sb, 0, e)];
    }
    __builtin_amdgcn_sched_barrier(0);
    hop_bwd<S, S, false>(a, a.B, s, 0, lb, sc, ar, ai, br, bi, top, bot);
  }
  stencil_site<S, S, false, Operand<S, DIR>, 1, 2>(a, xo, h, s, top, bot);
  // directions 2 and 3: neighbours inside the brick's in-plane sites take the
  // operand from LDS, the others (and every link) from memory
  {
    const unsigned L2 = (unsigned)a.L[2], L3 = (unsigned)a.L[3];
    const unsigned qi = (unsigned)q, x3 = qi % L3, x2 = (qi / L3) % L2;
    const int64_t zP = (int64_t)z * P, q0 = c * kBrickS;
#pragma unroll 1
    for (int mu = 2; mu < 4; ++mu) {
      const unsigned xm = mu == 2 ? x2 : x3, Lm = mu == 2 ? L2 : L3, sm = mu == 2 ? L3 : 1u;
      const int64_t qf = xm == Lm - 1 ? (int64_t)qi - (int64_t)(Lm - 1) * sm : (int64_t)qi + sm;
      const int64_t qb = xm == 0 ? (int64_t)qi + (int64_t)(Lm - 1) * sm : (int64_t)qi - sm;
      {
        S ar[4], ai[4], br[4], bi[4];
        cplx<S> lf[16];
        const int64_t i = qf - q0;
        if (i >= 0 && i < kBrickS) {
          from_lds(zl * kBrickS + (int)i, ar, ai, br, bi);
        } else {
          xo.template site<S>((zP + qf) * 4, ar, ai);
          xo.template site<S>(h + (zP + qf) * 4, br, bi);
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) lf[e] = a.U[link_index(s, mu, e)];
        __builtin_amdgcn_sched_barrier(0);
        hop_fwd<S, S, false>(a, a.B + mu * 16, s, mu, lf, sc, ar, ai, br, bi, top, bot);
      }
      {
        S ar[4], ai[4], br[4], bi[4];
        cplx<S> lb[16];
        const int64_t i = qb - q0;
        if (i >= 0 && i < kBrickS) {
          from_lds(zl * kBrickS + (int)i, ar, ai, br, bi);
        } else {
          xo.template site<S>((zP + qb) * 4, ar, ai);
          xo.template site<S>(h + (zP + qb) * 4, br, bi);
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) lb[e] = a.U[link_index(zP + qb, mu, e)];
        __builtin_amdgcn_sched_barrier(0);
        hop_bwd<S, S, false>(a, a.B + mu * 16, s, mu, lb, sc, ar, ai, br, bi, top, bot);
      }
    }
  }
  store_site<S, S>(yc + s * 4, top);
  store_site<S, S>(yc + h + s * 4, bot);
  double are = 0.0, aim = 0.0;
  if (apart || DIR) {   // the site's own operand components (LDS)
    S a0r[4], a0i[4], b0r[4], b0i[4];
    from_lds(t, a0r, a0i, b0r, b0i);
    if constexpr (DIR) {
      cx<S> pt[4], pb[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        pt[r] = cx<S>{a0r[r], a0i[r]};
        pb[r] = cx<S>{b0r[r], b0i[r]};
      }
      store_site<S, S>(pnew + s * 4, pt);
      store_site<S, S>(pnew + h + s * 4, pb);
    }
    if (apart) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        are += (double)a0r[r] * top[r].re + (double)a0i[r] * top[r].im +
               (double)b0r[r] * bot[r].re + (double)b0i[r] * bot[r].im;
        aim += (double)a0r[r] * top[r].im - (double)a0i[r] * top[r].re +
               (double)b0r[r] * bot[r].im - (double)b0i[r] * bot[r].re;
      }
    }
  }
  if (apart) {   // uniform over the grid
    are = block_sum<kStencilThreads>(are, sh);
    aim = block_sum<kStencilThreads>(aim, sh);
    if (threadIdx.x == 0) {
      apart[2 * blockIdx.x] = are;
      apart[2 * blockIdx.x + 1] = aim;
    }
  }
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {   // result valid in thread 0
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

// True residuals ||A x_c - lam_c x_c||^2 of many columns x_c = X + cols[c]*ldx
// with the links read once per group of columns: sixteen threads per site, thread
// (mu, r) computes the hops in direction mu of row r of both halves of
// (A x_c)(s) and keeps the link entries it multiplies in registers for every
// column (row r of U_mu(s), column r of U_mu(s - mu)); the four directions of
// a row are summed across lanes.  The site-independent B sits in LDS (per-site
// B is read per use).  FP64 products and accumulation on the stored vectors.
// A block walks the columns of its group (cpb of them; gridDim.y groups) in
// chunks of kResidCols with the links in registers, so the links are read
// once per group: once in all when the site blocks alone fill the device.
// partial[blk * ncols + c] = the share of column c of site block blk
// (stencil_resid_blocks blocks).
constexpr int kResidSites = kStencilThreads / 16;   // sites per block
constexpr int kResidCols = 16;                       // columns per chunk

// Site t (0..15) of residual block blockIdx.x.  When every extent is a
// multiple of 8 and the 8^4 boxes of the lattice come in multiples of eight,
// each run of 2048 workgroups covers eight boxes, box j of the run on XCD j
// (workgroup b runs on XCD b mod 8), a box's 256 workgroups in x0-slowest
// order, each two x2 rows of eight x3 sites.  The workgroups an XCD holds at
// once then cover a compact piece of one box, and a site's neighbours are
// mostly sites that the XCD is applying the same column to at about the same
// time (its L2), where consecutive sites put the neighbours in x2, x1 and x0
// on other XCDs (measured at 32^4 with about 112 columns per launch: 20.4 ->
// 19.1 ms; the kernel is then bound less by HBM than by its FP64 products
// and the data each lane loads).  Otherwise consecutive sites.
__device__ __forceinline__ int64_t resid_site(const int32_t L[4], int t) {
  const int64_t b = blockIdx.x;
  const int n0 = L[0] / 8, n1 = L[1] / 8, n2 = L[2] / 8, n3 = L[3] / 8;
  const bool boxes = L[0] % 8 == 0 && L[1] % 8 == 0 && L[2] % 8 == 0 && L[3] % 8 == 0 &&
                     ((int64_t)n0 * n1 * n2 * n3) % 8 == 0;
  if (!boxes) return b * kResidSites + t;
  int64_t box = (b >> 11) * 8 + (b & 7);
  const int l = (int)((b >> 3) & 255);
  const int b3 = (int)(box % n3); box /= n3;
  const int b2 = (int)(box % n2); box /= n2;
  const int b1 = (int)(box % n1);
  const int b0 = (int)(box / n1);
  const int64_t x0 = b0 * 8 + (l >> 5), x1 = b1 * 8 + ((l >> 2) & 7);
  const int64_t x2 = b2 * 8 + 2 * (l & 3) + (t >> 3), x3 = b3 * 8 + (t & 7);
  return ((x0 * L[1] + x1) * L[2] + x2) * L[3] + x3;
}

template <typename S, bool BSITE>
__global__ __launch_bounds__(kStencilThreads) void k_stencil_resid(StencilArgs<S> a,
                                                                   const cplx<S>* __restrict__ X,
                                                                   int64_t ldx,
                                                                   const int* __restrict__ cols,
                                                                   const double* __restrict__ lam,
                                                                   int ncols, int cpb,
                                                                   double* __restrict__ partial) {
  __shared__ cplx<S> Bs[64];
  __shared__ double red[kStencilThreads / 64][kResidCols];   // per-wavefront column sums
  const int r = threadIdx.x & 3, mu = (threadIdx.x >> 2) & 3;
  const int64_t s_raw = resid_site(a.L, threadIdx.x >> 4);
  const bool ok = s_raw < a.V;
  const int64_t s = ok ? s_raw : a.V - 1;   // in-bounds loads; the contribution is dropped
  const int64_t V = a.V, h = V * 4;
  if (!BSITE && threadIdx.x < 64) Bs[threadIdx.x] = a.B[threadIdx.x];
  const unsigned Ls[4] = {(unsigned)a.L[0], (unsigned)a.L[1], (unsigned)a.L[2], (unsigned)a.L[3]};
  const unsigned st[4] = {Ls[1] * Ls[2] * Ls[3], Ls[2] * Ls[3], Ls[3], 1u};
  unsigned xm;   // coordinate of s in direction mu
  {
    unsigned t = (unsigned)s, xc[4];
    xc[0] = t / st[0]; t -= xc[0] * st[0];
    xc[1] = t / st[1]; t -= xc[1] * st[1];
    xc[2] = t / st[2]; t -= xc[2] * st[2];
    xc[3] = t;
    xm = xc[mu];
  }
  const unsigned Lm = Ls[mu], sm = st[mu];
  const int64_t sf = (xm == Lm - 1) ? s - (int64_t)((Lm - 1) * sm) : s + sm;
  const int64_t sb = (xm == 0) ? s + (int64_t)((Lm - 1) * sm) : s - sm;
  cplx<S> uf[4], ub[4];   // uf[c] = U_mu(s)[r][c], ub[c] = U_mu(s - mu)[c][r]
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    uf[c] = a.U[link_index(s, mu, 4 * r + c)];
    ub[c] = a.U[link_index(sb, mu, 4 * c + r)];
  }
  __syncthreads();   // Bs
  const cplx<S>* Bm = Bs + mu * 16;   // site-independent B
  const double dg = a.diag, sc = a.scale;
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int colA = (int)blockIdx.y * cpb, colB = min(ncols, colA + cpb);
  for (int col0 = colA; col0 < colB; col0 += kResidCols) {
    const int col1 = min(colB, col0 + kResidCols);
    for (int col = col0; col < col1; ++col) {
      const int cc = col - col0;
      const cplx<S>* x = X + (int64_t)cols[col] * ldx;
      double tr = 0.0, ti = 0.0, br = 0.0, bi = 0.0;   // row r, direction mu
      if (mu == 0) {   // (diag - l) x(s), once per row
        const double l = lam[col];
        const cplx<S> xa = x[s * 4 + r], xb = x[h + s * 4 + r];
        tr = (dg - l) * (double)xa.x; ti = (dg - l) * (double)xa.y;
        br = (dg - l) * (double)xb.x; bi = (dg - l) * (double)xb.y;
      }
      {   // forward: U(s) a(s+mu), conj(U(s)) b(s+mu), B b(s+mu), conj(B) a(s+mu)
        double ar[4], ai[4], vr[4], vi[4];
        load_site<S, double>(x + sf * 4, ar, ai);
        load_site<S, double>(x + h + sf * 4, vr, vi);
        cx<double> t = {0, 0}, q = {0, 0}, tb = {0, 0}, qb = {0, 0};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const cplx<S> wv = BSITE ? a.B[link_index(s, mu, 4 * r + c)] : Bm[4 * r + c];
          const double ur = uf[c].x, ui = uf[c].y, wr = wv.x, wi = wv.y;
          mac(t, ur, ui, ar[c], ai[c]);
          mac_conj_a(q, ur, ui, vr[c], vi[c]);
          mac(tb, wr, wi, vr[c], vi[c]);
          mac_conj_a(qb, wr, wi, ar[c], ai[c]);
        }
        tr += sc * tb.re - t.re; ti += sc * tb.im - t.im;
        br -= q.re + sc * qb.re; bi -= q.im + sc * qb.im;
      }
      {   // backward: U(s-mu)^H a, U(s-mu)^T b, B(s-mu)^T b, B(s-mu)^H a at s - mu
        double ar[4], ai[4], vr[4], vi[4];
        load_site<S, double>(x + sb * 4, ar, ai);
        load_site<S, double>(x + h + sb * 4, vr, vi);
        cx<double> t = {0, 0}, q = {0, 0}, tb = {0, 0}, qb = {0, 0};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const cplx<S> wv = BSITE ? a.B[link_index(sb, mu, 4 * c + r)] : Bm[4 * c + r];
          const double ur = ub[c].x, ui = ub[c].y, wr = wv.x, wi = wv.y;
          mac_conj_a(t, ur, ui, ar[c], ai[c]);
          mac(q, ur, ui, vr[c], vi[c]);
          mac(tb, wr, wi, vr[c], vi[c]);
          mac_conj_a(qb, wr, wi, ar[c], ai[c]);
        }
        tr -= t.re + sc * tb.re; ti -= t.im + sc * tb.im;
        br += sc * qb.re - q.re; bi += sc * qb.im - q.im;
      }
      // the four directions of row r: lanes that differ in bits 2 and 3
#pragma unroll
      for (int o = 4; o <= 8; o <<= 1) {
        tr += __shfl_xor(tr, o); ti += __shfl_xor(ti, o);
        br += __shfl_xor(br, o); bi += __shfl_xor(bi, o);
      }
      double acc = (ok && mu == 0) ? tr * tr + ti * ti + br * br + bi * bi : 0.0;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
      if (lane == 0) red[w][cc] = acc;   // only this wavefront writes red[w]: no barrier per column
    }
    __syncthreads();
    for (int i = threadIdx.x; col0 + i < col1; i += kStencilThreads) {
      double tot = 0.0;
#pragma unroll
      for (int k = 0; k < kStencilThreads / 64; ++k) tot += red[k][i];
      partial[(int64_t)blockIdx.x * ncols + col0 + i] = tot;
    }
    __syncthreads();   // red is rewritten by the next chunk
  }
}

// Links from the caller's [mu][V][16] (site-major) layout into the
// operator's tiled copy (link_index); the padding of the last tile is zero.
template <typename S>
__global__ void k_links_tiled(const cplx<S>* __restrict__ src, cplx<S>* __restrict__ dst, int64_t V) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // destination index
  if (i >= link_elems(V)) return;
  const int64_t s = (i / (64 * kLinkTile)) * kLinkTile + i % kLinkTile;
  const int me = (int)((i / kLinkTile) % 64);                          // me = mu * 16 + e
  cplx<S> v;
  v.x = v.y = (S)0;
  if (s < V) v = src[((int64_t)(me / 16) * V + s) * 16 + me % 16];
  dst[i] = v;
}

// ------------------------------------------------------------------ dense
constexpr int kDenseThreads = 256;   // k_dense_resid: one wavefront per row

template <typename S, typename C, typename X>
__device__ __forceinline__ void dense_row(const DenseArgs<S>& a, const X& xo, int64_t r, cx<C>& s1,
                                          cx<C>& s2) {
  const int lane = threadIdx.x % 64;
  const cplx<S>* r11 = a.A11 + r * a.ld;
  const cplx<S>* r12 = a.A12 + r * a.ld;
  cx<C> p = {0, 0}, q = {0, 0};
  for (int64_t c = lane; c < a.h; c += 64) {
    const cplx<S> m11 = r11[c], m12 = r12[c];
    const cplx<S> va = xo.elem(c), vb = xo.elem(a.h + c);
    // s1 += A11 a + A12 b
    mac(p, (C)m11.x, (C)m11.y, (C)va.x, (C)va.y);
    mac(p, (C)m12.x, (C)m12.y, (C)vb.x, (C)vb.y);
    // s2 += A11 conj(b) - A12 conj(a)
    mac(q, (C)m11.x, (C)m11.y, (C)vb.x, -(C)vb.y);
    mac(q, (C)m12.x, (C)m12.y, -(C)va.x, (C)va.y);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    p.re += __shfl_xor(p.re, o);
    p.im += __shfl_xor(p.im, o);
    q.re += __shfl_xor(q.re, o);
    q.im += __shfl_xor(q.im, o);
  }
  s1 = p;
  s2 = q;
}

// k_dense_apply: kDenseRows rows per block.  The block's threads stride over
// the columns together (every wavefront reads 512 contiguous bytes of each
// row per column step), so the operand is read once per kDenseRows rows, and
// each thread issues the loads of kDenseUnroll column steps before any
// product, which keeps enough bytes in flight to stream the matrix.
constexpr int kDenseRows = 4;
template <typename S> constexpr int dense_unroll() { return sizeof(S) == 4 ? 4 : 2; }

template <typename S, int U, bool CHECK, typename X>
__device__ __forceinline__ void dense_cols(const DenseArgs<S>& a, const X& xo,
                                           const cplx<S>* const r11[kDenseRows],
                                           const cplx<S>* const r12[kDenseRows], int64_t c0,
                                           cx<S> p[kDenseRows], cx<S> q[kDenseRows]) {
  cplx<S> va[U], vb[U], m11[U][kDenseRows], m12[U][kDenseRows];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t c = c0 + (int64_t)u * kDenseThreads;
    const bool ok = !CHECK || c < a.h;
    const int64_t cc = ok ? c : 0;   // a clamped, in-bounds load; its terms are zeroed
    va[u] = xo.elem(cc);
    vb[u] = xo.elem(a.h + cc);
    if (!ok) va[u].x = va[u].y = vb[u].x = vb[u].y = (S)0;
#pragma unroll
    for (int k = 0; k < kDenseRows; ++k) {
      m11[u][k] = r11[k][cc];
      m12[u][k] = r12[k][cc];
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
#pragma unroll
    for (int k = 0; k < kDenseRows; ++k) {
      // s1 += A11 a + A12 b;  s2 += A11 conj(b) - A12 conj(a)
      mac(p[k], m11[u][k].x, m11[u][k].y, va[u].x, va[u].y);
      mac(p[k], m12[u][k].x, m12[u][k].y, vb[u].x, vb[u].y);
      mac(q[k], m11[u][k].x, m11[u][k].y, vb[u].x, -vb[u].y);
      mac(q[k], m12[u][k].x, m12[u][k].y, -va[u].x, va[u].y);
    }
  }
}

// As k_stencil_apply: with DIR the operand is p = r + beta p_old (p_old = x)
// and p is stored to pnew.
template <typename S, bool DIR>
__global__ __launch_bounds__(kDenseThreads) void k_dense_apply(DenseArgs<S> a,
                                                               const cplx<S>* __restrict__ x,
                                                               cplx<S>* __restrict__ y, int64_t ld,
                                                               double* __restrict__ apart,
                                                               const cplx<S>* __restrict__ dr,
                                                               const double* __restrict__ dbeta,
                                                               cplx<S>* __restrict__ pnew) {
  if (a.skip && *a.skip != 0.0) return;   // uniform over the grid
  constexpr int U = dense_unroll<S>(), NW = kDenseThreads / 64, R = kDenseRows;
  __shared__ S red[NW][R][4];
  __shared__ double sh[NW];
  const int64_t r0 = (int64_t)blockIdx.x * R;
  Operand<S, DIR> xo;
  if constexpr (DIR) xo = Operand<S, true>{dr, x, *dbeta};
  else xo = Operand<S, false>{x + (int64_t)blockIdx.y * ld};
  cplx<S>* yc = y + (int64_t)blockIdx.y * ld;
  const cplx<S>* r11[R];
  const cplx<S>* r12[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {   // rows past the end repeat the last row; not stored
    const int64_t r = r0 + k < a.h ? r0 + k : a.h - 1;
    r11[k] = a.A11 + r * a.ld;
    r12[k] = a.A12 + r * a.ld;
  }
  cx<S> p[R], q[R];
#pragma unroll
  for (int k = 0; k < R; ++k) p[k] = q[k] = cx<S>{(S)0, (S)0};
  int64_t c0 = threadIdx.x;
  for (; c0 + (int64_t)(U - 1) * kDenseThreads < a.h; c0 += (int64_t)U * kDenseThreads)
    dense_cols<S, U, false>(a, xo, r11, r12, c0, p, q);
  if (c0 < a.h) dense_cols<S, U, true>(a, xo, r11, r12, c0, p, q);
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
#pragma unroll
  for (int k = 0; k < R; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      p[k].re += __shfl_xor(p[k].re, o);
      p[k].im += __shfl_xor(p[k].im, o);
      q[k].re += __shfl_xor(q[k].re, o);
      q[k].im += __shfl_xor(q[k].im, o);
    }
    if (lane == 0) {
      red[w][k][0] = p[k].re;
      red[w][k][1] = p[k].im;
      red[w][k][2] = q[k].re;
      red[w][k][3] = q[k].im;
    }
  }
  __syncthreads();
  double are = 0.0, aim = 0.0;
  const int k = threadIdx.x;
  if (k < R && r0 + k < a.h) {   // thread k stores row r0 + k
    S v[4] = {(S)0, (S)0, (S)0, (S)0};
#pragma unroll
    for (int ww = 0; ww < NW; ++ww)
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] += red[ww][k][e];
    const int64_t r = r0 + k;
    cplx<S> t, b;
    t.x = v[0]; t.y = v[1];
    b.x = v[2]; b.y = -v[3];   // u_bot = conj(s2)
    yc[r] = t;
    yc[a.h + r] = b;
    if (apart || DIR) {
      const cplx<S> xt = xo.elem(r), xb = xo.elem(a.h + r);
      if constexpr (DIR) {
        pnew[r] = xt;
        pnew[a.h + r] = xb;
      }
      are = (double)xt.x * t.x + (double)xt.y * t.y + (double)xb.x * b.x + (double)xb.y * b.y;
      aim = (double)xt.x * t.y - (double)xt.y * t.x + (double)xb.x * b.y - (double)xb.y * b.x;
    }
  }
  if (apart) {
    are = block_sum<kDenseThreads>(are, sh);
    aim = block_sum<kDenseThreads>(aim, sh);
    if (threadIdx.x == 0) {
      apart[2 * blockIdx.x] = are;
      apart[2 * blockIdx.x + 1] = aim;
    }
  }
}

template <typename S>
__global__ __launch_bounds__(kDenseThreads) void k_dense_resid(DenseArgs<S> a,
                                                               const cplx<S>* __restrict__ X,
                                                               int64_t ldx,
                                                               const int* __restrict__ cols,
                                                               const double* __restrict__ lam,
                                                               double* __restrict__ partial) {
  __shared__ double sh[kDenseThreads / 64];
  const int64_t r = (int64_t)blockIdx.x * (kDenseThreads / 64) + threadIdx.x / 64;
  const int c = blockIdx.y;
  double acc = 0.0;
  if (r < a.h) {
    const cplx<S>* xc = X + (int64_t)cols[c] * ldx;
    cx<double> s1, s2;
    dense_row<S, double>(a, Operand<S, false>{xc}, r, s1, s2);
    if (threadIdx.x % 64 == 0) {
      const double l = lam[c];
      const cplx<S> xt = xc[r], xb = xc[a.h + r];
      const double tr = s1.re - l * (double)xt.x, ti = s1.im - l * (double)xt.y;
      const double br = s2.re - l * (double)xb.x, bi = -s2.im - l * (double)xb.y;
      acc = tr * tr + ti * ti + br * br + bi * bi;
    }
  }
  // only lane 0 of each wave holds a value; block_sum adds zeros elsewhere
  const double tot = block_sum<kDenseThreads>(acc, sh);
  if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * gridDim.y + c] = tot;
}

}  // namespace

int stencil_resid_blocks(int64_t V) { return (int)((V + kResidSites - 1) / kResidSites); }
int stencil_apply_blocks(int64_t V) { return (int)((V + kStencilThreads - 1) / kStencilThreads); }
int dense_apply_blocks(int64_t h) { return (int)((h + kDenseRows - 1) / kDenseRows); }
int dense_resid_blocks(int64_t h) { return (int)((h + kDenseThreads / 64 - 1) / (kDenseThreads / 64)); }

template <typename S, bool DIR>
hipError_t stencil_apply_impl(const StencilArgs<S>& a, const cplx<S>* x, cplx<S>* y, int64_t ld,
                              int nrhs, double* apart, const cplx<S>* dr, const double* dbeta,
                              cplx<S>* pnew, hipStream_t st) {
  dim3 grid((unsigned)((a.V + kStencilThreads - 1) / kStencilThreads), (unsigned)nrhs);
  if constexpr (sizeof(S) == 4) {
    const int64_t P = (int64_t)a.L[1] * a.L[2] * a.L[3];
    if (!a.b_per_site && P % (8 * kBrickS) == 0 && a.L[0] % kBrickZ == 0) {
      // plane-pair bricks (the grid covers V / 256 of them, exactly)
      hipLaunchKernelGGL((k_stencil_brick<S, DIR>), grid, dim3(kStencilThreads), 0, st, a, x, y, ld,
                         apart, dr, dbeta, pnew);
      return hipGetLastError();
    }
  }
  if (a.b_per_site)
    hipLaunchKernelGGL((k_stencil_apply<S, true, DIR>), grid, dim3(kStencilThreads), 0, st, a, x, y,
                       ld, apart, dr, dbeta, pnew);
  else
    hipLaunchKernelGGL((k_stencil_apply<S, false, DIR>), grid, dim3(kStencilThreads), 0, st, a, x,
                       y, ld, apart, dr, dbeta, pnew);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_stencil_apply(const StencilArgs<S>& a, const cplx<S>* x, cplx<S>* y, int64_t ld,
                                int nrhs, double* apart, hipStream_t st) {
  if (apart && nrhs != 1) return hipErrorInvalidValue;
  return stencil_apply_impl<S, false>(a, x, y, ld, nrhs, apart, nullptr, nullptr, nullptr, st);
}

template <typename S>
hipError_t launch_stencil_apply_dir(const StencilArgs<S>& a, const cplx<S>* r, const cplx<S>* pold,
                                    const double* beta, cplx<S>* pnew, cplx<S>* y, double* apart,
                                    hipStream_t st) {
  return stencil_apply_impl<S, true>(a, pold, y, a.V * 8, 1, apart, r, beta, pnew, st);
}

template <typename S>
hipError_t launch_stencil_resid(const StencilArgs<S>& a, const cplx<S>* X, int64_t ldx,
                                const int* cols, const double* lam, int ncols, double* partial,
                                int* nblk, hipStream_t st) {
  const int nb = stencil_resid_blocks(a.V);
  *nblk = nb;
  if (ncols <= 0) return hipSuccess;
  // column groups only as far as the site blocks alone leave the device short
  // of about 2048 workgroups (the links are read once per group)
  const int chunks = (ncols + kResidCols - 1) / kResidCols;
  const int groups = std::max(1, std::min(chunks, (2048 + nb - 1) / nb));
  const int cpb = (chunks + groups - 1) / groups * kResidCols;
  const dim3 grid((unsigned)nb, (unsigned)((ncols + cpb - 1) / cpb));
  if (a.b_per_site)
    hipLaunchKernelGGL((k_stencil_resid<S, true>), grid, dim3(kStencilThreads), 0, st, a, X, ldx,
                       cols, lam, ncols, cpb, partial);
  else
    hipLaunchKernelGGL((k_stencil_resid<S, false>), grid, dim3(kStencilThreads), 0, st, a, X, ldx,
                       cols, lam, ncols, cpb, partial);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_links_tiled(const cplx<S>* src, cplx<S>* dst, int64_t V, hipStream_t st) {
  const int64_t total = link_elems(V);
  hipLaunchKernelGGL(k_links_tiled<S>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, src,
                     dst, V);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_dense_apply(const DenseArgs<S>& a, const cplx<S>* x, cplx<S>* y, int64_t ldv,
                              int nrhs, double* apart, hipStream_t st) {
  if (apart && nrhs != 1) return hipErrorInvalidValue;
  dim3 grid((unsigned)dense_apply_blocks(a.h), (unsigned)nrhs);
  hipLaunchKernelGGL((k_dense_apply<S, false>), grid, dim3(kDenseThreads), 0, st, a, x, y, ldv,
                     apart, nullptr, nullptr, nullptr);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_dense_apply_dir(const DenseArgs<S>& a, const cplx<S>* r, const cplx<S>* pold,
                                  const double* beta, cplx<S>* pnew, cplx<S>* y, double* apart,
                                  hipStream_t st) {
  dim3 grid((unsigned)dense_apply_blocks(a.h), 1u);
  hipLaunchKernelGGL((k_dense_apply<S, true>), grid, dim3(kDenseThreads), 0, st, a, pold, y,
                     2 * a.h, apart, r, beta, pnew);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_dense_resid(const DenseArgs<S>& a, const cplx<S>* X, int64_t ldx,
                              const int* cols, const double* lam, int ncols, double* partial,
                              int* nblk, hipStream_t st) {
  const int nb = dense_resid_blocks(a.h);
  *nblk = nb;
  hipLaunchKernelGGL(k_dense_resid<S>, dim3((unsigned)nb, (unsigned)ncols), dim3(kDenseThreads), 0,
                     st, a, X, ldx, cols, lam, partial);
  return hipGetLastError();
}

#define JL_INST(S)                                                                               \
  template hipError_t launch_stencil_apply<S>(const StencilArgs<S>&, const cplx<S>*, cplx<S>*,   \
                                              int64_t, int, double*, hipStream_t);               \
  template hipError_t launch_stencil_resid<S>(const StencilArgs<S>&, const cplx<S>*, int64_t,    \
                                              const int*, const double*, int, double*, int*,     \
                                              hipStream_t);                                      \
  template hipError_t launch_links_tiled<S>(const cplx<S>*, cplx<S>*, int64_t, hipStream_t);       \
  template hipError_t launch_dense_apply<S>(const DenseArgs<S>&, const cplx<S>*, cplx<S>*,       \
                                            int64_t, int, double*, hipStream_t);                 \
  template hipError_t launch_dense_resid<S>(const DenseArgs<S>&, const cplx<S>*, int64_t,        \
                                            const int*, const double*, int, double*, int*,       \
                                            hipStream_t);                                        \
  template hipError_t launch_stencil_apply_dir<S>(const StencilArgs<S>&, const cplx<S>*,         \
                                                  const cplx<S>*, const double*, cplx<S>*,       \
                                                  cplx<S>*, double*, hipStream_t);               \
  template hipError_t launch_dense_apply_dir<S>(const DenseArgs<S>&, const cplx<S>*,             \
                                                const cplx<S>*, const double*, cplx<S>*,         \
                                                cplx<S>*, double*, hipStream_t);
JL_INST(float)
JL_INST(double)
#undef JL_INST

}  // namespace jl
