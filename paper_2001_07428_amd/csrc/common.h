// Internal declarations shared by the HIP kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace jl {

// Interleaved complex of storage type S.
template <typename S> struct cplx_t;
template <> struct cplx_t<float> { using type = float2; };
template <> struct cplx_t<double> { using type = double2; };
template <typename S> using cplx = typename cplx_t<S>::type;

// 16-byte vector of storage type S (two FP32 complex or one FP64 complex).
template <typename S> struct vec16_t;
template <> struct vec16_t<float> { using type = float4; };
template <> struct vec16_t<double> { using type = double2; };

constexpr int kWave = 64;

// ---------------------------------------------------------------- launchers
// Every launcher enqueues on `st` and returns the launch error (if any).

// Stencil operator data.  U: links in tiles of 64 sites, entry e of U_mu(s)
// at U[link_index(s, mu, e)] (the 64 sites of a tile fastest, then the entry
// mu * 16 + e, then the tile); B: the 4 direction matrices [mu][16], or with
// b_per_site the layout of U.
constexpr int kLinkTile = 64;
__host__ __device__ inline int64_t link_index(int64_t s, int mu, int e) {   // s >= 0
  const uint64_t u = (uint64_t)s;
  return (int64_t)((((u >> 6) * 64 + (uint64_t)(mu * 16 + e)) << 6) | (u & 63));
}
static_assert(kLinkTile == 64, "link_index assumes tiles of 64 sites");
// Elements of the tiled link copy for V sites (the last tile padded).
__host__ __device__ inline int64_t link_elems(int64_t V) { return (V + kLinkTile - 1) / kLinkTile * kLinkTile * 64; }
template <typename S> struct StencilArgs {
  const cplx<S>* U;
  const cplx<S>* B;
  int32_t L[4];
  int64_t V;
  int b_per_site;
  double diag;
  double scale;
  // When non-null, the apply kernels return at once while *skip != 0 (a
  // device flag: the conjugate-gradient loop sets it on convergence, so
  // launches queued past that point do no work).  Null for plain applies.
  const double* skip;
};

// y = A x for nrhs columns (ld = n), compute type = S.  With apart !=
// nullptr (nrhs == 1) each block also writes the FP64 partial sum of x^H y
// to apart[2*blk], apart[2*blk+1] (stencil_apply_blocks blocks).
template <typename S>
hipError_t launch_stencil_apply(const StencilArgs<S>& a, const cplx<S>* x, cplx<S>* y, int64_t ld,
                                int nrhs, double* apart, hipStream_t st);
int stencil_apply_blocks(int64_t V);
// One CG direction step fused into the apply (single column): the operand is
// p = r + beta p_old (beta = *beta on the device), y = A p, p is stored to
// pnew, and apart receives the partials of p^H y as above.
template <typename S>
hipError_t launch_stencil_apply_dir(const StencilArgs<S>& a, const cplx<S>* r, const cplx<S>* pold,
                                    const double* beta, cplx<S>* pnew, cplx<S>* y, double* apart,
                                    hipStream_t st);
// Per-block partial sums of ||A x_c - lam_c x_c||^2 (FP64 compute) for ncols
// columns x_c = X + cols[c]*ldx (cols, lam on the device); partial layout
// [blk][c]; *nblk = blocks per column.
// dst[link_index(s, mu, e)] = src[(mu * V + s) * 16 + e] for 4 directions
// (dst holds link_elems(V) elements; the padding is zeroed).
template <typename S>
hipError_t launch_links_tiled(const cplx<S>* src, cplx<S>* dst, int64_t V, hipStream_t st);

template <typename S>
hipError_t launch_stencil_resid(const StencilArgs<S>& a, const cplx<S>* X, int64_t ldx,
                                const int* cols, const double* lam, int ncols, double* partial,
                                int* nblk, hipStream_t st);
int stencil_resid_blocks(int64_t V);

// Dense operator: A11, A12 row-major h x h with row stride ld.
template <typename S> struct DenseArgs {
  const cplx<S>* A11;
  const cplx<S>* A12;
  int64_t h;
  int64_t ld;
  const double* skip;   // as StencilArgs::skip
};
template <typename S>
hipError_t launch_dense_apply(const DenseArgs<S>& a, const cplx<S>* x, cplx<S>* y, int64_t ldv,
                              int nrhs, double* apart, hipStream_t st);
int dense_apply_blocks(int64_t h);
template <typename S>   // as launch_stencil_apply_dir
hipError_t launch_dense_apply_dir(const DenseArgs<S>& a, const cplx<S>* r, const cplx<S>* pold,
                                  const double* beta, cplx<S>* pnew, cplx<S>* y, double* apart,
                                  hipStream_t st);
template <typename S>
hipError_t launch_dense_resid(const DenseArgs<S>& a, const cplx<S>* X, int64_t ldx,
                              const int* cols, const double* lam, int ncols, double* partial,
                              int* nblk, hipStream_t st);
int dense_resid_blocks(int64_t h);

// Case B operator (A = D D^H, twisted Eguchi-Kawai Wilson-Dirac, Sec. 4.2)
// in the canonical layout [psi_0; psi_2 | psi_1; psi_3] of su(N)
// coefficients.  All matrices Np x Np row-major (Np = N rounded up to 64),
// zero outside N x N.
template <typename S> struct ZJob {   // C = op(A) op(B); op 0 = as is, 1 = conjugate transpose
  const cplx<S>* A;
  const cplx<S>* B;
  cplx<S>* C;
  int opA, opB;
};
template <typename S> struct TekArgs {
  int N, Np;
  int64_t na;                 // N^2 - 1 coefficients per spin
  double kappa;
  cplx<S>* X;                 // [4][Np][Np] spin matrices (scratch)
  cplx<S>* H;                 // [16][Np][Np] half-spinors h (mu*4 + q; q < 2 for U h U^H)
  cplx<S>* FB;                // [16][Np][Np] U h U^H and U^H h U, same order
  double* zd;                 // [4][N] complex diagonal scratch (FP64)
  const double* proj;         // spin projection tables: B [2][4][2][4], A [2][4][4][2] complex
  const ZJob<S>* jobs1;       // 16 first products: U h, U^H h
  const ZJob<S>* jobs2;       // 16 second products: (U h) U^H, (U^H h) U
  const double* skip;         // as StencilArgs::skip
};
template <typename S> struct TekSrc {   // operand x, or p = r + beta x stored to pnew
  const cplx<S>* x;
  const cplx<S>* r;
  const double* beta;
  cplx<S>* pnew;
};
int tek_apply_blocks(int N);   // partial-sum blocks of one apply (apart / residual)
template <typename S>
hipError_t launch_tek_apply(const TekArgs<S>& a, const cplx<S>* x, cplx<S>* y, double* apart,
                            hipStream_t st);
template <typename S>   // as launch_stencil_apply_dir
hipError_t launch_tek_apply_dir(const TekArgs<S>& a, const cplx<S>* r, const cplx<S>* pold,
                                const double* beta, cplx<S>* pnew, cplx<S>* y, double* apart,
                                hipStream_t st);
// As launch_stencil_resid, with the column indices on the host (hcols).
template <typename S>
hipError_t launch_tek_resid(const TekArgs<S>& a, const cplx<S>* X, int64_t ldx, const int* hcols,
                            const double* lam, int ncols, double* partial, int* nblk,
                            hipStream_t st);

// ------------------------------------------------------- reorthogonalisation
// Basis V: ncol columns of length n = 2h, column stride ldv.
// dots: partial[blk][dots_stride(ncol)] = per block (Re, Im of v_i^H u, Re,
// Im of w_i^H u) for each column, then ||u||^2, then (with the local step,
// else zero) ||u - t v_jl||^2 before the beta term and the rounding.
__host__ __device__ constexpr int dots_stride(int ncol) { return 4 * ncol + 2; }
int reorth_dots_blocks(int64_t h, int es);   // partial rows written by dots; es: bytes per complex
// partial entries written by update (es: bytes per complex; jsym as for
// launch_reorth_update, whose long FP32 vectors take other blocks without it)
int reorth_update_blocks(int64_t h, int es, bool jsym = true);
constexpr int kReorthMaxCols = 2048;   // largest basis dots supports
// With tloc != nullptr the kernel first applies the local three-term step
// u <- u - t v_jl - beta v_{jl-1} (t = tloc[0] + i tloc[1] on the device,
// beta = 0 skips the second term), rounds u once to S, stores it, and then
// takes the inner products of the new u.
// groups > 1 splits the columns over gridDim.y (reorth_dots_groups); with
// tloc the locally updated u then goes to uout, which must not be u.  With
// beta2 (device) the second term uses beta = sqrt(*beta2) instead of `beta`.
template <typename S>
hipError_t launch_reorth_dots(const cplx<S>* V, int64_t ldv, int ncol, cplx<S>* u, int64_t h,
                              double* partial, int nblk, hipStream_t st,
                              const double* tloc = nullptr, double beta = 0.0, int jl = 0,
                              cplx<S>* uout = nullptr, int groups = 1,
                              const double* beta2 = nullptr);
int reorth_dots_groups(int64_t h, int es);
// update: u -= V c_v + W c_w (W = J V^*), coef = [4*ncol] FP64 (Re cv, Im cv,
// Re cw, Im cw per column); partial[blk] = ||u_new||^2 per block.
// jsym = false leaves out the W projection (standard Gram-Schmidt against V).
// The result goes to u, computed from uin (default u).  groups > 1 splits
// the columns (reorth_update_groups) and needs d: groups x n complex scratch.
// With fin the kernel also sums the block norms into *fin, using the counter
// *cnt (zero before the first launch, left zero; launches sharing it must not
// overlap).
template <typename S>
hipError_t launch_reorth_update(const cplx<S>* V, int64_t ldv, int ncol, cplx<S>* u, int64_t h,
                                const double* coef, double* partial, int nblk, hipStream_t st,
                                bool jsym = true, const cplx<S>* uin = nullptr, int groups = 1,
                                cplx<S>* d = nullptr, double* fin = nullptr,
                                unsigned* cnt = nullptr);
int reorth_update_groups(int64_t h, int es);
// out[c] = sum_b partial[b * stride + c] for c < ncols (deterministic order).
hipError_t launch_reduce_cols(const double* partial, int nblk, int stride, int ncols, double* out,
                              hipStream_t st);
// The same sum for many columns (the reorthogonalisation's dots_stride(ncol)
// inner products and norms), spread over reduce_wide_tiles(ncols) x reduce_wide_slices(nblk)
// workgroups.  scr: reduce_wide_scratch_doubles(nblk, ncols) doubles; cnt:
// reduce_wide_tiles(ncols) counters, zero before the first launch and left
// zero by every launch (launches that share them must not overlap).
// last_out (optional) also receives out[ncols - 2], out[ncols - 1].
int reduce_wide_slices(int nblk);
int reduce_wide_tiles(int ncols);
size_t reduce_wide_scratch_doubles(int nblk, int ncols);
hipError_t launch_reduce_wide(const double* partial, int nblk, int stride, int ncols, double* out,
                              double* scr, unsigned* cnt, hipStream_t st,
                              double* last_out = nullptr);
// u *= scale (n complex).
template <typename S>
hipError_t launch_scale(cplx<S>* u, int64_t n, double scale, hipStream_t st);
// u *= 1 / sqrt(*nrm2), nrm2 read on the device (n complex).
template <typename S>
hipError_t launch_scale_dev(cplx<S>* u, int64_t n, const double* nrm2, hipStream_t st);
// p[0 .. n) = 0 by a kernel (no memset node when the caller captures a graph).
hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t st);
// fill with a constant real value (n complex).
template <typename S>
hipError_t launch_fill(cplx<S>* u, int64_t n, double value, hipStream_t st);
// Y = J X^* for k columns.
template <typename S>
hipError_t launch_pair(const cplx<S>* X, int64_t ldx, cplx<S>* Y, int64_t ldy, int64_t h, int k,
                       hipStream_t st);
// Y[:, pairs[2 i]] = X[:, pairs[2 i + 1]] for i < npairs (pairs on the device).
template <typename S>
hipError_t launch_copy_pairs(const cplx<S>* X, int64_t ldx, cplx<S>* Y, int64_t ldy, int64_t n,
                             const int* pairs, int npairs, hipStream_t st);
// copy k columns of length n between column-major blocks.
template <typename S>
hipError_t launch_copy_cols(const cplx<S>* X, int64_t ldx, cplx<S>* Y, int64_t ldy, int64_t n,
                            int k, hipStream_t st);

// ------------------------------------------------- conjugate gradients (invert)
// Device scalars of one CG solve (doubles at cs[slot]).
enum CgSlot {
  CG_RR = 0, CG_ALPHA, CG_BETA, CG_THR, CG_DONE, CG_ITERS, CG_MAXIT, CG_BB, CG_CNT, CG_NSLOTS
};
// CG_DONE: 0 running, 1 stopped (converged or maxit), 2 p^H A p <= 0.
// CG_CNT: the fused step's finished-block counter (an unsigned in the slot).
int cg_blocks(int64_t n);   // partial sums written by the CG vector kernels
// x = 0, r = b, p = 0, beta = 0 (so the first fused apply forms p = b);
// starts the solve of A x = b (stop at ||r|| <= tol ||b||).
template <typename S>
hipError_t launch_cg_init(const cplx<S>* b, cplx<S>* x, cplx<S>* r, cplx<S>* p, int64_t n,
                          double* part, double* cs, double tol, int maxit, hipStream_t st);
// The rest of one iteration after q = A p (apart: the apply's napply
// partials of p^H q): alpha, x and r, beta and the stop test, in one launch.
// The next direction p = r + beta p is formed by the next apply.
template <typename S>
hipError_t launch_cg_step(cplx<S>* x, cplx<S>* r, cplx<S>* p, const cplx<S>* q, int64_t n,
                          const double* apart, int napply, double* part, double* cs,
                          hipStream_t st);
// u = x and the partials of v^H u (2 per block, cg_blocks(n) blocks).
template <typename S>
hipError_t launch_cg_finish(const cplx<S>* x, cplx<S>* u, const cplx<S>* v, int64_t n,
                            double* part, hipStream_t st);
// Partials of x^H x (cg_blocks(n) blocks).
template <typename S>
hipError_t launch_norm2(const cplx<S>* x, int64_t n, double* part, hipStream_t st);

// ------------------------------------------------------------ restart GEMM
// C (M x N, ldc) = A (M x K, lda) * B (K x N, ldb), real, column-major; A
// and C of storage type S, B and the MFMA accumulation of type T
// (instantiated: <float,double>, <double,double>).  With cmap (device, N
// ints) column c of the product is stored to column cmap[c] of C.
// Narrowest column tile of the GEMM: a launch pads its N columns to a
// multiple of kGemmTileN at most.
constexpr int kGemmTileN = 32;
template <typename S, typename T>
hipError_t launch_gemm_nn(const S* A, int64_t lda, const T* B, int64_t ldb, S* C, int64_t ldc,
                          int64_t M, int N, int K, hipStream_t st, const int* cmap = nullptr);

// ------------------------------------------------------- Ritz eigenproblem
// Symmetric eigen-decomposition of an m x m FP64 matrix by parallel cyclic
// Jacobi (one launch per round).  mp = m rounded up to even.
struct EigWork {
  double* A[2];   // (mp x mp) ping-pong; eigenvalues end on the diagonal
  double* Z;      // (mp x mp) eigenvectors (columns), updated in place
  double* off;    // [1] off-diagonal sum of squares
};
size_t eig_work_doubles(int m);
int eig_small_max();   // largest mp handled by launch_eig_small
// A[0] = T (m x m col-major, ldt) padded; Z = I.
hipError_t launch_eig_init(const double* T, int ldt, int m, EigWork w, hipStream_t st);
// Round r of a sweep: reads A[cur], writes A[1-cur], updates Z.
hipError_t launch_eig_round(int m, EigWork w, int cur, int r, hipStream_t st);
// off[0] = sum of squares of the off-diagonal entries of A[cur].
hipError_t launch_eig_offnorm(int m, EigWork w, int cur, hipStream_t st);
// Small problems: all sweeps in one workgroup; lam[m], Z (m x m, ldz).
hipError_t launch_eig_small(const double* T, int ldt, int m, double* lam, double* Z, int ldz,
                            int max_sweeps, hipStream_t st);
// Divide and conquer for the restart structure of T_m (m <= dc_max_m()):
// hs / ds hold theta[k], s[k], alpha[m - k], beta[m - k - 1] on the host /
// device (for k > 0 alpha[0] = t_kk and beta[0] = t_{k+1,k}; for k = 0 the
// whole tridiagonal).  *lam (m, unsorted) and *Z (m x m, ld *ldz) point into
// `work` (dc_work_doubles(m) doubles).
int dc_max_m();
size_t dc_work_doubles(int m);
hipError_t ritz_dc(int m, int k, const double* hs, const double* ds, double* work, const double** lam,
                   const double** Z, int* ldz, hipStream_t st);
// Sort: perm[r] = index of the r-th desired Ritz value (ascending unless
// descending), with lam_i = lam[i * lstride]; then lam_s[r], Zs[:, r] (FP64,
// m rows), Zc[:, r] (storage type, r < kcols), zlast[r] = Zs[m-1, r].
template <typename S>
hipError_t launch_ritz_sort(int m, const double* lam, int64_t lstride, const double* Z, int ldz,
                            int descending, int kcols, int* perm, double* lam_s, double* Zs, S* Zc,
                            double* zlast, hipStream_t st);

// ------------------------------------------------------------ batched solve
struct BatchProblem {
  int64_t h;          // half dimension (n = 2h)
  const void* A11;    // h x h row-major, row stride ld
  const void* A12;
  int64_t ld;
  void* X;            // n x nev output, column stride ldx
  int64_t ldx;
};
struct BatchParams {
  int nev, m, mwin, which, max_cycles, max_passes, min_passes, tol_relative;
  int lds_mat;        // LDS bytes per workgroup for a resident [A11 A12] (0: none)
  double tol;
};
// per-problem counters of the batched solve: cycles, n_mv, gs_passes, icnv,
// n_resid, then the device wall-clock ticks (constant rate) its workgroup spent
// in each phase (kBatchPhases of them)
constexpr int kBatchPhases = 5;   // apply, Gram-Schmidt, Rayleigh-Ritz, restart V Z, residuals
constexpr int kBatchStats = 5 + kBatchPhases;
struct BatchOut {
  double* evals;      // [count][nev]
  double* res;        // [count][nev]
  int* status;        // [count]
  int* stats;         // [count][kBatchStats]: cycles, n_mv, gs_passes, icnv, n_resid, phase ticks
};
size_t batched_lds_bytes(int64_t hmax, int m, int es);   // without the resident-matrix budget
size_t batched_slot_bytes(int64_t hmax, int m, int es);
hipError_t launch_batched_init(int* queue, hipStream_t st);
// One persistent launch of `blocks` workgroups of `threads` (128/256/512)
// threads; each pops ids (in the given order) from *queue and solves them.
// rpw (1, 2) rows per wavefront and unr (4, 8) column steps in flight in the
// operator apply; P.lds_mat bytes of LDS per workgroup hold the matrix of a
// problem that fits.
template <typename S>
hipError_t launch_batched(const BatchProblem* probs, const int* order, int count,
                          const BatchParams& P, int* queue, char* slots, size_t slot_bytes,
                          int64_t hmax, const BatchOut& out, int threads, int rpw, int unr,
                          int blocks, hipStream_t st);

}  // namespace jl
