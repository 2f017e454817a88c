// Thick-restart basis update V_k <- V_m Z[:, 0:k] (Alg. 1, V_m := V_m Z_m).
//
// Z is real, so the complex basis (interleaved, column-major, one vector per
// column) is a real (2n) x m column-major matrix and the update is a real
// GEMM C = A * B with M = 2n rows, K = m, N = k.  It is compute-bound at the
// stencil shapes, so it runs on the matrix cores: v_mfma_f64_16x16x4f64 for
// both bases (FP32 loads are converted to FP64, Z is FP64 and the result is
// rounded once to the storage type).  FP32 accumulation over K = m terms
// would leave a
// Ritz-vector error of about sqrt(m) u_32 that puts the true-residual floor
// above the mixed-precision tolerance.
//
// Block tile 128 x BN (BN = 128, 64 or 32), 4 wavefronts in 2 x 2, each
// 64 x BN/2 = 4 x BN/32 MFMA tiles (computed transposed so that stores run
// down the columns of C); K staged through LDS (as FP64) in steps of 8 with
// a register prefetch of the next step and two LDS buffers (one barrier per
// step).  Consecutive tiles of one row panel are placed on the same XCD so
// the A panel is shared through that XCD's L2.  A launch covers its N
// columns with 128-wide tiles and finishes the remainder with a 64-wide
// and a 32-wide tile, so at most 31 columns of MFMA work are padding
// (measured at M = 2^24, K = 500, FP32 A: 58.8 TFLOP/s at N = 256; N = 300
// in 128-wide tiles alone, 46.4 TFLOP/s).
#include "common.h"

#include <algorithm>
#include <type_traits>

namespace jl {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename S> struct Mfma;
template <> struct Mfma<double> {
  using acc_t = f64x4;
  static constexpr int BK = 8;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

constexpr int BM = 128, PAD = 16, LDT = BM + PAD;
constexpr int kThreads = 256;

// S: storage type of A and C; T: MFMA (accumulation) type, also the type of B.
template <typename S, typename T, int BN>
__global__ __launch_bounds__(kThreads, 2) void k_gemm_nn(const S* __restrict__ A, int64_t lda,
                                                      const T* __restrict__ B, int64_t ldb,
                                                      S* __restrict__ C, int64_t ldc, int64_t M,
                                                      int N, int K, int64_t tiles_m, int tiles_n,
                                                      const int* __restrict__ cmap) {
  using MF = Mfma<T>;
  constexpr int BK = MF::BK;
  constexpr int WN = BN / 2;                            // columns per wavefront
  constexpr int NJ = WN / 16;                           // MFMA tiles per wavefront row
  constexpr int AV = 16 / sizeof(S);                    // elements per 16-byte load
  constexpr int A_PER_T = BM * BK / kThreads;           // A elements per thread per step
  constexpr int B_PER_T = BN * BK / kThreads;
  static_assert(A_PER_T % AV == 0, "A loader");
  __shared__ T As[2][BK][LDT];
  __shared__ T Bs[2][BK][LDT];

  // XCD-aware tile order: hardware places block b on XCD b % 8; make the
  // tiles of one row panel consecutive on one XCD.
  const int64_t nblk = (int64_t)gridDim.x;
  const int64_t b = blockIdx.x;
  const int64_t per_xcd = nblk / 8;
  const int64_t logical = (b % 8) * per_xcd + b / 8;
  if (logical >= tiles_m * tiles_n) return;
  const int64_t tm = logical / tiles_n;
  const int tn = (int)(logical % tiles_n);
  const int64_t m0 = tm * BM;
  const int n0 = tn * BN;

  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int wm = wave / 2, wn = wave % 2;

  // A tile loader: thread -> (k, row chunk of A_PER_T contiguous rows)
  constexpr int A_TPK = BM / A_PER_T;                   // threads per k
  const int a_k = tid / A_TPK;
  const int a_r = (tid % A_TPK) * A_PER_T;
  // B tile loader: thread -> (col, k chunk of B_PER_T)
  constexpr int B_TPC = BK / B_PER_T;                   // threads per column
  const int b_c = tid / B_TPC;
  const int b_k = (tid % B_TPC) * B_PER_T;

  // Raw loads; the out-of-range values are zeroed when the registers are
  // stored to LDS, after the products, so nothing waits for the loads before
  // then.  Every load is unconditional, at an index clamped into the matrix:
  // a load under a condition is a branch the compiler closes by waiting for
  // it, which would serialise the prefetch of the next K step instead of
  // overlapping it with the products.  M is a multiple of AV (checked at
  // launch), so an A vector is wholly in range or not.
  S ra[A_PER_T];
  T rb[B_PER_T];
  bool a_in[A_PER_T / AV], b_in[B_PER_T];
  auto load = [&](int k0) {
    const int k = k0 + a_k;
    const int kc = k < K ? k : K - 1;
#pragma unroll
    for (int v = 0; v < A_PER_T; v += AV) {
      const int64_t row = m0 + a_r + v;
      a_in[v / AV] = k < K && row < M;
      const S* p = A + (int64_t)kc * lda + (row < M ? row : M - AV);
      if constexpr (AV == 4) {
        const float4 t = *reinterpret_cast<const float4*>(p);
        ra[v] = t.x; ra[v + 1] = t.y; ra[v + 2] = t.z; ra[v + 3] = t.w;
      } else {
        const double2 t = *reinterpret_cast<const double2*>(p);
        ra[v] = t.x; ra[v + 1] = t.y;
      }
    }
    const int col = n0 + b_c;
    const int colc = col < N ? col : N - 1;
#pragma unroll
    for (int e = 0; e < B_PER_T; ++e) {
      const int kk = k0 + b_k + e;
      b_in[e] = col < N && kk < K;
      rb[e] = B[(int64_t)colc * ldb + (kk < K ? kk : K - 1)];
    }
  };
  // B takes a 0/1 factor rather than a select, which the compiler would turn
  // back into a branch (the column test is uniform across the wavefront); the
  // clamped values are finite, so the product is 0.
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < A_PER_T; ++e) As[buf][a_k][a_r + e] = a_in[e / AV] ? (T)ra[e] : (T)0;
#pragma unroll
    for (int e = 0; e < B_PER_T; ++e) Bs[buf][b_k + e][b_c] = rb[e] * (b_in[e] ? (T)1 : (T)0);
  };

  typename MF::acc_t acc[4][NJ];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = typename MF::acc_t{0, 0, 0, 0};

  const int nk = (K + BK - 1) / BK;
  load(0);
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    store(buf);
    __syncthreads();
    load((kt + 1) * BK);   // past the last step the values are zeros and unused
    // the prefetch is issued before the products (the scheduler would
    // otherwise sink it below them and wait for it at once)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kr = ks * 4 + lane / 16;
      T a[4], bb[NJ];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[buf][kr][wm * 64 + i * 16 + lane % 16];
#pragma unroll
      for (int j = 0; j < NJ; ++j) bb[j] = Bs[buf][kr][wn * WN + j * 16 + lane % 16];
      // the transposed tile product (B^T A^T): the MFMA output then runs
      // along the rows of C in consecutive lanes
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = MF::op(bb[j], a[i], acc[i][j]);
    }
  }

  // Output layout of v_mfma_f64_16x16x4f64: lane l holds column l % 16 of the
  // 16 x 16 tile, register r holds row 4*r + l/16.  The tile here is C^T, so
  // lane l holds row l % 16 of C and register r column 4*r + l/16: each store
  // writes 16 consecutive rows of 4 columns.
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = m0 + wm * 64 + i * 16 + lane % 16;
    if (row >= M) continue;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = n0 + wn * WN + j * 16 + 4 * r + lane / 16;
        if (col < N) C[(int64_t)(cmap ? cmap[col] : col) * ldc + row] = (S)acc[i][j][r];
      }
    }
  }
}

}  // namespace

template <typename S, typename T, int BN>
hipError_t launch_tiles(const S* A, int64_t lda, const T* B, int64_t ldb, S* C, int64_t ldc, int64_t M,
                        int N, int K, hipStream_t st, const int* cmap) {
  const int64_t tm = (M + BM - 1) / BM;
  const int tn = (N + BN - 1) / BN;
  int64_t nblk = tm * tn;
  nblk = (nblk + 7) / 8 * 8;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_gemm_nn<S, T, BN>), dim3((unsigned)nblk), dim3(kThreads), 0, st, A, lda, B, ldb,
                     C, ldc, M, N, K, tm, tn, cmap);
  return hipGetLastError();
}

template <typename S, typename T>
hipError_t launch_gemm_nn(const S* A, int64_t lda, const T* B, int64_t ldb, S* C, int64_t ldc,
                          int64_t M, int N, int K, hipStream_t st, const int* cmap) {
  if (M <= 0 || N <= 0) return hipSuccess;
  // 16-byte vector loads/stores of A and C columns need 4-element (FP32) or
  // 2-element (FP64) alignment of every column start.
  const int AV = 16 / (int)sizeof(S);
  if ((lda % AV) || (ldc % AV) || (M % AV) || K <= 0 || ((uintptr_t)A % 16) || ((uintptr_t)C % 16))
    return hipErrorInvalidValue;
  // columns [c0, c0 + w) of the product: B and the output columns move with c0
  auto part = [&](auto tile, int c0, int w) -> hipError_t {
    constexpr int TB = decltype(tile)::value;
    return launch_tiles<S, T, TB>(A, lda, B + (int64_t)c0 * ldb, ldb, cmap ? C : C + (int64_t)c0 * ldc,
                                  ldc, M, w, K, st, cmap ? cmap + c0 : nullptr);
  };
  hipError_t e = hipSuccess;
  int full = N / 128 * 128;
  if (N - full > 96) full = N;   // the last 128-wide tile then pads fewer than 32 columns
  if (full > 0) e = part(std::integral_constant<int, 128>{}, 0, full);
  int c0 = full;
  if (e == hipSuccess && N - c0 > 32) {
    e = part(std::integral_constant<int, 64>{}, c0, std::min(64, N - c0));
    c0 += 64;
  }
  if (e == hipSuccess && N - c0 > 0) e = part(std::integral_constant<int, 32>{}, c0, N - c0);
  return e;
}

template hipError_t launch_gemm_nn<float, double>(const float*, int64_t, const double*, int64_t,
                                                  float*, int64_t, int64_t, int, int, hipStream_t,
                                                  const int*);
template hipError_t launch_gemm_nn<double, double>(const double*, int64_t, const double*, int64_t,
                                                   double*, int64_t, int64_t, int, int,
                                                   hipStream_t, const int*);

}  // namespace jl
