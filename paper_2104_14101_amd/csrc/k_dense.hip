// Dense kernels of the factorisation (Sec. 4.1) and of the Gaussian sketch, on the matrix
// cores of gfx950:
//   * gemm_kernel: C = alpha op(A) op(B) + beta C, FP64 (v_mfma_f64_16x16x4f64) or FP32
//     (v_mfma_f32_16x16x4f32), tiles up to 128 x 128, optional split-K over XCD-local row
//     ranges and a lower-triangle-only output; the products of the factorisation recursion and
//     of the Gaussian sketch;
//   * the Gram of the sketch, G = (SA)^T SA + nu^2 Lambda (m >= d), as split-K partials over
//     lower-triangle tiles reduced in a fixed order, with an optional BF16 form (FP32
//     accumulation, v_mfma_f32_32x32x16_bf16), and W = SA Lambda^-1 (SA)^T + nu^2 I (m < d);
//   * the Cholesky factor L of G and its inverse X = L^-1, by recursion on 2 x 2 block
//     partitions down to 128 x 128 nodes (one workgroup: two 64 x 64 leaves and three 64-wide
//     FP64 MFMA products in LDS); in a leaf one wavefront factorises column by column (lane =
//     row, next pivot updated ahead) while a second one inverts 8 rows behind it;
//   * the Gaussian sketch S A = G A / sqrt(m), its N(0, 1) entries generated in slabs from a
//     counter-based generator (Philox-4x64-10, Box-Muller), each exactly once per sketch.
#include "common.h"
#include "kernels.h"

namespace aes {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));

constexpr int BT = 64;   // output tile edge
constexpr int BKT = 16;  // K-step

// MFMA inner product over one K-step held in LDS (k-major tiles As[k][i], Bs[k][j]).
// Wave w owns the 32 x 32 quadrant (w >> 1, w & 1) as 2 x 2 blocks of 16 x 16.
__device__ __forceinline__ void mfma_ktile(const double (*As)[BT + 1], const double (*Bs)[BT + 1], int lane, int wm,
                                           int wn, d4 (&acc)[2][2]) {
#pragma unroll
  for (int kk = 0; kk < BKT / 4; ++kk) {
    const int kl = kk * 4 + (lane >> 4);
    double a[2], b[2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) a[bi] = As[kl][wm * 32 + bi * 16 + (lane & 15)];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) b[bj] = Bs[kl][wn * 32 + bj * 16 + (lane & 15)];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
  }
}

// Output element of lane `lane`, register r of block (bi, bj) for v_mfma_f64_16x16x4f64:
// row (lane/16) + 4*r, column lane%16 (measured on gfx950 against the oracle).
template <typename Store>
__device__ __forceinline__ void store_tile(const d4 (&acc)[2][2], int lane, int wm, int wn, int64_t m0, int64_t n0,
                                           Store st) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = m0 + wm * 32 + bi * 16 + (lane >> 4) + 4 * r;
        const int64_t j = n0 + wn * 32 + bj * 16 + (lane & 15);
        st(i, j, acc[bi][bj][r]);
      }
}

// MFMA 16 x 16 x 4 step for the element type, and the row held by register r of lane l in
// the 16 x 16 output block (measured on gfx950 against the oracle for both types).
template <typename T>
struct Mfma16;
template <>
struct Mfma16<double> {
  typedef d4 acc_t;
  __device__ __forceinline__ static acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma16<float> {
  typedef f4 acc_t;
  __device__ __forceinline__ static acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Tiled GEMM, 256 threads = 2 x 2 waves, wave tile (BM/2) x (BN/2) of 16 x 16 MFMA blocks.
// The next K-step is prefetched into registers while the current one is multiplied from LDS
// (double-buffered LDS, one barrier per K-step).
// MAP 0: grid (N tiles, M tiles, batch).  MAP 1 (split-K Gram, M == N, BM == BN): grid
// (splits, lower-triangle tiles); split z covers rows [z ksplit, min(K, (z+1) ksplit)) and the
// split index varies fastest, so that with a multiple of 8 splits each XCD (workgroups are
// dealt to the 8 XCDs round-robin) works on its own rows and shares them through its L2.
template <typename T, bool TA, bool TB, int BM, int BN, int BK, int MAP = 0>
__global__ __launch_bounds__(256) void gemm_kernel(int64_t M, int64_t N, int64_t K, double alpha,
                                                   const T* __restrict__ A, int64_t lda, int64_t sA,
                                                   const T* __restrict__ B, int64_t ldb, int64_t sB, double beta,
                                                   T* C, int64_t ldc, int64_t sC, int tri, int vec, int64_t ksplit,
                                                   int atri) {
  typedef Mfma16<T> MF;
  typedef typename MF::acc_t acc_t;
  // Each thread moves VW consecutive elements (16 bytes) along the contiguous direction of the
  // operand: rows of A^T / B (TA / !TB) or the K direction (!TA / TB).
  constexpr int VW = 16 / sizeof(T);
  constexpr int LA = BM * BK / 256, LB = BK * BN / 256;
  constexpr int LAV = LA / VW, LBV = LB / VW;
  static_assert(LAV * VW == LA && LBV * VW == LB, "tile too small for 16-byte loads");
  typedef T VT __attribute__((ext_vector_type(VW)));
  constexpr int WI = BM / 32, WJ = BN / 32;  // 16 x 16 blocks per wave
  int64_t bz, m0, n0;
  if (MAP == 0) {
    bz = blockIdx.z;
    m0 = (int64_t)blockIdx.y * BM;
    n0 = (int64_t)blockIdx.x * BN;
  } else {
    static_assert(MAP == 0 || BM == BN, "square tiles");
    bz = blockIdx.x;
    const int64_t t = blockIdx.y;
    int64_t ti = (int64_t)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while (ti * (ti + 1) / 2 > t) --ti;
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    m0 = ti * BM;
    n0 = (t - ti * (ti + 1) / 2) * BN;
    K = K - bz * ksplit;
    K = K < 0 ? 0 : (K > ksplit ? ksplit : K);
  }
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  if (tri && n0 > m0 + BM - 1) return;
  // atri (MAP 0, split-K with batch z covering global k = z ksplit + local k): A lower (1) or
  // upper (2) triangular, so only local k in [kbeg, kend) can meet nonzeros of the row tile
  int64_t kbeg = 0;
  if (MAP == 0 && atri == 1) {
    const int64_t e = m0 + BM - bz * ksplit;
    K = e < K ? (e < 0 ? 0 : e) : K;
  } else if (MAP == 0 && atri == 2) {
    const int64_t b0 = m0 - bz * ksplit;
    kbeg = b0 > 0 ? (b0 / BK) * BK : 0;
    if (kbeg > K) kbeg = K;
  }
  // interior tile with 16-byte aligned rows (vec: alignment checked by the host) and whole K-steps
  const bool interior = vec && m0 + BM <= M && n0 + BN <= N && K > kbeg && (K - kbeg) % BK == 0;
  __shared__ T As[2][BK][BM + 1], Bs[2][BK][BN + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wm = w >> 1, wn = w & 1;
  acc_t acc[WI][WJ];
#pragma unroll
  for (int bi = 0; bi < WI; ++bi)
#pragma unroll
    for (int bj = 0; bj < WJ; ++bj) acc[bi][bj] = acc_t{0, 0, 0, 0};
  T ra[LA], rb[LB];
  // (k, i) of element e of vector q of the A tile, (k, j) of the B tile
  auto a_at = [&](int q, int e, int& k, int& i) {
    const int idx = tid + q * 256;
    if (TA) { k = idx / (BM / VW); i = (idx % (BM / VW)) * VW + e; }
    else { k = (idx % (BK / VW)) * VW + e; i = idx / (BK / VW); }
  };
  auto b_at = [&](int q, int e, int& k, int& j) {
    const int idx = tid + q * 256;
    if (TB) { k = (idx % (BK / VW)) * VW + e; j = idx / (BK / VW); }
    else { k = idx / (BN / VW); j = (idx % (BN / VW)) * VW + e; }
  };
  auto load = [&](int64_t k0) {
    if (interior) {
#pragma unroll
      for (int q = 0; q < LAV; ++q) {
        int k, i;
        a_at(q, 0, k, i);
        const VT v = *reinterpret_cast<const VT*>(TA ? A + (k0 + k) * lda + m0 + i : A + (m0 + i) * lda + k0 + k);
#pragma unroll
        for (int e = 0; e < VW; ++e) ra[q * VW + e] = v[e];
      }
#pragma unroll
      for (int q = 0; q < LBV; ++q) {
        int k, j;
        b_at(q, 0, k, j);
        const VT v = *reinterpret_cast<const VT*>(TB ? B + (n0 + j) * ldb + k0 + k : B + (k0 + k) * ldb + n0 + j);
#pragma unroll
        for (int e = 0; e < VW; ++e) rb[q * VW + e] = v[e];
      }
    } else {
#pragma unroll
      for (int q = 0; q < LAV; ++q)
#pragma unroll
        for (int e = 0; e < VW; ++e) {
          int k, i;
          a_at(q, e, k, i);
          const int64_t gi = m0 + i, gk = k0 + k;
          ra[q * VW + e] = (gi < M && gk < K) ? (TA ? A[gk * lda + gi] : A[gi * lda + gk]) : T(0);
        }
#pragma unroll
      for (int q = 0; q < LBV; ++q)
#pragma unroll
        for (int e = 0; e < VW; ++e) {
          int k, j;
          b_at(q, e, k, j);
          const int64_t gj = n0 + j, gk = k0 + k;
          rb[q * VW + e] = (gj < N && gk < K) ? (TB ? B[gj * ldb + gk] : B[gk * ldb + gj]) : T(0);
        }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < LAV; ++q)
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        int k, i;
        a_at(q, e, k, i);
        As[buf][k][i] = ra[q * VW + e];
      }
#pragma unroll
    for (int q = 0; q < LBV; ++q)
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        int k, j;
        b_at(q, e, k, j);
        Bs[buf][k][j] = rb[q * VW + e];
      }
  };
  load(kbeg);
  store(0);
  __syncthreads();
  int cur = 0;
  for (int64_t k0 = kbeg; k0 < K; k0 += BK) {
    const bool more = k0 + BK < K;
    if (more) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kl = kk * 4 + (lane >> 4);
      T a[WI], b[WJ];
#pragma unroll
      for (int bi = 0; bi < WI; ++bi) a[bi] = As[cur][kl][wm * (BM / 2) + bi * 16 + (lane & 15)];
#pragma unroll
      for (int bj = 0; bj < WJ; ++bj) b[bj] = Bs[cur][kl][wn * (BN / 2) + bj * 16 + (lane & 15)];
#pragma unroll
      for (int bi = 0; bi < WI; ++bi)
#pragma unroll
        for (int bj = 0; bj < WJ; ++bj) acc[bi][bj] = MF::step(a[bi], b[bj], acc[bi][bj]);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
#pragma unroll
  for (int bi = 0; bi < WI; ++bi)
#pragma unroll
    for (int bj = 0; bj < WJ; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = m0 + wm * (BM / 2) + bi * 16 + MF::row(lane, r);
        const int64_t j = n0 + wn * (BN / 2) + bj * 16 + (lane & 15);
        if (i < M && j < N && (!tri || i >= j)) {
          double out = alpha * (double)acc[bi][bj][r];
          if (beta != 0.0) out += beta * (double)C[i * ldc + j];
          C[i * ldc + j] = (T)out;
        }
      }
}

template <typename T, bool TA, bool TB>
static void gemm_dispatch(int64_t M, int64_t N, int64_t K, double alpha, const T* A, int64_t lda, int64_t sA,
                          const T* B, int64_t ldb, int64_t sB, double beta, T* C, int64_t ldc, int64_t sC, int batch,
                          int tri, hipStream_t s, int atri, int64_t kofs) {
  const int64_t tiles128 = ceil_div(M, 128) * ceil_div(N, 128) * batch;
  // 16-byte vector loads need 16-byte aligned operand rows and whole K-steps (32 elements
  // covers every configuration's K-step)
  constexpr int VW = 16 / sizeof(T);
  const int vec = ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0) && lda % VW == 0 && ldb % VW == 0 &&
                  sA % VW == 0 && sB % VW == 0;
  if (N <= 32 && M >= 128) {
    // skinny products (multi-RHS matvecs, preconditioner applications): 128 x 32 tiles
    constexpr int BKS = sizeof(T) == 8 ? 16 : 32;
    dim3 grid(1u, (unsigned)ceil_div(M, 128), (unsigned)batch);
    hipLaunchKernelGGL((gemm_kernel<T, TA, TB, 128, 32, BKS>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, B,
                       ldb, sB, beta, C, ldc, sC, tri, vec, kofs, atri);
  } else if (M >= 128 && N >= 128 && tiles128 >= 128) {
    dim3 grid((unsigned)ceil_div(N, 128), (unsigned)ceil_div(M, 128), (unsigned)batch);
    hipLaunchKernelGGL((gemm_kernel<T, TA, TB, 128, 128, 16>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, B,
                       ldb, sB, beta, C, ldc, sC, tri, vec, kofs, atri);
  } else if (ceil_div(M, 64) * ceil_div(N, 64) * batch >= 512) {
    dim3 grid((unsigned)ceil_div(N, 64), (unsigned)ceil_div(M, 64), (unsigned)batch);
    hipLaunchKernelGGL((gemm_kernel<T, TA, TB, 64, 64, 32>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, B,
                       ldb, sB, beta, C, ldc, sC, tri, vec, kofs, atri);
  } else {
    // small products (the lower levels of the recursive factorisation): 32 x 32 tiles spread
    // the work over four times as many CUs
    dim3 grid((unsigned)ceil_div(N, 32), (unsigned)ceil_div(M, 32), (unsigned)batch);
    hipLaunchKernelGGL((gemm_kernel<T, TA, TB, 32, 32, 32>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, B,
                       ldb, sB, beta, C, ldc, sC, tri, vec, kofs, atri);
  }
  AES_LAUNCH_CHECK();
}

template <typename T>
static void gemm_any(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const T* A, int64_t lda,
                     int64_t sA, const T* B, int64_t ldb, int64_t sB, double beta, T* C, int64_t ldc, int64_t sC,
                     int batch, int tri, hipStream_t s, int atri, int64_t kofs) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (!ta && !tb)
    gemm_dispatch<T, false, false>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, tri, s, atri, kofs);
  else if (!ta && tb)
    gemm_dispatch<T, false, true>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, tri, s, atri, kofs);
  else if (ta && !tb)
    gemm_dispatch<T, true, false>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, tri, s, atri, kofs);
  else
    gemm_dispatch<T, true, true>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, tri, s, atri, kofs);
}

void gemm_f64(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
              int64_t sA, const double* B, int64_t ldb, int64_t sB, double beta, double* C, int64_t ldc, int64_t sC,
              int batch, int tri, hipStream_t s, int atri, int64_t kofs) {
  gemm_any<double>(ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, tri, s, atri, kofs);
}

void gemm_f32(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const float* A, int64_t lda,
              int64_t sA, const float* B, int64_t ldb, int64_t sB, double beta, float* C, int64_t ldc, int64_t sC,
              int batch, int tri, hipStream_t s) {
  gemm_any<float>(ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, tri, s, 0, 0);
}

// ---------------------------------------------------------------------------------------
// Gram of the sketch.
// ---------------------------------------------------------------------------------------
int gram_splits(int num_cu, int64_t m, int64_t d, bool fp64) {
  if (!fp64 || d >= 128) {
    // XCD-aware split-K over 128 x 128 tiles (gemm_kernel MAP 1 and the BF16 Gram): a multiple
    // of 8 splits, as few as keep the rounds of resident workgroups per XCD (two per CU) within
    // 5% of the best
    const int64_t nt = ceil_div(d, 128);
    const int64_t tiles = nt * (nt + 1) / 2;
    const int64_t slots = std::max<int64_t>(1, 2 * (int64_t)num_cu / 8);
    const int64_t max_q = std::max<int64_t>(1, std::min<int64_t>(4, m / (8 * 256)));
    double best = 1e30;
    for (int64_t q = 1; q <= max_q; ++q) best = std::min(best, (double)ceil_div(tiles * q, slots) / q);
    for (int64_t q = 1; q <= max_q; ++q)
      if ((double)ceil_div(tiles * q, slots) / q <= 1.05 * best) return (int)(8 * q);
    return 8;
  }
  // FP64 Gram with d < 128 (64 x 64 tiles), two workgroups per CU
  const int64_t tiles = ceil_div(d, BT) * (ceil_div(d, BT) + 1) / 2;
  const int64_t slots = 2 * (int64_t)num_cu;
  const int64_t max_s = std::min<int64_t>(16, std::max<int64_t>(1, m / 256));
  double best = 1e30;
  for (int64_t sp = 1; sp <= max_s; ++sp) best = std::min(best, (double)ceil_div(tiles * sp, slots) / sp);
  for (int64_t sp = 1; sp <= max_s; ++sp)
    if ((double)ceil_div(tiles * sp, slots) / sp <= 1.05 * best) return (int)sp;
  return 1;
}

// G[i,j] (lower, padded to dp) = [wprev gprev[i,j] +] sum_s part[s][i][j] + nu2 lam_i [i == j];
// identity padding; upper = 0.  gkeep[i,j] (lower d x d) gets the value before the diagonal term
// (gkeep may be gprev: each element is read and written by one thread).
template <typename TP>
__global__ void gram_reduce_kernel(const TP* __restrict__ part, int splits, int64_t d, int64_t dp, double nu2,
                                   const double* __restrict__ lam, double* __restrict__ G, const double* gprev,
                                   double wprev, double* gkeep) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= dp * dp) return;
  const int64_t i = e / dp, j = e % dp;
  double v = 0.0;
  if (i < d && j < d && i >= j) {
    // eight partials in flight per thread; summed in split order
    int s = 0;
    for (; s + 8 <= splits; s += 8) {
      TP x[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) x[q] = part[(int64_t)(s + q) * dp * dp + i * dp + j];
#pragma unroll
      for (int q = 0; q < 8; ++q) v += (double)x[q];
    }
    for (; s < splits; ++s) v += (double)part[(int64_t)s * dp * dp + i * dp + j];
    if (gprev) v += wprev * gprev[e];
    if (gkeep) gkeep[e] = v;
    if (i == j) v += nu2 * (lam ? lam[i] : 1.0);
  } else if (i == j) {
    v = 1.0;
  }
  G[e] = v;
}

void gram_tn(int64_t m, int64_t d, const double* SA, int64_t ldsa, double nu2, const double* lam, double* part,
             int splits, double* G, int64_t dp, hipStream_t s, const double* gprev, double wprev, double* gkeep) {
  // split z: rows [z rows, min(m, (z+1) rows)), rows a multiple of 32 (whole K-steps of the
  // vector path); splits past the end contribute zero tiles
  const int64_t rows = round_up(ceil_div(m, splits), 32);
  if (d >= 128) {
    const int64_t nt = ceil_div(d, 128);
    const int vec = ((uintptr_t)SA % 16 == 0) && ldsa % 2 == 0;
    dim3 grid((unsigned)splits, (unsigned)(nt * (nt + 1) / 2));
    hipLaunchKernelGGL((gemm_kernel<double, true, false, 128, 128, 16, 1>), grid, dim3(256), 0, s, d, d, m, 1.0, SA,
                       ldsa, rows * ldsa, SA, ldsa, rows * ldsa, 0.0, part, dp, dp * dp, 1, vec, rows, 0);
    AES_LAUNCH_CHECK();
  } else {
    const int full = (int)(m / rows);
    if (full > 0)
      gemm_f64(true, false, d, d, rows, 1.0, SA, ldsa, rows * ldsa, SA, ldsa, rows * ldsa, 0.0, part, dp, dp * dp,
               full, 1, s);
    const int64_t tail = m - (int64_t)full * rows;
    if (tail > 0)
      gemm_f64(true, false, d, d, tail, 1.0, SA + (int64_t)full * rows * ldsa, ldsa, 0,
               SA + (int64_t)full * rows * ldsa, ldsa, 0, 0.0, part + (int64_t)full * dp * dp, dp, 0, 1, 1, s);
    splits = full + (tail > 0 ? 1 : 0);
  }
  hipLaunchKernelGGL(gram_reduce_kernel<double>, dim3((unsigned)ceil_div(dp * dp, 256)), dim3(256), 0, s, part, splits,
                     d, dp, nu2, lam, G, gprev, wprev, gkeep);
  AES_LAUNCH_CHECK();
}

__global__ void scale_cols_kernel(int64_t m, int64_t d, const double* __restrict__ SA, int64_t ldsa,
                                  const double* __restrict__ invlam, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * d) return;
  const int64_t i = e / d, j = e % d;
  out[e] = SA[i * ldsa + j] * (invlam ? invlam[j] : 1.0);
}

__global__ void w_finish_kernel(int64_t m, int64_t mp, double nu2, double* __restrict__ W) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mp * mp) return;
  const int64_t i = e / mp, j = e % mp;
  if (i < m && j < m) {
    if (i == j) W[e] += nu2;
    else if (j > i) W[e] = 0.0;
  } else {
    W[e] = (i == j) ? 1.0 : 0.0;
  }
}

void gram_nt(int64_t m, int64_t d, const double* SA, int64_t ldsa, double nu2, const double* invlam, double* scaled,
             double* W, int64_t mp, hipStream_t s) {
  hipLaunchKernelGGL(scale_cols_kernel, dim3((unsigned)ceil_div(m * d, 256)), dim3(256), 0, s, m, d, SA, ldsa, invlam,
                     scaled);
  AES_LAUNCH_CHECK();
  gemm_f64(false, true, m, m, d, 1.0, scaled, d, 0, SA, ldsa, 0, 0.0, W, mp, 0, 1, 1, s);
  hipLaunchKernelGGL(w_finish_kernel, dim3((unsigned)ceil_div(mp * mp, 256)), dim3(256), 0, s, m, mp, nu2, W);
  AES_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------------------
// BF16 Gram on MFMA with FP32 accumulation (v_mfma_f32_32x32x16_bf16).  Tile 64 x 64 of
// G = SA^T SA, K-step 16 rows of SA; wave w computes the 32 x 32 block (w >> 1, w & 1).
// A-operand layout of the 32x32x16 bf16 MFMA: lane l supplies 8 consecutive k values
// k = 8*(l/32) .. +7 of row (l % 32); B likewise for column (l % 32); D: register r of lane l
// holds row 8*(r/4) + 4*(l/32)... see store below.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ short bf16_bits(__hip_bfloat16 v) { return *reinterpret_cast<short*>(&v); }

// BF16 Gram partials, XCD-aware split-K over lower-triangle 128 x 128 tiles (grid: splits x
// tiles, split fastest, as the FP64 Gram): part[z][i][j] = sum over split z's rows k of
// SA[k][i] SA[k][j] in FP32 (i >= j).  4 waves, each a 2 x 2 block of 32 x 32 outputs of
// v_mfma_f32_32x32x16_bf16 (register r of lane l: row 8(r/4) + 4(l/32) + r%4, column l%32);
// 32 rows of SA per K-step staged k-major in LDS through 16-byte loads, the next K-step
// prefetched into registers (double-buffered LDS, one barrier per K-step).
__global__ __launch_bounds__(256) void gram_bf16_kernel(int64_t m, int64_t d, const __hip_bfloat16* __restrict__ SA,
                                                        int64_t ldsa, int64_t rows_per_split,
                                                        float* __restrict__ part, int64_t dp, int vec) {
  constexpr int GT = 128, GK = 32, PADC = GT + 8;
  typedef short s8v __attribute__((ext_vector_type(8)));
  typedef float f16v __attribute__((ext_vector_type(16)));
  const int64_t split = blockIdx.x;
  const int64_t t = blockIdx.y;
  int64_t ti = (int64_t)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while (ti * (ti + 1) / 2 > t) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  const int64_t i0 = ti * GT, j0 = (t - ti * (ti + 1) / 2) * GT;
  const int64_t r_begin = split * rows_per_split;
  int64_t r_end = r_begin + rows_per_split;
  if (r_end > m) r_end = m;
  __shared__ __attribute__((aligned(16))) short Ti[2][GK][PADC], Tj[2][GK][PADC];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wm = w >> 1, wn = w & 1;
  const bool full_cols = vec && i0 + GT <= d && j0 + GT <= d;
  f16v acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f16v{};
  s8v ra[2], rb[2];
  // thread's two 16-byte pieces of each operand: row k = idx / 16, columns c8 .. c8 + 7
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = tid + 256 * q;
      const int k = idx >> 4, c8 = (idx & 15) * 8;
      const int64_t gk = k0 + k;
      if (gk < r_end && full_cols) {
        ra[q] = *reinterpret_cast<const s8v*>(SA + gk * ldsa + i0 + c8);
        rb[q] = *reinterpret_cast<const s8v*>(SA + gk * ldsa + j0 + c8);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          ra[q][e] = (gk < r_end && i0 + c8 + e < d) ? bf16_bits(SA[gk * ldsa + i0 + c8 + e]) : (short)0;
          rb[q][e] = (gk < r_end && j0 + c8 + e < d) ? bf16_bits(SA[gk * ldsa + j0 + c8 + e]) : (short)0;
        }
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = tid + 256 * q;
      const int k = idx >> 4, c8 = (idx & 15) * 8;
      *reinterpret_cast<s8v*>(&Ti[buf][k][c8]) = ra[q];
      *reinterpret_cast<s8v*>(&Tj[buf][k][c8]) = rb[q];
    }
  };
  if (r_begin < r_end) {
    load(r_begin);
    store(0);
    __syncthreads();
    int cur = 0;
    for (int64_t k0 = r_begin; k0 < r_end; k0 += GK) {
      const bool more = k0 + GK < r_end;
      if (more) load(k0 + GK);
#pragma unroll
      for (int ks = 0; ks < GK / 16; ++ks) {
        const int kb = ks * 16 + 8 * (lane >> 5);
        s8 a[2], b[2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int e = 0; e < 8; ++e) a[bi][e] = Ti[cur][kb + e][wm * 64 + bi * 32 + (lane & 31)];
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int e = 0; e < 8; ++e) b[bj][e] = Tj[cur][kb + e][wn * 64 + bj * 32 + (lane & 31)];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
            acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(b8, a[bi]),
                                                                  __builtin_bit_cast(b8, b[bj]), acc[bi][bj], 0, 0, 0);
      }
      if (more) store(cur ^ 1);
      __syncthreads();
      cur ^= 1;
    }
  }
  float* out = part + split * dp * dp;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t i = i0 + wm * 64 + bi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t j = j0 + wn * 64 + bj * 32 + (lane & 31);
        if (i < d && j < d && i >= j) out[i * dp + j] = acc[bi][bj][r];
      }
}

void gram_tn_bf16(int64_t m, int64_t d, const __hip_bfloat16* SA, int64_t ldsa, double nu2, const double* lam,
                  float* part, int splits, double* G, int64_t dp, hipStream_t s) {
  // split z: rows [z rows, min(m, (z+1) rows)), rows a multiple of the 32-row K-step
  const int64_t rows = round_up(ceil_div(m, splits), 32);
  const int64_t nt = ceil_div(d, 128);
  const int vec = ((uintptr_t)SA % 16 == 0) && ldsa % 8 == 0;
  dim3 grid((unsigned)splits, (unsigned)(nt * (nt + 1) / 2));
  hipLaunchKernelGGL(gram_bf16_kernel, grid, dim3(256), 0, s, m, d, SA, ldsa, rows, part, dp, vec);
  AES_LAUNCH_CHECK();
  hipLaunchKernelGGL(gram_reduce_kernel<float>, dim3((unsigned)ceil_div(dp * dp, 256)), dim3(256), 0, s, part, splits, d,
                     dp, nu2, lam, G, (const double*)nullptr, 0.0, (double*)nullptr);
  AES_LAUNCH_CHECK();
}

// out[e] = sum_s part[s * stride + e] (fixed order), e < count
__global__ void sum_parts_kernel(int64_t count, int splits, int64_t stride, const double* __restrict__ part,
                                 double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  double v = 0.0;
  for (int sp = 0; sp < splits; ++sp) v += part[(int64_t)sp * stride + e];
  out[e] = v;
}

void launch_sum_parts(int64_t count, int splits, int64_t stride, const double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s, count, splits, stride, part,
                     out);
  AES_LAUNCH_CHECK();
}

__global__ void f32_to_f64_kernel(int64_t count, const float* __restrict__ src, double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) dst[e] = (double)src[e];
}

void widen_f32(int64_t count, const float* src, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(f32_to_f64_kernel, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s, count, src, dst);
  AES_LAUNCH_CHECK();
}

__global__ void f64_to_f32_kernel(int64_t count, const double* __restrict__ src, float* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) dst[e] = (float)src[e];
}

void narrow_f64(int64_t count, const double* src, float* dst, hipStream_t s) {
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s, count, src, dst);
  AES_LAUNCH_CHECK();
}

__global__ void bf16_to_f64_kernel(int64_t m, int64_t d, const __hip_bfloat16* __restrict__ src, int64_t ld,
                                   double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * d) return;
  dst[e] = (double)(float)src[(e / d) * ld + (e % d)];
}

void gram_nt_bf16(int64_t m, int64_t d, const __hip_bfloat16* SA, int64_t ldsa, double nu2, const double* invlam,
                  double* sa64, double* scaled, double* W, int64_t mp, hipStream_t s) {
  // m < d: W is small (m x m); widen the BF16 sketch and reuse the FP64 path.
  hipLaunchKernelGGL(bf16_to_f64_kernel, dim3((unsigned)ceil_div(m * d, 256)), dim3(256), 0, s, m, d, SA, ldsa, sa64);
  AES_LAUNCH_CHECK();
  gram_nt(m, d, sa64, d, nu2, invlam, scaled, W, mp, s);
}

// ---------------------------------------------------------------------------------------
// Cholesky factor and its inverse, by recursion on 2 x 2 block partitions:
//   [A11  .  ]   L11 = chol(A11), X11 = L11^{-1}            (recursive)
//   [A21 A22 ]   L21 = A21 X11^T,  S = A22 - L21 L21^T
//                L22 = chol(S),    X22 = L22^{-1}            (recursive)
//                X21 = -X22 (L21 X11)
// Leaves are 64 x 64 blocks, factorised and inverted by one wavefront (below).
// ---------------------------------------------------------------------------------------
typedef double d2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)bits, l);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Leaf LDS: L row-major (Ls, read by the inverse wave and written out), L column-major (Lc,
// broadcast rows for the Cholesky wave's rank-1 updates), 1 / L[j][j].
struct LeafLds {
  double Ls[64][66];
  double Lc[64][66];
  double rdiag[64];
};

// Cholesky wave, step J (right-looking): lane i holds row i of the partially updated matrix in
// a[].  The pivot a[J] of lane J is broadcast with a cross-lane read, every lane scales its
// entry, the next column is updated at once (look-ahead: it holds the next pivot), and the
// remaining columns receive the rank-1 update with column J read back from Lc.  A barrier
// after every 8 steps releases the inverse wave.
template <int J>
struct LeafChol {
  __device__ __forceinline__ static void step(double (&a)[64], LeafLds& sm, int lane, bool& bad) {
    const double pj = readlane_d(a[J], J);
    const bool ok = pj > 0.0;  // uniform
    if (!ok) bad = true;
    const double piv = ok ? pj : 1.0;
    // 1/sqrt(piv): hardware estimate refined by two Newton steps (y <- y (3 - p y^2) / 2)
    double y = __builtin_amdgcn_rsq(piv);
    y = y * fma(-0.5 * piv, y * y, 1.5);
    y = y * fma(-0.5 * piv, y * y, 1.5);
    const double l = lane == J ? piv * y : (lane > J ? a[J] * y : 0.0);
    a[J] = l;
    sm.Ls[lane][J] = l;
    sm.Lc[J][lane] = l;
    if (lane == 0) sm.rdiag[J] = y;
    if constexpr (J + 1 < 64) {
      const double l1 = readlane_d(l, J + 1);
      a[J + 1] = fma(-l, l1, a[J + 1]);
    }
    if constexpr (J + 2 < 64) {
      // Lc[J][] written above by all lanes of this wave: LDS operations of one wave complete in order
      __builtin_amdgcn_s_waitcnt(0xC07F);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      constexpr int K0 = (J + 2) & ~1;  // 16-byte aligned start
#pragma unroll
      for (int k0 = K0; k0 < 64; k0 += 32) {
        d2 buf[16];
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (k0 + 2 * q < 64) buf[q] = *reinterpret_cast<const d2*>(&sm.Lc[J][k0 + 2 * q]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int k = k0 + 2 * q;
          if (k < 64 && k >= J + 2) a[k] = fma(-l, buf[q][0], a[k]);
          if (k + 1 < 64 && k + 1 >= J + 2) a[k + 1] = fma(-l, buf[q][1], a[k + 1]);
        }
      }
    }
    if constexpr ((J & 7) == 7) __syncthreads();
    LeafChol<J + 1>::step(a, sm, lane, bad);
  }
};
template <>
struct LeafChol<64> {
  __device__ __forceinline__ static void step(double (&)[64], LeafLds&, int, bool&) {}
};

// Inverse wave, step J: lane c owns column c of X = L^{-1} and runs the forward substitution
// x_J = (delta_Jc - sum_{k<J} L[J][k] x_k) / L[J][J] with row J of L read from Ls (batches of
// 16-byte broadcast reads).  Rows 8b .. 8b+7 are final after the Cholesky wave's barrier b.
template <int J>
struct LeafInv {
  __device__ __forceinline__ static void step(double (&x)[64], LeafLds& sm, int lane) {
    if constexpr ((J & 7) == 0) __syncthreads();
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k0 = 0; k0 < J; k0 += 32) {
      d2 buf[16];
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (k0 + 2 * q < J) buf[q] = *reinterpret_cast<const d2*>(&sm.Ls[J][k0 + 2 * q]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int k = k0 + 2 * q;
        if (k < J) s0 = fma(x[k], buf[q][0], s0);
        if (k + 1 < J) s1 = fma(x[k + 1], buf[q][1], s1);
      }
    }
    x[J] = (((J == lane) ? 1.0 : 0.0) - (s0 + s1)) * sm.rdiag[J];
    LeafInv<J + 1>::step(x, sm, lane);
  }
};
template <>
struct LeafInv<64> {
  __device__ __forceinline__ static void step(double (&)[64], LeafLds&, int) {}
};

// Factorises the 64 x 64 block held in sm.Ls (lower triangle read): on return sm.Ls holds L
// (zeros above the diagonal), sm.rdiag 1 / L[j][j], and wave 1's x[] column lane of L^{-1}.
// Wave 0 factorises, wave 1 inverts one 8-row block behind it; further waves of the workgroup
// only take part in the 8 barriers.  The caller synchronises before and after.
__device__ __forceinline__ void leaf_run(LeafLds& sm, int tid, bool& bad, double (&x)[64]) {
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (wave == 0) {
    double a[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) a[j] = (j <= lane) ? sm.Ls[lane][j] : 0.0;
    LeafChol<0>::step(a, sm, lane, bad);
  } else if (wave == 1) {
    LeafInv<0>::step(x, sm, lane);
  } else {
    for (int b = 0; b < 8; ++b) __syncthreads();
  }
}

// Leaf: Cholesky factor L (written over G, upper triangle zeroed) and X = L^{-1} of a 64 x 64
// block, by two wavefronts.
__global__ __launch_bounds__(128) void chol_inv_leaf_kernel(double* __restrict__ G, int64_t ld, double* __restrict__ X,
                                                            int64_t ldx, int* __restrict__ flag) {
  __shared__ __attribute__((aligned(16))) LeafLds sm;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  {
    double v[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) v[q] = G[(int64_t)(2 * q + (tid >> 6)) * ld + lane];  // coalesced staging
#pragma unroll
    for (int q = 0; q < 32; ++q) sm.Ls[2 * q + (tid >> 6)][lane] = v[q];
  }
  __syncthreads();
  bool bad = false;
  double x[64];
  leaf_run(sm, tid, bad, x);
  if (wave == 0) {
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll 8
    for (int i = 0; i < 64; ++i) G[(int64_t)i * ld + lane] = sm.Ls[i][lane];
    if (bad && lane == 0) atomicOr(flag, 1);
  } else {
#pragma unroll
    for (int i = 0; i < 64; ++i) X[(int64_t)i * ldx + lane] = (i >= lane) ? x[i] : 0.0;
  }
}

// 64 x 64 x 64 product on the workgroup's 4 waves: wave w accumulates rows 16w .. 16w+15,
// block bj columns 16bj .. 16bj+15; a_at(i, k), b_at(k, j) fetch the operands.
template <typename FA, typename FB>
__device__ __forceinline__ void mm64(FA a_at, FB b_at, d4 (&acc)[4], int lane, int wave) {
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const int k = kk * 4 + (lane >> 4);
    const double av = a_at(wave * 16 + (lane & 15), k);
    double bv[4];
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) bv[bj] = b_at(k, bj * 16 + (lane & 15));
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[bj], acc[bj], 0, 0, 0);
  }
}

// Node of the recursion with a 128 x 128 block, in one workgroup of 4 waves: leaf on A11,
// L21 = A21 X11^T, S = A22 - L21 L21^T, T2 = L21 X11, leaf on S, X21 = -X22 T2.  X (= L^{-1}) is
// written in full (the caller zero-fills the block above the diagonal); L only if keep_l.
struct NodeLds {
  LeafLds leaf;           // the leaves; leaf.Lc doubles as X11 / X22 between them
  double L21[64][65];
  double T2[64][65];
};

__global__ __launch_bounds__(256) void chol_inv_node128_kernel(double* __restrict__ G, int64_t ld,
                                                               double* __restrict__ X, int64_t ldx,
                                                               int* __restrict__ flag, int keep_l) {
  __shared__ __attribute__((aligned(16))) NodeLds sm;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const double* A21 = G + 64 * ld;
  const double* A22 = G + 64 * ld + 64;
  bool bad = false;
  double x[64];
  // ---- leaf on A11
  {
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = G[(int64_t)(4 * q + wave) * ld + lane];
#pragma unroll
    for (int q = 0; q < 16; ++q) sm.leaf.Ls[4 * q + wave][lane] = v[q];
  }
  __syncthreads();
  leaf_run(sm.leaf, tid, bad, x);
  __syncthreads();
  // X11 -> LDS (row-major in leaf.Lc) and X; L11 -> G
  if (wave == 1) {
#pragma unroll
    for (int i = 0; i < 64; ++i) {
      const double xv = (i >= lane) ? x[i] : 0.0;
      sm.leaf.Lc[i][lane] = xv;
      X[(int64_t)i * ldx + lane] = xv;
    }
  } else if (wave == 0 && keep_l) {
#pragma unroll 8
    for (int i = 0; i < 64; ++i) G[(int64_t)i * ld + lane] = sm.leaf.Ls[i][lane];
  }
  __syncthreads();
  // ---- L21 = A21 X11^T
  {
    d4 acc[4];
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bj] = d4{0.0, 0.0, 0.0, 0.0};
    mm64([&](int i, int k) { return A21[(int64_t)i * ld + k]; }, [&](int k, int j) { return sm.leaf.Lc[j][k]; }, acc,
         lane, wave);
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) sm.L21[wave * 16 + (lane >> 4) + 4 * r][bj * 16 + (lane & 15)] = acc[bj][r];
  }
  __syncthreads();
  // ---- S = A22 - L21 L21^T (into the leaf's input) and T2 = L21 X11
  {
    d4 acc[4];
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[bj][r] = A22[(int64_t)(wave * 16 + (lane >> 4) + 4 * r) * ld + bj * 16 + (lane & 15)];
    mm64([&](int i, int k) { return -sm.L21[i][k]; }, [&](int k, int j) { return sm.L21[j][k]; }, acc, lane, wave);
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) sm.leaf.Ls[wave * 16 + (lane >> 4) + 4 * r][bj * 16 + (lane & 15)] = acc[bj][r];
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bj] = d4{0.0, 0.0, 0.0, 0.0};
    mm64([&](int i, int k) { return sm.L21[i][k]; }, [&](int k, int j) { return sm.leaf.Lc[k][j]; }, acc, lane, wave);
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) sm.T2[wave * 16 + (lane >> 4) + 4 * r][bj * 16 + (lane & 15)] = acc[bj][r];
  }
  if (keep_l) {
    for (int e = tid; e < 64 * 64; e += 256) G[(int64_t)(64 + e / 64) * ld + e % 64] = sm.L21[e / 64][e % 64];
  }
  __syncthreads();
  // ---- leaf on S
  leaf_run(sm.leaf, tid, bad, x);
  __syncthreads();
  // X22 -> LDS (leaf.Lc) and X; L22 -> G
  double* X22 = X + 64 * ldx + 64;
  if (wave == 1) {
#pragma unroll
    for (int i = 0; i < 64; ++i) {
      const double xv = (i >= lane) ? x[i] : 0.0;
      sm.leaf.Lc[i][lane] = xv;
      X22[(int64_t)i * ldx + lane] = xv;
    }
  } else if (wave == 0 && keep_l) {
#pragma unroll 8
    for (int i = 0; i < 64; ++i) G[(int64_t)(64 + i) * ld + 64 + lane] = sm.leaf.Ls[i][lane];
  }
  __syncthreads();
  // ---- X21 = -X22 T2
  {
    d4 acc[4];
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bj] = d4{0.0, 0.0, 0.0, 0.0};
    mm64([&](int i, int k) { return -sm.leaf.Lc[i][k]; }, [&](int k, int j) { return sm.T2[k][j]; }, acc, lane, wave);
    double* X21 = X + 64 * ldx;
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) X21[(int64_t)(wave * 16 + (lane >> 4) + 4 * r) * ldx + bj * 16 + (lane & 15)] = acc[bj][r];
  }
  if (bad && tid == 0) atomicOr(flag, 1);
}

__global__ void copy_block_kernel(int64_t rows, int64_t cols, const double* __restrict__ src, int64_t lds,
                                  double* __restrict__ dst, int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e / cols, j = e % cols;
  dst[i * ldd + j] = src[i * lds + j];
}

static void cholinv_rec(double* G, double* X, int64_t ld, int64_t o, int64_t h, double* tmp, int* flag, bool keep_l,
                        hipStream_t s) {
  if (h == 64) {
    hipLaunchKernelGGL(chol_inv_leaf_kernel, dim3(1), dim3(128), 0, s, G + o * ld + o, ld, X + o * ld + o, ld, flag);
    AES_LAUNCH_CHECK();
    return;
  }
  if (h == 128) {
    hipLaunchKernelGGL(chol_inv_node128_kernel, dim3(1), dim3(256), 0, s, G + o * ld + o, ld, X + o * ld + o, ld, flag,
                       keep_l ? 1 : 0);
    AES_LAUNCH_CHECK();
    return;
  }
  const int64_t nb = h / 64;
  const int64_t h1 = 64 * ((nb + 1) / 2), h2 = h - h1;
  cholinv_rec(G, X, ld, o, h1, tmp, flag, keep_l, s);
  double* A21 = G + (o + h1) * ld + o;
  double* A22 = G + (o + h1) * ld + (o + h1);
  const double* X11 = X + o * ld + o;
  double* T1 = tmp;             // h2 x h1: L21
  double* T2 = tmp + h2 * h1;   // h2 x h1: L21 X11
  // L21 = A21 X11^T
  gemm_f64(false, true, h2, h1, h1, 1.0, A21, ld, 0, X11, ld, 0, 0.0, T1, h1, 0, 1, 0, s);
  if (keep_l) {
    hipLaunchKernelGGL(copy_block_kernel, dim3((unsigned)ceil_div(h2 * h1, 256)), dim3(256), 0, s, h2, h1, T1, h1, A21,
                       ld);
    AES_LAUNCH_CHECK();
  }
  // S = A22 - L21 L21^T (lower)
  gemm_f64(false, true, h2, h2, h1, -1.0, T1, h1, 0, T1, h1, 0, 1.0, A22, ld, 0, 1, 1, s);
  // T2 = L21 X11
  gemm_f64(false, false, h2, h1, h1, 1.0, T1, h1, 0, X11, ld, 0, 0.0, T2, h1, 0, 1, 0, s);
  cholinv_rec(G, X, ld, o + h1, h2, tmp + 2 * h2 * h1, flag, keep_l, s);
  // X21 = -X22 T2
  gemm_f64(false, false, h2, h1, h2, -1.0, X + (o + h1) * ld + (o + h1), ld, 0, T2, h1, 0, 0.0, X + (o + h1) * ld + o,
           ld, 0, 1, 0, s);
}

size_t cholinv_tmp_size(int64_t np) { return (size_t)np * np; }

void cholinv(double* G, int64_t np, double* Linv, double* tmp, int* flag, bool keep_l, hipStream_t s) {
  launch_fill(Linv, np * np, 0.0, s);
  cholinv_rec(G, Linv, np, 0, np, tmp, flag, keep_l, s);
}

// ---------------------------------------------------------------------------------------
// Gaussian sketch: SA (m x d) = G A / sqrt(m) with G_ij ~ N(0, 1) (Sec. 2.1).  Each entry of G
// is generated exactly once per sketch: a slab of K-rows at a time goes into the K-major buffer
// Gt (row r holds G[0..m, i0 + r]), and the slab is contracted with the same rows of A by the
// FP64 MFMA GEMM (the layout of the Gram, opA = Gt^T).  When the m x d output has too few
// tiles to fill the chip, the slab is cut into a batch of K-ranges writing partial products
// that are summed at the end in a fixed order.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gauss_gen_kernel(int64_t i0, int64_t rows, int64_t nq, int64_t mp,
                                                        uint64_t k0key, uint64_t k1key, double* __restrict__ Gt) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= nq) return;
  for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
    // four consecutive rows of G (4q .. 4q + 3) in column i0 + r come from one Philox block
    const Rand4 rn = philox4x64_10((uint64_t)(i0 + r), kStreamGauss, (uint64_t)q, 0, k0key, k1key);
    double z[4];
    gauss4(rn, z);
    double2* dst = reinterpret_cast<double2*>(Gt + r * mp + 4 * q);
    dst[0] = make_double2(z[0], z[1]);
    dst[1] = make_double2(z[2], z[3]);
  }
}

GaussPlan gauss_plan(int num_cu, int64_t n, int64_t d, int64_t m) {
  GaussPlan p;
  p.mp = round_up(m, 4);
  const int64_t tiles = ceil_div(m, 128) * ceil_div(d, 128);
  int64_t splits = std::min<int64_t>(64, std::max<int64_t>(1, ceil_div(2 * (int64_t)num_cu, tiles)));
  splits = std::min(splits, ceil_div(n, 64));
  // at most 2^25 generated entries resident at once (256 MiB)
  constexpr int64_t kBudget = int64_t(1) << 25;
  const int64_t cap = std::max<int64_t>(64, kBudget / (splits * p.mp) / 64 * 64);
  p.ks = std::min(round_up(ceil_div(n, splits), 64), cap);
  // every K-range of the first slab holds rows, so that slab initialises every output
  p.splits = (int)std::min(splits, ceil_div(n, p.ks));
  p.gt_elems = (size_t)p.splits * p.ks * p.mp;
  p.part_elems = p.splits > 1 ? (size_t)p.splits * m * d : 0;
  return p;
}

void launch_gauss_sketch(const GaussPlan& p, const double* A, int64_t n, int64_t d, int64_t lda, int64_t m,
                         uint64_t seed, int32_t problem, int64_t k, double* SA, double* gt, double* part,
                         hipStream_t s) {
  const RngKey key = make_key(seed, problem, k);
  const double alpha = 1.0 / std::sqrt((double)m);
  const int S = p.splits;
  double* out = S > 1 ? part : SA;
  const int64_t slab = (int64_t)S * p.ks, nq = p.mp / 4, md = m * d;
  for (int64_t base = 0; base < n; base += slab) {
    const int64_t rows = std::min(slab, n - base);
    dim3 grid((unsigned)ceil_div(nq, 256), (unsigned)std::min<int64_t>(rows, 16384));
    hipLaunchKernelGGL(gauss_gen_kernel, grid, dim3(256), 0, s, base, rows, nq, p.mp, key.k0, key.k1, gt);
    AES_LAUNCH_CHECK();
    const double beta = base > 0 ? 1.0 : 0.0;
    const int64_t full = rows / p.ks, rem = rows % p.ks;
    if (full > 0)
      gemm_f64(true, false, m, d, p.ks, alpha, gt, p.mp, p.ks * p.mp, A + base * lda, lda, p.ks * lda, beta, out, d,
               md, (int)full, 0, s);
    if (rem > 0)
      gemm_f64(true, false, m, d, rem, alpha, gt + full * p.ks * p.mp, p.mp, 0, A + (base + full * p.ks) * lda, lda,
               0, beta, out + full * md, d, 0, 1, 0, s);
  }
  if (S > 1) launch_sum_parts(md, S, md, part, SA, s);
}

}  // namespace aes
