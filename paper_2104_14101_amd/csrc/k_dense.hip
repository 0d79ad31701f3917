// Dense kernels on the FP64 (and BF16) matrix cores of gfx950:
//   * a tiled GEMM C = alpha op(A) op(B) + beta C (64 x 64 tiles, v_mfma_f64_16x16x4f64),
//     used for the Gram of the sketch, the Cholesky panels and trailing updates and the
//     triangular inverse;
//   * the Gram (SA)^T SA + nu^2 Lambda with split-K, and W = SA Lambda^{-1} SA^T + nu^2 I
//     (the two factorisation branches of Sec. 4.1);
//   * a blocked right-looking Cholesky (64 x 64 diagonal blocks factorised in LDS) and the
//     inverse of its lower-triangular factor;
//   * the Gaussian sketch S A = G A / sqrt(m) with the N(0,1) tile of G generated on chip
//     (Philox + Box-Muller) for every K-step, so G is never stored.
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

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_f64_kernel(int64_t M, int64_t N, int64_t K, double alpha,
                                                       const double* __restrict__ A, int64_t lda, int64_t sA,
                                                       const double* __restrict__ B, int64_t ldb, int64_t sB,
                                                       double beta, double* C, int64_t ldc, int64_t sC, int tri) {
  const int64_t bz = blockIdx.z;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  const int64_t m0 = (int64_t)blockIdx.y * BT, n0 = (int64_t)blockIdx.x * BT;
  if (tri && n0 > m0 + BT - 1) return;
  __shared__ double As[BKT][BT + 1], Bs[BKT][BT + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wm = w >> 1, wn = w & 1;
  d4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = d4{0.0, 0.0, 0.0, 0.0};

  for (int64_t k0 = 0; k0 < K; k0 += BKT) {
#pragma unroll
    for (int rep = 0; rep < 4; ++rep) {
      const int idx = tid + rep * 256;
      int i, k;
      if (!TA) {
        k = idx & 15;
        i = idx >> 4;
      } else {
        i = idx & 63;
        k = idx >> 6;
      }
      const int64_t gi = m0 + i, gk = k0 + k;
      double va = 0.0;
      if (gi < M && gk < K) va = TA ? A[gk * lda + gi] : A[gi * lda + gk];
      As[k][i] = va;
      int j;
      if (!TB) {
        j = idx & 63;
        k = idx >> 6;
      } else {
        k = idx & 15;
        j = idx >> 4;
      }
      const int64_t gj = n0 + j, gk2 = k0 + k;
      double vb = 0.0;
      if (gj < N && gk2 < K) vb = TB ? B[gj * ldb + gk2] : B[gk2 * ldb + gj];
      Bs[k][j] = vb;
    }
    __syncthreads();
    mfma_ktile(As, Bs, lane, wm, wn, acc);
    __syncthreads();
  }
  store_tile(acc, lane, wm, wn, m0, n0, [&](int64_t i, int64_t j, double v) {
    if (i < M && j < N && (!tri || i >= j)) {
      double out = alpha * v;
      if (beta != 0.0) out += beta * C[i * ldc + j];
      C[i * ldc + j] = out;
    }
  });
}

void gemm_f64(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
              int64_t sA, const double* B, int64_t ldb, int64_t sB, double beta, double* C, int64_t ldc, int64_t sC,
              int batch, int tri, hipStream_t s) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  dim3 grid((unsigned)ceil_div(N, BT), (unsigned)ceil_div(M, BT), (unsigned)batch);
  if (!ta && !tb)
    hipLaunchKernelGGL((gemm_f64_kernel<false, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB,
                       beta, C, ldc, sC, tri);
  else if (!ta && tb)
    hipLaunchKernelGGL((gemm_f64_kernel<false, true>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB,
                       beta, C, ldc, sC, tri);
  else if (ta && !tb)
    hipLaunchKernelGGL((gemm_f64_kernel<true, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB,
                       beta, C, ldc, sC, tri);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<true, true>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB,
                       beta, C, ldc, sC, tri);
  AES_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------------------
// Gram of the sketch.
// ---------------------------------------------------------------------------------------
int gram_splits(int num_cu, int64_t m, int64_t d) {
  const int64_t tiles = ceil_div(d, BT) * (ceil_div(d, BT) + 1) / 2;
  int64_t splits = ceil_div((int64_t)num_cu * 2, tiles);
  const int64_t max_by_k = ceil_div(m, 256);  // keep >= 256 rows per split
  if (splits > max_by_k) splits = max_by_k;
  if (splits > 64) splits = 64;
  return (int)(splits < 1 ? 1 : splits);
}

// G[i,j] (lower, padded to dp) = sum_s part[s][i][j] + nu2 lam_i [i == j]; identity padding; upper = 0
template <typename TP>
__global__ void gram_reduce_kernel(const TP* __restrict__ part, int splits, int64_t d, int64_t dp, double nu2,
                                   const double* __restrict__ lam, double* __restrict__ G) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= dp * dp) return;
  const int64_t i = e / dp, j = e % dp;
  double v = 0.0;
  if (i < d && j < d && i >= j) {
    for (int s = 0; s < splits; ++s) v += (double)part[(int64_t)s * dp * dp + i * dp + j];
    if (i == j) v += nu2 * (lam ? lam[i] : 1.0);
  } else if (i == j) {
    v = 1.0;
  }
  G[e] = v;
}

void gram_tn(int64_t m, int64_t d, const double* SA, int64_t ldsa, double nu2, const double* lam, double* part,
             int splits, double* G, int64_t dp, hipStream_t s) {
  const int64_t rows = ceil_div(m, splits);
  // splits with identical row counts except the last: run the full batch on `rows` rows
  // (the tail split reads rows up to m only through a separate call)
  const int full = (int)(m / rows);
  if (full > 0)
    gemm_f64(true, false, d, d, rows, 1.0, SA, ldsa, rows * ldsa, SA, ldsa, rows * ldsa, 0.0, part, dp, dp * dp, full,
             1, s);
  const int64_t tail = m - (int64_t)full * rows;
  if (tail > 0)
    gemm_f64(true, false, d, d, tail, 1.0, SA + (int64_t)full * rows * ldsa, ldsa, 0, SA + (int64_t)full * rows * ldsa,
             ldsa, 0, 0.0, part + (int64_t)full * dp * dp, dp, 0, 1, 1, s);
  const int used = full + (tail > 0 ? 1 : 0);
  hipLaunchKernelGGL(gram_reduce_kernel<double>, dim3((unsigned)ceil_div(dp * dp, 256)), dim3(256), 0, s, part, used, d,
                     dp, nu2, lam, G);
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

__global__ __launch_bounds__(256) void gram_bf16_kernel(int64_t m, int64_t d, const __hip_bfloat16* __restrict__ SA,
                                                        int64_t ldsa, int64_t rows_per_split,
                                                        float* __restrict__ part, int64_t dp) {
  const int64_t split = blockIdx.z;
  const int64_t r_begin = split * rows_per_split;
  int64_t r_end = r_begin + rows_per_split;
  if (r_end > m) r_end = m;
  const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
  if (j0 > i0 + 63) return;
  // k-major staging: Ts[k][c] for the 64 columns of the i tile and the j tile
  __shared__ short Ti[16][64 + 8], Tj[16][64 + 8];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wm = w >> 1, wn = w & 1;
  typedef float f16v __attribute__((ext_vector_type(16)));
  f16v accv = {};
  for (int64_t k0 = r_begin; k0 < r_end; k0 += 16) {
#pragma unroll
    for (int rep = 0; rep < 4; ++rep) {
      const int idx = tid + rep * 256;  // 0..1023 : 16 rows x 64 cols
      const int k = idx >> 6, c = idx & 63;
      const int64_t gk = k0 + k;
      short vi = 0, vj = 0;
      if (gk < r_end) {
        if (i0 + c < d) vi = bf16_bits(SA[gk * ldsa + i0 + c]);
        if (j0 + c < d) vj = bf16_bits(SA[gk * ldsa + j0 + c]);
      }
      Ti[k][c] = vi;
      Tj[k][c] = vj;
    }
    __syncthreads();
    s8 a, b;
    const int kb = 8 * (lane >> 5);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = Ti[kb + e][wm * 32 + (lane & 31)];
      b[e] = Tj[kb + e][wn * 32 + (lane & 31)];
    }
    accv = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(b8, a), __builtin_bit_cast(b8, b), accv, 0, 0, 0);
    __syncthreads();
  }
  float* out = part + split * dp * dp;
  // D layout of 32x32 MFMA: register r of lane l: row = 8*(r/4) + 4*(l/32) + (r%4), col = l%32
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t i = i0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const int64_t j = j0 + wn * 32 + (lane & 31);
    if (i < d && j < d && i >= j) out[i * dp + j] = accv[r];
  }
}

void gram_tn_bf16(int64_t m, int64_t d, const __hip_bfloat16* SA, int64_t ldsa, double nu2, const double* lam,
                  float* part, int splits, double* G, int64_t dp, hipStream_t s) {
  const int64_t rows = round_up(ceil_div(m, splits), 16);
  const int used = (int)ceil_div(m, rows);
  dim3 grid((unsigned)ceil_div(d, 64), (unsigned)ceil_div(d, 64), (unsigned)used);
  hipLaunchKernelGGL(gram_bf16_kernel, grid, dim3(256), 0, s, m, d, SA, ldsa, rows, part, dp);
  AES_LAUNCH_CHECK();
  hipLaunchKernelGGL(gram_reduce_kernel<float>, dim3((unsigned)ceil_div(dp * dp, 256)), dim3(256), 0, s, part, used, d,
                     dp, nu2, lam, G);
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
// Cholesky.
// ---------------------------------------------------------------------------------------
// Factorise one 64 x 64 diagonal block in LDS (lower), write L back (upper zeroed) and the
// inverse of L to dinv (64 x 64, ld 64).  flag set on a non-positive / NaN pivot.
__global__ __launch_bounds__(256) void potf2_inv_kernel(double* __restrict__ Gk, int64_t ld,
                                                        double* __restrict__ dinv, int* __restrict__ flag) {
  __shared__ double a[64][65];
  __shared__ double x[64][65];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int i = idx >> 6, j = idx & 63;
    a[i][j] = (j <= i) ? Gk[(int64_t)i * ld + j] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < 64; ++j) {
    if (tid == 0) {
      double piv = a[j][j];
      if (!(piv > 0.0)) {
        atomicOr(flag, 1);
        piv = 1.0;
      }
      a[j][j] = sqrt(piv);
    }
    __syncthreads();
    const double ljj = a[j][j];
    for (int i = j + 1 + tid; i < 64; i += 256) a[i][j] /= ljj;
    __syncthreads();
    const int w = 63 - j;
    for (int idx = tid; idx < w * w; idx += 256) {
      const int ii = j + 1 + idx / w, kk = j + 1 + idx % w;
      if (kk <= ii) a[ii][kk] -= a[ii][j] * a[kk][j];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int i = idx >> 6, j = idx & 63;
    Gk[(int64_t)i * ld + j] = (j <= i) ? a[i][j] : 0.0;
  }
  // inverse of the lower-triangular block, row by row: X[i][j] = -(sum_{k=j}^{i-1} L[i][k] X[k][j]) / L[i][i]
  for (int idx = tid; idx < 64 * 64; idx += 256) x[idx >> 6][idx & 63] = 0.0;
  __syncthreads();
  for (int i = 0; i < 64; ++i) {
    if (tid < 64) {
      const int j = tid;
      double v;
      if (j == i) {
        v = 1.0 / a[i][i];
      } else if (j < i) {
        double s = 0.0;
        for (int k = j; k < i; ++k) s += a[i][k] * x[k][j];
        v = -s / a[i][i];
      } else {
        v = 0.0;
      }
      x[i][j] = v;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < 64 * 64; idx += 256) dinv[idx] = x[idx >> 6][idx & 63];
}

void cholesky_inplace(double* G, int64_t np, double* dinv, int* flag, hipStream_t s) {
  const int64_t nb = np / 64;
  for (int64_t kb = 0; kb < nb; ++kb) {
    const int64_t k0 = kb * 64;
    double* Gk = G + k0 * np + k0;
    hipLaunchKernelGGL(potf2_inv_kernel, dim3(1), dim3(256), 0, s, Gk, np, dinv + kb * 4096, flag);
    AES_LAUNCH_CHECK();
    const int64_t rb = np - k0 - 64;
    if (rb > 0) {
      double* L21 = G + (k0 + 64) * np + k0;
      // L21 = A21 inv(L11)^T (in place: one column tile per workgroup row block)
      gemm_f64(false, true, rb, 64, 64, 1.0, L21, np, 0, dinv + kb * 4096, 64, 0, 0.0, L21, np, 0, 1, 0, s);
      // A22 -= L21 L21^T (lower)
      gemm_f64(false, true, rb, rb, 64, -1.0, L21, np, 0, L21, np, 0, 1.0, G + (k0 + 64) * np + (k0 + 64), np, 0, 1, 1,
               s);
    }
  }
}

__global__ void place_diag_inv_kernel(int64_t np, const double* __restrict__ dinv, double* __restrict__ Linv) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= np * np) return;
  const int64_t i = e / np, j = e % np;
  const int64_t bi = i >> 6, bj = j >> 6;
  Linv[e] = (bi == bj) ? dinv[bi * 4096 + (i & 63) * 64 + (j & 63)] : 0.0;
}

// Linv = L^{-1} by block diagonals: X_ij = -inv(L_ii) * sum_{k=j}^{i-1} L_ik X_kj, i = j + s.
void trtri_lower(const double* L, int64_t np, const double* dinv, double* Linv, double* tmp, hipStream_t s) {
  const int64_t nb = np / 64;
  hipLaunchKernelGGL(place_diag_inv_kernel, dim3((unsigned)ceil_div(np * np, 256)), dim3(256), 0, s, np, dinv, Linv);
  AES_LAUNCH_CHECK();
  const int64_t dstride = 64 * np + 64;
  for (int64_t sd = 1; sd < nb; ++sd) {
    const int batch = (int)(nb - sd);
    // T_j = L[(j+s) blk, j..j+s-1 blks] * X[j..j+s-1 blks, j blk]    (64 x 64, K = 64 s)
    gemm_f64(false, false, 64, 64, 64 * sd, 1.0, L + sd * 64 * np, np, dstride, Linv, np, dstride, 0.0, tmp, 64, 4096,
             batch, 0, s);
    // X_(j+s),j = -inv(L_(j+s)(j+s)) T_j
    gemm_f64(false, false, 64, 64, 64, -1.0, dinv + sd * 4096, 64, 4096, tmp, 64, 4096, 0.0, Linv + sd * 64 * np, np,
             dstride, batch, 0, s);
  }
}

// ---------------------------------------------------------------------------------------
// Gaussian sketch: SA (m x d) = G A / sqrt(m), G generated per K-step in LDS.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gauss_sketch_kernel(const double* __restrict__ A, int64_t n, int64_t d,
                                                           int64_t lda, int64_t m, uint64_t k0key, uint64_t k1key,
                                                           double scale, double* __restrict__ SA, int64_t ldsa) {
  const int64_t m0 = (int64_t)blockIdx.y * BT, n0 = (int64_t)blockIdx.x * BT;
  __shared__ double As[BKT][BT + 1], Bs[BKT][BT + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wm = w >> 1, wn = w & 1;
  d4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = d4{0.0, 0.0, 0.0, 0.0};
  const int gk_local = tid & 15, gq = tid >> 4;  // column of G in the K-step, row quad
  for (int64_t k0 = 0; k0 < n; k0 += BKT) {
    {
      const int64_t i = k0 + gk_local;
      double z[4] = {0.0, 0.0, 0.0, 0.0};
      if (i < n) {
        const Rand4 r = philox4x64_10((uint64_t)i, kStreamGauss, (uint64_t)(m0 / 4 + gq), 0, k0key, k1key);
        gauss4(r, z);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) As[gk_local][4 * gq + e] = z[e];
    }
#pragma unroll
    for (int rep = 0; rep < 4; ++rep) {
      const int idx = tid + rep * 256;
      const int j = idx & 63, k = idx >> 6;
      const int64_t gj = n0 + j, gk = k0 + k;
      Bs[k][j] = (gj < d && gk < n) ? A[gk * lda + gj] : 0.0;
    }
    __syncthreads();
    mfma_ktile(As, Bs, lane, wm, wn, acc);
    __syncthreads();
  }
  store_tile(acc, lane, wm, wn, m0, n0, [&](int64_t i, int64_t j, double v) {
    if (i < m && j < d) SA[i * ldsa + j] = v * scale;
  });
}

void launch_gauss_sketch(const double* A, int64_t n, int64_t d, int64_t lda, int64_t m, uint64_t seed, int32_t problem,
                         int64_t k, double* SA, int64_t ldsa, hipStream_t s) {
  const RngKey key = make_key(seed, problem, k);
  dim3 grid((unsigned)ceil_div(d, BT), (unsigned)ceil_div(m, BT));
  hipLaunchKernelGGL(gauss_sketch_kernel, grid, dim3(256), 0, s, A, n, d, lda, m, key.k0, key.k1,
                     1.0 / std::sqrt((double)m), SA, ldsa);
  AES_LAUNCH_CHECK();
}

}  // namespace aes
