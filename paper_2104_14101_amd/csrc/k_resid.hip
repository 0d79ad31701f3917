// Explicit residual r = b - A^T (A x) - nu^2 Lambda x (Algorithm 2's "r_t = b - H x_t") in
// compensated FP64: every product is split exactly into a rounded part and its error (TwoProd
// by fma) and every sum is carried as an unevaluated pair hi + lo (TwoSum), so the residual --
// a small difference of terms of the size of H x -- is formed as in about twice the working
// precision and rounded to FP64 once at the end.  Used by the refinement sweeps of the mixed
// precision and batched solves.
//   pass 1: z = A x as pairs (one wave per row of A);
//   pass 2: per row-block partials of A^T z as pairs (columns of A over the threads);
//   pass 3: the partials summed in a fixed order, then b - (.) - nu^2 lambda x, rounded.
// C right-hand sides (a power of two <= 32), x and r are d x C row-major.
#include "common.h"
#include "kernels.h"

// The error-free transformations below need every product rounded on its own and never fused
// with a following addition (a fused a*b + c would skip the rounding that TwoProd's correction
// term accounts for): no floating-point contraction in this file; fma only where written.
#pragma clang fp contract(off)

namespace aes {

namespace {

// Error-free transformations (plain operators: with contraction off each is rounded on its own).
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void fast_two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  e = b - (s - a);
}
__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e) {
  p = a * b;
  e = fma(a, b, -p);
}
// (hi, lo) += (bh, bl)
__device__ __forceinline__ void dd_add(double& hi, double& lo, double bh, double bl) {
  double s, e;
  two_sum(hi, bh, s, e);
  e = e + (lo + bl);
  fast_two_sum(s, e, hi, lo);
}
// (hi, lo) += a * (zh + zl): the product a zh exactly, a zl to working precision
__device__ __forceinline__ void dd_fma(double& hi, double& lo, double a, double zh, double zl) {
  double p, pe;
  two_prod(a, zh, p, pe);
  pe = fma(a, zl, pe);
  dd_add(hi, lo, p, pe);
}

constexpr int kRT = 256;  // threads per workgroup of the three passes

// pass 1: z[i][c] = sum_k A[i][k] x[k][c] as (zh, zl); lane l takes column c = l % C and every
// (64 / C)-th k; the lanes of a column are combined by a fixed-order tree of shuffles.
template <int C>
__global__ __launch_bounds__(kRT) void resid_ax_kernel(int64_t n, int64_t d, const double* __restrict__ A, int64_t lda,
                                                       const double* __restrict__ x, double* __restrict__ zh,
                                                       double* __restrict__ zl) {
  constexpr int S = 64 / C;
  const int lane = threadIdx.x & 63, c = lane % C, sl = lane / C;
  const int64_t wave = ((int64_t)blockIdx.x * kRT + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kRT) >> 6;
  for (int64_t i = wave; i < n; i += nwaves) {
    const double* Ai = A + i * lda;
    double hi = 0.0, lo = 0.0;
    for (int64_t k = sl; k < d; k += S) dd_fma(hi, lo, Ai[k], x[k * C + c], 0.0);
#pragma unroll
    for (int off = C; off < 64; off *= 2) {
      const double oh = __shfl_down(hi, off, 64), ol = __shfl_down(lo, off, 64);
      if (sl % (2 * (off / C)) == 0) dd_add(hi, lo, oh, ol);
    }
    if (sl == 0) {
      zh[i * C + c] = hi;
      zl[i * C + c] = lo;
    }
  }
}

// pass 2: part[b][j][c] = sum over the rows of block b of A[i][j] (zh + zl)[i][c]; thread t owns
// column c = t % C and the columns j0 + t / C + J s (J = 256 / C, s < 8) of its tile.
template <int C>
__global__ __launch_bounds__(kRT) void resid_atz_kernel(int64_t n, int64_t d, const double* __restrict__ A, int64_t lda,
                                                        const double* __restrict__ zh, const double* __restrict__ zl,
                                                        int64_t rows, double* __restrict__ ph, double* __restrict__ pl) {
  constexpr int J = kRT / C, S = 8;
  const int t = threadIdx.x, c = t % C, jj = t / C;
  const int64_t j0 = (int64_t)blockIdx.x * J * S;
  const int64_t r0 = (int64_t)blockIdx.y * rows, r1 = r0 + rows < n ? r0 + rows : n;
  double hi[S], lo[S];
#pragma unroll
  for (int s = 0; s < S; ++s) hi[s] = lo[s] = 0.0;
  for (int64_t i = r0; i < r1; ++i) {
    const double h = zh[i * C + c], l = zl[i * C + c];
    const double* Ai = A + i * lda + j0 + jj;
#pragma unroll
    for (int s = 0; s < S; ++s)
      if (j0 + jj + J * s < d) dd_fma(hi[s], lo[s], Ai[J * s], h, l);
  }
  const int64_t base = (int64_t)blockIdx.y * d * C;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int64_t j = j0 + jj + J * s;
    if (j < d) {
      ph[base + j * C + c] = hi[s];
      pl[base + j * C + c] = lo[s];
    }
  }
}

// pass 3: r = b - sum_b part[b] - nu^2 lambda x, the partials summed in block order, the nu^2
// lambda x term formed exactly as pairs (nu2 = nh + nl exactly), rounded once.
__global__ __launch_bounds__(kRT) void resid_combine_kernel(int64_t d, int C, int nrb, const double* __restrict__ ph,
                                                            const double* __restrict__ pl, const double* __restrict__ b,
                                                            int64_t ldb, const double* __restrict__ x,
                                                            const double* __restrict__ lam, double nu,
                                                            double* __restrict__ r, int64_t ldr) {
  const int64_t e = (int64_t)blockIdx.x * kRT + threadIdx.x;
  if (e >= d * C) return;
  const int64_t j = e / C;
  const int c = (int)(e - j * C);
  double qh = 0.0, ql = 0.0;
  for (int w = 0; w < nrb; ++w) dd_add(qh, ql, ph[(int64_t)w * d * C + e], pl[(int64_t)w * d * C + e]);
  // nu^2 lambda_j x_jc: nu^2 = nh + nl exactly, (lambda x) = ph2 + pe2 exactly, the pair product
  double nh, nl;
  two_prod(nu, nu, nh, nl);
  double lx, lxe;
  two_prod(lam ? lam[j] : 1.0, x[e], lx, lxe);
  double th, te;
  two_prod(nh, lx, th, te);
  te = fma(nh, lxe, fma(nl, lx, te));
  dd_add(qh, ql, th, te);
  // r = b - q
  double rh = b[j * ldb + c], rl = 0.0;
  dd_add(rh, rl, -qh, -ql);
  r[j * ldr + c] = rh + rl;
}

}  // namespace

int resid_blocks(int num_cu, int64_t n, int64_t d, int C, int64_t* rows) {
  const int64_t tiles = ceil_div(d, (int64_t)(kRT / C) * 8);
  const int64_t want = std::max<int64_t>(1, 4 * (int64_t)num_cu / tiles);
  int64_t nrb = std::min<int64_t>(want, ceil_div(n, 64));
  nrb = std::max<int64_t>(1, nrb);
  *rows = ceil_div(n, nrb);
  return (int)ceil_div(n, *rows);
}

void launch_residual_dd(int num_cu, int64_t n, int64_t d, int C, const double* A, int64_t lda, const double* b,
                        int64_t ldb, double nu, const double* lam, const double* x, double* zh, double* zl, double* ph,
                        double* pl, double* r, int64_t ldr, hipStream_t s) {
  int64_t rows = 0;
  const int nrb = resid_blocks(num_cu, n, d, C, &rows);
  const unsigned g1 = (unsigned)std::min<int64_t>(ceil_div(n, kRT / 64), 8 * (int64_t)num_cu);
  const dim3 g2((unsigned)ceil_div(d, (int64_t)(kRT / C) * 8), (unsigned)nrb);
#define AES_RESID_CASE(CV)                                                                                        \
  case CV:                                                                                                        \
    hipLaunchKernelGGL(resid_ax_kernel<CV>, dim3(g1), dim3(kRT), 0, s, n, d, A, lda, x, zh, zl);                  \
    AES_LAUNCH_CHECK();                                                                                           \
    hipLaunchKernelGGL(resid_atz_kernel<CV>, g2, dim3(kRT), 0, s, n, d, A, lda, zh, zl, rows, ph, pl);            \
    AES_LAUNCH_CHECK();                                                                                           \
    break;
  switch (C) {
    AES_RESID_CASE(1)
    AES_RESID_CASE(2)
    AES_RESID_CASE(4)
    AES_RESID_CASE(8)
    AES_RESID_CASE(16)
    AES_RESID_CASE(32)
    default:
      throw std::invalid_argument("compensated residual: C must be a power of two <= 32");
  }
#undef AES_RESID_CASE
  hipLaunchKernelGGL(resid_combine_kernel, dim3((unsigned)ceil_div(d * C, kRT)), dim3(kRT), 0, s, d, C, nrb, ph, pl, b,
                     ldb, x, lam, nu, r, ldr);
  AES_LAUNCH_CHECK();
}

size_t residual_dd_part_elems(int num_cu, int64_t n, int64_t d, int C) {
  int64_t rows = 0;
  const int nrb = resid_blocks(num_cu, n, d, C, &rows);
  return (size_t)nrb * d * C;
}

}  // namespace aes
