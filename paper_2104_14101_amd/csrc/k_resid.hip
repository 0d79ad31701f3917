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
// (hi, lo) = (ah, al) + (hi, lo): the same operation with the operands in the other order, so
// that two lanes exchanging their pairs compute bit-identical sums
__device__ __forceinline__ void dd_add2(double ah, double al, double& hi, double& lo) {
  double s, e;
  two_sum(ah, hi, s, e);
  e = e + (al + lo);
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

// pass 1 for C >= 8: a workgroup owns RB = R 256 / C consecutive rows (R = 4 for C >= 16, else
// 2); thread t takes column c = t % C of rows t / C + q 256 / C (q < R), R independent chains,
// summing k in increasing order.  K-chunks of 64 columns of the row block and the matching 64
// rows of x are staged in LDS, so x is read once per RB rows rather than once per row.
constexpr int kRK = 64;
constexpr int ax_tiled_rows(int C) { return (C >= 16 ? 4 : 2) * (kRT / C); }
template <int C>
__global__ __launch_bounds__(kRT) void resid_ax_tiled_kernel(int64_t n, int64_t d, const double* __restrict__ A,
                                                             int64_t lda, const double* __restrict__ x,
                                                             double* __restrict__ zh, double* __restrict__ zl) {
  constexpr int TR = kRT / C, RB = ax_tiled_rows(C), R = RB / TR;
  __shared__ double As[RB][kRK + 1];
  __shared__ double Xs[kRK][C];
  const int t = threadIdx.x, c = t % C, tr = t / C;
  const int64_t i0 = (int64_t)blockIdx.x * RB;
  double h[R], l[R];
#pragma unroll
  for (int q = 0; q < R; ++q) h[q] = l[q] = 0.0;
  for (int64_t k0 = 0; k0 < d; k0 += kRK) {
    const int kc = (int)(d - k0 < kRK ? d - k0 : kRK);
    // row block: element e = t + 256 q -> (row e / 64, column e % 64), 512 consecutive bytes per row
    static_assert(RB * kRK % kRT == 0 && kRK * C % kRT == 0, "tiles: whole rounds of the workgroup");
#pragma unroll
    for (int q = 0; q < RB * kRK / kRT; ++q) {
      const int e = t + kRT * q, r = e / kRK, k = e % kRK;
      const int64_t i = i0 + r;
      As[r][k] = (i < n && k < kc) ? A[i * lda + k0 + k] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kRK * C / kRT; ++q) {
      const int e = t + kRT * q, k = e / C, cc = e % C;
      Xs[k][cc] = k < kc ? x[(k0 + k) * C + cc] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < kc; ++k) {
      const double xv = Xs[k][c];
#pragma unroll
      for (int q = 0; q < R; ++q) dd_fma(h[q], l[q], As[tr + TR * q][k], xv, 0.0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int64_t i = i0 + tr + TR * q;
    if (i < n) {
      zh[i * C + c] = h[q];
      zl[i * C + c] = l[q];
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

// pass 2 for C >= 8, the same sums in the same order with the operands staged in LDS: chunks of
// RC rows of the workgroup's column tile of A and of (zh, zl) are loaded with coalesced reads (all
// of a chunk's loads in flight together), then every thread runs its S accumulators over the
// chunk's rows from LDS.
template <int C>
__global__ __launch_bounds__(kRT) void resid_atz_tiled_kernel(int64_t n, int64_t d, const double* __restrict__ A,
                                                              int64_t lda, const double* __restrict__ zh,
                                                              const double* __restrict__ zl, int64_t rows,
                                                              double* __restrict__ ph, double* __restrict__ pl) {
  constexpr int J = kRT / C, S = 8, W = J * S;  // W columns of A per workgroup
  constexpr int RC = W <= 128 ? 32 : 16;        // rows per chunk
  __shared__ double As[RC][W + 1];
  __shared__ double Zs[2][RC][C];
  const int t = threadIdx.x, c = t % C, jj = t / C;
  const int64_t j0 = (int64_t)blockIdx.x * W;
  const int64_t r0 = (int64_t)blockIdx.y * rows, r1 = r0 + rows < n ? r0 + rows : n;
  double hi[S], lo[S];
#pragma unroll
  for (int s = 0; s < S; ++s) hi[s] = lo[s] = 0.0;
  for (int64_t i0 = r0; i0 < r1; i0 += RC) {
    const int rc = (int)(r1 - i0 < RC ? r1 - i0 : RC);
    static_assert(RC * W % kRT == 0, "row chunk of A: whole rounds of the workgroup");
#pragma unroll
    for (int q = 0; q < RC * W / kRT; ++q) {
      const int e = t + kRT * q, r = e / W, j = e % W;
      As[r][j] = (r < rc && j0 + j < d) ? A[(i0 + r) * lda + j0 + j] : 0.0;
    }
    for (int e = t; e < RC * C; e += kRT) {
      const int r = e / C, cc = e % C;
      Zs[0][r][cc] = r < rc ? zh[(i0 + r) * C + cc] : 0.0;
      Zs[1][r][cc] = r < rc ? zl[(i0 + r) * C + cc] : 0.0;
    }
    __syncthreads();
    // no column bound here: columns past d hold zeros in As and add nothing (their sums are never
    // stored), and a branch per accumulator would serialise the S independent chains
    for (int r = 0; r < rc; ++r) {
      const double h = Zs[0][r][c], l = Zs[1][r][c];
#pragma unroll
      for (int s = 0; s < S; ++s) dd_fma(hi[s], lo[s], As[r][jj + J * s], h, l);
    }
    __syncthreads();
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

// Single-pass form for one column (d <= 4096, rows 16-byte aligned): a workgroup of 4 waves owns
// rows r0, r0 + G, ... (G workgroups); thread t owns the columns (j 256 + t) 2 + {0, 1}, j < NCH,
// keeps x for them and its partial A^T z as pairs in registers; each row's z = A_i x is reduced
// as pairs over the wave (butterfly) and the four waves (LDS, fixed order), then
// (part_hi, part_lo)[w][j] += A_ij z_i.  A is read once.
template <int NCH>
__global__ __launch_bounds__(kRT) void resid_fused_kernel(int64_t n, int d, const double* __restrict__ A, int64_t lda,
                                                          const double* __restrict__ x, double* __restrict__ ph,
                                                          double* __restrict__ pl) {
  typedef double dv2 __attribute__((ext_vector_type(2)));
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  __shared__ double redh[2][4], redl[2][4];
  double xv[NCH][2], qh[NCH][2], ql[NCH][2];
#pragma unroll
  for (int j = 0; j < NCH; ++j)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int col = (j * kRT + tid) * 2 + e;
      xv[j][e] = col < d ? x[col] : 0.0;
      qh[j][e] = ql[j][e] = 0.0;
    }
  int buf = 0;
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const double* Ai = A + i * lda;
    dv2 a[NCH];
#pragma unroll
    for (int j = 0; j < NCH; ++j) {
      const int col = (j * kRT + tid) * 2;
      a[j] = col < d ? __builtin_nontemporal_load(reinterpret_cast<const dv2*>(Ai + col)) : dv2{0.0, 0.0};
    }
    double hi = 0.0, lo = 0.0;
#pragma unroll
    for (int j = 0; j < NCH; ++j)
#pragma unroll
      for (int e = 0; e < 2; ++e) dd_fma(hi, lo, a[j][e], xv[j][e], 0.0);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double oh = __shfl_xor(hi, off, 64), ol = __shfl_xor(lo, off, 64);
      // both partners form the same pair sum (operands ordered by lane) so every lane ends equal
      if (lane & off)
        dd_add2(oh, ol, hi, lo);
      else
        dd_add(hi, lo, oh, ol);
    }
    if (lane == 0) {
      redh[buf][wid] = hi;
      redl[buf][wid] = lo;
    }
    __syncthreads();
    double zh = redh[buf][0], zl = redl[buf][0];
#pragma unroll
    for (int w = 1; w < 4; ++w) dd_add(zh, zl, redh[buf][w], redl[buf][w]);
    buf ^= 1;
#pragma unroll
    for (int j = 0; j < NCH; ++j)
#pragma unroll
      for (int e = 0; e < 2; ++e) dd_fma(qh[j][e], ql[j][e], a[j][e], zh, zl);
  }
  const int64_t base = (int64_t)blockIdx.x * d;
#pragma unroll
  for (int j = 0; j < NCH; ++j)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int col = (j * kRT + tid) * 2 + e;
      if (col < d) {
        ph[base + col] = qh[j][e];
        pl[base + col] = ql[j][e];
      }
    }
}

}  // namespace

// Workgroups of the single-pass form (each writes a d-length partial pair).
constexpr int kResidFusedWG = 512;

bool residual_dd_fused_ok(int64_t d, int C, const double* A, int64_t lda) {
  return C == 1 && d <= 4096 && d % 2 == 0 && lda % 2 == 0 && ((uintptr_t)A & 15) == 0;
}

int resid_blocks(int num_cu, int64_t n, int64_t d, int C, int64_t* rows) {
  const int64_t tiles = ceil_div(d, (int64_t)(kRT / C) * 8);
  const int64_t want = std::max<int64_t>(1, 8 * (int64_t)num_cu / tiles);
  int64_t nrb = std::min<int64_t>(want, ceil_div(n, 64));
  nrb = std::max<int64_t>(1, nrb);
  *rows = ceil_div(n, nrb);
  return (int)ceil_div(n, *rows);
}

void launch_residual_dd(int num_cu, int64_t n, int64_t d, int C, const double* A, int64_t lda, const double* b,
                        int64_t ldb, double nu, const double* lam, const double* x, double* zh, double* zl, double* ph,
                        double* pl, double* r, int64_t ldr, hipStream_t s) {
  if (residual_dd_fused_ok(d, C, A, lda)) {
    const int nwg = (int)std::min<int64_t>(kResidFusedWG, n);
    const int nch = (int)ceil_div(d, 2 * kRT);
#define AES_RFUSED(NC)                                                                                        \
  hipLaunchKernelGGL(resid_fused_kernel<NC>, dim3(nwg), dim3(kRT), 0, s, n, (int)d, A, lda, x, ph, pl); \
  break;
    switch (nch <= 1 ? 1 : nch <= 2 ? 2 : nch <= 4 ? 4 : 8) {
      case 1:
        AES_RFUSED(1)
      case 2:
        AES_RFUSED(2)
      case 4:
        AES_RFUSED(4)
      default:
        AES_RFUSED(8)
    }
#undef AES_RFUSED
    AES_LAUNCH_CHECK();
    hipLaunchKernelGGL(resid_combine_kernel, dim3((unsigned)ceil_div(d, kRT)), dim3(kRT), 0, s, d, 1, nwg, ph, pl, b,
                       ldb, x, lam, nu, r, ldr);
    AES_LAUNCH_CHECK();
    return;
  }
  int64_t rows = 0;
  const int nrb = resid_blocks(num_cu, n, d, C, &rows);
  const unsigned g1 = (unsigned)std::min<int64_t>(ceil_div(n, kRT / 64), 8 * (int64_t)num_cu);
  const dim3 g2((unsigned)ceil_div(d, (int64_t)(kRT / C) * 8), (unsigned)nrb);
#define AES_RESID_CASE(CV)                                                                                        \
  case CV:                                                                                                        \
    if (CV >= 8)                                                                                                  \
      hipLaunchKernelGGL(resid_ax_tiled_kernel<(CV >= 8 ? CV : 8)>, dim3((unsigned)ceil_div(n, ax_tiled_rows(CV >= 8 ? CV : 8))), \
                         dim3(kRT), 0, s, n, d, A, lda, x, zh, zl);                                               \
    else                                                                                                          \
      hipLaunchKernelGGL(resid_ax_kernel<CV>, dim3(g1), dim3(kRT), 0, s, n, d, A, lda, x, zh, zl);                \
    AES_LAUNCH_CHECK();                                                                                           \
    if (CV >= 8)                                                                                                  \
      hipLaunchKernelGGL(resid_atz_tiled_kernel<(CV >= 8 ? CV : 8)>, g2, dim3(kRT), 0, s, n, d, A, lda, zh, zl, rows, \
                         ph, pl);                                                                                 \
    else                                                                                                          \
      hipLaunchKernelGGL(resid_atz_kernel<CV>, g2, dim3(kRT), 0, s, n, d, A, lda, zh, zl, rows, ph, pl);          \
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
  if (C == 1 && d <= 4096) return std::max<size_t>((size_t)kResidFusedWG * d, 1);
  int64_t rows = 0;
  const int nrb = resid_blocks(num_cu, n, d, C, &rows);
  return (size_t)nrb * d * C;
}

}  // namespace aes
