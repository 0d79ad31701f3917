// Fused single-pass Hessian-vector product (the per-iteration O(nd) work of Sec. 4.1):
//     z = A v (kept on chip),  q = A^T z,  s = ||z||^2
// streaming every row of A from HBM exactly once.  Each workgroup owns a slice of rows and
// keeps its partial q (d values) in registers; partials are summed in a fixed order by
// hv_colsum, which also adds nu^2 Lambda v (deterministic, no floating-point atomics).
#include "common.h"
#include "kernels.h"

namespace aes {

template <typename T, int V>
struct VecT;
template <>
struct VecT<double, 1> {
  using type = double;
};
template <>
struct VecT<double, 2> {
  using type = double __attribute__((ext_vector_type(2)));
};
template <>
struct VecT<float, 1> {
  using type = float;
};
template <>
struct VecT<float, 4> {
  using type = float __attribute__((ext_vector_type(4)));
};

// Loads VEC consecutive elements (zero beyond nvalid); they stay in the storage type TA in
// registers and are widened to FP64 where they are used.
template <typename TA, int VEC>
__device__ __forceinline__ void load_vec(const TA* __restrict__ p, bool full, int nvalid, TA (&out)[VEC]) {
  using VT = typename VecT<TA, VEC>::type;
  if constexpr (VEC == 1) {
    out[0] = full ? __builtin_nontemporal_load(p) : TA(0);
  } else {
    if (full) {
      VT v = __builtin_nontemporal_load(reinterpret_cast<const VT*>(p));
#pragma unroll
      for (int i = 0; i < VEC; ++i) out[i] = v[i];
    } else {
#pragma unroll
      for (int i = 0; i < VEC; ++i) out[i] = i < nvalid ? p[i] : TA(0);
    }
  }
}

constexpr int kHvThreads = 256;

// One workgroup = 4 waves; thread t owns columns (j*256 + t)*VEC + [0, VEC) for j < NCH.
// Each step loads ROWS rows, reduces the ROWS partial dot products across the workgroup
// (wave transpose-reduction + LDS), then accumulates q += z_r * a_r.
template <typename TA, int VEC, int NCH, int ROWS>
__global__ __launch_bounds__(kHvThreads, 2) void hv_fused_kernel(const TA* __restrict__ A, int64_t n, int d,
                                                                  int64_t lda, const double* __restrict__ v,
                                                                  double* __restrict__ part,
                                                                  double* __restrict__ spart,
                                                                  const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  constexpr int CH = kHvThreads * VEC;  // columns per chunk
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  __shared__ double red[2][4][ROWS];

  double pr[NCH][VEC], qa[NCH][VEC];
#pragma unroll
  for (int j = 0; j < NCH; ++j)
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int col = j * CH + tid * VEC + e;
      pr[j][e] = col < d ? v[col] : 0.0;
      qa[j][e] = 0.0;
    }

  double ssum = 0.0;
  int buf = 0;
  const int64_t stride = (int64_t)gridDim.x * ROWS;
  for (int64_t r0 = (int64_t)blockIdx.x * ROWS; r0 < n; r0 += stride) {
    TA a[ROWS][NCH][VEC];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      const int64_t row = r0 + r;
      const bool rok = row < n;
      const TA* rp = A + (rok ? row : 0) * lda;
#pragma unroll
      for (int j = 0; j < NCH; ++j) {
        const int col = j * CH + tid * VEC;
        const int nvalid = d - col;
        load_vec<TA, VEC>(rp + col, rok && nvalid >= VEC, rok ? nvalid : 0, a[r][j]);
      }
    }
    double dot[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < NCH; ++j)
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc = fma((double)a[r][j][e], pr[j][e], acc);
      dot[r] = acc;
    }
    wave_transpose_sum<ROWS>(dot, lane);
    constexpr int shift = 6 - ilog2_c(ROWS);
    if ((lane & ((1 << shift) - 1)) == 0) red[buf][wid][(lane >> shift) & (ROWS - 1)] = dot[0];
    __syncthreads();
    double z[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) z[r] = (red[buf][0][r] + red[buf][1][r]) + (red[buf][2][r] + red[buf][3][r]);
    buf ^= 1;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      ssum = fma(z[r], z[r], ssum);
#pragma unroll
      for (int j = 0; j < NCH; ++j)
#pragma unroll
        for (int e = 0; e < VEC; ++e) qa[j][e] = fma(z[r], (double)a[r][j][e], qa[j][e]);
    }
  }
  double* out = part + (int64_t)blockIdx.x * d;
#pragma unroll
  for (int j = 0; j < NCH; ++j)
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int col = j * CH + tid * VEC + e;
      if (col < d) out[col] = qa[j][e];
    }
  if (tid == 0) spart[blockIdx.x] = ssum;
}

int hv_num_blocks(int num_cu, int64_t n) {
  int64_t nb = (int64_t)num_cu * 2;
  const int64_t groups = ceil_div(n, 4);
  if (nb > groups) nb = groups;
  return (int)(nb < 1 ? 1 : nb);
}

template <typename TA, int VEC, int NCH, int ROWS>
static void hv_launch_cfg(const TA* A, int64_t n, int64_t d, int64_t lda, const double* v, double* part,
                          double* spart, int nwg, hipStream_t s, const int* gate) {
  hipLaunchKernelGGL((hv_fused_kernel<TA, VEC, NCH, ROWS>), dim3(nwg), dim3(kHvThreads), 0, s, A, n, (int)d, lda,
                     v, part, spart, gate);
  AES_LAUNCH_CHECK();
}

template <>
void launch_hv_fused<double>(const double* A, int64_t n, int64_t d, int64_t lda, const double* v, double* part,
                             double* spart, int nwg, hipStream_t s, const int* gate) {
  const bool v2 = (d % 2 == 0) && (lda % 2 == 0) && ((uintptr_t)A % 16 == 0);
  if (v2) {
    if (d <= 512) return hv_launch_cfg<double, 2, 1, 16>(A, n, d, lda, v, part, spart, nwg, s, gate);
    if (d <= 1024) return hv_launch_cfg<double, 2, 2, 8>(A, n, d, lda, v, part, spart, nwg, s, gate);
    if (d <= 2048) return hv_launch_cfg<double, 2, 4, 8>(A, n, d, lda, v, part, spart, nwg, s, gate);
    if (d <= 4096) return hv_launch_cfg<double, 2, 8, 2>(A, n, d, lda, v, part, spart, nwg, s, gate);
    if (d <= 8192) return hv_launch_cfg<double, 2, 16, 1>(A, n, d, lda, v, part, spart, nwg, s, gate);
  } else {
    if (d <= 256) return hv_launch_cfg<double, 1, 1, 16>(A, n, d, lda, v, part, spart, nwg, s, gate);
    if (d <= 1024) return hv_launch_cfg<double, 1, 4, 8>(A, n, d, lda, v, part, spart, nwg, s, gate);
    if (d <= 2048) return hv_launch_cfg<double, 1, 8, 4>(A, n, d, lda, v, part, spart, nwg, s, gate);
    if (d <= 4096) return hv_launch_cfg<double, 1, 16, 1>(A, n, d, lda, v, part, spart, nwg, s, gate);
    if (d <= 8192) return hv_launch_cfg<double, 1, 32, 1>(A, n, d, lda, v, part, spart, nwg, s, gate);
  }
  throw std::invalid_argument("hv_fused: d > 8192 is not supported");
}

template <>
void launch_hv_fused<float>(const float* A, int64_t n, int64_t d, int64_t lda, const double* v, double* part,
                            double* spart, int nwg, hipStream_t s, const int* gate) {
  const bool v4 = (d % 4 == 0) && (lda % 4 == 0) && ((uintptr_t)A % 16 == 0);
  if (v4) {
    if (d <= 1024) return hv_launch_cfg<float, 4, 1, 8>(A, n, d, lda, v, part, spart, nwg, s, gate);
    if (d <= 2048) return hv_launch_cfg<float, 4, 2, 8>(A, n, d, lda, v, part, spart, nwg, s, gate);
    if (d <= 4096) return hv_launch_cfg<float, 4, 4, 4>(A, n, d, lda, v, part, spart, nwg, s, gate);
    if (d <= 8192) return hv_launch_cfg<float, 4, 8, 1>(A, n, d, lda, v, part, spart, nwg, s, gate);
  } else {
    if (d <= 256) return hv_launch_cfg<float, 1, 1, 16>(A, n, d, lda, v, part, spart, nwg, s, gate);
    if (d <= 1024) return hv_launch_cfg<float, 1, 4, 8>(A, n, d, lda, v, part, spart, nwg, s, gate);
    if (d <= 2048) return hv_launch_cfg<float, 1, 8, 4>(A, n, d, lda, v, part, spart, nwg, s, gate);
    if (d <= 4096) return hv_launch_cfg<float, 1, 16, 1>(A, n, d, lda, v, part, spart, nwg, s, gate);
    if (d <= 8192) return hv_launch_cfg<float, 1, 32, 1>(A, n, d, lda, v, part, spart, nwg, s, gate);
  }
  throw std::invalid_argument("hv_fused: d > 8192 is not supported");
}

// Second pass of the two-pass H.v for problems wider than the fused kernel takes (d > 8192):
// part[w][j] = sum over the rows i of row block w, in order, of z_i A[i, j] (z = A v from the
// first pass).  Workgroup (cb, w) covers columns [2048 cb, 2048 cb + 2048) of row block w;
// thread t owns the 16-byte vectors 256 v + t (v < 4) of that column block, so every load
// instruction of a wave covers 1 KiB of a row, and keeps four rows' loads in flight.
__global__ __launch_bounds__(256) void atz_kernel(const double* __restrict__ A, int64_t n, int64_t d, int64_t lda,
                                                  int vec, const double* __restrict__ z, int64_t rows,
                                                  double* __restrict__ part) {
  typedef double d2v __attribute__((ext_vector_type(2)));
  const int tid = threadIdx.x;
  const int64_t w = blockIdx.y;
  const int64_t i0 = w * rows;
  const int64_t i1 = i0 + rows < n ? i0 + rows : n;
  int64_t c0[4];
  bool full[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    c0[v] = (int64_t)blockIdx.x * 2048 + (int64_t)(v * 256 + tid) * 2;
    full[v] = vec && c0[v] + 2 <= d;
  }
  double acc[4][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
  for (int64_t i = i0; i < i1; i += 4) {
    double x[4][4][2], zi[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t r = i + u;
      const bool ok = r < i1;
      zi[u] = ok ? z[r] : 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (ok && full[v]) {
          const d2v y = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(A + r * lda + c0[v]));
          x[u][v][0] = y[0];
          x[u][v][1] = y[1];
        } else {
#pragma unroll
          for (int e = 0; e < 2; ++e) x[u][v][e] = (ok && c0[v] + e < d) ? A[r * lda + c0[v] + e] : 0.0;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int e = 0; e < 2; ++e) acc[v][e] = fma(zi[u], x[u][v][e], acc[v][e]);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int e = 0; e < 2; ++e)
      if (c0[v] + e < d) part[w * d + c0[v] + e] = acc[v][e];
}

int atz_blocks(int num_cu, int64_t n, int64_t d, int64_t* rows) {
  const int64_t cb = ceil_div(d, 2048);
  int64_t nrb = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 4), 4 * (int64_t)num_cu / cb));
  const int64_t r = round_up(ceil_div(n, nrb), 4);
  *rows = r;
  return (int)ceil_div(n, r);
}

void launch_atz(const double* A, int64_t n, int64_t d, int64_t lda, const double* z, double* part, int nrb,
                int64_t rows, hipStream_t s) {
  const int vec = ((uintptr_t)A % 16 == 0) && (lda % 2 == 0);
  hipLaunchKernelGGL(atz_kernel, dim3((unsigned)ceil_div(d, 2048), (unsigned)nrb), dim3(256), 0, s, A, n, d, lda, vec, z,
                     rows, part);
  AES_LAUNCH_CHECK();
}

// out[j, c] = sgn * (sum_w part[w][j][c] + nu2 * lam[j] * v[j, c]) + bsgn * b[j, c]
// 256 threads = 16 (j,c)-elements x 16 partial groups; a thread keeps 8 loads in flight and
// the groups are combined in a fixed order (deterministic).
template <typename TP>
__global__ __launch_bounds__(256) void hv_colsum_kernel(const TP* __restrict__ part, int nwg, int64_t total,
                                                        int C, const double* __restrict__ v,
                                                        const double* __restrict__ lam, double nu2, double sgn,
                                                        const double* __restrict__ b, double bsgn,
                                                        double* __restrict__ out, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ double sh[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t e = (int64_t)blockIdx.x * 16 + tx;
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (e < total) {
    int w = ty;
    for (; w + 16 * 7 < nwg; w += 16 * 8) {
      TP x[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = part[(int64_t)(w + 16 * k) * total + e];
#pragma unroll
      for (int k = 0; k < 8; ++k) a[k] += (double)x[k];
    }
    for (; w < nwg; w += 16) a[0] += (double)part[(int64_t)w * total + e];
  }
  sh[ty][tx] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  __syncthreads();
  for (int st = 8; st >= 1; st >>= 1) {
    if (ty < st) sh[ty][tx] += sh[ty + st][tx];
    __syncthreads();
  }
  if (ty == 0 && e < total) {
    const double sum = sh[0][tx];
    const int64_t j = e / C;
    const double lj = lam ? lam[j] : 1.0;
    double val = sgn * (sum + nu2 * lj * v[e]);
    if (b) val += bsgn * b[e];
    out[e] = val;
  }
}

void launch_hv_colsum(const double* part, int nwg, int64_t d, int C, const double* v, const double* lam, double nu2,
                      double sgn, const double* b, double bsgn, double* out, hipStream_t s, const int* gate) {
  const int64_t total = d * C;
  hipLaunchKernelGGL(hv_colsum_kernel<double>, dim3((unsigned)ceil_div(total, 16)), dim3(256), 0, s, part, nwg, total, C,
                     v, lam, nu2, sgn, b, bsgn, out, gate);
  AES_LAUNCH_CHECK();
}

void launch_hv_colsum_f32(const float* part, int nwg, int64_t d, int C, const double* v, const double* lam, double nu2,
                          double sgn, const double* b, double bsgn, double* out, hipStream_t s) {
  const int64_t total = d * C;
  hipLaunchKernelGGL(hv_colsum_kernel<float>, dim3((unsigned)ceil_div(total, 16)), dim3(256), 0, s, part, nwg, total, C,
                     v, lam, nu2, sgn, b, bsgn, out, nullptr);
  AES_LAUNCH_CHECK();
}

// out[c] = sum_i e[i,c]^2, out[C + c] = sum_i x[i,c]^2 (one workgroup, fixed-order tree)
__global__ __launch_bounds__(1024) void colnorm2_kernel(int64_t d, int C, const double* __restrict__ e,
                                                        const double* __restrict__ x, double* __restrict__ out) {
  __shared__ double b1[1024], b2[1024];
  const int tid = threadIdx.x, col = tid % C, tpc = 1024 / C;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = tid / C; i < d; i += tpc) {
    const double u = e[i * C + col], v = x[i * C + col];
    s1 += u * u;
    s2 += v * v;
  }
  b1[tid] = s1;
  b2[tid] = s2;
  __syncthreads();
  for (int st = 512; st >= C; st >>= 1) {
    if (tid < st) {
      b1[tid] += b1[tid + st];
      b2[tid] += b2[tid + st];
    }
    __syncthreads();
  }
  if (tid < C) {
    out[tid] = b1[tid];
    out[C + tid] = b2[tid];
  }
}

void launch_colnorm2(int64_t d, int C, const double* e, const double* x, double* out, hipStream_t s) {
  hipLaunchKernelGGL(colnorm2_kernel, dim3(1), dim3(1024), 0, s, d, C, e, x, out);
  AES_LAUNCH_CHECK();
}

}  // namespace aes
