// Sparse Johnson-Lindenstrauss transform with one non-zero per column (Sec. 2.1, s = 1):
// column i of S has a single +-1 in row h_i, so row r of S A is the signed sum of the rows of A
// hashed to r.  h_i and the sign come from Philox stream SJLT (h_i = high word of w0 * m).
//
// The sum is deterministic and in increasing row order: a stable counting sort orders the
// data rows by bucket (per-block counts in bucket-major order, an exclusive scan of the counts,
// then each block places its rows ranked by index), and one streaming pass over A adds the
// rows of every bucket in that order.  A is read once, each row as whole 16-byte vectors.
// With few buckets (long segments) a bucket is cut into Q equal pieces whose partial sums are
// added in piece order by a second, small kernel.
#include <cmath>

#include "common.h"
#include "kernels.h"

namespace aes {

constexpr int kSjBlk = 1024;  // data rows per counting block
constexpr int kSjItems = 64;  // most output items (bucket pieces) per reduction workgroup
constexpr int kScanChunk = 4096;

size_t sjlt_blocks(int64_t n) { return (size_t)ceil_div(n, kSjBlk); }

__global__ void sjlt_zero_kernel(int32_t* __restrict__ p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

// code[i] = h_i | (sign bit << 31); cnt[h * nblk + block] += 1
__global__ __launch_bounds__(kSjBlk) void sjlt_hash_kernel(uint64_t k0, uint64_t k1, int64_t n, int64_t m,
                                                           int64_t nblk, int32_t* __restrict__ code,
                                                           int32_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * kSjBlk + threadIdx.x;
  if (i >= n) return;
  const Rand4 r = philox4x64_10((uint64_t)i, kStreamSjlt, 0, 0, k0, k1);
  const int64_t h = (int64_t)__umul64hi(r.w[0], (uint64_t)m);
  code[i] = (int32_t)((uint32_t)h | ((uint32_t)(r.w[1] >> 63) << 31));
  atomicAdd(&cnt[h * nblk + blockIdx.x], 1);
}

// Exclusive scan of cnt (length len) in three steps over chunks of kScanChunk elements.
__global__ __launch_bounds__(256) void sjlt_chunk_sum_kernel(const int32_t* __restrict__ cnt, int64_t len,
                                                             int32_t* __restrict__ csum) {
  __shared__ int32_t ws[4];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  int32_t s = 0;
  for (int e = threadIdx.x; e < kScanChunk; e += 256)
    if (base + e < len) s += cnt[base + e];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) csum[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ __launch_bounds__(1024) void sjlt_top_scan_kernel(int32_t* __restrict__ csum, int64_t nch) {
  __shared__ int32_t sv[1024];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nch; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int32_t a = i < nch ? csum[i] : 0;
    sv[threadIdx.x] = a;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int32_t v = threadIdx.x >= off ? sv[threadIdx.x - off] : 0;
      __syncthreads();
      sv[threadIdx.x] += v;
      __syncthreads();
    }
    if (i < nch) csum[i] = carry + sv[threadIdx.x] - a;
    __syncthreads();
    if (threadIdx.x == 1023) carry += sv[1023];
    __syncthreads();
  }
}

// Each thread scans 16 consecutive elements; the 256 thread totals are scanned in LDS.
__global__ __launch_bounds__(256) void sjlt_chunk_scan_kernel(int32_t* __restrict__ cnt, int64_t len,
                                                              const int32_t* __restrict__ csum) {
  constexpr int E = kScanChunk / 256;
  __shared__ int32_t sv[256];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * E;
  int32_t v[E];
  int32_t tot = 0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    v[e] = base + e < len ? cnt[base + e] : 0;
    tot += v[e];
  }
  sv[threadIdx.x] = tot;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int32_t a = threadIdx.x >= off ? sv[threadIdx.x - off] : 0;
    __syncthreads();
    sv[threadIdx.x] += a;
    __syncthreads();
  }
  int32_t run = csum[blockIdx.x] + sv[threadIdx.x] - tot;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (base + e < len) cnt[base + e] = run;
    run += v[e];
  }
}

// perm[off[h * nblk + block] + rank] = code with the bucket replaced by the data row, where
// rank counts the earlier rows of the same block in the same bucket (a stable placement).
__global__ __launch_bounds__(kSjBlk) void sjlt_place_kernel(const int32_t* __restrict__ code, int64_t n,
                                                            int64_t nblk, const int32_t* __restrict__ off,
                                                            int32_t* __restrict__ perm) {
  __shared__ int32_t hb[kSjBlk];
  const int t = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kSjBlk + t;
  const int32_t c = i < n ? code[i] : -1;
  const int32_t h = i < n ? (c & 0x7fffffff) : -1;
  hb[t] = h;
  __syncthreads();
  if (i >= n) return;
  int rank = 0;
  for (int u = 0; u < t; ++u) rank += hb[u] == h;
  const int64_t dst = off[(int64_t)h * nblk + blockIdx.x] + rank;
  perm[dst] = (int32_t)((uint32_t)i | ((uint32_t)c & 0x80000000u));
}

// First sorted position of output item it (bucket it / Q, piece it % Q); n past the last.
__device__ __forceinline__ int32_t sjlt_item_begin(int64_t it, int Q, int64_t m, int64_t n, int64_t nblk,
                                                   const int32_t* __restrict__ off) {
  const int64_t r = it / Q, q = it - r * Q;
  if (r >= m) return (int32_t)n;
  const int64_t bs = off[r * nblk];
  const int64_t be = r + 1 < m ? off[(r + 1) * nblk] : n;
  return (int32_t)(bs + ((be - bs) * q) / Q);
}

template <typename TO, typename TA>
__device__ __forceinline__ TO sj_cvt(TA v) {
  return (TO)v;
}
template <>
__device__ __forceinline__ __hip_bfloat16 sj_cvt<__hip_bfloat16, float>(float v) {
  return __float2bfloat16(v);
}

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  using type = double __attribute__((ext_vector_type(2)));
};
template <>
struct Vec16<float> {
  using type = float __attribute__((ext_vector_type(4)));
};

// Workgroup (blockIdx.x, blockIdx.y) adds, for the items it0 .. it0 + G - 1, the signed rows of
// their sorted ranges into columns [blockIdx.y * 256 * VE * NV, +256 * VE * NV) and writes one
// output row per item (out row it).  Thread t owns the VE-element vectors v * 256 + t (v < NV),
// so each load instruction of a wave covers 1 KiB of a row.  The items' ranges are consecutive,
// so the workgroup streams one contiguous stretch of perm, RW rows in flight per thread.
template <typename TA, typename TO, int NV>
__global__ __launch_bounds__(256) void sjlt_reduce_kernel(const TA* __restrict__ A, int64_t lda, int64_t d, int vec,
                                                          const int32_t* __restrict__ perm,
                                                          const int32_t* __restrict__ off, int64_t nblk, int64_t n,
                                                          int64_t m, int Q, int G, TO* __restrict__ out,
                                                          int64_t ldo) {
  constexpr int VE = 16 / sizeof(TA);
  constexpr int RW = 16 / NV;
  using VT = typename Vec16<TA>::type;
  __shared__ int32_t iend[kSjItems + 1];
  __shared__ int32_t pl[256];
  const int tid = threadIdx.x;
  const int64_t it0 = (int64_t)blockIdx.x * G;
  const int nit = (int)std::min<int64_t>(G, m * Q - it0);
  if (tid <= nit) iend[tid] = sjlt_item_begin(it0 + tid, Q, m, n, nblk, off);
  __syncthreads();
  int64_t c0[NV];
  bool full[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    c0[v] = (int64_t)blockIdx.y * 256 * VE * NV + (int64_t)(v * 256 + tid) * VE;
    full[v] = vec && c0[v] + VE <= d;
  }
  TA acc[NV][VE];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int e = 0; e < VE; ++e) acc[v][e] = TA(0);
  int cur = 0;
  auto flush = [&]() {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (c0[v] < d) {
        TO* o = out + (it0 + cur) * ldo + c0[v];
#pragma unroll
        for (int e = 0; e < VE; ++e)
          if (c0[v] + e < d) o[e] = sj_cvt<TO>(acc[v][e]);
      }
#pragma unroll
      for (int e = 0; e < VE; ++e) acc[v][e] = TA(0);
    }
    ++cur;
  };
  const int32_t start = iend[0], end = iend[nit];
  for (int32_t base = start; base < end; base += 256) {
    __syncthreads();
    pl[tid] = base + tid < end ? perm[base + tid] : 0;
    __syncthreads();
    const int cnt = std::min<int32_t>(256, end - base);
    for (int u0 = 0; u0 < cnt; u0 += RW) {
      TA x[RW][NV][VE];
#pragma unroll
      for (int u = 0; u < RW; ++u) {
        // (the clamp keeps a corrupted entry inside A; a valid one is always < n)
        const int64_t row = std::min<int64_t>(pl[u0 + u < cnt ? u0 + u : 0] & 0x7fffffff, n - 1);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const TA* p = A + row * lda + c0[v];
          if (u0 + u < cnt && full[v]) {
            const VT y = __builtin_nontemporal_load(reinterpret_cast<const VT*>(p));
#pragma unroll
            for (int e = 0; e < VE; ++e) x[u][v][e] = y[e];
          } else {
#pragma unroll
            for (int e = 0; e < VE; ++e) x[u][v][e] = (u0 + u < cnt && c0[v] + e < d) ? p[e] : TA(0);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < RW; ++u) {
        if (u0 + u < cnt) {
          const int32_t j = base + u0 + u;
          while (j >= iend[cur + 1]) flush();
          const bool neg = pl[u0 + u] < 0;
#pragma unroll
          for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int e = 0; e < VE; ++e) acc[v][e] += neg ? -x[u][v][e] : x[u][v][e];
        }
      }
    }
  }
  while (cur < nit) flush();
}

// out[r, c] = sum over pieces q (in order) of part[(r Q + q), c]
template <typename TA, typename TO>
__global__ __launch_bounds__(256) void sjlt_combine_kernel(const TA* __restrict__ part, int64_t d, int Q,
                                                           TO* __restrict__ out) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (c >= d) return;
  const TA* p = part + r * Q * d + c;
  TA s = TA(0);
  for (int q = 0; q < Q; ++q) s += p[q * d];
  out[r * d + c] = sj_cvt<TO>(s);
}

// Vectors per thread of a reduction workgroup: whole 16-byte vectors of up to 1024 x VE columns.
static int sjlt_nv(int64_t d, int ve) {
  const int64_t nvec = ceil_div(d, 256 * ve);
  return nvec >= 4 ? 4 : (nvec >= 2 ? 2 : 1);
}

SjltPlan sjlt_plan(int64_t n, int64_t d, int64_t m, size_t elem) {
  SjltPlan p;
  p.nblk = (int64_t)sjlt_blocks(n);
  p.Q = (int)std::max<int64_t>(1, ceil_div(n, m * 64));
  // about 256 / NV rows (256 KiB of A at d = 2048 in FP64) per workgroup
  const int64_t per_item = std::max<int64_t>(1, ceil_div(n, m * p.Q));
  const int nv = sjlt_nv(d, (int)(16 / elem));
  p.G = (int)std::min<int64_t>(kSjItems, std::max<int64_t>(1, 256 / nv / per_item));
  p.count_elems = (size_t)(m * p.nblk);
  p.csum_elems = (size_t)std::max<int64_t>(1, ceil_div(m * p.nblk, kScanChunk));
  return p;
}

template <typename TA, typename TO>
static void launch_reduce(int nv, dim3 grid, hipStream_t s, const TA* A, int64_t lda, int64_t d, int vec,
                          const SjltScratch& sc, const SjltPlan& p, int64_t n, int64_t m, TO* out) {
  if (nv == 4)
    hipLaunchKernelGGL((sjlt_reduce_kernel<TA, TO, 4>), grid, dim3(256), 0, s, A, lda, d, vec, sc.perm, sc.cnt, p.nblk,
                       n, m, p.Q, p.G, out, d);
  else if (nv == 2)
    hipLaunchKernelGGL((sjlt_reduce_kernel<TA, TO, 2>), grid, dim3(256), 0, s, A, lda, d, vec, sc.perm, sc.cnt, p.nblk,
                       n, m, p.Q, p.G, out, d);
  else
    hipLaunchKernelGGL((sjlt_reduce_kernel<TA, TO, 1>), grid, dim3(256), 0, s, A, lda, d, vec, sc.perm, sc.cnt, p.nblk,
                       n, m, p.Q, p.G, out, d);
  AES_LAUNCH_CHECK();
}

template <typename TA, typename TO>
void launch_sjlt(const SjltPlan& p, const TA* A, int64_t n, int64_t d, int64_t lda, int64_t m, uint64_t seed,
                 int32_t problem, int64_t k, TO* SA, const SjltScratch& sc, hipStream_t s) {
  const RngKey key = make_key(seed, problem, k);
  const int64_t len = m * p.nblk;
  hipLaunchKernelGGL(sjlt_zero_kernel, dim3((unsigned)ceil_div(len, 256)), dim3(256), 0, s, sc.cnt, len);
  AES_LAUNCH_CHECK();
  hipLaunchKernelGGL(sjlt_hash_kernel, dim3((unsigned)p.nblk), dim3(kSjBlk), 0, s, key.k0, key.k1, n, m, p.nblk,
                     sc.code, sc.cnt);
  AES_LAUNCH_CHECK();
  const int64_t nch = ceil_div(len, kScanChunk);
  hipLaunchKernelGGL(sjlt_chunk_sum_kernel, dim3((unsigned)nch), dim3(256), 0, s, sc.cnt, len, sc.csum);
  AES_LAUNCH_CHECK();
  hipLaunchKernelGGL(sjlt_top_scan_kernel, dim3(1), dim3(1024), 0, s, sc.csum, nch);
  AES_LAUNCH_CHECK();
  hipLaunchKernelGGL(sjlt_chunk_scan_kernel, dim3((unsigned)nch), dim3(256), 0, s, sc.cnt, len, sc.csum);
  AES_LAUNCH_CHECK();
  hipLaunchKernelGGL(sjlt_place_kernel, dim3((unsigned)p.nblk), dim3(kSjBlk), 0, s, sc.code, n, p.nblk, sc.cnt,
                     sc.perm);
  AES_LAUNCH_CHECK();
  constexpr int VE = 16 / sizeof(TA);
  const int vec = ((uintptr_t)A % 16 == 0) && lda % VE == 0;
  const int64_t items = m * p.Q;
  const int nv = sjlt_nv(d, VE);
  dim3 grid((unsigned)ceil_div(items, p.G), (unsigned)ceil_div(d, 256 * VE * nv));
  if (p.Q == 1) {
    launch_reduce(nv, grid, s, A, lda, d, vec, sc, p, n, m, SA);
  } else {
    TA* part = reinterpret_cast<TA*>(sc.part);
    launch_reduce(nv, grid, s, A, lda, d, vec, sc, p, n, m, part);
    hipLaunchKernelGGL((sjlt_combine_kernel<TA, TO>), dim3((unsigned)ceil_div(d, 256), (unsigned)m), dim3(256), 0, s,
                       part, d, p.Q, SA);
    AES_LAUNCH_CHECK();
  }
}

template void launch_sjlt<double, double>(const SjltPlan&, const double*, int64_t, int64_t, int64_t, int64_t, uint64_t,
                                          int32_t, int64_t, double*, const SjltScratch&, hipStream_t);
template void launch_sjlt<float, float>(const SjltPlan&, const float*, int64_t, int64_t, int64_t, int64_t, uint64_t,
                                        int32_t, int64_t, float*, const SjltScratch&, hipStream_t);
template void launch_sjlt<float, __hip_bfloat16>(const SjltPlan&, const float*, int64_t, int64_t, int64_t, int64_t,
                                                 uint64_t, int32_t, int64_t, __hip_bfloat16*, const SjltScratch&,
                                                 hipStream_t);

}  // namespace aes
