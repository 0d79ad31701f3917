// Subsampled randomized Hadamard transform S A = (1/sqrt m) R H E A_pad (Sec. 2.1, with the
// zero padding of its footnote and the sqrt(n'/m) scale of the SRHT proof section):
//   * E: Rademacher signs of Philox stream SIGN (one per data row);
//   * R: the m padded rows with the smallest 64-bit Philox ROW keys (a uniform sample without
//     replacement), kept in increasing row order.  Selected by an exact radix select of the
//     m-th smallest key (eight 8-bit digit passes) and an order-preserving compaction;
//   * H: unnormalised Sylvester Walsh-Hadamard transform of order n' = 2^L along the rows,
//     done in ceil(L / 9) passes.  A pass transforms 2^b rows that differ in b consecutive
//     index bits: the tile (2^b rows x CW columns) is staged in LDS and transformed with
//     radix-8 butterflies held in registers (one LDS round trip per 3 bits).  The first pass
//     applies E and synthesises the zero padding rows; the last pass writes only the rows in R
//     (scaled by 1/sqrt m) and skips tiles that contain none.
#include <cmath>

#include "common.h"
#include "kernels.h"

namespace aes {

__global__ void signs_kernel(uint64_t k0, uint64_t k1, int64_t n, double* __restrict__ eps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Rand4 r = philox4x64_10((uint64_t)i, kStreamSign, 0, 0, k0, k1);
  eps[i] = (r.w[0] >> 63) ? -1.0 : 1.0;
}

void launch_signs(uint64_t seed, int32_t problem, int64_t k, int64_t n, double* eps, hipStream_t s) {
  const RngKey key = make_key(seed, problem, k);
  hipLaunchKernelGGL(signs_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, key.k0, key.k1, n, eps);
  AES_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------------------
// Row selection.
// state: [0] prefix (key value being built), [1] remaining rank, [2] unused, [3] unused
// ---------------------------------------------------------------------------------------
__global__ void rowkeys_kernel(uint64_t k0, uint64_t k1, int64_t npad, uint64_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  keys[i] = philox4x64_10((uint64_t)i, kStreamRow, 0, 0, k0, k1).w[0];
}

__global__ void select_init_kernel(uint64_t* __restrict__ state, uint32_t* __restrict__ hist, int64_t m) {
  const int t = threadIdx.x;
  for (int i = t; i < 256 * 8; i += blockDim.x) hist[i] = 0;
  if (t == 0) {
    state[0] = 0;
    state[1] = (uint64_t)(m - 1);
    state[2] = 0;
    state[3] = 0;
  }
}

__global__ __launch_bounds__(256) void select_hist_kernel(const uint64_t* __restrict__ keys, int64_t npad, int pass,
                                                          const uint64_t* __restrict__ state,
                                                          uint32_t* __restrict__ hist) {
  __shared__ uint32_t lh[256];
  lh[threadIdx.x] = 0;
  __syncthreads();
  const int shift = 56 - 8 * pass;
  const uint64_t prefix = state[0];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npad; i += stride) {
    const uint64_t key = keys[i];
    const bool match = pass == 0 || (key >> (shift + 8)) == (prefix >> (shift + 8));
    if (match) atomicAdd(&lh[(key >> shift) & 255], 1u);
  }
  __syncthreads();
  const uint32_t v = lh[threadIdx.x];
  if (v) atomicAdd(&hist[pass * 256 + threadIdx.x], v);
}

__global__ __launch_bounds__(256) void select_scan_kernel(int pass, uint64_t* __restrict__ state,
                                                          const uint32_t* __restrict__ hist) {
  __shared__ uint64_t cum[256];
  const int t = threadIdx.x;
  cum[t] = hist[pass * 256 + t];
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {  // inclusive Hillis-Steele scan
    const uint64_t v = t >= off ? cum[t - off] : 0;
    __syncthreads();
    cum[t] += v;
    __syncthreads();
  }
  const uint64_t rank = state[1];
  const uint64_t before = t ? cum[t - 1] : 0;
  __syncthreads();
  if (rank >= before && rank < cum[t]) {
    const int shift = 56 - 8 * pass;
    state[0] |= (uint64_t)t << shift;
    state[1] = rank - before;
  }
}

constexpr int kSelBlk = 1024;

size_t select_blocks(int64_t npad) { return (size_t)ceil_div(npad, kSelBlk); }

__global__ __launch_bounds__(kSelBlk) void select_count_kernel(const uint64_t* __restrict__ keys, int64_t npad,
                                                               const uint64_t* __restrict__ state,
                                                               uint32_t* __restrict__ blk) {
  __shared__ uint32_t cl[16], ce[16];
  const uint64_t T = state[0];
  const int64_t i = (int64_t)blockIdx.x * kSelBlk + threadIdx.x;
  const uint64_t key = i < npad ? keys[i] : ~0ull;
  const bool less = i < npad && key < T;
  const bool eq = i < npad && key == T;
  const uint64_t bl = __ballot(less), be = __ballot(eq);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    cl[w] = (uint32_t)__popcll(bl);
    ce[w] = (uint32_t)__popcll(be);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = 0, b = 0;
    for (int k = 0; k < kSelBlk / 64; ++k) {
      a += cl[k];
      b += ce[k];
    }
    blk[2 * blockIdx.x] = a;
    blk[2 * blockIdx.x + 1] = b;
  }
}

// Exclusive scan of the per-block (less, equal) counts (single workgroup, sequential chunks).
__global__ __launch_bounds__(1024) void select_blkscan_kernel(uint32_t* __restrict__ blk, int64_t nblk) {
  __shared__ uint32_t sa[1024], sb[1024];
  __shared__ uint32_t carry_a, carry_b;
  if (threadIdx.x == 0) {
    carry_a = 0;
    carry_b = 0;
  }
  __syncthreads();
  for (int64_t base = 0; base < nblk; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const uint32_t a = i < nblk ? blk[2 * i] : 0, b = i < nblk ? blk[2 * i + 1] : 0;
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const uint32_t va = threadIdx.x >= off ? sa[threadIdx.x - off] : 0;
      const uint32_t vb = threadIdx.x >= off ? sb[threadIdx.x - off] : 0;
      __syncthreads();
      sa[threadIdx.x] += va;
      sb[threadIdx.x] += vb;
      __syncthreads();
    }
    if (i < nblk) {
      blk[2 * i] = carry_a + sa[threadIdx.x] - a;
      blk[2 * i + 1] = carry_b + sb[threadIdx.x] - b;
    }
    __syncthreads();
    if (threadIdx.x == 1023) {
      carry_a += sa[1023];
      carry_b += sb[1023];
    }
    __syncthreads();
  }
}

// pos[i] = rank of padded row i in R (ascending row order) or -1.
__global__ __launch_bounds__(kSelBlk) void select_write_kernel(const uint64_t* __restrict__ keys, int64_t npad,
                                                               const uint64_t* __restrict__ state,
                                                               const uint32_t* __restrict__ blk,
                                                               int32_t* __restrict__ pos) {
  __shared__ uint32_t cl[16], ce[16];
  const uint64_t T = state[0];
  const uint64_t need = state[1] + 1;  // keys equal to T that are taken, in index order
  const int64_t i = (int64_t)blockIdx.x * kSelBlk + threadIdx.x;
  const uint64_t key = i < npad ? keys[i] : ~0ull;
  const bool less = i < npad && key < T;
  const bool eq = i < npad && key == T;
  const uint64_t bl = __ballot(less), be = __ballot(eq);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  if (lane == 0) {
    cl[w] = (uint32_t)__popcll(bl);
    ce[w] = (uint32_t)__popcll(be);
  }
  __syncthreads();
  uint32_t less_before = blk[2 * blockIdx.x], eq_before = blk[2 * blockIdx.x + 1];
  for (int k = 0; k < w; ++k) {
    less_before += cl[k];
    eq_before += ce[k];
  }
  less_before += (uint32_t)__popcll(bl & lt);
  eq_before += (uint32_t)__popcll(be & lt);
  if (i >= npad) return;
  int32_t p = -1;
  const uint64_t eqt = eq_before < need ? eq_before : need;
  if (less) p = (int32_t)(less_before + eqt);
  else if (eq && eq_before < need) p = (int32_t)(less_before + eq_before);
  pos[i] = p;
}

void launch_srht_select(uint64_t seed, int32_t problem, int64_t k, int64_t npad, int64_t m, const SelectScratch& sc,
                        hipStream_t s) {
  const RngKey key = make_key(seed, problem, k);
  hipLaunchKernelGGL(rowkeys_kernel, dim3((unsigned)ceil_div(npad, 256)), dim3(256), 0, s, key.k0, key.k1, npad, sc.keys);
  AES_LAUNCH_CHECK();
  hipLaunchKernelGGL(select_init_kernel, dim3(1), dim3(256), 0, s, sc.state, sc.hist, m);
  AES_LAUNCH_CHECK();
  int64_t hb = ceil_div(npad, 256 * 8);
  if (hb > 1024) hb = 1024;
  if (hb < 1) hb = 1;
  for (int pass = 0; pass < 8; ++pass) {
    hipLaunchKernelGGL(select_hist_kernel, dim3((unsigned)hb), dim3(256), 0, s, sc.keys, npad, pass, sc.state, sc.hist);
    AES_LAUNCH_CHECK();
    hipLaunchKernelGGL(select_scan_kernel, dim3(1), dim3(256), 0, s, pass, sc.state, sc.hist);
    AES_LAUNCH_CHECK();
  }
  const int64_t nblk = (int64_t)select_blocks(npad);
  hipLaunchKernelGGL(select_count_kernel, dim3((unsigned)nblk), dim3(kSelBlk), 0, s, sc.keys, npad, sc.state, sc.blk);
  AES_LAUNCH_CHECK();
  hipLaunchKernelGGL(select_blkscan_kernel, dim3(1), dim3(1024), 0, s, sc.blk, nblk);
  AES_LAUNCH_CHECK();
  hipLaunchKernelGGL(select_write_kernel, dim3((unsigned)nblk), dim3(kSelBlk), 0, s, sc.keys, npad, sc.state, sc.blk,
                     sc.pos);
  AES_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------------------
// Walsh-Hadamard passes.
// ---------------------------------------------------------------------------------------
template <typename T>
struct AccOf {
  using type = float;
};
template <>
struct AccOf<double> {
  using type = double;
};

template <typename TO, typename TA>
__device__ __forceinline__ TO cvt(TA v) {
  return (TO)v;
}
template <>
__device__ __forceinline__ __hip_bfloat16 cvt<__hip_bfloat16, float>(float v) {
  return __float2bfloat16(v);
}
template <>
__device__ __forceinline__ float cvt<float, __hip_bfloat16>(__hip_bfloat16 v) {
  return __bfloat162float(v);
}

constexpr int kMaxTileBits = 9;

// In-register Walsh-Hadamard of 2^NB values: v[q] for q < 2^NB.
template <typename TACC, int NB>
__device__ __forceinline__ void wht_reg(TACC (&v)[1 << NB]) {
#pragma unroll
  for (int h = 1; h < (1 << NB); h <<= 1)
#pragma unroll
    for (int q = 0; q < (1 << NB); ++q)
      if ((q & h) == 0) {
        const TACC a = v[q], b = v[q | h];
        v[q] = a + b;
        v[q | h] = a - b;
      }
}

template <typename TACC, int NB, int CW>
__device__ __forceinline__ void wht_group(TACC* tile, int R, int g, int tid) {
  // units: (R >> NB) index groups x (CW / VW) column vectors of 16 bytes
  constexpr int VW = 16 / sizeof(TACC);
  typedef TACC VT __attribute__((ext_vector_type(VW)));
  constexpr int CV = CW / VW;
  const int units = (R >> NB) * CV;
  for (int u = tid; u < units; u += 256) {
    const int c = (u % CV) * VW;
    const int jj = u / CV;
    const int j0 = ((jj >> g) << (g + NB)) | (jj & ((1 << g) - 1));
    VT v[1 << NB];
#pragma unroll
    for (int q = 0; q < (1 << NB); ++q) v[q] = *reinterpret_cast<const VT*>(&tile[(j0 + (q << g)) * CW + c]);
#pragma unroll
    for (int h = 1; h < (1 << NB); h <<= 1)
#pragma unroll
      for (int q = 0; q < (1 << NB); ++q)
        if ((q & h) == 0) {
          const VT x = v[q], y = v[q | h];
          v[q] = x + y;
          v[q | h] = x - y;
        }
#pragma unroll
    for (int q = 0; q < (1 << NB); ++q) *reinterpret_cast<VT*>(&tile[(j0 + (q << g)) * CW + c]) = v[q];
  }
}

// Radix-2^NB butterflies over v[q] at runtime NB (1..3), in the fixed bit order h = 1, 2, 4.
template <typename VT>
__device__ __forceinline__ void wht_reg_n(VT (&v)[8], int nb) {
  if (nb == 3) {
#pragma unroll
    for (int h = 1; h < 8; h <<= 1)
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if ((q & h) == 0) {
          const VT x = v[q], y = v[q | h];
          v[q] = x + y;
          v[q | h] = x - y;
        }
  } else if (nb == 2) {
#pragma unroll
    for (int h = 1; h < 4; h <<= 1)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if ((q & h) == 0) {
          const VT x = v[q], y = v[q | h];
          v[q] = x + y;
          v[q | h] = x - y;
        }
  } else if (nb == 1) {
    const VT x = v[0], y = v[1];
    v[0] = x + y;
    v[1] = x - y;
  }
}

// Radix-16 butterflies over v[q], in the fixed bit order h = 1, 2, 4, 8.
template <typename VT>
__device__ __forceinline__ void wht_reg16(VT (&v)[16]) {
#pragma unroll
  for (int h = 1; h < 16; h <<= 1)
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if ((q & h) == 0) {
        const VT x = v[q], y = v[q | h];
        v[q] = x + y;
        v[q | h] = x - y;
      }
}

// One WHT pass over index bits [s, s+b).  MODE: 0 first pass (src = A with signs, rows >= n
// are zero, dst = Y; tiles past n are skipped), 1 middle pass (Y -> Y), 2 last pass (Y -> SA,
// rows selected by pos, scale), 3 single pass (A -> SA).
// zero_bits > 0 (middle/last pass directly after the first): rows whose first-pass tile starts
// at or beyond n are known zero and not read.
// A thread moves VW consecutive columns (16 bytes of the accumulation type) of 2^nf rows: the
// lowest nf <= 3 tile bits are transformed in registers right after the loads, the highest
// nl <= 3 bits in registers right before the stores, and only the bits between take LDS
// round trips (3 bits each).  NF = 4 (b = 8 exactly): the low four bits after the loads and the
// high four before the stores, sixteen rows per thread each time, so the tile crosses LDS once.
template <typename TIN, typename TY, typename TOUT, int CW, int MODE, int NF>
__global__ __launch_bounds__(256) void wht_pass_kernel(const TIN* __restrict__ A, const TY* __restrict__ Ysrc,
                                                       TY* __restrict__ Ydst, TOUT* __restrict__ SA, int64_t ldsa,
                                                       int64_t n, int64_t d, int64_t lda, int64_t npad, int s, int b,
                                                       int zero_bits, const double* __restrict__ eps,
                                                       const int32_t* __restrict__ pos, double scale,
                                                       int a_aligned, const int32_t* __restrict__ need,
                                                       int check_tiles, int pw, int yperm) {
  using TACC = typename AccOf<TY>::type;
  // Y is stored in column panels of pw columns: element (row, col) at
  // (col / pw) * npad * pw + row * pw + col % pw, so that the strided tiles of the later passes
  // read rows of one panel rather than rows n' * 8 bytes apart
  const int pws = __builtin_ctz((unsigned)pw);  // pw is a power of two
  // yperm > 0 (two passes, the first over the low yperm index bits): a row is stored at its index
  // with the two bit fields swapped, so that a tile of the last pass (rows differing in the high
  // bits) is one contiguous block of the panel and the first pass writes with the stride instead
  const int lbits = __builtin_ctzll((unsigned long long)npad);
  auto ypos = [&](int64_t row, int64_t col) {
    if (yperm > 0) row = ((row & ((1ll << yperm) - 1)) << (lbits - yperm)) | (row >> yperm);
    return (((col >> pws) * npad + row) << pws) + (col & (int64_t)(pw - 1));
  };
  constexpr int VW = 16 / sizeof(TACC);  // columns per vector access
  constexpr int TPR = CW / VW;           // threads per row segment
  static_assert(NF != 4 || TPR == 16, "the radix-16 path maps 256 threads onto 16 x 16 units");
  if (NF == 4 && b != 8) return;  // launched only for 8-bit passes
  typedef TACC VT __attribute__((ext_vector_type(VW)));
  extern __shared__ unsigned char smem_raw[];
  TACC* tile = reinterpret_cast<TACC*>(smem_raw);
  const int tid = threadIdx.x;
  const int R = 1 << b;
  const int nf = NF == 4 ? 4 : (b < 3 ? b : 3);
  const int nl = NF == 4 ? 4 : ((b - nf) < 3 ? (b - nf) : 3);
  const int GF = 1 << nf, GL = 1 << nl;
  // column block fastest: concurrently resident workgroups cover whole rows of A / Y
  const int64_t tile_id = blockIdx.y;
  const int64_t lo = tile_id & ((1ll << s) - 1);
  const int64_t hi = tile_id >> s;
  const int64_t base = (hi << (s + b)) | lo;
  const int64_t c0 = (int64_t)blockIdx.x * CW;
  constexpr bool FIRST = MODE == 0 || MODE == 3;
  constexpr bool LAST = MODE == 2 || MODE == 3;

  if (MODE == 0 && base >= n) return;  // all-padding tile: implicit zeros
  // per-row flags of the tile kept in LDS: output row (last pass) or "needed" (pruned first pass)
  __shared__ int32_t rowflag[1 << kMaxTileBits];
  // last pass: with a sparse sample (check_tiles) the tile's rows are looked up first and a
  // tile without a selected row is skipped; with a dense one every tile has selected rows and
  // the lookups travel with the data loads (R <= 512: two rows per thread)
  int32_t pf0 = -1, pf1 = -1;
  if (LAST && check_tiles) {
    int found = 0;
    for (int j = tid; j < R; j += 256) {
      const int32_t pr = pos[base + ((int64_t)j << s)];
      rowflag[j] = pr;
      found |= pr >= 0;
    }
    if (!__syncthreads_or(found)) return;  // no selected row in this tile
  } else if (LAST) {
    if (tid < R) pf0 = pos[base + ((int64_t)tid << s)];
    if (tid + 256 < R) pf1 = pos[base + ((int64_t)(tid + 256) << s)];
  } else if (MODE == 0 && need) {
    for (int j = tid; j < R; j += 256) rowflag[j] = need[j];
  }
  const bool vec_in =
      ((d % VW) == 0) && (!FIRST || ((lda % VW) == 0 && sizeof(TIN) == sizeof(TACC) && a_aligned));
  // ---- load + first nf bits: unit u = (row group jg of GF rows, column vector) --------------
  // All loads of a batch (2 units x 8 rows of 16 bytes, with their signs) are issued before
  // any of them is consumed, so that a workgroup keeps its tile in flight.
  const int units_in = (R / GF) * TPR;
  if constexpr (NF == 4) {
    // one unit per thread: 16 rows j0 .. j0 + 15 of one column vector (units_in = 256)
    const int u = tid;
    const int cv = (u % TPR) * VW, j0 = (u / TPR) * 16;
    const int64_t col = c0 + cv;
    VT v[16];
    TACC sg[16];
    // every load of the unit is issued before any is used (the branch on vec_in sits outside
    // the row loops, so no row's load waits on another's use)
    if (vec_in) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int64_t row = base + ((int64_t)(j0 + q) << s);
        bool load = col < d;
        if (FIRST) load = load && row < n;
        else load = load && !(zero_bits > 0 && ((row >> zero_bits) << zero_bits) >= n);
        sg[q] = TACC(1);
        if (load) {
          if (FIRST) {
            v[q] = __builtin_nontemporal_load(
                reinterpret_cast<const VT*>(reinterpret_cast<const TACC*>(A) + row * lda + col));
            sg[q] = (TACC)eps[row];
          } else {
            v[q] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(Ysrc + ypos(row, col)));
          }
        } else {
#pragma unroll
          for (int e = 0; e < VW; ++e) v[q][e] = TACC(0);
        }
      }
    } else {
      for (int q = 0; q < 16; ++q) {
        const int64_t row = base + ((int64_t)(j0 + q) << s);
        bool load = true;
        if (FIRST) load = row < n;
        else load = !(zero_bits > 0 && ((row >> zero_bits) << zero_bits) >= n);
        sg[q] = TACC(1);
#pragma unroll
        for (int e = 0; e < VW; ++e) {
          TACC x = TACC(0);
          if (load && col + e < d) x = FIRST ? cvt<TACC>(A[row * lda + col + e]) : (TACC)Ysrc[ypos(row, col + e)];
          v[q][e] = x;
        }
        if (FIRST && load) sg[q] = (TACC)eps[row];
      }
    }
    if (FIRST) {
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = v[q] * sg[q];
    }
    wht_reg16(v);
#pragma unroll
    for (int q = 0; q < 16; ++q) *reinterpret_cast<VT*>(&tile[(j0 + q) * CW + cv]) = v[q];
  } else
  for (int u0 = 0; u0 < units_in; u0 += 256 * 2) {
    VT v[2][8];
    TACC sg[2][8];
    if (vec_in) {
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        const int u = u0 + tid + 256 * w;
        const int cv = (u % TPR) * VW, j0 = (u / TPR) * GF;
        const int64_t col = c0 + cv;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int64_t row = base + ((int64_t)(j0 + q) << s);
          bool load = q < GF && u < units_in && col < d;
          if (FIRST) load = load && row < n;
          else load = load && !(zero_bits > 0 && ((row >> zero_bits) << zero_bits) >= n);
          sg[w][q] = TACC(1);
          if (load) {
            if (FIRST) {
              v[w][q] = __builtin_nontemporal_load(
                  reinterpret_cast<const VT*>(reinterpret_cast<const TACC*>(A) + row * lda + col));
              sg[w][q] = (TACC)eps[row];
            } else {
              v[w][q] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(Ysrc + ypos(row, col)));
            }
          } else {
#pragma unroll
            for (int e = 0; e < VW; ++e) v[w][q][e] = TACC(0);
          }
        }
      }
    } else {
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        const int u = u0 + tid + 256 * w;
        const int cv = (u % TPR) * VW, j0 = (u / TPR) * GF;
        const int64_t col = c0 + cv;
        for (int q = 0; q < 8; ++q) {
          const int64_t row = base + ((int64_t)(j0 + q) << s);
          bool load = q < GF && u < units_in;
          if (FIRST) load = load && row < n;
          else load = load && !(zero_bits > 0 && ((row >> zero_bits) << zero_bits) >= n);
          sg[w][q] = TACC(1);
#pragma unroll
          for (int e = 0; e < VW; ++e) {
            TACC x = TACC(0);
            if (load && col + e < d) x = FIRST ? cvt<TACC>(A[row * lda + col + e]) : (TACC)Ysrc[ypos(row, col + e)];
            v[w][q][e] = x;
          }
          if (FIRST && load) sg[w][q] = (TACC)eps[row];
        }
      }
    }
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const int u = u0 + tid + 256 * w;
      if (u >= units_in) continue;
      if (FIRST) {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[w][q] = v[w][q] * sg[w][q];
      }
      wht_reg_n(v[w], nf);
      const int cv = (u % TPR) * VW, j0 = (u / TPR) * GF;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < GF) *reinterpret_cast<VT*>(&tile[(j0 + q) * CW + cv]) = v[w][q];
    }
  }
  if (LAST && !check_tiles) {
    if (tid < R) rowflag[tid] = pf0;
    if (tid + 256 < R) rowflag[tid + 256] = pf1;
  }
  __syncthreads();
  // ---- middle bits in LDS ---------------------------------------------------------------------
  for (int g = nf; g < b - nl; g += 3) {
    const int nb = (b - nl - g) >= 3 ? 3 : (b - nl - g);
    if (nb == 3) wht_group<TACC, 3, CW>(tile, R, g, tid);
    else if (nb == 2) wht_group<TACC, 2, CW>(tile, R, g, tid);
    else wht_group<TACC, 1, CW>(tile, R, g, tid);
    __syncthreads();
  }
  // ---- last nl bits + store: unit u = (row jl below bit b - nl, column vector) ---------------
  const int rl = R / GL;  // rows jl + q * rl, q < GL, form one group
  const int units_out = rl * TPR;
  if constexpr (NF == 4) {
    // one unit per thread: rows jl + 16 q (q < 16) of one column vector (units_out = 256)
    const int u = tid;
    const int cv = (u % TPR) * VW, jl = u / TPR;
    const int64_t col = c0 + cv;
    VT v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = *reinterpret_cast<const VT*>(&tile[(jl + q * 16) * CW + cv]);
    wht_reg16(v);
    if (col < d) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int j = jl + q * 16;
        const int64_t row = base + ((int64_t)j << s);
        if (LAST) {
          const int32_t pr = rowflag[j];
          if (pr < 0) continue;
#pragma unroll
          for (int e = 0; e < VW; ++e)
            if (col + e < d) {
              if constexpr (sizeof(TACC) == 8)
                SA[(int64_t)pr * ldsa + col + e] = (TOUT)(v[q][e] * scale);
              else
                SA[(int64_t)pr * ldsa + col + e] = cvt<TOUT>((float)(v[q][e] * (float)scale));
            }
        } else {
          if (MODE == 0 && need && !rowflag[j]) continue;
          if ((d % VW) == 0) {
            __builtin_nontemporal_store(v[q], reinterpret_cast<VT*>(Ydst + ypos(row, col)));
          } else {
#pragma unroll
            for (int e = 0; e < VW; ++e)
              if (col + e < d) Ydst[ypos(row, col + e)] = (TY)v[q][e];
          }
        }
      }
    }
    return;
  }
  for (int u = tid; u < units_out; u += 256) {
    const int cv = (u % TPR) * VW, jl = u / TPR;
    const int64_t col = c0 + cv;
    VT v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (q < GL) v[q] = *reinterpret_cast<const VT*>(&tile[(jl + q * rl) * CW + cv]);
    wht_reg_n(v, nl);
    if (col >= d) continue;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q >= GL) continue;
      const int j = jl + q * rl;
      const int64_t row = base + ((int64_t)j << s);
      if (LAST) {
        const int32_t pr = rowflag[j];
        if (pr < 0) continue;
#pragma unroll
        for (int e = 0; e < VW; ++e)
          if (col + e < d) {
            if constexpr (sizeof(TACC) == 8)
              SA[(int64_t)pr * ldsa + col + e] = (TOUT)(v[q][e] * scale);
            else
              SA[(int64_t)pr * ldsa + col + e] = cvt<TOUT>((float)(v[q][e] * (float)scale));
          }
      } else {
        if (MODE == 0 && need && !rowflag[j]) continue;  // no sampled row has these low index bits
        if ((d % VW) == 0) {
          __builtin_nontemporal_store(v[q], reinterpret_cast<VT*>(Ydst + ypos(row, col)));
        } else {
#pragma unroll
          for (int e = 0; e < VW; ++e)
            if (col + e < d) Ydst[ypos(row, col + e)] = (TY)v[q][e];
        }
      }
    }
  }
}

template <typename TIN, typename TY, typename TOUT, int CW, int MODE, int NF>
static void wht_launch_cw(int64_t npad, size_t shmem, hipStream_t st, const TIN* A, const TY* Ysrc, TY* Ydst, TOUT* SA,
                          int64_t ldsa, int64_t n, int64_t d, int64_t lda, int s, int b, int zero_bits,
                          const double* eps, const int32_t* pos, double scale, const int32_t* need,
                          int check_tiles, int pw, int yperm) {
  const int a_aligned = ((uintptr_t)A % 16) == 0;
  const dim3 grid((unsigned)ceil_div(d, CW), (unsigned)(npad >> b));
  hipLaunchKernelGGL((wht_pass_kernel<TIN, TY, TOUT, CW, MODE, NF>), grid, dim3(256), shmem, st, A, Ysrc, Ydst, SA, ldsa, n,
                     d, lda, npad, s, b, zero_bits, eps, pos, scale, a_aligned, need, check_tiles, pw, yperm);
  AES_LAUNCH_CHECK();
}

// Tile of 2^b rows x CW columns within 64 KB of LDS: 256-byte row segments for b <= 8,
// 128-byte segments for b = 9.
template <typename TIN, typename TY, typename TOUT, int MODE>
static void wht_launch(int64_t npad, hipStream_t st, const TIN* A, const TY* Ysrc, TY* Ydst, TOUT* SA, int64_t ldsa,
                       int64_t n, int64_t d, int64_t lda, int s, int b, int zero_bits, const double* eps,
                       const int32_t* pos, double scale, const int32_t* need, int check_tiles, int pw,
                       int yperm) {
  using TACC = typename AccOf<TY>::type;
  constexpr int CW_WIDE = 256 / sizeof(TACC), CW_NARROW = 128 / sizeof(TACC);
  // the radix-16 register path (one LDS crossing) measured faster for the last pass and for a
  // pruned first pass; a first pass that writes all of Y is faster with the radix-8 path
  const bool r16 = b == 8 && (MODE == 2 || (MODE == 0 && need != nullptr));
  if (r16)
    wht_launch_cw<TIN, TY, TOUT, CW_WIDE, MODE, 4>(npad, (size_t)(1 << b) * CW_WIDE * sizeof(TACC), st, A, Ysrc, Ydst,
                                                   SA, ldsa, n, d, lda, s, b, zero_bits, eps, pos, scale, need,
                                                   check_tiles, pw, yperm);
  else if (b <= 8)
    wht_launch_cw<TIN, TY, TOUT, CW_WIDE, MODE, 3>(npad, (size_t)(1 << b) * CW_WIDE * sizeof(TACC), st, A, Ysrc, Ydst,
                                                   SA, ldsa, n, d, lda, s, b, zero_bits, eps, pos, scale, need,
                                                   check_tiles, pw, yperm);
  else
    wht_launch_cw<TIN, TY, TOUT, CW_NARROW, MODE, 3>(npad, (size_t)(1 << b) * CW_NARROW * sizeof(TACC), st, A, Ysrc, Ydst,
                                                  SA, ldsa, n, d, lda, s, b, zero_bits, eps, pos, scale, need,
                                                  check_tiles, pw, yperm);
}

size_t srht_scratch_elems(int64_t npad, int64_t d) { return (size_t)npad * (size_t)round_up(d, 64); }

// need[j] = 1 if some sampled padded row has low index bits j (j < R0).
__global__ void need_mask_kernel(const int32_t* __restrict__ pos, int64_t npad, int R0, int32_t* __restrict__ need) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < npad && pos[i] >= 0) need[i & (R0 - 1)] = 1;
}

__global__ void zero_i32_kernel(int32_t* p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

template <typename TIN, typename TY, typename TOUT>
void launch_srht_apply(const TIN* A, int64_t n, int64_t d, int64_t lda, const double* eps, int64_t npad,
                       const int32_t* pos, int64_t m, TY* Y, TOUT* SA, int64_t ldsa, int32_t* need, hipStream_t st) {
  int L = 0;
  while ((1ll << L) < npad) ++L;
  constexpr int kBits = 9;  // at most 9 index bits per pass
  const int passes = L == 0 ? 1 : (L + kBits - 1) / kBits;
  const double scale = 1.0 / std::sqrt((double)m);
  // a tile of the last pass has 2^b rows; with at least 16 sampled rows per 1024 padded rows
  // (m >= n'/64) empty tiles are rare enough that checking for them costs more than it saves
  const int check_tiles = m * 64 < npad;
  // panel width of Y: the column block of the narrowest pass (passes have at most 8 bits
  // unless L > 16)
  using TACC = typename AccOf<TY>::type;
  const int pw = (passes > 1 && (L + passes - 1) / passes > 8) ? 128 / (int)sizeof(TACC) : 256 / (int)sizeof(TACC);
  const int yperm = passes == 2 ? (L + 1) / 2 : 0;
  int s = 0;
  int first_bits = 0;
  for (int p = 0; p < passes; ++p) {
    const int remaining = L - s;
    const int left = passes - p;
    const int b = (remaining + left - 1) / left;
    const int zero_bits = (p == 1) ? first_bits : 0;
    if (passes == 1) {
      wht_launch<TIN, TY, TOUT, 3>(npad, st, A, (const TY*)nullptr, (TY*)nullptr, SA, ldsa, n, d, lda, s, b, 0, eps, pos,
                                   scale, nullptr, check_tiles, pw, 0);
    } else if (p == 0) {
      const int32_t* nd = nullptr;
      if (passes == 2 && need && m <= (1ll << b) / 2) {
        const int R0 = 1 << b;
        hipLaunchKernelGGL(zero_i32_kernel, dim3((unsigned)ceil_div(R0, 256)), dim3(256), 0, st, need, R0);
        AES_LAUNCH_CHECK();
        hipLaunchKernelGGL(need_mask_kernel, dim3((unsigned)ceil_div(npad, 256)), dim3(256), 0, st, pos, npad, R0, need);
        AES_LAUNCH_CHECK();
        nd = need;
      }
      wht_launch<TIN, TY, TOUT, 0>(npad, st, A, (const TY*)nullptr, Y, SA, ldsa, n, d, lda, s, b, 0, eps, pos, scale,
                                   nd, 0, pw, yperm);
      first_bits = b;
    } else if (p == passes - 1) {
      wht_launch<TIN, TY, TOUT, 2>(npad, st, A, (const TY*)Y, (TY*)nullptr, SA, ldsa, n, d, lda, s, b, zero_bits, eps,
                                   pos, scale, nullptr, check_tiles, pw, yperm);
    } else {
      wht_launch<TIN, TY, TOUT, 1>(npad, st, A, (const TY*)Y, Y, SA, ldsa, n, d, lda, s, b, zero_bits, eps, pos, scale,
                                   nullptr, 0, pw, yperm);
    }
    s += b;
  }
}

template void launch_srht_apply<double, double, double>(const double*, int64_t, int64_t, int64_t, const double*, int64_t,
                                                        const int32_t*, int64_t, double*, double*, int64_t, int32_t*,
                                                        hipStream_t);
template void launch_srht_apply<float, float, float>(const float*, int64_t, int64_t, int64_t, const double*, int64_t,
                                                     const int32_t*, int64_t, float*, float*, int64_t, int32_t*,
                                                     hipStream_t);
template void launch_srht_apply<float, float, __hip_bfloat16>(const float*, int64_t, int64_t, int64_t, const double*,
                                                              int64_t, const int32_t*, int64_t, float*, __hip_bfloat16*,
                                                              int64_t, int32_t*, hipStream_t);

// ---------------------------------------------------------------------------------------
// Transform-reuse SRHT: SA[pos[i], :] = scale * Y[i, :] for the padded rows i with
// pos[i] >= 0 (Y is the stored normalised transform, npad x d, ld d).  One wave per padded row,
// four 8-byte loads in flight per lane.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gather_rows_kernel(int64_t npad, int64_t d, const double* __restrict__ Y,
                                                          const int32_t* __restrict__ pos, double scale,
                                                          double* __restrict__ SA, int64_t ldsa) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < npad; i += nwaves) {
    const int32_t r = pos[i];
    if (r < 0) continue;
    const double* src = Y + i * d;
    double* dst = SA + (int64_t)r * ldsa;
    int64_t j = lane;
    for (; j + 3 * 64 < d; j += 4 * 64) {
      double v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = src[j + 64 * k];
#pragma unroll
      for (int k = 0; k < 4; ++k) dst[j + 64 * k] = v[k] * scale;
    }
    for (; j < d; j += 64) dst[j] = src[j] * scale;
  }
}

void launch_gather_rows(int64_t npad, int64_t d, const double* Y, const int32_t* pos, double scale, double* SA,
                        int64_t ldsa, hipStream_t s) {
  if (npad <= 0 || d <= 0) return;
  int64_t blocks = ceil_div(npad, 4);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, s, npad, d, Y, pos, scale, SA, ldsa);
  AES_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------------------
// Nested SRHT: the key order of the padded rows.  A bucket sort on the top log2(npad) bits of
// the row key (uniform keys: about one per bucket): count per bucket, exclusive scan of the
// counts, scatter (integer atomics hand out the slots of a bucket in any order), then each
// bucket is insertion-sorted by (key, row), so the result does not depend on that order.
// ---------------------------------------------------------------------------------------
constexpr int kScanBlk = 1024;

size_t keyorder_sum_elems(int64_t npad) { return (size_t)ceil_div(npad, kScanBlk); }

__device__ __forceinline__ int64_t key_bucket(uint64_t key, int shift) {
  return shift >= 64 ? 0 : (int64_t)(key >> shift);
}

__global__ void keyorder_zero_kernel(int64_t npad, uint32_t* __restrict__ cnt, uint32_t* __restrict__ cur) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  cnt[i] = 0;
  cur[i] = 0;
}

__global__ void keyorder_count_kernel(const uint64_t* __restrict__ keys, int64_t npad, int shift,
                                      uint32_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  atomicAdd(&cnt[key_bucket(keys[i], shift)], 1u);
}

// off[i] = exclusive prefix of cnt within its block of kScanBlk; bsum[block] = the block's total
__global__ __launch_bounds__(kScanBlk) void keyorder_scan_block_kernel(const uint32_t* __restrict__ cnt, int64_t npad,
                                                                       uint32_t* __restrict__ off,
                                                                       uint32_t* __restrict__ bsum) {
  __shared__ uint32_t sv[kScanBlk];
  const int t = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kScanBlk + t;
  const uint32_t v = i < npad ? cnt[i] : 0u;
  sv[t] = v;
  __syncthreads();
  for (int o = 1; o < kScanBlk; o <<= 1) {
    const uint32_t a = t >= o ? sv[t - o] : 0u;
    __syncthreads();
    sv[t] += a;
    __syncthreads();
  }
  if (i < npad) off[i] = sv[t] - v;
  if (t == kScanBlk - 1) bsum[blockIdx.x] = sv[t];
}

// exclusive scan of the block totals in place (one workgroup, chunks of kScanBlk in order)
__global__ __launch_bounds__(kScanBlk) void keyorder_scan_sums_kernel(uint32_t* __restrict__ bsum, int64_t nb) {
  __shared__ uint32_t sv[kScanBlk];
  __shared__ uint32_t carry;
  const int t = threadIdx.x;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += kScanBlk) {
    const int64_t i = base + t;
    const uint32_t v = i < nb ? bsum[i] : 0u;
    sv[t] = v;
    __syncthreads();
    for (int o = 1; o < kScanBlk; o <<= 1) {
      const uint32_t a = t >= o ? sv[t - o] : 0u;
      __syncthreads();
      sv[t] += a;
      __syncthreads();
    }
    if (i < nb) bsum[i] = carry + sv[t] - v;
    __syncthreads();
    if (t == kScanBlk - 1) carry += sv[t];
    __syncthreads();
  }
}

__global__ void keyorder_scatter_kernel(const uint64_t* __restrict__ keys, int64_t npad, int shift,
                                        uint32_t* __restrict__ off, const uint32_t* __restrict__ bsum,
                                        uint32_t* __restrict__ cur, uint64_t* __restrict__ skey,
                                        int32_t* __restrict__ order) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  const uint64_t key = keys[i];
  const int64_t b = key_bucket(key, shift);
  const int64_t slot = (int64_t)off[b] + bsum[b / kScanBlk] + atomicAdd(&cur[b], 1u);
  skey[slot] = key;
  order[slot] = (int32_t)i;
}

// one thread per bucket: insertion sort of its slots by (key, row)
__global__ void keyorder_bucket_kernel(int64_t npad, const uint32_t* __restrict__ cnt,
                                       const uint32_t* __restrict__ off, const uint32_t* __restrict__ bsum,
                                       uint64_t* __restrict__ skey, int32_t* __restrict__ order) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= npad) return;
  const uint32_t len = cnt[b];
  if (len < 2) return;
  const int64_t base = (int64_t)off[b] + bsum[b / kScanBlk];
  for (uint32_t j = 1; j < len; ++j) {
    const uint64_t k = skey[base + j];
    const int32_t r = order[base + j];
    uint32_t q = j;
    while (q > 0) {
      const uint64_t kp = skey[base + q - 1];
      const int32_t rp = order[base + q - 1];
      if (kp < k || (kp == k && rp < r)) break;
      skey[base + q] = kp;
      order[base + q] = rp;
      --q;
    }
    skey[base + q] = k;
    order[base + q] = r;
  }
}

void launch_srht_key_order(uint64_t seed, int32_t problem, int64_t npad, const KeyOrderScratch& sc, int32_t* order,
                           hipStream_t s) {
  if (npad <= 0) return;
  const RngKey key = make_key(seed, problem, 0);
  const int shift = 64 - __builtin_ctzll((unsigned long long)npad);
  const unsigned g = (unsigned)ceil_div(npad, 256);
  const int64_t nb = ceil_div(npad, kScanBlk);
  hipLaunchKernelGGL(rowkeys_kernel, dim3(g), dim3(256), 0, s, key.k0, key.k1, npad, sc.keys);
  AES_LAUNCH_CHECK();
  hipLaunchKernelGGL(keyorder_zero_kernel, dim3(g), dim3(256), 0, s, npad, sc.cnt, sc.cur);
  AES_LAUNCH_CHECK();
  hipLaunchKernelGGL(keyorder_count_kernel, dim3(g), dim3(256), 0, s, sc.keys, npad, shift, sc.cnt);
  AES_LAUNCH_CHECK();
  hipLaunchKernelGGL(keyorder_scan_block_kernel, dim3((unsigned)nb), dim3(kScanBlk), 0, s, sc.cnt, npad, sc.off,
                     sc.bsum);
  AES_LAUNCH_CHECK();
  hipLaunchKernelGGL(keyorder_scan_sums_kernel, dim3(1), dim3(kScanBlk), 0, s, sc.bsum, nb);
  AES_LAUNCH_CHECK();
  hipLaunchKernelGGL(keyorder_scatter_kernel, dim3(g), dim3(256), 0, s, sc.keys, npad, shift, sc.off, sc.bsum, sc.cur,
                     sc.skey, order);
  AES_LAUNCH_CHECK();
  hipLaunchKernelGGL(keyorder_bucket_kernel, dim3(g), dim3(256), 0, s, npad, sc.cnt, sc.off, sc.bsum, sc.skey, order);
  AES_LAUNCH_CHECK();
}

// SA[r, :] = scale * Y[order[r], :] for r < m: one wave per output row, four 8-byte loads in
// flight per lane.
__global__ __launch_bounds__(256) void gather_ordered_kernel(int64_t m, int64_t d, const double* __restrict__ Y,
                                                             const int32_t* __restrict__ order, double scale,
                                                             double* __restrict__ SA, int64_t ldsa) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t r = wave; r < m; r += nwaves) {
    const double* src = Y + (int64_t)order[r] * d;
    double* dst = SA + r * ldsa;
    int64_t j = lane;
    for (; j + 3 * 64 < d; j += 4 * 64) {
      double v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = src[j + 64 * k];
#pragma unroll
      for (int k = 0; k < 4; ++k) dst[j + 64 * k] = v[k] * scale;
    }
    for (; j < d; j += 64) dst[j] = src[j] * scale;
  }
}

void launch_gather_ordered(int64_t m, int64_t d, const double* Y, const int32_t* order, double scale, double* SA,
                           int64_t ldsa, hipStream_t s) {
  if (m <= 0 || d <= 0) return;
  int64_t blocks = ceil_div(m, 4);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(gather_ordered_kernel, dim3((unsigned)blocks), dim3(256), 0, s, m, d, Y, order, scale, SA, ldsa);
  AES_LAUNCH_CHECK();
}

}  // namespace aes
