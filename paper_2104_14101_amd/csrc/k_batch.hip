// Grouped kernels of the batched step: every launch covers all problems of a batch (the
// matrix-variable solves of Sec. 5, many problems at once).  A problem takes part in a step
// when the host has set its run flag for the step and its device gate is open (set by the
// initialisation after a factorisation and by an accepted step's finish).
//
// Per step, for every active problem (C right-hand sides, Algorithm 2 / Algorithm 1):
//   prep:     VT = P^T (PCG direction; IHS: the candidate XP) in the type of the stored A,
//   H.P:      per-range partials of A^T (A P), each A tile read from HBM once (fused form), or
//             Z = A P then A^T Z (two-pass form, wide d),
//   colsum:   Q = sum of the partials + nu^2 Lambda P (IHS: RP = H XP - rhs),
//   candidate / apply (H_S^{-1} by the inverted factors, both branches of Sec. 4.1) / finish
//   (improvement test, commit, stop rule), then the flag blocks for the host.
//
// MFMA operand layout on gfx950 for v_mfma_{f32,f64}_16x16x4: lane l supplies A[l % 16][k = l / 16]
// and B[k = l / 16][l % 16]; the output row of register r is 4 (l / 16) + r for FP32 and
// l / 16 + 4 r for FP64, the column l % 16.  The reduction index k of a product may be permuted
// freely as long as both operands use the same permutation: lane group g = l / 16 takes the VW
// consecutive columns k0 + VW g .. k0 + VW g + VW - 1 over VW consecutive MFMA steps, so every
// operand is one 16-byte load.
#include <cmath>

#include "batch.h"
#include "common.h"
#include "kernels.h"
#include "vec_device.h"

namespace aes {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double dv2 __attribute__((ext_vector_type(2)));

template <typename T>
struct BMma;
template <>
struct BMma<float> {
  typedef f4 acc_t;
  typedef f4 vec_t;  // one 16-byte load
  static constexpr int VW = 4;
  __device__ __forceinline__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct BMma<double> {
  typedef d4 acc_t;
  typedef dv2 vec_t;
  static constexpr int VW = 2;
  __device__ __forceinline__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

__device__ __forceinline__ bool brun(const BProb& P, const BDyn& D) { return D.run != 0 && *P.gate != 0; }

constexpr int kR = 16;       // rows of A per block of the fused H.P
constexpr int kFT = 512;     // threads of the fused H.P (8 waves, two per SIMD: 256 VGPRs each)
constexpr int kZLD = 32;     // row length of the LDS copies of Z

template <typename T>
constexpr int lds_pad() {
  return sizeof(T) == 4 ? 4 : 2;  // row stride = 16 bytes mod 256: conflict-free 16-byte column reads
}
constexpr int kKG = 4;       // K-groups of the first product (waves (nb, kg) = (w & 1, w >> 1))

}  // namespace

size_t bhp_smem_bytes(bool fp64, int mb) {
  const size_t es = fp64 ? 8 : 4;
  const int ld = 256 * mb + (fp64 ? 2 : 4);
  return es * ((size_t)kR * ld + (size_t)kKG * kR * kZLD);
}

int bhp_fused_max_mb(bool fp64) { return fp64 ? 4 : 8; }

// Column-block class of a problem in the fused form (7 runs as 8: its 256-VGPR budget spills).
int bhp_fused_mb(bool fp64, int64_t d) {
  int mb = (int)((d + 255) / 256);
  if (!fp64 && mb == 7) mb = 8;
  return mb;
}

// ---------------------------------------------------------------------------------------
// prep: VT[n][k] = (T) V[k][n] for n < C, k < d; zero for n in [C, 16) and k in [d, kpad).
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void bprep_kernel(const BProb* __restrict__ probs, const BDyn* __restrict__ dyn,
                                                    bool ihs) {
  const BProb& P = probs[blockIdx.y];
  if (!brun(P, dyn[blockIdx.y])) return;
  const int C = P.C, NC = C < 16 ? 16 : C;
  const int64_t total = (int64_t)NC * P.kpad;
  const double* V = ihs ? P.XP : P.P;
  T* VT = static_cast<T*>(P.VT);
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int n = (int)(e / P.kpad);
    const int64_t k = e - (int64_t)n * P.kpad;
    VT[e] = (n < C && k < P.d) ? (T)V[k * C + n] : (T)0;
  }
}

template <typename T>
void launch_bprep(const BProb* probs, const BDyn* dyn, int nprob, int64_t max_elems, bool ihs, hipStream_t s) {
  const unsigned gx = (unsigned)std::min<int64_t>(64, ceil_div(max_elems, 256));
  hipLaunchKernelGGL(bprep_kernel<T>, dim3(gx, (unsigned)nprob), dim3(256), 0, s, probs, dyn, ihs);
  AES_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------------------
// Fused H.P: a workgroup owns a range of rows of one problem and accumulates the partial
// A_range^T (A_range P) (d x NC) in registers over blocks of 16 rows.  Each block of A is read
// from HBM once into LDS (through registers, the next block's loads in flight during the
// current block's products), then
//   stage 1: Z = A_blk P (16 x NC): waves (nb, kg) form partial products over K-groups of the
//            columns, summed in LDS in a fixed order;
//   stage 2: Q_w += A_blk[:, cols_w]^T Z: wave w owns 32 MB columns of A (rows of Q).
// d <= 256 MB; columns beyond d and rows beyond the range are zero in LDS.
// ---------------------------------------------------------------------------------------
template <typename T, int MB>
__global__ __launch_bounds__(kFT) void bhp_fused_kernel(const BProb* __restrict__ probs, const BDyn* __restrict__ dyn,
                                                        const BWork* __restrict__ work) {
  typedef BMma<T> M;
  typedef typename M::acc_t acc_t;
  typedef typename M::vec_t vec_t;
  constexpr int VW = M::VW;
  constexpr int KW = 256 * MB;              // columns held per block
  constexpr int LD = KW + lds_pad<T>();     // LDS row stride (elements)
  constexpr int KG = kKG;
  constexpr int KS = KW / KG;               // stage-1 columns per K-group
  constexpr int MW = 2 * MB;                // 16-column blocks of Q per wave
  constexpr int NV = kR * KW / VW / kFT;    // 16-byte vectors per thread per block
  static_assert(NV * VW * kFT == kR * KW, "block does not divide among the threads");
  const BWork wk = work[blockIdx.x];
  const BProb& P = probs[wk.p];
  if (!brun(P, dyn[wk.p])) return;
  __shared__ __align__(16) T As[kR * LD];       // [kR][LD]
  __shared__ __align__(16) T Zr[KG * kR * kZLD]; // [KG][kR][kZLD]; Zr[0] doubles as Z
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int C = P.C, NB = C > 16 ? 2 : 1;
  const int64_t d = P.d, lda = P.lda;
  const T* A = static_cast<const T*>(P.A);
  const T* VT = static_cast<const T*>(P.VT);
  const int64_t r0 = (int64_t)wk.r * P.rows;
  const int64_t r1 = r0 + P.rows < P.n ? r0 + P.rows : P.n;

  acc_t acc[MW][2];
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  // The host routes a problem here only when every row of A starts 16-byte aligned and d is a
  // multiple of the vector width, so each 16-byte vector lies wholly inside or outside [0, d).
  vec_t pf[NV];
  auto load_block = [&](int64_t b0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int f = tid + v * kFT;
      const int row = f / (KW / VW);
      const int64_t col = (int64_t)(f - row * (KW / VW)) * VW;
      const int64_t gr = b0 + row;
      vec_t x;
#pragma unroll
      for (int e = 0; e < VW; ++e) x[e] = 0;
      if (gr < r1 && col < d) x = __builtin_nontemporal_load(reinterpret_cast<const vec_t*>(A + gr * lda + col));
      pf[v] = x;
    }
  };
  auto store_block = [&]() {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int f = tid + v * kFT;
      const int row = f / (KW / VW);
      const int col = (f - row * (KW / VW)) * VW;
      *reinterpret_cast<vec_t*>(As + row * LD + col) = pf[v];
    }
  };

  if (r0 < r1) load_block(r0);
  for (int64_t b0 = r0; b0 < r1; b0 += kR) {
    __syncthreads();  // the previous block's stage 2 is done with As
    store_block();
    __syncthreads();
    if (b0 + kR < r1) load_block(b0 + kR);  // next block in flight during this block's products
    // ---- stage 1: Z partials over K-groups ----
    const int nb = w & 1, kg = w >> 1;
    if (kg < KG && nb < NB) {
      acc_t z;
#pragma unroll
      for (int r = 0; r < 4; ++r) z[r] = 0;
      const T* arow = As + l16 * LD + kg * KS + VW * g;
      const T* vrow = VT + (int64_t)(nb * 16 + l16) * P.kpad + kg * KS + VW * g;
#pragma unroll 2
      for (int k0 = 0; k0 < KS; k0 += 4 * VW) {
        const vec_t a = *reinterpret_cast<const vec_t*>(arow + k0);
        const vec_t b = *reinterpret_cast<const vec_t*>(vrow + k0);
#pragma unroll
        for (int e = 0; e < VW; ++e) z = M::mma(a[e], b[e], z);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) Zr[(kg * kR + M::row(lane, r)) * kZLD + nb * 16 + l16] = z[r];
    }
    __syncthreads();
    if (tid < kR * kZLD) {
      T s = Zr[tid];
#pragma unroll
      for (int q = 1; q < KG; ++q) s += Zr[q * kR * kZLD + tid];
      Zr[tid] = s;
    }
    __syncthreads();
    // ---- stage 2: Q_w += A_blk[:, cols_w]^T Z ----
#pragma unroll 1
    for (int s = 0; s < 4; ++s) {
      const int k = 4 * g + s;  // row of the block taken by lane group g at step s
      T bz[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) bz[j] = Zr[k * kZLD + j * 16 + l16];
#pragma unroll
      for (int i = 0; i < MW; ++i) {
        const T a = As[k * LD + (w * MW + i) * 16 + l16];
        acc[i][0] = M::mma(a, bz[0], acc[i][0]);
        if (NB > 1) acc[i][1] = M::mma(a, bz[1], acc[i][1]);
      }
    }
  }
  // ---- write the range's partial (rows j < d, columns n < C) ----
  T* part = static_cast<T*>(P.part) + (int64_t)wk.r * d * C;
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (j >= NB) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t col = (int64_t)(w * MW + i) * 16 + M::row(lane, r);
        const int n = j * 16 + l16;
        if (col < d && n < C) part[col * C + n] = acc[i][j][r];
      }
    }
}

template <typename T>
void launch_bhp_fused(const BProb* probs, const BDyn* dyn, const BWork* work, int nwork, int mb, hipStream_t s) {
  if (nwork <= 0) return;
#define AES_BHP_CASE(MBV)                                                                              \
  case MBV:                                                                                            \
    hipLaunchKernelGGL((bhp_fused_kernel<T, MBV>), dim3(nwork), dim3(kFT), 0, s, probs, dyn, work); \
    break;
  switch (mb) {
    AES_BHP_CASE(1)
    AES_BHP_CASE(2)
    AES_BHP_CASE(3)
    AES_BHP_CASE(4)
    default:
      if constexpr (sizeof(T) == 4) {
        switch (mb) {
          AES_BHP_CASE(5)
          AES_BHP_CASE(6)
          AES_BHP_CASE(8)
          default:
            throw std::invalid_argument("fused H.P: bad column-block count");
        }
      } else {
        throw std::invalid_argument("fused FP64 H.P takes d <= 1024");
      }
  }
#undef AES_BHP_CASE
  AES_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------------------
// Two-pass H.P (d beyond the fused form): Z = A P (work item: 64 rows), then per-range partials
// A_range^T Z_range (work item: row range r and a tile of 64 columns, packed as
// r * ceil(d / 64) + tile).  Four waves of 16 rows / columns each, NB blocks of 16 columns of P.
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void bz_kernel(const BProb* __restrict__ probs, const BDyn* __restrict__ dyn,
                                                 const BWork* __restrict__ work) {
  typedef BMma<T> M;
  typedef typename M::acc_t acc_t;
  typedef typename M::vec_t vec_t;
  constexpr int VW = M::VW;
  const BWork wk = work[blockIdx.x];
  const BProb& P = probs[wk.p];
  if (!brun(P, dyn[wk.p])) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int C = P.C, NB = C > 16 ? 2 : 1, NC = C < 16 ? 16 : C;
  const int64_t d = P.d, lda = P.lda;
  const T* A = static_cast<const T*>(P.A);
  const T* VT = static_cast<const T*>(P.VT);
  T* Z = static_cast<T*>(P.Z);
  const int64_t row = (int64_t)wk.r * 64 + w * 16 + l16;
  const bool vec_ok = (lda % VW == 0) && (d % VW == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  acc_t acc[2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[j][r] = 0;
  const T* arow = A + (row < P.n ? row : 0) * lda;
  for (int64_t k0 = 0; k0 < d; k0 += 4 * VW) {
    const int64_t kc = k0 + VW * g;
    vec_t a;
#pragma unroll
    for (int e = 0; e < VW; ++e) a[e] = 0;
    if (row < P.n) {
      if (vec_ok && kc + VW <= d) {
        a = *reinterpret_cast<const vec_t*>(arow + kc);
      } else {
#pragma unroll
        for (int e = 0; e < VW; ++e)
          if (kc + e < d) a[e] = arow[kc + e];
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (j >= NB) continue;
      const vec_t b = *reinterpret_cast<const vec_t*>(VT + (int64_t)(j * 16 + l16) * P.kpad + kc);
#pragma unroll
      for (int e = 0; e < VW; ++e) acc[j] = M::mma(a[e], b[e], acc[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (j >= NB) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = (int64_t)wk.r * 64 + w * 16 + M::row(lane, r);
      if (i < P.n) Z[i * NC + j * 16 + l16] = acc[j][r];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void batz_kernel(const BProb* __restrict__ probs, const BDyn* __restrict__ dyn,
                                                   const BWork* __restrict__ work) {
  typedef BMma<T> M;
  typedef typename M::acc_t acc_t;
  const BWork wk = work[blockIdx.x];
  const BProb& P = probs[wk.p];
  if (!brun(P, dyn[wk.p])) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int C = P.C, NB = C > 16 ? 2 : 1, NC = C < 16 ? 16 : C;
  const int64_t d = P.d, lda = P.lda;
  const int64_t tiles = (d + 63) / 64;
  const int64_t rr = wk.r / tiles, tile = wk.r - rr * tiles;
  const int64_t r0 = rr * P.rows, r1 = r0 + P.rows < P.n ? r0 + P.rows : P.n;
  const int64_t col = tile * 64 + w * 16 + l16;
  const T* A = static_cast<const T*>(P.A);
  const T* Z = static_cast<const T*>(P.Z);
  acc_t acc[2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[j][r] = 0;
  for (int64_t k0 = r0; k0 < r1; k0 += 4) {
    const int64_t k = k0 + g;
    const T a = (k < r1 && col < d) ? A[k * lda + col] : (T)0;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (j >= NB) continue;
      const T b = k < r1 ? Z[k * NC + j * 16 + l16] : (T)0;
      acc[j] = M::mma(a, b, acc[j]);
    }
  }
  T* part = static_cast<T*>(P.part) + rr * d * C;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (j >= NB) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t c = tile * 64 + w * 16 + M::row(lane, r);
      const int n = j * 16 + l16;
      if (c < d && n < C) part[c * C + n] = acc[j][r];
    }
  }
}

template <typename T>
void launch_bhp_twopass(const BProb* probs, const BDyn* dyn, const BWork* ztiles, int nz, const BWork* atiles, int na,
                        hipStream_t s) {
  if (nz > 0) {
    hipLaunchKernelGGL(bz_kernel<T>, dim3(nz), dim3(256), 0, s, probs, dyn, ztiles);
    AES_LAUNCH_CHECK();
  }
  if (na > 0) {
    hipLaunchKernelGGL(batz_kernel<T>, dim3(na), dim3(256), 0, s, probs, dyn, atiles);
    AES_LAUNCH_CHECK();
  }
}

// ---------------------------------------------------------------------------------------
// colsum: out = sum_{w < nrb} part[w] (fixed order, FP64) + nu^2 lam .* v;  PCG: Q = H P;
// IHS: RP = H XP - rhs.
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void bcolsum_kernel(const BProb* __restrict__ probs, const BDyn* __restrict__ dyn,
                                                      bool ihs) {
  const BProb& P = probs[blockIdx.y];
  if (!brun(P, dyn[blockIdx.y])) return;
  const int C = P.C;
  const int64_t total = P.d * C;
  const T* part = static_cast<const T*>(P.part);
  const double* v = ihs ? P.XP : P.P;
  double* out = ihs ? P.RP : P.Q;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    double s = 0.0;
    for (int w = 0; w < P.nrb; ++w) s += (double)part[(int64_t)w * total + e];
    const int64_t j = e / C;
    s += P.nu2 * P.lam[j] * v[e];
    if (ihs) s -= P.rhs[e];
    out[e] = s;
  }
}

template <typename T>
void launch_bcolsum(const BProb* probs, const BDyn* dyn, int nprob, int64_t max_elems, bool ihs, hipStream_t s) {
  const unsigned gx = (unsigned)std::min<int64_t>(128, ceil_div(max_elems, 256));
  hipLaunchKernelGGL(bcolsum_kernel<T>, dim3(gx, (unsigned)nprob), dim3(256), 0, s, probs, dyn, ihs);
  AES_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------------------
// Candidates (one workgroup of 1024 threads per problem).
//   PCG (and CG): pHp = p . q per column, alpha = D / pHp, xp = x + alpha p, rp = r - alpha q.
//   IHS: xp = x - mu s; Polyak-IHS: xp = (x - mu s) + beta (x - x_prev), x saved as the next
//   step's previous iterate (buffers alternating with the step parity).
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kVT) void bcandidate_kernel(const BProb* __restrict__ probs,
                                                         const BDyn* __restrict__ dyn, int method) {
  const BProb& P = probs[blockIdx.x];
  const BDyn& D = dyn[blockIdx.x];
  if (!brun(P, D)) return;
  const int C = P.C, tid = threadIdx.x, col = tid % C, tpc = kVT / C;
  const int64_t d = P.d;
  const int* active = P.active;
  if (method == 1 || method == 3) {
    const bool polyak = method == 3;
    const double* xprev = polyak ? (D.parity ? P.xpv1 : P.xpv0) : nullptr;
    double* xsave = polyak ? (D.parity ? P.xpv0 : P.xpv1) : nullptr;
    for (int64_t e = tid; e < d * C; e += kVT) {
      const double xe = P.X[e];
      double v = xe;
      if (active[e % C]) {
        v = xe - P.mu * P.P[e];
        if (xprev) v += P.beta * (xe - xprev[e]);
      }
      P.XP[e] = v;
      if (xsave) xsave[e] = xe;
    }
    return;
  }
  __shared__ double buf[kVT];
  __shared__ double alpha_s[64];
  double loc = 0.0;
#pragma unroll 4
  for (int64_t i = tid / C; i < d; i += tpc) loc += P.P[i * C + col] * P.Q[i * C + col];
  col_reduce(buf, loc, C);
  if (tid < C) {
    const double pHp = buf[tid];
    P.scal[5 * C + tid] = pHp;
    const double a = active[tid] ? P.scal[tid] / pHp : 0.0;
    P.scal[2 * C + tid] = a;
    alpha_s[tid] = a;
  }
  __syncthreads();
  const double a = alpha_s[col];
  if (active[col])
#pragma unroll 4
    for (int64_t i = tid / C; i < d; i += tpc) {
      const int64_t e = i * C + col;
      P.XP[e] = P.X[e] + a * P.P[e];
      P.RP[e] = P.R[e] - a * P.Q[e];
    }
}

void launch_bcandidate(const BProb* probs, const BDyn* dyn, int nprob, int method, hipStream_t s) {
  hipLaunchKernelGGL(bcandidate_kernel, dim3((unsigned)nprob), dim3(kVT), 0, s, probs, dyn, method);
  AES_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------------------
// Preconditioner product of slot `slot` (FP64 MFMA): y = (ysgn Mat[tri] (xs .* in) + zadd) .* rs * gs,
// work item: 64 output rows of one problem (four waves of 16 rows).
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void bapply_kernel(const BProb* __restrict__ probs, const BDyn* __restrict__ dyn,
                                                     const BWork* __restrict__ work, int slot) {
  typedef BMma<double> M;
  const BWork wk = work[blockIdx.x];
  const BProb& P = probs[wk.p];
  const BDyn& D = dyn[wk.p];
  if (!brun(P, D)) return;
  const BProd& pr = D.prod[slot];
  const int64_t m0 = (int64_t)wk.r * 64;
  if (pr.rows <= 0 || m0 >= pr.rows) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int C = P.C, NB = C > 16 ? 2 : 1;
  const int64_t K = pr.K, ld = pr.ld;
  const int64_t row = m0 + w * 16 + l16;
  const bool rok = row < pr.rows;
  int64_t klo = 0, khi = K;
  if (pr.tri == 1) khi = m0 + 64 < K ? m0 + 64 : K;
  if (pr.tri == 2) klo = (m0 / 8) * 8;
  const double* mrow = pr.mat + (rok ? row : 0) * ld;
  const bool vec_ok = (ld % 2 == 0) && ((reinterpret_cast<uintptr_t>(pr.mat) & 15) == 0);
  d4 acc[2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[j][r] = 0.0;
  for (int64_t k0 = klo; k0 < khi; k0 += 8) {
    const int64_t kc = k0 + 2 * g;
    dv2 a = {0.0, 0.0};
    if (rok) {
      if (vec_ok && kc + 2 <= K) {
        a = *reinterpret_cast<const dv2*>(mrow + kc);
      } else {
        if (kc < K) a[0] = mrow[kc];
        if (kc + 1 < K) a[1] = mrow[kc + 1];
      }
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int64_t k = kc + e;
        const bool keep = k < K && (pr.tri == 0 || (pr.tri == 1 ? k <= row : k >= row));
        if (!keep) a[e] = 0.0;
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (j >= NB) continue;
      const int n = j * 16 + l16;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int64_t k = kc + e;
        double b = 0.0;
        if (k < K && n < C) {
          b = pr.in[k * C + n];
          if (pr.xs) b *= pr.xs[k];
        }
        acc[j] = M::mma(a[e], b, acc[j]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (j >= NB) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = m0 + w * 16 + M::row(lane, r);
      const int n = j * 16 + l16;
      if (i < pr.rows && n < C) {
        double y = pr.ysgn * acc[j][r];
        if (pr.zadd) y += pr.zadd[i * C + n];
        if (pr.rs) y *= pr.rs[i];
        pr.out[i * C + n] = y * pr.gs;
      }
    }
  }
}

void launch_bapply(const BProb* probs, const BDyn* dyn, const BWork* tiles, int ntiles, int slot, hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(bapply_kernel, dim3((unsigned)ntiles), dim3(256), 0, s, probs, dyn, tiles, slot);
  AES_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------------------
// Finish (one workgroup per problem): decrement of the candidate, improvement test of
// Algorithm 2 / Algorithm 1 (log domain), commit if accepted, stop rule per column; the gate
// stays open iff the step was accepted, is finite and a column is still active.
// ---------------------------------------------------------------------------------------
template <bool IHS>
__global__ __launch_bounds__(kVT) void bfinish_kernel(const BProb* __restrict__ probs, const BDyn* __restrict__ dyn) {
  const BProb& P = probs[blockIdx.x];
  const BDyn& D = dyn[blockIdx.x];
  if (!brun(P, D)) return;
  __shared__ double buf[kVT];
  __shared__ double dp_s[64], xn_s[64], rz_s[64];
  __shared__ int accept_s;
  const int C = P.C, tid = threadIdx.x, col = tid % C, tpc = kVT / C;
  const int64_t d = P.d;
  int* active = P.active;
  double* scal = P.scal;
  const bool act = active[col] != 0;
  double l1 = 0.0, l2 = 0.0, l3 = 0.0;
  if (act)
#pragma unroll 4
    for (int64_t i = tid / C; i < d; i += tpc) {
      const int64_t e = i * C + col;
      l1 += P.RP[e] * P.RTP[e];
      l2 += P.XP[e] * P.XP[e];
      l3 += fabs(P.RP[e]);
    }
  col_reduce(buf, l1, C);
  if (tid < C) dp_s[tid] = IHS ? 0.5 * buf[tid] : buf[tid];
  __syncthreads();
  col_reduce(buf, l2, C);
  if (tid < C) xn_s[tid] = buf[tid];
  __syncthreads();
  col_reduce(buf, l3, C);
  if (tid < C) rz_s[tid] = buf[tid];
  __syncthreads();
  if (tid == 0) {
    double* fl = scal + 7 * C;
    bool fail = D.force != 0;
    bool nonfinite = false;
    double maxlr = -INFINITY;
    for (int c = 0; c < C; ++c) {
      if (!active[c]) continue;
      const double Dp = dp_s[c];
      const double a = IHS ? 1.0 : scal[2 * C + c];
      if (!isfinite(Dp) || !isfinite(a)) nonfinite = true;
      const double lr = Dp > 0.0 ? log(Dp) - log(scal[C + c]) : -INFINITY;
      scal[3 * C + c] = Dp;
      scal[6 * C + c] = lr;
      if (lr > maxlr) maxlr = lr;
      if (lr > D.thr) fail = true;
    }
    const bool accept = !nonfinite && (!fail || !P.adaptive || D.at_cap);
    fl[0] = fail ? 1.0 : 0.0;
    fl[2] = nonfinite ? 1.0 : 0.0;
    fl[3] = accept ? 1.0 : 0.0;
    fl[4] = maxlr;
    fl[7] = D.seq;
    accept_s = accept;
  }
  __syncthreads();
  if (!accept_s) {
    if (tid == 0) {
      int na = 0;
      for (int c = 0; c < C; ++c) na += active[c] != 0;
      scal[7 * C + 1] = (double)na;
      *P.gate = 0;
    }
    return;
  }
  if (act) {
    const double beta = IHS ? 0.0 : dp_s[col] / scal[col];
#pragma unroll 4
    for (int64_t i = tid / C; i < d; i += tpc) {
      const int64_t e = i * C + col;
      P.X[e] = P.XP[e];
      P.R[e] = P.RP[e];
      P.P[e] = IHS ? P.RTP[e] : P.RTP[e] + beta * P.P[e];
    }
  }
  __syncthreads();
  if (tid == 0) {
    int na = 0;
    double maxD = 0.0;
    for (int c = 0; c < C; ++c) {
      if (active[c]) {
        const double Dp = dp_s[c];
        scal[c] = Dp;
        const double Df = IHS ? 2.0 * Dp : Dp;
        const double D0f = IHS ? 2.0 * scal[4 * C + c] : scal[4 * C + c];
        if (stop_test(P.stop_rule, Df, D0f, xn_s[c], rz_s[c] == 0.0, D.stop_scale, P.stop_sr, P.tol2)) active[c] = 0;
      }
      na += active[c] != 0;
      if (scal[c] > maxD) maxD = scal[c];
    }
    scal[7 * C + 1] = (double)na;
    scal[7 * C + 5] = maxD;
    *P.gate = na > 0 ? 1 : 0;
  }
}

// Flag blocks of the problems that took part in the step (whether the step ran or their
// initialisation had closed the gate) into the packed host-read array.
__global__ void bflags_kernel(const BProb* __restrict__ probs, const BDyn* __restrict__ dyn, int nprob) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob || !dyn[p].run) return;
  const BProb& P = probs[p];
  if (!P.scal || !P.flags_out) return;  // a problem whose set-up failed
  for (int i = 0; i < 8; ++i) P.flags_out[i] = P.scal[7 * P.C + i];
}

void launch_bfinish(const BProb* probs, const BDyn* dyn, int nprob, bool ihs, hipStream_t s) {
  if (ihs)
    hipLaunchKernelGGL(bfinish_kernel<true>, dim3((unsigned)nprob), dim3(kVT), 0, s, probs, dyn);
  else
    hipLaunchKernelGGL(bfinish_kernel<false>, dim3((unsigned)nprob), dim3(kVT), 0, s, probs, dyn);
  AES_LAUNCH_CHECK();
  hipLaunchKernelGGL(bflags_kernel, dim3((unsigned)ceil_div(nprob, 64)), dim3(64), 0, s, probs, dyn, nprob);
  AES_LAUNCH_CHECK();
}

template void launch_bprep<float>(const BProb*, const BDyn*, int, int64_t, bool, hipStream_t);
template void launch_bprep<double>(const BProb*, const BDyn*, int, int64_t, bool, hipStream_t);
template void launch_bhp_fused<float>(const BProb*, const BDyn*, const BWork*, int, int, hipStream_t);
template void launch_bhp_fused<double>(const BProb*, const BDyn*, const BWork*, int, int, hipStream_t);
template void launch_bhp_twopass<float>(const BProb*, const BDyn*, const BWork*, int, const BWork*, int, hipStream_t);
template void launch_bhp_twopass<double>(const BProb*, const BDyn*, const BWork*, int, const BWork*, int, hipStream_t);
template void launch_bcolsum<float>(const BProb*, const BDyn*, int, int64_t, bool, hipStream_t);
template void launch_bcolsum<double>(const BProb*, const BDyn*, int, int64_t, bool, hipStream_t);

}  // namespace aes
