// Shared device helpers of the HIP library: error macros, the Philox4x64-10 generator,
// uniform/normal transforms and wavefront reductions (wave64, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

namespace aes {

struct HipError : std::runtime_error {
  explicit HipError(const std::string& s) : std::runtime_error(s) {}
};

#define AES_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::aes::HipError(std::string(#call) + ": " + hipGetErrorString(e_));         \
  } while (0)

#define AES_LAUNCH_CHECK() AES_HIP(hipGetLastError())

constexpr int kWave = 64;

// ---------------------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of
//   (c0, c1, c2, c3) <- (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))
// with the key bumped by the Weyl increments (W0, W1) before every round but the first.
// ---------------------------------------------------------------------------------------
struct Rand4 {
  uint64_t w[4];
};

__device__ __forceinline__ Rand4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  Rand4 out;
  out.w[0] = c0;
  out.w[1] = c1;
  out.w[2] = c2;
  out.w[3] = c3;
  return out;
}

enum Stream : uint64_t { kStreamSign = 1, kStreamRow = 2, kStreamGauss = 3, kStreamSjlt = 4 };

struct RngKey {
  uint64_t k0, k1;
};

__host__ __device__ inline RngKey make_key(uint64_t seed, int32_t problem, int64_t k) {
  RngKey key;
  key.k0 = seed;
  key.k1 = ((uint64_t)(uint32_t)problem << 32) | (uint64_t)(uint32_t)k;
  return key;
}

// (w >> 11 + 1) * 2^-53 in (0, 1]  and  (w >> 11) * 2^-53 in [0, 1)
__device__ __forceinline__ double u01_open0(uint64_t w) {
  return ((double)(w >> 11) + 1.0) * 0x1.0p-53;
}
__device__ __forceinline__ double u01(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

// Four N(0,1) values (sketch rows 4q..4q+3 of data column i) by Box-Muller on (w0,w1), (w2,w3).
__device__ __forceinline__ void gauss4(const Rand4& r, double out[4]) {
  const double two_pi = 6.283185307179586476925286766559;
  double ra = sqrt(-2.0 * log(u01_open0(r.w[0])));
  double aa = two_pi * u01(r.w[1]);
  double rb = sqrt(-2.0 * log(u01_open0(r.w[2])));
  double ab = two_pi * u01(r.w[3]);
  double sa, ca, sb, cb;
  sincos(aa, &sa, &ca);
  sincos(ab, &sb, &cb);
  out[0] = ra * ca;
  out[1] = ra * sa;
  out[2] = rb * cb;
  out[3] = rb * sb;
}

// ---------------------------------------------------------------------------------------
// Wavefront reductions (64 lanes).
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Reduce R values across the 64 lanes of a wave with log2(64) exchange levels, halving the
// number of live values at each of the first log2(R) levels.  On return v[0] of lane l holds
// the wave sum of value (l >> (6 - log2 R)) & (R - 1).
template <int R>
__device__ __forceinline__ void wave_transpose_sum(double (&v)[R], int lane) {
  static_assert(R >= 1 && R <= 64 && (R & (R - 1)) == 0, "R must be a power of two <= 64");
  int cnt = R;
  int bitpos = 5;
#pragma unroll
  for (int level = 0; level < 6; ++level) {
    if (cnt > 1) {
      const int half = cnt >> 1;
      const bool hi = (lane >> bitpos) & 1;
#pragma unroll
      for (int i = 0; i < R / 2; ++i) {
        if (i < half) {
          const double send = hi ? v[i] : v[i + half];
          const double keep = hi ? v[i + half] : v[i];
          v[i] = keep + __shfl_xor(send, 1 << bitpos, kWave);
        }
      }
      cnt = half;
    } else {
      v[0] += __shfl_xor(v[0], 1 << bitpos, kWave);
    }
    --bitpos;
  }
}

__host__ __device__ constexpr int ilog2_c(int x) { return x <= 1 ? 0 : 1 + ilog2_c(x >> 1); }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }
inline int64_t next_pow2(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

}  // namespace aes
