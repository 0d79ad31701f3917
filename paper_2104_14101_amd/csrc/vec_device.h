// Device helpers shared by the single-problem vector kernels (k_vec.hip) and the grouped
// kernels of the batched step (k_batch.hip): the fixed-order column reduction of a
// 1024-thread workgroup and the stop rules of the adaptive loop.
#pragma once

#include <hip/hip_runtime.h>

namespace aes {

constexpr int kVT = 1024;  // threads of the single-workgroup vector kernels

enum StopRule { kStopXrel = 0, kStopDtildeRel = 1, kStopFixed = 2, kStopRemark = 3 };

// Column-wise block sum: thread t contributes v to column t % C (C a power of two dividing
// 1024); on return buf[c] holds the sum for column c (fixed-order tree).
__device__ __forceinline__ void col_reduce(double* buf, double v, int C) {
  const int tid = threadIdx.x;
  buf[tid] = v;
  __syncthreads();
  for (int s = kVT / 2; s >= C; s >>= 1) {
    if (tid < s) buf[tid] += buf[tid + s];
    __syncthreads();
  }
}

// Stop rule of one column after a commit.  D is the decrement r^T H_S^{-1} r (Algorithm 2's;
// the IHS value doubled), D0 its value at the start, xn2 = ||x||^2:
//   XREL: (1 + sqrt rho) D <= nu^2 min(lambda) tol^2 ||x||^2 (stop_sr = 1 + sqrt rho, stop_scale =
//         nu^2 min(lambda) tol^2), from the decrement lemma and H >= nu^2 Lambda;
//   DTILDE_REL: D <= tol^2 D0;  REMARK: D / 2 <= stop_scale (the Remark on termination).
// A zero decrement or an exactly zero residual stops the column (exact convergence).
__device__ __forceinline__ bool stop_test(int rule, double Dfull, double D0full, double xn2, bool resid_zero,
                                          double stop_scale, double stop_sr, double tol2) {
  if (Dfull <= 0.0 || resid_zero) return true;
  switch (rule) {
    case kStopXrel:
      return stop_sr * Dfull <= stop_scale * xn2;
    case kStopDtildeRel:
      return Dfull <= tol2 * D0full;
    case kStopRemark:
      return 0.5 * Dfull <= stop_scale;
    default:
      return false;  // kStopFixed is decided by the host from the step count
  }
}

}  // namespace aes
