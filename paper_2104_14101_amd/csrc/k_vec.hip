// O(d) vector work of the adaptive PCG / IHS loops (Algorithm 2, Algorithm 1), the
// preconditioner applications as GEMVs with the inverted Cholesky factors (Sec. 4.1), and
// small helpers (copies, casts, the rank-2 gradient of the adjoint).
//
// Scalar state of a solve with C columns, `scal` (device doubles):
//   [0C) D      current decrement  r^T H_S^{-1} r  (IHS: 1/2 g^T H_S^{-1} g)
//   [1C) DI     decrement at the last restart index I
//   [2C) alpha  PCG step length of the pending candidate
//   [3C) Dp     decrement of the pending candidate
//   [4C) D0     decrement at the start (for the relative stop rule)
//   [5C) pHp    curvature of the pending candidate
//   [6C) lr     log(Dp / DI) of the pending candidate
//   [7C .. 7C+8) host-read flags: 0 fail, 1 number of active columns, 2 nonfinite,
//                3 accepted, 4 max log ratio over active columns, 5 max D over columns
#include <cmath>

#include "common.h"
#include "kernels.h"
#include "vec_device.h"

namespace aes {


// ---------------------------------------------------------------------------------------
// Wide form of the vector kernels (d * C >= kSplitElems, no device gate): the column sums
// are formed by a grid of G workgroups into partials, the single workgroup only combines the
// partials (fixed order) and decides, and the elementwise updates run on the grid again.
// Work buffer: 3 * G * C partials, then the commit record (accept, beta[C], active before[C]).
// ---------------------------------------------------------------------------------------
constexpr int64_t kSplitElems = 8192;
constexpr int kSplitMaxG = 256;

size_t vec_work_elems() { return (size_t)3 * kSplitMaxG * 64 + 2 * 64 + 1; }

static int split_groups(int64_t d, int C, const double* work, const int* gate) {
  const int64_t total = d * C;
  if (!work || gate || total < kSplitElems) return 0;
  return (int)std::min<int64_t>(kSplitMaxG, ceil_div(total, 2048));
}

// partials of NQ column sums over the flat d x C range; thread t of every workgroup only
// meets elements of column t % C (the grid stride is a multiple of 256 and C divides 256).
//   MODE 0: a.b               (PCG candidate: p.q)
//   MODE 1: a.b, x.x, |a|     (finish: rp.rtp, xp.xp, |rp|; init: r.rt, x.x, |r|)
// pcopy (init of PCG): pcopy = b on the active columns.
template <int MODE>
__global__ __launch_bounds__(256) void vec_partials_kernel(int64_t total, int C, const double* __restrict__ a,
                                                           const double* __restrict__ b, const double* __restrict__ x,
                                                           double* __restrict__ pcopy, const int* __restrict__ active,
                                                           double* __restrict__ part) {
  constexpr int NQ = MODE == 0 ? 1 : 3;
  __shared__ double sh[256];
  const int tid = threadIdx.x, G = gridDim.x, col = tid % C;
  double l[3] = {0.0, 0.0, 0.0};
  if (active[col]) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + tid; e < total; e += (int64_t)G * 256) {
      const double av = a[e], bv = b[e];
      l[0] = fma(av, bv, l[0]);
      if (MODE == 1) {
        if (x) l[1] = fma(x[e], x[e], l[1]);
        l[2] += fabs(av);
      }
      if (pcopy) pcopy[e] = bv;
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    sh[tid] = l[q];
    __syncthreads();
    for (int st = 128; st >= C; st >>= 1) {
      if (tid < st) sh[tid] += sh[tid + st];
      __syncthreads();
    }
    if (tid < C) part[((int64_t)q * G + blockIdx.x) * C + tid] = sh[tid];
    __syncthreads();
  }
}

// thread t of the single workgroup: sum of partials q of column t % C over the workgroups
// t / C, t / C + 1024 / C, ... (then col_reduce combines them in a fixed tree)
__device__ __forceinline__ double part_sum(const double* part, int q, int G, int C) {
  const int tid = threadIdx.x, col = tid % C, tpc = kVT / C;
  double v = 0.0;
  for (int w = tid / C; w < G; w += tpc) v += part[((int64_t)q * G + w) * C + col];
  return v;
}

__global__ __launch_bounds__(kVT) void pcg_candidate_kernel(int64_t d, int C, const double* __restrict__ spart, int nwg,
                                                            const double* __restrict__ lam, double nu2,
                                                            const double* __restrict__ x, const double* __restrict__ r,
                                                            const double* __restrict__ p, const double* __restrict__ q,
                                                            double* __restrict__ xp, double* __restrict__ rp,
                                                            double* __restrict__ scal, const int* __restrict__ active,
                                                            const int* __restrict__ gate,
                                                            const double* __restrict__ part, int G) {
  if (gate && *gate == 0) return;
  __shared__ double buf[kVT];
  __shared__ double alpha_s[64];
  const int tid = threadIdx.x, col = tid % C, tpc = kVT / C;
  double loc = 0.0;
  if (part) {
    if (active[col]) loc = part_sum(part, 0, G, C);
  } else if (spart) {
#pragma unroll 4
    for (int64_t i = tid / C; i < d; i += tpc) {
      const double pv = p[i * C + col];
      loc += (lam ? lam[i] : 1.0) * pv * pv;
    }
    loc *= nu2;
    for (int w = tid / C; w < nwg; w += tpc) loc += spart[(int64_t)w * C + col];
  } else {
#pragma unroll 4
    for (int64_t i = tid / C; i < d; i += tpc) loc += p[i * C + col] * q[i * C + col];
  }
  col_reduce(buf, loc, C);
  if (tid < C) {
    const double pHp = buf[tid];
    scal[5 * C + tid] = pHp;
    const double a = active[tid] ? scal[tid] / pHp : 0.0;
    scal[2 * C + tid] = a;
    alpha_s[tid] = a;
  }
  __syncthreads();
  if (part) return;  // the grid applies the step
  const double a = alpha_s[col];
  if (active[col])
#pragma unroll 4
    for (int64_t i = tid / C; i < d; i += tpc) {
      const int64_t e = i * C + col;
      xp[e] = x[e] + a * p[e];
      rp[e] = r[e] - a * q[e];
    }
}

__global__ void pcg_step_apply_kernel(int64_t total, int C, const double* __restrict__ x, const double* __restrict__ r,
                                      const double* __restrict__ p, const double* __restrict__ q,
                                      double* __restrict__ xp, double* __restrict__ rp,
                                      const double* __restrict__ scal, const int* __restrict__ active) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int c = (int)(e % C);
  if (!active[c]) return;
  const double a = scal[2 * C + c];
  xp[e] = x[e] + a * p[e];
  rp[e] = r[e] - a * q[e];
}

void launch_pcg_candidate(int64_t d, int C, const double* spart, int nwg, const double* lam, double nu2, const double* x,
                          const double* r, const double* p, const double* q, double* xp, double* rp, double* scal,
                          const int* active, hipStream_t s, const int* gate, double* work) {
  const int G = spart ? 0 : split_groups(d, C, work, gate);
  const int64_t total = d * C;
  if (G) {
    hipLaunchKernelGGL(vec_partials_kernel<0>, dim3(G), dim3(256), 0, s, total, C, p, q, nullptr, nullptr, active, work);
    AES_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(pcg_candidate_kernel, dim3(1), dim3(kVT), 0, s, d, C, spart, nwg, lam, nu2, x, r, p, q, xp, rp, scal,
                     active, gate, G ? work : nullptr, G);
  AES_LAUNCH_CHECK();
  if (G) {
    hipLaunchKernelGGL(pcg_step_apply_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, total, C, x, r, p, q,
                       xp, rp, scal, active);
    AES_LAUNCH_CHECK();
  }
}


// Shared tail of the PCG / IHS finish kernels.  `half` = 1 for the IHS decrement.
template <bool IHS>
__global__ __launch_bounds__(kVT) void finish_kernel(int64_t d, int C, double* __restrict__ x, double* __restrict__ r,
                                                     double* __restrict__ p, const double* __restrict__ xp,
                                                     const double* __restrict__ rp, const double* __restrict__ rtp,
                                                     double* __restrict__ scal, int* __restrict__ active,
                                                     int* __restrict__ gate, double thr, int force_reject,
                                                     int adaptive, int at_cap, int stop_rule, double stop_scale,
                                                     double stop_sr, double tol2, double seq,
                                                     const double* __restrict__ part, int G,
                                                     double* __restrict__ rec) {
  if (gate && *gate == 0) return;
  __shared__ double buf[kVT];
  __shared__ double dp_s[64], xn_s[64], rz_s[64];
  __shared__ int accept_s;
  const int tid = threadIdx.x, col = tid % C, tpc = kVT / C;
  const bool act = active[col] != 0;
  double l1 = 0.0, l2 = 0.0, l3 = 0.0;
  if (act && part) {
    l1 = part_sum(part, 0, G, C);
    l2 = part_sum(part, 1, G, C);
    l3 = part_sum(part, 2, G, C);
  } else if (act)
#pragma unroll 4
    for (int64_t i = tid / C; i < d; i += tpc) {
      const int64_t e = i * C + col;
      l1 += rp[e] * rtp[e];
      l2 += xp[e] * xp[e];
      l3 += fabs(rp[e]);
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
    bool fail = force_reject != 0;
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
      if (lr > thr) fail = true;
    }
    const bool accept = !nonfinite && (!fail || !adaptive || at_cap);
    fl[0] = fail ? 1.0 : 0.0;
    fl[2] = nonfinite ? 1.0 : 0.0;
    fl[3] = accept ? 1.0 : 0.0;
    fl[4] = maxlr;
    accept_s = accept;
  }
  __syncthreads();
  if (rec && tid == 0) rec[0] = accept_s ? 1.0 : 0.0;
  if (!accept_s) {
    if (tid == 0) {
      int na = 0;
      for (int c = 0; c < C; ++c) na += active[c] != 0;
      scal[7 * C + 1] = (double)na;
      scal[7 * C + 7] = seq;
      if (gate) *gate = 0;
    }
    return;
  }
  if (rec) {
    // the grid commits: beta and the active set before this step's stop test
    if (tid < C) {
      rec[1 + tid] = IHS ? 0.0 : dp_s[tid] / scal[tid];
      rec[1 + C + tid] = active[tid] ? 1.0 : 0.0;
    }
  } else if (act) {
    const double beta = IHS ? 0.0 : dp_s[col] / scal[col];
#pragma unroll 4
    for (int64_t i = tid / C; i < d; i += tpc) {
      const int64_t e = i * C + col;
      x[e] = xp[e];
      r[e] = rp[e];
      p[e] = IHS ? rtp[e] : rtp[e] + beta * p[e];
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
        if (stop_test(stop_rule, Df, D0f, xn_s[c], rz_s[c] == 0.0, stop_scale, stop_sr, tol2)) active[c] = 0;
      }
      na += active[c] != 0;
      if (scal[c] > maxD) maxD = scal[c];
    }
    scal[7 * C + 1] = (double)na;
    scal[7 * C + 5] = maxD;
    scal[7 * C + 7] = seq;
    if (gate) *gate = na > 0 ? 1 : 0;
  }
}

// Commit of an accepted step on the grid (wide form): x = xp, r = rp, p = rtp + beta p (IHS:
// p = rtp) on the columns that were active when the step was tested.
template <bool IHS>
__global__ void finish_commit_kernel(int64_t total, int C, double* __restrict__ x, double* __restrict__ r,
                                     double* __restrict__ p, const double* __restrict__ xp,
                                     const double* __restrict__ rp, const double* __restrict__ rtp,
                                     const double* __restrict__ rec) {
  if (rec[0] == 0.0) return;  // rejected: nothing to commit
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int c = (int)(e % C);
  if (rec[1 + C + c] == 0.0) return;
  x[e] = xp[e];
  r[e] = rp[e];
  p[e] = IHS ? rtp[e] : rtp[e] + rec[1 + c] * p[e];
}

template <bool IHS>
static void launch_finish(int64_t d, int C, double* x, double* r, double* p, const double* xp, const double* rp,
                          const double* rtp, double* scal, int* active, int* gate, double thr, int force_reject,
                          int adaptive, int at_cap, int stop_rule, double stop_scale, double stop_sr, double tol2,
                          hipStream_t s, double seq, double* work) {
  const int G = split_groups(d, C, work, gate);
  const int64_t total = d * C;
  double* rec = G ? work + (size_t)3 * kSplitMaxG * 64 : nullptr;
  if (G) {
    hipLaunchKernelGGL(vec_partials_kernel<1>, dim3(G), dim3(256), 0, s, total, C, rp, rtp, xp, nullptr, active, work);
    AES_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(finish_kernel<IHS>, dim3(1), dim3(kVT), 0, s, d, C, x, r, p, xp, rp, rtp, scal, active, gate, thr,
                     force_reject, adaptive, at_cap, stop_rule, stop_scale, stop_sr, tol2, seq, G ? work : nullptr, G,
                     rec);
  AES_LAUNCH_CHECK();
  if (G) {
    hipLaunchKernelGGL(finish_commit_kernel<IHS>, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, total, C, x, r,
                       p, xp, rp, rtp, rec);
    AES_LAUNCH_CHECK();
  }
}

void launch_pcg_finish(int64_t d, int C, double* x, double* r, double* p, const double* xp, const double* rp,
                       const double* rtp, double* scal, int* active, int* gate, double thr, int force_reject,
                       int adaptive, int at_cap, int stop_rule, double stop_scale, double stop_sr, double tol2,
                       hipStream_t s, double seq, double* work) {
  launch_finish<false>(d, C, x, r, p, xp, rp, rtp, scal, active, gate, thr, force_reject, adaptive, at_cap, stop_rule,
                       stop_scale, stop_sr, tol2, s, seq, work);
}

void launch_ihs_finish(int64_t d, int C, double* x, double* g, double* sd, const double* xp, const double* gp,
                       const double* sp, double* scal, int* active, int* gate, double thr, int force_reject,
                       int adaptive, int at_cap, int stop_rule, double stop_scale, double stop_sr, double tol2,
                       hipStream_t s, double seq, double* work) {
  launch_finish<true>(d, C, x, g, sd, xp, gp, sp, scal, active, gate, thr, force_reject, adaptive, at_cap, stop_rule,
                      stop_scale, stop_sr, tol2, s, seq, work);
}

// (Re)initialisation after a factorisation: p = rt (PCG), D = r.rt (x 1/2 for the IHS),
// DI = D, optionally D0 = D; then the stop rule at x.
template <bool IHS>
__global__ __launch_bounds__(kVT) void init_kernel(int64_t d, int C, const double* __restrict__ r,
                                                   const double* __restrict__ rt, double* __restrict__ p,
                                                   double* __restrict__ scal, int* __restrict__ active,
                                                   int stop_rule, double stop_scale, double stop_sr, double tol2,
                                                   const double* __restrict__ x, int set_d0, int* __restrict__ gate,
                                                   const int* __restrict__ chol_flag, const double* __restrict__ part,
                                                   int G) {
  __shared__ double buf[kVT];
  __shared__ double dd[64], xn[64], rz[64];
  const int tid = threadIdx.x, col = tid % C, tpc = kVT / C;
  const bool act = active[col] != 0;
  double l1 = 0.0, l2 = 0.0, l3 = 0.0;
  if (act && part) {  // sums (and the copy p = rt) formed by the grid
    l1 = part_sum(part, 0, G, C);
    l2 = part_sum(part, 1, G, C);
    l3 = part_sum(part, 2, G, C);
  } else if (act)
    for (int64_t i = tid / C; i < d; i += tpc) {
      const int64_t e = i * C + col;
      l1 += r[e] * rt[e];
      if (x) l2 += x[e] * x[e];
      l3 += fabs(r[e]);
      if (!IHS) p[e] = rt[e];
    }
  col_reduce(buf, l1, C);
  if (tid < C) dd[tid] = IHS ? 0.5 * buf[tid] : buf[tid];
  __syncthreads();
  col_reduce(buf, l2, C);
  if (tid < C) xn[tid] = buf[tid];
  __syncthreads();
  col_reduce(buf, l3, C);
  if (tid < C) rz[tid] = buf[tid];
  __syncthreads();
  if (tid == 0) {
    int na = 0;
    double maxD = 0.0;
    for (int c = 0; c < C; ++c) {
      if (active[c]) {
        scal[c] = dd[c];
        scal[C + c] = dd[c];
        if (set_d0) scal[4 * C + c] = dd[c];
        const double Df = IHS ? 2.0 * dd[c] : dd[c];
        const double D0f = IHS ? 2.0 * scal[4 * C + c] : scal[4 * C + c];
        if (stop_test(stop_rule, Df, D0f, xn[c], rz[c] == 0.0, stop_scale, stop_sr, tol2)) active[c] = 0;
        if (!isfinite(dd[c])) scal[7 * C + 2] = 1.0;
      }
      na += active[c] != 0;
      if (scal[c] > maxD) maxD = scal[c];
    }
    scal[7 * C + 1] = (double)na;
    scal[7 * C + 5] = maxD;
    // flag 6: the factorisation this initialisation follows met a non-positive pivot
    const bool bad = chol_flag && *chol_flag != 0;
    scal[7 * C + 6] = bad ? 1.0 : 0.0;
    scal[7 * C + 7] = -1.0;  // no step has run since this initialisation
    if (gate) *gate = (!bad && na > 0 && scal[7 * C + 2] == 0.0) ? 1 : 0;
  }
}

void launch_pcg_init(int64_t d, int C, const double* r, const double* rt, double* p, double* scal, int* active,
                     int* gate, int stop_rule, double stop_scale, double stop_sr, double tol2, const double* x,
                     int set_d0, hipStream_t s, const int* chol_flag, double* work) {
  const int G = split_groups(d, C, work, gate);
  if (G) {
    hipLaunchKernelGGL(vec_partials_kernel<1>, dim3(G), dim3(256), 0, s, d * C, C, r, rt, x, p, active, work);
    AES_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(init_kernel<false>, dim3(1), dim3(kVT), 0, s, d, C, r, rt, p, scal, active, stop_rule, stop_scale,
                     stop_sr, tol2, x, set_d0, gate, chol_flag, G ? work : nullptr, G);
  AES_LAUNCH_CHECK();
}

void launch_ihs_init(int64_t d, int C, const double* g, const double* sd, double* scal, int* active, int* gate,
                     int stop_rule, double stop_scale, double stop_sr, double tol2, const double* x, int set_d0,
                     hipStream_t s, const int* chol_flag, double* work) {
  const int G = split_groups(d, C, work, gate);
  if (G) {
    hipLaunchKernelGGL(vec_partials_kernel<1>, dim3(G), dim3(256), 0, s, d * C, C, g, sd, x, nullptr, active, work);
    AES_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(init_kernel<true>, dim3(1), dim3(kVT), 0, s, d, C, g, sd, nullptr, scal, active, stop_rule,
                     stop_scale, stop_sr, tol2, x, set_d0, gate, chol_flag, G ? work : nullptr, G);
  AES_LAUNCH_CHECK();
}

// xp = x - mu sd (IHS), or with xprev the heavy-ball step xp = (x - mu sd) + beta (x - xprev),
// which also saves x to xsave (the previous iterate of the next step)
__global__ void ihs_candidate_kernel(int64_t total, int C, const double* __restrict__ x, const double* __restrict__ sd,
                                     double mu, double* __restrict__ xp, const int* __restrict__ active,
                                     const int* __restrict__ gate, const double* __restrict__ xprev, double beta,
                                     double* __restrict__ xsave) {
  if (gate && *gate == 0) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const double xe = x[e];
  double v = xe;
  if (active[e % C]) {
    v = xe - mu * sd[e];
    if (xprev) v += beta * (xe - xprev[e]);
  }
  xp[e] = v;
  if (xsave) xsave[e] = xe;
}

void launch_ihs_candidate(int64_t d, int C, const double* x, const double* sd, double mu, double* xp, const int* active,
                          hipStream_t s, const int* gate, const double* xprev, double beta, double* xsave) {
  const int64_t total = d * C;
  hipLaunchKernelGGL(ihs_candidate_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, total, C, x, sd, mu, xp,
                     active, gate, xprev, beta, xsave);
  AES_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------------------
// Row-dot GEMV, one wave per row; C right-hand sides reduced with the transpose reduction.
// ---------------------------------------------------------------------------------------
template <int CC>
__global__ __launch_bounds__(256) void rowdot_kernel(int64_t nrows, int64_t ncols, const double* __restrict__ M,
                                                     int64_t ldm, int tri, const double* __restrict__ x,
                                                     const double* __restrict__ xs, double ysgn,
                                                     const double* __restrict__ zadd,
                                                     const double* __restrict__ rowscale, double gscale,
                                                     double* __restrict__ y, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < nrows; i += nwaves) {
    int64_t jlo = 0, jhi = ncols;
    if (tri == 1) jhi = i + 1 < ncols ? i + 1 : ncols;
    if (tri == 2) jlo = i;
    double acc[CC];
#pragma unroll
    for (int c = 0; c < CC; ++c) acc[c] = 0.0;
    const double* Mi = M + i * ldm;
    int64_t j = jlo + lane;
    if (CC == 1 && !xs) {
      // eight loads of the row (and of x) in flight per lane before they are consumed
      double acc2[4] = {0.0, 0.0, 0.0, 0.0};
      for (; j + 7 * 64 < jhi; j += 8 * 64) {
        double mv[8], xv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          mv[k] = Mi[j + 64 * k];
          xv[k] = x[j + 64 * k];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) acc2[k & 3] = fma(mv[k], xv[k], acc2[k & 3]);
      }
      acc[0] = (acc2[0] + acc2[1]) + (acc2[2] + acc2[3]);
    }
    for (; j < jhi; j += 64) {
      double mv = Mi[j];
      if (xs) mv *= xs[j];
#pragma unroll
      for (int c = 0; c < CC; ++c) acc[c] = fma(mv, x[j * CC + c], acc[c]);
    }
    wave_transpose_sum<CC>(acc, lane);
    constexpr int shift = 6 - ilog2_c(CC);
    if ((lane & ((1 << shift) - 1)) == 0) {
      const int c = (lane >> shift) & (CC - 1);
      double v = ysgn * acc[0];
      if (zadd) v += zadd[i * CC + c];
      if (rowscale) v *= rowscale[i];
      y[i * CC + c] = v * gscale;
    }
  }
}

void launch_rowdot(int64_t nrows, int64_t ncols, const double* M, int64_t ldm, int tri, const double* x, int C,
                   const double* xs, double ysgn, const double* zadd, const double* rowscale, double gscale, double* y,
                   hipStream_t s, const int* gate) {
  if (nrows <= 0) return;
  int64_t blocks = ceil_div(nrows, 4);
  if (blocks > 4096) blocks = 4096;
  dim3 g((unsigned)blocks), b(256);
  switch (C) {
    case 1: hipLaunchKernelGGL(rowdot_kernel<1>, g, b, 0, s, nrows, ncols, M, ldm, tri, x, xs, ysgn, zadd, rowscale, gscale, y, gate); break;
    case 2: hipLaunchKernelGGL(rowdot_kernel<2>, g, b, 0, s, nrows, ncols, M, ldm, tri, x, xs, ysgn, zadd, rowscale, gscale, y, gate); break;
    case 4: hipLaunchKernelGGL(rowdot_kernel<4>, g, b, 0, s, nrows, ncols, M, ldm, tri, x, xs, ysgn, zadd, rowscale, gscale, y, gate); break;
    case 8: hipLaunchKernelGGL(rowdot_kernel<8>, g, b, 0, s, nrows, ncols, M, ldm, tri, x, xs, ysgn, zadd, rowscale, gscale, y, gate); break;
    case 16: hipLaunchKernelGGL(rowdot_kernel<16>, g, b, 0, s, nrows, ncols, M, ldm, tri, x, xs, ysgn, zadd, rowscale, gscale, y, gate); break;
    case 32: hipLaunchKernelGGL(rowdot_kernel<32>, g, b, 0, s, nrows, ncols, M, ldm, tri, x, xs, ysgn, zadd, rowscale, gscale, y, gate); break;
    default: throw std::invalid_argument("rowdot: C must be a power of two <= 32");
  }
  AES_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------------------
// Helpers.
// ---------------------------------------------------------------------------------------
__global__ void copy_cols_kernel(int64_t rows, int C, const double* __restrict__ src, int64_t lds, int csrc,
                                 double* __restrict__ dst, int64_t ldd, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * C) return;
  const int64_t i = e / C;
  const int c = (int)(e % C);
  dst[i * ldd + c] = c < csrc ? src[i * lds + c] : 0.0;
}

void launch_copy_cols(int64_t rows, int C, const double* src, int64_t lds, int csrc, double* dst, int64_t ldd,
                      hipStream_t s, const int* gate) {
  if (rows * C <= 0) return;
  hipLaunchKernelGGL(copy_cols_kernel, dim3((unsigned)ceil_div(rows * C, 256)), dim3(256), 0, s, rows, C, src, lds, csrc,
                     dst, ldd, gate);
  AES_LAUNCH_CHECK();
}

__global__ void fill_kernel(double* p, int64_t count, double v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = v;
}

void launch_fill(double* p, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s, p, count, v);
  AES_LAUNCH_CHECK();
}

// dst[c, r] = src[r, c] * (colscale ? colscale[c] : 1)
__global__ void transpose_kernel(int64_t rows, int64_t cols, const double* __restrict__ src, int64_t lds,
                                 double* __restrict__ dst, int64_t ldd, const double* __restrict__ colscale) {
  __shared__ double t[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
  const double cs = (colscale && c0 + tx < cols) ? colscale[c0 + tx] : 1.0;
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = r0 + k, c = c0 + tx;
    t[k][tx] = (r < rows && c < cols) ? src[r * lds + c] * cs : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t c = c0 + k, r = r0 + tx;
    if (c < cols && r < rows) dst[c * ldd + r] = t[tx][k];
  }
}

void launch_transpose(int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst, int64_t ldd,
                      hipStream_t s, const double* colscale) {
  if (rows <= 0 || cols <= 0) return;
  if (ceil_div(rows, 32) > 65535) throw std::invalid_argument("transpose: more than 2^21 rows");
  dim3 g((unsigned)ceil_div(cols, 32), (unsigned)ceil_div(rows, 32));
  hipLaunchKernelGGL(transpose_kernel, g, dim3(256), 0, s, rows, cols, src, lds, dst, ldd, colscale);
  AES_LAUNCH_CHECK();
}

// Dual-form inputs: isl[j] = lambda_j^{-1/2} (1 without lambda); for column k < c
// u[j, k] = b[j, k] * isl[j] and v[j, k] = b[j, k] * isl[j]^2, columns c..C-1 zero.
__global__ void dual_prep_kernel(int64_t d, int C, int c, const double* __restrict__ b, int64_t ldb,
                                 const double* __restrict__ lambda, double* __restrict__ isl,
                                 double* __restrict__ u, double* __restrict__ v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d * C) return;
  const int64_t j = e / C;
  const int k = (int)(e % C);
  const double l = lambda ? lambda[j] : 1.0;
  const double is = 1.0 / sqrt(l);
  if (k == 0) isl[j] = is;
  const double bj = k < c ? b[j * ldb + k] : 0.0;
  u[e] = bj * is;
  v[e] = bj / l;
}

void launch_dual_prep(int64_t d, int C, int c, const double* b, int64_t ldb, const double* lambda, double* isl,
                      double* u, double* v, hipStream_t s) {
  if (d * C <= 0) return;
  hipLaunchKernelGGL(dual_prep_kernel, dim3((unsigned)ceil_div(d * C, 256)), dim3(256), 0, s, d, C, c, b, ldb, lambda,
                     isl, u, v);
  AES_LAUNCH_CHECK();
}

__global__ void inv_kernel(int64_t count, const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) dst[e] = src ? 1.0 / src[e] : 1.0;
}

void launch_inv(int64_t count, const double* src, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(inv_kernel, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s, count, src, dst);
  AES_LAUNCH_CHECK();
}

template <typename TO>
__global__ void cast_kernel(int64_t n, int64_t d, const double* __restrict__ A, int64_t lda, TO* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * d) return;
  out[e] = (TO)A[(e / d) * lda + (e % d)];
}

template <typename TO>
void launch_cast(int64_t n, int64_t d, const double* A, int64_t lda, TO* out, hipStream_t s) {
  hipLaunchKernelGGL(cast_kernel<TO>, dim3((unsigned)ceil_div(n * d, 256)), dim3(256), 0, s, n, d, A, lda, out);
  AES_LAUNCH_CHECK();
}
template void launch_cast<float>(int64_t, int64_t, const double*, int64_t, float*, hipStream_t);

__global__ void axpy_cols_kernel(int64_t total, int C, double* __restrict__ x, const double* __restrict__ e,
                                 const int* __restrict__ active) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  if (!active || active[i % C]) x[i] += e[i];
}

void launch_axpy_cols(int64_t d, int C, double* x, const double* e, const int* active, hipStream_t s) {
  const int64_t total = d * C;
  hipLaunchKernelGGL(axpy_cols_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, total, C, x, e, active);
  AES_LAUNCH_CHECK();
}

// dA[i, :] = -(z1_i y2 + z2_i y1), z1 = A y1, z2 = A y2: one wave per row, A read once.
__global__ __launch_bounds__(256) void grad_rank2_kernel(const double* __restrict__ A, int64_t n, int64_t d, int64_t lda,
                                                         const double* __restrict__ y1, const double* __restrict__ y2,
                                                         double* __restrict__ dA, int64_t ldda) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < n; i += nwaves) {
    const double* Ai = A + i * lda;
    double v[2] = {0.0, 0.0};
    for (int64_t j = lane; j < d; j += 64) {
      const double a = Ai[j];
      v[0] = fma(a, y1[j], v[0]);
      v[1] = fma(a, y2[j], v[1]);
    }
    const double z1 = wave_sum(v[0]);
    const double z2 = wave_sum(v[1]);
    double* Di = dA + i * ldda;
    for (int64_t j = lane; j < d; j += 64) Di[j] = -(z1 * y2[j] + z2 * y1[j]);
  }
}

void launch_grad_rank2(const double* A, int64_t n, int64_t d, int64_t lda, const double* y1, const double* y2, double* dA,
                       int64_t ldda, hipStream_t s) {
  int64_t blocks = ceil_div(n, 4);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(grad_rank2_kernel, dim3((unsigned)blocks), dim3(256), 0, s, A, n, d, lda, y1, y2, dA, ldda);
  AES_LAUNCH_CHECK();
}

}  // namespace aes
