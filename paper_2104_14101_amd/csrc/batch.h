// Grouped kernels of the batched step (k_batch.hip): one launch covers every active problem of a
// batch, reading each problem's operands from a device descriptor (BProb, fixed for the batch)
// and its per-step parameters from a second one (BDyn, rewritten by the host before every step).
// The step of all problems is therefore a fixed sequence of launches, captured once in a HIP
// graph and replayed once per step of the adaptive loop.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace aes {

// One product of the preconditioner application, y = (ysgn * Mat[tri] (xs .* in) + zadd) .* rs * gs
// (Mat rows x K, row-major with leading dimension ld; tri 0 full, 1 lower, 2 upper).  rows = 0:
// the slot is unused by the current factorisation branch.
struct BProd {
  const double* mat;
  const double* in;
  const double* xs;
  const double* zadd;
  const double* rs;
  double* out;
  int64_t rows, K, ld;
  double ysgn, gs;
  int32_t tri, pad_;
};

constexpr int kBProds = 4;

// Per-problem operands of the step (fixed for the batch).
struct BProb {
  const void* A;       // n x d, ld lda: the FP64 matrix or its FP32 copy (the kernel's type)
  int64_t lda, n, d;
  int32_t C;           // columns of the iterate blocks (power of two <= 32)
  int32_t nrb;         // row ranges of the H.P (partials)
  int64_t rows;        // rows per range
  int64_t kpad;        // d rounded up for the transposed operand (multiple of 32)
  void* VT;            // NC x kpad transposed operand of the product (type of A), NC = max(C, 16)
  void* Z;             // n x NC (type of A), two-pass form only
  void* part;          // nrb x d x C partial products (type of A)
  const double* lam;   // d
  double nu2;
  // iterate blocks (d x C, row-major)
  double *X, *R, *P, *Q, *XP, *RP, *RTP;
  const double* rhs;   // right-hand side of the current (inner) solve
  double *xpv0, *xpv1; // Polyak-IHS previous iterates (alternating by step parity)
  double* scal;        // 8C + 8 scalar state (layout of the single-problem vector kernels)
  int* active;         // C
  int* gate;           // 1: the next step runs (set by the initialisation and the finish)
  double* flags_out;   // 8 doubles of the packed host-read flag array
  // constants of the method and the stop rule
  double mu, beta;
  double stop_sr, tol2;
  int32_t stop_rule, adaptive;
};

// Per-step parameters of a problem, written by the host before every step.
struct BDyn {
  double thr;        // log c + (t+1-I) log phi (or the Polyak-IHS factor)
  double seq;        // step stamp, written to flag 7 when the step runs
  double stop_scale; // scale of the stop test (changes between refinement sweeps)
  int32_t run;       // 0: the problem takes no part in this step
  int32_t force;     // test hook: reject this step
  int32_t at_cap;    // m has reached its cap (a failed test is accepted)
  int32_t parity;    // t & 1 (Polyak-IHS previous-iterate buffers)
  BProd prod[kBProds];
};

// Work item of the grouped H.P: problem p, row range r.
struct BWork {
  int32_t p, r;
};

// Product kinds of the grouped H.P.
enum BHpKind { kBHpFused = 0, kBHpTwoPass = 1 };

size_t bhp_smem_bytes(bool fp64, int mb);
// MB: column blocks of 256 per wave (d <= 256 MB); largest MB the fused form takes per type.
int bhp_fused_max_mb(bool fp64);
int bhp_fused_mb(bool fp64, int64_t d);

// Launchers (all asynchronous on s).  `probs` and `dyn` are device arrays of nprob entries.
template <typename T>
void launch_bprep(const BProb* probs, const BDyn* dyn, int nprob, int64_t max_elems, bool ihs, hipStream_t s);
template <typename T>
void launch_bhp_fused(const BProb* probs, const BDyn* dyn, const BWork* work, int nwork, int mb, hipStream_t s);
template <typename T>
void launch_bhp_twopass(const BProb* probs, const BDyn* dyn, const BWork* ztiles, int nz, const BWork* atiles,
                        int na, hipStream_t s);
// Q (PCG) or RP = H XP - rhs (IHS) from the partials
template <typename T>
void launch_bcolsum(const BProb* probs, const BDyn* dyn, int nprob, int64_t max_elems, bool ihs, hipStream_t s);
void launch_bcandidate(const BProb* probs, const BDyn* dyn, int nprob, int method, hipStream_t s);
void launch_bapply(const BProb* probs, const BDyn* dyn, const BWork* tiles, int ntiles, int slot, hipStream_t s);
void launch_bfinish(const BProb* probs, const BDyn* dyn, int nprob, bool ihs, hipStream_t s);

}  // namespace aes
