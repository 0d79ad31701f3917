/*
 * aes.h -- C ABI of the adaptive sketching-based least-squares solver for MI355X (gfx950).
 *
 * Problem (Lacotte & Pilanci, arXiv 2104.14101, eq. "main optimization problem"):
 *     x* = argmin_x  1/2 x^T H x - b^T x,     H = A^T A + nu^2 Lambda,
 * with A in R^{n x d} dense, b in R^{d} (or R^{d x c}: c right-hand sides, the "matrix
 * variables" of Sec. 5), Lambda = diag(lambda) with lambda_i > 0, nu > 0.
 *
 * Conventions for every entry point
 *   - Matrices are row-major.  A is n x d with leading dimension lda >= d (elements).
 *     Right-hand sides and solutions are d x c with leading dimension ldb / ldx >= c; for
 *     c = 1 pass ld = 1 (a contiguous vector).
 *   - Pointers documented "device" are caller-owned HBM buffers on the handle's device; the
 *     library reads/writes them only during the call and never retains them, except an
 *     aes_ctx, which keeps a non-owning pointer to A until aes_ctx_free (A must stay valid and
 *     unchanged until then).  Pointers documented "host" are ordinary host memory.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.  All device work
 *     is enqueued on it.  The solve entry points block until their result is complete
 *     (the adaptive loop takes one host decision per iteration); the kernel-level entry points
 *     (aes_hv, aes_sketch, ...) are asynchronous on `stream`.
 *   - Errors are returned as aes_status; no C++ exception crosses the ABI.  A message for
 *     the last error on a handle is available from aes_last_error.  On AES_ERR_INVALID_ARG no
 *     output buffer has been written.
 *   - Random numbers: Philox4x64-10 keyed by (seed, (problem << 32) | k), k = index of the
 *     sketch within a solve; see the sketch entry points for the streams.
 */
#ifndef AES_H
#define AES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct aes_handle_s* aes_handle; /* device workspace pool; use from one host thread */
typedef struct aes_ctx_s* aes_ctx;       /* kept sketch + factor for adjoint solves */

typedef enum {
  AES_OK = 0,
  AES_ERR_INVALID_ARG = 1,  /* a size, pointer or option is out of range */
  AES_ERR_NOT_SPD = 2,      /* a Cholesky pivot of H_S (or W_S) was <= 0 or NaN */
  AES_ERR_NONFINITE = 3,    /* a step length or decrement became NaN/Inf */
  AES_ERR_MAX_ITER = 4,     /* max_iter accepted steps without meeting the stop rule;
                               x holds the last accepted iterate */
  AES_ERR_HIP = 5,          /* a HIP runtime call failed */
  AES_ERR_OOM = 6,          /* device workspace allocation failed */
  AES_ERR_NOT_IMPLEMENTED = 7
} aes_status;

/* AES_CG: the unpreconditioned conjugate-gradient baseline of the paper's numerical section
 * (Sec. 5): no sketch, FP64 only, stop rules XREL (with the identity for H_S:
 * r^T r <= (nu^2 min(lambda) tol)^2 ||x||^2), DTILDE_REL and FIXED. */
/* AES_POLYAK: the heavy-ball (Polyak-IHS) update of the appendix "Heavy-ball Acceleration and
 * Adaptivity", x+ = x - mu_rho H_S^{-1} grad f(x) + beta_rho (x - x_prev) with the corollary's
 * mu_rho = 2(1-rho)/(1+sqrt(1-rho)), beta_rho = (1-sqrt(1-rho))/(1+sqrt(1-rho)).  With
 * adaptive = 0 it is the fixed-m method; the adaptive form tests D+/D_I against
 * (1+sqrt rho)/(1-sqrt rho) alpha(tau, rho) beta_rho^omega(tau), tau = t+1-I (the corollary's
 * finite-time factor), and restarts the momentum (x_prev = x_t) after a resize.  The paper notes
 * that this factor is too loose for the adaptive form to be practical. */
typedef enum { AES_PCG = 0, AES_IHS = 1, AES_CG = 2, AES_POLYAK = 3 } aes_method;
/* AES_SRHT_REUSE: transform-reuse variant of the SRHT (not the paper's method; FP64 only).
 * S_k = sqrt(n'/m) R_k (H / sqrt(n')) E_0: the signs of index 0 for every sketch index k and the
 * row sample of index k.  Each S_k alone is an SRHT (Sec. 2.1), so a guarantee stated for one
 * SRHT holds for each of them and a union bound over the resizes applies, but the S_k share E_0
 * and H and are not independent.  A solve transforms A once (n' x d doubles kept in the handle's
 * workspace); every resize then only draws rows of the stored transform.
 * AES_SRHT_NESTED: the transform-reuse SRHT with nested row samples (not the paper's method;
 * FP64 only).  S_m = sqrt(n'/m) R_m (H / sqrt(n')) E_0, R_m the first m padded rows in
 * increasing order of their row keys of index 0 (ties: smaller row first), so each resize keeps
 * the rows it had; no sketch index is used.  Each S_m alone is the SRHT of index 0 with its rows
 * reordered.  Once m >= d the Gram grows incrementally: G_m' = (m/m') G_m plus the Gram of the
 * m' - m new rows, half the Gram flops of forming it again at a doubling. */
typedef enum {
  AES_SRHT = 0,
  AES_GAUSS = 1,
  AES_SJLT = 2,
  AES_SRHT_REUSE = 3,
  AES_SRHT_NESTED = 4
} aes_sketch_kind;
typedef enum {
  AES_FP64 = 0,       /* every step in FP64 */
  AES_MIXED = 1,      /* FP32-stored A for the PCG matvecs and the SRHT or SJLT (FP32 sums,
                         sketch rounded to BF16), BF16 MFMA Gram (FP32 accumulation), FP64
                         Cholesky, FP64 scalars and vectors, FP64 residual refinement (the
                         Gaussian sketch stays FP64) */
  AES_MIXED_FP32 = 2  /* as AES_MIXED with an FP32 sketch and an FP64 MFMA Gram of it (for small
                         nu, where a BF16 sketch or an FP32-accumulated Gram is too coarse) */
} aes_precision;
typedef enum {
  AES_STOP_XREL = 0,       /* (1+sqrt rho) D_t <= nu^2 min(lambda) tol^2 ||x_t||^2 (D = r^T H_S^-1 r) */
  AES_STOP_DTILDE_REL = 1, /* D_t <= tol^2 D_0 */
  AES_STOP_FIXED = 2,      /* exactly max_iter accepted steps */
  AES_STOP_REMARK = 3      /* 1/2 D_t <= tol / (m_delta + 1), Remark on termination, d_e := d */
} aes_stop_rule;

/* One attempted step of the adaptive loop (the axes of the paper's plots). */
typedef struct {
  int64_t t;          /* accepted-step counter before the attempt */
  int64_t m;          /* sketch size used by the attempt */
  int64_t k;          /* sketch index */
  double log_ratio;   /* max over active columns of log(D+ / D_I) */
  double threshold;   /* log c + (t+1-I) log phi */
  int32_t accept;
  int32_t pad_;
  double dtilde;      /* max over active columns of D (the preconditioned residual quantity of the
                         method) at the current iterate after the attempt: D_{t+1} when accepted,
                         else the unchanged D_t */
  double time_ms;     /* host milliseconds from the start of the solve to the attempt's flags */
} aes_trace_entry;

typedef struct {
  int32_t method;        /* aes_method, default AES_PCG */
  int32_t sketch;        /* aes_sketch_kind, default AES_SRHT */
  int32_t precision;     /* aes_precision, default AES_FP64 */
  int32_t stop;          /* aes_stop_rule, default AES_STOP_XREL */
  double rho;            /* in (0,1), default 1/8 (the adaptive guarantee assumes rho < 1/4) */
  int64_t m_init;        /* >= 1, default 1 */
  int64_t m_max;         /* cap on m; <= 0 means n' = 2^ceil(log2 n) */
  int64_t max_iter;      /* cap on accepted steps, default 200 */
  uint64_t seed;         /* Philox key word 0, default 0 */
  int32_t problem;       /* Philox stream id of the problem (key word 1 high half) */
  int32_t adaptive;      /* 1 (default): Algorithm 1/2; 0: fixed m = m_init, no test */
  int64_t force_reject_at;  /* test hook: reject the first candidate step at this t; -1 none */
  double inner_tol;      /* AES_MIXED: relative tolerance of each inner solve, default 1e-6 */
  int32_t max_refine;    /* AES_MIXED: cap on refinement sweeps, default 20 */
  int32_t trace_cap;     /* capacity of `trace` (entries) */
  aes_trace_entry* trace;   /* host, optional: filled with the attempted steps */
  const double* x0;         /* device d x c (ld = ldx) initial point, or NULL for 0 */
  int32_t profile;          /* 1: time every fused H.v launch with HIP events on `stream` */
  int32_t keep_fp32_copy;   /* AES_MIXED / AES_MIXED_FP32, default 0.  1: the caller promises that A
                               is unchanged since the last solve on this handle that cast the same
                               pointer with the same n, d, lda; the FP32 copy made then (kept in the
                               handle's pool) is reused instead of cast again.  A changed in place
                               under this promise gives results for the old A. */
} aes_options;

typedef struct {
  int64_t iterations;     /* accepted steps t (summed over sweeps for AES_MIXED) */
  int64_t attempts;       /* candidate steps (accepted + rejected) */
  int64_t final_m;        /* sketch size at exit */
  int64_t resketches;     /* number of times m was doubled */
  int64_t a_passes;       /* passes over A (H.v products and explicit residuals) */
  int64_t refine_sweeps;  /* AES_MIXED: outer refinement sweeps */
  int64_t trace_len;      /* entries written to options.trace (<= trace_cap) */
  double dtilde_final;    /* max over columns of the final decrement D */
  double time_sketch_ms;  /* host-measured wall time in sketch + factor phases */
  double time_total_ms;   /* host-measured wall time of the call */
  int32_t m_cap_reached;  /* a failed test was accepted because m reached its cap */
  int32_t status;         /* aes_status of the solve */
  double time_hv_ms;      /* options.profile: summed event time of the fused H.v kernels */
  int64_t hv_launches;    /* options.profile: number of fused H.v launches timed */
} aes_info;

/* Create a handle bound to HIP device `device` (allocates nothing large). */
aes_status aes_create(aes_handle* h, int device);
/* Release the handle and all its device workspace. */
aes_status aes_destroy(aes_handle h);
/* Message of the last error on `h` (static storage owned by the handle). */
const char* aes_last_error(aes_handle h);
/* Default options: PCG, SRHT, FP64, XREL, rho = 1/8, m_init = 1, max_iter = 200. */
void aes_default_options(aes_options* o);

/*
 * aes_solve -- adaptive PCG (Algorithm 2) or adaptive IHS (Algorithm 1 with the IHS update,
 * step mu = 1 - rho of Theorem "rate IHS"; AES_POLYAK and AES_CG select the heavy-ball variant
 * and the unpreconditioned baseline, see aes_method) for H x = b with the sketched preconditioner
 * H_S = (SA)^T SA + nu^2 Lambda, factorised as in Sec. 4.1 (Cholesky of H_S for m >= d,
 * Woodbury form with the Cholesky of W_S for m < d).  When the improvement test of the
 * algorithm fails, m doubles, a fresh S is drawn and the method restarts at x_t.
 *   A       device, n x d, row-major, lda >= d; 1 <= d <= 32768 (the single-pass fused
 *           H.v serves d <= 8192 with one right-hand side; wider problems and several
 *           right-hand sides use two MFMA products A v and A^T (A v) per step)
 *   b       device, d x c, ldb >= c, 1 <= c <= 32
 *   lambda  device, length d, all > 0; NULL means Lambda = I
 *   x       device, d x c output, ldx >= c
 *   info    host, output (may be NULL)
 * Returns AES_OK, or AES_ERR_MAX_ITER / NOT_SPD / NONFINITE with x = last accepted iterate.
 */
aes_status aes_solve(aes_handle h, void* stream, int64_t n, int64_t d, int64_t c,
                     const double* A, int64_t lda, const double* b, int64_t ldb, double nu,
                     const double* lambda, double tol, const aes_options* opt, double* x,
                     int64_t ldx, aes_info* info);

/*
 * aes_solve_direct -- the direct baseline of Sec. 5 (a Cholesky factorisation of the full
 * Hessian): G = A^T A + nu^2 Lambda in FP64 (O(n d^2) on MFMA), its lower Cholesky factor and
 * inverse factor (O(d^3)), then x = L^-T (L^-1 b).  No sketch, no iteration; the error of x is
 * that of a Cholesky solve, about kappa(H) times the unit roundoff.
 *   A       device, n x d, row-major, lda >= d; 1 <= d <= 32768
 *   b       device, d x c, ldb >= c, 1 <= c <= 32
 *   lambda  device, length d, all > 0; NULL means Lambda = I
 *   x       device, d x c output, ldx >= c (written only on success)
 * Workspace: four (d rounded up to 64)^2 FP64 matrices (plus split-K partials of the Gram) in the
 * handle's pool.  Synchronises `stream` to read the factorisation flag.  Returns AES_OK,
 * AES_ERR_INVALID_ARG (x untouched) or AES_ERR_NOT_SPD (a pivot was not positive; x untouched).
 */
aes_status aes_solve_direct(aes_handle h, void* stream, int64_t n, int64_t d, int64_t c, const double* A,
                            int64_t lda, const double* b, int64_t ldb, double nu, const double* lambda, double* x,
                            int64_t ldx);

/*
 * aes_solve_dual -- the same problem H x = b through its dual (Sec. 1, eq. "dual optimization
 * problem"), for n < d: with B = Lambda^{-1/2} A^T (d x n) the dual variable w in R^n solves
 * (B^T B + nu^2 I_n) w = A Lambda^{-1} b, which aes_solve's algorithm handles with data matrix B
 * (d rows, n columns) and Lambda = I; then x = Lambda^{-1} (b - A^T w) / nu^2 (from H x = b;
 * at the solution A x = w).  Arguments and layouts as in aes_solve, except:
 *   n       1 <= n <= 32768 (the dual has n unknowns); d is not limited
 *   opt     as in aes_solve; x0 must be NULL; the stop rule and tol apply to w, so the
 *           error of x is bounded through x - x* = -Lambda^{-1} A^T (w - w*) / nu^2
 *   info    of the dual solve: iterations, m and a_passes refer to B; the call adds one pass
 *           over A for A Lambda^{-1} b, one read of A and one write of B (d x n, kept in the
 *           handle's workspace) and one pass over B for x
 * Returns as aes_solve; on AES_ERR_MAX_ITER, x is mapped from the last accepted w.
 */
aes_status aes_solve_dual(aes_handle h, void* stream, int64_t n, int64_t d, int64_t c,
                          const double* A, int64_t lda, const double* b, int64_t ldb, double nu,
                          const double* lambda, double tol, const aes_options* opt, double* x,
                          int64_t ldx, aes_info* info);

/* One problem of a batch (all pointers device, layouts as in aes_solve). */
typedef struct {
  int64_t n, d, c;
  const double* A;
  int64_t lda;
  const double* b;
  int64_t ldb;
  double nu;
  const double* lambda;
  double* x;
  int64_t ldx;
} aes_problem;

/*
 * aes_solve_batched -- solves nprob independent problems (each with c right-hand sides that
 * share the problem's sketch, Sec. 5 "matrix variables").  Problem p draws its sketches from
 * Philox stream id p.  probs and infos are host arrays of length nprob.  The problems run
 * concurrently on up to 8 internal streams (default priority; the environment variable
 * AES_BATCH_WORKERS sets another count, 1..64) that wait for `stream`; the call returns when
 * all are done.
 */
aes_status aes_solve_batched(aes_handle h, void* stream, int64_t nprob, const aes_problem* probs,
                             double tol, const aes_options* opt, aes_info* infos);

/*
 * aes_solve_keep -- as aes_solve (single problem) and additionally returns a context holding
 * the last sketch, its factorisation and x*, for adjoint solves with the same H_S.
 */
aes_status aes_solve_keep(aes_handle h, void* stream, int64_t n, int64_t d, int64_t c,
                          const double* A, int64_t lda, const double* b, int64_t ldb, double nu,
                          const double* lambda, double tol, const aes_options* opt, double* x,
                          int64_t ldx, aes_info* info, aes_ctx* ctx);

/*
 * aes_adjoint_solve -- solves H lam = g (H symmetric) by the forward solve's method (adaptive
 * PCG, IHS or Polyak-IHS) starting from the context's sketch size and factorisation (resketching
 * only if the improvement test fails).
 *   g    device, d x c (ld = c);   lam  device, d x c output (ld = c)
 */
aes_status aes_adjoint_solve(aes_ctx ctx, void* stream, const double* g, double tol,
                             double* lam, aes_info* info);

/*
 * aes_grad -- gradients of L(x*) given the adjoint lam = H^{-1} dL/dx* (single column):
 *   dA = -(A x*) lam^T - (A lam) x*^T   (device n x d, ld = d; NULL to skip)
 *   dlognu = -2 nu^2 lam^T Lambda x*     (host scalar; NULL to skip)
 * db equals lam and is not computed here.
 */
aes_status aes_grad(aes_ctx ctx, void* stream, const double* lam, double* dA, double* dlognu);

void aes_ctx_free(aes_ctx ctx);

/*
 * Kernel-level entry points (asynchronous on `stream`; used by the parity tests).
 */

/* q = A^T (A p) + nu^2 lambda .* p  and  pHp = ||A p||^2 + nu^2 p^T Lambda p   (single pass
 * over A; the per-iteration product of Sec. 4.1 "Per-iteration cost").
 *   For d > 8192 (up to 32768) two streaming passes, z = A p then A^T z, and pHp = p . q.
 *   p, q: device length d.  pHp: device, 1 double.  lambda: device or NULL. */
aes_status aes_hv(aes_handle h, void* stream, int64_t n, int64_t d, const double* A, int64_t lda,
                  double nu, const double* lambda, const double* p, double* q, double* pHp);

/* aes_hv without any device allocation, for callers that cannot allocate (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same kernels and results as
 * aes_hv (bit-identical), with the per-workgroup partials and the pHp state in a static
 * device array of 33.7 MB that the library holds on every device it runs on until the process
 * ends (its address is resolved in aes_create).  Takes 1 <= d <= 8192 (AES_ERR_INVALID_ARG
 * otherwise).  Every call on a device shares that array and leaves its contents behind: calls
 * that overlap on one device (streams without mutual ordering) race and give wrong results.
 * Arguments as aes_hv; asynchronous on `stream`. */
aes_status aes_hv_noalloc(aes_handle h, void* stream, int64_t n, int64_t d, const double* A, int64_t lda,
                          double nu, const double* lambda, const double* p, double* q, double* pHp);

/* r = b - A^T (A x) - nu^2 Lambda x -- the explicit residual of Algorithm 2 ("compute
 * r_t = b - H x_t"), as the refinement sweeps of the mixed-precision and batched solves form it:
 * in compensated FP64 (every product split exactly by fma, every sum carried as an unevaluated
 * pair), rounded to FP64 once, so its error is about one rounding of r plus (n + d) u^2 times
 * |A|^T |A| |x| instead of (n + d) u |A|^T |A| |x|.  Two reads of A.
 *   A device n x d (lda); b, x device d x c (ldb, ldx); r device d x c output (ldr); c <= 32;
 *   lambda device length d or NULL; nu >= 0.  Asynchronous on `stream`. */
aes_status aes_residual(aes_handle h, void* stream, int64_t n, int64_t d, int64_t c, const double* A, int64_t lda,
                        const double* b, int64_t ldb, double nu, const double* lambda, const double* x, int64_t ldx,
                        double* r, int64_t ldr);

/* Tuner of the batched step's product A^T (A P) (the matrix-variable solves of Sec. 5): the average
 * time in milliseconds (*ms, host) of the grouped product for one n x d problem with
 * c <= 32 columns under a given plan, over `reps` launches after a warm-up launch.
 *   precision  AES_FP64 (the FP64 matrix) or AES_MIXED_FP32 (its FP32 copy, as the mixed modes)
 *   twopass    0: the fused single-read form (needs d <= 2048 in FP32, d <= 1024 in FP64, rows
 *              of A 16-byte aligned); 1: the two-pass form
 *   rows       rows of A per partial product (a multiple of 16)
 * The plans the library uses come from the file the tuning script writes (one per precision,
 * ceil(log2 n) and ceil(d / 256)); asynchronous work is complete when the call returns. */
aes_status aes_tune_hp(aes_handle h, void* stream, int64_t n, int64_t d, int64_t c, const double* A, int64_t lda,
                       int precision, int twopass, int64_t rows, int reps, double* ms);

/* Q = A^T (A P) + nu^2 Lambda P for c right-hand sides (P, Q device d x c, ld = c, c a power of
 * two <= 32) -- the per-step product of the matrix-variable solves (Sec. 5).  precision
 * AES_FP64: FP64 MFMA; AES_MIXED / AES_MIXED_FP32: A rounded to FP32 and FP32 MFMA products
 * with FP32 accumulation within row blocks, FP64 sums across them. */
aes_status aes_hv_multi(aes_handle h, void* stream, int64_t n, int64_t d, int64_t c, const double* A,
                        int64_t lda, double nu, const double* lambda, const double* P, double* Q,
                        int precision);

/* SA for sketch index k of size m (Sec. 2.1).  kind AES_SRHT: SA = (1/sqrt m) R H E A_pad,
 * H the unnormalised Sylvester Walsh-Hadamard matrix of order n' = 2^ceil(log2 n), E the
 * signs of stream SIGN, R the m padded rows with the smallest ROW keys (ascending order);
 * kind AES_GAUSS: SA = G A / sqrt m with G from stream GAUSS by Box-Muller;
 * kind AES_SJLT: the sparse embedding with one +-1 per column (s = 1): data row i goes, with
 * its sign, into sketch row h_i, both from stream SJLT; each sketch row sums its rows in
 * increasing order (n < 2^31; m may exceed n, leaving zero rows);
 * kind AES_SRHT_REUSE: SA = sqrt(n'/m) R_k Y with Y = (1/sqrt n') H E_0 A_pad (signs of index 0,
 * rows of index k), computed from scratch on every call;
 * kind AES_SRHT_NESTED: SA = sqrt(n'/m) Y[order[0..m)] with order the padded rows sorted by
 * their row keys of index 0 (k is not used; rows listed in that order).
 *   SA: device, m x d output (ld = d).  1 <= m <= n'. */
aes_status aes_sketch(aes_handle h, void* stream, int kind, int64_t n, int64_t d, const double* A,
                      int64_t lda, int64_t m, uint64_t seed, int32_t problem, int64_t k, double* SA);

/* Factorisation of H_S from SA (Sec. 4.1).  For m >= d writes G = SA^T SA + nu^2 Lambda and
 * its lower Cholesky factor L (both d x d, ld = d) to `G` and `L`; for m < d writes
 * W = SA Lambda^-1 SA^T + nu^2 I_m and L_W (m x m, ld = m).  Returns AES_ERR_NOT_SPD if a
 * pivot fails (synchronises the stream to read the flag). */
aes_status aes_factor(aes_handle h, void* stream, int64_t m, int64_t d, const double* SA, double nu,
                      const double* lambda, double* G, double* L);

/* v = H_S^{-1} z for the sketch SA (m x d), by the factorisation of Sec. 4.1 (builds it; the
 * solvers cache it instead).  z, v: device d x c (ld = c). */
aes_status aes_precond_apply(aes_handle h, void* stream, int64_t m, int64_t d, int64_t c,
                             const double* SA, double nu, const double* lambda, const double* z,
                             double* v);

#ifdef __cplusplus
}
#endif

#endif /* AES_H */
