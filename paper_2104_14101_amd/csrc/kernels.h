// Host-side launchers of the HIP kernels (all asynchronous on the given stream).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>

namespace aes {

// ---- fused H.v (k_hv.hip) ---------------------------------------------------------------
// Number of workgroups used by hv_fused for a problem (the size of the partial buffers).
int hv_num_blocks(int num_cu, int64_t n);
// part[w*d + j] (w < nwg) and spart[w]: per-workgroup partials of A^T (A v) and ||A v||^2.
// gate (optional, device): when *gate == 0 the launch does nothing (a speculatively enqueued
// step of the adaptive loop whose predecessor was not accepted).
template <typename TA>
void launch_hv_fused(const TA* A, int64_t n, int64_t d, int64_t lda, const double* v, double* part,
                     double* spart, int nwg, hipStream_t s, const int* gate = nullptr);
// Multi-RHS variant (C right-hand sides, V is d x C row-major): part[w][d][C], spart[w][C].
template <typename TA>
void launch_hv_multi(const TA* A, int64_t n, int64_t d, int64_t lda, const double* V, int C,
                     double* part, double* spart, int nwg, hipStream_t s);
// out[j,c] = sgn * (sum_w part[w][j][c] + nu2 * lam[j] * v[j,c]) + (b ? bsgn*b[j,c] : 0)
void launch_hv_colsum(const double* part, int nwg, int64_t d, int C, const double* v,
                      const double* lam, double nu2, double sgn, const double* b, double bsgn,
                      double* out, hipStream_t s, const int* gate = nullptr);

void launch_hv_colsum_f32(const float* part, int nwg, int64_t d, int C, const double* v, const double* lam,
                          double nu2, double sgn, const double* b, double bsgn, double* out, hipStream_t s);
// Two-pass H.v for wide problems (d > 8192): z = A v by launch_rowdot, then
// part[w][j] = sum_{i in row block w} z_i A[i, j] for the nrb row blocks of `rows` rows that
// atz_blocks chooses, then launch_hv_colsum over the nrb partials.
int atz_blocks(int num_cu, int64_t n, int64_t d, int64_t* rows);
void launch_atz(const double* A, int64_t n, int64_t d, int64_t lda, const double* z, double* part, int nrb,
                int64_t rows, hipStream_t s);
// out[c] = ||e[:, c]||^2, out[C + c] = ||x[:, c]||^2
void launch_colnorm2(int64_t d, int C, const double* e, const double* x, double* out, hipStream_t s);

// ---- vector kernels (k_vec.hip): one workgroup, C columns ------------------------------
struct StepScalars;  // defined in k_vec.hip
// PCG candidate: pHp_c = sum_w spart[w][c] + nu2 sum_j lam_j p_jc^2; alpha_c = D_c / pHp_c;
// xp = x + alpha p; rp = r - alpha q   (only for active columns)
void launch_pcg_candidate(int64_t d, int C, const double* spart, int nwg, const double* lam, double nu2,
                          const double* x, const double* r, const double* p, const double* q,
                          double* xp, double* rp, double* scal, const int* active, hipStream_t s,
                          const int* gate = nullptr, double* work = nullptr);
// PCG finish: Dp = rp . rtp per column; test; commit if accepted; stop rule.  See k_vec.hip.
// gate (optional): read first (0: do nothing), then set to 1 iff the step was accepted, is
// finite and a column is still active — the gate of the next, speculatively enqueued step.
// seq: written to flag 7 of the flag block when the step runs (the initialisations write -1).
void launch_pcg_finish(int64_t d, int C, double* x, double* r, double* p, const double* xp,
                       const double* rp, const double* rtp, double* scal, int* active, int* gate,
                       double thr, int force_reject, int adaptive, int at_cap, int stop_rule,
                       double stop_scale, double stop_sr, double tol2, hipStream_t s, double seq = -1.0,
                       double* work = nullptr);
// PCG (re)initialisation after a factorisation: rt = H_S^{-1} r given; p = rt; D = r.rt; DI = D.
// gate (optional): set to 1 iff finite and a column is active.  chol_flag (optional): the
// factorisation's failure flag, copied to flag 6 of the flag block (and closing the gate).
void launch_pcg_init(int64_t d, int C, const double* r, const double* rt, double* p, double* scal,
                     int* active, int* gate, int stop_rule, double stop_scale, double stop_sr,
                     double tol2, const double* x, int set_d0, hipStream_t s, const int* chol_flag = nullptr,
                     double* work = nullptr);
// IHS: xp = x - mu s; Polyak-IHS (xprev given): xp = (x - mu s) + beta (x - xprev), and x is
// copied to xsave (the previous iterate for the next step)
void launch_ihs_candidate(int64_t d, int C, const double* x, const double* sd, double mu, double* xp,
                          const int* active, hipStream_t s, const int* gate = nullptr,
                          const double* xprev = nullptr, double beta = 0.0, double* xsave = nullptr);
void launch_ihs_finish(int64_t d, int C, double* x, double* g, double* sd, const double* xp,
                       const double* gp, const double* sp, double* scal, int* active, int* gate,
                       double thr, int force_reject, int adaptive, int at_cap, int stop_rule,
                       double stop_scale, double stop_sr, double tol2, hipStream_t s, double seq = -1.0,
                       double* work = nullptr);
void launch_ihs_init(int64_t d, int C, const double* g, const double* sd, double* scal, int* active,
                     int* gate, int stop_rule, double stop_scale, double stop_sr, double tol2,
                     const double* x, int set_d0, hipStream_t s, const int* chol_flag = nullptr,
                     double* work = nullptr);
// Wide form of the vector kernels (d * C >= 8192 without a device gate): a work buffer of
// vec_work_elems() doubles for the grid's partial column sums and the commit record.
size_t vec_work_elems();

// ---- triangular / dense GEMV (k_vec.hip) ------------------------------------------------
// y[i, c] = (ysgn * sum_{j in tri(i)} M[i, j] * xs[j] * x[j, c] + (zadd ? zadd[i, c] : 0))
//           * (rowscale ? rowscale[i] : 1) * gscale
// tri: 0 full [0, ncols), 1 lower [0, i], 2 upper [i, ncols)
void launch_rowdot(int64_t nrows, int64_t ncols, const double* M, int64_t ldm, int tri,
                   const double* x, int C, const double* xs, double ysgn, const double* zadd,
                   const double* rowscale, double gscale, double* y, hipStream_t s,
                   const int* gate = nullptr);

// ---- misc (k_vec.hip) --------------------------------------------------------------------
void launch_copy_cols(int64_t rows, int C, const double* src, int64_t lds, int csrc, double* dst,
                      int64_t ldd, hipStream_t s, const int* gate = nullptr);
void launch_fill(double* p, int64_t count, double v, hipStream_t s);
// dst[c, r] = src[r, c] * (colscale ? colscale[c] : 1)
void launch_transpose(int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst,
                      int64_t ldd, hipStream_t s, const double* colscale = nullptr);
// Dual form (n < d): isl = Lambda^{-1/2}; u = Lambda^{-1/2} b and v = Lambda^{-1} b as d x C
// (C >= c, the extra columns zero).
void launch_dual_prep(int64_t d, int C, int c, const double* b, int64_t ldb, const double* lambda, double* isl,
                      double* u, double* v, hipStream_t s);
void launch_inv(int64_t count, const double* src, double* dst, hipStream_t s);
template <typename TO>
void launch_cast(int64_t n, int64_t d, const double* A, int64_t lda, TO* out, hipStream_t s);
void launch_axpy_cols(int64_t d, int C, double* x, const double* e, const int* active, hipStream_t s);

// ---- sketches (k_sketch.hip) -------------------------------------------------------------
struct SelectScratch {
  uint64_t* keys;      // npad
  int32_t* pos;        // npad: output row of padded row i, or -1
  uint32_t* hist;      // 256 * 8
  uint64_t* state;     // 4
  uint32_t* blk;       // 2 * nblk
};
size_t select_blocks(int64_t npad);
void launch_srht_select(uint64_t seed, int32_t problem, int64_t k, int64_t npad, int64_t m,
                        const SelectScratch& sc, hipStream_t s);
void launch_signs(uint64_t seed, int32_t problem, int64_t k, int64_t n, double* eps, hipStream_t s);
// Elements of the WHT scratch Y for a padded height npad and d columns.
size_t srht_scratch_elems(int64_t npad, int64_t d);
// FWHT-based SRHT: SA (m x d, ld d) from A (n x d, lda); Y scratch of srht_scratch_elems
// elements of type TY;
// need: scratch of 512 ints (or NULL) for the row pruning of a two-pass transform.
template <typename TIN, typename TY, typename TOUT>
void launch_srht_apply(const TIN* A, int64_t n, int64_t d, int64_t lda, const double* eps, int64_t npad,
                       const int32_t* pos, int64_t m, TY* Y, TOUT* SA, int64_t ldsa, int32_t* need, hipStream_t s);
// Transform-reuse SRHT: SA[pos[i], :] = scale * Y[i, :] for the padded rows with pos[i] >= 0
// (Y: the stored normalised transform, npad x d, ld d; pos from launch_srht_select).
void launch_gather_rows(int64_t npad, int64_t d, const double* Y, const int32_t* pos, double scale, double* SA,
                        int64_t ldsa, hipStream_t s);
// Nested SRHT: order[r] (r < npad) = the padded row with the r-th smallest row key of sketch
// index 0, ties to the smaller row.  Scratch: keys (npad), cnt / cur / off (npad each), skey
// (npad) and bsum (keyorder_sum_elems(npad)).
struct KeyOrderScratch {
  uint64_t* keys;
  uint32_t* cnt;
  uint32_t* cur;
  uint32_t* off;
  uint32_t* bsum;
  uint64_t* skey;
};
size_t keyorder_sum_elems(int64_t npad);
void launch_srht_key_order(uint64_t seed, int32_t problem, int64_t npad, const KeyOrderScratch& sc, int32_t* order,
                           hipStream_t s);
// SA[r, :] = scale * Y[order[r], :] for r < m (Y: the stored normalised transform, ld d).
void launch_gather_ordered(int64_t m, int64_t d, const double* Y, const int32_t* order, double scale, double* SA,
                           int64_t ldsa, hipStream_t s);
// Gaussian sketch SA (m x d, ld d) = G A / sqrt(m): the plan sizes the generated slab of G
// (gt_elems doubles) and the split-K partials (part_elems doubles, none with one split).
struct GaussPlan {
  int splits;
  int64_t ks;    // K-rows per split and slab
  int64_t mp;    // leading dimension of the slab (m rounded up to 4)
  size_t gt_elems;
  size_t part_elems;
};
GaussPlan gauss_plan(int num_cu, int64_t n, int64_t d, int64_t m);
void launch_gauss_sketch(const GaussPlan& p, const double* A, int64_t n, int64_t d, int64_t lda, int64_t m,
                         uint64_t seed, int32_t problem, int64_t k, double* SA, double* gt, double* part,
                         hipStream_t s);

// SJLT with one non-zero per column (k_sjlt.hip): SA (m x d, ld d) = S A.  n < 2^31.
struct SjltPlan {
  int64_t nblk;        // counting blocks of 1024 data rows
  int Q;               // pieces per bucket (partial sums combined in order when Q > 1)
  int G;               // output items per reduction workgroup
  size_t count_elems;  // int32 elements of SjltScratch::cnt (m * nblk)
  size_t csum_elems;   // int32 elements of SjltScratch::csum
};
struct SjltScratch {
  int32_t* code;  // n
  int32_t* cnt;   // count_elems: counts, then their exclusive scan (bucket-major offsets)
  int32_t* csum;  // csum_elems
  int32_t* perm;  // n: data rows sorted by bucket (stable), sign in bit 31
  void* part;     // Q > 1: m * Q * d elements of the input type
};
SjltPlan sjlt_plan(int64_t n, int64_t d, int64_t m, size_t elem);  // elem: bytes per element of A
template <typename TA, typename TO>
void launch_sjlt(const SjltPlan& p, const TA* A, int64_t n, int64_t d, int64_t lda, int64_t m, uint64_t seed,
                 int32_t problem, int64_t k, TO* SA, const SjltScratch& sc, hipStream_t s);

// ---- dense linear algebra on MFMA (k_dense.hip) ------------------------------------------
// C = alpha * opA(A) * opB(B) + beta * C, batched with element strides; tri = 1 writes only
// elements with row >= col (and skips tiles strictly above the diagonal).
// atri (split-K products, batch z covering global k = z kofs + local k): A lower (1) or upper (2)
// triangular — K-blocks of zeros are not read; a batch entry with none left writes zeros.
void gemm_f64(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
              int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB, double beta, double* C,
              int64_t ldc, int64_t sC, int batch, int tri, hipStream_t s, int atri = 0, int64_t kofs = 0);
void gemm_f32(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const float* A,
              int64_t lda, int64_t sA, const float* B, int64_t ldb, int64_t sB, double beta, float* C,
              int64_t ldc, int64_t sC, int batch, int tri, hipStream_t s);
void widen_f32(int64_t count, const float* src, double* dst, hipStream_t s);
// out[e] = sum_{s < splits} part[s * stride + e]
void launch_sum_parts(int64_t count, int splits, int64_t stride, const double* part, double* out, hipStream_t s);
void narrow_f64(int64_t count, const double* src, float* dst, hipStream_t s);
// Gram of a sketch with split-K: G (dp x dp, ld dp) lower = SA^T SA + nu2 diag(lam) (padding
// rows/cols beyond d get identity).  part: scratch of splits * dp * dp doubles.
// Incremental form: with gprev (dp x dp lower, a Gram without the nu2 diag(lam) term) the sum
// becomes wprev * gprev + SA^T SA; gkeep (may equal gprev) receives that sum before the diagonal
// term is added.
int gram_splits(int num_cu, int64_t m, int64_t d, bool fp64);
void gram_tn(int64_t m, int64_t d, const double* SA, int64_t ldsa, double nu2, const double* lam,
             double* part, int splits, double* G, int64_t dp, hipStream_t s, const double* gprev = nullptr,
             double wprev = 0.0, double* gkeep = nullptr);
// BF16 SA (m x d, ld ldsa) with FP32 accumulation on MFMA; G as above in FP64.
void gram_tn_bf16(int64_t m, int64_t d, const __hip_bfloat16* SA, int64_t ldsa, double nu2,
                  const double* lam, float* part, int splits, double* G, int64_t dp, hipStream_t s);
// W (mp x mp) lower = SA diag(1/lam) SA^T + nu2 I_m (padding gets identity).
void gram_nt(int64_t m, int64_t d, const double* SA, int64_t ldsa, double nu2, const double* invlam,
             double* scaled, double* W, int64_t mp, hipStream_t s);
void gram_nt_bf16(int64_t m, int64_t d, const __hip_bfloat16* SA, int64_t ldsa, double nu2,
                  const double* invlam, double* sa64, double* scaled, double* W, int64_t mp, hipStream_t s);
// Linv = L^{-1} for the lower Cholesky factor L of G (np x np, np % 64 == 0, lower triangle
// read); *flag != 0 on a non-positive or NaN pivot.  keep_l: L is written over G (upper
// triangle zeroed); otherwise G holds only the diagonal blocks of L afterwards.
// tmp: cholinv_tmp_size(np) doubles.
size_t cholinv_tmp_size(int64_t np);
void cholinv(double* G, int64_t np, double* Linv, double* tmp, int* flag, bool keep_l, hipStream_t s);

// ---- adjoint (k_vec.hip) ------------------------------------------------------------------
// dA[i, j] = -(z1[i] * y2[j] + z2[i] * y1[j]) with z1 = A y1, z2 = A y2 computed in-kernel.
void launch_grad_rank2(const double* A, int64_t n, int64_t d, int64_t lda, const double* y1,
                       const double* y2, double* dA, int64_t ldda, hipStream_t s);

// Allocation-free fused H.v (noalloc.hip): its scratch is a static device array whose address
// on each device is resolved once by noalloc_init (with that device current).
hipError_t noalloc_init(int device);
void hv_noalloc(int device, int num_cu, hipStream_t s, int64_t n, int64_t d, const double* A, int64_t lda, double nu,
                const double* lambda, const double* p, double* q, double* pHp);

// ---- compensated explicit residual (k_resid.hip) -----------------------------------------
// r = b - A^T (A x) - nu^2 Lambda x for C columns (x, b, r: d x C with leading dimensions C, ldb,
// ldr), formed in double-double arithmetic and rounded once.  Scratch: zh, zl (n x C) and ph, pl
// (residual_dd_part_elems doubles each).  lam: device or NULL (identity).
size_t residual_dd_part_elems(int num_cu, int64_t n, int64_t d, int C);
void launch_residual_dd(int num_cu, int64_t n, int64_t d, int C, const double* A, int64_t lda, const double* b,
                        int64_t ldb, double nu, const double* lam, const double* x, double* zh, double* zl, double* ph,
                        double* pl, double* r, int64_t ldr, hipStream_t s);

}  // namespace aes
