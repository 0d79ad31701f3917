// Host engine behind the C ABI: workspace pool, the adaptive PCG / IHS loops (Algorithm 2,
// Algorithm 1 with the IHS update), the cached factorisation of H_S (Sec. 4.1), the
// mixed-precision refinement driver, batched solves, and the kept context for adjoint solves.
//
// Control: every device step is enqueued on the caller's stream; the host reads back one
// small block of flags per attempted step (accepted / rejected / stopped), because the
// accept-or-resketch decision of the algorithms is data dependent.
#include <dlfcn.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <functional>
#include <initializer_list>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "aes.h"
#include "common.h"
#include "kernels.h"
#include "batch.h"

#include <rocprofiler-sdk-roctx/roctx.h>

using namespace aes;

// ---------------------------------------------------------------------------------------
// Handle and workspace.
// ---------------------------------------------------------------------------------------
struct aes_handle_s {
  int device = 0;
  int num_cu = 256;
  std::unordered_map<std::string, std::pair<void*, size_t>> bufs;
  std::string err;
  double* pinned = nullptr;  // host-visible flag block
  std::vector<hipEvent_t> events;  // pairs for timing the fused H.v launches

  hipEvent_t event(size_t i) {
    while (events.size() <= i) {
      hipEvent_t e;
      AES_HIP(hipEventCreate(&e));
      events.push_back(e);
    }
    return events[i];
  }

  std::mutex mu;  // guards bufs / events / err when batched workers share the handle

  // Source of the FP32 copy each pool buffer holds (options.keep_fp32_copy): written by every
  // cast into the buffer, dropped when the pool frees the buffer.
  struct F32Src {
    const void* A;
    int64_t n, d, lda;
  };
  std::unordered_map<void*, F32Src> f32src;
  bool f32_copy_of(void* buf, const void* A, int64_t n, int64_t d, int64_t lda) {
    std::lock_guard<std::mutex> lock(mu);
    auto it = f32src.find(buf);
    return it != f32src.end() && it->second.A == A && it->second.n == n && it->second.d == d && it->second.lda == lda;
  }
  void f32_copy_set(void* buf, const void* A, int64_t n, int64_t d, int64_t lda) {
    std::lock_guard<std::mutex> lock(mu);
    f32src[buf] = F32Src{A, n, d, lda};
  }

  template <typename T>
  T* buf(const std::string& name, size_t count) {
    std::lock_guard<std::mutex> lock(mu);
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    auto it = bufs.find(name);
    if (it != bufs.end() && it->second.second >= bytes) return static_cast<T*>(it->second.first);
    if (it != bufs.end()) {
      f32src.erase(it->second.first);
      AES_HIP(hipFree(it->second.first));
      bufs.erase(it);
    }
    void* p = nullptr;
    const size_t alloc = (bytes + 255) / 256 * 256;
    hipError_t e = hipMalloc(&p, alloc);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw std::bad_alloc();
    }
    bufs[name] = {p, alloc};
    return static_cast<T*>(p);
  }
  // Frees every pool buffer whose name is not listed (the stream work that used them must be
  // complete).
  void release_except(std::initializer_list<const char*> keep) {
    std::lock_guard<std::mutex> lock(mu);
    for (auto it = bufs.begin(); it != bufs.end();) {
      bool kept = false;
      for (const char* k : keep) kept = kept || it->first == k;
      if (kept) {
        ++it;
      } else {
        f32src.erase(it->second.first);
        AES_HIP(hipFree(it->second.first));
        it = bufs.erase(it);
      }
    }
  }
  void set_err(const std::string& e) {
    std::lock_guard<std::mutex> lock(mu);
    err = e;
  }
  void release() {
    for (auto& kv : bufs) (void)hipFree(kv.second.first);
    bufs.clear();
    f32src.clear();
    for (auto e : events) (void)hipEventDestroy(e);
    events.clear();
    if (pinned) (void)hipHostFree(pinned);
    pinned = nullptr;
  }
};

struct aes_ctx_s {
  aes_handle h = nullptr;  // private workspace holding the kept factorisation
  int64_t n = 0, d = 0, lda = 0;
  const double* A = nullptr;
  double nu = 0;
  bool has_lambda = false;
  aes_options opt{};
  int64_t m = 0, k = 0;
  double* xstar = nullptr;  // device, d (owned by h's pool: "ctx_xstar")
};

namespace {

// Host range of a phase (sketch and factor, iterate, refinement sweep, batch) for
// rocprofv3 --marker-trace; a no-op when no profiler is attached.
struct PhaseRange {
  explicit PhaseRange(const char* name) { roctxRangePushA(name); }
  ~PhaseRange() { roctxRangePop(); }
  PhaseRange(const PhaseRange&) = delete;
  PhaseRange& operator=(const PhaseRange&) = delete;
};

struct StatusError : std::runtime_error {
  aes_status st;
  StatusError(aes_status s, const std::string& m) : std::runtime_error(m), st(s) {}
};

inline double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct ProblemDesc {
  int64_t n, d, c;
  const double* A;
  int64_t lda;
  const double* b;
  int64_t ldb;
  double nu;
  const double* lambda;
  double* x;
  int64_t ldx;
};

// Widest d: the fused single-pass H.v keeps a d-vector slice per thread and takes d <= 8192;
// wider problems (and several right-hand sides) use the two-product MFMA path.
constexpr int64_t kMaxFusedD = 8192;
constexpr int64_t kMaxD = 32768;

void validate(const ProblemDesc& P, double tol, const aes_options& o) {
  auto bad = [](const char* m) { throw StatusError(AES_ERR_INVALID_ARG, m); };
  if (P.n < 1 || P.d < 1 || P.c < 1) bad("n, d and c must be >= 1");
  if (P.c > 32) bad("at most 32 right-hand sides per problem");
  if (P.d > kMaxD) bad("d > 32768 is not supported");
  if (P.lda < P.d) bad("lda < d");
  if (P.ldb < P.c || P.ldx < P.c) bad("ldb and ldx must be >= c");
  if (!P.A || !P.b || !P.x) bad("A, b and x must be non-null");
  if (!(std::isfinite(P.nu) && P.nu > 0)) bad("nu must be finite and > 0");
  if (!(o.rho > 0.0 && o.rho < 1.0)) bad("rho must lie in (0, 1)");
  if (o.m_init < 1) bad("m_init must be >= 1");
  if (o.stop != AES_STOP_FIXED && !(tol > 0)) bad("tol must be > 0");
  if (o.method != AES_PCG && o.method != AES_IHS && o.method != AES_CG && o.method != AES_POLYAK)
    bad("unknown method");
  if (o.method == AES_CG && o.precision != AES_FP64) bad("the CG baseline runs in FP64");
  if (o.method == AES_CG && o.stop == AES_STOP_REMARK) bad("the REMARK stop rule needs a sketch");
  if (o.sketch != AES_SRHT && o.sketch != AES_GAUSS && o.sketch != AES_SJLT && o.sketch != AES_SRHT_REUSE &&
      o.sketch != AES_SRHT_NESTED)
    bad("unknown sketch");
  if ((o.sketch == AES_SRHT_REUSE || o.sketch == AES_SRHT_NESTED) && o.precision != AES_FP64)
    bad("the transform-reuse SRHT runs in FP64");
  if (o.sketch == AES_SJLT && P.n >= (int64_t(1) << 31)) bad("the SJLT needs n < 2^31");
  if (o.precision < AES_FP64 || o.precision > AES_MIXED_FP32) bad("unknown precision");
  if (o.stop < 0 || o.stop > 3) bad("unknown stop rule");
  if (o.max_iter < 0) bad("max_iter must be >= 0");
}

double remark_m_delta(int64_t n, int64_t d) {
  const double de = (double)d, delta = 1.0 / (double)d;
  const double t = std::sqrt(de) + std::sqrt(8.0 * std::log(2.0 * (double)n / delta));
  return 16.0 * std::log(16.0 * de / delta) * t * t;
}

// ---------------------------------------------------------------------------------------
// Solver: one problem, C (power of two) internal columns.
// ---------------------------------------------------------------------------------------
class Solver {
 public:
  // ns: namespace of the problem's own buffers in the handle pool; sns: namespace of the
  // scratch that only lives within one eager phase (sketch, factorisation, an eager product),
  // shared by the problems of a batch (their eager work is ordered on one stream)
  Solver(aes_handle h, hipStream_t s, const ProblemDesc& P, const aes_options& o, double tol, const std::string& ns,
         const std::string& sns = std::string())
      : h_(h), s_(s), P_(P), o_(o), tol_(tol), ns_(ns), sns_(sns.empty() ? ns : sns) {
    n_ = P.n;
    d_ = P.d;
    c_ = P.c;
    C_ = (int)next_pow2(P.c);
    npad_ = next_pow2(n_);
    mcap_ = o.m_max > 0 ? std::min<int64_t>(o.m_max, npad_) : npad_;
    nu2_ = P.nu * P.nu;
    mixed_ = o.precision == AES_MIXED || o.precision == AES_MIXED_FP32;
    sketch32_ = o.precision == AES_MIXED_FP32;
    cg_ = o.method == AES_CG;
    fused_ = C_ == 1 && d_ <= kMaxFusedD;
    if (cg_) o_.adaptive = 0;  // the baseline has no sketch, no test and no resketch
    pinned_ = h->pinned;
  }
  ~Solver() {
    if (ss_) {
      (void)hipStreamSynchronize(ss_);
      (void)hipStreamDestroy(ss_);
    }
    if (spec_done_) (void)hipEventDestroy(spec_done_);
    if (spec_go_) (void)hipEventDestroy(spec_go_);
    for (hipEvent_t& e : fev_)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : sk_ev_) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  }
  Solver(const Solver&) = delete;
  Solver& operator=(const Solver&) = delete;

  // Buffers in the handle pool, namespaced per solver role.
  template <typename T>
  T* B(const char* name, size_t count) {
    return h_->buf<T>(ns_ + name, count);
  }
  template <typename T>
  T* S(const char* name, size_t count) {
    return h_->buf<T>(sns_ + name, count);
  }

  void setup_common() {
    const int64_t dc = d_ * C_;
    lam_ = B<double>("lam", d_);
    invlam_ = B<double>("invlam", d_);
    if (P_.lambda) {
      AES_HIP(hipMemcpyAsync(lam_, P_.lambda, d_ * sizeof(double), hipMemcpyDeviceToDevice, s_));
      launch_inv(d_, P_.lambda, invlam_, s_);
    } else {
      launch_fill(lam_, d_, 1.0, s_);
      launch_fill(invlam_, d_, 1.0, s_);
    }
    X_ = B<double>("X", dc);
    R_ = B<double>("R", dc);
    Pv_ = B<double>("P", dc);
    Q_ = B<double>("Q", dc);
    XP_ = B<double>("XP", dc);
    RP_ = B<double>("RP", dc);
    RTP_ = B<double>("RTP", dc);
    Bv_ = B<double>("B", dc);
    scal_ = B<double>("scal", 8 * C_ + 8);
    vw_ = B<double>("vec_work", vec_work_elems());
    active_ = B<int>("active", C_);
    nwg_ = hv_num_blocks(h_->num_cu, n_);
    if (!fused_) {
      // row splits of A^T Z: about four workgroups (of 128 columns) per CU in flight
      const int64_t col_tiles = ceil_div(d_, 128);
      const int64_t want = std::max<int64_t>(1, 4 * (int64_t)h_->num_cu / col_tiles);
      const int64_t split_rows = round_up(std::max<int64_t>(512, ceil_div(n_, want)), 32);
      msplit_ = (int)ceil_div(n_, split_rows);
      msplit_rows_ = split_rows;
      if (C_ == 1) atz_nrb_ = atz_blocks(h_->num_cu, n_, d_, &atz_rows_);
    }
    hv_scratch();
    AES_HIP(hipMemsetAsync(scal_, 0, (8 * C_ + 8) * sizeof(double), s_));
    launch_copy_cols(d_, C_, P_.b, P_.ldb, (int)c_, Bv_, C_, s_);
    std::vector<int> act(C_, 0);
    for (int j = 0; j < c_; ++j) act[j] = 1;
    AES_HIP(hipMemcpyAsync(active_, act.data(), C_ * sizeof(int), hipMemcpyHostToDevice, s_));
    if (mixed_) {
      // the FP32 copy feeds the inner products and every sketch of the mixed modes
      A32_ = B<float>("A32", (size_t)n_ * d_);
      // the caller may promise that A is the one the buffer was cast from and unchanged since
      if (!(o_.keep_fp32_copy && h_->f32_copy_of(A32_, P_.A, n_, d_, P_.lda))) {
        launch_cast<float>(n_, d_, P_.A, P_.lda, A32_, s_);
        h_->f32_copy_set(A32_, P_.A, n_, d_, P_.lda);
      }
      hv_scratch();
    }
    stop_scale_ = nu2_ * min_lambda() * tol_ * tol_;
    if (o_.stop == AES_STOP_REMARK) stop_scale_ = tol_ / (remark_m_delta(n_, d_) + 1.0);
    stop_sr_ = 1.0 + std::sqrt(o_.rho);
    if (cg_) {
      // ||x - x*|| <= ||r|| / (nu^2 min lambda): r^T r <= (nu^2 min lambda tol)^2 ||x||^2
      const double sc = nu2_ * min_lambda() * tol_;
      stop_scale_ = sc * sc;
      stop_sr_ = 1.0;
    }
    tol2_ = tol_ * tol_;
  }

  double min_lambda() {
    if (!P_.lambda) return 1.0;
    std::vector<double> hl(d_);
    AES_HIP(hipMemcpyAsync(hl.data(), P_.lambda, d_ * sizeof(double), hipMemcpyDeviceToHost, s_));
    AES_HIP(hipStreamSynchronize(s_));
    double mn = hl[0];
    for (double v : hl) {
      if (!(v > 0) || !std::isfinite(v)) throw StatusError(AES_ERR_INVALID_ARG, "lambda entries must be finite and > 0");
      mn = std::min(mn, v);
    }
    return mn;
  }

  // Scratch of the eager H.v, fetched from the pool at every use: within a batch it is shared by
  // all problems and may have grown (and moved) since this problem last used it.
  void hv_scratch() {
    if (fused_) {
      part_ = S<double>("part", (size_t)nwg_ * d_);
      spart_ = S<double>("spart", nwg_);
      return;
    }
    part_ = S<double>("part", (size_t)msplit_ * d_ * C_);
    Z_ = S<double>("Z", (size_t)n_ * C_);
    if (C_ == 1) atz_part_ = S<double>("atz_part", (size_t)atz_nrb_ * d_);
    if (mixed_) {
      V32_ = S<float>("V32", (size_t)d_ * C_);
      Z32_ = S<float>("Z32", (size_t)n_ * C_);
      part32_ = S<float>("part32", (size_t)msplit_ * d_ * C_);
    }
  }

  // out = sgn * (H v) + bsgn * b    (H = A^T A + nu^2 Lambda); A in FP64 or (inner) FP32.
  void hv(const double* v, double* out, double sgn, const double* bb, double bsgn, bool use32,
          const int* gate = nullptr) {
    hv_scratch();
    if (fused_) {
      const bool prof = o_.profile && !use32;
      if (prof) AES_HIP(hipEventRecord(h_->event(2 * n_events_), s_));
      if (use32)
        launch_hv_fused<float>(A32_, n_, d_, d_, v, part_, spart_, nwg_, s_, gate);
      else
        launch_hv_fused<double>(P_.A, n_, d_, P_.lda, v, part_, spart_, nwg_, s_, gate);
      if (prof) {
        AES_HIP(hipEventRecord(h_->event(2 * n_events_ + 1), s_));
        ++n_events_;
      }
      launch_hv_colsum(part_, nwg_, d_, 1, v, lam_, nu2_, sgn, bb, bsgn, out, s_, gate);
    } else if (C_ == 1 && !use32) {
      // wider than the fused pass: z = A v, then the row-block partials of A^T z (two streaming
      // passes over A), summed in a fixed order
      launch_rowdot(n_, d_, P_.A, P_.lda, 0, v, 1, nullptr, 1.0, nullptr, nullptr, 1.0, Z_, s_);
      launch_atz(P_.A, n_, d_, P_.lda, Z_, atz_part_, atz_nrb_, atz_rows_, s_);
      launch_hv_colsum(atz_part_, atz_nrb_, d_, 1, v, lam_, nu2_, sgn, bb, bsgn, out, s_);
    } else if (use32) {
      // FP32 storage and MFMA: Z = A V (n x C), partial Q_w = A_w^T Z_w over row blocks
      narrow_f64(d_ * C_, v, V32_, s_);
      gemm_f32(false, false, n_, C_, d_, 1.0, A32_, d_, 0, V32_, C_, 0, 0.0, Z32_, C_, 0, 1, 0, s_);
      const int full = (int)(n_ / msplit_rows_);
      if (full > 0)
        gemm_f32(true, false, d_, C_, msplit_rows_, 1.0, A32_, d_, msplit_rows_ * d_, Z32_, C_, msplit_rows_ * C_, 0.0,
                 part32_, C_, d_ * C_, full, 0, s_);
      const int64_t tail = n_ - (int64_t)full * msplit_rows_;
      int used = full;
      if (tail > 0) {
        gemm_f32(true, false, d_, C_, tail, 1.0, A32_ + (int64_t)full * msplit_rows_ * d_, d_, 0,
                 Z32_ + (int64_t)full * msplit_rows_ * C_, C_, 0, 0.0, part32_ + (int64_t)full * d_ * C_, C_, 0, 1, 0,
                 s_);
        ++used;
      }
      launch_hv_colsum_f32(part32_, used, d_, C_, v, lam_, nu2_, sgn, bb, bsgn, out, s_);
    } else {
      // Z = A V (n x C); partial Q_w = A_w^T Z_w over row splits; fixed-order column sum.
      gemm_f64(false, false, n_, C_, d_, 1.0, P_.A, P_.lda, 0, v, C_, 0, 0.0, Z_, C_, 0, 1, 0, s_);
      const int full = (int)(n_ / msplit_rows_);
      if (full > 0)
        gemm_f64(true, false, d_, C_, msplit_rows_, 1.0, P_.A, P_.lda, msplit_rows_ * P_.lda, Z_, C_,
                 msplit_rows_ * C_, 0.0, part_, C_, d_ * C_, full, 0, s_);
      const int64_t tail = n_ - (int64_t)full * msplit_rows_;
      int used = full;
      if (tail > 0) {
        gemm_f64(true, false, d_, C_, tail, 1.0, P_.A + (int64_t)full * msplit_rows_ * P_.lda, P_.lda, 0,
                 Z_ + (int64_t)full * msplit_rows_ * C_, C_, 0, 0.0, part_ + (int64_t)full * d_ * C_, C_, 0, 1, 0, s_);
        ++used;
      }
      launch_hv_colsum(part_, used, d_, C_, v, lam_, nu2_, sgn, bb, bsgn, out, s_);
    }
    ++a_passes_;
  }

  // ---- sketch + factorisation of H_S (Sec. 4.1) ----------------------------------------
  void sketch_factor() {
    PhaseRange range("aes sketch+factor");
    {
      std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
      AES_HIP(hipEventCreate(&ev.first));
      AES_HIP(hipEventCreate(&ev.second));
      sk_ev_.push_back(ev);
      AES_HIP(hipEventRecord(ev.first, s_));
    }
    const bool low = o_.sketch == AES_SRHT || o_.sketch == AES_SJLT;  // sketches of the FP32 copy
    const bool bf = mixed_ && !sketch32_ && low;
    const bool f32 = mixed_ && sketch32_ && low;
    woodbury_ = m_ < d_;
    if (bf) {
      SA16_ = S<__hip_bfloat16>("SA16", (size_t)m_ * d_);
    } else if (f32) {
      SA32_ = S<float>("SA32", (size_t)m_ * d_);
    } else {
      // the sketch itself is kept for the Woodbury form's products; for m >= d only its Gram is
      SA_ = woodbury_ ? B<double>("SA", (size_t)m_ * d_) : S<double>("SAg", (size_t)m_ * d_);
    }
    if (o_.sketch == AES_SRHT_REUSE || o_.sketch == AES_SRHT_NESTED) {
      // transform-reuse variants: Y = (H / sqrt(n')) E_0 A_pad once per solve (the SRHT of
      // index 0 at m = n', every row kept in order), then rows R_k of Y scaled by sqrt(n'/m);
      // nested: the first m rows of Y in key order (the key order is sorted once per solve)
      SelectScratch sc;
      sc.keys = S<uint64_t>("sel_keys", npad_);
      sc.pos = S<int32_t>("sel_pos", npad_);
      sc.hist = S<uint32_t>("sel_hist", 256 * 8);
      sc.state = S<uint64_t>("sel_state", 4);
      sc.blk = S<uint32_t>("sel_blk", 2 * select_blocks(npad_));
      if (!yr_ready_) {
        double* eps = S<double>("eps", n_);
        launch_signs(o_.seed, o_.problem, 0, n_, eps, s_);
        launch_srht_select(o_.seed, o_.problem, 0, npad_, npad_, sc, s_);
        yr_ = B<double>("Yreuse", (size_t)npad_ * d_);
        launch_srht_apply<double, double, double>(P_.A, n_, d_, P_.lda, eps, npad_, sc.pos, npad_,
                                                  S<double>("Y", srht_scratch_elems(npad_, d_)), yr_, d_,
                                                  S<int32_t>("need", 512), s_);
        if (o_.sketch == AES_SRHT_NESTED) {
          korder_ = B<int32_t>("nest_order", npad_);
          launch_srht_key_order(o_.seed, o_.problem, npad_, key_order_scratch(), korder_, s_);
          gnest_m_ = 0;
        }
        yr_ready_ = true;
      }
      const double scale = std::sqrt((double)npad_ / (double)m_);
      if (o_.sketch == AES_SRHT_NESTED) {
        launch_gather_ordered(m_, d_, yr_, korder_, scale, SA_, d_, s_);
      } else {
        launch_srht_select(o_.seed, o_.problem, k_, npad_, m_, sc, s_);
        launch_gather_rows(npad_, d_, yr_, sc.pos, scale, SA_, d_, s_);
      }
    } else if (o_.sketch == AES_SRHT && spec_pending_ && spec_k_ == k_ && spec_m_ == m_) {
      // this resize's sketch (same seed, index, size and type) was formed ahead on the side stream
      AES_HIP(hipStreamWaitEvent(s_, spec_done_, 0));
      if (bf)
        SA16_ = static_cast<__hip_bfloat16*>(spec_out_);
      else if (f32)
        SA32_ = static_cast<float*>(spec_out_);
      else
        SA_ = static_cast<double*>(spec_out_);
      spec_cur_ = spec_tgt_;
      spec_pending_ = false;
    } else if (o_.sketch == AES_SRHT) {
      double* eps = S<double>("eps", n_);
      launch_signs(o_.seed, o_.problem, k_, n_, eps, s_);
      SelectScratch sc;
      sc.keys = S<uint64_t>("sel_keys", npad_);
      sc.pos = S<int32_t>("sel_pos", npad_);
      sc.hist = S<uint32_t>("sel_hist", 256 * 8);
      sc.state = S<uint64_t>("sel_state", 4);
      sc.blk = S<uint32_t>("sel_blk", 2 * select_blocks(npad_));
      launch_srht_select(o_.seed, o_.problem, k_, npad_, m_, sc, s_);
      if (bf) {
        float* Y = S<float>("Y32", srht_scratch_elems(npad_, d_));
        launch_srht_apply<float, float, __hip_bfloat16>(A32_, n_, d_, d_, eps, npad_, sc.pos, m_, Y, SA16_, d_,
                                                        S<int32_t>("need", 512), s_);
      } else if (f32) {
        float* Y = S<float>("Y32", srht_scratch_elems(npad_, d_));
        launch_srht_apply<float, float, float>(A32_, n_, d_, d_, eps, npad_, sc.pos, m_, Y, SA32_, d_,
                                               S<int32_t>("need", 512), s_);
      } else {
        double* Y = S<double>("Y", srht_scratch_elems(npad_, d_));
        launch_srht_apply<double, double, double>(P_.A, n_, d_, P_.lda, eps, npad_, sc.pos, m_, Y, SA_, d_,
                                                  S<int32_t>("need", 512), s_);
      }
    } else if (o_.sketch == AES_SJLT) {
      const SjltPlan sp = sjlt_plan(n_, d_, m_, (bf || f32) ? sizeof(float) : sizeof(double));
      SjltScratch sc;
      sc.code = S<int32_t>("sj_code", n_);
      sc.cnt = S<int32_t>("sj_cnt", sp.count_elems);
      sc.csum = S<int32_t>("sj_csum", sp.csum_elems);
      sc.perm = S<int32_t>("sj_perm", n_);
      const size_t part = sp.Q > 1 ? (size_t)m_ * sp.Q * d_ : 0;
      if (bf) {
        sc.part = part ? S<float>("sj_part32", part) : nullptr;
        launch_sjlt<float, __hip_bfloat16>(sp, A32_, n_, d_, d_, m_, o_.seed, o_.problem, k_, SA16_, sc, s_);
      } else if (f32) {
        sc.part = part ? S<float>("sj_part32", part) : nullptr;
        launch_sjlt<float, float>(sp, A32_, n_, d_, d_, m_, o_.seed, o_.problem, k_, SA32_, sc, s_);
      } else {
        sc.part = part ? S<double>("sj_part", part) : nullptr;
        launch_sjlt<double, double>(sp, P_.A, n_, d_, P_.lda, m_, o_.seed, o_.problem, k_, SA_, sc, s_);
      }
    } else {
      const GaussPlan gp = gauss_plan(h_->num_cu, n_, d_, m_);
      launch_gauss_sketch(gp, P_.A, n_, d_, P_.lda, m_, o_.seed, o_.problem, k_, SA_, S<double>("gauss_gt", gp.gt_elems),
                          gp.part_elems ? S<double>("gauss_part", gp.part_elems) : nullptr, s_);
    }
    sketch_ahead(bf, f32);
    int* flag = B<int>("chol_flag", 1);  // read by the problem's next initialisation
    AES_HIP(hipMemsetAsync(flag, 0, sizeof(int), s_));
    factor_from_sa(bf ? 1 : (f32 ? 2 : 0), flag);
    // no wait here: the initialisation that follows copies the failure flag into the flag
    // block, which the host reads next
    chol_flag_ = flag;
    AES_HIP(hipEventRecord(sk_ev_.back().second, s_));
  }

  // SRHT solves of one problem: form the sketch of the next resize (index k + 1, size
  // min(2m, cap)) on a side stream while this resize's Gram, factorisation and the following
  // attempts run on the main one.  The sketch does not depend on the attempts, so a resize takes
  // it as it is (the same values a sketch at the resize would give); when no resize comes it is
  // discarded.  It writes one of two buffers in turn: the other holds the sketch in use, and the
  // one written last held the sketch of two resizes ago, whose readers have finished (the host
  // decided this resize after reading the flags of a later step).  Its scratch is its own; it is
  // used while the extra scratch fits in an eighth of the device's memory.
  void enable_sketch_ahead() {
    if (o_.sketch != AES_SRHT || !o_.adaptive || cg_) return;
    // the mixed modes sketch the FP32 copy (FP32 scratch) into BF16 (AES_MIXED) or FP32 output
    const double ey = mixed_ ? 4.0 : 8.0, es = !mixed_ ? 8.0 : (sketch32_ ? 4.0 : 2.0);
    const double bytes = ey * (double)srht_scratch_elems(npad_, d_) + 2.0 * es * (double)mcap_ * (double)d_;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return;
    spec_ok_ = bytes <= (double)total_b / kSketchAheadShare;
  }
  void sketch_ahead(bool bf, bool f32) {
    if (!spec_ok_ || m_ >= mcap_) return;
    const int64_t m2 = std::min<int64_t>(2 * m_, mcap_);
    if (!ss_) {
      AES_HIP(hipStreamCreateWithFlags(&ss_, hipStreamNonBlocking));
      AES_HIP(hipEventCreateWithFlags(&spec_go_, hipEventDisableTiming));
      AES_HIP(hipEventCreateWithFlags(&spec_done_, hipEventDisableTiming));
    }
    const int tgt = spec_cur_ == 0 ? 1 : 0;
    double* eps = S<double>("ahead_eps", n_);
    SelectScratch sc;
    sc.keys = S<uint64_t>("ahead_keys", npad_);
    sc.pos = S<int32_t>("ahead_pos", npad_);
    sc.hist = S<uint32_t>("ahead_hist", 256 * 8);
    sc.state = S<uint64_t>("ahead_state", 4);
    sc.blk = S<uint32_t>("ahead_blk", 2 * select_blocks(npad_));
    int32_t* need = S<int32_t>("ahead_need", 512);
    // ordered after everything enqueued on the main stream so far (the caller's writes of A, the
    // FP32 cast); this resize's Gram and factorisation come after this point and overlap it
    AES_HIP(hipEventRecord(spec_go_, s_));
    AES_HIP(hipStreamWaitEvent(ss_, spec_go_, 0));
    launch_signs(o_.seed, o_.problem, k_ + 1, n_, eps, ss_);
    launch_srht_select(o_.seed, o_.problem, k_ + 1, npad_, m2, sc, ss_);
    void* out;
    if (bf) {
      auto* o16 = B<__hip_bfloat16>(tgt ? "ahead_SA16_1" : "ahead_SA16_0", (size_t)m2 * d_);
      launch_srht_apply<float, float, __hip_bfloat16>(A32_, n_, d_, d_, eps, npad_, sc.pos, m2,
                                                      S<float>("ahead_Y32", srht_scratch_elems(npad_, d_)), o16, d_,
                                                      need, ss_);
      out = o16;
    } else if (f32) {
      auto* o32 = B<float>(tgt ? "ahead_SA32_1" : "ahead_SA32_0", (size_t)m2 * d_);
      launch_srht_apply<float, float, float>(A32_, n_, d_, d_, eps, npad_, sc.pos, m2,
                                             S<float>("ahead_Y32", srht_scratch_elems(npad_, d_)), o32, d_, need, ss_);
      out = o32;
    } else {
      auto* o64 = B<double>(tgt ? "ahead_SA1" : "ahead_SA0", (size_t)m2 * d_);
      launch_srht_apply<double, double, double>(P_.A, n_, d_, P_.lda, eps, npad_, sc.pos, m2,
                                                S<double>("ahead_Y", srht_scratch_elems(npad_, d_)), o64, d_, need,
                                                ss_);
      out = o64;
    }
    AES_HIP(hipEventRecord(spec_done_, ss_));
    spec_pending_ = true;
    spec_k_ = k_ + 1;
    spec_m_ = m2;
    spec_tgt_ = tgt;
    spec_out_ = out;
  }

  KeyOrderScratch key_order_scratch() {
    KeyOrderScratch k;
    k.keys = S<uint64_t>("ko_keys", npad_);
    k.cnt = S<uint32_t>("ko_cnt", npad_);
    k.cur = S<uint32_t>("ko_cur", npad_);
    k.off = S<uint32_t>("ko_off", npad_);
    k.bsum = S<uint32_t>("ko_bsum", keyorder_sum_elems(npad_));
    k.skey = S<uint64_t>("ko_skey", npad_);
    return k;
  }

  // Gram of the current sketch, its Cholesky factor and the inverse factor (Sec. 4.1).
  // sk: 0 FP64 sketch (SA_), 1 BF16 (SA16_), 2 FP32 (SA32_)
  void factor_from_sa(int sk, int* flag) {
    const bool bf = sk == 1;
    if (!woodbury_) {
      fp_ = round_up(d_, 64);
      double* G = S<double>("G", (size_t)fp_ * fp_);
      if (sk == 2) {
        // FP32 sketch, FP64 Gram: an FP32-accumulated Gram carries errors ~ u32 ||SA||^2,
        // above nu^2 Lambda once nu is small, and would not stay positive definite.
        SA_ = S<double>("SAg", (size_t)m_ * d_);
        widen_f32(m_ * d_, SA32_, SA_, s_);
        const int splits = gram_splits(h_->num_cu, m_, d_, true);
        double* part = S<double>("gram_part", (size_t)splits * fp_ * fp_);
        gram_tn(m_, d_, SA_, d_, nu2_, lam_, part, splits, G, fp_, s_);
      } else if (bf) {
        const int splits = gram_splits(h_->num_cu, m_, d_, false);
        float* part = S<float>("gram_part32", (size_t)splits * fp_ * fp_);
        gram_tn_bf16(m_, d_, SA16_, d_, nu2_, lam_, part, splits, G, fp_, s_);
      } else if (o_.sketch == AES_SRHT_NESTED) {
        // nested rows: the sketch of the last resize is the first gnest_m_ rows of this one (up
        // to its scale), so G = (gnest_m_ / m) G_last + the Gram of the new rows; the Gram
        // without the nu^2 Lambda term is kept for the next resize
        double* Gn = B<double>("nest_gram", (size_t)fp_ * fp_);
        const int64_t m0 = gnest_m_ > 0 && gnest_m_ < m_ ? gnest_m_ : 0;
        const int splits = gram_splits(h_->num_cu, m_ - m0, d_, true);
        double* part = S<double>("gram_part", (size_t)splits * fp_ * fp_);
        gram_tn(m_ - m0, d_, SA_ + m0 * d_, d_, nu2_, lam_, part, splits, G, fp_, s_, m0 ? Gn : nullptr,
                (double)m0 / (double)m_, Gn);
        gnest_m_ = m_;
      } else {
        const int splits = gram_splits(h_->num_cu, m_, d_, true);
        double* part = S<double>("gram_part", (size_t)splits * fp_ * fp_);
        gram_tn(m_, d_, SA_, d_, nu2_, lam_, part, splits, G, fp_, s_);
      }
      factor_and_invert(G, fp_, flag);
    } else {
      fp_ = round_up(m_, 64);
      double* W = S<double>("G", (size_t)fp_ * fp_);
      double* scaled = S<double>("sa_scaled", (size_t)m_ * d_);
      if (bf) {
        SA_ = B<double>("SA", (size_t)m_ * d_);
        gram_nt_bf16(m_, d_, SA16_, d_, nu2_, invlam_, SA_, scaled, W, fp_, s_);
      } else if (sk == 2) {
        SA_ = B<double>("SA", (size_t)m_ * d_);
        widen_f32(m_ * d_, SA32_, SA_, s_);
        gram_nt(m_, d_, SA_, d_, nu2_, invlam_, scaled, W, fp_, s_);
      } else {
        gram_nt(m_, d_, SA_, d_, nu2_, invlam_, scaled, W, fp_, s_);
      }
      factor_and_invert(W, fp_, flag);
      SAT_ = B<double>("SAT", (size_t)d_ * m_);
      launch_transpose(m_, d_, SA_, d_, SAT_, m_, s_);
    }
  }

  void factor_and_invert(double* G, int64_t np, int* flag) {
    Linv_ = B<double>("Linv", (size_t)np * np);
    LinvT_ = B<double>("LinvT", (size_t)np * np);
    double* tmp = S<double>("cholinv_tmp", cholinv_tmp_size(np));
    cholinv(G, np, Linv_, tmp, flag, false, s_);
    launch_transpose(np, np, Linv_, np, LinvT_, np, s_);
  }

  // v = H_S^{-1} z (z, v: d x C); the identity for the CG baseline
  void apply(const double* z, double* v, const int* gate = nullptr) {
    if (cg_) {
      launch_copy_cols(d_, C_, z, C_, C_, v, C_, s_, gate);
      return;
    }
    double* t1 = S<double>("ap_t1", (size_t)std::max(m_, d_) * C_);
    if (!woodbury_) {
      if (C_ >= 8) {
        // split-K skinny GEMMs over the padded factor (zero rows/columns beyond d)
        const int64_t np = fp_;
        int ns = 1;
        while (ns < 16 && np / (2 * ns) >= 128 && (np / (2 * ns)) % 64 == 0) ns *= 2;
        const int64_t Ks = np / ns;
        double* zp = S<double>("ap_zp", (size_t)np * C_);
        double* tp = S<double>("ap_tp", (size_t)np * C_);
        double* part = S<double>("ap_part", (size_t)ns * np * C_);
        if (np > d_) launch_fill(zp + d_ * C_, (np - d_) * C_, 0.0, s_);
        AES_HIP(hipMemcpyAsync(zp, z, d_ * C_ * sizeof(double), hipMemcpyDeviceToDevice, s_));
        gemm_f64(false, false, np, C_, Ks, 1.0, Linv_, np, Ks, zp, C_, Ks * C_, 0.0, part, C_, np * C_, ns, 0, s_, 1, Ks);
        launch_sum_parts(np * C_, ns, np * C_, part, tp, s_);
        gemm_f64(false, false, np, C_, Ks, 1.0, LinvT_, np, Ks, tp, C_, Ks * C_, 0.0, part, C_, np * C_, ns, 0, s_, 2, Ks);
        launch_sum_parts(d_ * C_, ns, np * C_, part, v, s_);
      } else {
        launch_rowdot(d_, d_, Linv_, fp_, 1, z, C_, nullptr, 1.0, nullptr, nullptr, 1.0, t1, s_, gate);
        launch_rowdot(d_, d_, LinvT_, fp_, 2, t1, C_, nullptr, 1.0, nullptr, nullptr, 1.0, v, s_, gate);
      }
    } else {
      double* u = S<double>("ap_u", (size_t)m_ * C_);
      double* w = S<double>("ap_w", (size_t)m_ * C_);
      launch_rowdot(m_, d_, SA_, d_, 0, z, C_, invlam_, 1.0, nullptr, nullptr, 1.0, u, s_, gate);
      launch_rowdot(m_, m_, Linv_, fp_, 1, u, C_, nullptr, 1.0, nullptr, nullptr, 1.0, t1, s_, gate);
      launch_rowdot(m_, m_, LinvT_, fp_, 2, t1, C_, nullptr, 1.0, nullptr, nullptr, 1.0, w, s_, gate);
      launch_rowdot(d_, m_, SAT_, m_, 0, w, C_, nullptr, -1.0, z, invlam_, 1.0 / nu2_, v, s_, gate);
    }
  }

  void read_flags() {
    AES_HIP(hipMemcpyAsync(pinned_, scal_ + 7 * C_, 8 * sizeof(double), hipMemcpyDeviceToHost, s_));
    AES_HIP(hipStreamSynchronize(s_));
    for (int i = 0; i < 8; ++i) fl_[i] = pinned_[i];
  }

  void trace(int64_t t, double lr, double thr, bool accept) {
    if (o_.trace && trace_len_ < o_.trace_cap) {
      aes_trace_entry& e = o_.trace[trace_len_++];
      e.t = t;
      e.m = m_;
      e.k = k_;
      e.log_ratio = lr;
      e.threshold = thr;
      e.accept = accept ? 1 : 0;
      e.pad_ = 0;
      e.dtilde = fl_[5];
      e.time_ms = now_ms() - t0_ms_;
    }
  }

  // ---- the adaptive loop --------------------------------------------------------------
  // Solves H x = rhs (device d x C), x initialised by the caller (x_is_zero tells whether
  // the initial point is 0).  Returns the status; fills the counters.
  aes_status adaptive(const double* rhs, double* x, bool x_is_zero, bool use32, int stop_rule, double stop_scale,
                      bool reuse_factor) {
    PhaseRange range("aes adaptive solve");
    // Polyak-IHS (heavy-ball appendix) runs the IHS step with momentum: mu_rho, beta_rho of the
    // corollary, x_prev = x_0 at the start and x_t after a resize; the test takes the
    // corollary's finite-time factor alpha(tau, rho) beta_rho^omega(tau) in place of phi^tau
    const bool polyak = o_.method == AES_POLYAK;
    const bool ihs = o_.method == AES_IHS || polyak;
    double phi, cc, mu = 0.0, beta = 0.0;
    const double sr = std::sqrt(o_.rho);
    if (ihs) {
      phi = o_.rho;
      cc = (1.0 + sr) / (1.0 - sr);
      mu = 1.0 - o_.rho;
      if (polyak) {
        const double q = std::sqrt(1.0 - o_.rho);
        mu = 2.0 * (1.0 - o_.rho) / (1.0 + q);
        beta = (1.0 - q) / (1.0 + q);
      }
    } else {
      const double q = std::sqrt(1.0 - o_.rho);
      phi = (1.0 - q) / (1.0 + q);
      cc = 4.0 * (1.0 + sr) / (1.0 - sr);
    }
    const double lphi = std::log(phi), lc = std::log(cc);
    auto thr_at = [&](int64_t tt, int64_t II) {
      return polyak ? lc + polyak_log_bound((double)(tt + 1 - II), beta) : thr_of(lc, lphi, tt, II);
    };
    // previous iterates of the heavy-ball step: step t reads xpv[t & 1] and writes x to xpv[(t+1) & 1]
    double* xpv[2] = {nullptr, nullptr};
    if (polyak) {
      xpv[0] = B<double>("XPV0", d_ * C_);
      xpv[1] = B<double>("XPV1", d_ * C_);
      AES_HIP(hipMemcpyAsync(xpv[0], x, d_ * C_ * sizeof(double), hipMemcpyDeviceToDevice, s_));
    }
    // With one right-hand side every kernel of a step is gated by a device word that the
    // previous step's finish (or the initialisation) sets when it accepted and has active
    // columns, so the next step is enqueued before the host has read the flags of the current
    // one; the host then reads them through an event on their own pinned slot.
    const bool spec = fused_;
    int* gate = spec ? B<int>("gate", 1) : nullptr;
    if (!reuse_factor && !cg_) sketch_factor();
    // initial residual / gradient
    if (ihs) {
      if (x_is_zero)
        launch_hv_colsum(nullptr, 0, d_, C_, x, lam_, 0.0, 0.0, rhs, -1.0, R_, s_);  // g = -b (no partials)
      else
        hv(x, R_, 1.0, rhs, -1.0, use32);  // g = H x - b
      apply(R_, Pv_);
      launch_ihs_init(d_, C_, R_, Pv_, scal_, active_, gate, stop_rule, stop_scale, stop_sr_, tol2_, x, 1, s_,
                      chol_flag_, vw_);
    } else {
      if (x_is_zero)
        AES_HIP(hipMemcpyAsync(R_, rhs, d_ * C_ * sizeof(double), hipMemcpyDeviceToDevice, s_));
      else
        hv(x, R_, -1.0, rhs, 1.0, use32);  // r = b - H x
      apply(R_, RTP_);
      launch_pcg_init(d_, C_, R_, RTP_, Pv_, scal_, active_, gate, stop_rule, stop_scale, stop_sr_, tol2_, x, 1, s_,
                      chol_flag_, vw_);
    }
    // Flags of an initialisation: read at once without speculation; with it, the first step is
    // enqueued behind the initialisation and its flags tell whether it ran (flag 7 = its
    // sequence number) or whether the initialisation closed the gate.
    bool after_init = true;
    auto check_init = [&]() -> aes_status {
      if (fl_[6] != 0.0) throw StatusError(AES_ERR_NOT_SPD, "Cholesky pivot of the sketched Hessian is not positive");
      return fl_[2] != 0.0 ? AES_ERR_NONFINITE : AES_OK;
    };
    if (!spec) {
      read_flags();
      if (check_init() != AES_OK) return AES_ERR_NONFINITE;
      after_init = false;
    }
    int64_t t = 0, I = 0;
    bool forced = false;
    double seq_ctr = 0.0;
    // one enqueued step: its index, forced-rejection flag, flag slot, first H.v event, stamp
    struct Step {
      int64_t t;
      int force;
      int slot;
      int64_t ev;
      double seq;
    };
    auto enqueue_step = [&](int64_t tt, int force, int slot) -> Step {
      const double thr = thr_at(tt, I);
      const int at_cap = m_ >= mcap_ ? 1 : 0;
      const int64_t ev = (o_.profile && !use32 && fused_) ? n_events_ : -1;
      const double seq = spec ? (seq_ctr += 1.0) : -1.0;
      if (ihs) {
        launch_ihs_candidate(d_, C_, x, Pv_, mu, XP_, active_, s_, gate, polyak ? xpv[tt & 1] : nullptr, beta,
                             polyak ? xpv[(tt + 1) & 1] : nullptr);
        hv(XP_, RP_, 1.0, rhs, -1.0, use32, gate);
        apply(RP_, RTP_, gate);
        launch_ihs_finish(d_, C_, x, R_, Pv_, XP_, RP_, RTP_, scal_, active_, gate, thr, force, o_.adaptive, at_cap,
                          stop_rule, stop_scale, stop_sr_, tol2_, s_, seq, vw_);
      } else {
        hv(Pv_, Q_, 1.0, nullptr, 0.0, use32, gate);
        launch_pcg_candidate(d_, C_, fused_ ? spart_ : nullptr, nwg_, lam_, nu2_, x, R_, Pv_, Q_, XP_, RP_, scal_,
                             active_, s_, gate, vw_);
        apply(RP_, RTP_, gate);
        launch_pcg_finish(d_, C_, x, R_, Pv_, XP_, RP_, RTP_, scal_, active_, gate, thr, force, o_.adaptive, at_cap,
                          stop_rule, stop_scale, stop_sr_, tol2_, s_, seq, vw_);
      }
      if (spec) {
        AES_HIP(hipMemcpyAsync(pinned_ + 8 * slot, scal_ + 7 * C_, 8 * sizeof(double), hipMemcpyDeviceToHost, s_));
        AES_HIP(hipEventRecord(flag_event(slot), s_));
      }
      return Step{tt, force, slot, ev, seq};
    };
    // an enqueued step that did not run: its pass and timing event do not count
    auto discard = [&](const Step& st) {
      --a_passes_;
      if (st.ev >= 0) skip_events_.push_back(st.ev);
    };
    auto force_at = [&](int64_t tt, bool already) {
      return (o_.adaptive && o_.force_reject_at >= 0 && tt == o_.force_reject_at && !already) ? 1 : 0;
    };
    bool have_next = false;
    Step next{};
    for (;;) {
      if (!after_init && fl_[1] <= 0.5) break;  // every column stopped
      if (t >= o_.max_iter) {
        if (have_next) discard(next);
        if (after_init) {
          read_flags();
          if (check_init() != AES_OK) return AES_ERR_NONFINITE;
          if (fl_[1] <= 0.5) break;
        }
        return stop_rule == AES_STOP_FIXED ? AES_OK : AES_ERR_MAX_ITER;
      }
      Step cur = have_next ? next : enqueue_step(t, force_at(t, forced), (int)(t & 1));
      have_next = false;
      if (spec && t + 1 < o_.max_iter) {
        // enqueue step t+1 as if step t is accepted (its force flag as the host would decide it)
        next = enqueue_step(t + 1, force_at(t + 1, forced || cur.force != 0), (int)((t + 1) & 1));
        have_next = true;
      }
      if (spec) {
        AES_HIP(hipEventSynchronize(flag_event(cur.slot)));
        for (int i = 0; i < 8; ++i) fl_[i] = pinned_[8 * cur.slot + i];
        if (fl_[7] != cur.seq) {
          // the initialisation before this step closed the gate: its own flags are in the block
          discard(cur);
          if (have_next) discard(next);
          have_next = false;
          if (check_init() != AES_OK) return AES_ERR_NONFINITE;
          break;  // stopped at the initialisation
        }
      } else {
        read_flags();
      }
      after_init = false;
      if (cur.force) forced = true;
      ++attempts_;
      const bool fail = fl_[0] != 0.0, accepted = fl_[3] != 0.0;
      trace(t, fl_[4], thr_at(t, I), accepted);
      if (fl_[2] != 0.0) {
        if (have_next) discard(next);
        return AES_ERR_NONFINITE;
      }
      if (accepted) {
        ++t;
        ++iters_;
        if (fail && o_.adaptive) m_cap_reached_ = 1;
        if (stop_rule == AES_STOP_FIXED && t >= o_.max_iter) {
          if (have_next) discard(next);
          return AES_OK;
        }
        if (fl_[1] <= 0.5 && have_next) {
          discard(next);  // stopped: the gate kept step t+1 from running
          have_next = false;
        }
        continue;
      }
      // rejected (the gate kept a speculative step t+1 from running): double m, fresh sketch,
      // restart at x_t (Algorithm 2 / Algorithm 1)
      if (have_next) {
        discard(next);
        have_next = false;
      }
      I = t;
      m_ = std::min<int64_t>(2 * m_, mcap_);
      ++k_;
      ++resketches_;
      sketch_factor();
      if (polyak)  // the momentum restarts at x_t with the new sketch
        AES_HIP(hipMemcpyAsync(xpv[t & 1], x, d_ * C_ * sizeof(double), hipMemcpyDeviceToDevice, s_));
      if (ihs) {
        apply(R_, Pv_);
        launch_ihs_init(d_, C_, R_, Pv_, scal_, active_, gate, stop_rule, stop_scale, stop_sr_, tol2_, x, 0, s_,
                        chol_flag_, vw_);
      } else {
        if (x_is_zero && t == 0)
          AES_HIP(hipMemcpyAsync(R_, rhs, d_ * C_ * sizeof(double), hipMemcpyDeviceToDevice, s_));
        else
          hv(x, R_, -1.0, rhs, 1.0, use32);  // explicit r_t = b - H x_t
        apply(R_, RTP_);
        launch_pcg_init(d_, C_, R_, RTP_, Pv_, scal_, active_, gate, stop_rule, stop_scale, stop_sr_, tol2_, x, 0, s_,
                        chol_flag_, vw_);
      }
      if (!spec) {
        read_flags();
        if (check_init() != AES_OK) return AES_ERR_NONFINITE;
      } else {
        after_init = true;
      }
    }
    if (have_next) discard(next);
    return AES_OK;
  }

  static double thr_of(double lc, double lphi, int64_t t, int64_t I) { return lc + (double)(t + 1 - I) * lphi; }
  // log of alpha(tau, rho) beta^omega(tau): nu = log2(tau) + 1, omega = tau - 2 nu,
  // alpha = 3^(nu (nu + 1)) (1 + 4 beta + beta^2)^(2 nu) (Polyak-IHS corollary)
  static double polyak_log_bound(double tau, double beta) {
    const double nu = std::log(tau) / std::log(2.0) + 1.0;
    const double la = nu * (nu + 1.0) * std::log(3.0) + 2.0 * nu * std::log(1.0 + 4.0 * beta + beta * beta);
    return la + (tau - 2.0 * nu) * std::log(beta);
  }

  hipEvent_t flag_event(int slot) {
    if (!fev_[slot]) AES_HIP(hipEventCreateWithFlags(&fev_[slot], hipEventDisableTiming));
    return fev_[slot];
  }

  aes_status run(aes_info* info, bool reuse_factor = false) {
    const double t0 = now_ms();
    aes_status st = AES_OK;
    try {
      setup_common();
      if (!reuse_factor) {
        m_ = cg_ ? 0 : std::min<int64_t>(o_.m_init, mcap_);
        k_ = 0;
      }
      const bool x0 = o_.x0 != nullptr;
      if (x0)
        launch_copy_cols(d_, C_, o_.x0, P_.ldx, (int)c_, X_, C_, s_);
      else
        AES_HIP(hipMemsetAsync(X_, 0, d_ * C_ * sizeof(double), s_));
      if (!mixed_) {
        st = adaptive(Bv_, X_, !x0, false, o_.stop, stop_scale_, reuse_factor);
      } else {
        st = run_mixed(x0);
      }
      if (st == AES_OK || st == AES_ERR_MAX_ITER || st == AES_ERR_NONFINITE)
        launch_copy_cols(d_, (int)c_, X_, C_, (int)c_, P_.x, P_.ldx, s_);
      AES_HIP(hipStreamSynchronize(s_));
    } catch (const StatusError& e) {
      st = e.st;
      h_->set_err(e.what());
    } catch (const HipError& e) {
      st = AES_ERR_HIP;
      h_->set_err(e.what());
    } catch (const std::bad_alloc&) {
      st = AES_ERR_OOM;
      h_->set_err("device workspace allocation failed");
    } catch (const std::invalid_argument& e) {
      st = AES_ERR_INVALID_ARG;
      h_->set_err(e.what());
    }
    // a sketch formed ahead for a resize that did not come still reads A: finish it before the
    // call returns
    if (ss_ && hipStreamSynchronize(ss_) != hipSuccess && st == AES_OK) st = AES_ERR_HIP;
    double hv_ms = 0.0;
    int64_t hv_n = 0;
    if (o_.profile && st != AES_ERR_HIP) {
      for (int64_t i = 0; i < n_events_; ++i) {
        if (std::find(skip_events_.begin(), skip_events_.end(), i) != skip_events_.end()) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h_->events[2 * i], h_->events[2 * i + 1]) == hipSuccess) {
          hv_ms += ms;
          ++hv_n;
        }
      }
    }
    if (info) {
      info->time_hv_ms = hv_ms;
      info->hv_launches = hv_n;
      info->iterations = iters_;
      info->attempts = attempts_;
      info->final_m = m_;
      info->resketches = resketches_;
      info->a_passes = a_passes_;
      info->refine_sweeps = sweeps_;
      info->trace_len = trace_len_;
      info->dtilde_final = fl_[5];
      double sk_ms = 0.0;
      if (st != AES_ERR_HIP)
        for (auto& e : sk_ev_) {
          float ms = 0.f;
          if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) sk_ms += ms;
        }
      info->time_sketch_ms = sk_ms;
      info->time_total_ms = now_ms() - t0;
      info->m_cap_reached = m_cap_reached_;
      info->status = st;
    }
    return st;
  }

  // Mixed precision: outer FP64 residual refinement around inner adaptive PCG/IHS solves
  // on the FP32-stored A with the BF16 sketch; the sketch state persists across sweeps.
  aes_status run_mixed(bool x0) {
    const int64_t dc = d_ * C_;
    double* E = B<double>("E", dc);
    double* Rr = B<double>("Rres", dc);
    double* nrm = B<double>("nrm", 2 * C_);
    bool first = true;
    bool x_zero = !x0;
    corr_ratio_ = 1.0;
    m_ = std::min<int64_t>(o_.m_init, mcap_);
    k_ = 0;
    const double inner = o_.inner_tol > 0 ? o_.inner_tol : 1e-6;
    double eta = inner;  // relative tolerance of the current inner solve
    std::vector<int> act(C_, 0);
    for (int j = 0; j < c_; ++j) act[j] = 1;
    std::vector<double> hn(2 * C_);
    for (int sweep = 0; sweep < std::max(1, o_.max_refine); ++sweep) {
      PhaseRange range("aes refinement sweep");
      ++sweeps_;
      // r = b - H x with the FP64 matrix (compensated once x is close)
      if (x_zero)
        AES_HIP(hipMemcpyAsync(Rr, Bv_, dc * sizeof(double), hipMemcpyDeviceToDevice, s_));
      else
        refine_residual(X_, Bv_, Rr);
      AES_HIP(hipMemsetAsync(E, 0, dc * sizeof(double), s_));
      AES_HIP(hipMemcpyAsync(active_, act.data(), C_ * sizeof(int), hipMemcpyHostToDevice, s_));
      aes_status st = adaptive(Rr, E, true, true, AES_STOP_XREL, nu2_ * min_lambda() * eta * eta, !first);
      first = false;
      if (st == AES_ERR_NONFINITE) return st;
      launch_axpy_cols(d_, C_, X_, E, nullptr, s_);
      x_zero = false;
      // per column: stop when ||e|| <= tol ||x|| / 4
      launch_colnorm2(d_, C_, E, X_, nrm, s_);
      AES_HIP(hipMemcpyAsync(hn.data(), nrm, 2 * C_ * sizeof(double), hipMemcpyDeviceToHost, s_));
      AES_HIP(hipStreamSynchronize(s_));
      bool done = true;
      corr_ratio_ = 0.0;
      for (int j = 0; j < c_; ++j) {
        const double en = std::sqrt(hn[j]), xn = std::sqrt(hn[C_ + j]);
        const bool ok = en <= 0.25 * tol_ * xn || xn == 0.0;
        if (act[j] && xn > 0.0) corr_ratio_ = std::max(corr_ratio_, en / xn);
        act[j] = ok ? 0 : 1;
        done = done && ok;
      }
      if (done) return AES_OK;
      eta = next_inner_tol(inner, eta);
    }
    return AES_ERR_MAX_ITER;
  }

  // Factorise H_S for a caller-given sketch SA (m x d, ld d) and apply it to z (d x C).
  void apply_external(int64_t m, const double* SA, const double* z, double* v) {
    lam_ = B<double>("lam", d_);
    invlam_ = B<double>("invlam", d_);
    if (P_.lambda) {
      AES_HIP(hipMemcpyAsync(lam_, P_.lambda, d_ * sizeof(double), hipMemcpyDeviceToDevice, s_));
      launch_inv(d_, P_.lambda, invlam_, s_);
    } else {
      launch_fill(lam_, d_, 1.0, s_);
      launch_fill(invlam_, d_, 1.0, s_);
    }
    m_ = m;
    woodbury_ = m_ < d_;
    SA_ = B<double>("SA", (size_t)m_ * d_);
    AES_HIP(hipMemcpyAsync(SA_, SA, (size_t)m_ * d_ * sizeof(double), hipMemcpyDeviceToDevice, s_));
    int* flag = B<int>("chol_flag", 1);
    AES_HIP(hipMemsetAsync(flag, 0, sizeof(int), s_));
    factor_from_sa(0, flag);
    int hflag = 0;
    AES_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s_));
    AES_HIP(hipStreamSynchronize(s_));
    if (hflag) throw StatusError(AES_ERR_NOT_SPD, "Cholesky pivot of the sketched Hessian is not positive");
    apply(z, v);
  }

  // Q = H P for the caller's P (d x C) without a solve (kernel-level entry point).
  void hv_external(const double* Pin, double* Qout, bool use32) {
    setup_common();
    hv(Pin, Qout, 1.0, nullptr, 0.0, use32);
  }
  void set_pinned(double* p) { pinned_ = p; }

  // ---- batch mode ----------------------------------------------------------------------
  // The steps of the adaptive loop run in the grouped kernels of a BatchEngine (one launch
  // sequence for all problems of a batch); this solver keeps the problem's control: the
  // (re)initialisations, resizes and restarts (Algorithm 2 / Algorithm 1), the refinement
  // sweeps of the mixed modes, the counters and the trace.
  enum BState { kBStep = 0, kBRefine = 1, kBDone = 2 };

  void batch_begin() {
    setup_common();
    // fixed addresses for the grouped step: the inverse factors at their largest padded size
    // (both branches: round_up(min(m, d), 64) <= round_up(d, 64)), the Woodbury operands at
    // d x d (m < d there), the products' intermediates
    const int64_t npm = round_up(d_, 64);
    (void)B<double>("Linv", (size_t)npm * npm);
    (void)B<double>("LinvT", (size_t)npm * npm);
    (void)B<double>("SA", (size_t)d_ * d_);
    (void)B<double>("SAT", (size_t)d_ * d_);
    bu_ = B<double>("bap_u", (size_t)d_ * C_);
    bt1_ = B<double>("bap_t1", (size_t)d_ * C_);
    bw_ = B<double>("bap_w", (size_t)d_ * C_);
    gate_ = B<int>("gate", 1);
    bihs_ = o_.method == AES_IHS || o_.method == AES_POLYAK;
    bpolyak_ = o_.method == AES_POLYAK;
    const double sr = std::sqrt(o_.rho);
    if (bihs_) {
      blphi_ = std::log(o_.rho);
      blc_ = std::log((1.0 + sr) / (1.0 - sr));
      bmu_ = 1.0 - o_.rho;
      if (bpolyak_) {
        const double q = std::sqrt(1.0 - o_.rho);
        bmu_ = 2.0 * (1.0 - o_.rho) / (1.0 + q);
        bbeta_ = (1.0 - q) / (1.0 + q);
      }
    } else {
      const double q = std::sqrt(1.0 - o_.rho);
      blphi_ = std::log((1.0 - q) / (1.0 + q));
      blc_ = std::log(4.0 * (1.0 + sr) / (1.0 - sr));
    }
    if (bpolyak_) {
      bxpv_[0] = B<double>("XPV0", d_ * C_);
      bxpv_[1] = B<double>("XPV1", d_ * C_);
    }
    m_ = cg_ ? 0 : std::min<int64_t>(o_.m_init, mcap_);
    k_ = 0;
    const bool x0 = o_.x0 != nullptr;
    if (x0)
      launch_copy_cols(d_, C_, o_.x0, P_.ldx, (int)c_, X_, C_, s_);
    else
      launch_fill(X_, d_ * C_, 0.0, s_);
    if (!mixed_) {
      inner_begin(Bv_, X_, !x0, false, o_.stop, stop_scale_, false);
    } else {
      bE_ = B<double>("E", d_ * C_);
      bRr_ = B<double>("Rres", d_ * C_);
      bnrm_ = B<double>("nrm", 2 * C_);
      bact_.assign(C_, 0);
      for (int j = 0; j < c_; ++j) bact_[j] = 1;
      const double inner = o_.inner_tol > 0 ? o_.inner_tol : 1e-6;
      binner_eta_ = inner;
      binner_scale_ = nu2_ * min_lambda() * inner * inner;
      bxzero_ = !x0;
      sweep_begin(true);
    }
  }

  // Start an inner adaptive solve of H x = rhs (Algorithm 2 / Algorithm 1): sketch and factor
  // unless the current factorisation is kept, then the initial residual and decrement.
  void inner_begin(const double* rhs, double* x, bool x_zero, bool use32, int stop_rule, double stop_scale,
                   bool reuse) {
    brhs_ = rhs;
    bx_ = x;
    bx_zero_ = x_zero;
    buse32_ = use32;
    bstop_ = stop_rule;
    bscale_ = stop_scale;
    bt_ = 0;
    bI_ = 0;
    bforced_ = false;
    if (bpolyak_) AES_HIP(hipMemcpyAsync(bxpv_[0], x, d_ * C_ * sizeof(double), hipMemcpyDeviceToDevice, s_));
    if (!reuse && !cg_) sketch_factor();
    binit(true);
    bstate_ = kBStep;
  }

  // (Re)initialisation at x after a factorisation: g or r, the preconditioned direction, D.
  void binit(bool first) {
    if (bihs_) {
      if (bx_zero_ && first)
        launch_hv_colsum(nullptr, 0, d_, C_, bx_, lam_, 0.0, 0.0, brhs_, -1.0, R_, s_);  // g = -b (no partials)
      else if (first)
        hv(bx_, R_, 1.0, brhs_, -1.0, buse32_);  // g = H x - b
      apply(R_, Pv_);
      launch_ihs_init(d_, C_, R_, Pv_, scal_, active_, gate_, bstop_, bscale_, stop_sr_, tol2_, bx_, first ? 1 : 0,
                      s_, chol_flag_, vw_);
    } else {
      if (bx_zero_ && bt_ == 0)
        AES_HIP(hipMemcpyAsync(R_, brhs_, d_ * C_ * sizeof(double), hipMemcpyDeviceToDevice, s_));
      else
        hv(bx_, R_, -1.0, brhs_, 1.0, buse32_);  // explicit r_t = b - H x_t
      apply(R_, RTP_);
      launch_pcg_init(d_, C_, R_, RTP_, Pv_, scal_, active_, gate_, bstop_, bscale_, stop_sr_, tol2_, bx_,
                      first ? 1 : 0, s_, chol_flag_, vw_);
    }
  }

  // One refinement sweep of the mixed modes: r = b - H x in FP64, then the inner solve of H e = r.
  void sweep_begin(bool first) {
    ++sweeps_;
    if (first) corr_ratio_ = 1.0;
    const int64_t dc = d_ * C_;
    if (bxzero_)
      AES_HIP(hipMemcpyAsync(bRr_, Bv_, dc * sizeof(double), hipMemcpyDeviceToDevice, s_));
    else
      refine_residual(X_, Bv_, bRr_);
    launch_fill(bE_, dc, 0.0, s_);
    AES_HIP(hipMemcpyAsync(active_, bact_.data(), C_ * sizeof(int), hipMemcpyHostToDevice, s_));
    inner_begin(bRr_, bE_, true, true, AES_STOP_XREL, binner_scale_, !first);
  }

  // The refinement residual r = b - H x with the FP64 matrix.  While the last correction was
  // larger than kCompensateBelow ||x|| in some column, x is still far from the solution and the
  // residual far above the rounding error of a plain FP64 product (about d u ||A||^2 ||x||), so the
  // plain product (one pass) gives all the digits the next inner solve can use; once every column's
  // correction is below that, the residual is formed in compensated arithmetic.
  static constexpr double kCompensateBelow = 1e-4;
  static constexpr double kCertifyTol = 0.1;
  // Relative tolerance of the next inner solve after a sweep run at `eta` that did not stop:
  // `inner`, or kCertifyTol for a sweep that only has to confirm convergence (the last correction
  // times its tolerance, the expected error of x, is already a tenth of the stop threshold; if x
  // is less accurate than that, the sweep's correction fails the stop test and a full sweep
  // follows).
  double next_inner_tol(double inner, double eta) const {
    return corr_ratio_ * eta <= 0.025 * tol_ ? std::max(inner, kCertifyTol) : inner;
  }
  void refine_residual(const double* x, const double* b, double* r) {
    if (corr_ratio_ > kCompensateBelow)
      hv(x, r, -1.0, b, 1.0, false);
    else
      residual_fp64(x, b, r);
  }

  // r = b - H x with the FP64 matrix in compensated arithmetic (the refinement residual: the
  // explicit residual of Algorithm 2 formed as in twice the working precision); two reads of A
  void residual_fp64(const double* x, const double* b, double* r) {
    double* zh = S<double>("rz_h", (size_t)n_ * C_);
    double* zl = S<double>("rz_l", (size_t)n_ * C_);
    const size_t pe = residual_dd_part_elems(h_->num_cu, n_, d_, C_);
    double* ph = S<double>("rp_h", pe);
    double* pl = S<double>("rp_l", pe);
    launch_residual_dd(h_->num_cu, n_, d_, C_, P_.A, P_.lda, b, C_, P_.nu, P_.lambda ? lam_ : nullptr, x, zh, zl, ph,
                       pl, r, C_, s_);
    a_passes_ += 2;
  }

  // Set-up for timing the grouped H.P alone (no sketch, no solve): buffers and an open gate.
  void batch_tune_setup() {
    setup_common();
    gate_ = B<int>("gate", 1);
    bx_ = X_;
    brhs_ = Bv_;
    launch_fill(X_, d_ * C_, 0.0, s_);
    launch_fill(Pv_, d_ * C_, 1.0, s_);
    AES_HIP(hipMemsetAsync(gate_, 0xff, sizeof(int), s_));  // nonzero: the gate is open
  }

  bool batch_fp32() const { return mixed_; }
  bool batch_ihs() const { return bihs_; }
  int64_t batch_n() const { return n_; }
  int64_t batch_d() const { return d_; }
  int batch_C() const { return C_; }
  int bstate() const { return bstate_; }
  aes_status bstatus() const { return bstatus_; }

  // Operands of the grouped step.  Ahp: the matrix the step multiplies by (FP32 copy or FP64).
  // kpad: length of the rows of the transposed operand (the fused form's column-block width)
  void batch_fill(BProb& bp, double* flags_out, int nrb, int64_t rows, bool twopass, int64_t kpad) {
    const bool f32 = mixed_;
    const size_t es = f32 ? sizeof(float) : sizeof(double);
    const int NC = C_ < 16 ? 16 : C_;
    bp = BProb{};
    bp.A = f32 ? (const void*)A32_ : (const void*)P_.A;
    bp.lda = f32 ? d_ : P_.lda;
    bp.n = n_;
    bp.d = d_;
    bp.C = C_;
    bp.nrb = nrb;
    bp.rows = rows;
    bp.kpad = kpad;
    bp.VT = h_->buf<unsigned char>(ns_ + "bVT", (size_t)NC * bp.kpad * es);
    bp.Z = twopass ? h_->buf<unsigned char>(ns_ + "bZ", (size_t)n_ * NC * es) : nullptr;
    bp.part = h_->buf<unsigned char>(ns_ + "bpart", (size_t)nrb * d_ * C_ * es);
    bp.lam = lam_;
    bp.nu2 = nu2_;
    bp.X = bx_;  // the iterate of the inner solve (the correction E in the mixed modes)
    bp.R = R_;
    bp.P = Pv_;
    bp.Q = Q_;
    bp.XP = XP_;
    bp.RP = RP_;
    bp.RTP = RTP_;
    bp.rhs = brhs_;
    bp.xpv0 = bxpv_[0];
    bp.xpv1 = bxpv_[1];
    bp.scal = scal_;
    bp.active = active_;
    bp.gate = gate_;
    bp.flags_out = flags_out;
    bp.mu = bmu_;
    bp.beta = bbeta_;
    bp.stop_sr = stop_sr_;
    bp.tol2 = tol2_;
    bp.stop_rule = bstop_;
    bp.adaptive = o_.adaptive;
  }
  // Step parameters (before every step of the batch).
  // ready: the problem's eager work (initialisation, resize) has completed; otherwise it sits
  // this step out and takes the next one
  void batch_dyn(BDyn& dy, bool ready) {
    dy = BDyn{};
    dy.run = (bstate_ == kBStep && ready) ? 1 : 0;
    if (!dy.run) return;
    dy.thr = bpolyak_ ? blc_ + polyak_log_bound((double)(bt_ + 1 - bI_), bbeta_) : thr_of(blc_, blphi_, bt_, bI_);
    bseq_ += 1.0;
    dy.seq = bseq_;
    dy.stop_scale = bscale_;
    dy.force = (o_.adaptive && o_.force_reject_at >= 0 && bt_ == o_.force_reject_at && !bforced_) ? 1 : 0;
    dy.at_cap = m_ >= mcap_ ? 1 : 0;
    dy.parity = (int)(bt_ & 1);
    // H_S^{-1} rp -> rtp: the products of the current branch (Sec. 4.1)
    auto prod = [](const double* mat, int64_t rows, int64_t K, int64_t ld, int tri, const double* in,
                   const double* xs, double ysgn, const double* zadd, const double* rs, double gs, double* out) {
      BProd p{};
      p.mat = mat;
      p.rows = rows;
      p.K = K;
      p.ld = ld;
      p.tri = tri;
      p.in = in;
      p.xs = xs;
      p.ysgn = ysgn;
      p.zadd = zadd;
      p.rs = rs;
      p.gs = gs;
      p.out = out;
      return p;
    };
    if (cg_) {
      dy.prod[0] = prod(nullptr, d_, 0, 0, 0, RP_, nullptr, 1.0, RP_, nullptr, 1.0, RTP_);  // identity
    } else if (!woodbury_) {
      dy.prod[0] = prod(Linv_, d_, d_, fp_, 1, RP_, nullptr, 1.0, nullptr, nullptr, 1.0, bt1_);
      dy.prod[1] = prod(LinvT_, d_, d_, fp_, 2, bt1_, nullptr, 1.0, nullptr, nullptr, 1.0, RTP_);
    } else {
      dy.prod[0] = prod(SA_, m_, d_, d_, 0, RP_, invlam_, 1.0, nullptr, nullptr, 1.0, bu_);
      dy.prod[1] = prod(Linv_, m_, m_, fp_, 1, bu_, nullptr, 1.0, nullptr, nullptr, 1.0, bt1_);
      dy.prod[2] = prod(LinvT_, m_, m_, fp_, 2, bt1_, nullptr, 1.0, nullptr, nullptr, 1.0, bw_);
      dy.prod[3] = prod(SAT_, d_, m_, m_, 0, bw_, nullptr, -1.0, RP_, invlam_, 1.0 / nu2_, RTP_);
    }
  }

  // Host side of a step (flags: the problem's flag block after the step).  Returns true when
  // the inner solve has ended and the mixed modes need their refinement check.
  bool batch_after(const double* fl) {
    beager_ = false;
    if (bstate_ != kBStep) return false;
    try {
      for (int i = 0; i < 8; ++i) fl_[i] = fl[i];
      if (fl_[7] != bseq_) {
        // the step did not run: the initialisation before it closed the gate
        if (fl_[6] != 0.0) throw StatusError(AES_ERR_NOT_SPD, "Cholesky pivot of the sketched Hessian is not positive");
        if (fl_[2] != 0.0) return bdone(AES_ERR_NONFINITE);
        return inner_end();
      }
      ++attempts_;
      ++a_passes_;
      const bool fail = fl_[0] != 0.0, accepted = fl_[3] != 0.0;
      const bool forced_now = o_.adaptive && o_.force_reject_at >= 0 && bt_ == o_.force_reject_at && !bforced_;
      if (forced_now) bforced_ = true;
      trace(bt_, fl_[4], bpolyak_ ? blc_ + polyak_log_bound((double)(bt_ + 1 - bI_), bbeta_) : thr_of(blc_, blphi_, bt_, bI_),
            accepted);
      if (fl_[2] != 0.0) return bdone(AES_ERR_NONFINITE);
      if (accepted) {
        ++bt_;
        ++iters_;
        if (fail && o_.adaptive) m_cap_reached_ = 1;
        if (fl_[1] <= 0.5) return inner_end();
        if (bt_ >= o_.max_iter) return at_max_iter();
        return false;
      }
      // rejected: double m, fresh sketch, restart at x_t
      beager_ = true;
      bI_ = bt_;
      m_ = std::min<int64_t>(2 * m_, mcap_);
      ++k_;
      ++resketches_;
      sketch_factor();
      if (bpolyak_) AES_HIP(hipMemcpyAsync(bxpv_[bt_ & 1], bx_, d_ * C_ * sizeof(double), hipMemcpyDeviceToDevice, s_));
      binit(false);
      return false;
    } catch (const StatusError& e) {
      h_->set_err(e.what());
      bdone(e.st);
    } catch (const HipError& e) {
      h_->set_err(e.what());
      bdone(AES_ERR_HIP);
    } catch (const std::bad_alloc&) {
      h_->set_err("device workspace allocation failed");
      bdone(AES_ERR_OOM);
    }
    return false;
  }

  // max_iter accepted steps: the FIXED rule's end, MAX_ITER otherwise; an inner solve of the
  // mixed modes ends its sweep instead (the refinement decides)
  bool at_max_iter() {
    if (mixed_) return inner_end();
    return bdone(bstop_ == AES_STOP_FIXED ? AES_OK : AES_ERR_MAX_ITER);
  }
  // Before a step: a problem already at max_iter (max_iter = 0) takes no step.
  bool batch_precheck() {
    if (bstate_ == kBStep && bt_ >= o_.max_iter) return at_max_iter();
    return false;
  }

  bool bdone(aes_status st) {
    bstatus_ = st;
    bstate_ = kBDone;
    return false;
  }

  // End of an inner solve: done (FP64), or the refinement update and its check (mixed).
  bool inner_end() {
    if (!mixed_) return bdone(AES_OK);
    launch_axpy_cols(d_, C_, X_, bE_, nullptr, s_);
    bxzero_ = false;
    launch_colnorm2(d_, C_, bE_, X_, bnrm_, s_);
    bstate_ = kBRefine;
    return true;
  }
  const double* batch_norms() const { return bnrm_; }
  // the last batch_after enqueued eager work (a resize and restart)
  bool batch_eager() const { return beager_; }

  // Refinement check (host copy of ||e||^2, ||x||^2 per column): stop when ||e|| <= tol ||x|| / 4.
  void batch_refine(const double* hn) {
    try {
      bool done = true;
      corr_ratio_ = 0.0;
      for (int j = 0; j < c_; ++j) {
        const double en = std::sqrt(hn[j]), xn = std::sqrt(hn[C_ + j]);
        const bool ok = en <= 0.25 * tol_ * xn || xn == 0.0;
        if (bact_[j] && xn > 0.0) corr_ratio_ = std::max(corr_ratio_, en / xn);
        bact_[j] = ok ? 0 : 1;
        done = done && ok;
      }
      if (done) {
        bdone(AES_OK);
        return;
      }
      if (sweeps_ >= std::max(1, o_.max_refine)) {
        bdone(AES_ERR_MAX_ITER);
        return;
      }
      binner_eta_ = next_inner_tol(o_.inner_tol > 0 ? o_.inner_tol : 1e-6, binner_eta_);
      binner_scale_ = nu2_ * min_lambda() * binner_eta_ * binner_eta_;
      sweep_begin(false);
    } catch (const StatusError& e) {
      h_->set_err(e.what());
      bdone(e.st);
    } catch (const HipError& e) {
      h_->set_err(e.what());
      bdone(AES_ERR_HIP);
    } catch (const std::bad_alloc&) {
      h_->set_err("device workspace allocation failed");
      bdone(AES_ERR_OOM);
    }
  }

  // Result and counters (after the batch has finished and the stream is idle).
  aes_status batch_result(aes_info* info, double t0) {
    aes_status st = bstatus_;
    try {
      if (st == AES_OK || st == AES_ERR_MAX_ITER || st == AES_ERR_NONFINITE)
        launch_copy_cols(d_, (int)c_, X_, C_, (int)c_, P_.x, P_.ldx, s_);
    } catch (const HipError& e) {
      h_->set_err(e.what());
      st = AES_ERR_HIP;
    }
    if (info) {
      info->time_hv_ms = 0.0;
      info->hv_launches = 0;
      info->iterations = iters_;
      info->attempts = attempts_;
      info->final_m = m_;
      info->resketches = resketches_;
      info->a_passes = a_passes_;
      info->refine_sweeps = sweeps_;
      info->trace_len = trace_len_;
      info->dtilde_final = fl_[5];
      double sk_ms = 0.0;
      if (st != AES_ERR_HIP)
        for (auto& e : sk_ev_) {
          float ms = 0.f;
          if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) sk_ms += ms;
        }
      info->time_sketch_ms = sk_ms;
      info->time_total_ms = now_ms() - t0;
      info->m_cap_reached = m_cap_reached_;
      info->status = st;
    }
    return st;
  }

  // accessors for the kept context
  int64_t m() const { return m_; }
  int64_t k() const { return k_; }
  void set_mk(int64_t m, int64_t k, bool woodbury, int64_t fp) {
    m_ = m;
    k_ = k;
    woodbury_ = woodbury;
    fp_ = fp;
  }
  void bind_factor() {
    // re-fetch kept factor buffers after setup (same names, same sizes)
    if (!woodbury_) {
      Linv_ = B<double>("Linv", (size_t)fp_ * fp_);
      LinvT_ = B<double>("LinvT", (size_t)fp_ * fp_);
    } else {
      Linv_ = B<double>("Linv", (size_t)fp_ * fp_);
      LinvT_ = B<double>("LinvT", (size_t)fp_ * fp_);
      SA_ = B<double>("SA", (size_t)m_ * d_);
      SAT_ = B<double>("SAT", (size_t)d_ * m_);
    }
  }
  bool woodbury() const { return woodbury_; }
  int64_t fp() const { return fp_; }
  double* X() const { return X_; }

 private:
  aes_handle h_;
  hipStream_t s_;
  ProblemDesc P_;
  aes_options o_;
  double tol_;
  // largest ||e|| / ||x|| of the last refinement sweep over the columns still refining
  double corr_ratio_ = 1.0;
  std::string ns_, sns_;
  int64_t n_, d_, c_;
  int C_;
  int64_t npad_, mcap_, m_ = 1, k_ = 0, fp_ = 64;
  double* yr_ = nullptr;   // transform-reuse SRHT: the stored normalised transform of A
  bool yr_ready_ = false;
  int32_t* korder_ = nullptr;  // nested SRHT: padded rows in increasing key order
  // sketch of the next resize formed ahead (FP64 SRHT, one problem)
  static constexpr double kSketchAheadShare = 8.0;  // extra scratch at most total memory / 8
  bool spec_ok_ = false, spec_pending_ = false;
  hipStream_t ss_ = nullptr;
  hipEvent_t spec_done_ = nullptr, spec_go_ = nullptr;
  int64_t spec_k_ = -1, spec_m_ = 0;
  int spec_cur_ = -1, spec_tgt_ = 0;
  void* spec_out_ = nullptr;
  int64_t gnest_m_ = 0;        // nested SRHT: rows behind the kept Gram (0: none)
  double nu2_;
  bool mixed_ = false, woodbury_ = false;
  double *lam_ = nullptr, *invlam_ = nullptr, *X_ = nullptr, *R_ = nullptr, *Pv_ = nullptr, *Q_ = nullptr,
         *XP_ = nullptr, *RP_ = nullptr, *RTP_ = nullptr, *Bv_ = nullptr, *scal_ = nullptr;
  int* active_ = nullptr;
  double *part_ = nullptr, *spart_ = nullptr, *Z_ = nullptr;
  int nwg_ = 1, msplit_ = 1;
  int64_t msplit_rows_ = 1;
  float* A32_ = nullptr;
  float *V32_ = nullptr, *Z32_ = nullptr, *part32_ = nullptr, *SA32_ = nullptr;
  bool sketch32_ = false;
  double* pinned_ = nullptr;
  double *SA_ = nullptr, *SAT_ = nullptr, *Linv_ = nullptr, *LinvT_ = nullptr;
  __hip_bfloat16* SA16_ = nullptr;
  double stop_scale_ = 0, stop_sr_ = 1, tol2_ = 0;
  double fl_[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t iters_ = 0, attempts_ = 0, resketches_ = 0, a_passes_ = 0, sweeps_ = 0, trace_len_ = 0;
  double t0_ms_ = now_ms();  // start of the solve (trace time stamps)
  int m_cap_reached_ = 0;
  int64_t n_events_ = 0;
  std::vector<int64_t> skip_events_;  // timing events of speculative steps that did not run
  hipEvent_t fev_[2] = {nullptr, nullptr};  // flag-copy events of the two pinned slots
  std::vector<std::pair<hipEvent_t, hipEvent_t>> sk_ev_;  // start / end of every sketch + factorisation
  double* atz_part_ = nullptr;
  int atz_nrb_ = 0;
  int64_t atz_rows_ = 0;
  double* vw_ = nullptr;  // work buffer of the wide vector kernels
  bool fused_ = true;  // single-RHS fused H.v (and the speculative step pipeline)
  bool cg_ = false;
  const int* chol_flag_ = nullptr;
  // batch mode
  BState bstate_ = kBStep;
  aes_status bstatus_ = AES_OK;
  const double* brhs_ = nullptr;
  double* bx_ = nullptr;
  bool bx_zero_ = true, buse32_ = false, bxzero_ = true;
  int bstop_ = 0;
  double bscale_ = 0.0, binner_scale_ = 0.0;
  double binner_eta_ = 1e-6;  // relative tolerance of the current inner solve (batched refinement)
  int64_t bt_ = 0, bI_ = 0;
  bool bforced_ = false;
  double bseq_ = 0.0;
  double blc_ = 0.0, blphi_ = 0.0, bmu_ = 0.0, bbeta_ = 0.0;
  bool bihs_ = false, bpolyak_ = false;
  double* bxpv_[2] = {nullptr, nullptr};
  double *bu_ = nullptr, *bt1_ = nullptr, *bw_ = nullptr, *bE_ = nullptr, *bRr_ = nullptr, *bnrm_ = nullptr;
  int* gate_ = nullptr;
  std::vector<int> bact_;
  bool beager_ = false;
};

// ---------------------------------------------------------------------------------------
// Batched solves (Sec. 5 "matrix variables", many problems): each problem keeps its own
// Solver for the control of Algorithm 2 / Algorithm 1 (resizes, restarts, refinement sweeps),
// while the step of every problem that is stepping runs as one fixed sequence of grouped
// launches (k_batch.hip), captured once in a HIP graph and replayed once per step.  Between
// replays the host reads every problem's flag block (one copy) and enqueues the eager work of
// the problems that were rejected (sketch, factorisation, explicit residual, initialisation) or
// finished an inner solve (refinement).
// ---------------------------------------------------------------------------------------
struct HpPlan {
  bool twopass = false;
  int64_t rows = 0;  // rows per range of the partial products
};

// Tuned plans of the grouped H.P, one per (precision, ceil(log2 n), ceil(d / 256)) bucket, read
// once from a text file (lines "fp32|fp64 <log2 n> <d blocks> fused|twopass <rows> ..."): the
// file named by AES_TUNE_FILE, else tune/hp_plans.txt beside the library's directory.
struct HpTuned {
  std::mutex mu;
  bool loaded = false;
  std::unordered_map<std::string, HpPlan> plans;
};
HpTuned& hp_tuned_table() {
  static HpTuned t;
  return t;
}
std::string hp_bucket(int64_t n, int64_t d, bool fp32) {
  int lg = 0;
  while ((int64_t(1) << lg) < n) ++lg;
  return std::string(fp32 ? "fp32 " : "fp64 ") + std::to_string(lg) + " " + std::to_string(ceil_div(d, 256));
}
void hp_tuned_load(HpTuned& t) {
  t.loaded = true;
  std::string path;
  if (const char* e = std::getenv("AES_TUNE_FILE")) {
    path = e;
  } else {
    Dl_info info;
    if (dladdr(reinterpret_cast<void*>(&hp_tuned_table), &info) && info.dli_fname) {
      std::string lib = info.dli_fname;
      const size_t sl = lib.rfind('/');
      const std::string dir = sl == std::string::npos ? std::string(".") : lib.substr(0, sl);
      path = dir + "/../tune/hp_plans.txt";
    }
  }
  if (path.empty()) return;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof(line), f)) {
    char prec[8], kind[16];
    int lg = 0, db = 0;
    long long rows = 0;
    if (line[0] == '#') continue;
    if (std::sscanf(line, "%7s %d %d %15s %lld", prec, &lg, &db, kind, &rows) != 5) continue;
    HpPlan p;
    p.twopass = std::strcmp(kind, "twopass") == 0;
    p.rows = rows;
    if (rows <= 0 || (!p.twopass && std::strcmp(kind, "fused") != 0)) continue;
    t.plans[std::string(prec) + " " + std::to_string(lg) + " " + std::to_string(db)] = p;
  }
  std::fclose(f);
}
bool hp_tuned(int64_t n, int64_t d, bool fp32, HpPlan* out) {
  HpTuned& t = hp_tuned_table();
  std::lock_guard<std::mutex> lock(t.mu);
  if (!t.loaded) hp_tuned_load(t);
  auto it = t.plans.find(hp_bucket(n, d, fp32));
  if (it == t.plans.end()) return false;
  *out = it->second;
  return true;
}

// Plan of the grouped H.P for one problem.  It depends only on the problem's shape (so a
// problem gives the same sums alone and in a batch): the tuned plan of its bucket when there is
// one and it applies, else the default (fused when the shape allows it).
HpPlan hp_plan(int64_t n, int64_t d, bool fp32, bool vec_ok) {
  const bool fused_ok = vec_ok && bhp_fused_mb(!fp32, d) <= bhp_fused_max_mb(!fp32);
  HpPlan p;
  if (hp_tuned(n, d, fp32, &p) && (p.twopass || fused_ok)) return p;
  p.twopass = !fused_ok;
  if (!p.twopass)
    p.rows = std::max<int64_t>(64, std::min<int64_t>(512, round_up(ceil_div(n, 256), 16)));
  else
    p.rows = std::max<int64_t>(512, round_up(ceil_div(n, 64), 64));
  return p;
}

class BatchEngine {
 public:
  BatchEngine(aes_handle h, hipStream_t caller, const std::vector<ProblemDesc>& probs, const aes_options& o,
              double tol, const std::vector<int32_t>& ids)
      : h_(h), caller_(caller), P_(probs), o_(o), tol_(tol), ids_(ids) {}
  ~BatchEngine() { cleanup(); }

  aes_status run(aes_info* infos) {
    PhaseRange range("aes batched solve");
    const double t0 = now_ms();
    const int np = (int)P_.size();
    AES_HIP(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
    AES_HIP(hipEventCreateWithFlags(&ready_, hipEventDisableTiming));
    AES_HIP(hipEventRecord(ready_, caller_));
    AES_HIP(hipStreamWaitEvent(s_, ready_, 0));
    // the eager phases of problem p run on worker stream p % W (default priority) with that
    // stream's own scratch namespace; the step waits for all of them through events
    const int W = std::min(np, kWorkers);
    ws_.assign(W, nullptr);
    wev_.assign(W, nullptr);
    for (int w = 0; w < W; ++w) {
      AES_HIP(hipStreamCreateWithFlags(&ws_[w], hipStreamNonBlocking));
      AES_HIP(hipEventCreateWithFlags(&wev_[w], hipEventDisableTiming));
      AES_HIP(hipStreamWaitEvent(ws_[w], ready_, 0));
    }
    so_.resize(np);
    for (int p = 0; p < np; ++p) {
      aes_options op = o_;
      op.problem = ids_[p];
      so_[p] = std::make_unique<Solver>(h_, ws_[p % W], P_[p], op, tol_, "b" + std::to_string(p) + ".",
                                        "bs" + std::to_string(p % W) + ".");
    }
    // per-problem set-up (eager): casts, the first sketch and factorisation, the initialisation
    for (int p = 0; p < np; ++p) {
      try {
        so_[p]->batch_begin();
      } catch (const StatusError& e) {
        h_->set_err(e.what());
        so_[p]->bdone(e.st);
      } catch (const std::bad_alloc&) {
        h_->set_err("device workspace allocation failed");
        so_[p]->bdone(AES_ERR_OOM);
      }
    }
    build(np);
    const bool graph = graph_enabled();
    if (graph) capture();
    // A problem whose eager work (set-up, resize and restart, refinement sweep) is still running
    // on its worker stream sits steps out until an event says it is done, so a long resize does
    // not hold the other problems back; its own sequence of operations is the same either way.
    AES_HIP(hipEventCreateWithFlags(&sev_, hipEventDisableTiming));
    pev_.assign(np, nullptr);
    nev_.assign(np, nullptr);
    for (int p = 0; p < np; ++p) {
      AES_HIP(hipEventCreateWithFlags(&pev_[p], hipEventDisableTiming));
      AES_HIP(hipEventCreateWithFlags(&nev_[p], hipEventDisableTiming));
    }
    std::vector<char> pending(np, 0), refine_wait(np, 0);
    auto mark_eager = [&](int p) {
      AES_HIP(hipEventRecord(pev_[p], ws_[p % ws_.size()]));
      pending[p] = 1;
    };
    auto start_refine = [&](int p) {
      // ||e||^2, ||x||^2 of the finished inner solve, copied to the host behind its eager work
      hipStream_t w = ws_[p % ws_.size()];
      AES_HIP(hipMemcpyAsync(hnrm_ + 64 * p, so_[p]->batch_norms(), 2 * so_[p]->batch_C() * sizeof(double),
                             hipMemcpyDeviceToHost, w));
      AES_HIP(hipEventRecord(nev_[p], w));
      refine_wait[p] = 1;
    };
    for (int p = 0; p < np; ++p) mark_eager(p);
    for (;;) {
      bool any = false, waiting = false;
      for (int p = 0; p < np; ++p) {
        if (refine_wait[p]) {
          const hipError_t q = hipEventQuery(nev_[p]);
          if (q == hipSuccess) {
            refine_wait[p] = 0;
            so_[p]->batch_refine(hnrm_ + 64 * p);
            if (so_[p]->bstate() == Solver::kBStep) mark_eager(p);
          } else if (q != hipErrorNotReady) {
            AES_HIP(q);
          }
        }
        if (so_[p]->batch_precheck()) {
          mark_eager(p);
          start_refine(p);
        }
        bool ready = true;
        if (so_[p]->bstate() == Solver::kBStep && pending[p]) {
          const hipError_t q = hipEventQuery(pev_[p]);
          if (q == hipSuccess) {
            pending[p] = 0;
            AES_HIP(hipStreamWaitEvent(s_, pev_[p], 0));  // orders the step after it (complete already)
          } else if (q == hipErrorNotReady) {
            ready = false;
          } else {
            AES_HIP(q);
          }
        }
        so_[p]->batch_dyn(hdyn_[p], ready);
        any = any || hdyn_[p].run != 0;
        waiting = waiting || refine_wait[p] || (so_[p]->bstate() == Solver::kBStep && !ready);
      }
      if (any) {
        AES_HIP(hipMemcpyAsync(ddyn_, hdyn_, np * sizeof(BDyn), hipMemcpyHostToDevice, s_));
        if (graph)
          AES_HIP(hipGraphLaunch(exec_, s_));
        else
          enqueue_step();
        AES_HIP(hipMemcpyAsync(hflags_, dflags_, (size_t)np * 8 * sizeof(double), hipMemcpyDeviceToHost, s_));
        AES_HIP(hipEventRecord(sev_, s_));
        AES_HIP(hipStreamSynchronize(s_));
        ++steps_;
        // eager work enqueued from here on is ordered after the step on every worker stream
        for (hipStream_t w : ws_) AES_HIP(hipStreamWaitEvent(w, sev_, 0));
        for (int p = 0; p < np; ++p) {
          if (!hdyn_[p].run) continue;
          const bool refine_now = so_[p]->batch_after(hflags_ + 8 * p);
          if (so_[p]->batch_eager()) mark_eager(p);
          if (refine_now) start_refine(p);
        }
        continue;
      }
      bool all_done = true;
      for (int p = 0; p < np; ++p) all_done = all_done && so_[p]->bstate() == Solver::kBDone;
      if (all_done) break;
      if (!waiting) throw HipError("batched solve made no progress");
      // nothing can step: wait for the earliest outstanding eager work
      for (int p = 0; p < np; ++p) {
        if (refine_wait[p]) {
          AES_HIP(hipEventSynchronize(nev_[p]));
          break;
        }
        if (so_[p]->bstate() == Solver::kBStep && pending[p]) {
          AES_HIP(hipEventSynchronize(pev_[p]));
          break;
        }
      }
    }
    aes_status worst = AES_OK;
    for (int p = 0; p < np; ++p) {
      const aes_status st = so_[p]->batch_result(infos ? &infos[p] : nullptr, t0);
      if (st != AES_OK && worst == AES_OK) worst = st;
    }
    for (hipStream_t w : ws_) AES_HIP(hipStreamSynchronize(w));
    AES_HIP(hipStreamSynchronize(s_));
    return worst;
  }

  int64_t steps() const { return steps_; }

  // Average time (ms) of the grouped H.P (prep, products, column sums) of one problem under a
  // given plan, over `reps` launches after one warm-up launch.  For the tuner of the plans.
  double time_hp(const HpPlan& plan, int reps) {
    AES_HIP(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
    AES_HIP(hipEventCreateWithFlags(&ready_, hipEventDisableTiming));
    AES_HIP(hipEventRecord(ready_, caller_));
    AES_HIP(hipStreamWaitEvent(s_, ready_, 0));
    so_.resize(1);
    so_[0] = std::make_unique<Solver>(h_, s_, P_[0], o_, tol_, "tune.", "tune_s.");
    so_[0]->batch_tune_setup();
    fp32_ = so_[0]->batch_fp32();
    np_ = 1;
    const int64_t n = P_[0].n, d = P_[0].d;
    const int mb = bhp_fused_mb(!fp32_, d);
    if (!plan.twopass && mb > bhp_fused_max_mb(!fp32_)) throw StatusError(AES_ERR_INVALID_ARG, "the fused form takes no such d");
    const int64_t kpad = plan.twopass ? round_up(d, 256) : 256 * (int64_t)mb;
    const int nrb = (int)ceil_div(n, plan.rows);
    dflags_ = h_->buf<double>("tune.flags", 8);
    dprob_ = h_->buf<BProb>("tune.prob", 1);
    ddyn_ = h_->buf<BDyn>("tune.dyn", 1);
    BProb hp;
    so_[0]->batch_fill(hp, dflags_, nrb, plan.rows, plan.twopass, kpad);
    BDyn dy{};
    dy.run = 1;
    std::vector<BWork> work, z, a;
    if (!plan.twopass) {
      for (int r = 0; r < nrb; ++r) work.push_back(BWork{0, r});
    } else {
      for (int64_t t = 0; t < ceil_div(n, 64); ++t) z.push_back(BWork{0, (int32_t)t});
      const int64_t ct = ceil_div(d, 64);
      for (int64_t r = 0; r < nrb; ++r)
        for (int64_t t = 0; t < ct; ++t) a.push_back(BWork{0, (int32_t)(r * ct + t)});
    }
    BWork* dw = work.empty() ? nullptr : h_->buf<BWork>("tune.fw", work.size());
    BWork* dz = z.empty() ? nullptr : h_->buf<BWork>("tune.zw", z.size());
    BWork* da = a.empty() ? nullptr : h_->buf<BWork>("tune.aw", a.size());
    AES_HIP(hipMemcpyAsync(dprob_, &hp, sizeof(BProb), hipMemcpyHostToDevice, s_));
    AES_HIP(hipMemcpyAsync(ddyn_, &dy, sizeof(BDyn), hipMemcpyHostToDevice, s_));
    if (dw) AES_HIP(hipMemcpyAsync(dw, work.data(), work.size() * sizeof(BWork), hipMemcpyHostToDevice, s_));
    if (dz) AES_HIP(hipMemcpyAsync(dz, z.data(), z.size() * sizeof(BWork), hipMemcpyHostToDevice, s_));
    if (da) AES_HIP(hipMemcpyAsync(da, a.data(), a.size() * sizeof(BWork), hipMemcpyHostToDevice, s_));
    const int64_t vt = (int64_t)std::max(16, so_[0]->batch_C()) * kpad, dc = d * so_[0]->batch_C();
    auto once = [&]() {
      if (fp32_) {
        launch_bprep<float>(dprob_, ddyn_, 1, vt, false, s_);
        if (dw) launch_bhp_fused<float>(dprob_, ddyn_, dw, (int)work.size(), mb, s_);
        if (dz) launch_bhp_twopass<float>(dprob_, ddyn_, dz, (int)z.size(), da, (int)a.size(), s_);
        launch_bcolsum<float>(dprob_, ddyn_, 1, dc, false, s_);
      } else {
        launch_bprep<double>(dprob_, ddyn_, 1, vt, false, s_);
        if (dw) launch_bhp_fused<double>(dprob_, ddyn_, dw, (int)work.size(), mb, s_);
        if (dz) launch_bhp_twopass<double>(dprob_, ddyn_, dz, (int)z.size(), da, (int)a.size(), s_);
        launch_bcolsum<double>(dprob_, ddyn_, 1, dc, false, s_);
      }
    };
    once();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    AES_HIP(hipEventCreate(&e0));
    AES_HIP(hipEventCreate(&e1));
    AES_HIP(hipEventRecord(e0, s_));
    for (int i = 0; i < reps; ++i) once();
    AES_HIP(hipEventRecord(e1, s_));
    AES_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    const hipError_t te = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    AES_HIP(te);
    return (double)ms / std::max(reps, 1);
  }

 private:
  static constexpr int kWorkers = 8;

  // the step stream waits for the eager work enqueued on every worker stream
  void join_workers() {
    for (size_t w = 0; w < ws_.size(); ++w) {
      AES_HIP(hipEventRecord(wev_[w], ws_[w]));
      AES_HIP(hipStreamWaitEvent(s_, wev_[w], 0));
    }
  }

  static bool graph_enabled() {
    const char* e = std::getenv("AES_BATCH_GRAPH");
    return !(e && e[0] == '0');
  }

  void build(int np) {
    fp32_ = so_[0]->batch_fp32();
    ihs_ = so_[0]->batch_ihs();
    method_ = o_.method;
    np_ = np;
    dflags_ = h_->buf<double>("bt.flags", (size_t)np * 8);
    dprob_ = h_->buf<BProb>("bt.prob", np);
    ddyn_ = h_->buf<BDyn>("bt.dyn", np);
    AES_HIP(hipHostMalloc((void**)&hdyn_, np * sizeof(BDyn), hipHostMallocDefault));
    AES_HIP(hipHostMalloc((void**)&hflags_, (size_t)np * 8 * sizeof(double), hipHostMallocDefault));
    AES_HIP(hipHostMalloc((void**)&hnrm_, (size_t)np * 64 * sizeof(double), hipHostMallocDefault));
    std::vector<BProb> hp(np);
    std::vector<BWork> z, a, tiles;
    std::vector<std::vector<BWork>> fw(9);
    const size_t es = fp32_ ? sizeof(float) : sizeof(double);
    for (int p = 0; p < np; ++p) {
      Solver& so = *so_[p];
      const int64_t n = so.batch_n(), d = so.batch_d();
      const int vw = (int)(16 / es);
      const ProblemDesc& P = P_[p];
      // the FP32 copy is dense (ld d) in a 256-byte aligned pool buffer
      const bool vec_ok = fp32_ ? d % vw == 0
                                : (d % vw == 0 && P.lda % vw == 0 && (reinterpret_cast<uintptr_t>(P.A) & 15) == 0);
      const HpPlan hpp = hp_plan(n, d, fp32_, vec_ok);
      const int nrb = (int)ceil_div(n, hpp.rows);
      // the fused form reads whole column blocks of 256 * mb of the transposed operand
      const int64_t kpad = hpp.twopass ? round_up(d, 256) : 256 * (int64_t)bhp_fused_mb(!fp32_, d);
      so.batch_fill(hp[p], dflags_ + 8 * p, nrb, hpp.rows, hpp.twopass, kpad);
      max_vt_ = std::max<int64_t>(max_vt_, (int64_t)std::max(16, so.batch_C()) * kpad);
      max_dc_ = std::max<int64_t>(max_dc_, d * so.batch_C());
      if (!hpp.twopass) {
        const int mb = bhp_fused_mb(!fp32_, d);
        for (int r = 0; r < nrb; ++r) fw[mb].push_back(BWork{p, r});
      } else {
        for (int64_t t = 0; t < ceil_div(n, 64); ++t) z.push_back(BWork{p, (int32_t)t});
        const int64_t ct = ceil_div(d, 64);
        for (int64_t r = 0; r < nrb; ++r)
          for (int64_t t = 0; t < ct; ++t) a.push_back(BWork{p, (int32_t)(r * ct + t)});
      }
      for (int64_t t = 0; t < ceil_div(d, 64); ++t) tiles.push_back(BWork{p, (int32_t)t});
    }
    join_workers();  // the descriptors point at buffers the set-up initialised
    AES_HIP(hipMemcpyAsync(dprob_, hp.data(), np * sizeof(BProb), hipMemcpyHostToDevice, s_));
    auto upload = [&](const std::vector<BWork>& v, const char* name) -> BWork* {
      if (v.empty()) return nullptr;
      BWork* dv = h_->buf<BWork>(name, v.size());
      AES_HIP(hipMemcpyAsync(dv, v.data(), v.size() * sizeof(BWork), hipMemcpyHostToDevice, s_));
      return dv;
    };
    for (int mb = 1; mb <= 8; ++mb) {
      fwork_[mb] = upload(fw[mb], ("bt.fw" + std::to_string(mb)).c_str());
      nfwork_[mb] = (int)fw[mb].size();
    }
    zwork_ = upload(z, "bt.zw");
    nz_ = (int)z.size();
    awork_ = upload(a, "bt.aw");
    na_ = (int)a.size();
    tiles_ = upload(tiles, "bt.tiles");
    ntiles_ = (int)tiles.size();
    // the host vectors must outlive the asynchronous copies
    AES_HIP(hipStreamSynchronize(s_));
  }

  // The step of every problem (run flag and device gate decide who takes part).
  void enqueue_step() {
    if (fp32_)
      enqueue_typed<float>();
    else
      enqueue_typed<double>();
  }
  template <typename T>
  void enqueue_typed() {
    if (ihs_) launch_bcandidate(dprob_, ddyn_, np_, method_, s_);  // xp = x - mu s (+ momentum)
    launch_bprep<T>(dprob_, ddyn_, np_, max_vt_, ihs_, s_);
    for (int mb = 1; mb <= 8; ++mb)
      if (nfwork_[mb]) launch_bhp_fused<T>(dprob_, ddyn_, fwork_[mb], nfwork_[mb], mb, s_);
    if (nz_ || na_) launch_bhp_twopass<T>(dprob_, ddyn_, zwork_, nz_, awork_, na_, s_);
    launch_bcolsum<T>(dprob_, ddyn_, np_, max_dc_, ihs_, s_);
    if (!ihs_) launch_bcandidate(dprob_, ddyn_, np_, method_, s_);  // alpha, xp, rp
    const int slots = method_ == AES_CG ? 1 : kBProds;
    for (int sl = 0; sl < slots; ++sl) launch_bapply(dprob_, ddyn_, tiles_, ntiles_, sl, s_);
    launch_bfinish(dprob_, ddyn_, np_, ihs_, s_);
  }

  void capture() {
    hipGraph_t g = nullptr;
    AES_HIP(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
    try {
      enqueue_step();
    } catch (...) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(s_, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      throw;
    }
    AES_HIP(hipStreamEndCapture(s_, &g));
    const hipError_t e = hipGraphInstantiate(&exec_, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    AES_HIP(e);
  }

  void cleanup() {
    for (hipStream_t w : ws_)
      if (w) (void)hipStreamSynchronize(w);
    if (s_) (void)hipStreamSynchronize(s_);
    if (exec_) (void)hipGraphExecDestroy(exec_);
    exec_ = nullptr;
    so_.clear();
    if (hdyn_) (void)hipHostFree(hdyn_);
    if (hflags_) (void)hipHostFree(hflags_);
    if (hnrm_) (void)hipHostFree(hnrm_);
    hdyn_ = nullptr;
    hflags_ = nullptr;
    hnrm_ = nullptr;
    if (ready_) (void)hipEventDestroy(ready_);
    ready_ = nullptr;
    for (hipEvent_t e : wev_)
      if (e) (void)hipEventDestroy(e);
    wev_.clear();
    if (sev_) (void)hipEventDestroy(sev_);
    sev_ = nullptr;
    for (hipEvent_t e : pev_)
      if (e) (void)hipEventDestroy(e);
    pev_.clear();
    for (hipEvent_t e : nev_)
      if (e) (void)hipEventDestroy(e);
    nev_.clear();
    for (hipStream_t w : ws_)
      if (w) (void)hipStreamDestroy(w);
    ws_.clear();
    if (s_) (void)hipStreamDestroy(s_);
    s_ = nullptr;
  }

  aes_handle h_;
  hipStream_t caller_;
  std::vector<ProblemDesc> P_;
  aes_options o_;
  double tol_;
  std::vector<int32_t> ids_;
  hipStream_t s_ = nullptr;
  hipEvent_t ready_ = nullptr;
  std::vector<hipStream_t> ws_;
  std::vector<hipEvent_t> wev_;
  std::vector<hipEvent_t> pev_, nev_;  // per problem: end of its eager work; its norms on the host
  hipEvent_t sev_ = nullptr;           // end of the last step
  hipGraphExec_t exec_ = nullptr;
  std::vector<std::unique_ptr<Solver>> so_;
  bool fp32_ = false, ihs_ = false;
  int method_ = 0, np_ = 0;
  BProb* dprob_ = nullptr;
  BDyn* ddyn_ = nullptr;
  BDyn* hdyn_ = nullptr;
  double *dflags_ = nullptr, *hflags_ = nullptr, *hnrm_ = nullptr;
  BWork* fwork_[9] = {};
  int nfwork_[9] = {};
  BWork *zwork_ = nullptr, *awork_ = nullptr, *tiles_ = nullptr;
  int nz_ = 0, na_ = 0, ntiles_ = 0;
  int64_t max_vt_ = 0, max_dc_ = 0;
  int64_t steps_ = 0;
};

aes_status guard(aes_handle h, const std::function<void()>& f) {
  try {
    f();
    return AES_OK;
  } catch (const StatusError& e) {
    if (h) h->err = e.what();
    return e.st;
  } catch (const HipError& e) {
    if (h) h->err = e.what();
    return AES_ERR_HIP;
  } catch (const std::bad_alloc&) {
    if (h) h->err = "device workspace allocation failed";
    return AES_ERR_OOM;
  } catch (const std::invalid_argument& e) {
    if (h) h->err = e.what();
    return AES_ERR_INVALID_ARG;
  } catch (const std::exception& e) {
    if (h) h->err = e.what();
    return AES_ERR_HIP;
  }
}

void set_device(aes_handle h) { AES_HIP(hipSetDevice(h->device)); }

}  // namespace

// ---------------------------------------------------------------------------------------
// C ABI.
// ---------------------------------------------------------------------------------------
extern "C" {

void aes_default_options(aes_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->method = AES_PCG;
  o->sketch = AES_SRHT;
  o->precision = AES_FP64;
  o->stop = AES_STOP_XREL;
  o->rho = 0.125;
  o->m_init = 1;
  o->m_max = 0;
  o->max_iter = 200;
  o->seed = 0;
  o->problem = 0;
  o->adaptive = 1;
  o->force_reject_at = -1;
  o->inner_tol = 1e-6;
  o->max_refine = 20;
  o->trace_cap = 0;
  o->trace = nullptr;
  o->x0 = nullptr;
}

aes_status aes_create(aes_handle* out, int device) {
  if (!out) return AES_ERR_INVALID_ARG;
  *out = nullptr;
  auto h = std::make_unique<aes_handle_s>();
  h->device = device;
  aes_status st = guard(h.get(), [&] {
    int count = 0;
    AES_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) throw StatusError(AES_ERR_INVALID_ARG, "no such device");
    AES_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    AES_HIP(hipGetDeviceProperties(&prop, device));
    h->num_cu = prop.multiProcessorCount;
    AES_HIP(hipHostMalloc((void**)&h->pinned, 64 * sizeof(double), hipHostMallocDefault));
    // device address of the allocation-free entry point's static workspace on this device
    AES_HIP(noalloc_init(device));
  });
  if (st != AES_OK) return st;
  *out = h.release();
  return AES_OK;
}

aes_status aes_destroy(aes_handle h) {
  if (!h) return AES_ERR_INVALID_ARG;
  (void)hipSetDevice(h->device);
  h->release();
  delete h;
  return AES_OK;
}

const char* aes_last_error(aes_handle h) { return h ? h->err.c_str() : "null handle"; }

static aes_status solve_impl(aes_handle h, void* stream, const ProblemDesc& P, double tol, const aes_options* opt,
                             aes_info* info, const std::string& ns, Solver** keep) {
  if (!h) return AES_ERR_INVALID_ARG;
  aes_options o;
  if (opt)
    o = *opt;
  else
    aes_default_options(&o);
  aes_status st = guard(h, [&] {
    set_device(h);
    validate(P, tol, o);
  });
  if (st != AES_OK) {
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->status = st;
    }
    return st;
  }
  if (P.c > 1 && !keep) {
    // several right-hand sides: the grouped step of the batched engine (one problem), so that a
    // problem solved alone and within a batch takes the same arithmetic
    aes_status bst = AES_OK;
    st = guard(h, [&] {
      BatchEngine eng(h, (hipStream_t)stream, std::vector<ProblemDesc>{P}, o, tol, std::vector<int32_t>{o.problem});
      bst = eng.run(info);
    });
    if (st != AES_OK && info) {
      std::memset(info, 0, sizeof(*info));
      info->status = st;
    }
    return st != AES_OK ? st : bst;
  }
  auto* solver = new Solver(h, (hipStream_t)stream, P, o, tol, ns);
  if (!keep) solver->enable_sketch_ahead();
  st = solver->run(info);
  if (keep)
    *keep = solver;
  else
    delete solver;
  return st;
}

aes_status aes_solve(aes_handle h, void* stream, int64_t n, int64_t d, int64_t c, const double* A, int64_t lda,
                     const double* b, int64_t ldb, double nu, const double* lambda, double tol, const aes_options* opt,
                     double* x, int64_t ldx, aes_info* info) {
  ProblemDesc P{n, d, c, A, lda, b, ldb, nu, lambda, x, ldx};
  aes_status st = AES_OK;
  try {
    st = solve_impl(h, stream, P, tol, opt, info, "s.", nullptr);
  } catch (const StatusError& e) {
    if (h) h->err = e.what();
    st = e.st;
  }
  return st;
}

aes_status aes_solve_dual(aes_handle h, void* stream, int64_t n, int64_t d, int64_t c, const double* A, int64_t lda,
                          const double* b, int64_t ldb, double nu, const double* lambda, double tol,
                          const aes_options* opt, double* x, int64_t ldx, aes_info* info) {
  // Dual problem of Sec. 1: with B = Lambda^{-1/2} A^T (d x n), solve
  // (B^T B + nu^2 I_n) w = A Lambda^{-1} b by the primal solver, then
  // x = Lambda^{-1/2} (Lambda^{-1/2} b - B w) / nu^2 (primal optimality: H x = b, A x = w).
  if (!h) return AES_ERR_INVALID_ARG;
  aes_options o;
  if (opt)
    o = *opt;
  else
    aes_default_options(&o);
  hipStream_t s = (hipStream_t)stream;
  const int C = (int)next_pow2(std::max<int64_t>(c, 1));
  double *Bm = nullptr, *w = nullptr, *bd = nullptr, *isl = nullptr, *u = nullptr, *v = nullptr, *xp = nullptr;
  aes_status st = guard(h, [&] {
    set_device(h);
    auto bad = [](const char* m) { throw StatusError(AES_ERR_INVALID_ARG, m); };
    if (n < 1 || d < 1 || c < 1) bad("n, d and c must be >= 1");
    if (n > kMaxD) bad("the dual form needs n <= 32768");
    if (c > 32) bad("at most 32 right-hand sides per problem");
    if (lda < d) bad("lda < d");
    if (ldb < c || ldx < c) bad("ldb and ldx must be >= c");
    if (!A || !b || !x) bad("A, b and x must be non-null");
    if (o.x0) bad("the dual form takes no start point");
    // the dual problem as the primal solver will see it (placeholder pointers)
    validate(ProblemDesc{d, n, c, A, n, b, C, nu, nullptr, x, C}, tol, o);
    Bm = h->buf<double>("dual.B", (size_t)d * n);
    w = h->buf<double>("dual.w", (size_t)n * C);
    bd = h->buf<double>("dual.bd", (size_t)n * C);
    isl = h->buf<double>("dual.isl", d);
    u = h->buf<double>("dual.u", (size_t)d * C);
    v = h->buf<double>("dual.v", (size_t)d * C);
    xp = h->buf<double>("dual.x", (size_t)d * C);
    launch_dual_prep(d, C, (int)c, b, ldb, lambda, isl, u, v, s);
    launch_rowdot(n, d, A, lda, 0, v, C, nullptr, 1.0, nullptr, nullptr, 1.0, bd, s);  // A Lambda^{-1} b
    launch_transpose(n, d, A, lda, Bm, n, s, isl);                                    // Lambda^{-1/2} A^T
    launch_fill(w, n * C, 0.0, s);
  });
  if (st != AES_OK) {
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->status = st;
    }
    return st;
  }
  try {
    st = solve_impl(h, stream, ProblemDesc{d, n, c, Bm, n, bd, C, nu, nullptr, w, C}, tol, &o, info, "s.", nullptr);
  } catch (const StatusError& e) {
    h->err = e.what();
    st = e.st;
  }
  if (st != AES_OK && st != AES_ERR_MAX_ITER) return st;
  const aes_status st2 = guard(h, [&] {
    set_device(h);
    launch_rowdot(d, n, Bm, n, 0, w, C, nullptr, -1.0, u, isl, 1.0 / (nu * nu), xp, s);
    launch_copy_cols(d, (int)c, xp, C, (int)c, x, ldx, s);
    AES_HIP(hipStreamSynchronize(s));
  });
  if (st2 != AES_OK && info) info->status = st2;
  return st2 != AES_OK ? st2 : st;
}

aes_status aes_solve_batched(aes_handle h, void* stream, int64_t nprob, const aes_problem* probs, double tol,
                             const aes_options* opt, aes_info* infos) {
  if (!h || nprob < 0 || (nprob > 0 && !probs)) return AES_ERR_INVALID_ARG;
  if (nprob == 0) return AES_OK;
  aes_options o;
  if (opt)
    o = *opt;
  else
    aes_default_options(&o);
  o.trace = nullptr;
  o.trace_cap = 0;
  o.profile = 0;
  o.x0 = nullptr;
  // validate everything first: on INVALID_ARG nothing is written
  for (int64_t p = 0; p < nprob; ++p) {
    const aes_problem& q = probs[p];
    ProblemDesc P{q.n, q.d, q.c, q.A, q.lda, q.b, q.ldb, q.nu, q.lambda, q.x, q.ldx};
    aes_status st = guard(h, [&] { validate(P, tol, o); });
    if (st != AES_OK) return st;
  }
  // all problems step together in the grouped kernels (one graph launch per step); problem p
  // draws its sketches from Philox stream p
  std::vector<ProblemDesc> P;
  std::vector<int32_t> ids;
  for (int64_t p = 0; p < nprob; ++p) {
    const aes_problem& q = probs[p];
    P.push_back(ProblemDesc{q.n, q.d, q.c, q.A, q.lda, q.b, q.ldb, q.nu, q.lambda, q.x, q.ldx});
    ids.push_back((int32_t)p);
  }
  aes_status bst = AES_OK;
  const aes_status st = guard(h, [&] {
    set_device(h);
    BatchEngine eng(h, (hipStream_t)stream, P, o, tol, ids);
    bst = eng.run(infos);
  });
  if (st != AES_OK && infos)
    for (int64_t p = 0; p < nprob; ++p) {
      std::memset(&infos[p], 0, sizeof(aes_info));
      infos[p].status = st;
    }
  return st != AES_OK ? st : bst;
}

aes_status aes_solve_keep(aes_handle h, void* stream, int64_t n, int64_t d, int64_t c, const double* A, int64_t lda,
                          const double* b, int64_t ldb, double nu, const double* lambda, double tol,
                          const aes_options* opt, double* x, int64_t ldx, aes_info* info, aes_ctx* ctx) {
  if (!h || !ctx) return AES_ERR_INVALID_ARG;
  *ctx = nullptr;
  if (c != 1) {
    h->err = "aes_solve_keep supports c = 1";
    return AES_ERR_INVALID_ARG;
  }
  aes_options o;
  if (opt)
    o = *opt;
  else
    aes_default_options(&o);
  if (o.precision != AES_FP64) {
    h->err = "aes_solve_keep supports FP64";
    return AES_ERR_INVALID_ARG;
  }
  if (o.method == AES_CG) {
    h->err = "aes_solve_keep needs a sketched preconditioner (PCG, IHS or Polyak-IHS)";
    return AES_ERR_INVALID_ARG;
  }
  auto c2 = std::make_unique<aes_ctx_s>();
  aes_status st = aes_create(&c2->h, h->device);
  if (st != AES_OK) return st;
  ProblemDesc P{n, d, c, A, lda, b, ldb, nu, lambda, x, ldx};
  Solver* keep = nullptr;
  st = solve_impl(c2->h, stream, P, tol, &o, info, "s.", &keep);
  if (st != AES_OK) {
    h->err = c2->h->err;
    delete keep;
    aes_destroy(c2->h);
    return st;
  }
  c2->n = n;
  c2->d = d;
  c2->lda = lda;
  c2->A = A;
  c2->nu = nu;
  c2->has_lambda = lambda != nullptr;
  c2->opt = o;
  c2->opt.trace = nullptr;
  c2->opt.trace_cap = 0;
  c2->opt.x0 = nullptr;
  c2->m = keep->m();
  c2->k = keep->k();
  st = guard(h, [&] {
    c2->xstar = c2->h->buf<double>("ctx_xstar", d);
    AES_HIP(hipMemcpyAsync(c2->xstar, x, d * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
    if (lambda) {
      double* lk = c2->h->buf<double>("ctx_lambda", d);
      AES_HIP(hipMemcpyAsync(lk, lambda, d * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
    }
    AES_HIP(hipStreamSynchronize((hipStream_t)stream));
  });
  delete keep;
  if (st != AES_OK) {
    aes_destroy(c2->h);
    return st;
  }
  // Between the forward and the adjoint solve the context holds only what the adjoint reuses:
  // the sketch (Woodbury branch), the inverse factor and its transpose, x* and Lambda.  The
  // rest of the pool (the transform scratch, Gram partials, vectors) is released now and
  // re-allocated by the adjoint solve as it needs it.
  st = guard(h, [&] {
    set_device(c2->h);
    c2->h->release_except({"s.SA", "s.SAT", "s.Linv", "s.LinvT", "ctx_xstar", "ctx_lambda"});
  });
  if (st != AES_OK) {
    aes_destroy(c2->h);
    return st;
  }
  *ctx = c2.release();
  return AES_OK;
}

aes_status aes_adjoint_solve(aes_ctx ctx, void* stream, const double* g, double tol, double* lam, aes_info* info) {
  if (!ctx || !g || !lam) return AES_ERR_INVALID_ARG;
  aes_handle h = ctx->h;
  const double* lk = ctx->has_lambda ? h->buf<double>("ctx_lambda", ctx->d) : nullptr;
  ProblemDesc P{ctx->n, ctx->d, 1, ctx->A, ctx->lda, g, 1, ctx->nu, lk, lam, 1};
  aes_status st = guard(h, [&] {
    set_device(h);
    validate(P, tol, ctx->opt);
  });
  if (st != AES_OK) return st;
  // Same workspace names as the forward solve: the kept SA / factor are reused as H_S, and
  // the sketch stream continues at index k+1 if the improvement test asks for a resize.
  Solver solver(h, (hipStream_t)stream, P, ctx->opt, tol, "s.");
  solver.set_mk(ctx->m, ctx->k, ctx->m < ctx->d, round_up(ctx->m < ctx->d ? ctx->m : ctx->d, 64));
  st = guard(h, [&] { solver.bind_factor(); });
  if (st != AES_OK) return st;
  st = solver.run(info, true);
  if (st == AES_OK) {
    ctx->m = solver.m();
    ctx->k = solver.k();
  }
  return st;
}

aes_status aes_grad(aes_ctx ctx, void* stream, const double* lam, double* dA, double* dlognu) {
  if (!ctx || !lam) return AES_ERR_INVALID_ARG;
  aes_handle h = ctx->h;
  return guard(h, [&] {
    set_device(h);
    hipStream_t s = (hipStream_t)stream;
    if (dA) launch_grad_rank2(ctx->A, ctx->n, ctx->d, ctx->lda, ctx->xstar, lam, dA, ctx->d, s);
    if (dlognu) {
      // -2 nu^2 lam^T Lambda x*  (a 1 x d row-dot with the diagonal as the column scale)
      double* out = h->buf<double>("grad_out", 1);
      const double* lk = ctx->has_lambda ? h->buf<double>("ctx_lambda", ctx->d) : nullptr;
      launch_rowdot(1, ctx->d, lam, ctx->d, 0, ctx->xstar, 1, lk, 1.0, nullptr, nullptr, 1.0, out, s);
      double v = 0;
      AES_HIP(hipMemcpyAsync(&v, out, sizeof(double), hipMemcpyDeviceToHost, s));
      AES_HIP(hipStreamSynchronize(s));
      *dlognu = -2.0 * ctx->nu * ctx->nu * v;
    }
  });
}

void aes_ctx_free(aes_ctx ctx) {
  if (!ctx) return;
  if (ctx->h) aes_destroy(ctx->h);
  delete ctx;
}

aes_status aes_hv(aes_handle h, void* stream, int64_t n, int64_t d, const double* A, int64_t lda, double nu,
                  const double* lambda, const double* p, double* q, double* pHp) {
  if (!h) return AES_ERR_INVALID_ARG;
  return guard(h, [&] {
    if (n < 1 || d < 1 || lda < d || !A || !p || !q || !(nu >= 0)) throw StatusError(AES_ERR_INVALID_ARG, "bad arguments");
    if (d > kMaxD) throw StatusError(AES_ERR_INVALID_ARG, "d > 32768 is not supported");
    set_device(h);
    hipStream_t s = (hipStream_t)stream;
    const int nwg = hv_num_blocks(h->num_cu, n);
    double* spart = nullptr;  // wide problems: pHp = p . q
    if (d <= kMaxFusedD) {
      double* part = h->buf<double>("hv.part", (size_t)nwg * d);
      spart = h->buf<double>("hv.spart", nwg);
      launch_hv_fused<double>(A, n, d, lda, p, part, spart, nwg, s);
      launch_hv_colsum(part, nwg, d, 1, p, lambda, nu * nu, 1.0, nullptr, 0.0, q, s);
    } else {
      int64_t rows = 0;
      const int nrb = atz_blocks(h->num_cu, n, d, &rows);
      double* z = h->buf<double>("hv.z", n);
      double* part = h->buf<double>("hv.atz", (size_t)nrb * d);
      launch_rowdot(n, d, A, lda, 0, p, 1, nullptr, 1.0, nullptr, nullptr, 1.0, z, s);
      launch_atz(A, n, d, lda, z, part, nrb, rows, s);
      launch_hv_colsum(part, nrb, d, 1, p, lambda, nu * nu, 1.0, nullptr, 0.0, q, s);
    }
    if (pHp) {
      // ||A p||^2 + nu^2 p^T Lambda p: the candidate kernel's reduction with a zero state
      double* scal = h->buf<double>("hv.scal", 16);
      int* act = h->buf<int>("hv.act", 1);
      double* dummy = h->buf<double>("hv.dummy", 2 * d);
      AES_HIP(hipMemsetAsync(scal, 0, 16 * sizeof(double), s));
      AES_HIP(hipMemsetAsync(act, 0, sizeof(int), s));
      launch_pcg_candidate(d, 1, spart, nwg, lambda, nu * nu, p, p, p, q, dummy, dummy + d, scal, act, s);
      AES_HIP(hipMemcpyAsync(pHp, scal + 5, sizeof(double), hipMemcpyDeviceToDevice, s));
    }
  });
}

aes_status aes_residual(aes_handle h, void* stream, int64_t n, int64_t d, int64_t c, const double* A, int64_t lda,
                        const double* b, int64_t ldb, double nu, const double* lambda, const double* x, int64_t ldx,
                        double* r, int64_t ldr) {
  if (!h) return AES_ERR_INVALID_ARG;
  return guard(h, [&] {
    if (n < 1 || d < 1 || c < 1 || c > 32 || lda < d || ldb < c || ldx < c || ldr < c || !A || !b || !x || !r ||
        !(std::isfinite(nu) && nu >= 0))
      throw StatusError(AES_ERR_INVALID_ARG, "bad arguments");
    set_device(h);
    hipStream_t s = (hipStream_t)stream;
    const int C = (int)next_pow2(c);
    // x and b into C-column blocks (zero padding columns), the residual back to the caller's layout
    double* xc = h->buf<double>("res.x", (size_t)d * C);
    double* bc = h->buf<double>("res.b", (size_t)d * C);
    double* rc = h->buf<double>("res.r", (size_t)d * C);
    launch_copy_cols(d, C, x, ldx, (int)c, xc, C, s);
    launch_copy_cols(d, C, b, ldb, (int)c, bc, C, s);
    const size_t pe = residual_dd_part_elems(h->num_cu, n, d, C);
    launch_residual_dd(h->num_cu, n, d, C, A, lda, bc, C, nu, lambda, xc, h->buf<double>("res.zh", (size_t)n * C),
                       h->buf<double>("res.zl", (size_t)n * C), h->buf<double>("res.ph", pe),
                       h->buf<double>("res.pl", pe), rc, C, s);
    launch_copy_cols(d, (int)c, rc, C, (int)c, r, ldr, s);
  });
}

aes_status aes_tune_hp(aes_handle h, void* stream, int64_t n, int64_t d, int64_t c, const double* A, int64_t lda,
                       int precision, int twopass, int64_t rows, int reps, double* ms) {
  if (!h || !ms) return AES_ERR_INVALID_ARG;
  return guard(h, [&] {
    if (n < 1 || d < 1 || c < 1 || c > 32 || lda < d || !A || rows < 16 || rows % 16 || reps < 1)
      throw StatusError(AES_ERR_INVALID_ARG, "bad arguments (rows a multiple of 16)");
    if (d > kMaxD) throw StatusError(AES_ERR_INVALID_ARG, "d > 32768 is not supported");
    if (precision != AES_FP64 && precision != AES_MIXED_FP32) throw StatusError(AES_ERR_INVALID_ARG, "precision");
    set_device(h);
    aes_options o;
    aes_default_options(&o);
    o.precision = precision;
    const int C = (int)next_pow2(c);
    double* b = h->buf<double>("tune.b", (size_t)d * C);
    double* x = h->buf<double>("tune.x", (size_t)d * C);
    launch_fill(b, d * C, 0.0, (hipStream_t)stream);
    HpPlan plan;
    plan.twopass = twopass != 0;
    plan.rows = rows;
    BatchEngine eng(h, (hipStream_t)stream, std::vector<ProblemDesc>{ProblemDesc{n, d, C, A, lda, b, C, 1.0, nullptr, x, C}},
                    o, 1e-10, std::vector<int32_t>{0});
    *ms = eng.time_hp(plan, reps);
  });
}

aes_status aes_hv_noalloc(aes_handle h, void* stream, int64_t n, int64_t d, const double* A, int64_t lda, double nu,
                          const double* lambda, const double* p, double* q, double* pHp) {
  if (!h) return AES_ERR_INVALID_ARG;
  return guard(h, [&] {
    if (n < 1 || d < 1 || lda < d || !A || !p || !q || !(nu >= 0)) throw StatusError(AES_ERR_INVALID_ARG, "bad arguments");
    if (d > kMaxFusedD) throw StatusError(AES_ERR_INVALID_ARG, "aes_hv_noalloc takes d <= 8192");
    set_device(h);
    hv_noalloc(h->device, h->num_cu, (hipStream_t)stream, n, d, A, lda, nu, lambda, p, q, pHp);
  });
}

aes_status aes_hv_multi(aes_handle h, void* stream, int64_t n, int64_t d, int64_t c, const double* A, int64_t lda,
                        double nu, const double* lambda, const double* P, double* Q, int precision) {
  if (!h) return AES_ERR_INVALID_ARG;
  return guard(h, [&] {
    if (n < 1 || d < 1 || c < 1 || c > 32 || (c & (c - 1)) || lda < d || !A || !P || !Q || !(nu >= 0))
      throw StatusError(AES_ERR_INVALID_ARG, "bad arguments (c must be a power of two <= 32)");
    if (precision < AES_FP64 || precision > AES_MIXED_FP32) throw StatusError(AES_ERR_INVALID_ARG, "bad precision");
    set_device(h);
    aes_options o;
    aes_default_options(&o);
    o.precision = precision;
    ProblemDesc Pd{n, d, c, A, lda, P, c, nu, lambda, Q, c};
    Solver so(h, (hipStream_t)stream, Pd, o, 1e-10, "hm.");
    so.hv_external(P, Q, precision != AES_FP64);
  });
}

aes_status aes_sketch(aes_handle h, void* stream, int kind, int64_t n, int64_t d, const double* A, int64_t lda,
                      int64_t m, uint64_t seed, int32_t problem, int64_t k, double* SA) {
  if (!h) return AES_ERR_INVALID_ARG;
  return guard(h, [&] {
    const int64_t npad = next_pow2(n);
    if (n < 1 || d < 1 || lda < d || m < 1 || m > npad || !A || !SA || k < 0)
      throw StatusError(AES_ERR_INVALID_ARG, "bad arguments");
    set_device(h);
    hipStream_t s = (hipStream_t)stream;
    if (kind == AES_SRHT) {
      double* eps = h->buf<double>("sk.eps", n);
      launch_signs(seed, problem, k, n, eps, s);
      SelectScratch sc;
      sc.keys = h->buf<uint64_t>("sk.keys", npad);
      sc.pos = h->buf<int32_t>("sk.pos", npad);
      sc.hist = h->buf<uint32_t>("sk.hist", 256 * 8);
      sc.state = h->buf<uint64_t>("sk.state", 4);
      sc.blk = h->buf<uint32_t>("sk.blk", 2 * select_blocks(npad));
      launch_srht_select(seed, problem, k, npad, m, sc, s);
      double* Y = h->buf<double>("sk.Y", srht_scratch_elems(npad, d));
      launch_srht_apply<double, double, double>(A, n, d, lda, eps, npad, sc.pos, m, Y, SA, d,
                                                h->buf<int32_t>("sk.need", 512), s);
    } else if (kind == AES_SRHT_REUSE) {
      double* eps = h->buf<double>("sk.eps", n);
      launch_signs(seed, problem, 0, n, eps, s);
      SelectScratch sc;
      sc.keys = h->buf<uint64_t>("sk.keys", npad);
      sc.pos = h->buf<int32_t>("sk.pos", npad);
      sc.hist = h->buf<uint32_t>("sk.hist", 256 * 8);
      sc.state = h->buf<uint64_t>("sk.state", 4);
      sc.blk = h->buf<uint32_t>("sk.blk", 2 * select_blocks(npad));
      launch_srht_select(seed, problem, 0, npad, npad, sc, s);
      double* Yr = h->buf<double>("sk.Yreuse", (size_t)npad * d);
      launch_srht_apply<double, double, double>(A, n, d, lda, eps, npad, sc.pos, npad,
                                                h->buf<double>("sk.Y", srht_scratch_elems(npad, d)), Yr, d,
                                                h->buf<int32_t>("sk.need", 512), s);
      launch_srht_select(seed, problem, k, npad, m, sc, s);
      launch_gather_rows(npad, d, Yr, sc.pos, std::sqrt((double)npad / (double)m), SA, d, s);
    } else if (kind == AES_SRHT_NESTED) {
      double* eps = h->buf<double>("sk.eps", n);
      launch_signs(seed, problem, 0, n, eps, s);
      SelectScratch sc;
      sc.keys = h->buf<uint64_t>("sk.keys", npad);
      sc.pos = h->buf<int32_t>("sk.pos", npad);
      sc.hist = h->buf<uint32_t>("sk.hist", 256 * 8);
      sc.state = h->buf<uint64_t>("sk.state", 4);
      sc.blk = h->buf<uint32_t>("sk.blk", 2 * select_blocks(npad));
      launch_srht_select(seed, problem, 0, npad, npad, sc, s);
      double* Yr = h->buf<double>("sk.Yreuse", (size_t)npad * d);
      launch_srht_apply<double, double, double>(A, n, d, lda, eps, npad, sc.pos, npad,
                                                h->buf<double>("sk.Y", srht_scratch_elems(npad, d)), Yr, d,
                                                h->buf<int32_t>("sk.need", 512), s);
      KeyOrderScratch ko;
      ko.keys = sc.keys;
      ko.cnt = h->buf<uint32_t>("sk.ko_cnt", npad);
      ko.cur = h->buf<uint32_t>("sk.ko_cur", npad);
      ko.off = h->buf<uint32_t>("sk.ko_off", npad);
      ko.bsum = h->buf<uint32_t>("sk.ko_bsum", keyorder_sum_elems(npad));
      ko.skey = h->buf<uint64_t>("sk.ko_skey", npad);
      int32_t* order = h->buf<int32_t>("sk.ko_order", npad);
      launch_srht_key_order(seed, problem, npad, ko, order, s);
      launch_gather_ordered(m, d, Yr, order, std::sqrt((double)npad / (double)m), SA, d, s);
    } else if (kind == AES_SJLT) {
      if (n >= (int64_t(1) << 31)) throw StatusError(AES_ERR_INVALID_ARG, "the SJLT needs n < 2^31");
      const SjltPlan sp = sjlt_plan(n, d, m, sizeof(double));
      SjltScratch sc;
      sc.code = h->buf<int32_t>("sk.sj_code", n);
      sc.cnt = h->buf<int32_t>("sk.sj_cnt", sp.count_elems);
      sc.csum = h->buf<int32_t>("sk.sj_csum", sp.csum_elems);
      sc.perm = h->buf<int32_t>("sk.sj_perm", n);
      sc.part = sp.Q > 1 ? h->buf<double>("sk.sj_part", (size_t)m * sp.Q * d) : nullptr;
      launch_sjlt<double, double>(sp, A, n, d, lda, m, seed, problem, k, SA, sc, s);
    } else if (kind == AES_GAUSS) {
      const GaussPlan gp = gauss_plan(h->num_cu, n, d, m);
      launch_gauss_sketch(gp, A, n, d, lda, m, seed, problem, k, SA, h->buf<double>("sk.gt", gp.gt_elems),
                          gp.part_elems ? h->buf<double>("sk.part", gp.part_elems) : nullptr, s);
    } else {
      throw StatusError(AES_ERR_INVALID_ARG, "unknown sketch kind");
    }
  });
}

aes_status aes_factor(aes_handle h, void* stream, int64_t m, int64_t d, const double* SA, double nu,
                      const double* lambda, double* G, double* L) {
  if (!h) return AES_ERR_INVALID_ARG;
  return guard(h, [&] {
    if (m < 1 || d < 1 || !SA || !G || !L || !(nu > 0)) throw StatusError(AES_ERR_INVALID_ARG, "bad arguments");
    set_device(h);
    hipStream_t s = (hipStream_t)stream;
    const bool wb = m < d;
    const int64_t dim = wb ? m : d;
    const int64_t fp = round_up(dim, 64);
    double* Gp = h->buf<double>("fa.G", (size_t)fp * fp);
    double* invlam = h->buf<double>("fa.invlam", d);
    launch_inv(d, lambda, invlam, s);
    if (!wb) {
      const int splits = gram_splits(h->num_cu, m, d, true);
      double* part = h->buf<double>("fa.part", (size_t)splits * fp * fp);
      gram_tn(m, d, SA, d, nu * nu, lambda, part, splits, Gp, fp, s);
    } else {
      double* scaled = h->buf<double>("fa.scaled", (size_t)m * d);
      gram_nt(m, d, SA, d, nu * nu, invlam, scaled, Gp, fp, s);
    }
    // G (unpadded, full symmetric from the lower triangle)
    launch_copy_cols(dim, (int)dim, Gp, fp, (int)dim, G, dim, s);
    int* flag = h->buf<int>("fa.flag", 1);
    AES_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    double* linv = h->buf<double>("fa.linv", (size_t)fp * fp);
    double* tmp = h->buf<double>("fa.tmp", cholinv_tmp_size(fp));
    cholinv(Gp, fp, linv, tmp, flag, true, s);
    launch_copy_cols(dim, (int)dim, Gp, fp, (int)dim, L, dim, s);
    int hf = 0;
    AES_HIP(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    AES_HIP(hipStreamSynchronize(s));
    if (hf) throw StatusError(AES_ERR_NOT_SPD, "Cholesky pivot is not positive");
  });
}

aes_status aes_solve_direct(aes_handle h, void* stream, int64_t n, int64_t d, int64_t c, const double* A, int64_t lda,
                            const double* b, int64_t ldb, double nu, const double* lambda, double* x, int64_t ldx) {
  // The direct baseline of Sec. 5: H = A^T A + nu^2 Lambda formed in full (the Gram kernel with
  // S = I, O(n d^2)), its Cholesky factor and inverse factor (O(d^3)), x = L^-T (L^-1 b).
  if (!h) return AES_ERR_INVALID_ARG;
  return guard(h, [&] {
    auto bad = [](const char* m) { throw StatusError(AES_ERR_INVALID_ARG, m); };
    if (n < 1 || d < 1 || c < 1) bad("n, d and c must be >= 1");
    if (c > 32) bad("at most 32 right-hand sides");
    if (d > kMaxD) bad("d must be <= 32768");
    if (lda < d) bad("lda < d");
    if (ldb < c || ldx < c) bad("ldb and ldx must be >= c");
    if (!A || !b || !x) bad("A, b and x must be non-null");
    if (!(nu > 0) || !std::isfinite(nu)) bad("nu must be finite and > 0");
    set_device(h);
    hipStream_t s = (hipStream_t)stream;
    const int C = (int)next_pow2(c);
    const int64_t fp = round_up(d, 64);
    double* G = h->buf<double>("dir.G", (size_t)fp * fp);
    const int splits = gram_splits(h->num_cu, n, d, true);
    double* part = h->buf<double>("dir.part", (size_t)splits * fp * fp);
    gram_tn(n, d, A, lda, nu * nu, lambda, part, splits, G, fp, s);
    int* flag = h->buf<int>("dir.flag", 1);
    AES_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    double* linv = h->buf<double>("dir.linv", (size_t)fp * fp);
    double* linvT = h->buf<double>("dir.linvT", (size_t)fp * fp);
    cholinv(G, fp, linv, h->buf<double>("dir.tmp", cholinv_tmp_size(fp)), flag, false, s);
    launch_transpose(fp, fp, linv, fp, linvT, fp, s);
    double* bc = h->buf<double>("dir.b", (size_t)d * C);
    double* t = h->buf<double>("dir.t", (size_t)d * C);
    double* xc = h->buf<double>("dir.x", (size_t)d * C);
    launch_copy_cols(d, C, b, ldb, (int)c, bc, C, s);
    launch_rowdot(d, d, linv, fp, 1, bc, C, nullptr, 1.0, nullptr, nullptr, 1.0, t, s);
    launch_rowdot(d, d, linvT, fp, 2, t, C, nullptr, 1.0, nullptr, nullptr, 1.0, xc, s);
    int hf = 0;
    AES_HIP(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    AES_HIP(hipStreamSynchronize(s));
    if (hf) throw StatusError(AES_ERR_NOT_SPD, "Cholesky pivot is not positive");
    launch_copy_cols(d, (int)c, xc, C, (int)c, x, ldx, s);
  });
}

aes_status aes_precond_apply(aes_handle h, void* stream, int64_t m, int64_t d, int64_t c, const double* SA, double nu,
                             const double* lambda, const double* z, double* v) {
  if (!h) return AES_ERR_INVALID_ARG;
  return guard(h, [&] {
    if (m < 1 || d < 1 || c < 1 || c > 32 || (c & (c - 1)) || !SA || !z || !v || !(nu > 0))
      throw StatusError(AES_ERR_INVALID_ARG, "bad arguments (c must be a power of two <= 32)");
    set_device(h);
    hipStream_t s = (hipStream_t)stream;
    // Build a solver state around the given sketch (no A needed for the application).
    aes_options o;
    aes_default_options(&o);
    ProblemDesc P{std::max<int64_t>(m, 1), d, c, SA, d, z, c, nu, lambda, v, c};
    Solver so(h, s, P, o, 1e-10, "pa.");
    so.apply_external(m, SA, z, v);
  });
}

}  // extern "C"
