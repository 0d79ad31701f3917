// Allocation-free variant of the fused H.v entry point: the per-workgroup partials and the
// small state of the pHp reduction live in a file-scope device array instead of the handle's
// workspace pool, so the call makes no hipMalloc / hipFree (for code under graph capture and
// serving loops that must not allocate).
//
// Every call on a device shares that device's array and leaves its contents behind; calls that
// overlap on one device (different streams without ordering) race on it.
#include <mutex>

#include "aes.h"
#include "common.h"
#include "kernels.h"

using namespace aes;

namespace {

// Limits of the array: d up to the fused pass's width, at most 512 workgroups of partials.
constexpr int64_t kNaMaxD = 8192;
constexpr int64_t kNaMaxWG = 512;
// layout in doubles: part (kNaMaxWG x kNaMaxD) | spart (kNaMaxWG) | scal (16) | xp, rp (2 x kNaMaxD) | act (8)
constexpr int64_t kNaPart = 0;
constexpr int64_t kNaSpart = kNaPart + kNaMaxWG * kNaMaxD;
constexpr int64_t kNaScal = kNaSpart + kNaMaxWG;
constexpr int64_t kNaDummy = kNaScal + 16;
constexpr int64_t kNaAct = kNaDummy + 2 * kNaMaxD;
constexpr int64_t kNaTotal = kNaAct + 8;  // 4,211,224 doubles = 33.7 MB

__device__ __align__(256) double scratch[kNaTotal];

constexpr int kNaMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kNaMaxDevices] = {};  // device address of `scratch` on each device

__global__ void na_zero_int_kernel(int* p) { *p = 0; }

}  // namespace

namespace aes {

// Resolves the device address of the array on `device`, which must be the current device.
// Called once per device from aes_create; later calls return the cached address.
hipError_t noalloc_init(int device) {
  if (device < 0 || device >= kNaMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_ptr[device] = static_cast<double*>(p);
  return hipSuccess;
}

double* noalloc_scratch(int device) {
  if (device < 0 || device >= kNaMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_ptr[device];
}

// Fused H.v (d <= 8192) with the partials in the device array; same kernels, grid and order of
// summation as aes_hv, so the results are bit-identical.
void hv_noalloc(int device, int num_cu, hipStream_t s, int64_t n, int64_t d, const double* A, int64_t lda, double nu,
                const double* lambda, const double* p, double* q, double* pHp) {
  if (d > kNaMaxD) throw std::invalid_argument("aes_hv_noalloc: d > 8192 exceeds its static workspace");
  double* base = noalloc_scratch(device);
  if (!base) throw HipError("aes_hv_noalloc: the static workspace of this device is not resolved (aes_create)");
  const int nwg = hv_num_blocks(num_cu, n);
  if (nwg > kNaMaxWG) throw HipError("aes_hv_noalloc: too many workgroups for the static workspace");
  double* part = base + kNaPart;
  double* spart = base + kNaSpart;
  launch_hv_fused<double>(A, n, d, lda, p, part, spart, nwg, s);
  launch_hv_colsum(part, nwg, d, 1, p, lambda, nu * nu, 1.0, nullptr, 0.0, q, s);
  if (pHp) {
    // ||A p||^2 + nu^2 p^T Lambda p by the candidate kernel with an inactive column (it writes
    // only scal[5]; the inactive flag must start at zero: cleared by a kernel, no memset)
    double* scal = base + kNaScal;
    double* dummy = base + kNaDummy;
    int* act = reinterpret_cast<int*>(base + kNaAct);
    hipLaunchKernelGGL(na_zero_int_kernel, dim3(1), dim3(1), 0, s, act);
    AES_LAUNCH_CHECK();
    launch_pcg_candidate(d, 1, spart, nwg, lambda, nu * nu, p, p, p, q, dummy, dummy + d, scal, act, s);
    AES_HIP(hipMemcpyAsync(pHp, scal + 5, sizeof(double), hipMemcpyDeviceToDevice, s));
  }
}

}  // namespace aes
