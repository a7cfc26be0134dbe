// Linear XEB on the device (Eq. (1) of the paper: F = 2^n / k sum_i |amp_i|^2 - 1)
// as a compensated FP64 reduction in a fixed order, in two passes:
//  1. workgroup g sums |amp|^2 over strings [g C, (g + 1) C) (C = kXebChunk):
//     each thread a Neumaier sum over its strings in increasing order, then a
//     TwoSum tree over the workgroup; the (sum, compensation) pair goes to
//     partial slot g of a scratch buffer;
//  2. one workgroup sums the partial pairs in the same way and writes F.
// The chunking depends only on k, so the result is the same on any device
// and in every launch form.
//
// Scratch layout (device, 16-byte aligned): slot 0 holds F (one double), slots
// 1..G the partial pairs (double2), G = ceil(k / C).  Every launch writes all
// the slots it reads, so the scratch needs no clearing.

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "compensated.h"
#include "plan.h"

namespace xeb {
namespace {

constexpr int kXebThreads = 256;
constexpr int kXebFinalThreads = 1024;

// Fixed-order TwoSum tree over a workgroup's (s, c) pairs in LDS; returns the
// compensated total in thread 0.
template <int N>
__device__ __forceinline__ double2 tree_sum(double s, double c, double* ss, double* cc) {
  const int t = threadIdx.x;
  ss[t] = s;
  cc[t] = c;
  __syncthreads();
  for (int w = N / 2; w > 0; w >>= 1) {
    if (t < w) {
      double sum, err;
      two_sum(ss[t], ss[t + w], sum, err);
      ss[t] = sum;
      cc[t] = cc[t] + cc[t + w] + err;
    }
    __syncthreads();
  }
  return make_double2(ss[0], cc[0]);
}

__global__ void __launch_bounds__(kXebThreads) k_xeb_partial(const double2* amps, int64_t k,
                                                             double2* partial) {
  __shared__ double ss[kXebThreads];
  __shared__ double cc[kXebThreads];
  const int64_t begin = int64_t(blockIdx.x) * kXebChunk;
  const int64_t end = begin + kXebChunk < k ? begin + kXebChunk : k;
  double s = 0.0, c = 0.0;
  for (int64_t i = begin + threadIdx.x; i < end; i += kXebThreads) {
    const double2 a = amps[i];
    neumaier(s, c, a.x * a.x + a.y * a.y);
  }
  const double2 r = tree_sum<kXebThreads>(s, c, ss, cc);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__global__ void __launch_bounds__(kXebFinalThreads) k_xeb_final(const double2* partial, int64_t groups,
                                                                 int64_t k, int n, double* out) {
  __shared__ double ss[kXebFinalThreads];
  __shared__ double cc[kXebFinalThreads];
  double s = 0.0, c = 0.0;
  for (int64_t g = threadIdx.x; g < groups; g += kXebFinalThreads) {
    const double2 p = partial[g];
    neumaier(s, c, p.x);
    c += p.y;
  }
  const double2 r = tree_sum<kXebFinalThreads>(s, c, ss, cc);
  if (threadIdx.x == 0) out[0] = ldexp(r.x + r.y, n) / double(k) - 1.0;
}

}  // namespace

// Both passes: partial pairs in `partial` (groups slots), F in *out.
void launch_xeb_into(const double2* amps, int64_t k, int n_qubits, double2* partial, double* out,
                     hipStream_t s) {
  const int64_t groups = (k + kXebChunk - 1) / kXebChunk;
  k_xeb_partial<<<dim3(unsigned(groups)), dim3(kXebThreads), 0, s>>>(amps, k, partial);
  k_xeb_final<<<dim3(1), dim3(kXebFinalThreads), 0, s>>>(partial, groups, k, n_qubits, out);
}

// Chunk partials of the allocation-free form: one array per device for the
// life of the process, never allocated by a call.  Host code must not use
// this name as a device address: it takes the address that
// hipGetSymbolAddress returns for the current device (see static_scratch).
static __device__ __align__(256) double2 scratch[kXebStaticGroups];

// Device address of `scratch` on device `dev`, looked up once per device with
// that device current.
double2* static_scratch(int dev) {
  static std::mutex mu;
  static double2* ptr[kMaxDevices] = {};
  if (dev < 0 || dev >= kMaxDevices) fail(XEB_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) fail(XEB_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    ptr[dev] = static_cast<double2*>(p);
  }
  return ptr[dev];
}

uint64_t xeb_scratch_bytes(int64_t k) {
  const int64_t groups = k > 0 ? (k + kXebChunk - 1) / kXebChunk : 0;
  return uint64_t(1 + groups) * 16;
}

void launch_xeb(const double2* amps, int64_t k, int n_qubits, void* scratch_dev, hipStream_t s) {
  if (k <= 0) return;
  double2* slots = static_cast<double2*>(scratch_dev);
  launch_xeb_into(amps, k, n_qubits, slots + 1, reinterpret_cast<double*>(slots), s);
}

void launch_xeb_static(const double2* amps, int64_t k, int n_qubits, double* F_dev, hipStream_t s) {
  if (k <= 0) fail(XEB_EINVAL, "XEB of an empty batch");
  if (k > kXebStaticMaxStrings)
    fail(XEB_ELIMIT, "k = " + std::to_string(k) + " exceeds the allocation-free limit of " +
                         std::to_string(kXebStaticMaxStrings) + " strings");
  if (n_qubits < 1 || n_qubits > 64) fail(XEB_EINVAL, "n_qubits must be in [1, 64]");
  if (!amps || !F_dev) fail(XEB_EINVAL, "amps or F is NULL");
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  double2* partial = static_scratch(dev);
  launch_xeb_into(amps, k, n_qubits, partial, F_dev, s);
  hip_check(hipGetLastError(), "xeb launch");
}

}  // namespace xeb
