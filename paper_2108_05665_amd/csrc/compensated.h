// FP64 compensated summation helpers shared by the device kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace xeb {

// Neumaier's improved Kahan summation: s + c carries the running sum, c the
// rounding error of every addition so far.
__device__ __forceinline__ void neumaier(double& s, double& c, double x) {
  const double t = s + x;
  if (fabs(s) >= fabs(x))
    c += (s - t) + x;
  else
    c += (x - t) + s;
  s = t;
}

// Error-free sum of two doubles (Knuth's TwoSum): s + e == a + b exactly.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

}  // namespace xeb
