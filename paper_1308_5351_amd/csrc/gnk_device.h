// Device helpers shared by the pair kernels (Cauchy sums of the operators and
// of the geometric derivatives).
#pragma once

#include <hip/hip_runtime.h>

namespace gnk {

// Pointers into global memory. In the device pass they carry address space 1,
// so wave-uniform loads through them compile to scalar loads (a generic
// pointer read from a table in memory would give per-lane flat loads). The
// host pass only parses kernel bodies and keeps plain pointers.
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using gptr = __attribute__((address_space(1))) T*;
#else
template <class T>
using gptr = T*;
#endif

// v_rcp_f64 is accurate to about 2^-24 on gfx950; one Newton step brings the
// reciprocal to about 2^-48 (a few ulp), below the rounding of the sums.
__device__ __forceinline__ double refine_rcp(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  const double e = __builtin_fma(-d, r, 1.0);
  return __builtin_fma(r, e, r);
}

}  // namespace gnk
