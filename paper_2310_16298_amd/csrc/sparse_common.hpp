// Shared pieces of the nonzero-tap gather kernels (GENERAL stencils).
#pragma once

#include "device_common.hpp"

namespace stencil {

// Value of v in lane t (t wave-uniform), as a wave-uniform value.
template <typename T>
__device__ __forceinline__ T lane_value(T v, int t) {
  if constexpr (sizeof(T) == 4) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), t));
  } else {
    const long long u = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(u & 0xffffffffLL), t);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), t);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
  }
}

}  // namespace stencil
