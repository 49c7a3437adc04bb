// Wave-uniform broadcast of one lane's value (v_readlane): no LDS round trip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace svk {

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const uint64_t b = __double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

}  // namespace svk
