// Small device helpers shared by the kernel files.
#pragma once
#include <hip/hip_runtime.h>

namespace fb {

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).
// Remap the linear block id so that each XCD walks one contiguous range of work:
// XCD x receives the ids [x q + min(x, r), ...) of length q + (x < r), where
// total = 8 q + r.
__device__ __forceinline__ int xcd_remap(int lin, int total) {
  const int q = total >> 3, r = total & 7, x = lin & 7;
  return x * q + min(x, r) + (lin >> 3);
}

// Workgroup barrier that waits only for this wave's LDS operations, not for its global
// loads: loads issued for a later stage stay in flight across it.  Only LDS data may be
// exchanged through it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

}  // namespace fb
