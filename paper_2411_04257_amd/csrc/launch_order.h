// Workgroup launch order on an 8-XCD device (host and device arithmetic).
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define LB_LO_FN __host__ __device__ __forceinline__
#else
#define LB_LO_FN static inline
#endif

namespace lb {

// The device hands a launch's workgroups to its 8 XCDs in turn (workgroup L
// to XCD L mod 8).  xcd_contiguous(L, total) renumbers them so that each XCD
// takes a contiguous, ordered range of [0, total): XCD x holds
// floor(total / 8) numbers, one more if x < total mod 8, after those of XCDs
// 0..x-1.  A bijection of [0, total).
LB_LO_FN uint32_t xcd_contiguous(uint32_t L, uint32_t total) {
  const uint32_t x = L & 7u, i = L >> 3, q = total >> 3, r = total & 7u;
  return x * q + (x < r ? x : r) + i;
}

}  // namespace lb
