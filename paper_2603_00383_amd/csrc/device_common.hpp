// Device helpers shared by the kernel sources.
#pragma once

#include "kernels.hpp"

namespace seas {

__device__ __forceinline__ int64_t ring_slot(int64_t t, int64_t R) {
  int64_t s = t % R;
  return s < 0 ? s + R : s;
}

typedef float mfma_f4 __attribute__((ext_vector_type(4)));

static inline int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace seas
