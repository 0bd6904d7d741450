// Device helper of the batched stages (HIP sources only): the curve a
// workgroup of a batched launch belongs to.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace nu {

// begin[c] is the first workgroup of curve c, begin[n_curves] the total:
// returns the last c with begin[c] <= b and sets local = b - begin[c].
__device__ __forceinline__ int batch_find(const int* __restrict__ begin, int n_curves, int b, int& local) {
  int lo = 0, hi = n_curves - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= b) lo = mid; else hi = mid - 1;
  }
  local = b - begin[lo];
  return lo;
}

}  // namespace nu
