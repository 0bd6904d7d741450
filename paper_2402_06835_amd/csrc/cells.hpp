// Device helpers of the (duration, epoch slot) cell grid, shared by the
// linear-search kernels (HIP sources only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace nu {

struct DurList {
  int n;
  int d[MAX_ND];     // box lengths in slots (ascending for the q kernels, caller order for the epilogue)
  int perm[MAX_ND];  // q kernels: caller index of the k-th ascending duration
  int off[MAX_ND];   // template searches: offset of the duration's shape in the concatenated shapes
};

__device__ __forceinline__ int64_t lower_bound_i64(const int64_t* __restrict__ a, int64_t n, int64_t v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Samples with lattice index below a: from the table T[s] = that count for
// s in [0, n_epochs], by binary search outside it.
__device__ __forceinline__ int64_t count_below(const int64_t* __restrict__ lattice, int64_t n,
                                               const int32_t* __restrict__ T, int64_t n_epochs, int64_t a) {
  return (a >= 0 && a <= n_epochs) ? (int64_t)T[a] : lower_bound_i64(lattice, n, a);
}

// Orders one wave's LDS writes before its later LDS reads (the waves of these
// kernels never share LDS rows, so no workgroup barrier is needed).
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace nu
