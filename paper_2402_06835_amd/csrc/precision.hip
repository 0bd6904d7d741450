// Reduced-precision triangular inverse support: FP64 <-> FP32 copies of the
// lower TB-blocks, and the block band moved between the inverse and the
// refinement buffer.
//
// The mixed inverse X = L^-1 is formed by the same bottom-up doubling as the
// FP64 one, with the level products in FP32 on the matrix cores; the FP64
// diagonal blocks (from the factorisation) are kept. One Newton step
//   X1 = X + X (I - L X) = 2 X - X (L X)
// is then applied to the blocks within `w` of the diagonal, in FP64. For
// triangular matrices, block (I, J) of either product involves only the
// blocks J..I, so the band is refined exactly from the band alone. The box
// sums q of the linear search draw almost all of their weight from that
// band, where the refinement restores FP64 accuracy.
#include "internal.hpp"

namespace nu {

// dst = (float) src on the lower blocks (bi >= bj), or on the diagonal blocks only
__global__ __launch_bounds__(256) void cvt_f64_f32_kernel(const double* __restrict__ src, float* __restrict__ dst,
                                                          int64_t np, int diag_only, int cb0, int cb1) {
  const int bi = blockIdx.y, bj = diag_only ? blockIdx.y : cb0 + (int)blockIdx.x;
  if (bj > bi || bj < cb0 || bj >= cb1) return;
  const double* s = src + (int64_t)bi * TB * np + (int64_t)bj * TB;
  float* d = dst + (int64_t)bi * TB * np + (int64_t)bj * TB;
  for (int idx = threadIdx.x; idx < TB * TB; idx += 256) {
    const int r = idx >> 7, c = idx & (TB - 1);
    d[(int64_t)r * np + c] = (float)s[(int64_t)r * np + c];
  }
}

// dst = (float) src on the lower blocks (bi >= bj) of block columns [cb0, cb1),
// or on their diagonal blocks only
hipError_t launch_cvt_f64_f32(hipStream_t s, const double* src, float* dst, int64_t np, int diag_only, int cb0,
                              int cb1) {
  const int nb = (int)(np / TB);
  cb0 = cb0 < 0 ? 0 : cb0;
  cb1 = cb1 > nb ? nb : cb1;
  if (cb1 <= cb0) return hipSuccess;
  hipLaunchKernelGGL(cvt_f64_f32_kernel, dim3(diag_only ? 1u : (unsigned)(cb1 - cb0), (unsigned)nb), dim3(256), 0, s,
                     src, dst, np, diag_only, cb0, cb1);
  return hipGetLastError();
}

// dst = (double) src on the strictly lower blocks (bi > bj)
__global__ __launch_bounds__(256) void cvt_f32_f64_kernel(const float* __restrict__ src, double* __restrict__ dst,
                                                          int64_t np) {
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bj >= bi) return;
  const float* s = src + (int64_t)bi * TB * np + (int64_t)bj * TB;
  double* d = dst + (int64_t)bi * TB * np + (int64_t)bj * TB;
  for (int idx = threadIdx.x; idx < TB * TB; idx += 256) {
    const int r = idx >> 7, c = idx & (TB - 1);
    d[(int64_t)r * np + c] = (double)s[(int64_t)r * np + c];
  }
}

hipError_t launch_cvt_f32_f64(hipStream_t s, const float* src, double* dst, int64_t np) {
  const unsigned nb = (unsigned)(np / TB);
  hipLaunchKernelGGL(cvt_f32_f64_kernel, dim3(nb, nb), dim3(256), 0, s, src, dst, np);
  return hipGetLastError();
}

// Band blocks (I, I - d), d = 1..w, between X (np x np) and the band buffer
// (block (I, d) at ((I * (w + 1) + d) * TB * TB), TB x TB row-major).
__global__ __launch_bounds__(256) void band_copy_kernel(double* __restrict__ X, int64_t np,
                                                        double* __restrict__ band, int w, int to_band) {
  const int e = blockIdx.x;
  const int I = e / w, d = 1 + e % w, J = I - d;
  if (J < 0) return;
  double* x = X + (int64_t)I * TB * np + (int64_t)J * TB;
  double* b = band + ((int64_t)I * (w + 1) + d) * TB * TB;
  for (int idx = threadIdx.x; idx < TB * TB; idx += 256) {
    const int r = idx >> 7, c = idx & (TB - 1);
    if (to_band)
      b[idx] = x[(int64_t)r * np + c];
    else
      x[(int64_t)r * np + c] = b[idx];
  }
}

hipError_t launch_band_copy(hipStream_t s, double* X, int64_t np, double* band, int w, int to_band) {
  const int nb = (int)(np / TB);
  if (w <= 0 || nb <= 1) return hipSuccess;
  hipLaunchKernelGGL(band_copy_kernel, dim3((unsigned)(nb * w)), dim3(256), 0, s, X, np, band, w, to_band);
  return hipGetLastError();
}

}  // namespace nu
