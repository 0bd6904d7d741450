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
#include "batch_dev.hpp"
#include "internal.hpp"

namespace nu {

// one TB x TB block (bi, bj) of dst = (float) src
__device__ __forceinline__ void cvt_f64_f32_block(const double* __restrict__ src, float* __restrict__ dst, int64_t np,
                                                  int bi, int bj) {
  const double* s = src + (int64_t)bi * TB * np + (int64_t)bj * TB;
  float* d = dst + (int64_t)bi * TB * np + (int64_t)bj * TB;
  for (int idx = threadIdx.x; idx < TB * TB; idx += 256) {
    const int r = idx >> 7, c = idx & (TB - 1);
    d[(int64_t)r * np + c] = (float)s[(int64_t)r * np + c];
  }
}

// dst = (float) src on the lower blocks (bi >= bj), or on the diagonal blocks only
__global__ __launch_bounds__(256) void cvt_f64_f32_kernel(const double* __restrict__ src, float* __restrict__ dst,
                                                          int64_t np, int diag_only, int cb0, int cb1) {
  const int bi = blockIdx.y, bj = diag_only ? blockIdx.y : cb0 + (int)blockIdx.x;
  if (bj > bi || bj < cb0 || bj >= cb1) return;
  cvt_f64_f32_block(src, dst, np, bi, bj);
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

__device__ __forceinline__ void cvt_f32_f64_block(const float* __restrict__ src, double* __restrict__ dst, int64_t np,
                                                  int bi, int bj) {
  const float* s = src + (int64_t)bi * TB * np + (int64_t)bj * TB;
  double* d = dst + (int64_t)bi * TB * np + (int64_t)bj * TB;
  for (int idx = threadIdx.x; idx < TB * TB; idx += 256) {
    const int r = idx >> 7, c = idx & (TB - 1);
    d[(int64_t)r * np + c] = (double)s[(int64_t)r * np + c];
  }
}

// dst = (double) src on the strictly lower blocks (bi > bj)
__global__ __launch_bounds__(256) void cvt_f32_f64_kernel(const float* __restrict__ src, double* __restrict__ dst,
                                                          int64_t np) {
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bj >= bi) return;
  cvt_f32_f64_block(src, dst, np, bi, bj);
}

hipError_t launch_cvt_f32_f64(hipStream_t s, const float* src, double* dst, int64_t np) {
  const unsigned nb = (unsigned)(np / TB);
  hipLaunchKernelGGL(cvt_f32_f64_kernel, dim3(nb, nb), dim3(256), 0, s, src, dst, np);
  return hipGetLastError();
}

// Band blocks (I, I - d), d = 1..w, between X (np x np) and the band buffer
// (block (I, d) at ((I * (w + 1) + d) * TB * TB), TB x TB row-major).
__device__ __forceinline__ void band_copy_block(double* __restrict__ X, int64_t np, double* __restrict__ band, int w,
                                                int to_band, int e) {
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

__global__ __launch_bounds__(256) void band_copy_kernel(double* __restrict__ X, int64_t np,
                                                        double* __restrict__ band, int w, int to_band) {
  band_copy_block(X, np, band, w, to_band, (int)blockIdx.x);
}

hipError_t launch_band_copy(hipStream_t s, double* X, int64_t np, double* band, int w, int to_band) {
  const int nb = (int)(np / TB);
  if (w <= 0 || nb <= 1) return hipSuccess;
  hipLaunchKernelGGL(band_copy_kernel, dim3((unsigned)(nb * w)), dim3(256), 0, s, X, np, band, w, to_band);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched forms (one launch for every curve of a batch; workgroups numbered
// curve after curve, see CurveJob)

// (bi, bj) of the u-th block of the lower block triangle, row by row
__device__ __forceinline__ void lower_block(int u, int& bi, int& bj) {
  int r = (int)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= u) ++r;
  while (r * (r + 1) / 2 > u) --r;
  bi = r;
  bj = u - r * (r + 1) / 2;
}

// L32 = (float) L on every lower block
__global__ __launch_bounds__(256) void batch_cvt_l_kernel(const CurveJob* __restrict__ jobs,
                                                          const int* __restrict__ begin, int n_curves) {
  int u, bi, bj;
  const CurveJob& J = jobs[batch_find(begin, n_curves, (int)blockIdx.x, u)];
  lower_block(u, bi, bj);
  cvt_f64_f32_block(J.L, J.L32, J.np, bi, bj);
}

// X32 = (float) X on the diagonal blocks
__global__ __launch_bounds__(256) void batch_cvt_xd_kernel(const CurveJob* __restrict__ jobs,
                                                           const int* __restrict__ begin, int n_curves) {
  int u;
  const CurveJob& J = jobs[batch_find(begin, n_curves, (int)blockIdx.x, u)];
  cvt_f64_f32_block(J.X, J.X32, J.np, u, u);
}

// X = (double) X32 on the strictly lower blocks
__global__ __launch_bounds__(256) void batch_cvt_back_kernel(const CurveJob* __restrict__ jobs,
                                                             const int* __restrict__ begin, int n_curves) {
  int u, bi, bj;
  const CurveJob& J = jobs[batch_find(begin, n_curves, (int)blockIdx.x, u)];
  lower_block(u, bi, bj);
  cvt_f32_f64_block(J.X32, J.X, J.np, bi + 1, bj);  // strictly lower: row blocks 1.. against the triangle
}

__global__ __launch_bounds__(256) void batch_band_copy_kernel(const CurveJob* __restrict__ jobs,
                                                              const int* __restrict__ begin, int n_curves, int w,
                                                              int to_band) {
  int u;
  const CurveJob& J = jobs[batch_find(begin, n_curves, (int)blockIdx.x, u)];
  band_copy_block(J.X, J.np, J.bandX, w, to_band, u);
}

hipError_t launch_batch_cvt_l(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_cvt_l_kernel, dim3((unsigned)total), dim3(256), 0, s, jobs, begin, n_curves);
  return hipGetLastError();
}

hipError_t launch_batch_cvt_xd(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_cvt_xd_kernel, dim3((unsigned)total), dim3(256), 0, s, jobs, begin, n_curves);
  return hipGetLastError();
}

hipError_t launch_batch_cvt_back(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_cvt_back_kernel, dim3((unsigned)total), dim3(256), 0, s, jobs, begin, n_curves);
  return hipGetLastError();
}

hipError_t launch_batch_band_copy(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total,
                                  int w, int to_band) {
  if (total <= 0 || w <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_band_copy_kernel, dim3((unsigned)total), dim3(256), 0, s, jobs, begin, n_curves, w,
                     to_band);
  return hipGetLastError();
}

}  // namespace nu
