// Covariance build and the per-step diagonal-block kernel of the blocked
// Cholesky factorisation (gp_factor).
//
// K[n][m] = k_SHO(|t_n - t_m|) + sigma_w^2 delta_nm with the SHO covariance of
// Appendix A; ln|K| = 2 sum ln L_nn enters Eq. 5.
#include "internal.hpp"

namespace nu {

// SHO covariance of Appendix A, branch by quality factor.
__device__ __forceinline__ double sho_cov(double tau, double amp, double omega, double q) {
  const double x = omega * tau / (2.0 * q);
  const double env = amp * amp * exp(-x);
  if (q == 0.5) return env * (1.0 + omega * tau);
  if (q < 0.5) {
    const double f = sqrt(1.0 - 4.0 * q * q);
    return env * (cosh(f * x) + sinh(f * x) / f);
  }
  const double g = sqrt(4.0 * q * q - 1.0);
  double s, c;
  sincos(g * x, &s, &c);
  return env * (c + s / g);
}

// Lower triangle of K, padded: rows/columns n >= N hold the identity.
// Grid: (np/64, np/64) blocks of 64 x 64; upper blocks exit at once.
__global__ __launch_bounds__(256) void kbuild_kernel(const double* __restrict__ t, int64_t n, int64_t np,
                                                     double amp, double omega, double q, double s2w,
                                                     double* __restrict__ K) {
  const int64_t br = blockIdx.y, bc = blockIdx.x;
  if (bc > br) return;
  const int64_t r0 = br * 64, c0 = bc * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 columns x 4 rows per pass
  const int64_t col = c0 + tx;
  const double tc = col < n ? t[col] : 0.0;
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t row = r0 + rr;
    if (col > row) continue;
    double v;
    if (row < n && col < n) {
      v = sho_cov(fabs(t[row] - tc), amp, omega, q);
      if (row == col) v += s2w;
    } else {
      v = (row == col) ? 1.0 : 0.0;
    }
    K[row * np + col] = v;
  }
}

hipError_t launch_kbuild(hipStream_t s, const double* t, int64_t n, int64_t np, const nu_sho& th, double* K) {
  dim3 grid((unsigned)(np / 64), (unsigned)(np / 64));
  hipLaunchKernelGGL(kbuild_kernel, grid, dim3(256), 0, s, t, n, np, th.amp, th.omega, th.q,
                     th.sigma_w * th.sigma_w, K);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Diagonal block of step k: factor the TB x TB block in LDS, write L_kk (zeros
// above the diagonal), then invert it in place and write X_kk = L_kk^-1 into
// the inverse's diagonal block (zeros above the diagonal).
//
// Inverse storage while in LDS: the strictly lower part of X_kk is kept
// transposed in the strictly upper part of the array (free once L_kk is
// lower), its diagonal in xd[]. The inverse is built bottom-up: the four
// 32 x 32 diagonal blocks by forward substitution, then two doubling levels
//   X21 = -X_C (L21 X_A)
// for the 2 x 2 block partition [[A, 0], [L21, C]].
// ---------------------------------------------------------------------------
constexpr int DB = TB;       // 128
constexpr int DPAD = DB + 1;

__device__ __forceinline__ double xinv(const double (*a)[DPAD], const double* xd, int r, int c) {
  // element (r, c) of the inverse, r >= c, within an already-inverted block
  return r == c ? xd[r] : a[c][r];
}

// One doubling level: nodes at A-block offsets a0 = node*2*BS, C-block at a0+BS.
template <int BS, int NODES>
__device__ void inverse_level(double (*a)[DPAD], const double* xd) {
  constexpr int PER_NODE = BS * BS;
  constexpr int TOTAL = PER_NODE * NODES;
  constexpr int PER_THREAD = TOTAL / 256;
  static_assert(TOTAL % 256 == 0, "level must split evenly over 256 threads");
  const int tid = threadIdx.x;
  // T = L21 X_A, stored at a[a0 + j][c0 + i] (upper region of this node, free)
#pragma unroll
  for (int u = 0; u < PER_THREAD; ++u) {
    const int idx = tid + 256 * u;
    const int node = idx / PER_NODE, e = idx % PER_NODE;
    const int i = e / BS, j = e % BS;
    const int a0 = node * 2 * BS, c0 = a0 + BS;
    double acc = 0.0;
    for (int k = j; k < BS; ++k) acc = fma(a[c0 + i][a0 + k], xinv(a, xd, a0 + k, a0 + j), acc);
    a[a0 + j][c0 + i] = acc;
  }
  __syncthreads();
  // X21 = -X_C T into registers, then overwrite T
  double out[PER_THREAD];
#pragma unroll
  for (int u = 0; u < PER_THREAD; ++u) {
    const int idx = tid + 256 * u;
    const int node = idx / PER_NODE, e = idx % PER_NODE;
    const int i = e / BS, j = e % BS;
    const int a0 = node * 2 * BS, c0 = a0 + BS;
    double acc = 0.0;
    for (int k = 0; k <= i; ++k) acc = fma(xinv(a, xd, c0 + i, c0 + k), a[a0 + j][c0 + k], acc);
    out[u] = -acc;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER_THREAD; ++u) {
    const int idx = tid + 256 * u;
    const int node = idx / PER_NODE, e = idx % PER_NODE;
    const int i = e / BS, j = e % BS;
    const int a0 = node * 2 * BS, c0 = a0 + BS;
    a[a0 + j][c0 + i] = out[u];
  }
  __syncthreads();
}

__global__ __launch_bounds__(256, 1) void potrf_diag_kernel(double* __restrict__ L, int64_t ld, int64_t off,
                                                           int step, double* __restrict__ logdet_parts,
                                                           int64_t* __restrict__ status, double* __restrict__ X,
                                                           int64_t ldx) {
  __shared__ double a[DB][DPAD];
  __shared__ double xd[DB];
  __shared__ double piv;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < DB * DB; idx += 256) {
    const int r = idx / DB, c = idx - (idx / DB) * DB;
    a[r][c] = c <= r ? L[(off + r) * ld + off + c] : 0.0;
  }
  __syncthreads();
  double logsum = 0.0;
  // right-looking, one column at a time; thread (s, rpar) owns column s and
  // the rows r >= s of parity rpar in the trailing update
  const int s_col = tid & (DB - 1), rpar = tid >> 7;
  for (int c = 0; c < DB; ++c) {
    if (tid == 0) {
      const double p = a[c][c];
      if (!(p > 0.0) && *status < 0) *status = off + c;
      const double d = sqrt(p);
      a[c][c] = d;
      piv = d;
      logsum += log(d);
    }
    __syncthreads();
    if (tid > c && tid < DB) a[tid][c] = a[tid][c] / piv;
    __syncthreads();
    if (s_col > c) {
      const double asc = a[s_col][c];
      for (int r = s_col + rpar; r < DB; r += 2) a[r][s_col] = fma(-a[r][c], asc, a[r][s_col]);
    }
    __syncthreads();
  }
  if (tid == 0) logdet_parts[step] = 2.0 * logsum;
  for (int idx = tid; idx < DB * DB; idx += 256) {
    const int r = idx / DB, c = idx - (idx / DB) * DB;
    L[(off + r) * ld + off + c] = c <= r ? a[r][c] : 0.0;
  }
  __syncthreads();
  // ---- inverse of the four 32 x 32 diagonal blocks: wave w, lane = column ----
  {
    const int w = tid >> 6, lane = tid & 63;
    const int b0 = w * 32;
    if (lane < 32) {
      const int c = lane;
      double x[32];
#pragma unroll
      for (int r = 0; r < 32; ++r) {
        double acc = (r == c) ? 1.0 : 0.0;
#pragma unroll
        for (int s = 0; s < r; ++s)
          if (s >= c) acc = fma(-a[b0 + r][b0 + s], x[s], acc);
        x[r] = (r >= c) ? acc / a[b0 + r][b0 + r] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < 32; ++r) {
        if (r == c) xd[b0 + c] = x[r];
        if (r > c) a[b0 + c][b0 + r] = x[r];
      }
    }
  }
  __syncthreads();
  inverse_level<32, 2>(a, xd);
  inverse_level<64, 1>(a, xd);
  for (int idx = tid; idx < DB * DB; idx += 256) {
    const int r = idx / DB, c = idx - (idx / DB) * DB;
    X[(off + r) * ldx + off + c] = r > c ? a[c][r] : (r == c ? xd[r] : 0.0);
  }
}

hipError_t launch_potrf_diag(hipStream_t s, double* L, int64_t ld, int64_t off, int step, double* logdet_parts,
                             int64_t* status, double* Xdiag, int64_t ldx) {
  hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, s, L, ld, off, step, logdet_parts, status, Xdiag,
                     ldx);
  return hipGetLastError();
}

__global__ void fill_i64_kernel(int64_t* __restrict__ p, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

hipError_t launch_fill_i64(hipStream_t s, int64_t* p, int64_t v) {
  hipLaunchKernelGGL(fill_i64_kernel, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

__global__ void logdet_reduce_kernel(const double* __restrict__ parts, int nparts, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += parts[i];
    *out = s;
  }
}

hipError_t launch_logdet_reduce(hipStream_t s, const double* parts, int nparts, double* out) {
  hipLaunchKernelGGL(logdet_reduce_kernel, dim3(1), dim3(64), 0, s, parts, nparts, out);
  return hipGetLastError();
}

}  // namespace nu
