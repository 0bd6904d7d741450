// Covariance build and the per-step diagonal-block kernel of the blocked
// Cholesky factorisation (gp_factor).
//
// K[n][m] = k_SHO(|t_n - t_m|) + sigma_w^2 delta_nm with the SHO covariance of
// Appendix A; ln|K| = 2 sum ln L_nn enters Eq. 5.
#include <algorithm>

#include "batch_dev.hpp"
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
// One 64 x 64 block (br, bc), bc <= br, per workgroup.
__device__ __forceinline__ void kbuild_block(const double* __restrict__ t, int64_t n, int64_t np,
                                             const nu_sho* __restrict__ th, double* __restrict__ K, int64_t br,
                                             int64_t bc) {
  const double amp = th->amp, omega = th->omega, q = th->q, s2w = th->sigma_w * th->sigma_w;
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

// Grid: (np/64, np/64) blocks; upper blocks exit at once.
__global__ __launch_bounds__(256) void kbuild_kernel(const double* __restrict__ t, int64_t n, int64_t np,
                                                     const nu_sho* __restrict__ th, double* __restrict__ K) {
  const int64_t br = blockIdx.y, bc = blockIdx.x;
  if (bc > br) return;
  kbuild_block(t, n, np, th, K, br, bc);
}

// Lower triangle of K for a sum-of-terms covariance (nu_kernel), same layout.
__global__ __launch_bounds__(256) void kbuild_terms_kernel(const double* __restrict__ t, int64_t n, int64_t np,
                                                           const nu_kernel* __restrict__ kp, double* __restrict__ K) {
  const int64_t br = blockIdx.y, bc = blockIdx.x;
  if (bc > br) return;
  const nu_kernel k = *kp;
  const double s2w = k.sigma_w * k.sigma_w;
  const int64_t r0 = br * 64, c0 = bc * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t col = c0 + tx;
  const double tc = col < n ? t[col] : 0.0;
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t row = r0 + rr;
    if (col > row) continue;
    double v;
    if (row < n && col < n) {
      const double tau = fabs(t[row] - tc);
      v = 0.0;
      for (int s = 0; s < k.n_sho; ++s) v += sho_cov(tau, k.sho_amp[s], k.sho_omega[s], k.sho_q[s]);
      for (int e = 0; e < k.n_exp; ++e) v += k.exp_sigma[e] * k.exp_sigma[e] * exp(-tau / k.exp_ell[e]);
      if (row == col) v += s2w;
    } else {
      v = (row == col) ? 1.0 : 0.0;
    }
    K[row * np + col] = v;
  }
}

hipError_t launch_kbuild_terms(hipStream_t s, const double* t, int64_t n, int64_t np, const nu_kernel* k_dev,
                               double* K) {
  dim3 grid((unsigned)(np / 64), (unsigned)(np / 64));
  hipLaunchKernelGGL(kbuild_terms_kernel, grid, dim3(256), 0, s, t, n, np, k_dev, K);
  return hipGetLastError();
}

// theta is read from device memory, so a captured graph picks up new values
hipError_t launch_kbuild(hipStream_t s, const double* t, int64_t n, int64_t np, const nu_sho* th_dev, double* K) {
  dim3 grid((unsigned)(np / 64), (unsigned)(np / 64));
  hipLaunchKernelGGL(kbuild_kernel, grid, dim3(256), 0, s, t, n, np, th_dev, K);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Diagonal block of step k: factor the TB x TB block in LDS, write L_kk (zeros
// above the diagonal), and its inverse X_kk = L_kk^-1 into the diagonal block
// of the inverse (zeros above the diagonal).
//
// Blocked right-looking by 16: each 16 x 16 diagonal piece is factored by all
// threads with one barrier per pair of columns, the rows below it are solved against
// it by substitution (one row per thread), and the trailing pieces are
// updated on the matrix cores. The inverse starts from the eight piece
// inverses (forward substitution, one column per lane) and is completed by
// three doubling levels X21 = -X_C (L21 X_A) for the 2 x 2 partitions 16|16,
// 32|32, 64|64, also on the matrix cores.
//
// Inverse storage while in LDS: X[r][c] (r > c) is kept at a[c][r] (the
// strictly upper part, free once L is lower), its diagonal in xd[].
// ---------------------------------------------------------------------------
constexpr int DB = TB;       // 128
constexpr int DPAD = DB + 1;
constexpr int SB = 16;       // piece edge
constexpr int NSB = DB / SB; // 8

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));

// 1/x: the hardware estimate r with a third-order correction (e = 1 - x r,
// 1/x = r (1 + e + e^2 + ...); measured |e| <= 2^-24.4, result within 1 ulp)
__device__ __forceinline__ double rcp_nr(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

// 1/sqrt(x) for positive normal x: the hardware estimate r with a
// third-order correction. With h = 1 - x r^2, 1/sqrt(x) = r (1 - h)^(-1/2)
// = r (1 + h/2 + 3 h^2/8 + ...); the estimate has |h| <= 2^-23.2 (measured on
// gfx950 over 1e-300 .. 1e300), which leaves a truncation below 2^-70 and a
// result within 1.3 ulp.
__device__ __forceinline__ double rsq_nr(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  const double h = fma(-x * r, r, 1.0);
  return fma(r * h, fma(h, 0.375, 0.5), r);
}

__device__ __forceinline__ double xget(const double (*a)[DPAD], const double* xd, int r, int c) {
  return r > c ? a[c][r] : (r == c ? xd[r] : 0.0);
}

__device__ __forceinline__ dbl4 mfma64(double av, double bv, dbl4 acc) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
}

// X[r][c] of the in-LDS inverse when r > c is known to hold (a block strictly
// below the diagonal)
__device__ __forceinline__ double xlow(const double (*a)[DPAD], int r, int c) { return a[c][r]; }

// One doubling level of the in-block inverse: NODES nodes of edge 2*BS (the
// A part at a0 = node*2*BS, the C part at c0 = a0 + BS), NB = BS/16 pieces a
// side. The NB waves of a node each take one piece row (first product) or one
// piece column (second product), so every wave does the same number of
// 16 x 16 x 16 products, and every loop bound is a compile-time constant
// (straight-line code whose LDS reads the compiler issues ahead of the
// MFMAs). The sums run over the same k in the same order as a plain loop.
template <int BS, int NODES>
__device__ void inverse_level(double (*a)[DPAD], const double* xd) {
  constexpr int NB = BS / SB;
  static_assert(NB * NODES == 4, "one wave per piece row of a node");
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int node = wave / NB, wi = wave % NB;
  const int a0 = node * 2 * BS, c0 = a0 + BS;
  // T = L21 X_A: this wave's piece row bi = wi, pieces bj = 0..NB-1, k over
  // blocks bj..NB-1 (X_A is lower); kept at a[a0 + j][c0 + i] until X21 replaces it
  {
    const int bi = wi;
    dbl4 acc[NB];
#pragma unroll
    for (int bj = 0; bj < NB; ++bj) {
      acc[bj] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int bk = bj; bk < NB; ++bk)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int k = a0 + bk * SB + q * 4 + lk, col = a0 + bj * SB + lr;
          const double xa = bk > bj ? xlow(a, k, col) : xget(a, xd, k, col);
          acc[bj] = mfma64(a[c0 + bi * SB + lr][k], xa, acc[bj]);
        }
    }
#pragma unroll
    for (int bj = 0; bj < NB; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) a[a0 + bj * SB + lr][c0 + bi * SB + lk + 4 * v] = acc[bj][v];
  }
  __syncthreads();
  // X21 = -X_C T: this wave's piece column bj = wi, pieces bi = 0..NB-1, k over
  // blocks 0..bi (X_C is lower)
  const int bj = wi;
  dbl4 res[NB];
#pragma unroll
  for (int bi = 0; bi < NB; ++bi) {
    res[bi] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int bk = 0; bk <= bi; ++bk)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = c0 + bi * SB + lr, k = c0 + bk * SB + q * 4 + lk;
        const double xc = bk < bi ? xlow(a, row, k) : xget(a, xd, row, k);
        res[bi] = mfma64(-xc, a[a0 + bj * SB + lr][k], res[bi]);
      }
  }
  __syncthreads();
#pragma unroll
  for (int bi = 0; bi < NB; ++bi)
#pragma unroll
    for (int v = 0; v < 4; ++v) a[a0 + bj * SB + lr][c0 + bi * SB + lk + 4 * v] = res[bi][v];
  __syncthreads();
}

__global__ __launch_bounds__(256, 1) void potrf_diag_kernel(const PotrfJob* __restrict__ jobs) {
  __builtin_amdgcn_s_setprio(2);  // on the factorisation's critical chain: issue ahead of co-resident waves
  const PotrfJob J = jobs[blockIdx.x];
  NU_GLOBAL double* __restrict__ L = (NU_GLOBAL double*)J.L;
  NU_GLOBAL double* __restrict__ X = (NU_GLOBAL double*)J.X;
  NU_GLOBAL int64_t* __restrict__ status = (NU_GLOBAL int64_t*)J.status;
  const int64_t ld = J.ld, ldx = J.ld, off = J.off;
  __shared__ double a[DB][DPAD];
  __shared__ double xd[DB];
  __shared__ double rdg[DB];  // 1 / L_cc
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  // load the lower triangle, two columns per 16-byte load, all loads in
  // flight at once (thread tid reads columns 2 (tid & 63), +1 of rows
  // tid >> 6, +4, +8, ...); the upper triangle is set to zero
  {
    const int c = 2 * (tid & 63), r0 = tid >> 6;
    const NU_GLOBAL double* src = L + (off + r0) * ld + off + c;
    dbl2 v[DB * DB / 512];
#pragma unroll
    for (int u = 0; u < DB * DB / 512; ++u)
      v[u] = c <= r0 + 4 * u ? *(const NU_GLOBAL dbl2*)(src + 4 * u * ld) : dbl2{0.0, 0.0};
#pragma unroll
    for (int u = 0; u < DB * DB / 512; ++u) {
      const int r = r0 + 4 * u;
      a[r][c] = v[u][0];
      a[r][c + 1] = c + 1 <= r ? v[u][1] : 0.0;
    }
  }
  __syncthreads();
  // 16-byte stores of rows [r0, r1) x columns [c0, c1) of a block of L or X
  // (columns an even count), value(r, c) from LDS
  auto store_rect = [&](NU_GLOBAL double* dst, int64_t ldd, int r0, int r1, int c0, int c1, auto value) {
    const int w = (c1 - c0) / 2, cnt = (r1 - r0) * w;
    for (int idx = tid; idx < cnt; idx += 256) {
      const int r = r0 + idx / w, c = c0 + 2 * (idx % w);
      const dbl2 v = {value(r, c), value(r, c + 1)};
      *(NU_GLOBAL dbl2*)(dst + (off + r) * ldd + off + c) = v;
    }
  };
  auto lval = [&](int r, int c) { return c <= r ? a[r][c] : 0.0; };
  auto xval = [&](int r, int c) { return xget(a, xd, r, c); };
  const int pr = tid >> 4, ps = tid & 15;  // (row, column) of a 16 x 16 piece owned by this thread
  for (int kb = 0; kb < NSB; ++kb) {
    const int o = kb * SB;
    // (a) factor the 16 x 16 diagonal piece two columns per barrier: with the
    // unscaled pivot block P = [[p00, p01], [p01, p11]] of columns c, c+1,
    //   a_rs -= [a_rc, a_r,c+1] P^-1 [a_sc, a_s,c+1]^T   (s > c+1, r >= s),
    // while the previous pair is scaled into L (neither phase touches what the
    // other reads): L_rc = a_rc / sqrt(p00), and with the Schur complement
    // z = p11 - p01^2 / p00, L_r,c+1 = (a_r,c+1 - a_rc p01 / p00) / sqrt(z).
    // The last pair is scaled after the loop.
    double q00 = 1.0, q01 = 0.0, q11 = 1.0;  // pivot block of the previous pair
    for (int c = 0; c <= SB; c += 2) {
      if (c > 0 && tid < SB && tid >= c - 2) {
        const int r = tid, c0 = c - 2;
        // 1/sqrt of the two pivots; sqrt(x) = x / sqrt(x) and 1/p00 = (1/sqrt(p00))^2
        const double rd0 = rsq_nr(q00);
        const double iq00 = rd0 * rd0;
        const double z = q11 - q01 * q01 * iq00;
        const double rd1 = rsq_nr(z);
        if (r == c0) {
          if (!(q00 > 0.0) && *status < 0) *status = off + o + c0;
          else if (!(z > 0.0) && *status < 0) *status = off + o + c0 + 1;
          rdg[o + c0] = rd0;
          rdg[o + c0 + 1] = rd1;
        }
        const double ar0 = a[o + r][o + c0];
        a[o + r][o + c0] = (r == c0) ? q00 * rd0 : ar0 * rd0;
        if (r > c0) {
          const double ar1 = a[o + r][o + c0 + 1];
          a[o + r][o + c0 + 1] = (r == c0 + 1) ? z * rd1 : (ar1 - ar0 * q01 * iq00) * rd1;
        }
      }
      if (c < SB) {
        const double p00 = a[o + c][o + c], p01 = a[o + c + 1][o + c], p11 = a[o + c + 1][o + c + 1];
        const double rdet = rcp_nr(p00 * p11 - p01 * p01);
        if (ps > c + 1 && ps <= pr) {
          const double r0 = a[o + pr][o + c], r1 = a[o + pr][o + c + 1];
          const double u = (r0 * p11 - r1 * p01) * rdet, v = (r1 * p00 - r0 * p01) * rdet;
          a[o + pr][o + ps] = fma(-u, a[o + ps][o + c], fma(-v, a[o + ps][o + c + 1], a[o + pr][o + ps]));
        }
        q00 = p00;
        q01 = p01;
        q11 = p11;
      }
      __syncthreads();
    }
    // (b) rows below the piece: solve x L_dd^T = a_row by substitution
    const int nrow = DB - o - SB;
    if (tid < nrow) {
      const int r = o + SB + tid;
      double x[SB];
#pragma unroll
      for (int c = 0; c < SB; ++c) {
        double acc = a[r][o + c];
#pragma unroll
        for (int s2 = 0; s2 < c; ++s2) acc = fma(-x[s2], a[o + c][o + s2], acc);
        x[c] = acc * rdg[o + c];
      }
#pragma unroll
      for (int c = 0; c < SB; ++c) a[r][o + c] = x[c];
    }
    __syncthreads();
    // columns [o, o + 16) of L are final: store them (zeros above the
    // diagonal) while the rest of the block is factored
    store_rect(L, ld, 0, DB, o, o + SB, lval);
    // (c) trailing pieces (i, j), kb < j <= i: A_ij -= P_i P_j^T on the matrix cores
    const int m = NSB - 1 - kb;
    for (int t = wave; t < m * (m + 1) / 2; t += 4) {
      int ii = 0;
      while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
      const int jj = t - ii * (ii + 1) / 2;
      const int i0 = (kb + 1 + ii) * SB, j0 = (kb + 1 + jj) * SB;
      dbl4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = a[i0 + lk + 4 * v][j0 + lr];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = o + q * 4 + lk;
        acc = mfma64(-a[i0 + lr][k], a[j0 + lr][k], acc);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) a[i0 + lk + 4 * v][j0 + lr] = acc[v];
    }
    __syncthreads();
  }
  // ln|L_kk| = sum of ln of the diagonal: two per lane of wave 0, then a
  // fixed-order butterfly
  if (wave == 0) {
    double v = log(a[lane][lane]) + log(a[lane + 64][lane + 64]);
#pragma unroll
    for (int offs = 32; offs > 0; offs >>= 1) v += __shfl_xor(v, offs, 64);
    if (lane == 0) ((NU_GLOBAL double*)J.parts)[J.step] = 2.0 * v;
  }
  // inverses of the eight 16 x 16 diagonal pieces, all at once: wave w takes
  // pieces w (lanes 0-15) and w + 4 (lanes 16-31), lane j forms column j by
  // forward substitution
  if (lane < 2 * SB) {
    const int o = (wave + 4 * (lane >> 4)) * SB, j = lane & 15;
    double x[SB];
#pragma unroll
    for (int i = 0; i < SB; ++i) {
      double acc = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int s2 = 0; s2 < i; ++s2) acc = fma(-a[o + i][o + s2], x[s2], acc);
      x[i] = (i >= j) ? acc * rdg[o + i] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < SB; ++i) {
      if (i > j) a[o + j][o + i] = x[i];
      if (i == j) xd[o + j] = x[i];
    }
  }
  __syncthreads();
  inverse_level<16, 4>(a, xd);
  inverse_level<32, 2>(a, xd);
  // the two 64 x 64 diagonal blocks of X and the zeros right of the first are
  // final (the last level only reads them): stored while it runs
  store_rect(X, ldx, 0, DB / 2, 0, DB, xval);
  store_rect(X, ldx, DB / 2, DB, DB / 2, DB, xval);
  inverse_level<64, 1>(a, xd);
  store_rect(X, ldx, DB / 2, DB, 0, DB / 2, xval);
}

// one workgroup per job (one diagonal block per factor of a batch)
hipError_t launch_potrf_diag(hipStream_t s, const PotrfJob* jobs, int njobs) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(potrf_diag_kernel, dim3((unsigned)njobs), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

__global__ void fill_i64_kernel(int64_t* __restrict__ p, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

hipError_t launch_fill_i64(hipStream_t s, int64_t* p, int64_t v) {
  hipLaunchKernelGGL(fill_i64_kernel, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

__global__ void copy_i64_kernel(const int64_t* __restrict__ src, int64_t* __restrict__ dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

hipError_t launch_copy_i64(hipStream_t s, const int64_t* src, int64_t* dst) {
  hipLaunchKernelGGL(copy_i64_kernel, dim3(1), dim3(64), 0, s, src, dst);
  return hipGetLastError();
}

// outputs of a light curve whose covariance could not be factored: every
// cell invalid (depth 0, var +inf, dll 0) and no event at any period
__global__ void fill_invalid_cells_kernel(int64_t count, double* __restrict__ depth, double* __restrict__ var,
                                          double* __restrict__ dll, uint8_t* __restrict__ valid) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    depth[i] = 0.0;
    var[i] = INFINITY;
    dll[i] = 0.0;
    valid[i] = 0;
  }
}

hipError_t launch_fill_invalid_cells(hipStream_t s, int64_t count, double* depth, double* var, double* dll,
                                     uint8_t* valid) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_invalid_cells_kernel, dim3((unsigned)blocks), dim3(256), 0, s, count, depth, var, dll,
                     valid);
  return hipGetLastError();
}

__global__ void fill_no_event_kernel(int64_t n_p, double* __restrict__ q_snr, int64_t* __restrict__ best_phase,
                                     int32_t* __restrict__ best_dur, double* __restrict__ best_depth,
                                     double* __restrict__ best_sigma, double* __restrict__ best_lnp,
                                     int64_t* __restrict__ best_period) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 == 0 && best_period) *best_period = -1;
  for (int64_t i = i0; i < n_p; i += (int64_t)gridDim.x * blockDim.x) {
    q_snr[i] = 0.0;
    best_phase[i] = -1;
    best_dur[i] = -1;
    best_depth[i] = 0.0;
    best_sigma[i] = 0.0;
    best_lnp[i] = -INFINITY;
  }
}

hipError_t launch_fill_no_event(hipStream_t s, int64_t n_p, double* q_snr, int64_t* best_phase, int32_t* best_dur,
                                double* best_depth, double* best_sigma, double* best_lnp, int64_t* best_period) {
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n_p + 255) / 256, 4096));
  hipLaunchKernelGGL(fill_no_event_kernel, dim3((unsigned)blocks), dim3(256), 0, s, n_p, q_snr, best_phase, best_dur,
                     best_depth, best_sigma, best_lnp, best_period);
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

// ---------------------------------------------------------------------------
// Batched stages of the factorisation (one launch for every curve of a batch)

// status = -1 of every curve (one thread per curve)
__global__ __launch_bounds__(64) void batch_init_kernel(const CurveJob* __restrict__ jobs, int n_curves) {
  const int c = blockIdx.x * 64 + threadIdx.x;
  if (c < n_curves) *jobs[c].status = -1;
}

hipError_t launch_batch_init(hipStream_t s, const CurveJob* jobs, int n_curves) {
  hipLaunchKernelGGL(batch_init_kernel, dim3((unsigned)((n_curves + 63) / 64)), dim3(64), 0, s, jobs, n_curves);
  return hipGetLastError();
}

__global__ __launch_bounds__(64) void batch_collect_kernel(const CurveJob* __restrict__ jobs, int n_curves,
                                                           int64_t* __restrict__ status_out,
                                                           double* __restrict__ logdet_out) {
  const int c = blockIdx.x * 64 + threadIdx.x;
  if (c >= n_curves) return;
  const CurveJob& J = jobs[c];
  status_out[J.curve] = *J.status;
  logdet_out[J.curve] = *J.logdet;
}

hipError_t launch_batch_collect(hipStream_t s, const CurveJob* jobs, int n_curves, int64_t* status_out,
                                double* logdet_out) {
  hipLaunchKernelGGL(batch_collect_kernel, dim3((unsigned)((n_curves + 63) / 64)), dim3(64), 0, s, jobs, n_curves,
                     status_out, logdet_out);
  return hipGetLastError();
}

// lower 64 x 64 blocks of every curve's K, numbered row by row within a curve
__global__ __launch_bounds__(256) void batch_kbuild_kernel(const CurveJob* __restrict__ jobs,
                                                           const int* __restrict__ begin, int n_curves) {
  int u;
  const int c = batch_find(begin, n_curves, (int)blockIdx.x, u);
  const CurveJob& J = jobs[c];
  int64_t br = (int64_t)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5);
  while ((br + 1) * (br + 2) / 2 <= u) ++br;
  while (br * (br + 1) / 2 > u) --br;
  const int64_t bc = u - br * (br + 1) / 2;
  kbuild_block(J.t, J.n, J.np, J.theta, J.L, br, bc);
}

hipError_t launch_batch_kbuild(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_kbuild_kernel, dim3((unsigned)total), dim3(256), 0, s, jobs, begin, n_curves);
  return hipGetLastError();
}

// ln|K| of every curve (one workgroup per curve; the same order as logdet_reduce_kernel)
__global__ __launch_bounds__(64) void batch_logdet_kernel(const CurveJob* __restrict__ jobs) {
  const CurveJob& J = jobs[blockIdx.x];
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int i = 0; i < J.nblk; ++i) sum += J.parts[i];
    *J.logdet = sum;
  }
}

hipError_t launch_batch_logdet(hipStream_t s, const CurveJob* jobs, int n_curves) {
  hipLaunchKernelGGL(batch_logdet_kernel, dim3((unsigned)n_curves), dim3(64), 0, s, jobs);
  return hipGetLastError();
}

}  // namespace nu
