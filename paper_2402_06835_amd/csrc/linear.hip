// Linear search (Section 2.2, Eqs. 5-6) on top of the factor K = L L^T and the
// triangular inverse X = L^-1.
//
// For the cell (duration j, epoch slot i) the design is X_ij = [A | b] with
// b = -1 on the box samples [lo, hi). With G0 = A^T K^-1 A, the Schur
// complement of the trend block gives the box coefficient of Eq. 6 exactly:
//   q = b^T K^-1 b = ||L^-1 b||^2 = sum_n (sum_{m in [lo,hi)} X[n][m])^2
//   g = A^T K^-1 b = -sum_{n in [lo,hi)} (K^-1 A)[n]
//   h = b^T K^-1 r0 = -sum_{n in [lo,hi)} (K^-1 r0)[n],   r0 = f - A w0
//   S = q - g^T G0^-1 g,  depth = h / S,  var = 1 / S,  dll = h^2 / (2 S)
// where w0 is the trend-only fit and dll = ln L_ij - ln L_0 (Eq. 5).
//
// Kernels, in launch order:
//   pack_v        V = [A | f] row-major
//   rows_matvec   Y = X V                 (whitened trend and flux; one wave per row)
//   null_solve    trend-only GLS, r~0 = f~ - A~ w0, chi2_0, ln L_0
//   cols_matvec   Z = X^T [A~ | r~0] = [K^-1 A | K^-1 r0]   (row-chunk partials + reduce)
// With an inverse X computed in reduced precision, Y and Z each get one step
// of iterative refinement against the FP64 factor: Y += X (V - L Y) and
// Z += X^T (W - L^T Z).
//   q_partial     per cell, sum over a row chunk of the squared box window sums of X
//   cell_epilogue per cell: g, h from window sums of Z, Schur complement, outputs
#include <algorithm>

#include "batch_dev.hpp"
#include "cells.hpp"
#include "internal.hpp"

namespace nu {

__device__ __forceinline__ void slot_count_at(const int64_t* __restrict__ lattice, int64_t n, int64_t n_epochs,
                                              int32_t* __restrict__ T, int64_t s) {
  if (s <= n_epochs) T[s] = (int32_t)lower_bound_i64(lattice, n, s);
}

__global__ __launch_bounds__(256) void slot_count_kernel(const int64_t* __restrict__ lattice, int64_t n,
                                                         int64_t n_epochs, int32_t* __restrict__ T) {
  slot_count_at(lattice, n, n_epochs, T, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

hipError_t launch_slot_count(hipStream_t s, const int64_t* lattice, int64_t n, int64_t n_epochs, int32_t* T) {
  hipLaunchKernelGGL(slot_count_kernel, dim3((unsigned)((n_epochs + 1 + 255) / 256)), dim3(256), 0, s, lattice, n,
                     n_epochs, T);
  return hipGetLastError();
}

// The lattice the searches assume: lattice[0] == 0, strictly increasing,
// lattice[n - 1] == n_epochs - 1. One workgroup; *ok = 1 if it holds, else 0.
// The trend fit reads the flag, so a lattice that breaks it leaves every cell
// invalid and ln L_0 = NaN (the call itself does not synchronise to report it).
__device__ __forceinline__ void lattice_check_block(const int64_t* __restrict__ lattice, int64_t n, int64_t n_epochs,
                                                    int* __restrict__ ok) {
  bool bad = false;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const int64_t v = lattice[i];
    if (i == 0) bad = bad || v != 0;
    else bad = bad || v <= lattice[i - 1];
    if (i == n - 1) bad = bad || v != n_epochs - 1;
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) *ok = bad ? 0 : 1;
}

__global__ __launch_bounds__(256) void lattice_check_kernel(const int64_t* __restrict__ lattice, int64_t n,
                                                            int64_t n_epochs, int* __restrict__ ok) {
  lattice_check_block(lattice, n, n_epochs, ok);
}

hipError_t launch_lattice_check(hipStream_t s, const int64_t* lattice, int64_t n, int64_t n_epochs, int* ok) {
  hipLaunchKernelGGL(lattice_check_kernel, dim3(1), dim3(256), 0, s, lattice, n, n_epochs, ok);
  return hipGetLastError();
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------
// V = [A | f] packed row-major (np x YCOLS): column c < m1 is trend column c,
// column m1 is the flux.
__device__ __forceinline__ void pack_v_at(const double* __restrict__ A, int m1, const double* __restrict__ f,
                                          int64_t n, double* __restrict__ V, int64_t r) {
  if (r >= n) return;
#pragma unroll
  for (int c = 0; c < YCOLS; ++c) V[r * YCOLS + c] = c < m1 ? A[c * n + r] : (c == m1 ? f[r] : 0.0);
}

__global__ __launch_bounds__(256) void pack_v_kernel(const double* __restrict__ A, int m1,
                                                     const double* __restrict__ f, int64_t n,
                                                     double* __restrict__ V) {
  pack_v_at(A, m1, f, n, V, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

hipError_t launch_pack_v(hipStream_t s, const double* A, int m1, const double* f, int64_t n, double* V) {
  hipLaunchKernelGGL(pack_v_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, m1, f, n, V);
  return hipGetLastError();
}

// out[r] = base[r] + alpha * sum_{m <= r} M[r][m] V[m]   (nv columns, row-major,
// lower-triangular M; entries above the diagonal are never read), in two
// launches: partial sums over column chunks of cw columns, then the
// fixed-order sum of the chunks (cols_reduce_kernel, shared with the
// transposed product). A wave owns RPW consecutive rows and one column chunk
// and streams its 64-column pieces of V once for all RPW rows (each lane: one
// column of the piece, its nv values of V, and one element of every row);
// fixed-order wave reductions at the end. The chunks keep each wave's chain of
// dependent loads short and give the long rows at the bottom of the triangle
// as many waves as they need. Chunks right of a wave's rows write zeros, so
// every partial is defined. out may alias base.
constexpr int RPW = 8;

template <int NV>
__device__ __forceinline__ void rows_partial_block(const double* __restrict__ M, int64_t ldm, int64_t n, int64_t np,
                                                   const double* __restrict__ V, int cw, double* __restrict__ partial,
                                                   int bx, int chunk) {
  const int64_t r0 = ((int64_t)bx * 4 + (threadIdx.x >> 6)) * RPW;
  const int lane = threadIdx.x & 63;
  if (r0 >= n) return;
  const int rows = (int)min((int64_t)RPW, n - r0);
  const int64_t rlast = r0 + rows - 1;
  double acc[RPW][NV];
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int c = 0; c < NV; ++c) acc[i][c] = 0.0;
  const int64_t mb = (int64_t)chunk * cw, me = min(rlast + 1, mb + cw);
  for (int64_t m0 = mb; m0 < me; m0 += 64) {
    const int64_t m = m0 + lane;
    double v[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] = m <= rlast ? V[m * YCOLS + c] : 0.0;
    double x[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) x[i] = (i < rows && m <= r0 + i) ? M[(r0 + i) * ldm + m] : 0.0;
#pragma unroll
    for (int i = 0; i < RPW; ++i)
#pragma unroll
      for (int c = 0; c < NV; ++c) acc[i][c] = fma(x[i], v[c], acc[i][c]);
  }
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int c = 0; c < NV; ++c) acc[i][c] = wave_sum(acc[i][c]);
  // lane i * 8 + c writes row r0 + i, column c of this chunk's partial
  const int wi = lane >> 3, wc = lane & 7;
  double mine = 0.0;
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int c = 0; c < NV; ++c)
      if (i == wi && c == wc) mine = acc[i][c];
  if (wi < rows) partial[((int64_t)chunk * np + r0 + wi) * YCOLS + wc] = wc < NV ? mine : 0.0;
}

template <int NV>
__global__ __launch_bounds__(256) void rows_partial_kernel(const double* __restrict__ M, int64_t ldm, int64_t n,
                                                           int64_t np, const double* __restrict__ V, int cw,
                                                           double* __restrict__ partial) {
  rows_partial_block<NV>(M, ldm, n, np, V, cw, partial, (int)blockIdx.x, (int)blockIdx.y);
}

// ---------------------------------------------------------------------------
// Block-wide sum of one double per thread; fixed order (wave butterflies, then
// the four wave totals in order). All threads get the result.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

// status: the factor's status word (a failed factorisation: >= 0), or null
__device__ __forceinline__ void null_solve_block(double* __restrict__ Y, int64_t n, int m1,
                                                 const double* __restrict__ logdet, const int* __restrict__ lattice_ok,
                                                 const int64_t* __restrict__ status, NullFit* __restrict__ nf,
                                                 double* __restrict__ null_out) {
  __shared__ double red[4];
  __shared__ double S[MAX_M1 + 1][MAX_M1 + 1];
  __shared__ double w0s[MAX_M1];
  __shared__ int ok_s;
  const int tid = threadIdx.x;
  const int nv = m1 + 1;
  for (int a = 0; a < nv; ++a)
    for (int b = a; b < nv; ++b) {
      double acc = 0.0;
      for (int64_t r = tid; r < n; r += 256) acc = fma(Y[r * YCOLS + a], Y[r * YCOLS + b], acc);
      acc = block_sum(acc, red);
      if (tid == 0) S[a][b] = S[b][a] = acc;
    }
  __syncthreads();
  if (tid == 0) {
    // Cholesky of G0 = A~^T A~ and w0 = G0^-1 A~^T f~
    double Lg[MAX_M1][MAX_M1];
    int ok = 1;
    for (int i = 0; i < m1; ++i)
      for (int j = 0; j <= i; ++j) {
        double v = S[i][j];
        for (int k = 0; k < j; ++k) v -= Lg[i][k] * Lg[j][k];
        if (i == j) {
          if (!(v > 0.0)) ok = 0;
          Lg[i][i] = sqrt(v);
        } else {
          Lg[i][j] = v / Lg[j][j];
        }
      }
    double y[MAX_M1];
    for (int i = 0; i < m1; ++i) {
      double v = S[i][m1];
      for (int k = 0; k < i; ++k) v -= Lg[i][k] * y[k];
      y[i] = v / Lg[i][i];
    }
    for (int i = m1 - 1; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < m1; ++k) v -= Lg[k][i] * w0s[k];
      w0s[i] = v / Lg[i][i];
    }
    for (int i = 0; i < MAX_M1; ++i)
      for (int j = 0; j < MAX_M1; ++j) nf->G0chol[i * MAX_M1 + j] = (i < m1 && j <= i) ? Lg[i][j] : 0.0;
    for (int i = 0; i < m1; ++i) nf->w0[i] = w0s[i];
    // a failed factorisation leaves ln|K| non-finite: no cell is valid then;
    // nor with a lattice the searches cannot use
    if (!isfinite(*logdet)) ok = 0;
    if (lattice_ok && !*lattice_ok) ok = 0;
    if (status && *status >= 0) ok = 0;
    nf->ok = ok;
    ok_s = ok;
  }
  __syncthreads();
  // r~0 = f~ - A~ w0 (overwrites the f~ column), chi2_0 = ||r~0||^2
  double acc = 0.0;
  for (int64_t r = tid; r < n; r += 256) {
    double v = Y[r * YCOLS + m1];
    for (int a = 0; a < m1; ++a) v -= Y[r * YCOLS + a] * w0s[a];
    Y[r * YCOLS + m1] = v;
    acc = fma(v, v, acc);
  }
  acc = block_sum(acc, red);
  if (tid == 0) {
    const double ld = *logdet;
    const double lnl0 = -0.5 * acc - 0.5 * ld - 0.5 * (double)n * log(2.0 * M_PI);
    nf->chi2_0 = acc;
    nf->lnl0 = lnl0;
    nf->logdet = ld;
    if (null_out) {
      null_out[0] = ok_s ? lnl0 : NAN;
      null_out[1] = acc;
      null_out[2] = ld;
    }
  }
}

__global__ __launch_bounds__(256) void null_solve_kernel(double* __restrict__ Y, int64_t n, int m1,
                                                         const double* __restrict__ logdet,
                                                         const int* __restrict__ lattice_ok, NullFit* __restrict__ nf,
                                                         double* __restrict__ null_out) {
  null_solve_block(Y, n, m1, logdet, lattice_ok, nullptr, nf, null_out);
}

hipError_t launch_null_solve(hipStream_t s, double* Y, int64_t n, int m1, const double* logdet,
                             const int* lattice_ok, NullFit* nf, double* null_out) {
  hipLaunchKernelGGL(null_solve_kernel, dim3(1), dim3(256), 0, s, Y, n, m1, logdet, lattice_ok, nf, null_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// out[m] = base[m] + alpha * sum_{n >= m} M[n][m] W[n]   (nv columns,
// row-major, lower-triangular M). Workgroup = 256 columns x a chunk of rows;
// partials per chunk, then a fixed-order reduction. out may alias base.
// The operands are read through global-address-space views: a batch passes
// pointers read from its job records, generic to the compiler, and the row of
// W shared by a wave then came in by per-lane flat loads instead of scalar
// loads.
__device__ __forceinline__ void cols_partial_block(const double* __restrict__ M_, int64_t ldm, int64_t n, int64_t np,
                                                   const double* __restrict__ W_, int nv, int rowchunk,
                                                   double* __restrict__ partial, int bx, int chunk) {
  const NU_GLOBAL double* __restrict__ M = (const NU_GLOBAL double*)M_;
  const NU_GLOBAL double* __restrict__ W = (const NU_GLOBAL double*)W_;
  const int64_t m = (int64_t)bx * 256 + threadIdx.x;
  if (m >= np) return;
  const int64_t r0 = (int64_t)chunk * rowchunk;
  const int64_t r1 = min(n, r0 + rowchunk);
  double acc[YCOLS];
#pragma unroll
  for (int c = 0; c < YCOLS; ++c) acc[c] = 0.0;
  const int64_t c0 = (int64_t)bx * 256;
  if (m < n) {
    // eight rows per step: eight independent loads in flight per thread
    int64_t r = max(r0, c0);
    for (; r + 8 <= r1; r += 8) {
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = (m <= r + u) ? M[(r + u) * ldm + m] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const NU_GLOBAL double* wr = W + (r + u) * YCOLS;
#pragma unroll
        for (int c = 0; c < YCOLS; ++c)
          if (c < nv) acc[c] = fma(x[u], wr[c], acc[c]);
      }
    }
    for (; r < r1; ++r) {
      const double x = (m <= r) ? M[r * ldm + m] : 0.0;
      const NU_GLOBAL double* wr = W + r * YCOLS;
#pragma unroll
      for (int c = 0; c < YCOLS; ++c)
        if (c < nv) acc[c] = fma(x, wr[c], acc[c]);
    }
  }
  NU_GLOBAL double* o = (NU_GLOBAL double*)partial + ((int64_t)chunk * np + m) * YCOLS;
#pragma unroll
  for (int c = 0; c < YCOLS; ++c) o[c] = acc[c];
}

__global__ __launch_bounds__(256) void cols_partial_kernel(const double* __restrict__ M, int64_t ldm, int64_t n,
                                                           int64_t np, const double* __restrict__ W, int nv,
                                                           int rowchunk, double* __restrict__ partial) {
  cols_partial_block(M, ldm, n, np, W, nv, rowchunk, partial, (int)blockIdx.x, (int)blockIdx.y);
}

// out[e] = base[e] + alpha * sum_c partial[c][e] for e < tot (elements of the
// np x YCOLS layout), the chunks in order
__device__ __forceinline__ void cols_reduce_at(const double* __restrict__ partial, int64_t np, int nchunks,
                                               const double* base, double alpha, double* out, int64_t tot,
                                               int64_t e) {
  if (e >= tot) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += partial[(int64_t)c * np * YCOLS + e];
  out[e] = (base ? base[e] : 0.0) + alpha * s;
}

__global__ __launch_bounds__(256) void cols_reduce_kernel(const double* __restrict__ partial, int64_t np,
                                                          int nchunks, const double* base, double alpha,
                                                          double* out, int64_t tot) {
  cols_reduce_at(partial, np, nchunks, base, alpha, out, tot, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

hipError_t launch_rows_matvec(hipStream_t s, const double* M, int64_t ldm, int64_t n, int64_t np, const double* V,
                              int nv, double* partial, int cw, int nchunks, const double* base, double alpha,
                              double* out) {
  if (cw <= 0 || cw % 64 != 0 || (int64_t)nchunks * cw < n) return hipErrorInvalidValue;
  const int64_t waves = (n + RPW - 1) / RPW;
  const dim3 g((unsigned)((waves + 3) / 4), (unsigned)nchunks), b(256);
  switch (nv) {
    case 1: hipLaunchKernelGGL(rows_partial_kernel<1>, g, b, 0, s, M, ldm, n, np, V, cw, partial); break;
    case 2: hipLaunchKernelGGL(rows_partial_kernel<2>, g, b, 0, s, M, ldm, n, np, V, cw, partial); break;
    case 3: hipLaunchKernelGGL(rows_partial_kernel<3>, g, b, 0, s, M, ldm, n, np, V, cw, partial); break;
    case 4: hipLaunchKernelGGL(rows_partial_kernel<4>, g, b, 0, s, M, ldm, n, np, V, cw, partial); break;
    case 5: hipLaunchKernelGGL(rows_partial_kernel<5>, g, b, 0, s, M, ldm, n, np, V, cw, partial); break;
    case 6: hipLaunchKernelGGL(rows_partial_kernel<6>, g, b, 0, s, M, ldm, n, np, V, cw, partial); break;
    case 7: hipLaunchKernelGGL(rows_partial_kernel<7>, g, b, 0, s, M, ldm, n, np, V, cw, partial); break;
    case 8: hipLaunchKernelGGL(rows_partial_kernel<8>, g, b, 0, s, M, ldm, n, np, V, cw, partial); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // rows n .. np - 1 of the partials are never written; the sum covers rows < n only
  const int64_t tot = n * YCOLS;
  hipLaunchKernelGGL(cols_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, partial, np, nchunks,
                     base, alpha, out, tot);
  return hipGetLastError();
}

hipError_t launch_cols_matvec(hipStream_t s, const double* M, int64_t ldm, int64_t n, int64_t np, const double* W,
                              int nv, double* partial, int rowchunk, int nchunks, const double* base, double alpha,
                              double* out) {
  hipLaunchKernelGGL(cols_partial_kernel, dim3((unsigned)(np / 256 + (np % 256 ? 1 : 0)), (unsigned)nchunks),
                     dim3(256), 0, s, M, ldm, n, np, W, nv, rowchunk, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t tot = np * YCOLS;
  hipLaunchKernelGGL(cols_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, partial, np, nchunks,
                     base, alpha, out, tot);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// q partial sums. A wave owns 64 consecutive epoch slots (one per lane) and
// one chunk of rows; the four waves of a workgroup take adjacent slot groups
// over the same rows, so their overlapping row segments meet in cache. The
// union of the boxes of a wave's slots spans the sample segment
// [seg_lo, seg_hi), at most 64 + dmax samples; a row of X restricted to it
// (entries above the diagonal read as 0) is turned into inclusive prefix sums
// in registers, each lane holding RUN consecutive entries: a serial prefix
// within the lane, one wave scan of the lane totals, then the lane's offset.
// The prefix row goes to the wave's own LDS row, from which each lane takes
// the two ends of each of its boxes: box sum = P[hi] - P[lo]. Rows go two at
// a time (two independent scan chains), the next two rows' segments loading
// meanwhile. No workgroup barrier:
// the waves are independent, and LDS order within a wave needs only a
// compiler fence.
constexpr int QCH = 256;  // slots per workgroup (4 waves x 64)

template <int RUN>
__device__ __forceinline__ void q_partial_block(const double* __restrict__ X, int64_t ldx, int64_t n,
                                                const int64_t* __restrict__ lattice, const int32_t* __restrict__ T,
                                                int64_t n_epochs, const DurList& dl, int rowchunk,
                                                double* __restrict__ qpart, int bx, int chunk) {
  constexpr int SEG = 64 * RUN;  // segment capacity of a wave
  __shared__ double prefix[4][2][SEG + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t slot = (int64_t)bx * QCH + wave * 64 + lane;
  const bool active = slot < n_epochs;
  int64_t lo[MAX_ND], hi[MAX_ND];
  int64_t my_lo = INT64_MAX, my_hi = INT64_MIN;
#pragma unroll
  for (int k = 0; k < MAX_ND; ++k) {
    lo[k] = hi[k] = 0;
    if (k < dl.n && active) {
      const int64_t a = slot - dl.d[k] / 2;
      lo[k] = count_below(lattice, n, T, n_epochs, a);
      hi[k] = count_below(lattice, n, T, n_epochs, a + dl.d[k]);
      my_lo = min(my_lo, lo[k]);
      my_hi = max(my_hi, hi[k]);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    my_lo = min(my_lo, (int64_t)__shfl_xor(my_lo, off, 64));
    my_hi = max(my_hi, (int64_t)__shfl_xor(my_hi, off, 64));
  }
  const int64_t seg_lo = my_lo, seg_hi = my_hi;  // empty wave: seg_lo > seg_hi
  double* P0 = prefix[wave][0];
  double* P1 = prefix[wave][1];
  double q[MAX_ND];
  int rl[MAX_ND], rh[MAX_ND];
#pragma unroll
  for (int k = 0; k < MAX_ND; ++k) {
    q[k] = 0.0;
    rl[k] = (int)(lo[k] - seg_lo);
    rh[k] = (int)(hi[k] - seg_lo);
  }
  const int64_t r0 = max((int64_t)chunk * rowchunk, seg_lo);
  const int64_t r1 = min(n, (int64_t)chunk * rowchunk + rowchunk);
  if (seg_hi > seg_lo && seg_hi - seg_lo <= SEG && r0 < r1) {
    if (lane == 0) P0[0] = P1[0] = 0.0;
    const int64_t m0 = seg_lo + lane * RUN;  // this lane's first column
    // row r restricted to the segment; rows at or past r1 read as 0
    // global loads (a batch's X is a generic pointer read from its job record,
    // and flat loads would also hold up the waits for the LDS prefix)
    auto load_row = [&](int64_t r, double (&v)[RUN]) {
      const NU_GLOBAL double* x = (const NU_GLOBAL double*)X + r * ldx;
#pragma unroll
      for (int e = 0; e < RUN; ++e) {
        const int64_t m = m0 + e;
        v[e] = (r < r1 && m < seg_hi && m <= r) ? x[m] : 0.0;
      }
    };
    // inclusive prefix of the segment into P[1..]
    auto scan_store = [&](double (&v)[RUN], double* P) {
#pragma unroll
      for (int e = 1; e < RUN; ++e) v[e] += v[e - 1];
      double incl = v[RUN - 1];
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const double y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
      }
      const double excl = incl - v[RUN - 1];
#pragma unroll
      for (int e = 0; e < RUN; ++e) P[1 + lane * RUN + e] = v[e] + excl;
    };
    // two rows per pass, the next two rows' loads in flight meanwhile
    double n0[RUN], n1[RUN];
    load_row(r0, n0);
    load_row(r0 + 1, n1);
    for (int64_t r = r0; r < r1; r += 2) {
      double v0[RUN], v1[RUN];
#pragma unroll
      for (int e = 0; e < RUN; ++e) {
        v0[e] = n0[e];
        v1[e] = n1[e];
      }
      if (r + 2 < r1) {
        load_row(r + 2, n0);
        load_row(r + 3, n1);
      }
      scan_store(v0, P0);
      scan_store(v1, P1);
      wave_lds_fence();
      if (active) {
#pragma unroll
        for (int k = 0; k < MAX_ND; ++k)
          if (k < dl.n) {
            const double s0 = P0[rh[k]] - P0[rl[k]];
            const double s1 = P1[rh[k]] - P1[rl[k]];
            q[k] = fma(s0, s0, q[k]);
            q[k] = fma(s1, s1, q[k]);
          }
      }
      wave_lds_fence();
    }
  }
  if (active) {
#pragma unroll
    for (int k = 0; k < MAX_ND; ++k)
      if (k < dl.n) qpart[((int64_t)chunk * dl.n + dl.perm[k]) * n_epochs + slot] = q[k];
  }
}

template <int RUN>
__global__ __launch_bounds__(256) void q_partial_kernel(const double* __restrict__ X, int64_t ldx, int64_t n,
                                                        const int64_t* __restrict__ lattice,
                                                        const int32_t* __restrict__ T, int64_t n_epochs,
                                                        DurList dl, int rowchunk, double* __restrict__ qpart) {
  q_partial_block<RUN>(X, ldx, n, lattice, T, n_epochs, dl, rowchunk, qpart, (int)blockIdx.x, (int)blockIdx.y);
}

hipError_t launch_q_partial(hipStream_t s, const double* X, int64_t ldx, int64_t n, const int64_t* lattice,
                            const int32_t* T, int64_t n_epochs, const int32_t* dur_sorted, int n_d, int dmax,
                            int rowchunk, int nchunks, double* qpart) {
  // dur_sorted: host array [2 * n_d]: ascending durations, then their caller indices
  DurList dl{};
  dl.n = n_d;
  for (int k = 0; k < n_d; ++k) {
    dl.d[k] = dur_sorted[k];
    dl.perm[k] = dur_sorted[n_d + k];
  }
  // a wave's segment: at most 64 slots plus the longest box, in samples
  const int seg = 64 + dmax;
  const dim3 g((unsigned)((n_epochs + QCH - 1) / QCH), (unsigned)nchunks), b(256);
  if (seg <= 64 * 2) hipLaunchKernelGGL(q_partial_kernel<2>, g, b, 0, s, X, ldx, n, lattice, T, n_epochs, dl, rowchunk, qpart);
  else if (seg <= 64 * 3) hipLaunchKernelGGL(q_partial_kernel<3>, g, b, 0, s, X, ldx, n, lattice, T, n_epochs, dl, rowchunk, qpart);
  else if (seg <= 64 * 5) hipLaunchKernelGGL(q_partial_kernel<5>, g, b, 0, s, X, ldx, n, lattice, T, n_epochs, dl, rowchunk, qpart);
  else if (seg <= 64 * 9) hipLaunchKernelGGL(q_partial_kernel<9>, g, b, 0, s, X, ldx, n, lattice, T, n_epochs, dl, rowchunk, qpart);
  else if (seg <= 64 * 17) hipLaunchKernelGGL(q_partial_kernel<17>, g, b, 0, s, X, ldx, n, lattice, T, n_epochs, dl, rowchunk, qpart);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per cell: q from the partial sums, g = A^T K^-1 b and h = b^T K^-1 r0 as
// (weighted) window sums of Z, the Schur complement of the trend block, and
// the outputs. With TPL the box is the duration's shape: sample r of the
// window weighs shapes[off_j + lattice[r] - a].
template <bool TPL>
__device__ __forceinline__ void cell_epilogue_at(const double* __restrict__ qpart, int nchunks,
                                                 const int64_t* __restrict__ lattice, const int32_t* __restrict__ T,
                                                 int64_t n, int64_t n_epochs, const DurList& dl,
                                                 const double* __restrict__ Z, int m1, const NullFit* __restrict__ nf,
                                                 const double* __restrict__ shapes, double* __restrict__ depth,
                                                 double* __restrict__ var, double* __restrict__ dll,
                                                 uint8_t* __restrict__ valid, int64_t cell) {
  if (cell >= (int64_t)dl.n * n_epochs) return;
  const int j = (int)(cell / n_epochs);
  const int64_t i = cell - (int64_t)j * n_epochs;
  double q = 0.0;
  for (int c = 0; c < nchunks; ++c) q += qpart[((int64_t)c * dl.n + j) * n_epochs + i];
  const int d = dl.d[j];
  const int64_t a = i - d / 2;
  const int64_t lo = count_below(lattice, n, T, n_epochs, a);
  const int64_t hi = count_below(lattice, n, T, n_epochs, a + d);
  bool ok = (hi > lo) && nf->ok;
  double h = 0.0, g[MAX_M1];
#pragma unroll
  for (int c = 0; c < MAX_M1; ++c) g[c] = 0.0;
  if (ok) {
    for (int64_t r = lo; r < hi; ++r) {
      const double* zr = Z + r * YCOLS;
      double wgt = 1.0;
      if (TPL) {  // the sample's window offset; in [0, d) for a lattice the searches accept
        const int64_t o = lattice[r] - a;
        wgt = (o >= 0 && o < d) ? shapes[dl.off[j] + (int)o] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < MAX_M1; ++c)
        if (c < m1) g[c] = fma(-wgt, zr[c], g[c]);
      h = fma(-wgt, zr[m1], h);
    }
  }
  // S = q - g^T G0^-1 g via y = chol(G0)^-1 g
  double gg = 0.0, y[MAX_M1];
#pragma unroll
  for (int r = 0; r < MAX_M1; ++r) {
    if (r < m1) {
      double v = g[r];
#pragma unroll
      for (int k = 0; k < MAX_M1; ++k)
        if (k < r) v -= nf->G0chol[r * MAX_M1 + k] * y[k];
      y[r] = v / nf->G0chol[r * MAX_M1 + r];
      gg = fma(y[r], y[r], gg);
    } else {
      y[r] = 0.0;
    }
  }
  // a box in the span of the trend columns leaves S at rounding level: singular
  const double S = q - gg;
  ok = ok && (S > 1e-12 * q) && isfinite(S) && isfinite(h);
  const int64_t o = (int64_t)j * n_epochs + i;
  if (ok) {
    const double dep = h / S;
    depth[o] = dep;
    var[o] = 1.0 / S;
    dll[o] = 0.5 * h * dep;
    valid[o] = 1;
  } else {
    depth[o] = 0.0;
    var[o] = INFINITY;
    dll[o] = 0.0;
    valid[o] = 0;
  }
}

template <bool TPL>
__global__ __launch_bounds__(256) void cell_epilogue_kernel(const double* __restrict__ qpart, int nchunks,
                                                            const int64_t* __restrict__ lattice,
                                                            const int32_t* __restrict__ T, int64_t n,
                                                            int64_t n_epochs, DurList dl,
                                                            const double* __restrict__ Z, int m1,
                                                            const NullFit* __restrict__ nf,
                                                            const double* __restrict__ shapes,
                                                            double* __restrict__ depth, double* __restrict__ var,
                                                            double* __restrict__ dll, uint8_t* __restrict__ valid) {
  cell_epilogue_at<TPL>(qpart, nchunks, lattice, T, n, n_epochs, dl, Z, m1, nf, shapes, depth, var, dll, valid,
                        (int64_t)blockIdx.x * 256 + threadIdx.x);
}

hipError_t launch_cell_epilogue(hipStream_t s, const double* qpart, int nchunks, const int64_t* lattice,
                                const int32_t* T, int64_t n, int64_t n_epochs, const int32_t* dur, int n_d,
                                const double* Z, int m1, const NullFit* nf, double* depth, double* var, double* dll,
                                uint8_t* valid, const double* shapes) {
  DurList dl{};
  dl.n = n_d;
  int off = 0;
  for (int k = 0; k < n_d; ++k) {
    dl.d[k] = dur[k];
    dl.perm[k] = k;
    dl.off[k] = off;
    off += dur[k];
  }
  const int64_t cells = (int64_t)n_d * n_epochs;
  const dim3 g((unsigned)((cells + 255) / 256)), b(256);
  if (shapes)
    hipLaunchKernelGGL(cell_epilogue_kernel<true>, g, b, 0, s, qpart, nchunks, lattice, T, n, n_epochs, dl, Z, m1,
                       nf, shapes, depth, var, dll, valid);
  else
    hipLaunchKernelGGL(cell_epilogue_kernel<false>, g, b, 0, s, qpart, nchunks, lattice, T, n, n_epochs, dl, Z, m1,
                       nf, shapes, depth, var, dll, valid);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// q of template cells: q = sum_r (sum_m X[r][m] b_m)^2 with b the shape of the
// cell on its window. As in q_partial, a wave owns 64 consecutive epoch slots
// and one chunk of rows; here a row is laid out by lattice slot in the wave's
// LDS rows (zeros on slots without a sample), so every window is a contiguous
// run of it, and the shape value at a window offset is the same for every
// lane (a broadcast read of the shapes, staged once per workgroup in LDS).
// RR rows go per pass, so each shape value read serves RR rows; the window
// loop runs four offsets at a time so neighbouring row reads pair up. The span
// of slots a wave's windows cover is 64 + dmax; RUN slots per lane.
template <int RUN, int RR>
__global__ __launch_bounds__(256) void q_template_kernel(const double* __restrict__ X, int64_t ldx, int64_t n,
                                                         const int64_t* __restrict__ lattice,
                                                         const int32_t* __restrict__ T, int64_t n_epochs, DurList dl,
                                                         const double* __restrict__ shapes, int shape_total,
                                                         int half_max, int dmax, int rowchunk,
                                                         double* __restrict__ qpart) {
  constexpr int SPAN = 64 * RUN;
  __shared__ double sh[MAX_SHAPE];
  __shared__ double rows[4][RR][SPAN];
  for (int t = threadIdx.x; t < shape_total; t += 256) sh[t] = shapes[t];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t s0 = (int64_t)blockIdx.x * QCH + wave * 64;  // first slot of the wave
  const int64_t slot = s0 + lane;
  const int chunk = blockIdx.y;
  const bool active = slot < n_epochs;
  const int64_t base = s0 - half_max;  // slot of row position 0
  // the sample (if any) on each of the lane's RUN slots
  int64_t msamp[RUN];
  int64_t my_lo = INT64_MAX, my_hi = INT64_MIN;
#pragma unroll
  for (int e = 0; e < RUN; ++e) {
    const int64_t sl = base + lane * RUN + e;
    const int64_t m = count_below(lattice, n, T, n_epochs, sl);
    const bool present = m < n && lattice[m] == sl;
    msamp[e] = present ? m : -1;
    if (present) {
      my_lo = min(my_lo, m);
      my_hi = max(my_hi, m + 1);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    my_lo = min(my_lo, (int64_t)__shfl_xor(my_lo, off, 64));
    my_hi = max(my_hi, (int64_t)__shfl_xor(my_hi, off, 64));
  }
  // duration k's window covers offsets [wlo[k], wlo[k] + d_k) from the lane's base position
  int wlo[MAX_ND];
#pragma unroll
  for (int k = 0; k < MAX_ND; ++k) wlo[k] = k < dl.n ? half_max - dl.d[k] / 2 : 0;
  double q[MAX_ND];
#pragma unroll
  for (int k = 0; k < MAX_ND; ++k) q[k] = 0.0;
  const int64_t r0 = max((int64_t)chunk * rowchunk, my_lo);
  const int64_t r1 = min(n, (int64_t)chunk * rowchunk + rowchunk);
  if (my_hi > my_lo) {
    for (int64_t r = r0; r < r1; r += RR) {
#pragma unroll
      for (int rr = 0; rr < RR; ++rr) {
        const int64_t row = r + rr;
        const double* x = X + row * ldx;
#pragma unroll
        for (int e = 0; e < RUN; ++e) {
          const int64_t m = msamp[e];
          rows[wave][rr][lane * RUN + e] = (row < r1 && m >= 0 && m <= row) ? x[m] : 0.0;
        }
      }
      wave_lds_fence();
      if (active) {
#pragma unroll
        for (int k = 0; k < MAX_ND; ++k) {
          if (k < dl.n) {
            const double* shp = sh + dl.off[k];
            const int d = dl.d[k];
            const int p0 = lane + wlo[k];
            double acc[RR];
#pragma unroll
            for (int rr = 0; rr < RR; ++rr) acc[rr] = 0.0;
            int i = 0;
            for (; i + 4 <= d; i += 4) {
              double w[4];
#pragma unroll
              for (int t = 0; t < 4; ++t) w[t] = shp[i + t];
#pragma unroll
              for (int rr = 0; rr < RR; ++rr)
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[rr] = fma(w[t], rows[wave][rr][p0 + i + t], acc[rr]);
            }
            for (; i < d; ++i) {
              const double w = shp[i];
#pragma unroll
              for (int rr = 0; rr < RR; ++rr) acc[rr] = fma(w, rows[wave][rr][p0 + i], acc[rr]);
            }
#pragma unroll
            for (int rr = 0; rr < RR; ++rr) q[k] = fma(acc[rr], acc[rr], q[k]);
          }
        }
      }
      wave_lds_fence();
    }
  }
  if (active) {
    for (int k = 0; k < dl.n; ++k) qpart[((int64_t)chunk * dl.n + dl.perm[k]) * n_epochs + slot] = q[k];
  }
}

// The same sums on the matrix cores, for windows up to 256 slots. One wave
// per workgroup owns 64 slots (four 16-slot tiles) and takes 16 rows per pass:
// for duration k, C[r][l] = sum_m A[r][m] B[m][l] with A the rows laid out by
// slot (m counted from the tile's first window position) and B the banded
// Toeplitz matrix B[m][l] = s_k[m - l] (0 outside the shape), so each
// v_mfma_f64_16x16x4f64 step takes 4 offsets m for 16 rows x 16 slots. The B
// fragment depends on m - l only, so one read of the shape serves all four
// tiles; the squares of C summed over the rows give q.
typedef double qdbl4 __attribute__((ext_vector_type(4)));
constexpr int QT_ROWS = 16;
constexpr int QT_SH0 = 16;  // zeros before a staged shape: m - lr >= -15
constexpr int QT_SH1 = 24;  // zeros after it: m - lr < d + 18
constexpr int QT_PAD = 9;  // zeros after a row (the last MFMA step may reach past the span); odd, so the 16 rows of a read fall in distinct banks

template <int RUN>
__global__ __launch_bounds__(64) void q_template_mfma_kernel(const double* __restrict__ X, int64_t ldx, int64_t n,
                                                             const int64_t* __restrict__ lattice,
                                                             const int32_t* __restrict__ T, int64_t n_epochs,
                                                             DurList dl, const double* __restrict__ shapes,
                                                             int shape_total, int half_max, int rowchunk,
                                                             double* __restrict__ qpart) {
  constexpr int SPAN = 64 * RUN;
  constexpr int LDR = SPAN + QT_PAD;
  // shapes with QT_SH0 zeros before and QT_SH1 after each, so that the B
  // fragment is one unconditional read (no branch splits the MFMA loop)
  __shared__ double sh[MAX_SHAPE + (QT_SH0 + QT_SH1) * MAX_ND];
  __shared__ double rows[QT_ROWS][LDR];
  const int lane = threadIdx.x;
  const int padded = shape_total + (QT_SH0 + QT_SH1) * dl.n;
  for (int t = lane; t < padded; t += 64) sh[t] = 0.0;
  for (int t = lane; t < QT_ROWS * QT_PAD; t += 64) rows[t / QT_PAD][SPAN + t % QT_PAD] = 0.0;
  __syncthreads();
  for (int k = 0; k < dl.n; ++k) {
    const int po = dl.off[k] + (QT_SH0 + QT_SH1) * dl.perm[k] + QT_SH0;
    for (int t = lane; t < dl.d[k]; t += 64) sh[po + t] = shapes[dl.off[k] + t];
  }
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t s0 = (int64_t)blockIdx.x * 64;  // first slot of the wave
  const int64_t slot = s0 + lane;
  const int chunk = blockIdx.y;
  const bool active = slot < n_epochs;
  const int64_t base = s0 - half_max;  // slot of row position 0
  int64_t msamp[RUN];
  int64_t my_lo = INT64_MAX, my_hi = INT64_MIN;
#pragma unroll
  for (int e = 0; e < RUN; ++e) {
    const int64_t sl = base + lane * RUN + e;
    const int64_t m = count_below(lattice, n, T, n_epochs, sl);
    const bool present = m < n && lattice[m] == sl;
    msamp[e] = present ? m : -1;
    if (present) {
      my_lo = min(my_lo, m);
      my_hi = max(my_hi, m + 1);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    my_lo = min(my_lo, (int64_t)__shfl_xor(my_lo, off, 64));
    my_hi = max(my_hi, (int64_t)__shfl_xor(my_hi, off, 64));
  }
  double q[MAX_ND];
#pragma unroll
  for (int k = 0; k < MAX_ND; ++k) q[k] = 0.0;
  const int64_t r0 = max((int64_t)chunk * rowchunk, my_lo);
  const int64_t r1 = min(n, (int64_t)chunk * rowchunk + rowchunk);
  __syncthreads();
  if (my_hi > my_lo) {
    for (int64_t r = r0; r < r1; r += QT_ROWS) {
#pragma unroll
      for (int rr = 0; rr < QT_ROWS; ++rr) {
        const int64_t row = r + rr;
        const double* x = X + row * ldx;
#pragma unroll
        for (int e = 0; e < RUN; ++e) {
          const int64_t m = msamp[e];
          rows[rr][lane * RUN + e] = (row < r1 && m >= 0 && m <= row) ? x[m] : 0.0;
        }
      }
      wave_lds_fence();
#pragma unroll
      for (int k = 0; k < MAX_ND; ++k) {
        if (k < dl.n) {
          const int d = dl.d[k];
          // B fragment of step st: shape value at m - lr = 4 st + lk - lr, zero outside [0, d)
          const double* shb = sh + dl.off[k] + (QT_SH0 + QT_SH1) * dl.perm[k] + QT_SH0 + lk - lr;
          const int w0 = half_max - d / 2;  // window start of tile slot 0, in row positions
          const double* ar = &rows[lr][w0 + lk];
          const int steps = (QT_ROWS - 1 + d + 3) / 4;
          qdbl4 acc[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) acc[t] = qdbl4{0.0, 0.0, 0.0, 0.0};
          // operands of step st + 1 are read while step st's products run (the
          // padding keeps the read past the last step inside the arrays)
          double bv = shb[0], av[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) av[t] = ar[16 * t];
          for (int st = 0; st < steps; ++st) {
            const double bn = shb[4 * st + 4];
            double an[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) an[t] = ar[16 * t + 4 * st + 4];
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv, acc[t], 0, 0, 0);
            bv = bn;
#pragma unroll
            for (int t = 0; t < 4; ++t) av[t] = an[t];
          }
          // column lr of tile t: rows lk + 4v; sum the squares over the 16 rows
          double mine = 0.0;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            double s2 = 0.0;
#pragma unroll
            for (int v = 0; v < 4; ++v) s2 = fma(acc[t][v], acc[t][v], s2);
            s2 += __shfl_xor(s2, 16, 64);
            s2 += __shfl_xor(s2, 32, 64);
            if (t == lk) mine = s2;  // lane 16 t + lr is slot 16 t + lr
          }
          q[k] += mine;
        }
      }
      wave_lds_fence();
    }
  }
  if (active) {
    for (int k = 0; k < dl.n; ++k) qpart[((int64_t)chunk * dl.n + dl.perm[k]) * n_epochs + slot] = q[k];
  }
}

hipError_t launch_q_template(hipStream_t s, const double* X, int64_t ldx, int64_t n, const int64_t* lattice,
                             const int32_t* T, int64_t n_epochs, const int32_t* dur_sorted, const int32_t* dur,
                             int n_d, const double* shapes, int dmax, int rowchunk, int nchunks, double* qpart) {
  // dur_sorted: host [2 n_d]: ascending durations, then their caller indices; dur: caller order
  int offs[MAX_ND];
  int total = 0;
  for (int k = 0; k < n_d; ++k) {
    offs[k] = total;
    total += dur[k];
  }
  if (total > MAX_SHAPE) return hipErrorInvalidValue;
  DurList dl{};
  dl.n = n_d;
  for (int k = 0; k < n_d; ++k) {
    dl.d[k] = dur_sorted[k];
    dl.perm[k] = dur_sorted[n_d + k];
    dl.off[k] = offs[dl.perm[k]];
  }
  const int span = 64 + dmax;
  const int half = dmax / 2;
  const dim3 g((unsigned)((n_epochs + QCH - 1) / QCH), (unsigned)nchunks), b(256);
#define NU_QT(RUN, RR)                                                                                            \
  hipLaunchKernelGGL((q_template_kernel<RUN, RR>), g, b, 0, s, X, ldx, n, lattice, T, n_epochs, dl, shapes, total, \
                     half, dmax, rowchunk, qpart)
#define NU_QTM(RUN)                                                                                               \
  hipLaunchKernelGGL((q_template_mfma_kernel<RUN>), dim3((unsigned)((n_epochs + 63) / 64), (unsigned)nchunks),       \
                     dim3(64), 0, s, X, ldx, n, lattice, T, n_epochs, dl, shapes, total, half, rowchunk, qpart)
  if (span <= 64 * 2) NU_QTM(2);
  else if (span <= 64 * 3) NU_QTM(3);
  else if (span <= 64 * 5) NU_QTM(5);
  else if (span <= 64 * 9) NU_QT(9, 2);
  else if (span <= 64 * 17) NU_QT(17, 1);
#undef NU_QT
#undef NU_QTM
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched forms of the linear search (one launch for every curve of a batch;
// workgroups numbered curve after curve, see CurveJob). The bodies are those
// of the single-curve kernels, so each curve's outputs are bitwise the same.

__device__ __forceinline__ double* job_panel(const CurveJob& J, int sel) {
  switch (sel) {
    case PS_V: return J.V;
    case PS_Y: return J.Y;
    case PS_R: return J.R;
    case PS_Z: return J.Z;
    case PS_RZ: return J.Rz;
    default: return nullptr;
  }
}

__global__ __launch_bounds__(256) void batch_lattice_check_kernel(const CurveJob* __restrict__ jobs) {
  const CurveJob& J = jobs[blockIdx.x];
  lattice_check_block(J.lattice, J.n, J.n_epochs, J.lattice_ok);
}

__global__ __launch_bounds__(256) void batch_pack_v_kernel(const CurveJob* __restrict__ jobs,
                                                           const int* __restrict__ begin, int n_curves, int m1) {
  int u;
  const CurveJob& J = jobs[batch_find(begin, n_curves, (int)blockIdx.x, u)];
  pack_v_at(J.A, m1, J.f, J.n, J.V, (int64_t)u * 256 + threadIdx.x);
}

// workgroups of the row products of one curve: row groups x column chunks
__host__ __device__ inline int rows_groups(int64_t n) { return (int)(((n + RPW - 1) / RPW + 3) / 4); }

template <int NV>
__global__ __launch_bounds__(256) void batch_rows_partial_kernel(const CurveJob* __restrict__ jobs,
                                                                 const int* __restrict__ begin, int n_curves,
                                                                 int mat, int vin) {
  int u;
  const CurveJob& J = jobs[batch_find(begin, n_curves, (int)blockIdx.x, u)];
  const int gx = rows_groups(J.n);
  rows_partial_block<NV>(mat == MS_L ? J.L : J.X, J.np, J.n, J.np, job_panel(J, vin), LIN_RCW, J.xpart, u % gx,
                         u / gx);
}

// out = base + alpha * (sum of the chunks), over tot(J) elements; rows: n YCOLS, columns: np YCOLS
template <bool ROWS>
__global__ __launch_bounds__(256) void batch_reduce_kernel(const CurveJob* __restrict__ jobs,
                                                           const int* __restrict__ begin, int n_curves, int base,
                                                           double alpha, int out) {
  int u;
  const CurveJob& J = jobs[batch_find(begin, n_curves, (int)blockIdx.x, u)];
  const int64_t tot = (ROWS ? J.n : J.np) * YCOLS;
  cols_reduce_at(J.xpart, J.np, ROWS ? J.rchunks : J.xchunks, job_panel(J, base), alpha, job_panel(J, out), tot,
                 (int64_t)u * 256 + threadIdx.x);
}

__global__ __launch_bounds__(256) void batch_null_kernel(const CurveJob* __restrict__ jobs, int m1) {
  const CurveJob& J = jobs[blockIdx.x];
  null_solve_block(J.Y, J.n, m1, J.logdet, J.lattice_ok, J.status, J.nf, J.null_out);
}

__global__ __launch_bounds__(256) void batch_cols_partial_kernel(const CurveJob* __restrict__ jobs,
                                                                 const int* __restrict__ begin, int n_curves, int nv,
                                                                 int mat, int win) {
  int u;
  const CurveJob& J = jobs[batch_find(begin, n_curves, (int)blockIdx.x, u)];
  const int gx = (int)((J.np + 255) / 256);
  cols_partial_block(mat == MS_L ? J.L : J.X, J.np, J.n, J.np, job_panel(J, win), nv, LIN_XRC, J.xpart, u % gx,
                     u / gx);
}

__global__ __launch_bounds__(256) void batch_slot_count_kernel(const CurveJob* __restrict__ jobs,
                                                               const int* __restrict__ begin, int n_curves) {
  int u;
  const CurveJob& J = jobs[batch_find(begin, n_curves, (int)blockIdx.x, u)];
  slot_count_at(J.lattice, J.n, J.n_epochs, J.slot_count, (int64_t)u * 256 + threadIdx.x);
}

template <int RUN>
__global__ __launch_bounds__(256) void batch_q_partial_kernel(const CurveJob* __restrict__ jobs,
                                                              const int* __restrict__ begin, int n_curves,
                                                              DurList dl) {
  int u;
  const CurveJob& J = jobs[batch_find(begin, n_curves, (int)blockIdx.x, u)];
  const int gx = (int)((J.n_epochs + QCH - 1) / QCH);
  q_partial_block<RUN>(J.X, J.np, J.n, J.lattice, J.slot_count, J.n_epochs, dl, LIN_QRC, J.qpart, u % gx, u / gx);
}

__global__ __launch_bounds__(256) void batch_epilogue_kernel(const CurveJob* __restrict__ jobs,
                                                             const int* __restrict__ begin, int n_curves, DurList dl,
                                                             int m1) {
  int u;
  const CurveJob& J = jobs[batch_find(begin, n_curves, (int)blockIdx.x, u)];
  cell_epilogue_at<false>(J.qpart, J.qchunks, J.lattice, J.slot_count, J.n, J.n_epochs, dl, J.Z, m1, J.nf, nullptr,
                          J.depth, J.var, J.dll, J.valid, (int64_t)u * 256 + threadIdx.x);
}

hipError_t launch_batch_lattice_check(hipStream_t s, const CurveJob* jobs, int n_curves) {
  hipLaunchKernelGGL(batch_lattice_check_kernel, dim3((unsigned)n_curves), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_batch_pack_v(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total,
                               int m1) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_pack_v_kernel, dim3((unsigned)total), dim3(256), 0, s, jobs, begin, n_curves, m1);
  return hipGetLastError();
}

hipError_t launch_batch_rows(hipStream_t s, const CurveJob* jobs, const int* begin, const int* begin_red,
                             int n_curves, int total, int total_red, int nv, int mat, int vin, int base, double alpha,
                             int out) {
  if (total <= 0) return hipSuccess;
  const dim3 g((unsigned)total), b(256);
  switch (nv) {
    case 1: hipLaunchKernelGGL(batch_rows_partial_kernel<1>, g, b, 0, s, jobs, begin, n_curves, mat, vin); break;
    case 2: hipLaunchKernelGGL(batch_rows_partial_kernel<2>, g, b, 0, s, jobs, begin, n_curves, mat, vin); break;
    case 3: hipLaunchKernelGGL(batch_rows_partial_kernel<3>, g, b, 0, s, jobs, begin, n_curves, mat, vin); break;
    case 4: hipLaunchKernelGGL(batch_rows_partial_kernel<4>, g, b, 0, s, jobs, begin, n_curves, mat, vin); break;
    case 5: hipLaunchKernelGGL(batch_rows_partial_kernel<5>, g, b, 0, s, jobs, begin, n_curves, mat, vin); break;
    case 6: hipLaunchKernelGGL(batch_rows_partial_kernel<6>, g, b, 0, s, jobs, begin, n_curves, mat, vin); break;
    case 7: hipLaunchKernelGGL(batch_rows_partial_kernel<7>, g, b, 0, s, jobs, begin, n_curves, mat, vin); break;
    case 8: hipLaunchKernelGGL(batch_rows_partial_kernel<8>, g, b, 0, s, jobs, begin, n_curves, mat, vin); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || total_red <= 0) return e;
  hipLaunchKernelGGL(batch_reduce_kernel<true>, dim3((unsigned)total_red), b, 0, s, jobs, begin_red, n_curves, base,
                     alpha, out);
  return hipGetLastError();
}

hipError_t launch_batch_null(hipStream_t s, const CurveJob* jobs, int n_curves, int m1) {
  hipLaunchKernelGGL(batch_null_kernel, dim3((unsigned)n_curves), dim3(256), 0, s, jobs, m1);
  return hipGetLastError();
}

hipError_t launch_batch_cols(hipStream_t s, const CurveJob* jobs, const int* begin, const int* begin_red,
                             int n_curves, int total, int total_red, int nv, int mat, int win, int base, double alpha,
                             int out) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_cols_partial_kernel, dim3((unsigned)total), dim3(256), 0, s, jobs, begin, n_curves, nv, mat,
                     win);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || total_red <= 0) return e;
  hipLaunchKernelGGL(batch_reduce_kernel<false>, dim3((unsigned)total_red), dim3(256), 0, s, jobs, begin_red, n_curves,
                     base, alpha, out);
  return hipGetLastError();
}

hipError_t launch_batch_slot_count(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_slot_count_kernel, dim3((unsigned)total), dim3(256), 0, s, jobs, begin, n_curves);
  return hipGetLastError();
}

hipError_t launch_batch_q_partial(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total,
                                  const int32_t* dur_sorted, int n_d, int dmax) {
  if (total <= 0) return hipSuccess;
  DurList dl{};
  dl.n = n_d;
  for (int k = 0; k < n_d; ++k) {
    dl.d[k] = dur_sorted[k];
    dl.perm[k] = dur_sorted[n_d + k];
  }
  const int seg = 64 + dmax;
  const dim3 g((unsigned)total), b(256);
  if (seg <= 64 * 2) hipLaunchKernelGGL(batch_q_partial_kernel<2>, g, b, 0, s, jobs, begin, n_curves, dl);
  else if (seg <= 64 * 3) hipLaunchKernelGGL(batch_q_partial_kernel<3>, g, b, 0, s, jobs, begin, n_curves, dl);
  else if (seg <= 64 * 5) hipLaunchKernelGGL(batch_q_partial_kernel<5>, g, b, 0, s, jobs, begin, n_curves, dl);
  else if (seg <= 64 * 9) hipLaunchKernelGGL(batch_q_partial_kernel<9>, g, b, 0, s, jobs, begin, n_curves, dl);
  else if (seg <= 64 * 17) hipLaunchKernelGGL(batch_q_partial_kernel<17>, g, b, 0, s, jobs, begin, n_curves, dl);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_batch_epilogue(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total,
                                 const int32_t* dur, int n_d, int m1) {
  if (total <= 0) return hipSuccess;
  DurList dl{};
  dl.n = n_d;
  for (int k = 0; k < n_d; ++k) {
    dl.d[k] = dur[k];
    dl.perm[k] = k;
    dl.off[k] = 0;
  }
  hipLaunchKernelGGL(batch_epilogue_kernel, dim3((unsigned)total), dim3(256), 0, s, jobs, begin, n_curves, dl, m1);
  return hipGetLastError();
}

// workgroups of a linear-search stage for one curve (the grids of the single-curve launches)
int64_t linear_stage_blocks(int stage, const CurveJob& J, int n_d) {
  switch (stage) {
    case BS_CHECK: return 1;
    case BS_PACKV: return (J.n + 255) / 256;
    case BS_ROWS: return (int64_t)rows_groups(J.n) * J.rchunks;
    case BS_ROWS_RED: return (J.n * YCOLS + 255) / 256;
    case BS_NULL: return 1;
    case BS_COLS: return (J.np + 255) / 256 * J.xchunks;
    case BS_COLS_RED: return (J.np * YCOLS + 255) / 256;
    case BS_SLOTS: return (J.n_epochs + 1 + 255) / 256;
    case BS_QPART: return (J.n_epochs + QCH - 1) / QCH * J.qchunks;
    case BS_EPI: return ((int64_t)n_d * J.n_epochs + 255) / 256;
    default: return 0;
  }
}

}  // namespace nu
