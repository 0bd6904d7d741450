// Grouped GEMM on the gfx950 matrix cores, FP64 (v_mfma_f64_16x16x4_f64) and
// FP32 (v_mfma_f32_16x16x4_f32).
//
// One launch runs a list of problems C = alpha * op(A) op(B) + beta * C; each
// workgroup owns one 128 x 128 (or, for launches with few tiles, 64 x 64)
// output tile of one problem. 256 threads = 4 waves in a 2 x 2 arrangement,
// each wave a 64 x 64 (32 x 32) sub-tile held as 4 x 4 (2 x 2) MFMA
// accumulators of 16 x 16. The k loop stages 16-deep slices of A and op(B)
// through LDS (k-major, double buffered; one barrier per slice).
//
// This is the dense contraction of the factorisation: the trailing updates
// and panels of the blocked Cholesky, and both products of every level of the
// triangular inverse X = L^-1 that whitens the box design of the linear search.
#include "internal.hpp"

// Accumulator layout of v_mfma_f32_16x16x4_f32 (set from the lane probe)
#ifndef MFMA_F32_ROW_INTERLEAVED
#define MFMA_F32_ROW_INTERLEAVED 0
#endif

namespace nu {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

constexpr int GBK = 16;
constexpr int LPAD = 4;

// Tile order within a problem: groups of GROUP tile-rows, column-major inside
// a group, so any run of consecutive tiles covers a compact block of rows and
// columns (their A row panels and B column panels meet in cache). For the
// lower-triangular tile set the same grouping is applied to the rows: the
// rectangular part of a group (columns left of its diagonal) comes first,
// then its triangle.
constexpr int GROUP = 16;

template <int BM>
__device__ __forceinline__ void tile_of(const GemmProblem& P, int t, int& tm, int& tn) {
  if (P.flags & G_C_LOWER_TILES) {
    const int T = P.M / BM;
    int r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    while (r * (r + 1) / 2 > t) --r;
    int g0 = (r / GROUP) * GROUP;
    const int R = min(GROUP, T - g0);
    int u = t - g0 * (g0 + 1) / 2;
    if (u < g0 * R) {
      tn = u / R;
      tm = g0 + u % R;
    } else {
      u -= g0 * R;
      int c = 0;
      while (u >= R - c) {
        u -= R - c;
        ++c;
      }
      tn = g0 + c;
      tm = g0 + c + u;
    }
  } else {
    const int Tm = P.M / BM, Tn = P.tiles_n;
    const int g = t / (GROUP * Tn);
    const int g0 = g * GROUP;
    const int R = min(GROUP, Tm - g0);
    const int u = t - g * GROUP * Tn;
    tn = u / R;
    tm = g0 + u % R;
  }
}

// Matrix-core operation per element type: the accumulator of one 16 x 16 x 4
// product and the row that item i of a lane holds (measured on gfx950: the
// f64 accumulator interleaves rows by 4, the f32 one holds 4 consecutive rows).
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef dbl4 acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int i) { return lk + 4 * i; }
};
template <>
struct Mfma<float> {
  typedef flt4 acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int i) { return MFMA_F32_ROW_INTERLEAVED ? lk + 4 * i : 4 * lk + i; }
};

// E consecutive elements from global memory into registers, 16-byte loads
template <typename T, int E>
__device__ __forceinline__ void loadE(const T* p, T (&r)[E]) {
  constexpr int PER = 16 / sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(PER)));
  const vec_t* v = reinterpret_cast<const vec_t*>(p);
#pragma unroll
  for (int i = 0; i < E / PER; ++i) {
    const vec_t x = v[i];
#pragma unroll
    for (int e = 0; e < PER; ++e) r[i * PER + e] = x[e];
  }
}

// BM x BM output tile per workgroup (BM = 128 or 64), 4 waves in a 2 x 2
// arrangement of (BM/2) x (BM/2) sub-tiles.
template <typename T, int BM>
__global__ __launch_bounds__(256, 2) void gemm_kernel(const GemmProblem* __restrict__ probs, int nprob) {
  constexpr int BN = BM;
  constexpr int E = BM * GBK / 256;  // elements per thread per operand slice
  constexpr int WT = BM / 2;         // wave sub-tile edge
  constexpr int NB = WT / 16;        // MFMA blocks per wave sub-tile edge
  __shared__ T As[2][GBK][BM + LPAD];
  __shared__ T Bs[2][GBK][BN + LPAD];
  typedef typename Mfma<T>::acc_t acc_t;

  // Workgroups go to the 8 XCDs round-robin, so the tiles resident at once
  // are consecutive tiles of the grouped order: a compact block of rows x
  // columns whose panels all XCDs stream together (shared last-level cache).
  const int tile = blockIdx.x;
  int lo = 0, hi = nprob - 1;  // last problem with tile_begin <= tile
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
  }
  const GemmProblem P = probs[lo];
  int tm, tn;
  tile_of<BM>(P, tile - P.tile_begin, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  int kb = 0, ke = P.K;
  if (P.flags & G_A_LOWER) ke = min(ke, m0 + BM);
  if (P.flags & G_B_LOWER) kb = max(kb, n0);
  if (P.flags & G_B_UPPER) ke = min(ke, n0 + BN);
  const int nk = ke > kb ? (ke - kb) / GBK : 0;
  const bool bt = (P.flags & G_BT) != 0;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WT, wn = (wave & 1) * WT;
  const int lr = lane & 15, lk = lane >> 4;

  // global -> register staging: "row-major M x K -> [k][m]" pattern for A (and B^T)
  const int ar = tid / (GBK / E), akh = (tid % (GBK / E)) * E;
  // "row-major K x N -> [k][n]" pattern for B
  const int bk = tid / (BN / E), bnc = (tid % (BN / E)) * E;

  const T* A = static_cast<const T*>(P.A);
  const T* B = static_cast<const T*>(P.B);
  const T* Ap = A + (int64_t)(m0 + ar) * P.lda + akh;
  const T* Bp = bt ? B + (int64_t)(n0 + ar) * P.ldb + akh : B + (int64_t)bk * P.ldb + n0 + bnc;

  T ra[E], rb[E];
  auto gload = [&](int k0) {
    loadE<T, E>(Ap + k0, ra);
    loadE<T, E>(bt ? Bp + k0 : Bp + (int64_t)k0 * P.ldb, rb);
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < E; ++i) As[buf][akh + i][ar] = ra[i];
    if (bt) {
#pragma unroll
      for (int i = 0; i < E; ++i) Bs[buf][akh + i][ar] = rb[i];
    } else {
#pragma unroll
      for (int i = 0; i < E; ++i) Bs[buf][bk][bnc + i] = rb[i];
    }
  };

  acc_t acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  if (nk > 0) {
    gload(kb);
    lstore(0);
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
      const int buf = it & 1;
      if (it + 1 < nk) gload(kb + (it + 1) * GBK);
#pragma unroll
      for (int kk = 0; kk < GBK / 4; ++kk) {
        T a[NB], b[NB];
#pragma unroll
        for (int mi = 0; mi < NB; ++mi) a[mi] = As[buf][kk * 4 + lk][wm + mi * 16 + lr];
#pragma unroll
        for (int ni = 0; ni < NB; ++ni) b[ni] = Bs[buf][kk * 4 + lk][wn + ni * 16 + lr];
#pragma unroll
        for (int mi = 0; mi < NB; ++mi)
#pragma unroll
          for (int ni = 0; ni < NB; ++ni) acc[mi][ni] = Mfma<T>::op(a[mi], b[ni], acc[mi][ni]);
      }
      if (it + 1 < nk) lstore(buf ^ 1);
      __syncthreads();
    }
  }

  const T alpha = (T)P.alpha, beta = (T)P.beta;
  T* C = static_cast<T*>(P.C);
#pragma unroll
  for (int mi = 0; mi < NB; ++mi)
#pragma unroll
    for (int ni = 0; ni < NB; ++ni)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = m0 + wm + mi * 16 + Mfma<T>::row(lk, i);
        const int col = n0 + wn + ni * 16 + lr;
        T* c = C + (int64_t)row * P.ldc + col;
        T v = alpha * acc[mi][ni][i];
        if (beta != (T)0) v = fma(beta, *c, v);
        *c = v;
      }
}

hipError_t launch_gemm(hipStream_t s, const GemmProblem* dprobs, int nprob, int total_tiles, int f32, int tile) {
  if (total_tiles <= 0) return hipSuccess;
  const dim3 g((unsigned)total_tiles), b(256);
  if (f32) {
    if (tile == 64) hipLaunchKernelGGL((gemm_kernel<float, 64>), g, b, 0, s, dprobs, nprob);
    else hipLaunchKernelGGL((gemm_kernel<float, 128>), g, b, 0, s, dprobs, nprob);
  } else {
    if (tile == 64) hipLaunchKernelGGL((gemm_kernel<double, 64>), g, b, 0, s, dprobs, nprob);
    else hipLaunchKernelGGL((gemm_kernel<double, 128>), g, b, 0, s, dprobs, nprob);
  }
  return hipGetLastError();
}

}  // namespace nu
