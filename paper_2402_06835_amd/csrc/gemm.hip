// Grouped GEMM on the gfx950 matrix cores, FP64 (v_mfma_f64_16x16x4_f64) and
// FP32 (v_mfma_f32_16x16x4_f32).
//
// One launch runs a list of problems C = alpha * op(A) op(B) + beta * C; each
// workgroup owns one 128 x 128 output tile of one problem (or, for launches
// with few tiles, 64 x 64, or 64 x 128 where C aliases A). 256 threads = 4
// waves in a 2 x 2 arrangement, each wave a quarter of the tile held as 16 x 16
// MFMA accumulators. The k loop stages 16-deep slices of A and op(B) through
// LDS (k-major, double buffered; one barrier per slice).
//
// A problem may write C over its own A (the Cholesky panel, times the inverse
// of the diagonal block) only if every tile spans all N columns: a tile reads
// whole rows of A, and another tile of the same rows must not overwrite them
// while it does.
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

// BM x BN output tile per workgroup ((128, 128), (64, 64) or (64, 128)),
// 4 waves in a 2 x 2 arrangement of (BM/2) x (BN/2) sub-tiles.
template <typename T, int BM, int BN>
__global__ __launch_bounds__(256, 2) void gemm_kernel(const GemmProblem* __restrict__ probs, int nprob) {
  constexpr int EA = BM * GBK / 256;  // elements per thread of an A slice
  constexpr int EB = BN * GBK / 256;  // elements per thread of a B slice
  constexpr int NBM = BM / 32;        // MFMA blocks per wave sub-tile, rows
  constexpr int NBN = BN / 32;        // and columns
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
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
  const int lr = lane & 15, lk = lane >> 4;

  // global -> register staging: "row-major M x K -> [k][m]" pattern for A (and B^T)
  const int ar = tid / (GBK / EA), akh = (tid % (GBK / EA)) * EA;
  const int br = tid / (GBK / EB), bkh = (tid % (GBK / EB)) * EB;
  // "row-major K x N -> [k][n]" pattern for B
  const int bk = tid / (BN / EB), bnc = (tid % (BN / EB)) * EB;

  const T* A = static_cast<const T*>(P.A);
  const T* B = static_cast<const T*>(P.B);
  const T* Ap = A + (int64_t)(m0 + ar) * P.lda + akh;
  const T* Bp = bt ? B + (int64_t)(n0 + br) * P.ldb + bkh : B + (int64_t)bk * P.ldb + n0 + bnc;

  T ra[EA], rb[EB];
  auto gload = [&](int k0) {
    loadE<T, EA>(Ap + k0, ra);
    loadE<T, EB>(bt ? Bp + k0 : Bp + (int64_t)k0 * P.ldb, rb);
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < EA; ++i) As[buf][akh + i][ar] = ra[i];
    if (bt) {
#pragma unroll
      for (int i = 0; i < EB; ++i) Bs[buf][bkh + i][br] = rb[i];
    } else {
#pragma unroll
      for (int i = 0; i < EB; ++i) Bs[buf][bk][bnc + i] = rb[i];
    }
  };

  acc_t acc[NBM][NBN];
#pragma unroll
  for (int i = 0; i < NBM; ++i)
#pragma unroll
    for (int j = 0; j < NBN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  if (nk > 0) {
    gload(kb);
    lstore(0);
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
      const int buf = it & 1;
      if (it + 1 < nk) gload(kb + (it + 1) * GBK);
#pragma unroll
      for (int kk = 0; kk < GBK / 4; ++kk) {
        T a[NBM], b[NBN];
#pragma unroll
        for (int mi = 0; mi < NBM; ++mi) a[mi] = As[buf][kk * 4 + lk][wm + mi * 16 + lr];
#pragma unroll
        for (int ni = 0; ni < NBN; ++ni) b[ni] = Bs[buf][kk * 4 + lk][wn + ni * 16 + lr];
#pragma unroll
        for (int mi = 0; mi < NBM; ++mi)
#pragma unroll
          for (int ni = 0; ni < NBN; ++ni) acc[mi][ni] = Mfma<T>::op(a[mi], b[ni], acc[mi][ni]);
      }
      if (it + 1 < nk) lstore(buf ^ 1);
      __syncthreads();
    }
  }

  const T alpha = (T)P.alpha, beta = (T)P.beta;
  T* C = static_cast<T*>(P.C);
#pragma unroll
  for (int mi = 0; mi < NBM; ++mi)
#pragma unroll
    for (int ni = 0; ni < NBN; ++ni)
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

template <typename T>
void launch_typed(hipStream_t s, const GemmProblem* dprobs, int nprob, dim3 g, int tm, int tn) {
  const dim3 b(256);
  if (tm == 64 && tn == 64) hipLaunchKernelGGL((gemm_kernel<T, 64, 64>), g, b, 0, s, dprobs, nprob);
  else if (tm == 64) hipLaunchKernelGGL((gemm_kernel<T, 64, 128>), g, b, 0, s, dprobs, nprob);
  else hipLaunchKernelGGL((gemm_kernel<T, 128, 128>), g, b, 0, s, dprobs, nprob);
}

hipError_t launch_gemm(hipStream_t s, const GemmProblem* dprobs, int nprob, int total_tiles, int f32, int tile_m,
                       int tile_n) {
  if (total_tiles <= 0) return hipSuccess;
  if (!((tile_m == 128 && tile_n == 128) || (tile_m == 64 && (tile_n == 64 || tile_n == 128))))
    return hipErrorInvalidValue;
  const dim3 g((unsigned)total_tiles);
  if (f32) launch_typed<float>(s, dprobs, nprob, g, tile_m, tile_n);
  else launch_typed<double>(s, dprobs, nprob, g, tile_m, tile_n);
  return hipGetLastError();
}

}  // namespace nu
