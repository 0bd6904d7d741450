// Grouped GEMM on the gfx950 matrix cores, FP64 (v_mfma_f64_16x16x4_f64),
// FP32 (v_mfma_f32_16x16x4_f32) and split BF16 (v_mfma_f32_16x16x32_bf16 on
// FP32 data, see gemm_bf16x3_kernel).
//
// One launch runs a list of problems C = alpha * op(A) op(B) + beta * C; each
// workgroup owns one 128 x 128 output tile of one problem (or, for launches
// with few tiles, 64 x 64, or 64 x 128 where C aliases A). 256 threads = 4
// waves in a 2 x 2 arrangement, each wave a quarter of the tile held as 16 x 16
// MFMA accumulators. The k loop stages 16-deep slices of A and op(B) through
// LDS (k-major, double buffered; one barrier per slice). The slices come in by
// buffer loads: per slice a descriptor on the tile's first row, built in
// scalar registers, plus one fixed 32-bit offset per lane, so the loop does no
// vector address arithmetic and the loads of slice it + 2 stay in flight
// while slice it is computed. (With 64-bit vector addresses the compiler put
// the next addresses into registers of loads still in flight and waited for
// every load at the top of the loop: standalone 16384^2 x 768 FP64 products
// 67.7 -> 70.3 TFLOP/s, FP32 8192^3 products 142.8 -> 146 TFLOP/s.)
//
// A problem may write C over its own A (the Cholesky panel, times the inverse
// of the diagonal block) only if every tile spans all N columns: a tile reads
// whole rows of A, and another tile of the same rows must not overwrite them
// while it does.
//
// This is the dense contraction of the factorisation: the trailing updates
// and panels of the blocked Cholesky, and both products of every level of the
// triangular inverse X = L^-1 that whitens the box design of the linear search.
#include <hip/hip_ext.h>

#include "internal.hpp"

// LDS stores of the next k-slice interleaved with the MFMAs of the current one
#ifndef NU_GEMM_INTERLEAVE
#define NU_GEMM_INTERLEAVE 1
#endif

// Accumulator layout of v_mfma_f32_16x16x4_f32 (set from the lane probe)
#ifndef MFMA_F32_ROW_INTERLEAVED
#define MFMA_F32_ROW_INTERLEAVED 0
#endif

namespace nu {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef float flt2 __attribute__((ext_vector_type(2)));

constexpr int GBK = 16;
// LDS row padding of the staged slices, per element type
#ifndef NU_LPAD_F32
#define NU_LPAD_F32 4
#endif
template <typename T>
struct Lpad {
  static constexpr int v = 4;
};
template <>
struct Lpad<float> {
  static constexpr int v = NU_LPAD_F32;
};

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
  } else if (P.flags & G_A_LOWER) {
    // a lower A gives row group g about g + 1 slices of k per tile: the
    // heaviest groups go first, so the launch ends on light tiles
    const int Tm = P.M / BM, Tn = P.tiles_n;
    const int G = (Tm + GROUP - 1) / GROUP, Rl = Tm - (G - 1) * GROUP;
    int g, u, R;
    if (t < Rl * Tn) {
      g = G - 1;
      u = t;
      R = Rl;
    } else {
      const int t2 = t - Rl * Tn;
      g = G - 2 - t2 / (GROUP * Tn);
      u = t2 - (t2 / (GROUP * Tn)) * GROUP * Tn;
      R = GROUP;
    }
    tn = u / R;
    tm = g * GROUP + u % R;
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
__device__ __forceinline__ void loadE(const NU_GLOBAL T* p, T (&r)[E]) {
  constexpr int PER = 16 / sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(PER)));
  const NU_GLOBAL vec_t* v = reinterpret_cast<const NU_GLOBAL vec_t*>(p);
#pragma unroll
  for (int i = 0; i < E / PER; ++i) {
    const vec_t x = v[i];
#pragma unroll
    for (int e = 0; e < PER; ++e) r[i * PER + e] = x[e];
  }
}

typedef int int4v __attribute__((ext_vector_type(4)));
// raw buffer descriptor over [p, p + 4 GiB): no stride, unformatted 32-bit data
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, -1, 0x00020000);
}
// E consecutive elements at byte offset voff of a buffer, 16-byte loads
template <typename T, int E>
__device__ __forceinline__ void bloadE(__amdgpu_buffer_rsrc_t rs, uint32_t voff, T (&r)[E]) {
  constexpr int PER = 16 / sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(PER)));
#pragma unroll
  for (int i = 0; i < E / PER; ++i) {
    const vec_t x = __builtin_bit_cast(vec_t, __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 16u * i, 0, 0));
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
  constexpr int LPAD = Lpad<T>::v;
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
  if (P.flags & G_PRIO) __builtin_amdgcn_s_setprio(2);
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

  // two register sets: the global loads of slice it + 2 are issued while
  // slice it is computed, two slices ahead of their LDS store
  T ra0[EA], rb0[EB], ra1[EA], rb1[EB];
  // buffer loads: a descriptor on the tile's first row of A (of B) per slice,
  // built in scalar registers, and one loop-invariant 32-bit lane offset, so
  // no per-slice vector address arithmetic (a tile's rows span far less than
  // 2^32 bytes for any matrix that fits the device)
  const char* Abase = (const char*)P.A + (int64_t)m0 * P.lda * (int64_t)sizeof(T);
  const char* Bbase = (const char*)P.B + (bt ? (int64_t)n0 * P.ldb : (int64_t)n0) * (int64_t)sizeof(T);
  const uint32_t aoff = (uint32_t)(((int64_t)ar * P.lda + akh) * (int64_t)sizeof(T));
  const uint32_t boff = (uint32_t)((bt ? (int64_t)br * P.ldb + bkh : (int64_t)bk * P.ldb + bnc) * (int64_t)sizeof(T));
  const int64_t bstep = bt ? (int64_t)sizeof(T) : (int64_t)P.ldb * (int64_t)sizeof(T);
  auto gload = [&](int k0, T (&ra)[EA], T (&rb)[EB]) {
    bloadE<T, EA>(make_rsrc(Abase + (int64_t)k0 * (int64_t)sizeof(T)), aoff, ra);
    bloadE<T, EB>(make_rsrc(Bbase + (int64_t)k0 * bstep), boff, rb);
  };
  auto lstore = [&](int buf, const T (&ra)[EA], const T (&rb)[EB]) {
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

  // part q of 4 of the LDS store of a slice (a quarter of each thread's A and B
  // elements). The B element i of a thread goes to Bs[k0 + i dk][n0 + i dn]:
  // along k for B stored transposed, along n otherwise (no branch in the loop).
  const int bs_k0 = bt ? bkh : bk, bs_n0 = bt ? br : bnc, bs_step = bt ? BN + LPAD : 1;
  auto lstore_part = [&](int q, int buf, const T (&ra)[EA], const T (&rb)[EB]) {
    constexpr int QA = (EA + 3) / 4, QB = (EB + 3) / 4;
#pragma unroll
    for (int i = q * QA; i < (q + 1) * QA && i < EA; ++i) As[buf][akh + i][ar] = ra[i];
    T* bb = &Bs[buf][bs_k0][bs_n0];
#pragma unroll
    for (int i = q * QB; i < (q + 1) * QB && i < EB; ++i) bb[i * bs_step] = rb[i];
  };
  // slice it from buffer buf; with `store`, the next slice goes into the other
  // buffer a quarter after each k-step, so the LDS stores issue among the MFMAs
  // instead of after them (the other buffer was last read before the previous
  // barrier)
  auto compute = [&](int buf, const T (&ran)[EA], const T (&rbn)[EB]) {
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
#if NU_GEMM_INTERLEAVE
      lstore_part(kk, buf ^ 1, ran, rbn);
#endif
    }
#if !NU_GEMM_INTERLEAVE
    lstore(buf ^ 1, ran, rbn);
#endif
  };
  // one slice: compute buffer it & 1 (slice it), refill the register set
  // that held slice it with slice it + 2, store slice it + 1 from the other.
  // The loads and stores are unconditional (near the end of the k range the
  // last slice is loaded again, and a store goes to a buffer no one reads any
  // more), so the loop body has no branch: the compiler then counts the loads
  // in flight exactly (a conditional load forced a wait for all of them) and
  // schedules the LDS reads of a k-step among the MFMAs of the previous one.
  auto step = [&](int it, T (&rac)[EA], T (&rbc)[EB], T (&ran)[EA], T (&rbn)[EB]) {
    gload(kb + min(it + 2, nk - 1) * GBK, rac, rbc);
    // keep the loads ahead of the products (the scheduler would otherwise
    // sink them and give their registers to the LDS operands)
    __builtin_amdgcn_sched_barrier(0);
    compute(it & 1, ran, rbn);
    __syncthreads();
  };

  if (nk > 0) {
    gload(kb, ra0, rb0);
    gload(kb + min(1, nk - 1) * GBK, ra1, rb1);
    lstore(0, ra0, rb0);
    __syncthreads();
    for (int it = 0; it < nk; it += 2) {
      step(it, ra0, rb0, ra1, rb1);
      if (it + 1 < nk) step(it + 1, ra1, rb1, ra0, rb0);
    }
  }

  const T alpha = (T)P.alpha, beta = (T)P.beta;
  NU_GLOBAL T* C = (NU_GLOBAL T*)P.C + (int64_t)(m0 + wm) * P.ldc + n0 + wn + lr;
  auto cptr = [&](int mi, int ni, int i) { return C + (int64_t)(mi * 16 + Mfma<T>::row(lk, i)) * P.ldc + ni * 16; };
  if (beta != (T)0) {
    // the loads of C of a row block all in flight before its stores (a store
    // could alias a later load as far as the compiler knows, which would
    // otherwise serialise every load behind the previous store)
#pragma unroll
    for (int mi = 0; mi < NBM; ++mi) {
      T cv[NBN][4];
#pragma unroll
      for (int ni = 0; ni < NBN; ++ni)
#pragma unroll
        for (int i = 0; i < 4; ++i) cv[ni][i] = *cptr(mi, ni, i);
#pragma unroll
      for (int ni = 0; ni < NBN; ++ni)
#pragma unroll
        for (int i = 0; i < 4; ++i) *cptr(mi, ni, i) = fma(beta, cv[ni][i], alpha * acc[mi][ni][i]);
    }
  } else {
#pragma unroll
    for (int mi = 0; mi < NBM; ++mi)
#pragma unroll
      for (int ni = 0; ni < NBN; ++ni)
#pragma unroll
        for (int i = 0; i < 4; ++i) *cptr(mi, ni, i) = alpha * acc[mi][ni][i];
  }
}

// ---------------------------------------------------------------------------
// Split BF16 products with FP32 accumulation. Every FP32 operand x is held as
// hi + lo, hi = x rounded to BF16 and lo = (x - hi) rounded to BF16 (x - hi is
// exact in FP32), which carries 16 of x's 24 significand bits; a product is
// taken as lo_a hi_b + hi_a lo_b + hi_a hi_b, leaving out lo_a lo_b (2^-16
// relative). One v_mfma_f32_16x16x32_bf16 covers 32 k at the BF16 rate, so
// the three products cost about a fifth of the FP32 matrix-core time of
// v_mfma_f32_16x16x4_f32. The relative error per product is ~2^-16 instead of
// 2^-24; the triangular inverse built this way gets a wider FP64 band step.
//
// Operands are FP32 in memory (A row-major M x K, B row-major K x N; no G_BT
// and no G_C_IS_A), split once while a slice is staged: LDS holds the hi and
// lo halves k-contiguous per row of A and per column of B, so each lane
// fetches its 8 k of a 16 x 16 x 32 operand with one 16-byte read (row stride
// 80 bytes: the 16 rows of a quarter-wave fall on disjoint banks). A and B
// take k in the same lane order, which is all the product needs.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int SBK = 32;        // k depth of a slice: one MFMA
constexpr int SROW = SBK + 8;  // LDS row stride in BF16 elements

__device__ __forceinline__ void split8(const float (&x)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)x[e];
    hi[e] = h;
    lo[e] = (__bf16)(x[e] - (float)h);
  }
}

template <int BM, int BN>
__global__ __launch_bounds__(256, 2) void gemm_bf16x3_kernel(const GemmProblem* __restrict__ probs, int nprob) {
  constexpr int NBM = BM / 32, NBN = BN / 32;  // MFMA blocks per wave sub-tile
  constexpr int EA = BM * SBK / 256;           // A elements per thread and slice: one row segment
  constexpr int APR = SBK / EA;                // threads per A row
  constexpr int NBC = BN / 64;                 // B columns per thread (8 k each)
  constexpr int BCT = BN / NBC;                // threads across the B columns
  static_assert(EA % 8 == 0 && 256 / BCT * 8 == SBK, "staging layout");
  __shared__ __attribute__((aligned(16))) __bf16 Ah[2][BM][SROW];
  __shared__ __attribute__((aligned(16))) __bf16 Al[2][BM][SROW];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[2][BN][SROW];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[2][BN][SROW];

  const int tile = blockIdx.x;
  int lo_p = 0, hi_p = nprob - 1;  // last problem with tile_begin <= tile
  while (lo_p < hi_p) {
    const int mid = (lo_p + hi_p + 1) >> 1;
    if (probs[mid].tile_begin <= tile) lo_p = mid; else hi_p = mid - 1;
  }
  const GemmProblem P = probs[lo_p];
  int tm, tn;
  tile_of<BM>(P, tile - P.tile_begin, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  int kb = 0, ke = P.K;
  if (P.flags & G_A_LOWER) ke = min(ke, m0 + BM);
  if (P.flags & G_B_LOWER) kb = max(kb, n0);
  if (P.flags & G_B_UPPER) ke = min(ke, n0 + BN);
  const int nk = ke > kb ? (ke - kb) / SBK : 0;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
  const int lr = lane & 15, lg = lane >> 4;

  const int ar = tid / APR, ak = (tid % APR) * EA;         // A: one row, EA consecutive k
  const int bc = (tid % BCT) * NBC, bk = (tid / BCT) * 8;  // B: NBC columns, 8 consecutive k
  const NU_GLOBAL float* Ap = (const NU_GLOBAL float*)P.A + (int64_t)(m0 + ar) * P.lda + ak;
  const NU_GLOBAL float* Bp = (const NU_GLOBAL float*)P.B + (int64_t)bk * P.ldb + n0 + bc;

  float ra[EA], rb[NBC][8];
  auto gload = [&](int k0) {
    loadE<float, EA>(Ap + k0, ra);
    const NU_GLOBAL float* b = Bp + (int64_t)k0 * P.ldb;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if constexpr (NBC == 2) {
        const flt2 v = *reinterpret_cast<const NU_GLOBAL flt2*>(b + (int64_t)r * P.ldb);
        rb[0][r] = v[0];
        rb[1][r] = v[1];
      } else {
        rb[0][r] = b[(int64_t)r * P.ldb];
      }
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int h = 0; h < EA / 8; ++h) {
      float x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = ra[h * 8 + e];
      bf16x8 vh, vl;
      split8(x, vh, vl);
      *reinterpret_cast<bf16x8*>(&Ah[buf][ar][ak + h * 8]) = vh;
      *reinterpret_cast<bf16x8*>(&Al[buf][ar][ak + h * 8]) = vl;
    }
#pragma unroll
    for (int c = 0; c < NBC; ++c) {
      bf16x8 vh, vl;
      split8(rb[c], vh, vl);
      *reinterpret_cast<bf16x8*>(&Bh[buf][bc + c][bk]) = vh;
      *reinterpret_cast<bf16x8*>(&Bl[buf][bc + c][bk]) = vl;
    }
  };

  flt4 acc[NBM][NBN];
#pragma unroll
  for (int i = 0; i < NBM; ++i)
#pragma unroll
    for (int j = 0; j < NBN; ++j) acc[i][j] = flt4{0, 0, 0, 0};

  if (nk > 0) {
    gload(kb);
    lstore(0);
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
      const int buf = it & 1;
      if (it + 1 < nk) gload(kb + (it + 1) * SBK);
      bf16x8 ah[NBM], al[NBM], bh[NBN], bl[NBN];
#pragma unroll
      for (int mi = 0; mi < NBM; ++mi) {
        ah[mi] = *reinterpret_cast<const bf16x8*>(&Ah[buf][wm + mi * 16 + lr][lg * 8]);
        al[mi] = *reinterpret_cast<const bf16x8*>(&Al[buf][wm + mi * 16 + lr][lg * 8]);
      }
#pragma unroll
      for (int ni = 0; ni < NBN; ++ni) {
        bh[ni] = *reinterpret_cast<const bf16x8*>(&Bh[buf][wn + ni * 16 + lr][lg * 8]);
        bl[ni] = *reinterpret_cast<const bf16x8*>(&Bl[buf][wn + ni * 16 + lr][lg * 8]);
      }
      // small terms first; each pass is NBM * NBN independent accumulations
#pragma unroll
      for (int mi = 0; mi < NBM; ++mi)
#pragma unroll
        for (int ni = 0; ni < NBN; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[mi], bh[ni], acc[mi][ni], 0, 0, 0);
#pragma unroll
      for (int mi = 0; mi < NBM; ++mi)
#pragma unroll
        for (int ni = 0; ni < NBN; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mi], bl[ni], acc[mi][ni], 0, 0, 0);
#pragma unroll
      for (int mi = 0; mi < NBM; ++mi)
#pragma unroll
        for (int ni = 0; ni < NBN; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mi], bh[ni], acc[mi][ni], 0, 0, 0);
      if (it + 1 < nk) lstore(buf ^ 1);
      __syncthreads();
    }
  }

  // accumulator of a 16 x 16 block: lane (lr, lg) holds column lr, rows 4 lg .. 4 lg + 3
  const float alpha = (float)P.alpha, beta = (float)P.beta;
  NU_GLOBAL float* C = (NU_GLOBAL float*)P.C + (int64_t)(m0 + wm) * P.ldc + n0 + wn + lr;
  auto cptr = [&](int mi, int ni, int i) { return C + (int64_t)(mi * 16 + 4 * lg + i) * P.ldc + ni * 16; };
  if (beta != 0.0f) {
#pragma unroll
    for (int mi = 0; mi < NBM; ++mi) {
      float cv[NBN][4];
#pragma unroll
      for (int ni = 0; ni < NBN; ++ni)
#pragma unroll
        for (int i = 0; i < 4; ++i) cv[ni][i] = *cptr(mi, ni, i);
#pragma unroll
      for (int ni = 0; ni < NBN; ++ni)
#pragma unroll
        for (int i = 0; i < 4; ++i) *cptr(mi, ni, i) = fmaf(beta, cv[ni][i], alpha * acc[mi][ni][i]);
    }
  } else {
#pragma unroll
    for (int mi = 0; mi < NBM; ++mi)
#pragma unroll
      for (int ni = 0; ni < NBN; ++ni)
#pragma unroll
        for (int i = 0; i < 4; ++i) *cptr(mi, ni, i) = alpha * acc[mi][ni][i];
  }
}

// With events, the launch records them itself at the start and end of its
// dispatch (hipExtLaunchKernelGGL).
template <typename K>
void launch_one(K kernel, dim3 g, hipStream_t s, hipEvent_t e0, hipEvent_t e1, const GemmProblem* dprobs, int nprob) {
  if (e0 || e1) hipExtLaunchKernelGGL(kernel, g, dim3(256), 0, s, e0, e1, 0, dprobs, nprob);
  else hipLaunchKernelGGL(kernel, g, dim3(256), 0, s, dprobs, nprob);
}

template <typename T>
void launch_typed(hipStream_t s, const GemmProblem* dprobs, int nprob, dim3 g, int tm, int tn, hipEvent_t e0,
                  hipEvent_t e1) {
  if (tm == 64 && tn == 64) launch_one(gemm_kernel<T, 64, 64>, g, s, e0, e1, dprobs, nprob);
  else if (tm == 64) launch_one(gemm_kernel<T, 64, 128>, g, s, e0, e1, dprobs, nprob);
  else launch_one(gemm_kernel<T, 128, 128>, g, s, e0, e1, dprobs, nprob);
}

hipError_t launch_gemm(hipStream_t s, const GemmProblem* dprobs, int nprob, int total_tiles, int kind, int tile_m,
                       int tile_n, hipEvent_t start, hipEvent_t stop) {
  if (total_tiles <= 0) return hipSuccess;
  if (!((tile_m == 128 && tile_n == 128) || (tile_m == 64 && (tile_n == 64 || tile_n == 128))))
    return hipErrorInvalidValue;
  const dim3 g((unsigned)total_tiles);
  switch (kind) {
    case GK_F64: launch_typed<double>(s, dprobs, nprob, g, tile_m, tile_n, start, stop); break;
    case GK_F32: launch_typed<float>(s, dprobs, nprob, g, tile_m, tile_n, start, stop); break;
    case GK_BF16X3:
      // square tiles only (64 x 128 serves the in-place panels, which this kind never runs)
      if (tile_m != tile_n) return hipErrorInvalidValue;
      if (tile_m == 64) launch_one(gemm_bf16x3_kernel<64, 64>, g, s, start, stop, dprobs, nprob);
      else launch_one(gemm_bf16x3_kernel<128, 128>, g, s, start, stop, dprobs, nprob);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nu
