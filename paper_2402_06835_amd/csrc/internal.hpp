// Internal declarations shared by the HIP sources of the transit-search library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "nuance_mi355x.h"

namespace nu {

// Block edge of the dense factorisation: matrices are padded to a multiple of
// TB (identity on the padded diagonal), every GEMM problem is a multiple of
// TB in M and N, and the diagonal blocks factored in LDS are TB x TB.
constexpr int TB = 128;
constexpr int MAX_M1 = 7;        // trend columns
constexpr int YCOLS = 8;         // row stride of the whitened [A | f] panel
constexpr int MAX_ND = 16;       // durations per search
constexpr int MAX_DUR = 1024;    // samples per box

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// One C = alpha * op(A) * op(B) + beta * C problem of a grouped launch.
// All matrices are row-major. A is M x K (lda), op(B) is K x N: B itself is
// K x N (ldb) or, with G_BT, N x K (ldb). Triangular flags restrict the
// k-range per output tile to where the triangular operand is non-zero; the
// zero entries inside that range must be stored zeros.
enum GemmFlags : int {
  G_BT = 1,             // B stored transposed (N x K)
  G_A_LOWER = 2,        // A lower triangular: k < m0 + TB
  G_B_LOWER = 4,        // op(B) lower triangular: k >= n0
  G_B_UPPER = 8,        // op(B) upper triangular: k < n0 + TB
  G_C_LOWER_TILES = 16  // only tiles with row block >= column block
};

struct GemmProblem {
  const void* A;  // element type given by the launch (double or float)
  const void* B;
  void* C;
  int64_t lda, ldb, ldc;
  int M, N, K;
  int flags;
  double alpha, beta;
  int tiles_n;
  int tile_begin;
  int tile_count;
  int pad_;
};

struct NullFit {
  double G0chol[MAX_M1 * MAX_M1];  // lower Cholesky factor of A^T K^-1 A
  double w0[MAX_M1];
  double chi2_0;
  double lnl0;
  double logdet;
  int ok;
  int pad_;
};

}  // namespace nu

struct nu_timing_slot {
  int64_t launches = 0;
  double ms = 0.0;
  double work = 0.0;
};

struct nu_pending_event {
  std::string name;
  hipEvent_t start, stop;
  double work;
};

struct nu_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  // growable device workspace
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // kernel timing
  bool timing = false;
  std::vector<nu_pending_event> pending;
  std::vector<hipEvent_t> free_events;
  std::map<std::string, nu_timing_slot> timings;
  std::vector<std::string> timing_names;
};

namespace nu {
// one grouped launch: problems [first, first + count) of a schedule
struct Range {
  int first = 0, count = 0, tiles = 0;
  int tile = TB;  // output tile edge of the launch (128 or 64)
  double flops = 0.0;
};
constexpr int BAND_W = 2;  // block diagonals refined after a reduced-precision inverse
}  // namespace nu

struct nu_factor {
  int device = 0;
  int64_t n = 0;    // samples
  int64_t np = 0;   // padded to a multiple of TB
  double* L = nullptr;       // np x np row-major; lower triangle = Cholesky factor
  double* X = nullptr;       // np x np row-major; lower triangle = L^-1 (diagonal blocks at factor time)
  double* T = nullptr;       // workspace of the triangular-inverse levels
  size_t t_elems = 0;
  double* small = nullptr;   // logdet parts, logdet, status
  nu::NullFit* nullfit = nullptr;
  // FP64 schedule: Cholesky and triangular inverse
  nu::GemmProblem* probs = nullptr;
  std::vector<nu::GemmProblem> sched;
  std::vector<nu::Range> panel, pupd, trail, t1, t2;
  // reduced-precision inverse (allocated on first use)
  float* L32 = nullptr;
  float* X32 = nullptr;
  double* bandP = nullptr;   // (I, d) blocks of L X on the band, stored by column block
  double* bandX = nullptr;   // refined band blocks
  nu::GemmProblem* probs32 = nullptr;
  std::vector<nu::GemmProblem> sched32;
  std::vector<nu::Range> t1_32, t2_32, bandp, bandx;
  int inverse_kind = 0;  // 0 none, 1 FP64, 2 FP32 levels + refinement
  double logdet = 0.0;
};

namespace nu {

// error helpers (capi.cpp)
nu_status set_error(nu_ctx* ctx, nu_status st, const std::string& msg);
nu_status check_hip(nu_ctx* ctx, hipError_t e, const char* what);
void* ctx_workspace(nu_ctx* ctx, size_t bytes, nu_status* st);

// kernel timing (capi.cpp)
void timing_begin(nu_ctx* ctx, hipStream_t s, hipEvent_t* start);
void timing_end(nu_ctx* ctx, hipStream_t s, const char* name, hipEvent_t start, double work);

// launchers (*.hip)
hipError_t launch_kbuild(hipStream_t s, const double* t, int64_t n, int64_t np, const nu_sho& th, double* K);
hipError_t launch_gemm(hipStream_t s, const GemmProblem* dprobs, int nprob, int total_tiles, int f32, int tile);
hipError_t launch_potrf_diag(hipStream_t s, double* L, int64_t ld, int64_t off, int step, double* logdet_parts,
                             int64_t* status, double* Xdiag, int64_t ldx);
hipError_t launch_fill_i64(hipStream_t s, int64_t* p, int64_t v);
hipError_t launch_cvt_f64_f32(hipStream_t s, const double* src, float* dst, int64_t np, int diag_only);
hipError_t launch_cvt_f32_f64(hipStream_t s, const float* src, double* dst, int64_t np);
hipError_t launch_band_copy(hipStream_t s, double* X, int64_t np, double* band, int w, int to_band);
hipError_t launch_logdet_reduce(hipStream_t s, const double* parts, int nparts, double* out);

hipError_t launch_pack_v(hipStream_t s, const double* A, int m1, const double* f, int64_t n, double* V);
hipError_t launch_rows_matvec(hipStream_t s, const double* M, int64_t ldm, int64_t n, const double* V, int nv,
                              const double* base, double alpha, double* out);
hipError_t launch_null_solve(hipStream_t s, double* Y, int64_t n, int m1, const double* logdet, NullFit* nf,
                             double* null_out);
hipError_t launch_cols_matvec(hipStream_t s, const double* M, int64_t ldm, int64_t n, int64_t np, const double* W,
                              int nv, double* partial, int rowchunk, int nchunks, const double* base, double alpha,
                              double* out);
hipError_t launch_q_partial(hipStream_t s, const double* X, int64_t ldx, int64_t n, const int64_t* lattice,
                            int64_t n_epochs, const int32_t* dur_sorted, int n_d, int dmax, int rowchunk,
                            int nchunks, double* qpart);
hipError_t launch_cell_epilogue(hipStream_t s, const double* qpart, int nchunks, const int64_t* lattice, int64_t n,
                                int64_t n_epochs, const int32_t* dur, const int32_t* dur_rank, int n_d,
                                const double* Z, int m1, const NullFit* nf, double* depth, double* var, double* dll,
                                uint8_t* valid);
hipError_t launch_fold(hipStream_t s, const double* depth, const double* var, const double* dll,
                       const uint8_t* valid, int n_d, int64_t n_epochs, double dt, const double* periods, int64_t n_p,
                       int sign, double* q_snr, int64_t* best_phase, int32_t* best_dur, double* best_depth,
                       double* best_sigma, double* best_lnp, double* packed);
size_t fold_workspace_doubles(int n_d, int64_t n_epochs);
hipError_t launch_best_period(hipStream_t s, const double* q_snr, int64_t n_p, int64_t* out);

}  // namespace nu
