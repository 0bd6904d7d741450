// Internal declarations shared by the HIP sources of the transit-search library.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <memory>
#include <map>
#include <string>
#include <vector>

#include "nuance_mi355x.h"

namespace nu {

// Block edge of the dense factorisation: matrices are padded to a multiple of
// TB (identity on the padded diagonal), every GEMM problem is a multiple of
// TB in M and N, and the diagonal blocks factored in LDS are TB x TB.
constexpr int TB = 128;

// Device pointers read out of a problem or job record are generic (flat)
// pointers to the compiler, and a flat load also counts against the LDS wait
// counter: every wait for an LDS read in a k loop would then wait for the
// global loads of the next slice too. Kernels cast such pointers to the global
// address space, which gives global_load / global_store.
#define NU_GLOBAL __attribute__((address_space(1)))
constexpr int MAX_M1 = 7;        // trend columns
constexpr int YCOLS = 8;         // row stride of the whitened [A | f] panel
// Algorithmic FP64 flops of the periodic fold per event visit (one event of
// one (phase, duration) cell; Eq. 8 with the estimates of Eq. B4): linear
// interpolation of depth, var and dll (3 flops each), the sums of 1/v, d/v and
// dll (5), and the terms (d - D)^2 / (v + sigma^2) and 1 + sigma^2 / v of the
// chi^2 and the log product (8).
constexpr double FOLD_FLOPS_PER_VISIT = 22.0;
constexpr int MAX_ND = 16;       // durations per search
constexpr int MAX_DUR = 1024;    // samples per box
constexpr int MAX_SEG = 32;      // segments of a segmented periodic search
constexpr int MAX_SHAPE = 2048;  // values of all shapes of a template search together
// Partials of the linear search's passes over X and L: rows per partial of the
// transposed products, columns per partial of the row products, rows per
// partial of the box sums of squares (measured choices, see run_linear)
constexpr int LIN_XRC = 512;
constexpr int LIN_RCW = 2048;
constexpr int LIN_QRC = 256;

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
  G_C_LOWER_TILES = 16,  // only tiles with row block >= column block (square tiles)
  G_C_IS_A = 32,         // C overwrites A's rows: every tile must span all N columns
  G_PRIO = 64            // the tile's waves take issue priority over other kernels' waves on their CU
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

// Launch classes of the dense schedule. Each class takes 64 x 64 output tiles
// when a launch has fewer 128 x 128 tiles than its threshold.
enum TuneClass { TC_PANEL = 0, TC_PUPD, TC_TRAIL, TC_INV64, TC_INV32, TC_BAND, TC_INVB, TC_COUNT };
struct Tuning {
  int small_below[TC_COUNT] = {512, 512, 512, 512, 512, 512, 512};
};

// Arithmetic of a grouped GEMM launch: FP64, FP32, or split BF16 products on
// FP32 data (hi + lo halves, three products, FP32 accumulation).
enum GemmKind { GK_F64 = 0, GK_F32 = 1, GK_BF16X3 = 2 };

// Block diagonals refined in FP64 after a reduced-precision inverse: the
// split-BF16 products leave ~2^-16 relative error where FP32 leaves 2^-24, so
// more of the near-diagonal weight of the box sums is restored in FP64.
constexpr int BAND_W_F32 = 2;
constexpr int BAND_W_BF16X3 = 8;
inline int band_width(int prec) { return prec == NU_BF16X3_REFINE ? BAND_W_BF16X3 : BAND_W_F32; }
// Steps of iterative refinement of the whitened trend and flux (Y = X V) and
// of their back-substitution (Z = X^T W) against the FP64 factor. Each step
// shrinks the error by about cond(K) times the inverse's relative error, so
// the split-BF16 inverse (2^-16) needs a second step where FP32 (2^-24) does
// not.
constexpr int REFINE_STEPS_F32 = 1;
constexpr int REFINE_STEPS_BF16X3 = 2;
inline int refine_steps(int prec) {
  return prec == NU_BF16X3_REFINE ? REFINE_STEPS_BF16X3 : prec == NU_FP32_REFINE ? REFINE_STEPS_F32 : 0;
}
inline int gemm_kind_of(int prec) {
  return prec == NU_BF16X3_REFINE ? GK_BF16X3 : prec == NU_FP32_REFINE ? GK_F32 : GK_F64;
}

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

namespace nu {
// Device bytes counted against a context's workspace limit (0: none): its
// search workspace and batch arena, and the buffers of the factors, graphs,
// networks and batch calls made on it. Every object holding such buffers
// shares the count, since it may outlive its context.
struct MemCount {
  std::atomic<size_t> live{0};
  size_t limit = 0;
};
// the part of its context's count one object holds
struct MemHold {
  std::shared_ptr<MemCount> count;
  size_t bytes = 0;
  void release() {
    if (count) count->live -= bytes;
    bytes = 0;
  }
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
  // growable device workspace of the searches
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // device arena of the batch factors, kept between calls
  void* arena = nullptr;
  size_t arena_bytes = 0;
  // device memory counted against the workspace limit
  std::shared_ptr<nu::MemCount> mem = std::make_shared<nu::MemCount>();
  // kernel timing (only of the launches whose name starts with timing_only, when set)
  bool timing = false;
  std::string timing_only;
  std::vector<nu_pending_event> pending;
  std::vector<hipEvent_t> free_events;
  std::map<std::string, nu_timing_slot> timings;
  std::vector<std::string> timing_names;
  // tile policy of the dense launches (set by the autotuner)
  nu::Tuning tuning;
  // the Cholesky's step loop (created on first use): the diagonal blocks,
  // panels and lookahead updates on s_fac; the rest of each trailing update
  // on s_rest, which leaves LOOKAHEAD_FREE_CUS compute units to s_fac
  hipStream_t s_fac = nullptr, s_rest = nullptr;
  // the periodic search of a batch wave, beside the next wave's factorisation
  // (created on first use; default priority, non-blocking)
  hipStream_t s_fold = nullptr;
  hipEvent_t ev_fork = nullptr, ev_pan = nullptr, ev_rest = nullptr, ev_join = nullptr;
  bool lookahead = true;
  // early inverse of a factorisation: its streams (both on the top s_inv_cus
  // CUs; early phases alternate between them, so a phase released late does
  // not queue behind an earlier phase's products), the event that releases a
  // phase and the event of each stream's last phase; the precision it is
  // started for (-1: none) and the CUs asked for (0: three quarters)
  hipStream_t s_inv[2] = {nullptr, nullptr};
  int s_inv_cus = 0;
  hipEvent_t ev_split = nullptr, ev_inv[2] = {nullptr, nullptr};
  int prefetch_prec = -1, prefetch_cus = 0;
  // pinned host staging of small host-to-device uploads (template shapes); the
  // event marks the last copy out of it
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t pinned_ev = nullptr;
  // this device's fixed scratch array of the allocation-free periodic search
  double* scratch = nullptr;
};

namespace nu {
// one grouped launch: problems [first, first + count) of a schedule
struct Range {
  int first = 0, count = 0, tiles = 0;
  int tile_m = TB, tile_n = TB;  // output tile of the launch: 128 x 128, 64 x 64 or 64 x 128
  double flops = 0.0;
};

// One diagonal block of the blocked Cholesky (one workgroup of a launch).
struct PotrfJob {
  double* L;            // the factor, row-major, leading dimension ld
  double* X;            // the inverse, same layout
  double* parts;        // per-step ln|L_kk| terms
  int64_t* status;      // first failing pivot, or -1
  int64_t ld;
  int64_t off;          // row and column of the block's first element
  int step;             // block index
  int pad_;
};

// Schedule of the dense work of one or more factors run together: grouped
// GEMM launches whose problem lists span every factor, and the diagonal
// blocks of each Cholesky step as one launch of one workgroup per factor.
struct Plan {
  std::vector<GemmProblem> sched;
  GemmProblem* dprobs = nullptr;
  std::vector<PotrfJob> jobs;
  PotrfJob* djobs = nullptr;
  std::vector<int> job_first, job_count;  // per Cholesky step
  std::vector<Range> panel, pupd;        // per Cholesky step
  std::vector<Range> next, rest;          // per step: the trailing update after a panel's last block, split
                                          // into the next panel's columns and the rest
  std::vector<Range> t1, t2;              // per inverse level, deepest first
  // a single factor's inverse split into phases by the columns they read
  // (phase k: columns left of cuts[k]; the last: all), each a list of
  // launches; empty: t1/t2 instead
  std::vector<std::vector<Range>> phases;
  std::vector<int> cuts;
  Range bandp, bandx;
  bool built = false;
};
void plan_release(Plan& P);

}  // namespace nu

struct nu_factor {
  int device = 0;
  int64_t n = 0;    // samples
  int64_t np = 0;   // padded to a multiple of TB
  int nblk = 0;     // np / TB
  double* L = nullptr;       // np x np row-major; lower triangle = Cholesky factor
  double* X = nullptr;       // np x np row-major; lower triangle = L^-1 (diagonal blocks at factor time)
  double* T = nullptr;       // workspace of the triangular-inverse levels
  size_t t_elems = 0;
  double* small = nullptr;   // [nblk] logdet parts, logdet, status (int64), theta (4), spare
  nu::NullFit* nullfit = nullptr;
  nu_sho theta_host{};       // source of the theta upload of the last factorisation
  bool general = false;      // K from kernel_dev() (a nu_kernel) instead of theta_dev()
  nu_kernel kernel_host{};   // source of the kernel upload of the last general factorisation
  nu::Plan plan64;           // Cholesky + FP64 inverse
  // reduced-precision inverse (allocated on first use)
  float* L32 = nullptr;
  float* X32 = nullptr;
  double* bandP = nullptr;   // (I, d) blocks of L X on the band, stored by column block
  double* bandX = nullptr;   // refined band blocks
  int band_w = 0;            // widest band the band buffers hold
  size_t band_bytes = 0;     // device bytes of the band buffers it allocated
  nu::Plan plan32;           // reduced-precision inverse + FP64 band step
  int plan32_prec = 0;       // the nu_precision plan32 was built for
  int inverse_kind = 0;  // 0 none, else 1 + the nu_precision X was formed in
  double logdet = 0.0;
  bool owns_memory = true;   // false: buffers carved from the context's arena
  nu::MemHold hold;          // its buffers' share of the context's memory count
  double* parts() const { return small; }
  double* logdet_dev() const { return small + nblk; }
  int64_t* status_dev() const { return reinterpret_cast<int64_t*>(small + nblk + 1); }
  nu_sho* theta_dev() const { return reinterpret_cast<nu_sho*>(small + nblk + 2); }
  nu_kernel* kernel_dev() const { return reinterpret_cast<nu_kernel*>(small + nblk + 8); }
};
// doubles of `small` after the per-block parts: logdet, status, theta (4), spare (2), a nu_kernel
constexpr int FACTOR_SMALL_EXTRA = 8 + (int)((sizeof(nu_kernel) + 7) / 8);

namespace nu {

// error helpers (capi.cpp)
nu_status set_error(nu_ctx* ctx, nu_status st, const std::string& msg);
nu_status check_hip(nu_ctx* ctx, hipError_t e, const char* what);
void* ctx_workspace(nu_ctx* ctx, size_t bytes, nu_status* st);
// NU_ERR_OOM if the context's count, less `replaced`, plus `bytes` exceeds its limit
nu_status mem_check(nu_ctx* ctx, size_t bytes, size_t replaced, const char* what);
// hipMalloc counted against the context's limit, on behalf of `hold`
nu_status ctx_malloc(nu_ctx* ctx, void** p, size_t bytes, MemHold& hold, const char* what);
// what a batch call may still place (the limit less what is held outside the arena; SIZE_MAX: no limit)
size_t mem_headroom(const nu_ctx* ctx, size_t replaced);
// host -> device copy on the context's stream through the pinned staging buffer
nu_status ctx_upload(nu_ctx* ctx, const void* host, size_t bytes, void* dev);
// template shapes: validates n_d shapes of dur_samples_host[j] values each (finite, total <= MAX_SHAPE)
nu_status validate_shapes(nu_ctx* ctx, const double* shapes_host, const int32_t* dur_samples_host, int n_d);

// kernel timing (capi.cpp): events on the context's stream around a launch
void timing_begin(nu_ctx* ctx, hipStream_t s, const char* name, hipEvent_t* start);
// events that a launch records itself (start and end of its own dispatch, no
// marker of their own in the stream), both null when `name` is not timed;
// timing_add queues them
void timing_pair(nu_ctx* ctx, const char* name, hipEvent_t* start, hipEvent_t* stop);
void timing_add(nu_ctx* ctx, const char* name, hipEvent_t start, hipEvent_t stop, double work);
void timing_end(nu_ctx* ctx, hipStream_t s, const char* name, hipEvent_t start, double work);
void resolve_timing(nu_ctx* ctx);  // synchronises the stream, folds pending events into the totals
struct Timed {
  nu_ctx* ctx;
  hipStream_t stream;
  const char* name;
  double work;
  hipEvent_t start;
  Timed(nu_ctx* c, const char* n, double w) : Timed(c, c->stream, n, w) {}
  Timed(nu_ctx* c, hipStream_t s, const char* n, double w) : ctx(c), stream(s), name(n), work(w) {
    timing_begin(c, s, n, &start);
  }
  ~Timed() { timing_end(ctx, stream, name, start, work); }
};

// Host wall time of a phase of a call (allocation, planning, waits, frees),
// accumulated under "host:<name>" when timing is on.
struct HostTimed {
  nu_ctx* ctx;
  const char* name;
  double t0;
  HostTimed(nu_ctx* c, const char* n);
  ~HostTimed();
};

// engine (engine.cpp)
void plan_cholesky(const std::vector<nu_factor*>& Fs, const Tuning& tu, Plan& P);
void plan_inverse(const std::vector<nu_factor*>& Fs, int kind, const Tuning& tu, Plan& P, bool split = false);
void plan_band(const std::vector<nu_factor*>& Fs, int w, const Tuning& tu, Plan& P);
size_t inverse_t_elems(int nblk);
nu_status plan_upload(nu_ctx* ctx, Plan& P);
size_t factor_bytes(int64_t n, int prec, size_t t_min = 0);
nu_status factor_alloc(nu_ctx* ctx, int64_t n, bool own_plan, nu_factor** out);
nu_status factor_place(nu_ctx* ctx, int64_t n, int prec, char** cursor, nu_factor** out, size_t t_min = 0);
void* ctx_arena(nu_ctx* ctx, size_t bytes, nu_status* st);
nu_status alloc_mixed(nu_ctx* ctx, nu_factor* F, int prec);
nu_status ensure_plan32(nu_ctx* ctx, nu_factor* F, int prec);
void factor_free(nu_factor* F);
nu_status launch_range(nu_ctx* ctx, const Plan& P, const Range& r, const char* name, int kind,
                       hipStream_t s = nullptr);  // s = nullptr: the context's stream
nu_status ensure_factor_streams(nu_ctx* ctx);
nu_status ensure_inverse_stream(nu_ctx* ctx, int compute_units);
void destroy_factor_streams(nu_ctx* ctx);
// The reduced-precision inverse of a single factor started inside its
// factorisation: each early phase as soon as the Cholesky has finished the
// columns it reads, beside the remaining steps, the last phase after them.
struct EarlyInverse {
  nu_factor* F = nullptr;
  int prec = 0;              // NU_FP32_REFINE or NU_BF16X3_REFINE; F->plan32 is built for it
  mutable int started = 0;   // out: the early phases enqueued (the rest is due)
};
nu_status run_factor(nu_ctx* ctx, const std::vector<nu_factor*>& Fs, const Plan& P,
                     const std::vector<const double*>& ts, const std::vector<const nu_sho*>& theta_dev,
                     const EarlyInverse* early = nullptr);
// the Cholesky's step loop alone (diagonal blocks, panels, trailing updates of P)
nu_status run_factor_steps(nu_ctx* ctx, const Plan& P, const EarlyInverse* early = nullptr);
nu_status read_factor_status(nu_ctx* ctx, const std::vector<nu_factor*>& Fs, std::vector<int64_t>& status);
nu_status run_inverse_fp64(nu_ctx* ctx, const Plan& P);
nu_status run_inverse_mixed(nu_ctx* ctx, const std::vector<nu_factor*>& Fs, const Plan& P, int prec);
nu_status run_inverse_phase(nu_ctx* ctx, nu_factor* F, const Plan& P, int prec, int k, hipStream_t s);
nu_status run_inverse_post(nu_ctx* ctx, nu_factor* F, const Plan& P, int prec);
size_t linear_ws_bytes(int64_t n, int n_d, int64_t n_epochs);
nu_status validate_linear(nu_ctx* ctx, int64_t n, const double* f, const double* A, int m1, const int64_t* lattice,
                          int64_t n_epochs, const int32_t* dur_samples_host, int n_d, nu_precision prec,
                          const void* depth, const void* var, const void* dll, const void* valid);
// shapes_host: NULL for boxes, else the concatenated template shapes (caller order; copied into ws)
nu_status run_linear(nu_ctx* ctx, nu_factor* F, const double* f, const double* A, int m1, const int64_t* lattice,
                     int64_t n_epochs, const int32_t* dur_samples_host, int n_d, int prec, double* depth,
                     double* var, double* dll, uint8_t* valid, double* null_out, double* ws,
                     const double* shapes_host = nullptr);
size_t linear_ss_ws_bytes(int64_t n, const nu_kernel& k, int n_d, int64_t n_epochs);
nu_status run_linear_ss(nu_ctx* ctx, const double* t, int64_t n, const nu_kernel& k, const double* f, const double* A,
                        int m1, const int64_t* lattice, int64_t n_epochs, const int32_t* dur_samples_host, int n_d,
                        const double* shapes_host, double* depth, double* var, double* dll, uint8_t* valid,
                        double* null_out, double* ws, int64_t** status_dev);
size_t periodic_ws_bytes(int n_d, int64_t n_epochs);
nu_status validate_periodic(nu_ctx* ctx, int n_d, int64_t n_epochs, double dt, int64_t n_p, int log_term_sign);
nu_status run_periodic(nu_ctx* ctx, const double* depth, const double* var, const double* dll, const uint8_t* valid,
                       int n_d, int64_t n_epochs, double dt, const double* periods, int64_t n_p, int log_term_sign,
                       double* q_snr, int64_t* best_phase, int32_t* best_dur, double* best_depth, double* best_sigma,
                       double* best_lnp, int64_t* best_period_index, double* ws);
nu_status validate_theta(nu_ctx* ctx, const nu_sho* theta);

// launchers (*.hip)
hipError_t launch_kbuild(hipStream_t s, const double* t, int64_t n, int64_t np, const nu_sho* th_dev, double* K);
hipError_t launch_kbuild_terms(hipStream_t s, const double* t, int64_t n, int64_t np, const nu_kernel* k_dev,
                               double* K);
nu_status validate_kernel(nu_ctx* ctx, const nu_kernel* k);
hipError_t launch_gemm(hipStream_t s, const GemmProblem* dprobs, int nprob, int total_tiles, int kind, int tile_m,
                       int tile_n, hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
hipError_t launch_potrf_diag(hipStream_t s, const PotrfJob* jobs, int njobs);
hipError_t launch_copy_i64(hipStream_t s, const int64_t* src, int64_t* dst);
hipError_t launch_fill_invalid_cells(hipStream_t s, int64_t count, double* depth, double* var, double* dll,
                                     uint8_t* valid);
hipError_t launch_fill_no_event(hipStream_t s, int64_t n_p, double* q_snr, int64_t* best_phase, int32_t* best_dur,
                                double* best_depth, double* best_sigma, double* best_lnp, int64_t* best_period);
hipError_t launch_fill_i64(hipStream_t s, int64_t* p, int64_t v);
hipError_t launch_cvt_f64_f32(hipStream_t s, const double* src, float* dst, int64_t np, int diag_only, int cb0,
                              int cb1);
hipError_t launch_cvt_f32_f64(hipStream_t s, const float* src, double* dst, int64_t np);
hipError_t launch_band_copy(hipStream_t s, double* X, int64_t np, double* band, int w, int to_band);
hipError_t launch_logdet_reduce(hipStream_t s, const double* parts, int nparts, double* out);

hipError_t launch_pack_v(hipStream_t s, const double* A, int m1, const double* f, int64_t n, double* V);
hipError_t launch_rows_matvec(hipStream_t s, const double* M, int64_t ldm, int64_t n, int64_t np, const double* V,
                              int nv, double* partial, int cw, int nchunks, const double* base, double alpha,
                              double* out);
// lattice_ok: device flag from launch_lattice_check (NULL: not checked)
hipError_t launch_null_solve(hipStream_t s, double* Y, int64_t n, int m1, const double* logdet,
                             const int* lattice_ok, NullFit* nf, double* null_out);
hipError_t launch_lattice_check(hipStream_t s, const int64_t* lattice, int64_t n, int64_t n_epochs, int* ok);
hipError_t launch_cols_matvec(hipStream_t s, const double* M, int64_t ldm, int64_t n, int64_t np, const double* W,
                              int nv, double* partial, int rowchunk, int nchunks, const double* base, double alpha,
                              double* out);
hipError_t launch_slot_count(hipStream_t s, const int64_t* lattice, int64_t n, int64_t n_epochs, int32_t* T);
hipError_t launch_q_partial(hipStream_t s, const double* X, int64_t ldx, int64_t n, const int64_t* lattice,
                            const int32_t* T, int64_t n_epochs, const int32_t* dur_sorted, int n_d, int dmax,
                            int rowchunk, int nchunks, double* qpart);
// shapes: NULL for boxes, else the concatenated template shapes on the device (caller order)
hipError_t launch_cell_epilogue(hipStream_t s, const double* qpart, int nchunks, const int64_t* lattice,
                                const int32_t* T, int64_t n, int64_t n_epochs, const int32_t* dur, int n_d,
                                const double* Z, int m1, const NullFit* nf, double* depth, double* var, double* dll,
                                uint8_t* valid, const double* shapes = nullptr);
// q of template cells from the rows of X (shapes on the device, caller order; dur_sorted as for q_partial)
hipError_t launch_q_template(hipStream_t s, const double* X, int64_t ldx, int64_t n, const int64_t* lattice,
                             const int32_t* T, int64_t n_epochs, const int32_t* dur_sorted, const int32_t* dur,
                             int n_d, const double* shapes, int dmax, int rowchunk, int nchunks, double* qpart);
hipError_t launch_fold(hipStream_t s, const double* depth, const double* var, const double* dll,
                       const uint8_t* valid, int n_d, int64_t n_epochs, double dt, const double* periods, int64_t n_p,
                       int sign, double* q_snr, int64_t* best_phase, int32_t* best_dur, double* best_depth,
                       double* best_sigma, double* best_lnp, double* packed);
size_t fold_workspace_doubles(int n_d, int64_t n_epochs);
// The fixed device array of the allocation-free periodic search (fold.hip):
// its size, and its address on `device` (looked up once per device, with that
// device current; the same pointer afterwards).
constexpr size_t FOLD_SCRATCH_DOUBLES = NU_PERIODIC_SCRATCH_BYTES / sizeof(double);
hipError_t fold_scratch_ptr(int device, double** out);
size_t fold_segments_workspace_doubles(int n_d, const int64_t* len, int n_seg);
hipError_t launch_fold_segments(hipStream_t s, const double* depth, const double* var, const double* dll,
                                const uint8_t* valid, int n_d, int n_seg, const int64_t* seg_len,
                                const int64_t* seg_off, double dt, const double* periods, int64_t n_p, int sign,
                                double* q_snr, int64_t* best_phase, int32_t* best_dur, double* best_depth,
                                double* best_sigma, double* best_lnp, double* packed);
hipError_t launch_mask_transit(hipStream_t s, double* depth, double* var, double* dll, uint8_t* valid, int n_d,
                               int64_t n_t, double p, int64_t m, int h);
hipError_t launch_best_period(hipStream_t s, const double* q_snr, int64_t n_p, int64_t* out);

// State-space linear search (statespace.hip): the phases after the step
// coefficients, each one launch on the stream.
enum SsPhase {
  SS_RICCATI = 0, SS_FORWARD, SS_BACKWARD, SS_BOX, SS_TEMPLATE,
  // the chunked (parallel-in-time) forms of the first three
  SS_PAR_RICCATI, SS_PAR_FORWARD, SS_PAR_BACKWARD
};
struct SsArgs {
  int n_sho = 0, n_exp = 0;
  int64_t n = 0;
  nu_kernel kernel{};                   // by value: a kernel argument of the first phase
  const double* step = nullptr;         // [n - 1][7 n_sho + 2 n_exp]
  double* gain = nullptr;               // [n][1 + J]
  double* Gm = nullptr;                 // [n + 1][J][J]
  double* logdet = nullptr;             // 1 (NaN on failure)
  int64_t* status = nullptr;            // first failing sample or -1
  const double* V = nullptr;            // [n][YCOLS]
  double* Y = nullptr;                  // [n][YCOLS]
  double* Z = nullptr;                  // [n][YCOLS]
  int nv = 0;
  const int64_t* lattice = nullptr;
  const int32_t* slot_count = nullptr;
  int64_t n_epochs = 0;
  const int32_t* dur_sorted = nullptr;  // host [2 n_d]: ascending durations, then their caller indices
  const int32_t* dur = nullptr;         // host [n_d], caller order
  int n_d = 0;
  const double* shapes = nullptr;       // device, concatenated template shapes (caller order), or NULL: boxes
  double* qbox = nullptr;               // [n_d][n_epochs]
  double* chunk = nullptr;              // chunked path: ss_chunk_ws_doubles(n, J) doubles
};
// the chunked path: its workspace, and whether it applies to a kernel (at most
// 6 states, sigma_w > 0, every term of positive variance)
size_t ss_chunk_ws_doubles(int64_t n, int J);
bool ss_chunked_applies(const nu_kernel& k);
hipError_t launch_ss_step(hipStream_t s, const double* t, int64_t n, const nu_kernel& k, double* step);
hipError_t launch_ss(int phase, hipStream_t s, const SsArgs& A);

// ---------------------------------------------------------------------------
// Batched stages: one launch runs a stage of the search for every curve of a
// batch. Each curve's record holds its sizes and the device pointers of its
// factor, search workspace, inputs and outputs; a launch's workgroups are
// numbered curve after curve, and begin[c] (per stage kind) is the first
// workgroup of curve c (begin[n_curves] the total), so a workgroup finds its
// curve by binary search and its own index within that curve's grid.
struct CurveJob {
  // factor
  const double* t;
  const nu_sho* theta;
  double *L, *X;
  float *L32, *X32;
  double* bandX;
  double* parts;    // per-block ln|L_kk| terms
  double* logdet;   // then the status word (int64) right after it
  int64_t* status;
  NullFit* nf;
  int64_t n, np;
  int nblk, xchunks, rchunks, qchunks;
  // linear search: inputs, workspace (inside the factor's T region), outputs
  const double* f;
  const double* A;  // n x m1 column-major, or null
  const int64_t* lattice;
  int64_t n_epochs;
  double *V, *Y, *R, *Z, *Rz, *xpart, *qpart;
  int32_t* slot_count;
  int* lattice_ok;
  double *depth, *var, *dll;
  uint8_t* valid;
  double* null_out;  // 3 doubles or null
  // periodic search
  double* packed;
  double dt;
  double *q_snr, *best_depth, *best_sigma, *best_lnp;
  int64_t* best_phase;
  int32_t* best_dur;
  int64_t* best_index;  // or null
  // the caller's index of the curve (where its status and ln|K| are collected)
  int64_t curve;
};

// stage kinds (rows of the begin table)
enum BatchStage {
  BS_INIT = 0, BS_KBUILD, BS_LOGDET, BS_CVT_L, BS_CVT_XD, BS_CVT_BACK, BS_BAND, BS_CHECK, BS_PACKV, BS_ROWS,
  BS_ROWS_RED, BS_NULL, BS_COLS, BS_COLS_RED, BS_SLOTS, BS_QPART, BS_EPI, BS_FOLD_PACK, BS_BEST, BS_COUNT
};
// workgroups of stage `stage` for one curve (n_d durations, band width w, n_p periods)
int64_t batch_stage_blocks(int stage, const CurveJob& J, int n_d, int band_w);
// doubles of one curve's linear-search workspace (the packed fold grid is kept
// apart, so a wave's fold can run while the next wave reuses the workspace)
size_t batch_search_ws_doubles(int64_t n, int n_d, int64_t n_epochs);
// carve a curve's linear-search workspace from ws
void batch_carve_search_ws(CurveJob& J, double* ws, int n_d);

// GEMV passes of the linear search: the matrix (X or L), the vector panel
// read, the base added and the panel written (fields of CurveJob)
enum PanelSel { PS_NONE = -1, PS_V = 0, PS_Y, PS_R, PS_Z, PS_RZ };
enum MatSel { MS_X = 0, MS_L = 1 };

hipError_t launch_batch_init(hipStream_t s, const CurveJob* jobs, int n_curves);
// status_out[J.curve] = status, logdet_out[J.curve] = ln|K| of every curve of the launch
hipError_t launch_batch_collect(hipStream_t s, const CurveJob* jobs, int n_curves, int64_t* status_out,
                                double* logdet_out);
hipError_t launch_batch_kbuild(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total);
hipError_t launch_batch_logdet(hipStream_t s, const CurveJob* jobs, int n_curves);
hipError_t launch_batch_cvt_l(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total);
hipError_t launch_batch_cvt_xd(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total);
hipError_t launch_batch_cvt_back(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total);
hipError_t launch_batch_band_copy(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total,
                                  int w, int to_band);
hipError_t launch_batch_lattice_check(hipStream_t s, const CurveJob* jobs, int n_curves);
hipError_t launch_batch_pack_v(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total,
                               int m1);
hipError_t launch_batch_rows(hipStream_t s, const CurveJob* jobs, const int* begin, const int* begin_red,
                             int n_curves, int total, int total_red, int nv, int mat, int vin, int base, double alpha,
                             int out);
hipError_t launch_batch_null(hipStream_t s, const CurveJob* jobs, int n_curves, int m1);
hipError_t launch_batch_cols(hipStream_t s, const CurveJob* jobs, const int* begin, const int* begin_red,
                             int n_curves, int total, int total_red, int nv, int mat, int win, int base, double alpha,
                             int out);
hipError_t launch_batch_slot_count(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total);
hipError_t launch_batch_q_partial(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total,
                                  const int32_t* dur_sorted, int n_d, int dmax);
hipError_t launch_batch_epilogue(hipStream_t s, const CurveJob* jobs, const int* begin, int n_curves, int total,
                                 const int32_t* dur, int n_d, int m1);
hipError_t launch_batch_fold(hipStream_t s, const CurveJob* jobs, const int* begin_pack, int n_curves,
                             int total_pack, int n_d, const double* periods, int64_t n_p, int sign);
hipError_t launch_batch_best(hipStream_t s, const CurveJob* jobs, int n_curves, int64_t n_p,
                             const int64_t* status_out);

}  // namespace nu
