// C ABI of the transit-search library: argument validation, context and
// factor objects, launch schedules of the blocked factorisation and of the
// triangular inverse, kernel timing. No exception crosses the boundary.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "internal.hpp"

using namespace nu;

namespace nu {

nu_status set_error(nu_ctx* ctx, nu_status st, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return st;
}

nu_status check_hip(nu_ctx* ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return NU_OK;
  return set_error(ctx, e == hipErrorOutOfMemory ? NU_ERR_OOM : NU_ERR_DEVICE,
                   std::string(what) + ": " + hipGetErrorString(e));
}

void* ctx_workspace(nu_ctx* ctx, size_t bytes, nu_status* st) {
  *st = NU_OK;
  if (bytes <= ctx->ws_bytes) return ctx->ws;
  // the old buffer may still be in use by enqueued work
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess && ctx->ws) e = hipFree(ctx->ws);
  ctx->ws = nullptr;
  ctx->ws_bytes = 0;
  if (e == hipSuccess) e = hipMalloc(&ctx->ws, bytes);
  if (e != hipSuccess) {
    *st = check_hip(ctx, e, "workspace allocation");
    ctx->ws = nullptr;
    return nullptr;
  }
  ctx->ws_bytes = bytes;
  return ctx->ws;
}

void timing_begin(nu_ctx* ctx, hipStream_t s, hipEvent_t* start) {
  *start = nullptr;
  if (!ctx->timing) return;
  if (ctx->free_events.empty()) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return;
    ctx->free_events.push_back(ev);
  }
  *start = ctx->free_events.back();
  ctx->free_events.pop_back();
  hipEventRecord(*start, s);
}

void timing_end(nu_ctx* ctx, hipStream_t s, const char* name, hipEvent_t start, double work) {
  if (!ctx->timing || !start) return;
  hipEvent_t stop;
  if (ctx->free_events.empty()) {
    if (hipEventCreate(&stop) != hipSuccess) return;
  } else {
    stop = ctx->free_events.back();
    ctx->free_events.pop_back();
  }
  hipEventRecord(stop, s);
  ctx->pending.push_back({name, start, stop, work});
}

}  // namespace nu

namespace {

void resolve_timing(nu_ctx* ctx) {
  if (ctx->pending.empty()) return;
  hipStreamSynchronize(ctx->stream);
  for (auto& p : ctx->pending) {
    float ms = 0.0f;
    hipEventElapsedTime(&ms, p.start, p.stop);
    auto it = ctx->timings.find(p.name);
    if (it == ctx->timings.end()) {
      ctx->timing_names.push_back(p.name);
      it = ctx->timings.emplace(p.name, nu_timing_slot{}).first;
    }
    it->second.launches += 1;
    it->second.ms += ms;
    it->second.work += p.work;
    ctx->free_events.push_back(p.start);
    ctx->free_events.push_back(p.stop);
  }
  ctx->pending.clear();
}

struct Timed {
  nu_ctx* ctx;
  const char* name;
  double work;
  hipEvent_t start;
  Timed(nu_ctx* c, const char* n, double w) : ctx(c), name(n), work(w) { timing_begin(c, c->stream, &start); }
  ~Timed() { timing_end(ctx, ctx->stream, name, start, work); }
};

int tiles_of(const GemmProblem& g, int tile) {
  const int tm = g.M / tile, tn = g.N / tile;
  return (g.flags & G_C_LOWER_TILES) ? tm * (tm + 1) / 2 : tm * tn;
}

// Launches with fewer 128 x 128 tiles than one round of workgroups on the chip
// (256 CUs x 2) use 64 x 64 tiles instead: four times the workgroups, each a
// quarter of the work.
constexpr int SMALL_LAUNCH_TILES = 512;

// useful flops of a problem (zeros of triangular operands not counted)
double useful_flops(const GemmProblem& g) {
  const double M = g.M, N = g.N, K = g.K;
  if (g.flags & G_C_LOWER_TILES) return M * (M + 1) * K;          // 2 K per lower element
  if (g.flags & (G_B_LOWER | G_B_UPPER)) return M * N * (N + 1);  // triangular N x N right factor
  if (g.flags & G_A_LOWER) return N * M * (M + 1);                // triangular M x M left factor
  if ((g.flags & G_BT) && g.K == TB && g.N == TB) return M * N * (K + 1);  // panel: triangular X_kk^T
  return 2.0 * M * N * K;
}

// append one launch's problems, numbering tiles from 0 within the launch
Range add_launch(std::vector<GemmProblem>& sched, std::vector<GemmProblem> probs) {
  Range r;
  r.first = (int)sched.size();
  r.count = (int)probs.size();
  int big = 0;
  for (auto& p : probs) big += tiles_of(p, TB);
  r.tile = big < SMALL_LAUNCH_TILES ? 64 : TB;
  int t = 0;
  for (auto& p : probs) {
    p.tiles_n = p.N / r.tile;
    p.tile_begin = t;
    p.tile_count = tiles_of(p, r.tile);
    t += p.tile_count;
    r.flops += useful_flops(p);
    sched.push_back(p);
  }
  r.tiles = t;
  return r;
}

// element (row, col) of a row-major matrix with leading dimension ld and element size es
inline const void* at(const void* base, int64_t row, int64_t col, int64_t ld, size_t es) {
  return static_cast<const char*>(base) + (size_t)(row * ld + col) * es;
}
inline void* at(void* base, int64_t row, int64_t col, int64_t ld, size_t es) {
  return static_cast<char*>(base) + (size_t)(row * ld + col) * es;
}

GemmProblem prob(const void* A, int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, int M, int N, int K,
                 int flags, double alpha, double beta) {
  GemmProblem g{};
  g.A = A;
  g.B = B;
  g.C = C;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.M = M;
  g.N = N;
  g.K = K;
  g.flags = flags;
  g.alpha = alpha;
  g.beta = beta;
  return g;
}

// Outer panel width of the Cholesky, in TB blocks: each panel is factored
// block by block (diagonal block, its column, the update of the panel's
// remaining columns), then the trailing matrix gets one update of depth
// PANEL * TB.
constexpr int PANEL = 4;

void plan_cholesky(nu_factor* F) {
  const int64_t np = F->np;
  const int nblk = (int)(np / TB);
  F->panel.assign(nblk, Range());
  F->pupd.assign(nblk, Range());
  F->trail.assign(nblk, Range());
  const size_t es = sizeof(double);
  for (int p0 = 0; p0 < nblk; p0 += PANEL) {
    const int pw = std::min(PANEL, nblk - p0);
    for (int k = p0; k < p0 + pw; ++k) {
      const int64_t off = (int64_t)k * TB;
      const int rest = (int)(np - off - TB);
      if (rest <= 0) continue;
      void* col = at(F->L, off + TB, off, np, es);  // rows below the diagonal block, block column k
      const void* xkk = at(F->X, off, off, np, es);
      F->panel[k] = add_launch(F->sched, {prob(col, np, xkk, np, col, np, rest, TB, TB, G_BT, 1.0, 0.0)});
      const int inner = (p0 + pw - k - 1) * TB;  // columns of this panel right of block k
      if (inner > 0)
        F->pupd[k] = add_launch(F->sched, {prob(col, np, col, np, at(col, 0, TB, np, es), np, rest, inner, TB, G_BT,
                                                -1.0, 1.0)});
    }
    const int64_t t0 = (int64_t)(p0 + pw) * TB;
    const int rest2 = (int)(np - t0);
    if (rest2 > 0) {
      const void* pan = at(F->L, t0, (int64_t)p0 * TB, np, es);  // trailing rows, panel columns
      F->trail[p0] = add_launch(F->sched, {prob(pan, np, pan, np, at(F->L, t0, t0, np, es), np, rest2, rest2,
                                                pw * TB, G_BT | G_C_LOWER_TILES, -1.0, 1.0)});
    }
  }
}

struct Node {
  int a, mid, b;
};

void build_tree(int a, int b, int depth, std::vector<std::vector<Node>>& levels) {
  if (b - a < 2) return;
  const int mid = a + (b - a + 1) / 2;
  if ((int)levels.size() <= depth) levels.resize(depth + 1);
  levels[depth].push_back({a, mid, b});
  build_tree(a, mid, depth + 1, levels);
  build_tree(mid, b, depth + 1, levels);
}

// Triangular inverse X = L^-1, bottom-up over a binary tree of the TB blocks:
// for the node [[A, 0], [L21, C]], T = L21 X_A then X21 = -X_C T. Leaves are
// the diagonal-block inverses. Returns the workspace (elements) T needs.
size_t plan_inverse(int64_t np, const void* L, void* X, void* T, size_t es, std::vector<GemmProblem>& sched,
                    std::vector<Range>& t1, std::vector<Range>& t2) {
  const int nblk = (int)(np / TB);
  std::vector<std::vector<Node>> levels;
  build_tree(0, nblk, 0, levels);
  size_t tmax = 0;
  t1.clear();
  t2.clear();
  for (int d = (int)levels.size() - 1; d >= 0; --d) {
    std::vector<GemmProblem> p1, p2;
    size_t off_t = 0;
    for (const Node& nd : levels[d]) {
      const int64_t a0 = (int64_t)nd.a * TB, m0 = (int64_t)nd.mid * TB;
      const int na = (nd.mid - nd.a) * TB, nc = (nd.b - nd.mid) * TB;
      void* Tn = at(T, 0, (int64_t)off_t, 0, es);
      p1.push_back(prob(at(L, m0, a0, np, es), np, at(X, a0, a0, np, es), np, Tn, na, nc, na, na, G_B_LOWER, 1.0,
                        0.0));
      p2.push_back(prob(at(X, m0, m0, np, es), np, Tn, na, at(X, m0, a0, np, es), np, nc, na, nc, G_A_LOWER, -1.0,
                        0.0));
      off_t += (size_t)na * nc;
    }
    tmax = std::max(tmax, off_t);
    t1.push_back(add_launch(sched, p1));
    t2.push_back(add_launch(sched, p2));
  }
  return tmax;
}

// One Newton step X1 = 2 X - X (L X) on the blocks within BAND_W of the
// diagonal, FP64: P(I, J) = sum_{K=J..I} L(I, K) X(K, J) for I - J <= w, stored
// by column block (the blocks P(J..J+w, J) stacked), then
// X1(I, J) = 2 X(I, J) - sum_{K=J..I} X(I, K) P(K, J) for 1 <= I - J <= w, into
// the band buffer (which holds X(I, J) on entry).
void plan_band(nu_factor* F) {
  const int64_t np = F->np;
  const int nblk = (int)(np / TB), w = BAND_W;
  const size_t es = sizeof(double);
  const int64_t bs = (int64_t)TB * TB;
  std::vector<GemmProblem> pp, px;
  for (int I = 0; I < nblk; ++I)
    for (int d = 0; d <= w && d <= I; ++d) {
      const int J = I - d;
      pp.push_back(prob(at(F->L, (int64_t)I * TB, (int64_t)J * TB, np, es), np,
                        at(F->X, (int64_t)J * TB, (int64_t)J * TB, np, es), np,
                        F->bandP + ((int64_t)J * (w + 1) + d) * bs, TB, TB, TB, (d + 1) * TB, 0, 1.0, 0.0));
      if (d >= 1)
        px.push_back(prob(at(F->X, (int64_t)I * TB, (int64_t)J * TB, np, es), np,
                          F->bandP + (int64_t)J * (w + 1) * bs, TB, F->bandX + ((int64_t)I * (w + 1) + d) * bs, TB,
                          TB, TB, (d + 1) * TB, 0, -1.0, 2.0));
    }
  F->bandp.assign(1, add_launch(F->sched32, pp));
  F->bandx.assign(1, px.empty() ? Range() : add_launch(F->sched32, px));
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

nu_status launch_range(nu_ctx* ctx, const GemmProblem* dprobs, const Range& r, const char* name, int f32 = 0) {
  if (r.tiles == 0) return NU_OK;
  Timed tm(ctx, name, r.flops);
  return check_hip(ctx, launch_gemm(ctx->stream, dprobs + r.first, r.count, r.tiles, f32, r.tile), name);
}

nu_status upload(nu_ctx* ctx, GemmProblem** dst, const std::vector<GemmProblem>& src) {
  nu_status st = check_hip(ctx, hipMalloc(dst, std::max<size_t>(src.size(), 1) * sizeof(GemmProblem)),
                           "alloc schedule");
  if (st != NU_OK || src.empty()) return st;
  return check_hip(ctx, hipMemcpy(*dst, src.data(), src.size() * sizeof(GemmProblem), hipMemcpyHostToDevice),
                   "upload schedule");
}

nu_status validate_theta(nu_ctx* ctx, const nu_sho* theta) {
  const nu_sho& th = *theta;
  if (!(std::isfinite(th.amp) && th.amp >= 0.0) || !finite_pos(th.omega) || !finite_pos(th.q) ||
      !(std::isfinite(th.sigma_w) && th.sigma_w >= 0.0))
    return set_error(ctx, NU_ERR_ARG, "gp_factor: need finite amp >= 0, omega > 0, q > 0, sigma_w >= 0");
  return NU_OK;
}

// K build, blocked Cholesky, ln|K|, status; synchronises once.
nu_status factor_compute(nu_ctx* ctx, nu_factor* F, const double* t, const nu_sho& th, double* logdet_host,
                         int64_t* fail_pivot_host) {
  const int64_t n = F->n, np = F->np;
  const int nblk = (int)(np / TB);
  double* parts = F->small;
  double* logdet_dev = F->small + nblk;
  int64_t* status = reinterpret_cast<int64_t*>(F->small + nblk + 1);
  F->inverse_kind = 0;
  nu_status st = check_hip(ctx, launch_fill_i64(ctx->stream, status, -1), "status init");
  if (st != NU_OK) return st;
  {
    Timed tm(ctx, "kbuild", (double)n * (double)(n + 1) / 2.0);
    st = check_hip(ctx, launch_kbuild(ctx->stream, t, n, np, th, F->L), "kbuild");
  }
  // Blocked right-looking Cholesky, two levels: within a panel of PANEL
  // blocks, diagonal block -> its column (times the diagonal block's inverse)
  // -> update of the panel's remaining columns; after the panel, one trailing
  // update of depth PANEL * TB on the whole chip.
  for (int k = 0; st == NU_OK && k < nblk; ++k) {
    {
      Timed tm(ctx, "potrf_diag", (double)TB * TB * TB * 2.0 / 3.0);
      st = check_hip(ctx, launch_potrf_diag(ctx->stream, F->L, np, (int64_t)k * TB, k, parts, status, F->X, np),
                     "potrf_diag");
    }
    if (st == NU_OK) st = launch_range(ctx, F->probs, F->panel[k], "gemm_f64:panel");
    if (st == NU_OK) st = launch_range(ctx, F->probs, F->pupd[k], "gemm_f64:panel_update");
    if (st == NU_OK && (k + 1) % PANEL == 0)
      st = launch_range(ctx, F->probs, F->trail[k + 1 - PANEL], "gemm_f64:trailing");
  }
  if (st == NU_OK) st = check_hip(ctx, launch_logdet_reduce(ctx->stream, parts, nblk, logdet_dev), "logdet");
  if (st != NU_OK) return st;
  struct {
    double logdet;
    int64_t status;
  } hostv{};
  st = check_hip(ctx, hipMemcpyAsync(&hostv.logdet, logdet_dev, sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
                 "read logdet");
  if (st == NU_OK)
    st = check_hip(ctx, hipMemcpyAsync(&hostv.status, status, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream),
                   "read status");
  if (st == NU_OK) st = check_hip(ctx, hipStreamSynchronize(ctx->stream), "gp_factor sync");
  if (st != NU_OK) return st;
  if (hostv.status >= 0) {
    if (fail_pivot_host) *fail_pivot_host = hostv.status;
    return set_error(ctx, NU_ERR_NOT_PD,
                     "gp_factor: covariance not positive definite at pivot " + std::to_string(hostv.status));
  }
  F->logdet = hostv.logdet;
  if (logdet_host) *logdet_host = hostv.logdet;
  return NU_OK;
}

// allocations and schedules of the reduced-precision inverse (first use only)
nu_status ensure_mixed(nu_ctx* ctx, nu_factor* F) {
  if (F->probs32) return NU_OK;
  const int64_t np = F->np;
  const int nblk = (int)(np / TB);
  const size_t band_elems = (size_t)nblk * (BAND_W + 1) * TB * TB;
  nu_status st = check_hip(ctx, hipMalloc(&F->L32, (size_t)np * np * sizeof(float)), "alloc L32");
  if (st == NU_OK) st = check_hip(ctx, hipMalloc(&F->X32, (size_t)np * np * sizeof(float)), "alloc X32");
  if (st == NU_OK) st = check_hip(ctx, hipMalloc(&F->bandP, band_elems * sizeof(double)), "alloc band");
  if (st == NU_OK) st = check_hip(ctx, hipMalloc(&F->bandX, band_elems * sizeof(double)), "alloc band");
  if (st != NU_OK) return st;
  F->sched32.clear();
  // the FP32 level products reuse the FP64 T workspace (the same element count fits)
  plan_inverse(np, F->L32, F->X32, F->T, sizeof(float), F->sched32, F->t1_32, F->t2_32);
  plan_band(F);
  return upload(ctx, &F->probs32, F->sched32);
}

nu_status inverse_fp64(nu_ctx* ctx, nu_factor* F) {
  nu_status st = NU_OK;
  for (size_t l = 0; st == NU_OK && l < F->t1.size(); ++l) {
    st = launch_range(ctx, F->probs, F->t1[l], "gemm_f64:inverse");
    if (st == NU_OK) st = launch_range(ctx, F->probs, F->t2[l], "gemm_f64:inverse");
  }
  return st;
}

nu_status inverse_mixed(nu_ctx* ctx, nu_factor* F) {
  nu_status st = ensure_mixed(ctx, F);
  if (st != NU_OK) return st;
  const int64_t np = F->np;
  {
    Timed tm(ctx, "convert", 0.0);
    st = check_hip(ctx, launch_cvt_f64_f32(ctx->stream, F->L, F->L32, np, 0), "convert L");
    if (st == NU_OK) st = check_hip(ctx, launch_cvt_f64_f32(ctx->stream, F->X, F->X32, np, 1), "convert X diag");
  }
  for (size_t l = 0; st == NU_OK && l < F->t1_32.size(); ++l) {
    st = launch_range(ctx, F->probs32, F->t1_32[l], "gemm_f32:inverse", 1);
    if (st == NU_OK) st = launch_range(ctx, F->probs32, F->t2_32[l], "gemm_f32:inverse", 1);
  }
  if (st == NU_OK) {
    Timed tm(ctx, "convert", 0.0);
    st = check_hip(ctx, launch_cvt_f32_f64(ctx->stream, F->X32, F->X, np), "convert X");
  }
  // one Newton step on the blocks within BAND_W of the diagonal
  if (st == NU_OK) st = check_hip(ctx, launch_band_copy(ctx->stream, F->X, np, F->bandX, BAND_W, 1), "band copy");
  if (st == NU_OK) st = launch_range(ctx, F->probs32, F->bandp[0], "gemm_f64:band");
  if (st == NU_OK) st = launch_range(ctx, F->probs32, F->bandx[0], "gemm_f64:band");
  if (st == NU_OK) st = check_hip(ctx, launch_band_copy(ctx->stream, F->X, np, F->bandX, BAND_W, 0), "band copy");
  return st;
}

}  // namespace

// ===========================================================================
extern "C" {

nu_status nu_ctx_create(int device, void* stream, nu_ctx** out) {
  if (!out) return NU_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return NU_ERR_DEVICE;
  if (device < 0 || device >= ndev) return NU_ERR_ARG;
  nu_ctx* ctx = new (std::nothrow) nu_ctx();
  if (!ctx) return NU_ERR_OOM;
  ctx->device = device;
  ctx->stream = (hipStream_t)stream;
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return NU_ERR_DEVICE;
  }
  *out = ctx;
  return NU_OK;
}

void nu_ctx_destroy(nu_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  if (ctx->ws) hipFree(ctx->ws);
  for (auto& p : ctx->pending) {
    hipEventDestroy(p.start);
    hipEventDestroy(p.stop);
  }
  for (auto e : ctx->free_events) hipEventDestroy(e);
  delete ctx;
}

nu_status nu_ctx_set_stream(nu_ctx* ctx, void* stream) {
  if (!ctx) return NU_ERR_ARG;
  ctx->stream = (hipStream_t)stream;
  return NU_OK;
}

const char* nu_ctx_last_error(const nu_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

nu_status nu_ctx_enable_timing(nu_ctx* ctx, int enable) {
  if (!ctx) return NU_ERR_ARG;
  ctx->timing = enable != 0;
  return NU_OK;
}

nu_status nu_ctx_timing_reset(nu_ctx* ctx) {
  if (!ctx) return NU_ERR_ARG;
  resolve_timing(ctx);
  ctx->timings.clear();
  ctx->timing_names.clear();
  return NU_OK;
}

int nu_ctx_timing_count(nu_ctx* ctx) {
  if (!ctx) return 0;
  resolve_timing(ctx);
  return (int)ctx->timing_names.size();
}

nu_status nu_ctx_timing_entry(nu_ctx* ctx, int index, const char** name_host, int64_t* launches_host,
                              double* total_ms_host, double* work_units_host) {
  if (!ctx) return NU_ERR_ARG;
  resolve_timing(ctx);
  if (index < 0 || index >= (int)ctx->timing_names.size())
    return set_error(ctx, NU_ERR_ARG, "timing index out of range");
  const std::string& nm = ctx->timing_names[index];
  const nu_timing_slot& s = ctx->timings[nm];
  if (name_host) *name_host = nm.c_str();
  if (launches_host) *launches_host = s.launches;
  if (total_ms_host) *total_ms_host = s.ms;
  if (work_units_host) *work_units_host = s.work;
  return NU_OK;
}

// ---------------------------------------------------------------------------
nu_status nu_gp_factor(nu_ctx* ctx, const double* t, int64_t n, const nu_sho* theta, nu_factor** out,
                       double* logdet_host, int64_t* fail_pivot_host) {
  if (!ctx) return NU_ERR_ARG;
  if (!t || !theta || !out) return set_error(ctx, NU_ERR_ARG, "gp_factor: null argument");
  *out = nullptr;
  if (fail_pivot_host) *fail_pivot_host = -1;
  if (n < 1 || n > (int64_t)1 << 17) return set_error(ctx, NU_ERR_ARG, "gp_factor: n must be in [1, 131072]");
  nu_status st = validate_theta(ctx, theta);
  if (st != NU_OK) return st;
  st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;

  nu_factor* F = new (std::nothrow) nu_factor();
  if (!F) return set_error(ctx, NU_ERR_OOM, "gp_factor: host allocation");
  F->device = ctx->device;
  F->n = n;
  F->np = round_up(n, TB);
  const int64_t np = F->np;
  const int nblk = (int)(np / TB);
  auto fail = [&](nu_status s) {
    nu_factor_destroy(F);
    return s;
  };
  st = check_hip(ctx, hipMalloc(&F->L, (size_t)np * np * sizeof(double)), "alloc L");
  if (st == NU_OK) st = check_hip(ctx, hipMalloc(&F->X, (size_t)np * np * sizeof(double)), "alloc X");
  if (st != NU_OK) return fail(st);
  {
    std::vector<GemmProblem> tmp;
    std::vector<Range> a, b;
    F->t_elems = std::max<size_t>(plan_inverse(np, F->L, F->X, nullptr, sizeof(double), tmp, a, b), 1);
  }
  st = check_hip(ctx, hipMalloc(&F->T, F->t_elems * sizeof(double)), "alloc T");
  if (st == NU_OK) st = check_hip(ctx, hipMalloc(&F->small, (size_t)(nblk + 4) * sizeof(double)), "alloc small");
  if (st == NU_OK) st = check_hip(ctx, hipMalloc(&F->nullfit, sizeof(NullFit)), "alloc nullfit");
  if (st != NU_OK) return fail(st);
  plan_cholesky(F);
  plan_inverse(np, F->L, F->X, F->T, sizeof(double), F->sched, F->t1, F->t2);
  st = upload(ctx, &F->probs, F->sched);
  if (st != NU_OK) return fail(st);
  st = factor_compute(ctx, F, t, *theta, logdet_host, fail_pivot_host);
  if (st != NU_OK) return fail(st);
  *out = F;
  return NU_OK;
}

nu_status nu_gp_factor_into(nu_ctx* ctx, nu_factor* F, const double* t, int64_t n, const nu_sho* theta,
                            double* logdet_host, int64_t* fail_pivot_host) {
  if (!ctx) return NU_ERR_ARG;
  if (!F || !t || !theta) return set_error(ctx, NU_ERR_ARG, "gp_factor_into: null argument");
  if (fail_pivot_host) *fail_pivot_host = -1;
  if (F->device != ctx->device) return set_error(ctx, NU_ERR_ARG, "gp_factor_into: factor on another device");
  if (n != F->n) return set_error(ctx, NU_ERR_ARG, "gp_factor_into: n differs from the factor's");
  nu_status st = validate_theta(ctx, theta);
  if (st != NU_OK) return st;
  st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  return factor_compute(ctx, F, t, *theta, logdet_host, fail_pivot_host);
}

void nu_factor_destroy(nu_factor* F) {
  if (!F) return;
  hipSetDevice(F->device);
  hipDeviceSynchronize();
  void* bufs[] = {F->L, F->X, F->T, F->small, F->nullfit, F->probs, F->L32, F->X32, F->bandP, F->bandX, F->probs32};
  for (void* b : bufs)
    if (b) hipFree(b);
  delete F;
}

int64_t nu_factor_n(const nu_factor* F) { return F ? F->n : -1; }

// ---------------------------------------------------------------------------
nu_status nu_linear_search(nu_ctx* ctx, nu_factor* F, const double* f, const double* A, int m1,
                           const int64_t* lattice, int64_t n_epochs, const int32_t* dur_samples_host, int n_d,
                           nu_precision prec, double* depth, double* var, double* dll, uint8_t* valid,
                           double* null_out) {
  if (!ctx) return NU_ERR_ARG;
  if (!F || !f || !lattice || !dur_samples_host || !depth || !var || !dll || !valid)
    return set_error(ctx, NU_ERR_ARG, "linear_search: null argument");
  if (F->device != ctx->device) return set_error(ctx, NU_ERR_ARG, "linear_search: factor on another device");
  if (m1 < 0 || m1 > MAX_M1) return set_error(ctx, NU_ERR_ARG, "linear_search: m1 must be in [0, 7]");
  if (m1 > 0 && !A) return set_error(ctx, NU_ERR_ARG, "linear_search: A is NULL with m1 > 0");
  if (F->n < m1 + 1) return set_error(ctx, NU_ERR_ARG, "linear_search: need n >= m1 + 1");
  if (n_d < 1 || n_d > MAX_ND) return set_error(ctx, NU_ERR_ARG, "linear_search: n_d must be in [1, 16]");
  if (n_epochs < 1 || n_epochs > ((int64_t)1 << 31))
    return set_error(ctx, NU_ERR_ARG, "linear_search: n_epochs must be in [1, 2^31]");
  if (n_epochs < F->n) return set_error(ctx, NU_ERR_ARG, "linear_search: n_epochs must be >= n (strict lattice)");
  int dmax = 0;
  for (int j = 0; j < n_d; ++j) {
    if (dur_samples_host[j] < 1 || dur_samples_host[j] > MAX_DUR)
      return set_error(ctx, NU_ERR_ARG, "linear_search: durations must be in [1, 1024] slots");
    dmax = std::max(dmax, (int)dur_samples_host[j]);
  }
  if (prec != NU_FP64 && prec != NU_FP32_REFINE)
    return set_error(ctx, NU_ERR_UNSUPPORTED, "linear_search: precision not available in this build");
  nu_status st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  const int64_t n = F->n, np = F->np;
  const bool mixed = prec == NU_FP32_REFINE;

  // triangular inverse X = L^-1 (kept in the factor for further searches)
  const int want = mixed ? 2 : 1;
  if (F->inverse_kind != want) {
    st = mixed ? inverse_mixed(ctx, F) : inverse_fp64(ctx, F);
    if (st != NU_OK) return st;
    F->inverse_kind = want;
  }

  // workspace: V, Y, R, Z, Rz (np x 8), column partials, q partials
  const int xrc = 1024;
  const int xchunks = (int)((n + xrc - 1) / xrc);
  const int qrc = 2048;
  const int qchunks = (int)((n + qrc - 1) / qrc);
  const size_t yz = (size_t)np * YCOLS;
  const size_t need = (5 * yz + (size_t)xchunks * yz + (size_t)qchunks * n_d * n_epochs) * sizeof(double);
  double* ws = (double*)ctx_workspace(ctx, need, &st);
  if (!ws) return st;
  double* V = ws;
  double* Y = V + yz;
  double* R = Y + yz;
  double* Z = R + yz;
  double* Rz = Z + yz;
  double* xpart = Rz + yz;
  double* qpart = xpart + (size_t)xchunks * yz;
  const double* logdet_dev = F->small + (np / TB);
  const int nv = m1 + 1;
  const double gemv_bytes = (double)n * (double)(n + 1) / 2.0 * 8.0;

  st = check_hip(ctx, launch_pack_v(ctx->stream, A, m1, f, n, V), "pack_v");
  if (st != NU_OK) return st;
  {
    // Y = X V, refined once against L when X is the mixed inverse
    Timed tm(ctx, "rows_matvec", gemv_bytes * (mixed ? 3 : 1));
    st = check_hip(ctx, launch_rows_matvec(ctx->stream, F->X, np, n, V, nv, nullptr, 1.0, Y), "rows_matvec");
    if (mixed && st == NU_OK)
      st = check_hip(ctx, launch_rows_matvec(ctx->stream, F->L, np, n, Y, nv, V, -1.0, R), "rows_matvec");
    if (mixed && st == NU_OK)
      st = check_hip(ctx, launch_rows_matvec(ctx->stream, F->X, np, n, R, nv, Y, 1.0, Y), "rows_matvec");
  }
  if (st != NU_OK) return st;
  {
    Timed tm(ctx, "null_solve", 0.0);
    st = check_hip(ctx, launch_null_solve(ctx->stream, Y, n, m1, logdet_dev, F->nullfit, null_out), "null_solve");
  }
  if (st != NU_OK) return st;
  {
    // Z = X^T [A~ | r~0], refined once against L^T when X is the mixed inverse
    Timed tm(ctx, "cols_matvec", gemv_bytes * (mixed ? 3 : 1));
    st = check_hip(ctx, launch_cols_matvec(ctx->stream, F->X, np, n, np, Y, nv, xpart, xrc, xchunks, nullptr, 1.0, Z),
                   "cols_matvec");
    if (mixed && st == NU_OK)
      st = check_hip(ctx, launch_cols_matvec(ctx->stream, F->L, np, n, np, Z, nv, xpart, xrc, xchunks, Y, -1.0, Rz),
                     "cols_matvec");
    if (mixed && st == NU_OK)
      st = check_hip(ctx, launch_cols_matvec(ctx->stream, F->X, np, n, np, Rz, nv, xpart, xrc, xchunks, Z, 1.0, Z),
                     "cols_matvec");
  }
  if (st != NU_OK) return st;
  // ascending durations (nested boxes) with their caller indices
  std::vector<int32_t> order(n_d);
  for (int j = 0; j < n_d; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return dur_samples_host[a] < dur_samples_host[b]; });
  std::vector<int32_t> sorted(2 * n_d);
  for (int k = 0; k < n_d; ++k) {
    sorted[k] = dur_samples_host[order[k]];
    sorted[n_d + k] = order[k];
  }
  {
    Timed tm(ctx, "q_partial", 0.0);
    st = check_hip(ctx, launch_q_partial(ctx->stream, F->X, np, n, lattice, n_epochs, sorted.data(), n_d, dmax, qrc,
                                         qchunks, qpart),
                   "q_partial");
  }
  if (st != NU_OK) return st;
  {
    Timed tm(ctx, "cell_epilogue", 0.0);
    st = check_hip(ctx, launch_cell_epilogue(ctx->stream, qpart, qchunks, lattice, n, n_epochs, dur_samples_host,
                                             nullptr, n_d, Z, m1, F->nullfit, depth, var, dll, valid),
                   "cell_epilogue");
  }
  return st;
}

// ---------------------------------------------------------------------------
nu_status nu_periodic_search(nu_ctx* ctx, const double* depth, const double* var, const double* dll,
                             const uint8_t* valid, int n_d, int64_t n_epochs, double dt, const double* periods,
                             int64_t n_p, int log_term_sign, double* q_snr, int64_t* best_phase, int32_t* best_dur,
                             double* best_depth, double* best_sigma, double* best_lnp, int64_t* best_period_index) {
  if (!ctx) return NU_ERR_ARG;
  if (!depth || !var || !dll || !valid || !periods || !q_snr || !best_phase || !best_dur || !best_depth ||
      !best_sigma || !best_lnp)
    return set_error(ctx, NU_ERR_ARG, "periodic_search: null argument");
  if (n_d < 1 || n_d > MAX_ND) return set_error(ctx, NU_ERR_ARG, "periodic_search: n_d must be in [1, 16]");
  if (n_epochs < 1 || n_epochs > ((int64_t)1 << 31))
    return set_error(ctx, NU_ERR_ARG, "periodic_search: n_epochs must be in [1, 2^31]");
  if (!finite_pos(dt)) return set_error(ctx, NU_ERR_ARG, "periodic_search: dt must be finite and > 0");
  if (n_p < 1 || n_p > ((int64_t)1 << 31) - 1)
    return set_error(ctx, NU_ERR_ARG, "periodic_search: n_p must be in [1, 2^31)");
  if (log_term_sign != 1 && log_term_sign != -1)
    return set_error(ctx, NU_ERR_ARG, "periodic_search: log_term_sign must be +1 or -1");
  nu_status st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  double* packed = (double*)ctx_workspace(ctx, fold_workspace_doubles(n_d, n_epochs) * sizeof(double), &st);
  if (!packed) return st;
  {
    // algorithmic bytes: 24 per event visit (depth, var, dll of one interpolated event), n_d * n_epochs per period
    Timed tm(ctx, "fold", 24.0 * (double)n_d * (double)n_epochs * (double)n_p);
    st = check_hip(ctx, launch_fold(ctx->stream, depth, var, dll, valid, n_d, n_epochs, dt, periods, n_p,
                                    log_term_sign, q_snr, best_phase, best_dur, best_depth, best_sigma, best_lnp,
                                    packed),
                   "fold");
  }
  if (st != NU_OK) return st;
  if (best_period_index) {
    Timed tm(ctx, "best_period", 0.0);
    st = check_hip(ctx, launch_best_period(ctx->stream, q_snr, n_p, best_period_index), "best_period");
  }
  return st;
}

}  // extern "C"
