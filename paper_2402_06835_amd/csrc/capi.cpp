// C ABI of the transit-search library, single-curve entry points: argument
// validation, context and factor objects, kernel timing. The schedules and
// enqueue sequences live in the engine. No exception crosses the boundary.
#include <algorithm>
#include <chrono>
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

nu_status mem_check(nu_ctx* ctx, size_t bytes, size_t replaced, const char* what) {
  const MemCount& m = *ctx->mem;
  const size_t live = m.live.load() - replaced;
  if (m.limit && (bytes > m.limit || live > m.limit - bytes))
    return set_error(ctx, NU_ERR_OOM,
                     std::string(what) + ": " + std::to_string(bytes) + " bytes would exceed the context's limit of " +
                         std::to_string(m.limit) + " bytes (" + std::to_string(live) + " in use)");
  return NU_OK;
}

nu_status ctx_malloc(nu_ctx* ctx, void** p, size_t bytes, MemHold& hold, const char* what) {
  *p = nullptr;
  nu_status st = mem_check(ctx, bytes, 0, what);
  if (st == NU_OK) st = check_hip(ctx, hipMalloc(p, bytes), what);
  if (st != NU_OK) {
    *p = nullptr;
    return st;
  }
  if (!hold.count) hold.count = ctx->mem;
  ctx->mem->live += bytes;
  hold.bytes += bytes;
  return NU_OK;
}

size_t mem_headroom(const nu_ctx* ctx, size_t replaced) {
  const MemCount& m = *ctx->mem;
  if (!m.limit) return SIZE_MAX;
  const size_t live = m.live.load() - replaced;
  return live >= m.limit ? 0 : m.limit - live;
}

// the context's own growable buffer (workspace or arena): grown to `bytes`
// when smaller, counted against the limit
static void* ctx_grow(nu_ctx* ctx, void** buf, size_t* have, size_t bytes, const char* what, nu_status* st) {
  *st = NU_OK;
  if (bytes <= *have) return *buf;
  *st = mem_check(ctx, bytes, *have, what);
  if (*st != NU_OK) return nullptr;
  // the old buffer may still be in use by enqueued work
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess && *buf) e = hipFree(*buf);
  ctx->mem->live -= *have;
  *buf = nullptr;
  *have = 0;
  if (e == hipSuccess) e = hipMalloc(buf, bytes);
  if (e != hipSuccess) {
    *st = check_hip(ctx, e, what);
    *buf = nullptr;
    return nullptr;
  }
  ctx->mem->live += bytes;
  *have = bytes;
  return *buf;
}

void* ctx_workspace(nu_ctx* ctx, size_t bytes, nu_status* st) {
  return ctx_grow(ctx, &ctx->ws, &ctx->ws_bytes, bytes, "workspace allocation", st);
}

nu_status ctx_upload(nu_ctx* ctx, const void* host, size_t bytes, void* dev) {
  if (bytes == 0) return NU_OK;
  // the previous copy out of the staging buffer must be done before it is overwritten
  if (ctx->pinned_ev) {
    nu_status st = check_hip(ctx, hipEventSynchronize(ctx->pinned_ev), "upload wait");
    if (st != NU_OK) return st;
  } else {
    nu_status st = check_hip(ctx, hipEventCreateWithFlags(&ctx->pinned_ev, hipEventDisableTiming), "upload event");
    if (st != NU_OK) return st;
  }
  if (bytes > ctx->pinned_bytes) {
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
    nu_status st = check_hip(ctx, hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault), "pinned staging");
    if (st != NU_OK) return st;
    ctx->pinned_bytes = bytes;
  }
  std::memcpy(ctx->pinned, host, bytes);
  nu_status st = check_hip(ctx, hipMemcpyAsync(dev, ctx->pinned, bytes, hipMemcpyHostToDevice, ctx->stream),
                           "upload");
  if (st == NU_OK) st = check_hip(ctx, hipEventRecord(ctx->pinned_ev, ctx->stream), "upload event");
  return st;
}

nu_status validate_shapes(nu_ctx* ctx, const double* shapes_host, const int32_t* dur_samples_host, int n_d) {
  int64_t total = 0;
  for (int j = 0; j < n_d; ++j) total += dur_samples_host[j];
  if (total > MAX_SHAPE)
    return set_error(ctx, NU_ERR_ARG, "template search: the shapes together may hold at most 2048 values");
  for (int64_t k = 0; k < total; ++k)
    if (!std::isfinite(shapes_host[k])) return set_error(ctx, NU_ERR_ARG, "template search: shape values must be finite");
  return NU_OK;
}

void* ctx_arena(nu_ctx* ctx, size_t bytes, nu_status* st) {
  return ctx_grow(ctx, &ctx->arena, &ctx->arena_bytes, bytes, "arena allocation", st);
}

void timing_begin(nu_ctx* ctx, hipStream_t s, const char* name, hipEvent_t* start) {
  *start = nullptr;
  if (!ctx->timing) return;
  if (!ctx->timing_only.empty() && std::strncmp(name, ctx->timing_only.c_str(), ctx->timing_only.size()) != 0) return;
  if (ctx->free_events.empty()) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return;
    ctx->free_events.push_back(ev);
  }
  *start = ctx->free_events.back();
  ctx->free_events.pop_back();
  (void)hipEventRecord(*start, s);
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
  (void)hipEventRecord(stop, s);
  ctx->pending.push_back({name, start, stop, work});
}

void timing_pair(nu_ctx* ctx, const char* name, hipEvent_t* start, hipEvent_t* stop) {
  *start = *stop = nullptr;
  if (!ctx->timing) return;
  if (!ctx->timing_only.empty() && std::strncmp(name, ctx->timing_only.c_str(), ctx->timing_only.size()) != 0) return;
  while (ctx->free_events.size() < 2) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return;
    ctx->free_events.push_back(ev);
  }
  *start = ctx->free_events.back();
  ctx->free_events.pop_back();
  *stop = ctx->free_events.back();
  ctx->free_events.pop_back();
}

void timing_add(nu_ctx* ctx, const char* name, hipEvent_t start, hipEvent_t stop, double work) {
  if (start && stop) ctx->pending.push_back({name, start, stop, work});
}

static double wall_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

HostTimed::HostTimed(nu_ctx* c, const char* n) : ctx(c), name(n), t0(c->timing ? wall_ms() : 0.0) {}

HostTimed::~HostTimed() {
  if (!ctx->timing) return;
  const std::string key = std::string("host:") + name;
  auto it = ctx->timings.find(key);
  if (it == ctx->timings.end()) {
    ctx->timing_names.push_back(key);
    it = ctx->timings.emplace(key, nu_timing_slot{}).first;
  }
  it->second.launches += 1;
  it->second.ms += wall_ms() - t0;
}

void resolve_timing(nu_ctx* ctx) {
  if (ctx->pending.empty()) return;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& p : ctx->pending) {
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, p.start, p.stop);
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

nu_status validate_theta(nu_ctx* ctx, const nu_sho* theta) {
  const nu_sho& th = *theta;
  auto finite_pos = [](double x) { return std::isfinite(x) && x > 0.0; };
  if (!(std::isfinite(th.amp) && th.amp >= 0.0) || !finite_pos(th.omega) || !finite_pos(th.q) ||
      !(std::isfinite(th.sigma_w) && th.sigma_w >= 0.0))
    return set_error(ctx, NU_ERR_ARG, "gp_factor: need finite amp >= 0, omega > 0, q > 0, sigma_w >= 0");
  return NU_OK;
}

nu_status validate_kernel(nu_ctx* ctx, const nu_kernel* k) {
  auto finite_pos = [](double x) { return std::isfinite(x) && x > 0.0; };
  auto finite_nonneg = [](double x) { return std::isfinite(x) && x >= 0.0; };
  if (k->n_sho < 0 || k->n_sho > 4 || k->n_exp < 0 || k->n_exp > 4)
    return set_error(ctx, NU_ERR_ARG, "kernel: n_sho and n_exp must be in [0, 4]");
  for (int s = 0; s < k->n_sho; ++s)
    if (!finite_nonneg(k->sho_amp[s]) || !finite_pos(k->sho_omega[s]) || !finite_pos(k->sho_q[s]))
      return set_error(ctx, NU_ERR_ARG, "kernel: SHO terms need finite amp >= 0, omega > 0, q > 0");
  for (int e = 0; e < k->n_exp; ++e)
    if (!finite_nonneg(k->exp_sigma[e]) || !finite_pos(k->exp_ell[e]))
      return set_error(ctx, NU_ERR_ARG, "kernel: exponential terms need finite sigma >= 0, ell > 0");
  if (!finite_nonneg(k->sigma_w)) return set_error(ctx, NU_ERR_ARG, "kernel: need finite sigma_w >= 0");
  return NU_OK;
}

}  // namespace nu

namespace {

// K build (from the uploaded theta or kernel), blocked Cholesky, ln|K|;
// synchronises once for the status. With an inverse precision set on the
// context (nu_ctx_set_inverse_prefetch), the factor's reduced-precision
// inverse for it is computed here too, its early phases inside the
// factorisation.
nu_status factor_run(nu_ctx* ctx, nu_factor* F, const double* t, double* logdet_host, int64_t* fail_pivot_host) {
  std::vector<nu_factor*> one{F};
  nu_status st = NU_OK;
  EarlyInverse early;
  const bool prefetch = ctx->prefetch_prec > 0;
  if (prefetch) {
    early.F = F;
    early.prec = ctx->prefetch_prec;
    st = ensure_plan32(ctx, F, early.prec);
  }
  if (st == NU_OK) st = run_factor(ctx, one, F->plan64, {t}, {F->theta_dev()}, prefetch ? &early : nullptr);
  if (st == NU_OK && prefetch) {
    // the phases the factorisation did not start, then the last one
    for (int k = early.started; st == NU_OK && k + 1 < (int)F->plan32.phases.size(); ++k)
      st = run_inverse_phase(ctx, F, F->plan32, early.prec, k, ctx->stream);
    if (st == NU_OK)
      st = F->plan32.phases.empty() ? run_inverse_mixed(ctx, one, F->plan32, early.prec)
                                    : run_inverse_post(ctx, F, F->plan32, early.prec);
  }
  std::vector<int64_t> status;
  if (st == NU_OK) st = read_factor_status(ctx, one, status);
  if (st != NU_OK) return st;
  if (status[0] >= 0) {
    if (fail_pivot_host) *fail_pivot_host = status[0];
    return set_error(ctx, NU_ERR_NOT_PD,
                     "gp_factor: covariance not positive definite at pivot " + std::to_string(status[0]));
  }
  if (prefetch) F->inverse_kind = 1 + early.prec;
  if (logdet_host) *logdet_host = F->logdet;
  return NU_OK;
}

nu_status factor_compute_kernel(nu_ctx* ctx, nu_factor* F, const double* t, const nu_kernel& k, double* logdet_host,
                                int64_t* fail_pivot_host) {
  F->general = true;
  F->kernel_host = k;
  nu_status st = check_hip(ctx, hipMemcpyAsync(F->kernel_dev(), &F->kernel_host, sizeof(nu_kernel),
                                               hipMemcpyHostToDevice, ctx->stream),
                           "upload kernel");
  if (st != NU_OK) return st;
  return factor_run(ctx, F, t, logdet_host, fail_pivot_host);
}

// theta upload, K build, blocked Cholesky, ln|K|; synchronises once for the status
nu_status factor_compute(nu_ctx* ctx, nu_factor* F, const double* t, const nu_sho& th, double* logdet_host,
                         int64_t* fail_pivot_host) {
  F->general = false;
  F->theta_host = th;
  nu_status st = check_hip(ctx, hipMemcpyAsync(F->theta_dev(), &F->theta_host, sizeof(nu_sho), hipMemcpyHostToDevice,
                                               ctx->stream),
                           "upload theta");
  if (st != NU_OK) return st;
  return factor_run(ctx, F, t, logdet_host, fail_pivot_host);
}

}  // namespace

// ===========================================================================
extern "C" {

nu_status nu_ctx_create(int device, void* stream, size_t workspace_limit_bytes, nu_ctx** out) {
  if (!out) return NU_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return NU_ERR_DEVICE;
  if (device < 0 || device >= ndev) return NU_ERR_ARG;
  nu_ctx* ctx = new (std::nothrow) nu_ctx();
  if (!ctx) return NU_ERR_OOM;
  ctx->device = device;
  ctx->stream = (hipStream_t)stream;
  ctx->mem->limit = workspace_limit_bytes;
  if (hipSetDevice(device) != hipSuccess || nu::fold_scratch_ptr(device, &ctx->scratch) != hipSuccess) {
    delete ctx;
    return NU_ERR_DEVICE;
  }
  *out = ctx;
  return NU_OK;
}

void nu_ctx_destroy(nu_ctx* ctx) {
  if (!ctx) return;
  // Called after the HIP runtime has shut down (a context released during
  // process exit), the device objects went with the runtime: free the host
  // side only, and touch nothing on the device.
  if (hipSetDevice(ctx->device) != hipSuccess) {
    delete ctx;
    return;
  }
  (void)hipStreamSynchronize(ctx->stream);
  nu::destroy_factor_streams(ctx);
  if (ctx->s_fold) {
    (void)hipStreamSynchronize(ctx->s_fold);
    (void)hipStreamDestroy(ctx->s_fold);
  }
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->arena) (void)hipFree(ctx->arena);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->pinned_ev) (void)hipEventDestroy(ctx->pinned_ev);
  for (auto& p : ctx->pending) {
    (void)hipEventDestroy(p.start);
    (void)hipEventDestroy(p.stop);
  }
  for (auto e : ctx->free_events) (void)hipEventDestroy(e);
  delete ctx;
}

nu_status nu_ctx_release_memory(nu_ctx* ctx) {
  if (!ctx) return NU_ERR_ARG;
  nu_status st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st == NU_OK) st = check_hip(ctx, hipStreamSynchronize(ctx->stream), "release sync");
  if (st != NU_OK) return st;
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->arena) (void)hipFree(ctx->arena);
  ctx->mem->live -= ctx->ws_bytes + ctx->arena_bytes;
  ctx->ws = ctx->arena = nullptr;
  ctx->ws_bytes = ctx->arena_bytes = 0;
  return NU_OK;
}

size_t nu_ctx_device_bytes(const nu_ctx* ctx) { return ctx ? ctx->mem->live.load() : 0; }

nu_status nu_ctx_set_stream(nu_ctx* ctx, void* stream) {
  if (!ctx) return NU_ERR_ARG;
  ctx->stream = (hipStream_t)stream;
  return NU_OK;
}

const char* nu_ctx_last_error(const nu_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

nu_status nu_ctx_set_inverse_prefetch(nu_ctx* ctx, int prec, int compute_units) {
  if (!ctx) return NU_ERR_ARG;
  if (prec != -1 && prec != NU_FP32_REFINE && prec != NU_BF16X3_REFINE)
    return set_error(ctx, NU_ERR_ARG, "inverse prefetch: precision must be NU_FP32_REFINE, NU_BF16X3_REFINE or -1");
  if (compute_units < 0) return set_error(ctx, NU_ERR_ARG, "inverse prefetch: compute_units must be >= 0");
  ctx->prefetch_prec = prec;
  ctx->prefetch_cus = compute_units;
  return NU_OK;
}

nu_status nu_ctx_enable_timing(nu_ctx* ctx, int enable) {
  if (!ctx) return NU_ERR_ARG;
  ctx->timing = enable != 0;
  return NU_OK;
}

nu_status nu_ctx_set_timing_filter(nu_ctx* ctx, const char* prefix) {
  if (!ctx) return NU_ERR_ARG;
  ctx->timing_only = prefix ? prefix : "";
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
  nu_factor* F = nullptr;
  st = factor_alloc(ctx, n, true, &F);
  if (st != NU_OK) return st;
  st = factor_compute(ctx, F, t, *theta, logdet_host, fail_pivot_host);
  if (st != NU_OK) {
    factor_free(F);
    return st;
  }
  *out = F;
  return NU_OK;
}

// The stellar-variability kernel of Section 3.2 as terms of a nu_kernel. An
// SHO term of power S0 has k(0) = S0 omega Q, which is what nu_kernel's
// amplitude squares; the two modes share the variance sigma^2 in the ratio
// 1 : f.
nu_status nu_rotation_kernel(double sigma, double period, double q0, double dq, double f, double sigma_short,
                             double ell_short, double sigma_long, double ell_long, double sigma_w,
                             nu_kernel* out_host) {
  if (!out_host) return NU_ERR_ARG;
  const double in[] = {sigma, period, q0, dq, f, sigma_short, ell_short, sigma_long, ell_long, sigma_w};
  for (double v : in)
    if (!std::isfinite(v)) return NU_ERR_ARG;
  const double q1 = 0.5 + q0 + dq, q2 = 0.5 + q0;
  if (!(sigma >= 0.0 && period > 0.0 && q0 > 0.0 && dq >= 0.0 && f >= 0.0 && sigma_short >= 0.0 &&
        ell_short > 0.0 && sigma_long >= 0.0 && ell_long > 0.0 && sigma_w >= 0.0))
    return NU_ERR_ARG;
  const double w1 = 4.0 * M_PI * q1 / (period * std::sqrt(4.0 * q1 * q1 - 1.0));
  const double w2 = 2.0 * w1;
  const double s1 = sigma * sigma / ((1.0 + f) * w1 * q1);
  const double s2 = f * sigma * sigma / ((1.0 + f) * w2 * q2);
  nu_kernel k{};
  k.n_sho = 2;
  k.n_exp = 2;
  k.sho_amp[0] = std::sqrt(s1 * w1 * q1);
  k.sho_omega[0] = w1;
  k.sho_q[0] = q1;
  k.sho_amp[1] = std::sqrt(s2 * w2 * q2);
  k.sho_omega[1] = w2;
  k.sho_q[1] = q2;
  k.exp_sigma[0] = sigma_short;
  k.exp_ell[0] = ell_short;
  k.exp_sigma[1] = sigma_long;
  k.exp_ell[1] = ell_long;
  k.sigma_w = sigma_w;
  *out_host = k;
  return NU_OK;
}

nu_status nu_gp_factor_kernel(nu_ctx* ctx, const double* t, int64_t n, const nu_kernel* kernel_host,
                              nu_factor** out, double* logdet_host, int64_t* fail_pivot_host) {
  if (!ctx) return NU_ERR_ARG;
  if (!t || !kernel_host || !out) return set_error(ctx, NU_ERR_ARG, "gp_factor_kernel: null argument");
  *out = nullptr;
  if (fail_pivot_host) *fail_pivot_host = -1;
  if (n < 1 || n > (int64_t)1 << 17) return set_error(ctx, NU_ERR_ARG, "gp_factor_kernel: n must be in [1, 131072]");
  nu_status st = validate_kernel(ctx, kernel_host);
  if (st != NU_OK) return st;
  st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  nu_factor* F = nullptr;
  st = factor_alloc(ctx, n, true, &F);
  if (st != NU_OK) return st;
  st = factor_compute_kernel(ctx, F, t, *kernel_host, logdet_host, fail_pivot_host);
  if (st != NU_OK) {
    factor_free(F);
    return st;
  }
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

void nu_factor_destroy(nu_factor* F) { factor_free(F); }

int64_t nu_factor_n(const nu_factor* F) { return F ? F->n : -1; }

// ---------------------------------------------------------------------------
nu_status nu_linear_search(nu_ctx* ctx, nu_factor* F, const double* f, const double* A, int m1,
                           const int64_t* lattice, int64_t n_epochs, const int32_t* dur_samples_host, int n_d,
                           nu_precision prec, double* depth, double* var, double* dll, uint8_t* valid,
                           double* null_out) {
  if (!ctx) return NU_ERR_ARG;
  if (!F) return set_error(ctx, NU_ERR_ARG, "linear_search: null argument");
  if (F->device != ctx->device) return set_error(ctx, NU_ERR_ARG, "linear_search: factor on another device");
  nu_status st = validate_linear(ctx, F->n, f, A, m1, lattice, n_epochs, dur_samples_host, n_d, prec, depth, var,
                                 dll, valid);
  if (st != NU_OK) return st;
  st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  const bool mixed = prec != NU_FP64;

  // triangular inverse X = L^-1 (kept in the factor for further searches)
  const int want = 1 + (int)prec;
  if (F->inverse_kind != want) {
    if (mixed) {
      st = ensure_plan32(ctx, F, prec);
      if (st == NU_OK) st = run_inverse_mixed(ctx, {F}, F->plan32, prec);
    } else {
      st = run_inverse_fp64(ctx, F->plan64);
    }
    if (st != NU_OK) return st;
    F->inverse_kind = want;
  }
  double* ws = (double*)ctx_workspace(ctx, linear_ws_bytes(F->n, n_d, n_epochs), &st);
  if (!ws) return st;
  return run_linear(ctx, F, f, A, m1, lattice, n_epochs, dur_samples_host, n_d, prec, depth, var, dll, valid,
                    null_out, ws);
}

// ---------------------------------------------------------------------------
nu_status nu_linear_search_template(nu_ctx* ctx, nu_factor* F, const double* f, const double* A, int m1,
                                    const int64_t* lattice, int64_t n_epochs, const int32_t* dur_samples_host,
                                    int n_d, const double* shapes_host, nu_precision prec, double* depth,
                                    double* var, double* dll, uint8_t* valid, double* null_out) {
  if (!ctx) return NU_ERR_ARG;
  if (!F || !shapes_host) return set_error(ctx, NU_ERR_ARG, "linear_search_template: null argument");
  if (F->device != ctx->device) return set_error(ctx, NU_ERR_ARG, "linear_search_template: factor on another device");
  nu_status st = validate_linear(ctx, F->n, f, A, m1, lattice, n_epochs, dur_samples_host, n_d, prec, depth, var,
                                 dll, valid);
  if (st == NU_OK) st = validate_shapes(ctx, shapes_host, dur_samples_host, n_d);
  if (st != NU_OK) return st;
  st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  const bool mixed = prec != NU_FP64;
  const int want = 1 + (int)prec;
  if (F->inverse_kind != want) {
    if (mixed) {
      st = ensure_plan32(ctx, F, prec);
      if (st == NU_OK) st = run_inverse_mixed(ctx, {F}, F->plan32, prec);
    } else {
      st = run_inverse_fp64(ctx, F->plan64);
    }
    if (st != NU_OK) return st;
    F->inverse_kind = want;
  }
  double* ws = (double*)ctx_workspace(ctx, linear_ws_bytes(F->n, n_d, n_epochs), &st);
  if (!ws) return st;
  return run_linear(ctx, F, f, A, m1, lattice, n_epochs, dur_samples_host, n_d, prec, depth, var, dll, valid,
                    null_out, ws, shapes_host);
}

// ---------------------------------------------------------------------------
nu_status nu_linear_search_ss(nu_ctx* ctx, const double* t, int64_t n, const nu_kernel* kernel_host, const double* f,
                              const double* A, int m1, const int64_t* lattice, int64_t n_epochs,
                              const int32_t* dur_samples_host, int n_d, const double* shapes_host, double* depth,
                              double* var, double* dll, uint8_t* valid, double* null_out, int64_t* fail_index_host) {
  if (!ctx) return NU_ERR_ARG;
  if (!t || !kernel_host) return set_error(ctx, NU_ERR_ARG, "linear_search_ss: null argument");
  nu_status st = validate_kernel(ctx, kernel_host);
  if (st != NU_OK) return st;
  if (kernel_host->n_sho + kernel_host->n_exp < 1)
    return set_error(ctx, NU_ERR_ARG, "linear_search_ss: the kernel needs at least one SHO or exponential term");
  if (n < 1 || n > ((int64_t)1 << 31)) return set_error(ctx, NU_ERR_ARG, "linear_search_ss: n must be in [1, 2^31]");
  st = validate_linear(ctx, n, f, A, m1, lattice, n_epochs, dur_samples_host, n_d, NU_FP64, depth, var, dll, valid);
  if (st == NU_OK && shapes_host) st = validate_shapes(ctx, shapes_host, dur_samples_host, n_d);
  if (st != NU_OK) return st;
  st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  double* ws = (double*)ctx_workspace(ctx, linear_ss_ws_bytes(n, *kernel_host, n_d, n_epochs), &st);
  if (!ws) return st;
  int64_t* status_dev = nullptr;
  st = run_linear_ss(ctx, t, n, *kernel_host, f, A, m1, lattice, n_epochs, dur_samples_host, n_d, shapes_host, depth,
                     var, dll, valid, null_out, ws, &status_dev);
  if (st != NU_OK || !fail_index_host) return st;
  int64_t fail = -1;
  st = check_hip(ctx, hipMemcpyAsync(&fail, status_dev, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream),
                 "hipMemcpyAsync");
  if (st == NU_OK) st = check_hip(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  if (st != NU_OK) return st;
  *fail_index_host = fail;
  if (fail >= 0)
    return set_error(ctx, NU_ERR_NOT_PD,
                     "linear_search_ss: innovation variance not positive at sample " + std::to_string(fail));
  return NU_OK;
}

// ---------------------------------------------------------------------------
nu_status nu_mask_transit(nu_ctx* ctx, double* depth, double* var, double* dll, uint8_t* valid, int n_d,
                          int64_t n_epochs, double dt, double period, int64_t phase, int half_width) {
  if (!ctx) return NU_ERR_ARG;
  if (!depth || !var || !dll || !valid) return set_error(ctx, NU_ERR_ARG, "mask_transit: null argument");
  if (n_d < 1 || n_d > MAX_ND) return set_error(ctx, NU_ERR_ARG, "mask_transit: n_d must be in [1, 16]");
  if (n_epochs < 1 || n_epochs > ((int64_t)1 << 31))
    return set_error(ctx, NU_ERR_ARG, "mask_transit: n_epochs must be in [1, 2^31]");
  if (!(std::isfinite(dt) && dt > 0.0)) return set_error(ctx, NU_ERR_ARG, "mask_transit: dt must be finite and > 0");
  const double p = period / dt;
  if (!(std::isfinite(p) && p >= 1.0 && p <= 1e15))
    return set_error(ctx, NU_ERR_ARG, "mask_transit: period must be at least one cadence (and finite)");
  if (phase < 0 || phase >= n_epochs) return set_error(ctx, NU_ERR_ARG, "mask_transit: phase must be in [0, n_epochs)");
  if (half_width < 1 || half_width > MAX_DUR)
    return set_error(ctx, NU_ERR_ARG, "mask_transit: half_width must be in [1, 1024] slots");
  nu_status st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  Timed tm(ctx, "mask_transit", 0.0);
  return check_hip(ctx, launch_mask_transit(ctx->stream, depth, var, dll, valid, n_d, n_epochs, p, phase, half_width),
                   "mask_transit");
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
  nu_status st = validate_periodic(ctx, n_d, n_epochs, dt, n_p, log_term_sign);
  if (st != NU_OK) return st;
  st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  double* ws = (double*)ctx_workspace(ctx, periodic_ws_bytes(n_d, n_epochs), &st);
  if (!ws) return st;
  return run_periodic(ctx, depth, var, dll, valid, n_d, n_epochs, dt, periods, n_p, log_term_sign, q_snr,
                      best_phase, best_dur, best_depth, best_sigma, best_lnp, best_period_index, ws);
}

// ---------------------------------------------------------------------------
// The periodic search of nu_periodic_search without any allocation: the
// packed grid goes to the device's fixed scratch array (looked up in
// nu_ctx_create), and the kernels are the same, so the outputs are bitwise
// those of nu_periodic_search. No kernel timing is recorded for it.
nu_status nu_periodic_search_noalloc(nu_ctx* ctx, const double* depth, const double* var, const double* dll,
                                     const uint8_t* valid, int n_d, int64_t n_epochs, double dt,
                                     const double* periods, int64_t n_p, int log_term_sign, double* q_snr,
                                     int64_t* best_phase, int32_t* best_dur, double* best_depth, double* best_sigma,
                                     double* best_lnp, int64_t* best_period_index) {
  if (!ctx) return NU_ERR_ARG;
  if (!depth || !var || !dll || !valid || !periods || !q_snr || !best_phase || !best_dur || !best_depth ||
      !best_sigma || !best_lnp)
    return set_error(ctx, NU_ERR_ARG, "periodic_search_noalloc: null argument");
  nu_status st = validate_periodic(ctx, n_d, n_epochs, dt, n_p, log_term_sign);
  if (st != NU_OK) return st;
  if (fold_workspace_doubles(n_d, n_epochs) > FOLD_SCRATCH_DOUBLES)
    return set_error(ctx, NU_ERR_ARG,
                     "periodic_search_noalloc: 24 n_d (n_epochs + 64) bytes exceed the scratch of " +
                         std::to_string(NU_PERIODIC_SCRATCH_BYTES) + " bytes");
  if (!ctx->scratch) return set_error(ctx, NU_ERR_DEVICE, "periodic_search_noalloc: no scratch on this device");
  st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  st = check_hip(ctx, launch_fold(ctx->stream, depth, var, dll, valid, n_d, n_epochs, dt, periods, n_p, log_term_sign,
                                  q_snr, best_phase, best_dur, best_depth, best_sigma, best_lnp, ctx->scratch),
                 "fold");
  if (st == NU_OK && best_period_index)
    st = check_hip(ctx, launch_best_period(ctx->stream, q_snr, n_p, best_period_index), "best_period");
  return st;
}

// ---------------------------------------------------------------------------
nu_status nu_periodic_search_segments(nu_ctx* ctx, const double* depth, const double* var, const double* dll,
                                      const uint8_t* valid, int n_d, int n_seg, const int64_t* seg_len_host,
                                      const int64_t* seg_off_host, double dt, const double* periods, int64_t n_p,
                                      int log_term_sign, double* q_snr, int64_t* best_phase, int32_t* best_dur,
                                      double* best_depth, double* best_sigma, double* best_lnp,
                                      int64_t* best_period_index) {
  if (!ctx) return NU_ERR_ARG;
  if (!depth || !var || !dll || !valid || !periods || !q_snr || !best_phase || !best_dur || !best_depth ||
      !best_sigma || !best_lnp || !seg_len_host || !seg_off_host)
    return set_error(ctx, NU_ERR_ARG, "periodic_search_segments: null argument");
  if (n_seg < 1 || n_seg > MAX_SEG)
    return set_error(ctx, NU_ERR_ARG, "periodic_search_segments: n_seg must be in [1, 32]");
  for (int s = 0; s < n_seg; ++s) {
    if (seg_len_host[s] < 1 || seg_off_host[s] < 0)
      return set_error(ctx, NU_ERR_ARG, "periodic_search_segments: segment lengths >= 1 and offsets >= 0 required");
    if (s > 0 && seg_off_host[s] < seg_off_host[s - 1] + seg_len_host[s - 1] + 64)
      return set_error(ctx, NU_ERR_ARG,
                       "periodic_search_segments: segments must be ascending and at least 64 slots apart");
  }
  const int64_t extent = seg_off_host[n_seg - 1] + seg_len_host[n_seg - 1];
  nu_status st = validate_periodic(ctx, n_d, extent, dt, n_p, log_term_sign);
  if (st != NU_OK) return st;
  st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  double* ws =
      (double*)ctx_workspace(ctx, fold_segments_workspace_doubles(n_d, seg_len_host, n_seg) * sizeof(double), &st);
  if (!ws) return st;
  int64_t cells = 0;
  for (int s = 0; s < n_seg; ++s) cells += (int64_t)n_d * seg_len_host[s];
  {
    Timed tm(ctx, "fold", FOLD_FLOPS_PER_VISIT * (double)cells * (double)n_p);
    st = check_hip(ctx, launch_fold_segments(ctx->stream, depth, var, dll, valid, n_d, n_seg, seg_len_host,
                                             seg_off_host, dt, periods, n_p, log_term_sign, q_snr, best_phase,
                                             best_dur, best_depth, best_sigma, best_lnp, ws),
                   "fold_segments");
  }
  if (st == NU_OK && best_period_index) {
    Timed tm(ctx, "best_period", 0.0);
    st = check_hip(ctx, launch_best_period(ctx->stream, q_snr, n_p, best_period_index), "best_period");
  }
  return st;
}

}  // extern "C"
