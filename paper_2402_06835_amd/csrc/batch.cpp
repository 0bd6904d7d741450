// Batched search of light curves of uneven length, captured graphs of the
// whole single-curve search, and the tile autotuner.
//
// Batch: the curves are ordered by length (longest first) and cut into waves
// whose factors fit the device-memory budget; the factors of a wave are carved
// from one device arena that the context keeps for later calls (allocating
// and freeing hundreds of GB per call costs seconds). Within a wave every dense stage
// is one launch for all curves: the diagonal blocks of Cholesky step k are
// one launch of one workgroup per curve that has a block k, and the panel,
// panel-update, trailing and inverse-level products of all curves form the
// problem list of one grouped GEMM launch. The linear and periodic searches
// then run curve by curve (each of their launches already covers the chip).
#include <algorithm>
#include <cmath>
#include <new>
#include <numeric>

#include "internal.hpp"

using namespace nu;

struct nu_graph {
  int device = 0;
  nu_factor* F = nullptr;
  double* ws = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

nu_status fail_batch(nu_ctx* ctx, std::vector<nu_factor*>& Fs, Plan* P, Plan* Q, nu_status st) {
  (void)hipStreamSynchronize(ctx->stream);
  if (P) plan_release(*P);
  if (Q) plan_release(*Q);
  for (nu_factor* F : Fs) factor_free(F);
  Fs.clear();
  return st;
}

const char* class_timing_name(int c) {
  static const char* names[TC_COUNT] = {"gemm_f64:panel",   "gemm_f64:panel_update", "gemm_f64:trailing",
                                        "gemm_f64:inverse", "gemm_f32:inverse",      "gemm_f64:band",
                                        "gemm_bf16x3:inverse"};
  return names[c];
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
nu_status nu_search_batch(nu_ctx* ctx, int n_curves, const int64_t* sample_off_host, const int64_t* epoch_off_host,
                          const double* t, const double* f, const double* A, int m1, const int64_t* lattice,
                          const nu_sho* theta_host, const double* dt_host, const int32_t* dur_samples_host, int n_d,
                          const double* periods, int64_t n_p, nu_precision prec, int log_term_sign,
                          size_t memory_budget_bytes, double* depth, double* var, double* dll, uint8_t* valid,
                          double* null_out, double* q_snr, int64_t* best_phase, int32_t* best_dur,
                          double* best_depth, double* best_sigma, double* best_lnp, int64_t* best_period_index,
                          double* logdet_host, int64_t* fail_pivot_host) {
  if (!ctx) return NU_ERR_ARG;
  if (n_curves < 1) return set_error(ctx, NU_ERR_ARG, "search_batch: n_curves must be >= 1");
  if (!sample_off_host || !epoch_off_host || !t || !theta_host || !dt_host || !periods || !q_snr || !best_phase ||
      !best_dur || !best_depth || !best_sigma || !best_lnp)
    return set_error(ctx, NU_ERR_ARG, "search_batch: null argument");
  if (sample_off_host[0] != 0 || epoch_off_host[0] != 0)
    return set_error(ctx, NU_ERR_ARG, "search_batch: offsets must start at 0");
  for (int c = 0; c < n_curves; ++c) {
    const int64_t n = sample_off_host[c + 1] - sample_off_host[c];
    const int64_t ne = epoch_off_host[c + 1] - epoch_off_host[c];
    if (n < 1 || n > (int64_t)1 << 17)
      return set_error(ctx, NU_ERR_ARG, "search_batch: every curve needs 1 .. 131072 samples");
    nu_status st = validate_theta(ctx, &theta_host[c]);
    if (st == NU_OK)
      st = validate_linear(ctx, n, f, A, m1, lattice, ne, dur_samples_host, n_d, prec, depth, var, dll, valid);
    if (st == NU_OK) st = validate_periodic(ctx, n_d, ne, dt_host[c], n_p, log_term_sign);
    if (st != NU_OK) return set_error(ctx, st, ctx->last_error + " (curve " + std::to_string(c) + ")");
  }
  nu_status st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  const bool mixed = prec != NU_FP64;

  // shared workspace of the per-curve searches, sized for the largest curve
  size_t ws_need = 0;
  for (int c = 0; c < n_curves; ++c) {
    const int64_t n = sample_off_host[c + 1] - sample_off_host[c];
    const int64_t ne = epoch_off_host[c + 1] - epoch_off_host[c];
    ws_need = std::max({ws_need, linear_ws_bytes(n, n_d, ne), periodic_ws_bytes(n_d, ne)});
  }
  double* ws = (double*)ctx_workspace(ctx, ws_need, &st);
  if (!ws) return st;

  // the budget counts the arena this context already holds as available
  size_t budget = memory_budget_bytes;
  if (budget == 0) {
    size_t free_b = 0, total_b = 0;
    st = check_hip(ctx, hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    if (st != NU_OK) return st;
    budget = (free_b + ctx->arena_bytes) / 10 * 9;
  }

  // longest curves first, cut into waves that fit the budget
  std::vector<int> order(n_curves);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return sample_off_host[a + 1] - sample_off_host[a] > sample_off_host[b + 1] - sample_off_host[b];
  });
  std::vector<std::vector<int>> waves;
  size_t used = 0;
  for (int c : order) {
    const size_t need = factor_bytes(sample_off_host[c + 1] - sample_off_host[c], prec);
    if (need > budget)
      return set_error(ctx, NU_ERR_OOM, "search_batch: curve " + std::to_string(c) +
                                            " does not fit the device-memory budget");
    if (waves.empty() || used + need > budget) {
      waves.emplace_back();
      used = 0;
    }
    waves.back().push_back(c);
    used += need;
  }
  size_t arena_need = 0;
  for (const auto& wave : waves) {
    size_t b = 0;
    for (int c : wave) b += factor_bytes(sample_off_host[c + 1] - sample_off_host[c], prec);
    arena_need = std::max(arena_need, b);
  }
  char* arena = nullptr;
  {
    HostTimed ht(ctx, "batch_arena");
    arena = (char*)ctx_arena(ctx, arena_need, &st);
  }
  if (!arena) return st;

  int n_failed = 0;
  int first_failed = -1;
  for (const auto& wave : waves) {
    std::vector<nu_factor*> Fs;
    {
      HostTimed ht(ctx, "batch_place");
      char* cursor = arena;
      for (int c : wave) {
        nu_factor* F = nullptr;
        st = factor_place(ctx, sample_off_host[c + 1] - sample_off_host[c], prec, &cursor, &F);
        if (st != NU_OK) break;
        Fs.push_back(F);
        F->theta_host = theta_host[c];
        st = check_hip(ctx, hipMemcpyAsync(F->theta_dev(), &F->theta_host, sizeof(nu_sho), hipMemcpyHostToDevice,
                                           ctx->stream),
                       "upload theta");
        if (st != NU_OK) break;
      }
    }
    if (st != NU_OK) return fail_batch(ctx, Fs, nullptr, nullptr, st);
    Plan P, Q;
    {
      HostTimed ht(ctx, "batch_plan");
      plan_cholesky(Fs, ctx->tuning, P);
      st = plan_upload(ctx, P);
    }
    std::vector<const double*> ts;
    std::vector<const nu_sho*> th;
    for (size_t i = 0; i < wave.size(); ++i) {
      ts.push_back(t + sample_off_host[wave[i]]);
      th.push_back(Fs[i]->theta_dev());
    }
    if (st == NU_OK) st = run_factor(ctx, Fs, P, ts, th);
    std::vector<int64_t> status;
    if (st == NU_OK) {
      HostTimed ht(ctx, "batch_factor_wait");
      st = read_factor_status(ctx, Fs, status);
    }
    if (st != NU_OK) return fail_batch(ctx, Fs, &P, &Q, st);

    std::vector<nu_factor*> ok;
    for (size_t i = 0; i < wave.size(); ++i) {
      const int c = wave[i];
      if (logdet_host) logdet_host[c] = Fs[i]->logdet;
      if (fail_pivot_host) fail_pivot_host[c] = status[i];
      if (status[i] < 0) {
        ok.push_back(Fs[i]);
      } else {
        if (first_failed < 0) first_failed = c;
        ++n_failed;
      }
    }
    if (!ok.empty()) {
      HostTimed ht(ctx, "batch_inverse_setup");
      if (mixed) {
        if (st == NU_OK) {
          plan_inverse(ok, gemm_kind_of(prec), ctx->tuning, Q);
          plan_band(ok, band_width(prec), ctx->tuning, Q);
          st = plan_upload(ctx, Q);
        }
        if (st == NU_OK) st = run_inverse_mixed(ctx, ok, Q, prec);
      } else {
        plan_inverse(ok, GK_F64, ctx->tuning, Q);
        st = plan_upload(ctx, Q);
        if (st == NU_OK) st = run_inverse_fp64(ctx, Q);
      }
    }
    for (size_t i = 0; st == NU_OK && i < wave.size(); ++i) {
      const int c = wave[i];
      const int64_t s0 = sample_off_host[c], e0 = epoch_off_host[c];
      const int64_t ne = epoch_off_host[c + 1] - e0;
      const int64_t cells = (int64_t)n_d * e0;
      double* qs = q_snr + (int64_t)c * n_p;
      int64_t* bp = best_phase + (int64_t)c * n_p;
      int32_t* bd = best_dur + (int64_t)c * n_p;
      double* bdep = best_depth + (int64_t)c * n_p;
      double* bsig = best_sigma + (int64_t)c * n_p;
      double* blnp = best_lnp + (int64_t)c * n_p;
      int64_t* bpi = best_period_index ? best_period_index + c : nullptr;
      if (status[i] >= 0) {
        st = check_hip(ctx, launch_fill_invalid_cells(ctx->stream, (int64_t)n_d * ne, depth + cells, var + cells,
                                                      dll + cells, valid + cells),
                       "fill invalid");
        if (st == NU_OK)
          st = check_hip(ctx, launch_fill_no_event(ctx->stream, n_p, qs, bp, bd, bdep, bsig, blnp, bpi),
                         "fill no event");
        continue;
      }
      st = run_linear(ctx, Fs[i], f + s0, m1 > 0 ? A + (int64_t)m1 * s0 : nullptr, m1, lattice + s0, ne,
                      dur_samples_host, n_d, prec, depth + cells, var + cells, dll + cells, valid + cells,
                      null_out ? null_out + 3 * (int64_t)c : nullptr, ws);
      if (st == NU_OK)
        st = run_periodic(ctx, depth + cells, var + cells, dll + cells, valid + cells, n_d, ne, dt_host[c],
                          periods, n_p, log_term_sign, qs, bp, bd, bdep, bsig, blnp, bpi, ws);
    }
    // the factors go before the next wave is allocated
    nu_status st2;
    {
      HostTimed ht(ctx, "batch_wait_free");
      st2 = fail_batch(ctx, Fs, &P, &Q, st);
    }
    if (st2 != NU_OK) return st2;
  }
  if (n_failed > 0)
    return set_error(ctx, NU_ERR_NOT_PD,
                     "search_batch: " + std::to_string(n_failed) + " covariance(s) not positive definite (first: curve " +
                         std::to_string(first_failed) + "); their outputs hold no candidate");
  return NU_OK;
}

// ---------------------------------------------------------------------------
nu_status nu_graph_create(nu_ctx* ctx, const double* t, int64_t n, const nu_sho* theta_dev, const double* f,
                          const double* A, int m1, const int64_t* lattice, int64_t n_epochs,
                          const int32_t* dur_samples_host, int n_d, nu_precision prec, double dt,
                          const double* periods, int64_t n_p, int log_term_sign, double* depth, double* var,
                          double* dll, uint8_t* valid, double* null_out, double* q_snr, int64_t* best_phase,
                          int32_t* best_dur, double* best_depth, double* best_sigma, double* best_lnp,
                          int64_t* best_period_index, int64_t* status_dev, nu_graph** out) {
  if (!ctx) return NU_ERR_ARG;
  if (!out || !t || !theta_dev || !status_dev || !periods || !q_snr || !best_phase || !best_dur || !best_depth ||
      !best_sigma || !best_lnp)
    return set_error(ctx, NU_ERR_ARG, "graph_create: null argument");
  *out = nullptr;
  if (n < 1 || n > (int64_t)1 << 17) return set_error(ctx, NU_ERR_ARG, "graph_create: n must be in [1, 131072]");
  nu_status st = validate_linear(ctx, n, f, A, m1, lattice, n_epochs, dur_samples_host, n_d, prec, depth, var, dll,
                                 valid);
  if (st == NU_OK) st = validate_periodic(ctx, n_d, n_epochs, dt, n_p, log_term_sign);
  if (st != NU_OK) return st;
  st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  const bool mixed = prec != NU_FP64;

  nu_graph* g = new (std::nothrow) nu_graph();
  if (!g) return set_error(ctx, NU_ERR_OOM, "graph_create: host allocation");
  g->device = ctx->device;
  auto fail = [&](nu_status s) {
    nu_graph_destroy(g);
    return s;
  };
  // every allocation happens before the capture
  st = factor_alloc(ctx, n, true, &g->F);
  if (st == NU_OK && mixed) st = ensure_plan32(ctx, g->F, prec);
  if (st == NU_OK)
    st = check_hip(ctx, hipMalloc(&g->ws, std::max(linear_ws_bytes(n, n_d, n_epochs), periodic_ws_bytes(n_d, n_epochs))),
                   "alloc graph workspace");
  if (st != NU_OK) return fail(st);

  hipStream_t cs = nullptr;
  st = check_hip(ctx, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
  if (st != NU_OK) return fail(st);
  const hipStream_t saved_stream = ctx->stream;
  const bool saved_timing = ctx->timing;
  ctx->stream = cs;
  ctx->timing = false;
  st = check_hip(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
  if (st == NU_OK) {
    nu_factor* F = g->F;
    std::vector<nu_factor*> one{F};
    nu_status cst = run_factor(ctx, one, F->plan64, {t}, {theta_dev});
    if (cst == NU_OK) cst = check_hip(ctx, launch_copy_i64(cs, F->status_dev(), status_dev), "status copy");
    if (cst == NU_OK) cst = mixed ? run_inverse_mixed(ctx, one, F->plan32, prec) : run_inverse_fp64(ctx, F->plan64);
    if (cst == NU_OK)
      cst = run_linear(ctx, F, f, A, m1, lattice, n_epochs, dur_samples_host, n_d, prec, depth, var, dll, valid,
                       null_out, g->ws);
    if (cst == NU_OK)
      cst = run_periodic(ctx, depth, var, dll, valid, n_d, n_epochs, dt, periods, n_p, log_term_sign, q_snr,
                         best_phase, best_dur, best_depth, best_sigma, best_lnp, best_period_index, g->ws);
    st = check_hip(ctx, hipStreamEndCapture(cs, &g->graph), "end capture");
    if (cst != NU_OK) st = cst;
  }
  ctx->stream = saved_stream;
  ctx->timing = saved_timing;
  (void)hipStreamDestroy(cs);
  if (st == NU_OK) st = check_hip(ctx, hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0), "instantiate");
  if (st != NU_OK) return fail(st);
  *out = g;
  return NU_OK;
}

nu_status nu_graph_launch(nu_ctx* ctx, nu_graph* g) {
  if (!ctx) return NU_ERR_ARG;
  if (!g || !g->exec) return set_error(ctx, NU_ERR_ARG, "graph_launch: null graph");
  if (g->device != ctx->device) return set_error(ctx, NU_ERR_ARG, "graph_launch: graph on another device");
  nu_status st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  return check_hip(ctx, hipGraphLaunch(g->exec, ctx->stream), "graph launch");
}

void nu_graph_destroy(nu_graph* g) {
  if (!g) return;
  if (hipSetDevice(g->device) != hipSuccess) {  // the runtime has shut down: host side only
    factor_free(g->F);
    delete g;
    return;
  }
  (void)hipDeviceSynchronize();
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->ws) (void)hipFree(g->ws);
  factor_free(g->F);
  delete g;
}

// ---------------------------------------------------------------------------
nu_status nu_ctx_get_tuning(const nu_ctx* ctx, int launch_class, int* small_below_host) {
  if (!ctx || !small_below_host || launch_class < 0 || launch_class >= TC_COUNT) return NU_ERR_ARG;
  *small_below_host = ctx->tuning.small_below[launch_class];
  return NU_OK;
}

nu_status nu_ctx_set_tuning(nu_ctx* ctx, int launch_class, int small_below) {
  if (!ctx) return NU_ERR_ARG;
  if (launch_class < 0 || launch_class >= TC_COUNT || small_below < 0)
    return set_error(ctx, NU_ERR_ARG, "set_tuning: class in [0, 7) and threshold >= 0 required");
  ctx->tuning.small_below[launch_class] = small_below;
  return NU_OK;
}

nu_status nu_ctx_autotune(nu_ctx* ctx, int64_t n, nu_precision prec) {
  if (!ctx) return NU_ERR_ARG;
  if (n < TB || n > (int64_t)1 << 17) return set_error(ctx, NU_ERR_ARG, "autotune: n must be in [128, 131072]");
  if (prec != NU_FP64 && prec != NU_FP32_REFINE && prec != NU_BF16X3_REFINE)
    return set_error(ctx, NU_ERR_ARG, "autotune: unknown precision");
  nu_status st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  const bool mixed = prec != NU_FP64;
  // a well-conditioned synthetic covariance on a unit-spaced grid
  std::vector<double> th(n);
  for (int64_t i = 0; i < n; ++i) th[i] = (double)i;
  double* t_dev = nullptr;
  nu_factor* F = nullptr;
  st = check_hip(ctx, hipMalloc(&t_dev, n * sizeof(double)), "autotune alloc");
  if (st == NU_OK) st = check_hip(ctx, hipMemcpy(t_dev, th.data(), n * sizeof(double), hipMemcpyHostToDevice), "copy");
  if (st == NU_OK) st = factor_alloc(ctx, n, false, &F);
  if (st == NU_OK && mixed) st = alloc_mixed(ctx, F, prec);
  if (st == NU_OK) {
    F->theta_host = nu_sho{1.0, 0.3, 2.0, 0.5};
    st = check_hip(ctx, hipMemcpy(F->theta_dev(), &F->theta_host, sizeof(nu_sho), hipMemcpyHostToDevice), "copy");
  }

  // the caller's timing state is put aside while the trials are timed
  resolve_timing(ctx);
  const bool saved_timing = ctx->timing;
  auto saved_timings = ctx->timings;
  auto saved_names = ctx->timing_names;
  const int candidates[] = {512, 0, 256, 1024, 2048, 1 << 30};
  double best_ms[TC_COUNT];
  int best_thr[TC_COUNT];
  for (int c = 0; c < TC_COUNT; ++c) {
    best_ms[c] = INFINITY;
    best_thr[c] = ctx->tuning.small_below[c];
  }
  std::vector<nu_factor*> one{F};
  for (int cand : candidates) {
    if (st != NU_OK) break;
    Tuning tu;
    for (int c = 0; c < TC_COUNT; ++c) tu.small_below[c] = cand;
    Plan P, Q;
    plan_cholesky(one, tu, P);
    plan_inverse(one, GK_F64, tu, P);
    st = plan_upload(ctx, P);
    if (st == NU_OK && mixed) {
      plan_inverse(one, gemm_kind_of(prec), tu, Q);
      plan_band(one, band_width(prec), tu, Q);
      st = plan_upload(ctx, Q);
    }
    for (int rep = 0; st == NU_OK && rep < 2; ++rep) {  // the second repetition is the one kept
      ctx->timings.clear();
      ctx->timing_names.clear();
      ctx->timing = true;
      st = run_factor(ctx, one, P, {t_dev}, {F->theta_dev()});
      if (st == NU_OK) st = run_inverse_fp64(ctx, P);
      if (st == NU_OK && mixed) st = run_inverse_mixed(ctx, one, Q, prec);
      resolve_timing(ctx);
      ctx->timing = false;
    }
    if (st == NU_OK)
      for (int c = 0; c < TC_COUNT; ++c) {
        auto it = ctx->timings.find(class_timing_name(c));
        if (it != ctx->timings.end() && it->second.ms < best_ms[c]) {
          best_ms[c] = it->second.ms;
          best_thr[c] = cand;
        }
      }
    (void)hipStreamSynchronize(ctx->stream);
    plan_release(P);
    plan_release(Q);
  }
  ctx->timing = saved_timing;
  ctx->timings = saved_timings;
  ctx->timing_names = saved_names;
  factor_free(F);
  if (t_dev) (void)hipFree(t_dev);
  if (st != NU_OK) return st;
  for (int c = 0; c < TC_COUNT; ++c) ctx->tuning.small_below[c] = best_thr[c];
  return NU_OK;
}

}  // extern "C"
