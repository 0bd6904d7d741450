// Batched search of light curves of uneven length, its captured graph, captured
// graphs of the whole single-curve search, and the tile autotuner.
//
// Batch: the curves are ordered by length (longest first) and cut into waves
// whose factors fit the device-memory budget; the factors of a wave (and each
// curve's search workspace, inside its factor's inverse workspace) are carved
// from one device arena that the context keeps for later calls (allocating
// and freeing hundreds of GB per call costs seconds). Every stage of a wave is
// one launch for all its curves: the covariance build, the diagonal blocks of
// each Cholesky step (one workgroup per curve) and the grouped GEMMs of its
// panel, panel-update and trailing products, each level of the inverse, every
// pass of the linear search, the fold over (period, curve) and the best
// periods. A wave's fold and best periods run on a second stream beside the
// next wave's factorisation (vector work beside matrix-core work), reading
// grids kept outside the arena. The per-curve records (CurveJob) and stage tables are built and
// uploaded before anything is enqueued, and a failed factorisation is handled
// on the device (its cells come out invalid), so the enqueue sequence neither
// allocates nor synchronises: the eager call waits once, at its end, and the
// same sequence is captured as one graph for replay.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>

#include "internal.hpp"

using namespace nu;

struct nu_graph {
  int device = 0;
  nu_factor* F = nullptr;
  double* ws = nullptr;
  MemHold hold;  // ws against the context's limit
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

const char* class_timing_name(int c) {
  static const char* names[TC_COUNT] = {"gemm_f64:panel",   "gemm_f64:panel_update", "gemm_f64:trailing",
                                        "gemm_f64:inverse", "gemm_f32:inverse",      "gemm_f64:band",
                                        "gemm_bf16x3:inverse"};
  return names[c];
}

// ---------------------------------------------------------------------------
// A batch cut into waves whose factors fit the memory budget; every wave is
// searched by one launch per stage for all its curves (see CurveJob), its
// factors carved from one arena reused wave after wave. Built on the host
// before anything is enqueued (plans and tables uploaded), so that the
// enqueue sequence itself allocates and synchronises nothing and can be
// captured into a graph.
struct BatchWave {
  std::vector<int> curves;       // caller indices, longest first
  std::vector<nu_factor*> Fs;    // placed in the arena
  std::vector<CurveJob> jobs;    // host copies of the device records
  std::vector<int> begin;        // [BS_COUNT][n + 1]
  std::vector<int> total;        // workgroups per stage
  Plan P, Q;                     // Cholesky; inverse (+ band)
  CurveJob* djobs = nullptr;
  int* dbegin = nullptr;
  int n() const { return (int)curves.size(); }
  const int* b(int stage) const { return dbegin + (size_t)stage * (n() + 1); }
};

struct BatchInputs {
  int n_curves = 0;
  const int64_t *sample_off = nullptr, *epoch_off = nullptr;
  const double *t = nullptr, *f = nullptr, *A = nullptr;
  int m1 = 0;
  const int64_t* lattice = nullptr;
  const nu_sho* theta_dev = nullptr;  // device, one per curve
  const double* dt_host = nullptr;
  const int32_t* dur = nullptr;       // host, caller order
  int n_d = 0;
  const double* periods = nullptr;
  int64_t n_p = 0;
  int prec = 0, sign = 1;
  double *depth = nullptr, *var = nullptr, *dll = nullptr;
  uint8_t* valid = nullptr;
  double *null_out = nullptr, *q_snr = nullptr, *best_depth = nullptr, *best_sigma = nullptr, *best_lnp = nullptr;
  int64_t* best_phase = nullptr;
  int32_t* best_dur = nullptr;
  int64_t* best_index = nullptr;
  int64_t* status_out = nullptr;  // device, one per curve
  double* logdet_out = nullptr;   // device, one per curve
};

struct BatchRun {
  std::vector<BatchWave> waves;
  void* tables = nullptr;    // device: every wave's jobs and begin tables
  double* packed = nullptr;  // device: every curve's packed fold grid (outside the arena)
  std::vector<hipEvent_t> ev_lin, ev_fold;  // per wave: linear search done, fold done
  MemHold hold;                             // tables and grids against the context's limit
  ~BatchRun() {
    hold.release();
    for (auto& w : waves) {
      plan_release(w.P);
      plan_release(w.Q);
      for (nu_factor* F : w.Fs) factor_free(F);
    }
    if (tables) (void)hipFree(tables);
    if (packed) (void)hipFree(packed);
    for (hipEvent_t e : ev_lin) (void)hipEventDestroy(e);
    for (hipEvent_t e : ev_fold) (void)hipEventDestroy(e);
  }
};

int64_t curve_n(const BatchInputs& in, int c) { return in.sample_off[c + 1] - in.sample_off[c]; }
int64_t curve_ne(const BatchInputs& in, int c) { return in.epoch_off[c + 1] - in.epoch_off[c]; }
size_t curve_t_min(const BatchInputs& in, int c) { return batch_search_ws_doubles(curve_n(in, c), in.n_d, curve_ne(in, c)); }
size_t curve_bytes(const BatchInputs& in, int c) { return factor_bytes(curve_n(in, c), in.prec, curve_t_min(in, c)); }

// every curve's packed fold grid and record, held for the whole call outside
// the waves (the records' bound: one wave per curve at most)
size_t batch_grid_bytes(const BatchInputs& in) {
  size_t grids = (size_t)in.n_curves * (sizeof(CurveJob) + 2 * BS_COUNT * sizeof(int) + 512);
  for (int c = 0; c < in.n_curves; ++c) grids += fold_workspace_doubles(in.n_d, curve_ne(in, c)) * sizeof(double);
  return grids;
}

// waves of curves (longest first) whose factors fit `budget` bytes; the arena size they need
nu_status plan_waves(nu_ctx* ctx, const BatchInputs& in, size_t budget, std::vector<std::vector<int>>& waves,
                     size_t& arena_need) {
  std::vector<int> order(in.n_curves);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return curve_n(in, a) > curve_n(in, b); });
  const size_t grids = batch_grid_bytes(in);
  if (grids >= budget)
    return set_error(ctx, NU_ERR_OOM, "search_batch: the fold grids do not fit the device-memory budget");
  budget -= grids;
  size_t used = 0;
  for (int c : order) {
    const size_t need = curve_bytes(in, c);
    if (need > budget)
      return set_error(ctx, NU_ERR_OOM,
                       "search_batch: curve " + std::to_string(c) + " does not fit the device-memory budget");
    if (waves.empty() || used + need > budget) {
      waves.emplace_back();
      used = 0;
    }
    waves.back().push_back(c);
    used += need;
  }
  arena_need = 0;
  for (const auto& w : waves) {
    size_t b = 0;
    for (int c : w) b += curve_bytes(in, c);
    arena_need = std::max(arena_need, b);
  }
  return NU_OK;
}

// factors, records, stage tables and schedules of every wave; uploads them
nu_status build_batch(nu_ctx* ctx, const BatchInputs& in, const std::vector<std::vector<int>>& waves, char* arena,
                      BatchRun& run) {
  const bool mixed = in.prec != NU_FP64;
  const int bw = mixed ? band_width(in.prec) : 0;
  size_t table_bytes = 0;
  run.waves.resize(waves.size());
  for (size_t wi = 0; wi < waves.size(); ++wi) {
    BatchWave& W = run.waves[wi];
    W.curves = waves[wi];
    char* cursor = arena;
    for (int c : W.curves) {
      nu_factor* F = nullptr;
      nu_status st = factor_place(ctx, curve_n(in, c), in.prec, &cursor, &F, curve_t_min(in, c));
      if (st != NU_OK) return st;
      W.Fs.push_back(F);
      CurveJob J{};
      const int64_t s0 = in.sample_off[c], e0 = in.epoch_off[c], cells = (int64_t)in.n_d * e0;
      J.t = in.t + s0;
      J.theta = in.theta_dev + c;
      J.L = F->L;
      J.X = F->X;
      J.L32 = F->L32;
      J.X32 = F->X32;
      J.bandX = F->bandX;
      J.parts = F->parts();
      J.logdet = F->logdet_dev();
      J.status = F->status_dev();
      J.nf = F->nullfit;
      J.n = F->n;
      J.np = F->np;
      J.nblk = F->nblk;
      J.f = in.f + s0;
      J.A = in.m1 > 0 ? in.A + (int64_t)in.m1 * s0 : nullptr;
      J.lattice = in.lattice + s0;
      J.n_epochs = curve_ne(in, c);
      batch_carve_search_ws(J, F->T, in.n_d);
      J.depth = in.depth + cells;
      J.var = in.var + cells;
      J.dll = in.dll + cells;
      J.valid = in.valid + cells;
      J.null_out = in.null_out ? in.null_out + 3 * (int64_t)c : nullptr;
      J.dt = in.dt_host[c];
      J.q_snr = in.q_snr + (int64_t)c * in.n_p;
      J.best_phase = in.best_phase + (int64_t)c * in.n_p;
      J.best_dur = in.best_dur + (int64_t)c * in.n_p;
      J.best_depth = in.best_depth + (int64_t)c * in.n_p;
      J.best_sigma = in.best_sigma + (int64_t)c * in.n_p;
      J.best_lnp = in.best_lnp + (int64_t)c * in.n_p;
      J.best_index = in.best_index ? in.best_index + c : nullptr;
      J.curve = c;
      W.jobs.push_back(J);
    }
    const int n = W.n();
    W.begin.assign((size_t)BS_COUNT * (n + 1), 0);
    W.total.assign(BS_COUNT, 0);
    for (int stg = 0; stg < BS_COUNT; ++stg) {
      int64_t acc = 0;
      for (int i = 0; i < n; ++i) {
        W.begin[(size_t)stg * (n + 1) + i] = (int)acc;
        acc += batch_stage_blocks(stg, W.jobs[i], in.n_d, bw);
      }
      if (acc > INT32_MAX) return set_error(ctx, NU_ERR_ARG, "search_batch: a stage exceeds 2^31 workgroups");
      W.begin[(size_t)stg * (n + 1) + n] = (int)acc;
      W.total[stg] = (int)acc;
    }
    table_bytes += (size_t)n * sizeof(CurveJob) + W.begin.size() * sizeof(int) + 256;
    plan_cholesky(W.Fs, ctx->tuning, W.P);
    nu_status st = plan_upload(ctx, W.P);
    if (st != NU_OK) return st;
    if (mixed) {
      plan_inverse(W.Fs, gemm_kind_of(in.prec), ctx->tuning, W.Q);
      plan_band(W.Fs, bw, ctx->tuning, W.Q);
    } else {
      plan_inverse(W.Fs, GK_F64, ctx->tuning, W.Q);
    }
    st = plan_upload(ctx, W.Q);
    if (st != NU_OK) return st;
  }
  // the packed fold grids live outside the arena, so a wave's fold can run
  // while the next wave's factors overwrite the arena
  size_t packed_doubles = 0;
  for (const BatchWave& W : run.waves)
    for (const CurveJob& J : W.jobs) packed_doubles += fold_workspace_doubles(in.n_d, J.n_epochs);
  nu_status st = ctx_malloc(ctx, (void**)&run.packed, std::max<size_t>(packed_doubles, 1) * sizeof(double), run.hold,
                            "alloc batch fold grids");
  if (st != NU_OK) return st;
  size_t poff = 0;
  for (BatchWave& W : run.waves)
    for (CurveJob& J : W.jobs) {
      J.packed = run.packed + poff;
      poff += fold_workspace_doubles(in.n_d, J.n_epochs);
    }
  if (!ctx->s_fold)  // created here, never under a capture
    st = check_hip(ctx, hipStreamCreateWithFlags(&ctx->s_fold, hipStreamNonBlocking), "fold stream");
  if (st != NU_OK) return st;
  run.ev_lin.assign(run.waves.size(), nullptr);
  run.ev_fold.assign(run.waves.size(), nullptr);
  for (size_t w = 0; st == NU_OK && w < run.waves.size(); ++w) {
    st = check_hip(ctx, hipEventCreateWithFlags(&run.ev_lin[w], hipEventDisableTiming), "batch event");
    if (st == NU_OK) st = check_hip(ctx, hipEventCreateWithFlags(&run.ev_fold[w], hipEventDisableTiming), "batch event");
  }
  if (st != NU_OK) return st;
  st = ctx_malloc(ctx, &run.tables, table_bytes, run.hold, "alloc batch tables");
  if (st != NU_OK) return st;
  std::vector<char> host(table_bytes);
  size_t off = 0;
  for (BatchWave& W : run.waves) {
    const size_t jb = (size_t)W.n() * sizeof(CurveJob);
    std::memcpy(host.data() + off, W.jobs.data(), jb);
    W.djobs = reinterpret_cast<CurveJob*>(static_cast<char*>(run.tables) + off);
    off += jb;
    const size_t bb = W.begin.size() * sizeof(int);
    std::memcpy(host.data() + off, W.begin.data(), bb);
    W.dbegin = reinterpret_cast<int*>(static_cast<char*>(run.tables) + off);
    off = (off + bb + 255) / 256 * 256;
  }
  return check_hip(ctx, hipMemcpy(run.tables, host.data(), table_bytes, hipMemcpyHostToDevice),
                   "upload batch tables");
}

// the stages of one wave, each one launch for all its curves
nu_status enqueue_wave(nu_ctx* ctx, const BatchInputs& in, const BatchWave& W) {
  hipStream_t s = ctx->stream;
  const int n = W.n(), m1 = in.m1, nv = m1 + 1, n_d = in.n_d;
  const bool mixed = in.prec != NU_FP64;
  const int kind = gemm_kind_of(in.prec), steps = refine_steps(in.prec), bw = mixed ? band_width(in.prec) : 0;
  double kflops = 0.0;
  for (const CurveJob& J : W.jobs) kflops += (double)J.n * (double)(J.n + 1) / 2.0;
  nu_status st = check_hip(ctx, launch_batch_init(s, W.djobs, n), "batch init");
  if (st == NU_OK) {
    Timed tm(ctx, "kbuild", kflops);
    st = check_hip(ctx, launch_batch_kbuild(s, W.djobs, W.b(BS_KBUILD), n, W.total[BS_KBUILD]), "kbuild");
  }
  if (st == NU_OK) st = run_factor_steps(ctx, W.P);
  if (st == NU_OK) st = check_hip(ctx, launch_batch_logdet(s, W.djobs, n), "logdet");
  // the triangular inverse
  if (st == NU_OK && mixed) {
    const char* level_name = kind == GK_BF16X3 ? "gemm_bf16x3:inverse" : "gemm_f32:inverse";
    {
      Timed tm(ctx, "convert", 0.0);
      st = check_hip(ctx, launch_batch_cvt_l(s, W.djobs, W.b(BS_CVT_L), n, W.total[BS_CVT_L]), "convert L");
      if (st == NU_OK)
        st = check_hip(ctx, launch_batch_cvt_xd(s, W.djobs, W.b(BS_CVT_XD), n, W.total[BS_CVT_XD]), "convert X");
    }
    for (size_t l = 0; st == NU_OK && l < W.Q.t1.size(); ++l) {
      st = launch_range(ctx, W.Q, W.Q.t1[l], level_name, kind);
      if (st == NU_OK) st = launch_range(ctx, W.Q, W.Q.t2[l], level_name, kind);
    }
    if (st == NU_OK) {
      Timed tm(ctx, "convert", 0.0);
      st = check_hip(ctx, launch_batch_cvt_back(s, W.djobs, W.b(BS_CVT_BACK), n, W.total[BS_CVT_BACK]), "convert X");
    }
    if (st == NU_OK)
      st = check_hip(ctx, launch_batch_band_copy(s, W.djobs, W.b(BS_BAND), n, W.total[BS_BAND], bw, 1), "band copy");
    if (st == NU_OK) st = launch_range(ctx, W.Q, W.Q.bandp, "gemm_f64:band", GK_F64);
    if (st == NU_OK) st = launch_range(ctx, W.Q, W.Q.bandx, "gemm_f64:band", GK_F64);
    if (st == NU_OK)
      st = check_hip(ctx, launch_batch_band_copy(s, W.djobs, W.b(BS_BAND), n, W.total[BS_BAND], bw, 0), "band copy");
  } else if (st == NU_OK) {
    st = run_inverse_fp64(ctx, W.Q);
  }
  // the linear search
  double gemv_bytes = 0.0;
  for (const CurveJob& J : W.jobs) gemv_bytes += (double)J.n * (double)(J.n + 1) / 2.0 * 8.0;
  if (st == NU_OK) st = check_hip(ctx, launch_batch_lattice_check(s, W.djobs, n), "lattice_check");
  if (st == NU_OK) st = check_hip(ctx, launch_batch_pack_v(s, W.djobs, W.b(BS_PACKV), n, W.total[BS_PACKV], m1), "pack_v");
  auto rows = [&](int mat, int vin, int base, double alpha, int out) {
    return check_hip(ctx, launch_batch_rows(s, W.djobs, W.b(BS_ROWS), W.b(BS_ROWS_RED), n, W.total[BS_ROWS],
                                            W.total[BS_ROWS_RED], nv, mat, vin, base, alpha, out),
                     "rows_matvec");
  };
  auto cols = [&](int mat, int win, int base, double alpha, int out) {
    return check_hip(ctx, launch_batch_cols(s, W.djobs, W.b(BS_COLS), W.b(BS_COLS_RED), n, W.total[BS_COLS],
                                            W.total[BS_COLS_RED], nv, mat, win, base, alpha, out),
                     "cols_matvec");
  };
  if (st == NU_OK) {
    Timed tm(ctx, "rows_matvec", gemv_bytes * (1 + 2 * steps));
    st = rows(MS_X, PS_V, PS_NONE, 1.0, PS_Y);
    for (int r = 0; r < steps && st == NU_OK; ++r) {
      st = rows(MS_L, PS_Y, PS_V, -1.0, PS_R);
      if (st == NU_OK) st = rows(MS_X, PS_R, PS_Y, 1.0, PS_Y);
    }
  }
  if (st == NU_OK) {
    Timed tm(ctx, "null_solve", 0.0);
    st = check_hip(ctx, launch_batch_null(s, W.djobs, n, m1), "null_solve");
  }
  if (st == NU_OK) {
    Timed tm(ctx, "cols_matvec", gemv_bytes * (1 + 2 * steps));
    st = cols(MS_X, PS_Y, PS_NONE, 1.0, PS_Z);
    for (int r = 0; r < steps && st == NU_OK; ++r) {
      st = cols(MS_L, PS_Z, PS_Y, -1.0, PS_RZ);
      if (st == NU_OK) st = cols(MS_X, PS_RZ, PS_Z, 1.0, PS_Z);
    }
  }
  std::vector<int32_t> order(n_d), sorted(2 * n_d);
  for (int j = 0; j < n_d; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return in.dur[a] < in.dur[b]; });
  int dmax = 0;
  for (int k = 0; k < n_d; ++k) {
    sorted[k] = in.dur[order[k]];
    sorted[n_d + k] = order[k];
    dmax = std::max(dmax, (int)in.dur[k]);
  }
  if (st == NU_OK) {
    Timed tm(ctx, "q_partial", 0.0);
    st = check_hip(ctx, launch_batch_slot_count(s, W.djobs, W.b(BS_SLOTS), n, W.total[BS_SLOTS]), "slot_count");
    if (st == NU_OK)
      st = check_hip(ctx, launch_batch_q_partial(s, W.djobs, W.b(BS_QPART), n, W.total[BS_QPART], sorted.data(), n_d,
                                                 dmax),
                     "q_partial");
  }
  if (st == NU_OK) {
    Timed tm(ctx, "cell_epilogue", 0.0);
    st = check_hip(ctx, launch_batch_epilogue(s, W.djobs, W.b(BS_EPI), n, W.total[BS_EPI], in.dur, n_d, m1),
                   "cell_epilogue");
  }
  // statuses and ln|K| by curve index, before the next wave overwrites the arena
  if (st == NU_OK)
    st = check_hip(ctx, launch_batch_collect(s, W.djobs, n, in.status_out, in.logdet_out), "batch collect");
  return st;
}

// the periodic search of one wave on stream s (its grids outside the arena)
nu_status enqueue_wave_fold(nu_ctx* ctx, const BatchInputs& in, const BatchWave& W, hipStream_t s) {
  const int n = W.n(), n_d = in.n_d;
  nu_status st;
  {
    double visits = 0.0;
    for (const CurveJob& J : W.jobs) visits += (double)n_d * (double)J.n_epochs * (double)in.n_p;
    Timed tm(ctx, s, "fold", FOLD_FLOPS_PER_VISIT * visits);
    st = check_hip(ctx, launch_batch_fold(s, W.djobs, W.b(BS_FOLD_PACK), n, W.total[BS_FOLD_PACK], n_d, in.periods,
                                          in.n_p, in.sign),
                   "fold");
  }
  if (st == NU_OK) {
    Timed tm(ctx, s, "best_period", 0.0);
    st = check_hip(ctx, launch_batch_best(s, W.djobs, n, in.n_p, in.status_out), "best_period");
  }
  return st;
}

// Every wave: factorisation, inverse and linear search on the context's
// stream; then its periodic search on the fold stream, which runs beside the
// next wave's factorisation (the fold is VALU work, the factorisation matrix-
// core work). The context's stream joins the fold stream at the end.
nu_status enqueue_batch(nu_ctx* ctx, const BatchInputs& in, BatchRun& run) {
  nu_status st = NU_OK;
  bool forked = false;
  for (size_t w = 0; st == NU_OK && w < run.waves.size(); ++w) {
    st = enqueue_wave(ctx, in, run.waves[w]);
    if (st == NU_OK) st = check_hip(ctx, hipEventRecord(run.ev_lin[w], ctx->stream), "batch fork");
    if (st == NU_OK) st = check_hip(ctx, hipStreamWaitEvent(ctx->s_fold, run.ev_lin[w], 0), "batch fork");
    if (st == NU_OK) {
      forked = true;
      st = enqueue_wave_fold(ctx, in, run.waves[w], ctx->s_fold);
    }
    if (st == NU_OK) st = check_hip(ctx, hipEventRecord(run.ev_fold[w], ctx->s_fold), "batch join");
  }
  if (forked) {  // join (also after an error: the caller's stream must not run ahead of the fold stream)
    const size_t last = run.waves.size() - 1;
    nu_status sj = check_hip(ctx, hipEventRecord(run.ev_fold[last], ctx->s_fold), "batch join");
    if (sj == NU_OK) sj = check_hip(ctx, hipStreamWaitEvent(ctx->stream, run.ev_fold[last], 0), "batch join");
    if (st == NU_OK) st = sj;
  }
  return st;
}

nu_status validate_batch(nu_ctx* ctx, int n_curves, const int64_t* sample_off_host, const int64_t* epoch_off_host,
                         const double* t, const double* f, const double* A, int m1, const int64_t* lattice,
                         const double* dt_host, const int32_t* dur_samples_host, int n_d, const double* periods,
                         int64_t n_p, nu_precision prec, int log_term_sign, double* depth, double* var, double* dll,
                         uint8_t* valid, const void* q_snr, const void* best_phase, const void* best_dur,
                         const void* best_depth, const void* best_sigma, const void* best_lnp) {
  if (n_curves < 1) return set_error(ctx, NU_ERR_ARG, "search_batch: n_curves must be >= 1");
  if (!sample_off_host || !epoch_off_host || !t || !dt_host || !periods || !q_snr || !best_phase || !best_dur ||
      !best_depth || !best_sigma || !best_lnp)
    return set_error(ctx, NU_ERR_ARG, "search_batch: null argument");
  if (sample_off_host[0] != 0 || epoch_off_host[0] != 0)
    return set_error(ctx, NU_ERR_ARG, "search_batch: offsets must start at 0");
  for (int c = 0; c < n_curves; ++c) {
    const int64_t n = sample_off_host[c + 1] - sample_off_host[c];
    const int64_t ne = epoch_off_host[c + 1] - epoch_off_host[c];
    if (n < 1 || n > (int64_t)1 << 17)
      return set_error(ctx, NU_ERR_ARG, "search_batch: every curve needs 1 .. 131072 samples");
    nu_status st = validate_linear(ctx, n, f, A, m1, lattice, ne, dur_samples_host, n_d, prec, depth, var, dll, valid);
    if (st == NU_OK) st = validate_periodic(ctx, n_d, ne, dt_host[c], n_p, log_term_sign);
    if (st != NU_OK) return set_error(ctx, st, ctx->last_error + " (curve " + std::to_string(c) + ")");
  }
  return NU_OK;
}

}  // namespace

struct nu_batch_graph {
  int device = 0;
  MemHold hold;             // arena and logdet against the context's limit
  void* arena = nullptr;    // the graph's own factors
  double* logdet = nullptr;  // ln|K| per curve when the caller passes none
  BatchRun run;              // schedules, tables, placed factors
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

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
  if (!theta_host) return set_error(ctx, NU_ERR_ARG, "search_batch: null argument");
  nu_status st = validate_batch(ctx, n_curves, sample_off_host, epoch_off_host, t, f, A, m1, lattice, dt_host,
                                dur_samples_host, n_d, periods, n_p, prec, log_term_sign, depth, var, dll, valid, q_snr,
                                best_phase, best_dur, best_depth, best_sigma, best_lnp);
  if (st != NU_OK) return st;
  for (int c = 0; c < n_curves; ++c) {
    st = validate_theta(ctx, &theta_host[c]);
    if (st != NU_OK) return set_error(ctx, st, ctx->last_error + " (curve " + std::to_string(c) + ")");
  }
  st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;

  BatchInputs in;
  in.n_curves = n_curves;
  in.sample_off = sample_off_host;
  in.epoch_off = epoch_off_host;
  in.t = t;
  in.f = f;
  in.A = A;
  in.m1 = m1;
  in.lattice = lattice;
  in.dt_host = dt_host;
  in.dur = dur_samples_host;
  in.n_d = n_d;
  in.periods = periods;
  in.n_p = n_p;
  in.prec = prec;
  in.sign = log_term_sign;
  in.depth = depth;
  in.var = var;
  in.dll = dll;
  in.valid = valid;
  in.null_out = null_out;
  in.q_snr = q_snr;
  in.best_phase = best_phase;
  in.best_dur = best_dur;
  in.best_depth = best_depth;
  in.best_sigma = best_sigma;
  in.best_lnp = best_lnp;
  in.best_index = best_period_index;

  // per-curve hyperparameters, statuses and ln|K| in the context's workspace
  const size_t small_bytes = (size_t)n_curves * (sizeof(nu_sho) + sizeof(int64_t) + sizeof(double));
  char* small = (char*)ctx_workspace(ctx, small_bytes, &st);
  if (!small) return st;
  in.theta_dev = reinterpret_cast<const nu_sho*>(small);
  in.status_out = reinterpret_cast<int64_t*>(small + (size_t)n_curves * sizeof(nu_sho));
  in.logdet_out = reinterpret_cast<double*>(small + (size_t)n_curves * (sizeof(nu_sho) + sizeof(int64_t)));
  st = ctx_upload(ctx, theta_host, (size_t)n_curves * sizeof(nu_sho), small);
  if (st != NU_OK) return st;

  // the budget counts the arena this context already holds as available
  size_t budget = memory_budget_bytes;
  if (budget == 0) {
    size_t free_b = 0, total_b = 0;
    st = check_hip(ctx, hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    if (st != NU_OK) return st;
    budget = (free_b + ctx->arena_bytes) / 10 * 9;
  }
  budget = std::min(budget, mem_headroom(ctx, ctx->arena_bytes));  // the arena is replaced
  std::vector<std::vector<int>> waves;
  size_t arena_need = 0;
  st = plan_waves(ctx, in, budget, waves, arena_need);
  if (st != NU_OK) return st;
  if (arena_need > ctx->arena_bytes && ctx->arena_bytes > 0) {
    // The budget follows the free memory, so from call to call the first wave
    // can gain a curve and outgrow the arena, whose replacement (a wait, a free
    // and an allocation of up to hundreds of GB) costs seconds. The arena held
    // is kept when a plan within it needs no more waves.
    size_t largest = 0;
    for (int c = 0; c < n_curves; ++c) largest = std::max(largest, curve_bytes(in, c));
    if (largest <= ctx->arena_bytes) {
      std::vector<std::vector<int>> within;
      size_t need = 0;
      if (plan_waves(ctx, in, ctx->arena_bytes + batch_grid_bytes(in), within, need) == NU_OK &&
          within.size() <= waves.size()) {
        waves.swap(within);
        arena_need = need;
      }
    }
  }
  char* arena = nullptr;
  {
    HostTimed ht(ctx, "batch_arena");
    arena = (char*)ctx_arena(ctx, arena_need, &st);
  }
  if (!arena) return st;
  BatchRun run;
  {
    HostTimed ht(ctx, "batch_plan");
    st = build_batch(ctx, in, waves, arena, run);
  }
  if (st == NU_OK) st = enqueue_batch(ctx, in, run);
  std::vector<int64_t> status(n_curves, -1);
  std::vector<double> logdet(n_curves, 0.0);
  if (st == NU_OK) {
    HostTimed ht(ctx, "batch_wait");
    st = check_hip(ctx, hipMemcpyAsync(status.data(), in.status_out, (size_t)n_curves * sizeof(int64_t),
                                       hipMemcpyDeviceToHost, ctx->stream),
                   "read statuses");
    if (st == NU_OK)
      st = check_hip(ctx, hipMemcpyAsync(logdet.data(), in.logdet_out, (size_t)n_curves * sizeof(double),
                                         hipMemcpyDeviceToHost, ctx->stream),
                     "read logdets");
    if (st == NU_OK) st = check_hip(ctx, hipStreamSynchronize(ctx->stream), "batch sync");
  } else {
    (void)hipStreamSynchronize(ctx->stream);  // nothing of the run may be freed while it is queued
  }
  if (st != NU_OK) return st;
  int n_failed = 0, first_failed = -1;
  for (int c = 0; c < n_curves; ++c) {
    if (logdet_host) logdet_host[c] = logdet[c];
    if (fail_pivot_host) fail_pivot_host[c] = status[c];
    if (status[c] >= 0) {
      if (first_failed < 0) first_failed = c;
      ++n_failed;
    }
  }
  if (n_failed > 0)
    return set_error(ctx, NU_ERR_NOT_PD,
                     "search_batch: " + std::to_string(n_failed) + " covariance(s) not positive definite (first: curve " +
                         std::to_string(first_failed) + "); their outputs hold no candidate");
  return NU_OK;
}

// ---------------------------------------------------------------------------
nu_status nu_batch_graph_create(nu_ctx* ctx, int n_curves, const int64_t* sample_off_host,
                                const int64_t* epoch_off_host, const double* t, const double* f, const double* A,
                                int m1, const int64_t* lattice, const nu_sho* theta_dev, const double* dt_host,
                                const int32_t* dur_samples_host, int n_d, const double* periods, int64_t n_p,
                                nu_precision prec, int log_term_sign, size_t memory_budget_bytes, double* depth,
                                double* var, double* dll, uint8_t* valid, double* null_out, double* q_snr,
                                int64_t* best_phase, int32_t* best_dur, double* best_depth, double* best_sigma,
                                double* best_lnp, int64_t* best_period_index, int64_t* status_dev,
                                double* logdet_dev, nu_batch_graph** out) {
  if (!ctx) return NU_ERR_ARG;
  if (!out || !theta_dev || !status_dev) return set_error(ctx, NU_ERR_ARG, "batch_graph_create: null argument");
  *out = nullptr;
  nu_status st = validate_batch(ctx, n_curves, sample_off_host, epoch_off_host, t, f, A, m1, lattice, dt_host,
                                dur_samples_host, n_d, periods, n_p, prec, log_term_sign, depth, var, dll, valid, q_snr,
                                best_phase, best_dur, best_depth, best_sigma, best_lnp);
  if (st != NU_OK) return st;
  st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  nu_batch_graph* g = new (std::nothrow) nu_batch_graph();
  if (!g) return set_error(ctx, NU_ERR_OOM, "batch_graph_create: host allocation");
  g->device = ctx->device;
  auto fail = [&](nu_status e) {
    nu_batch_graph_destroy(g);
    return e;
  };
  BatchInputs in;
  in.n_curves = n_curves;
  in.sample_off = sample_off_host;
  in.epoch_off = epoch_off_host;
  in.t = t;
  in.f = f;
  in.A = A;
  in.m1 = m1;
  in.lattice = lattice;
  in.theta_dev = theta_dev;
  in.dt_host = dt_host;
  in.dur = dur_samples_host;
  in.n_d = n_d;
  in.periods = periods;
  in.n_p = n_p;
  in.prec = prec;
  in.sign = log_term_sign;
  in.depth = depth;
  in.var = var;
  in.dll = dll;
  in.valid = valid;
  in.null_out = null_out;
  in.q_snr = q_snr;
  in.best_phase = best_phase;
  in.best_dur = best_dur;
  in.best_depth = best_depth;
  in.best_sigma = best_sigma;
  in.best_lnp = best_lnp;
  in.best_index = best_period_index;
  in.status_out = status_dev;
  if (!logdet_dev) {
    st = ctx_malloc(ctx, (void**)&g->logdet, (size_t)n_curves * sizeof(double), g->hold, "alloc logdet");
    if (st != NU_OK) return fail(st);
    logdet_dev = g->logdet;
  }
  in.logdet_out = logdet_dev;
  // every allocation happens before the capture: the graph's own arena, schedules and tables
  size_t budget = memory_budget_bytes;
  if (budget == 0) {
    size_t free_b = 0, total_b = 0;
    st = check_hip(ctx, hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    if (st != NU_OK) return fail(st);
    budget = free_b / 10 * 9;
  }
  budget = std::min(budget, mem_headroom(ctx, 0));
  std::vector<std::vector<int>> waves;
  size_t arena_need = 0;
  st = plan_waves(ctx, in, budget, waves, arena_need);
  if (st == NU_OK) st = ctx_malloc(ctx, &g->arena, std::max<size_t>(arena_need, 256), g->hold, "alloc graph arena");
  if (st == NU_OK) st = build_batch(ctx, in, waves, (char*)g->arena, g->run);
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
    const nu_status cst = enqueue_batch(ctx, in, g->run);
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

nu_status nu_batch_graph_launch(nu_ctx* ctx, nu_batch_graph* g) {
  if (!ctx) return NU_ERR_ARG;
  if (!g || !g->exec) return set_error(ctx, NU_ERR_ARG, "batch_graph_launch: null graph");
  if (g->device != ctx->device) return set_error(ctx, NU_ERR_ARG, "batch_graph_launch: graph on another device");
  nu_status st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  return check_hip(ctx, hipGraphLaunch(g->exec, ctx->stream), "batch graph launch");
}

void nu_batch_graph_destroy(nu_batch_graph* g) {
  if (!g) return;
  g->hold.release();
  if (hipSetDevice(g->device) != hipSuccess) {  // the runtime has shut down: host side only
    for (auto& w : g->run.waves) {
      w.P = Plan();
      w.Q = Plan();
      for (nu_factor*& F : w.Fs) {
        F->plan64 = Plan();
        F->plan32 = Plan();
        delete F;
        F = nullptr;
      }
      w.Fs.clear();
    }
    g->run.waves.clear();
    g->run.tables = nullptr;
    g->run.packed = nullptr;
    g->run.ev_lin.clear();
    g->run.ev_fold.clear();
    delete g;
    return;
  }
  (void)hipDeviceSynchronize();
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->arena) (void)hipFree(g->arena);
  if (g->logdet) (void)hipFree(g->logdet);
  delete g;  // the schedules, tables and factor records go with g->run
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
    st = ctx_malloc(ctx, (void**)&g->ws,
                    std::max(linear_ws_bytes(n, n_d, n_epochs), periodic_ws_bytes(n_d, n_epochs)), g->hold,
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
  g->hold.release();
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
  MemHold hold;
  st = ctx_malloc(ctx, (void**)&t_dev, n * sizeof(double), hold, "autotune alloc");
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
  hold.release();
  if (st != NU_OK) return st;
  for (int c = 0; c < TC_COUNT; ++c) ctx->tuning.small_below[c] = best_thr[c];
  return NU_OK;
}

}  // extern "C"
