// C ABI of the learned warm start and of the hyperparameter fit it seeds:
// the GP sampler, the trend-profiled likelihood, the plain start, BFGS, and
// the CNN object (parameters, Adam state, activations).
//
// The fit (maximum likelihood of the trend-only model of Eq. 5 with the trend
// solved linearly, Section 3.2) runs BFGS on x = (ln amp, ln P_rot, ln Q,
// ln sigma_w) for all curves in lockstep: every likelihood evaluation of an
// iteration (the central-difference gradient, each line-search trial) is one
// launch of the Kalman-filter kernel over all (curve, theta) pairs; the
// 4 x 4 BFGS updates are host arithmetic.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "internal.hpp"
#include "learned.hpp"

using namespace nu;

struct nu_cnn {
  int device = 0;
  bool half = false;
  int max_batch = 0;
  int64_t n = 0;
  float* p = nullptr;        // FP32 master parameters
  _Float16* p16 = nullptr;   // FP16 copy (half mode)
  float* m = nullptr;        // Adam moments
  float* v = nullptr;
  float* g = nullptr;        // gradient
  float* loss = nullptr;     // device scalar of the last step
  CnnBuffers buf{};
  void* arena = nullptr;     // activations and scratch
  MemHold hold;              // the arena against the context's limit
  int64_t step = 0;
};

namespace {

constexpr double LOG_BOUNDS[4][2] = {{-12.0, 0.0},      // amp in [6e-6, 1]
                                     {-4.0, 4.0},       // P_rot in [0.018, 55] time units
                                     {-0.6, 9.2},       // Q in [0.55, 1e4]
                                     {-14.0, -1.0}};    // sigma_w in [8e-7, 0.37]

nu_sho theta_of(const double* x) {
  const double amp = std::exp(x[0]), prot = std::exp(x[1]), q = std::exp(x[2]), sw = std::exp(x[3]);
  const double om = q > 0.5 ? 4.0 * M_PI * q / (prot * std::sqrt(4.0 * q * q - 1.0)) : 2.0 * M_PI / prot;
  return nu_sho{amp, om, q, sw};
}

double clampd(double v, double lo, double hi) { return std::min(hi, std::max(lo, v)); }

struct FitCurve {
  double x[4], f, g[4], H[16];
  int iters = 0, evals = 0;
  bool done = false;
};

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
nu_status nu_gp_sample(nu_ctx* ctx, const double* t, int64_t n, int n_curves, const nu_sho* theta, uint64_t seed,
                       uint64_t curve_base, int n_bins, double* flux, float* input, float* target,
                       nu_sho* theta_out) {
  if (!ctx) return NU_ERR_ARG;
  if (!t || n < 2 || n_curves < 1) return set_error(ctx, NU_ERR_ARG, "gp_sample: need t, n >= 2, n_curves >= 1");
  if (input && (n_bins < 1 || n_bins > 512))
    return set_error(ctx, NU_ERR_ARG, "gp_sample: n_bins must be in [1, 512]");
  if (!flux && !input && !target && !theta_out) return set_error(ctx, NU_ERR_ARG, "gp_sample: no output requested");
  nu_status st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  double* bm = nullptr;
  if (input) {
    bm = (double*)ctx_workspace(ctx, (size_t)n_curves * n_bins * sizeof(double), &st);
    if (!bm) return st;
  }
  Timed tm(ctx, "gp_sample", (double)n_curves * (double)n);
  return check_hip(ctx, launch_gp_sample(ctx->stream, t, n, n_curves, theta, seed, curve_base, input ? n_bins : 0,
                                         flux, bm, theta_out, target, input),
                   "gp_sample");
}

// ---------------------------------------------------------------------------
nu_status nu_gp_nll(nu_ctx* ctx, int n_curves, const int64_t* sample_off, const double* t, const double* f,
                    const double* A, int m1, const nu_sho* theta, int n_eval, double* nll) {
  if (!ctx) return NU_ERR_ARG;
  if (n_curves < 1 || n_eval < 1 || !sample_off || !t || !f || !theta || !nll)
    return set_error(ctx, NU_ERR_ARG, "gp_nll: null argument or empty batch");
  if (m1 < 0 || m1 > MAX_M1 || (m1 > 0 && !A)) return set_error(ctx, NU_ERR_ARG, "gp_nll: m1 in [0, 7] with A");
  nu_status st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  Timed tm(ctx, "kalman_nll", (double)n_curves * n_eval);
  return check_hip(ctx, launch_kalman_nll(ctx->stream, t, f, A, m1, sample_off, n_curves, theta, n_eval, nll),
                   "kalman_nll");
}

// ---------------------------------------------------------------------------
nu_status nu_plain_init(nu_ctx* ctx, int n_curves, const int64_t* sample_off, const double* t, const double* f,
                        const double* prot_grid, int n_grid, double* x0) {
  if (!ctx) return NU_ERR_ARG;
  if (n_curves < 1 || n_grid < 1 || !sample_off || !t || !f || !prot_grid || !x0)
    return set_error(ctx, NU_ERR_ARG, "plain_init: null argument or empty input");
  nu_status st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  double* ws = (double*)ctx_workspace(ctx, ((size_t)n_curves * 3 + (size_t)n_curves * n_grid) * sizeof(double), &st);
  if (!ws) return st;
  Timed tm(ctx, "plain_init", 0.0);
  return check_hip(ctx, launch_plain_init(ctx->stream, t, f, sample_off, n_curves, prot_grid, n_grid, ws,
                                          ws + 3 * n_curves, x0),
                   "plain_init");
}

// ---------------------------------------------------------------------------
nu_status nu_fit_hyper(nu_ctx* ctx, int n_curves, const int64_t* sample_off_host, const double* t, const double* f,
                       const double* A, int m1, const double* x0_host, int max_iter, double gtol, double* x_host,
                       double* nll_host, int32_t* n_eval_host, int32_t* iters_host) {
  if (!ctx) return NU_ERR_ARG;
  if (n_curves < 1 || !sample_off_host || !t || !f || !x0_host || !x_host || max_iter < 0 || !(gtol > 0.0))
    return set_error(ctx, NU_ERR_ARG, "fit_hyper: null argument, empty batch, max_iter < 0 or gtol <= 0");
  if (m1 < 0 || m1 > MAX_M1 || (m1 > 0 && !A)) return set_error(ctx, NU_ERR_ARG, "fit_hyper: m1 in [0, 7] with A");
  nu_status st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  const int NE = 9;  // centre + central differences in 4 coordinates
  const double h = 1e-4;
  // device buffers: offsets, thetas, results
  const size_t off_b = (size_t)(n_curves + 1) * sizeof(int64_t);
  const size_t th_b = (size_t)n_curves * NE * sizeof(nu_sho);
  const size_t nl_b = (size_t)n_curves * NE * sizeof(double);
  char* ws = (char*)ctx_workspace(ctx, off_b + th_b + nl_b + 512, &st);
  if (!ws) return st;
  int64_t* d_off = (int64_t*)ws;
  nu_sho* d_th = (nu_sho*)(ws + ((off_b + 255) / 256) * 256);
  double* d_nll = (double*)((char*)d_th + ((th_b + 255) / 256) * 256);
  st = check_hip(ctx, hipMemcpyAsync(d_off, sample_off_host, off_b, hipMemcpyHostToDevice, ctx->stream), "offsets");
  if (st != NU_OK) return st;
  std::vector<nu_sho> th((size_t)n_curves * NE);
  std::vector<double> nl((size_t)n_curves * NE);

  // evaluate NLL at the first `ne` thetas of every curve (rows with fewer used pad with the centre)
  auto evaluate = [&](int ne) -> nu_status {
    nu_status s2 = check_hip(ctx, hipMemcpyAsync(d_th, th.data(), (size_t)n_curves * ne * sizeof(nu_sho),
                                                 hipMemcpyHostToDevice, ctx->stream),
                             "thetas");
    if (s2 == NU_OK) {
      Timed tm(ctx, "kalman_nll", (double)n_curves * ne);
      s2 = check_hip(ctx, launch_kalman_nll(ctx->stream, t, f, A, m1, d_off, n_curves, d_th, ne, d_nll), "kalman_nll");
    }
    if (s2 == NU_OK)
      s2 = check_hip(ctx, hipMemcpyAsync(nl.data(), d_nll, (size_t)n_curves * ne * sizeof(double),
                                         hipMemcpyDeviceToHost, ctx->stream),
                     "nll");
    if (s2 == NU_OK) s2 = check_hip(ctx, hipStreamSynchronize(ctx->stream), "fit sync");
    return s2;
  };
  auto clampx = [&](double* x) {
    for (int k = 0; k < 4; ++k) x[k] = clampd(x[k], LOG_BOUNDS[k][0], LOG_BOUNDS[k][1]);
  };

  // NU_TRACE_FIT=1 prints every curve's iterations to stderr (a debugging aid)
  const bool trace = std::getenv("NU_TRACE_FIT") != nullptr;
  std::vector<FitCurve> C(n_curves);
  // value and gradient at the current points of the curves in `which`
  auto value_and_grad = [&](std::vector<int>& which) -> nu_status {
    for (int c = 0; c < n_curves; ++c) {
      const FitCurve& fc = C[c];
      for (int e = 0; e < NE; ++e) {
        double x[4] = {fc.x[0], fc.x[1], fc.x[2], fc.x[3]};
        if (e > 0) x[(e - 1) / 2] += ((e - 1) % 2 == 0 ? h : -h);
        th[(size_t)c * NE + e] = theta_of(x);
      }
    }
    nu_status s2 = evaluate(NE);
    if (s2 != NU_OK) return s2;
    for (int c : which) {
      FitCurve& fc = C[c];
      fc.f = nl[(size_t)c * NE];
      for (int k = 0; k < 4; ++k) fc.g[k] = (nl[(size_t)c * NE + 1 + 2 * k] - nl[(size_t)c * NE + 2 + 2 * k]) / (2 * h);
      fc.evals += NE;
    }
    return NU_OK;
  };

  std::vector<int> all(n_curves);
  for (int c = 0; c < n_curves; ++c) {
    all[c] = c;
    std::memcpy(C[c].x, x0_host + 4 * c, sizeof(double) * 4);
    clampx(C[c].x);
    for (int k = 0; k < 16; ++k) C[c].H[k] = (k % 5 == 0) ? 1e-4 : 0.0;  // start: a short scaled-gradient step
  }
  st = value_and_grad(all);
  if (st != NU_OK) return st;
  for (FitCurve& fc : C) {
    const double gmax = std::max({std::fabs(fc.g[0]), std::fabs(fc.g[1]), std::fabs(fc.g[2]), std::fabs(fc.g[3])});
    fc.done = !(gmax > gtol) || !std::isfinite(fc.f);
    // first inverse-Hessian guess: unit step along the gradient direction
    const double gn = std::sqrt(fc.g[0] * fc.g[0] + fc.g[1] * fc.g[1] + fc.g[2] * fc.g[2] + fc.g[3] * fc.g[3]);
    if (gn > 0.0)
      for (int k = 0; k < 4; ++k) fc.H[5 * k] = 0.1 / gn;
  }
  for (int it = 0; it < max_iter; ++it) {
    std::vector<int> act;
    for (int c = 0; c < n_curves; ++c)
      if (!C[c].done) act.push_back(c);
    if (act.empty()) break;
    // direction p = -H g, backtracking line search (Armijo), all active curves per launch
    std::vector<double> p((size_t)n_curves * 4, 0.0), alpha(n_curves, 1.0), xn((size_t)n_curves * 4);
    std::vector<char> accepted(n_curves, 0);
    for (int c : act) {
      FitCurve& fc = C[c];
      double slope = 0.0;
      for (int a = 0; a < 4; ++a) {
        double v = 0.0;
        for (int b = 0; b < 4; ++b) v -= fc.H[a * 4 + b] * fc.g[b];
        p[4 * c + a] = v;
        slope += v * fc.g[a];
      }
      if (!(slope < 0.0)) {  // not a descent direction: restart from the scaled gradient
        const double gn = std::sqrt(fc.g[0] * fc.g[0] + fc.g[1] * fc.g[1] + fc.g[2] * fc.g[2] + fc.g[3] * fc.g[3]);
        for (int k = 0; k < 16; ++k) fc.H[k] = (k % 5 == 0) ? 0.1 / gn : 0.0;
        for (int a = 0; a < 4; ++a) p[4 * c + a] = -fc.H[5 * a] * fc.g[a];
      }
    }
    for (int trial = 0; trial < 30; ++trial) {
      bool any = false;
      for (int c = 0; c < n_curves; ++c) {
        // curves still searching get a new trial point; the others keep theirs (or their current x)
        if (!C[c].done && !accepted[c]) {
          double x[4];
          std::memcpy(x, C[c].x, sizeof x);
          for (int a = 0; a < 4; ++a) x[a] += alpha[c] * p[4 * c + a];
          clampx(x);
          std::memcpy(&xn[4 * c], x, sizeof x);
          any = true;
        } else if (!accepted[c]) {
          std::memcpy(&xn[4 * c], C[c].x, sizeof C[c].x);
        }
        th[c] = theta_of(&xn[4 * c]);
      }
      if (!any) break;
      st = evaluate(1);
      if (st != NU_OK) return st;
      for (int c : act) {
        if (accepted[c]) continue;
        FitCurve& fc = C[c];
        fc.evals += 1;
        double dec = 0.0;
        for (int a = 0; a < 4; ++a) dec += (xn[4 * c + a] - fc.x[a]) * fc.g[a];
        if (std::isfinite(nl[c]) && nl[c] <= fc.f + 1e-4 * dec) accepted[c] = 1;
        else alpha[c] *= 0.5;
      }
    }
    std::vector<double> xold((size_t)n_curves * 4), gold((size_t)n_curves * 4), fold(n_curves);
    for (int c : act) {
      FitCurve& fc = C[c];
      std::memcpy(&xold[4 * c], fc.x, sizeof fc.x);
      std::memcpy(&gold[4 * c], fc.g, sizeof fc.g);
      fold[c] = fc.f;
      if (accepted[c]) std::memcpy(fc.x, &xn[4 * c], sizeof fc.x);
      else fc.done = true;  // no decrease along the direction: converged to the evaluation noise
    }
    st = value_and_grad(act);
    if (st != NU_OK) return st;
    for (int c : act) {
      FitCurve& fc = C[c];
      fc.iters += 1;
      if (!accepted[c]) {
        if (trace) std::fprintf(stderr, "[fit] curve %d iter %d: line search found no decrease\n", c, fc.iters);
        std::memcpy(fc.x, &xold[4 * c], sizeof fc.x);
        fc.f = fold[c];
        std::memcpy(fc.g, &gold[4 * c], sizeof fc.g);
        continue;
      }
      double s[4], y[4], sy = 0.0;
      for (int a = 0; a < 4; ++a) {
        s[a] = fc.x[a] - xold[4 * c + a];
        y[a] = fc.g[a] - gold[4 * c + a];
        sy += s[a] * y[a];
      }
      if (sy > 1e-12) {  // BFGS update of the inverse Hessian
        double Hy[4], yHy = 0.0;
        for (int a = 0; a < 4; ++a) {
          Hy[a] = 0.0;
          for (int b = 0; b < 4; ++b) Hy[a] += fc.H[a * 4 + b] * y[b];
          yHy += y[a] * Hy[a];
        }
        const double r = 1.0 / sy;
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b)
            fc.H[a * 4 + b] += (1.0 + yHy * r) * r * s[a] * s[b] - r * (Hy[a] * s[b] + s[a] * Hy[b]);
      }
      const double gmax = std::max({std::fabs(fc.g[0]), std::fabs(fc.g[1]), std::fabs(fc.g[2]), std::fabs(fc.g[3])});
      if (!(gmax > gtol) || std::fabs(fold[c] - fc.f) <= 1e-12 * std::max(1.0, std::fabs(fc.f))) fc.done = true;
      if (trace)
        std::fprintf(stderr, "[fit] curve %d iter %d f %.10g (was %.10g) gmax %.3g alpha %.3g sy %.3g done %d\n", c,
                     fc.iters, fc.f, fold[c], gmax, alpha[c], sy, (int)fc.done);
    }
  }
  for (int c = 0; c < n_curves; ++c) {
    std::memcpy(x_host + 4 * c, C[c].x, sizeof C[c].x);
    if (nll_host) nll_host[c] = C[c].f;
    if (n_eval_host) n_eval_host[c] = C[c].evals;
    if (iters_host) iters_host[c] = C[c].iters;
  }
  return NU_OK;
}

// ---------------------------------------------------------------------------
int64_t nu_cnn_param_count(void) { return cnn_param_count(); }

nu_status nu_cnn_create(nu_ctx* ctx, int half_precision, int max_batch, nu_cnn** out) {
  if (!ctx) return NU_ERR_ARG;
  if (!out || max_batch < 1 || max_batch > 65536)
    return set_error(ctx, NU_ERR_ARG, "cnn_create: need out and 1 <= max_batch <= 65536");
  *out = nullptr;
  nu_status st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != NU_OK) return st;
  nu_cnn* M = new (std::nothrow) nu_cnn();
  if (!M) return set_error(ctx, NU_ERR_OOM, "cnn_create: host allocation");
  M->device = ctx->device;
  M->half = half_precision != 0;
  M->max_batch = max_batch;
  M->n = cnn_param_count();
  const int64_t n = M->n;
  // one allocation: parameters, FP16 copy, Adam moments, gradient, loss, activations, partials
  std::vector<size_t> sizes = {(size_t)n * 4, (size_t)n * 2, (size_t)n * 4, (size_t)n * 4, (size_t)n * 4, 256};
  for (int l = 0; l < CNN_LAYERS; ++l) sizes.push_back((size_t)max_batch * CNN_CH * (CNN_IN >> (l + 1)) * 4);
  for (int l = 0; l < CNN_LAYERS; ++l) sizes.push_back((size_t)max_batch * CNN_CH * (CNN_IN >> (l + 1)) * 4);
  const size_t nchunks = (size_t)(max_batch + CNN_WCHUNK - 1) / CNN_WCHUNK;
  sizes.push_back((size_t)max_batch * CNN_CH * 4);
  sizes.push_back((size_t)max_batch * CNN_OUT * 4);
  sizes.push_back((size_t)max_batch * CNN_OUT * 4);
  sizes.push_back((size_t)max_batch * 4);
  sizes.push_back(nchunks * CNN_CH * CNN_CH * CNN_KW * 4);
  size_t total = 0;
  for (size_t& sz : sizes) {
    sz = (sz + 255) / 256 * 256;
    total += sz;
  }
  st = ctx_malloc(ctx, &M->arena, total, M->hold, "alloc cnn");
  if (st == NU_OK) st = check_hip(ctx, hipMemset(M->arena, 0, total), "clear cnn");
  if (st != NU_OK) {
    nu_cnn_destroy(M);
    return st;
  }
  char* p = (char*)M->arena;
  size_t i = 0;
  auto take = [&]() {
    char* r = p;
    p += sizes[i++];
    return r;
  };
  M->p = (float*)take();
  M->p16 = (_Float16*)take();
  M->m = (float*)take();
  M->v = (float*)take();
  M->g = (float*)take();
  M->loss = (float*)take();
  for (int l = 0; l < CNN_LAYERS; ++l) M->buf.y[l] = (float*)take();
  for (int l = 0; l < CNN_LAYERS; ++l) M->buf.dz[l] = (float*)take();
  M->buf.h = (float*)take();
  M->buf.out = (float*)take();
  M->buf.dO = (float*)take();
  M->buf.sq = (float*)take();
  M->buf.part = (float*)take();
  *out = M;
  return NU_OK;
}

void nu_cnn_destroy(nu_cnn* M) {
  if (!M) return;
  M->hold.release();
  if (hipSetDevice(M->device) != hipSuccess) {  // the runtime has shut down: host side only
    delete M;
    return;
  }
  (void)hipDeviceSynchronize();
  if (M->arena) (void)hipFree(M->arena);
  delete M;
}

nu_status nu_cnn_set_params(nu_ctx* ctx, nu_cnn* M, const float* params_host) {
  if (!ctx) return NU_ERR_ARG;
  if (!M || !params_host) return set_error(ctx, NU_ERR_ARG, "cnn_set_params: null argument");
  nu_status st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st == NU_OK)
    st = check_hip(ctx, hipMemcpy(M->p, params_host, (size_t)M->n * 4, hipMemcpyHostToDevice), "upload params");
  if (st == NU_OK) st = check_hip(ctx, launch_to_half(ctx->stream, M->p, M->p16, M->n), "to half");
  // fresh Adam state
  if (st == NU_OK) st = check_hip(ctx, hipMemset(M->m, 0, (size_t)M->n * 4), "clear m");
  if (st == NU_OK) st = check_hip(ctx, hipMemset(M->v, 0, (size_t)M->n * 4), "clear v");
  if (st == NU_OK) st = check_hip(ctx, hipStreamSynchronize(ctx->stream), "set params sync");
  M->step = 0;
  return st;
}

nu_status nu_cnn_init(nu_ctx* ctx, nu_cnn* M, uint64_t seed) {
  if (!ctx) return NU_ERR_ARG;
  if (!M) return set_error(ctx, NU_ERR_ARG, "cnn_init: null model");
  nu_status st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st == NU_OK) st = check_hip(ctx, launch_cnn_init(ctx->stream, M->p, M->n, seed), "cnn init");
  if (st == NU_OK) st = check_hip(ctx, launch_to_half(ctx->stream, M->p, M->p16, M->n), "to half");
  if (st == NU_OK) st = check_hip(ctx, hipMemsetAsync(M->m, 0, (size_t)M->n * 4, ctx->stream), "clear m");
  if (st == NU_OK) st = check_hip(ctx, hipMemsetAsync(M->v, 0, (size_t)M->n * 4, ctx->stream), "clear v");
  M->step = 0;
  return st;
}

nu_status nu_cnn_get_params(nu_ctx* ctx, nu_cnn* M, float* params_host) {
  if (!ctx) return NU_ERR_ARG;
  if (!M || !params_host) return set_error(ctx, NU_ERR_ARG, "cnn_get_params: null argument");
  nu_status st = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st == NU_OK)
    st = check_hip(ctx, hipMemcpyAsync(params_host, M->p, (size_t)M->n * 4, hipMemcpyDeviceToHost, ctx->stream),
                   "download params");
  if (st == NU_OK) st = check_hip(ctx, hipStreamSynchronize(ctx->stream), "get params sync");
  return st;
}

static nu_status cnn_check(nu_ctx* ctx, nu_cnn* M, const float* input, int batch, const char* what) {
  if (!ctx) return NU_ERR_ARG;
  if (!M || !input) return set_error(ctx, NU_ERR_ARG, std::string(what) + ": null argument");
  if (batch < 1 || batch > M->max_batch)
    return set_error(ctx, NU_ERR_ARG, std::string(what) + ": batch must be in [1, max_batch]");
  if (M->device != ctx->device) return set_error(ctx, NU_ERR_ARG, std::string(what) + ": model on another device");
  return check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
}

nu_status nu_cnn_forward(nu_ctx* ctx, nu_cnn* M, const float* input, int batch, float* out, double* x_log) {
  nu_status st = cnn_check(ctx, M, input, batch, "cnn_forward");
  if (st != NU_OK) return st;
  float* o = out ? out : M->buf.out;
  {
    Timed tm(ctx, "cnn_forward", 0.0);
    st = check_hip(ctx, launch_cnn_forward(ctx->stream, M->buf, M->p, M->p16, M->half, input, batch, o), "cnn fwd");
  }
  if (st == NU_OK && x_log)
    st = check_hip(ctx, launch_outputs_to_log(ctx->stream, o, batch, nullptr, x_log), "to log");
  return st;
}

nu_status nu_warm_start(nu_ctx* ctx, nu_cnn* M, const float* input, int batch, const double* x_plain,
                        double* x_out) {
  nu_status st = cnn_check(ctx, M, input, batch, "warm_start");
  if (st != NU_OK) return st;
  if (!x_plain || !x_out) return set_error(ctx, NU_ERR_ARG, "warm_start: null argument");
  {
    Timed tm(ctx, "cnn_forward", 0.0);
    st = check_hip(ctx, launch_cnn_forward(ctx->stream, M->buf, M->p, M->p16, M->half, input, batch, M->buf.out),
                   "cnn fwd");
  }
  if (st == NU_OK)
    st = check_hip(ctx, launch_outputs_to_log(ctx->stream, M->buf.out, batch, x_plain, x_out), "warm start");
  return st;
}

nu_status nu_cnn_gradient(nu_ctx* ctx, nu_cnn* M, const float* input, const float* target, int batch, float* grad,
                          float* loss) {
  nu_status st = cnn_check(ctx, M, input, batch, "cnn_gradient");
  if (st != NU_OK) return st;
  if (!target) return set_error(ctx, NU_ERR_ARG, "cnn_gradient: null target");
  Timed tm(ctx, "cnn_train", 0.0);
  st = check_hip(ctx, launch_cnn_forward(ctx->stream, M->buf, M->p, M->p16, M->half, input, batch, M->buf.out),
                 "cnn fwd");
  if (st == NU_OK)
    st = check_hip(ctx, launch_cnn_backward(ctx->stream, M->buf, M->p, M->p16, M->half, input, target, batch,
                                            grad ? grad : M->g, loss ? loss : M->loss),
                   "cnn bwd");
  return st;
}

nu_status nu_cnn_train_step(nu_ctx* ctx, nu_cnn* M, const float* input, const float* target, int batch, float lr,
                            float* loss) {
  nu_status st = nu_cnn_gradient(ctx, M, input, target, batch, M ? M->g : nullptr, loss);
  if (st != NU_OK) return st;
  if (!(lr > 0.f)) return set_error(ctx, NU_ERR_ARG, "cnn_train_step: lr must be > 0");
  M->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)M->step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)M->step)));
  Timed tm(ctx, "adam", 0.0);
  return check_hip(ctx, launch_adam(ctx->stream, M->p, M->p16, M->g, M->m, M->v, M->n, lr, b1, b2, 1e-8f, c1, c2),
                   "adam");
}

}  // extern "C"
