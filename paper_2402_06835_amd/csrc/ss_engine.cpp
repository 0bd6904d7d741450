// Host side of the state-space linear search (statespace.hip): workspace
// layout and the enqueue sequence of one search.
#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace nu {

// The cells of the dense linear search from the Kalman form of a sum-of-terms
// covariance, with no N x N matrix anywhere.

namespace {
struct SsWs {
  double *V, *Y, *Z, *step, *gain, *Gm, *qbox, *shapes, *chunk, *logdet;
  int64_t* status;
  int* lattice_ok;
  NullFit* nf;
  int32_t* slot_count;
};

// layout of the workspace; with base == nullptr only the size is computed
size_t ss_layout(int64_t n, int J, int ts, int n_d, int64_t n_epochs, double* base, SsWs* w) {
  size_t off = 0;
  auto take = [&](size_t doubles) {
    double* p = base ? base + off : nullptr;
    off += round_up((int64_t)doubles, 32);  // 256-byte aligned pieces
    return p;
  };
  SsWs l{};
  l.V = take((size_t)n * YCOLS);
  l.Y = take((size_t)n * YCOLS);
  l.Z = take((size_t)n * YCOLS);
  l.step = take((size_t)std::max<int64_t>(n - 1, 1) * ts);
  l.gain = take((size_t)n * (J + 1));
  l.Gm = take((size_t)(n + 1) * J * J);
  l.qbox = take((size_t)n_d * n_epochs);
  l.shapes = take(MAX_SHAPE);
  l.chunk = take(ss_chunk_ws_doubles(n, J));
  l.logdet = take(2);
  l.status = reinterpret_cast<int64_t*>(l.logdet + 1);
  l.lattice_ok = reinterpret_cast<int*>(take(1));
  l.nf = reinterpret_cast<NullFit*>(take((sizeof(NullFit) + 7) / 8));
  l.slot_count = reinterpret_cast<int32_t*>(take(((size_t)n_epochs + 2) / 2));
  if (w) *w = l;
  return off * sizeof(double);
}
}  // namespace

size_t linear_ss_ws_bytes(int64_t n, const nu_kernel& k, int n_d, int64_t n_epochs) {
  return ss_layout(n, 2 * k.n_sho + k.n_exp, 7 * k.n_sho + 2 * k.n_exp, n_d, n_epochs, nullptr, nullptr);
}

nu_status run_linear_ss(nu_ctx* ctx, const double* t, int64_t n, const nu_kernel& k, const double* f, const double* A,
                        int m1, const int64_t* lattice, int64_t n_epochs, const int32_t* dur_samples_host, int n_d,
                        const double* shapes_host, double* depth, double* var, double* dll, uint8_t* valid,
                        double* null_out, double* ws, int64_t** status_dev) {
  const int J = 2 * k.n_sho + k.n_exp, ts = 7 * k.n_sho + 2 * k.n_exp;
  SsWs w{};
  ss_layout(n, J, ts, n_d, n_epochs, ws, &w);
  if (status_dev) *status_dev = w.status;
  SsArgs a;
  a.n_sho = k.n_sho;
  a.n_exp = k.n_exp;
  a.n = n;
  a.kernel = k;
  a.step = w.step;
  a.gain = w.gain;
  a.Gm = w.Gm;
  a.logdet = w.logdet;
  a.status = w.status;
  a.V = w.V;
  a.Y = w.Y;
  a.Z = w.Z;
  a.nv = m1 + 1;
  a.lattice = lattice;
  a.slot_count = w.slot_count;
  a.n_epochs = n_epochs;
  a.n_d = n_d;
  a.dur = dur_samples_host;
  a.shapes = shapes_host ? w.shapes : nullptr;
  a.qbox = w.qbox;
  a.chunk = w.chunk;
  const bool chunked = ss_chunked_applies(k);
  // ascending durations (the boxes of one start are nested) with their caller indices
  std::vector<int32_t> order(n_d);
  for (int j = 0; j < n_d; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return dur_samples_host[x] < dur_samples_host[y]; });
  std::vector<int32_t> sorted(2 * n_d);
  for (int j = 0; j < n_d; ++j) {
    sorted[j] = dur_samples_host[order[j]];
    sorted[n_d + j] = order[j];
  }
  a.dur_sorted = sorted.data();
  nu_status st = NU_OK;
  if (shapes_host) {
    size_t total = 0;
    for (int j = 0; j < n_d; ++j) total += (size_t)dur_samples_host[j];
    st = ctx_upload(ctx, shapes_host, total * sizeof(double), w.shapes);
    if (st != NU_OK) return st;
  }
  st = check_hip(ctx, launch_lattice_check(ctx->stream, lattice, n, n_epochs, w.lattice_ok), "lattice_check");
  if (st == NU_OK) st = check_hip(ctx, launch_pack_v(ctx->stream, A, m1, f, n, w.V), "pack_v");
  if (st != NU_OK) return st;
  {
    Timed tm(ctx, "ss_step", 0.0);
    st = check_hip(ctx, launch_ss_step(ctx->stream, t, n, k, w.step), "ss_step");
  }
  if (st != NU_OK) return st;
  {
    Timed tm(ctx, "ss_riccati", 0.0);
    st = check_hip(ctx, launch_ss(chunked ? SS_PAR_RICCATI : SS_RICCATI, ctx->stream, a), "ss_riccati");
  }
  if (st != NU_OK) return st;
  {
    Timed tm(ctx, "ss_forward", 0.0);
    st = check_hip(ctx, launch_ss(chunked ? SS_PAR_FORWARD : SS_FORWARD, ctx->stream, a), "ss_forward");
  }
  if (st != NU_OK) return st;
  {
    Timed tm(ctx, "null_solve", 0.0);
    st = check_hip(ctx, launch_null_solve(ctx->stream, w.Y, n, m1, w.logdet, w.lattice_ok, w.nf, null_out), "null_solve");
  }
  if (st != NU_OK) return st;
  {
    Timed tm(ctx, "ss_backward", 0.0);
    st = check_hip(ctx, launch_ss(chunked ? SS_PAR_BACKWARD : SS_BACKWARD, ctx->stream, a), "ss_backward");
  }
  if (st != NU_OK) return st;
  {
    Timed tm(ctx, "ss_box", 0.0);
    st = check_hip(ctx, launch_slot_count(ctx->stream, lattice, n, n_epochs, w.slot_count), "slot_count");
    if (st == NU_OK)
      st = check_hip(ctx, launch_ss(shapes_host ? SS_TEMPLATE : SS_BOX, ctx->stream, a),
                     shapes_host ? "ss_template" : "ss_box");
  }
  if (st != NU_OK) return st;
  Timed tm(ctx, "cell_epilogue", 0.0);
  return check_hip(ctx, launch_cell_epilogue(ctx->stream, w.qbox, 1, lattice, w.slot_count, n, n_epochs,
                                             dur_samples_host, n_d, w.Z, m1, w.nf, depth, var, dll, valid, a.shapes),
                   "cell_epilogue");
}

}  // namespace nu
