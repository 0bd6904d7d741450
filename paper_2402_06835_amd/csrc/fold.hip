// Periodic search (Sections 2.3-2.4): fold of the single-event grid over
// phases, common-depth combination (Eq. 8 with the estimates of Eq. B4), the
// argmax of Eq. 9 and Q(P) = depth / sigma; then the best period.
//
// One workgroup per trial period; thread = phase m of one duration j at a
// time. Consecutive threads read consecutive epoch slots m + floor(k p), so
// each event gather is one coalesced segment per wave. Interpolation and the
// sums are evaluated exactly as written (this file is compiled without
// floating-point contraction), in increasing k.
#include "internal.hpp"

namespace nu {

struct Best {
  double val;    // lnP
  int64_t flat;  // m * n_d + j
  double dep, s2;
};

// true if a beats b: larger lnP, ties to the smaller flat index
__device__ __forceinline__ bool beats(const Best& a, const Best& b) {
  if (a.flat < 0) return false;
  if (b.flat < 0) return true;
  return a.val > b.val || (a.val == b.val && a.flat < b.flat);
}

// event k of phase m: slot position m + k p; returns false when outside the grid
struct Ev {
  double d, v, l;
  bool use;
};

__device__ __forceinline__ bool event_at(const double* __restrict__ D, const double* __restrict__ V,
                                         const double* __restrict__ LL, const uint8_t* __restrict__ ok, int64_t n_t,
                                         int64_t m, double kp, bool need_l, Ev& e) {
  const double base = floor(kp);
  const int64_t i0 = m + (int64_t)base;
  if (i0 > n_t - 1) return false;  // this and every later event lie past the grid
  const double w = kp - base;
  e.use = false;
  if (w == 0.0) {
    if (ok[i0]) {
      e.d = D[i0];
      e.v = V[i0];
      e.l = need_l ? LL[i0] : 0.0;
      e.use = true;
    }
  } else if (i0 + 1 <= n_t - 1 && ok[i0] && ok[i0 + 1]) {
    const double u = 1.0 - w;
    e.d = u * D[i0] + w * D[i0 + 1];
    e.v = u * V[i0] + w * V[i0 + 1];
    e.l = need_l ? u * LL[i0] + w * LL[i0 + 1] : 0.0;
    e.use = true;
  }
  return true;
}

__global__ __launch_bounds__(256) void fold_kernel(const double* __restrict__ depth, const double* __restrict__ var,
                                                   const double* __restrict__ dll, const uint8_t* __restrict__ valid,
                                                   int n_d, int64_t n_t, double dt,
                                                   const double* __restrict__ periods, double sign,
                                                   double* __restrict__ q_snr, int64_t* __restrict__ best_phase,
                                                   int32_t* __restrict__ best_dur, double* __restrict__ best_depth,
                                                   double* __restrict__ best_sigma, double* __restrict__ best_lnp) {
  __shared__ Best red[256];
  const int64_t ip = blockIdx.x;
  const int tid = threadIdx.x;
  const double P = periods[ip];
  const double p = P / dt;
  Best best{-INFINITY, -1, 0.0, 0.0};
  // periods below one cadence or absurdly long are reported as having no event
  if (p >= 1.0 && p <= 1e15) {
    const double nph_d = ceil(p);
    const int64_t nph = nph_d < (double)n_t ? (int64_t)nph_d : n_t;  // phases >= n_t hold no event
    for (int j = 0; j < n_d; ++j) {
      const double* D = depth + (int64_t)j * n_t;
      const double* V = var + (int64_t)j * n_t;
      const double* LL = dll + (int64_t)j * n_t;
      const uint8_t* OK = valid + (int64_t)j * n_t;
      for (int64_t mb = 0; mb < nph; mb += 256) {
        const int64_t m = mb + tid;
        if (m >= nph) continue;
        // pass 1: Eq. B4 estimates and the sum of single-event log-likelihood gains
        double s_w = 0.0, s_wd = 0.0, s_ll = 0.0;
        int64_t cnt = 0;
        for (int64_t k = 0;; ++k) {
          Ev e;
          if (!event_at(D, V, LL, OK, n_t, m, (double)k * p, true, e)) break;
          if (e.use) {
            s_w = s_w + 1.0 / e.v;
            s_wd = s_wd + e.d / e.v;
            s_ll = s_ll + e.l;
            ++cnt;
          }
        }
        if (cnt == 0) continue;
        const double s2 = 1.0 / s_w;
        const double dc = s2 * s_wd;
        // pass 2: the common-depth terms of Eq. 8
        double corr = 0.0;
        for (int64_t k = 0;; ++k) {
          Ev e;
          if (!event_at(D, V, LL, OK, n_t, m, (double)k * p, false, e)) break;
          if (e.use) {
            const double dd = e.d - dc;
            const double term = sign * (log(e.v) - log(s2 + e.v)) + dd * dd / (e.v + s2);
            corr = corr + term;
          }
        }
        const double lnp = s_ll - 0.5 * corr;
        Best cand{lnp, m * (int64_t)n_d + j, dc, s2};
        if (lnp == lnp && lnp > -INFINITY && beats(cand, best)) best = cand;
      }
    }
  }
  red[tid] = best;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off && beats(red[tid + off], red[tid])) red[tid] = red[tid + off];
    __syncthreads();
  }
  if (tid == 0) {
    const Best b = red[0];
    if (b.flat >= 0) {
      const double s = sqrt(b.s2);
      q_snr[ip] = b.dep / s;
      best_phase[ip] = b.flat / n_d;
      best_dur[ip] = (int32_t)(b.flat % n_d);
      best_depth[ip] = b.dep;
      best_sigma[ip] = s;
      best_lnp[ip] = b.val;
    } else {
      q_snr[ip] = 0.0;
      best_phase[ip] = -1;
      best_dur[ip] = -1;
      best_depth[ip] = 0.0;
      best_sigma[ip] = 0.0;
      best_lnp[ip] = -INFINITY;
    }
  }
}

hipError_t launch_fold(hipStream_t s, const double* depth, const double* var, const double* dll,
                       const uint8_t* valid, int n_d, int64_t n_epochs, double dt, const double* periods, int64_t n_p,
                       int sign, double* q_snr, int64_t* best_phase, int32_t* best_dur, double* best_depth,
                       double* best_sigma, double* best_lnp) {
  hipLaunchKernelGGL(fold_kernel, dim3((unsigned)n_p), dim3(256), 0, s, depth, var, dll, valid, n_d, n_epochs, dt,
                     periods, (double)sign, q_snr, best_phase, best_dur, best_depth, best_sigma, best_lnp);
  return hipGetLastError();
}

// First period of largest Q (NaN never wins).
__global__ __launch_bounds__(1024) void best_period_kernel(const double* __restrict__ q, int64_t n_p,
                                                           int64_t* __restrict__ out) {
  __shared__ double rv[1024];
  __shared__ int64_t ri[1024];
  const int tid = threadIdx.x;
  double bv = -INFINITY;
  int64_t bi = -1;
  for (int64_t i = tid; i < n_p; i += 1024) {
    const double v = q[i];
    if (v > bv) {  // indices rise within a thread: strict > keeps the first
      bv = v;
      bi = i;
    }
  }
  rv[tid] = bv;
  ri[tid] = bi;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (tid < off) {
      const double v = rv[tid + off];
      const int64_t i = ri[tid + off];
      if (i >= 0 && (ri[tid] < 0 || v > rv[tid] || (v == rv[tid] && i < ri[tid]))) {
        rv[tid] = v;
        ri[tid] = i;
      }
    }
    __syncthreads();
  }
  if (tid == 0) *out = ri[0];
}

hipError_t launch_best_period(hipStream_t s, const double* q_snr, int64_t n_p, int64_t* out) {
  hipLaunchKernelGGL(best_period_kernel, dim3(1), dim3(1024), 0, s, q_snr, n_p, out);
  return hipGetLastError();
}

}  // namespace nu
