// The hyperparameter fit the search needs first (maximum likelihood of the
// trend-only model of Eq. 5 with the trend solved linearly, Section 3.2) and
// the learned warm start for it:
//
//   gp_sample_kernel      training curves drawn from the SHO process (exact
//                         discretisation of the oscillator's state-space
//                         model, Appendix A) plus white noise, random numbers
//                         from Philox-4x32-10 (Salmon et al., SC'11); the bin
//                         means of each curve are accumulated on the fly
//   bin_normalise_kernel  CNN input: bin means over their median, minus one,
//                         times 100 (empty bins 0); median by a bitonic sort
//   kalman_nll_kernel     -ln L_0 for many (curve, theta) pairs: the Kalman
//                         filter's innovations whiten [A | f] (prediction-
//                         error decomposition), two passes (trend fit, then
//                         the residual) so chi^2 does not cancel
//   lomb_scargle_kernel,  the plain start: Lomb-Scargle power over a period
//   moments_kernel,       grid, its first argmax, std(f) and the rms of
//   plain_init_kernel     second differences
//   conv_*_kernel         the CNN's stride-2 width-7 convolutions as implicit
//                         GEMMs on the matrix cores (FP16 inputs with FP32
//                         accumulation, or FP32), forward, input gradient
//                         (with the previous ReLU's mask) and weight gradient
//   head_*_kernel         global average pool, linear head, squared error
//   adam_kernel           Adam, writing the FP16 copy of the weights
#include <algorithm>
#include <cmath>

#include "internal.hpp"
#include "learned.hpp"

namespace nu {

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Philox-4x32-10 and normals

struct U4 {
  uint32_t v[4];
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return U4{{c0, c1, c2, c3}};
}

// strictly inside (0, 1): k < 2^52 from the top 26 bits of two words, (k + 1/2) 2^-52
__device__ __forceinline__ double uniform01(uint32_t a, uint32_t b) {
  return ((double)(a >> 6) * 67108864.0 + (double)(b >> 6) + 0.5) * (1.0 / 4503599627370496.0);
}

// Box-Muller of the two uniforms of one draw
__device__ __forceinline__ void normal_pair(const U4& w, double& z0, double& z1) {
  const double u1 = uniform01(w.v[0], w.v[1]);
  const double u2 = uniform01(w.v[2], w.v[3]);
  const double r = sqrt(-2.0 * log(u1));
  double s, c;
  sincos(2.0 * M_PI * u2, &s, &c);
  z0 = r * c;
  z1 = r * s;
}

__device__ __forceinline__ U4 draw(uint64_t n, uint64_t curve, uint32_t stream, uint64_t seed) {
  return philox((uint32_t)n, (uint32_t)curve, (uint32_t)(curve >> 32), stream, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// ---------------------------------------------------------------------------
// SHO state-space model: x'' + (omega/Q) x' + omega^2 x = white forcing, with
// stationary covariance Pinf = diag(amp^2, amp^2 omega^2). Over a step h the
// state moves by Phi = exp(F h) = e^{-a h} [[C + a S, S], [-omega^2 S, C - a S]],
// a = omega / 2Q, with C = cos(b h), S = sin(b h)/b (b^2 = omega^2 - a^2, Q > 1/2),
// C = 1, S = h (Q = 1/2), C = cosh(b h), S = sinh(b h)/b (b^2 = a^2 - omega^2,
// Q < 1/2), and the process noise of the step is Qd = Pinf - Phi Pinf Phi^T.

struct Step {
  double p00, p01, p10, p11;  // Phi
  double q00, q01, q11;       // Qd
};

__device__ Step sho_step(double amp, double om, double q, double h) {
  const double a = om / (2.0 * q);
  double C, S;
  if (q == 0.5) {
    C = 1.0;
    S = h;
  } else if (q > 0.5) {
    const double b = om * sqrt(1.0 - 1.0 / (4.0 * q * q));
    double sn, cs;
    sincos(b * h, &sn, &cs);
    C = cs;
    S = sn / b;
  } else {
    const double b = om * sqrt(1.0 / (4.0 * q * q) - 1.0);
    C = cosh(b * h);
    S = sinh(b * h) / b;
  }
  const double e = exp(-a * h);
  Step st;
  st.p00 = e * (C + a * S);
  st.p01 = e * S;
  st.p10 = -e * om * om * S;
  st.p11 = e * (C - a * S);
  const double v0 = amp * amp, v1 = amp * amp * om * om;
  st.q00 = v0 - (st.p00 * st.p00 * v0 + st.p01 * st.p01 * v1);
  st.q01 = -(st.p00 * st.p10 * v0 + st.p01 * st.p11 * v1);
  st.q11 = v1 - (st.p10 * st.p10 * v0 + st.p11 * st.p11 * v1);
  return st;
}

__device__ __forceinline__ double omega_from_rotation(double prot, double q) {
  return q > 0.5 ? 4.0 * M_PI * q / (prot * sqrt(4.0 * q * q - 1.0)) : 2.0 * M_PI / prot;
}

__device__ __forceinline__ double rotation_from_omega(double om, double q) {
  return q > 0.5 ? 4.0 * M_PI * q / (om * sqrt(4.0 * q * q - 1.0)) : 2.0 * M_PI / om;
}

// ---------------------------------------------------------------------------
// Sampler: one thread per curve, samples in time order, bin means on the fly.

__global__ __launch_bounds__(64) void gp_sample_kernel(const double* __restrict__ t, int64_t n, int n_curves,
                                                       const nu_sho* __restrict__ theta_in, uint64_t seed,
                                                       uint64_t curve_base, int n_bins,
                                                       double* __restrict__ flux, double* __restrict__ bin_mean,
                                                       nu_sho* __restrict__ theta_out, float* __restrict__ target) {
  const int c = blockIdx.x * 64 + threadIdx.x;
  if (c >= n_curves) return;
  const uint64_t curve = curve_base + (uint64_t)c;
  double amp, om, q, sw, prot;
  if (theta_in) {
    const nu_sho th = theta_in[c];
    amp = th.amp;
    om = th.omega;
    q = th.q;
    sw = th.sigma_w;
    prot = rotation_from_omega(om, q);
  } else {
    const U4 w0 = draw(0, curve, STREAM_THETA, seed), w1 = draw(1, curve, STREAM_THETA, seed);
    const uint32_t w[8] = {w0.v[0], w0.v[1], w0.v[2], w0.v[3], w1.v[0], w1.v[1], w1.v[2], w1.v[3]};
    double v[4];
    for (int i = 0; i < 4; ++i) {
      const double lo = log(prior_lo(i)), hi = log(prior_hi(i));
      v[i] = exp(lo + uniform01(w[2 * i], w[2 * i + 1]) * (hi - lo));
    }
    amp = v[0];
    prot = v[1];
    q = v[2];
    sw = v[3];
    om = omega_from_rotation(prot, q);
  }
  if (theta_out) theta_out[c] = nu_sho{amp, om, q, sw};
  if (target) {
    const double v[4] = {amp, prot, q, sw};
    for (int i = 0; i < 4; ++i) {
      const double lo = log(prior_lo(i)), hi = log(prior_hi(i));
      target[(int64_t)c * 4 + i] = (float)((log(v[i]) - 0.5 * (lo + hi)) / ((hi - lo) / sqrt(12.0)));
    }
  }
  double* bm = bin_mean ? bin_mean + (int64_t)c * n_bins : nullptr;
  if (bm)
    for (int b = 0; b < n_bins; ++b) bm[b] = NAN;
  const double t0 = t[0], span = t[n - 1] - t[0];
  double z0, z1;
  normal_pair(draw(0, curve, STREAM_INITIAL, seed), z0, z1);
  double x0 = amp * z0, x1 = amp * om * z1;
  double hprev = -1.0;
  Step st{};
  double c00 = 0.0, c10 = 0.0, c11 = 0.0;
  int cur = -1;
  double s = 0.0, cnt = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double ti = t[i];
    if (i > 0) {
      const double h = ti - t[i - 1];
      if (h != hprev) {
        st = sho_step(amp, om, q, h);
        c00 = sqrt(fmax(st.q00, 0.0));
        c10 = c00 > 0.0 ? st.q01 / c00 : 0.0;
        c11 = sqrt(fmax(st.q11 - c10 * c10, 0.0));
        hprev = h;
      }
      double za, zb;
      normal_pair(draw(i, curve, STREAM_PROCESS, seed), za, zb);
      const double n0 = st.p00 * x0 + st.p01 * x1 + c00 * za;
      const double n1 = st.p10 * x0 + st.p11 * x1 + (c10 * za + c11 * zb);
      x0 = n0;
      x1 = n1;
    }
    double zw, unused;
    normal_pair(draw(i, curve, STREAM_WHITE, seed), zw, unused);
    const double f = 1.0 + x0 + sw * zw;
    if (flux) flux[(int64_t)c * n + i] = f;
    if (bm) {
      const int b = min(n_bins - 1, (int)floor((ti - t0) / span * n_bins));
      if (b != cur) {
        if (cur >= 0) bm[cur] = s / cnt;
        cur = b;
        s = 0.0;
        cnt = 0.0;
      }
      s += f;
      cnt += 1.0;
    }
  }
  if (bm && cur >= 0) bm[cur] = s / cnt;
}

// One workgroup per curve: median of the non-empty bin means (bitonic sort of
// 512 keys, empty bins last), then the normalised input.
__global__ __launch_bounds__(256) void bin_normalise_kernel(const double* __restrict__ bin_mean, int n_bins,
                                                            float* __restrict__ input) {
  __shared__ double key[512];
  __shared__ int count;
  const int c = blockIdx.x, tid = threadIdx.x;
  const double* bm = bin_mean + (int64_t)c * n_bins;
  if (tid == 0) count = 0;
  __syncthreads();
  int mine = 0;
  for (int i = tid; i < 512; i += 256) {
    const double v = i < n_bins ? bm[i] : NAN;
    const bool ok = !isnan(v);
    key[i] = ok ? v : INFINITY;
    mine += ok;
  }
  atomicAdd(&count, mine);  // integer count: order-independent
  for (int k = 2; k <= 512; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      __syncthreads();
      for (int i = tid; i < 512; i += 256) {
        const int p = i ^ j;
        if (p > i) {
          const bool up = (i & k) == 0;
          const double a = key[i], b = key[p];
          if ((a > b) == up) {
            key[i] = b;
            key[p] = a;
          }
        }
      }
    }
  __syncthreads();
  const int m = count;
  const double med = m == 0 ? 1.0 : ((m & 1) ? key[m / 2] : (key[m / 2 - 1] + key[m / 2]) / 2.0);
  for (int i = tid; i < n_bins; i += 256) {
    const double v = bm[i];
    input[(int64_t)c * n_bins + i] = isnan(v) ? 0.0f : (float)(100.0 * (v / med - 1.0));
  }
}

hipError_t launch_gp_sample(hipStream_t s, const double* t, int64_t n, int n_curves, const nu_sho* theta_in,
                            uint64_t seed, uint64_t curve_base, int n_bins, double* flux, double* bin_mean,
                            nu_sho* theta_out, float* target, float* input) {
  hipLaunchKernelGGL(gp_sample_kernel, dim3((unsigned)((n_curves + 63) / 64)), dim3(64), 0, s, t, n, n_curves,
                     theta_in, seed, curve_base, n_bins, flux, bin_mean, theta_out, target);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !input) return e;
  hipLaunchKernelGGL(bin_normalise_kernel, dim3((unsigned)n_curves), dim3(256), 0, s, bin_mean, n_bins, input);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Trend-profiled likelihood by the Kalman filter, one thread per (curve, theta).

struct Filter {
  double P00, P01, P11;
  double amp, om, q, sw2;
  double hprev;
  Step st;
  __device__ void start(const nu_sho& th) {
    amp = th.amp;
    om = th.omega;
    q = th.q;
    sw2 = th.sigma_w * th.sigma_w;
    P00 = amp * amp;
    P01 = 0.0;
    P11 = amp * amp * om * om;
    hprev = -1.0;
  }
  // predict the covariance over a step h (the means are moved by the caller with st)
  __device__ void predict(double h) {
    if (h != hprev) {
      st = sho_step(amp, om, q, h);
      hprev = h;
    }
    const double a00 = st.p00 * P00 + st.p01 * P01, a01 = st.p00 * P01 + st.p01 * P11;
    const double a10 = st.p10 * P00 + st.p11 * P01, a11 = st.p10 * P01 + st.p11 * P11;
    P00 = a00 * st.p00 + a01 * st.p01 + st.q00;
    P01 = a00 * st.p10 + a01 * st.p11 + st.q01;
    P11 = a10 * st.p10 + a11 * st.p11 + st.q11;
  }
  // innovation variance, then the covariance update with gain (P00, P01) / S
  __device__ double update() {
    const double S = P00 + sw2;
    const double k0 = P00 / S, k1 = P01 / S;
    const double n00 = P00 - k0 * P00, n01 = P01 - k0 * P01, n11 = P11 - k1 * P01;
    P00 = n00;
    P01 = n01;
    P11 = n11;
    return S;
  }
};

// M1 trend columns (a template parameter, so the per-thread state stays in registers)
template <int M1>
__global__ __launch_bounds__(64) void kalman_nll_kernel(const double* __restrict__ t, const double* __restrict__ f,
                                                        const double* __restrict__ A,
                                                        const int64_t* __restrict__ off, int n_curves,
                                                        const nu_sho* __restrict__ theta, int n_eval,
                                                        double* __restrict__ nll) {
  constexpr int KC = M1 + 1;  // columns [A | f]
  const int idx = blockIdx.x * 64 + threadIdx.x;
  if (idx >= n_curves * n_eval) return;
  const int c = idx / n_eval;
  const int64_t s0 = off[c], n = off[c + 1] - s0;
  const double* tc = t + s0;
  const double* fc = f + s0;
  const double* Ac = M1 > 0 ? A + (int64_t)M1 * s0 : nullptr;
  const nu_sho th = theta[idx];
  Filter F;
  // pass 1: whitened Gram of [A | f] and ln|K|
  F.start(th);
  double x0[KC], x1[KC], G[KC * (KC + 1) / 2];
#pragma unroll
  for (int j = 0; j < KC; ++j) x0[j] = x1[j] = 0.0;
#pragma unroll
  for (int j = 0; j < KC * (KC + 1) / 2; ++j) G[j] = 0.0;
  double logdet = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (i > 0) {
      F.predict(tc[i] - tc[i - 1]);
#pragma unroll
      for (int j = 0; j < KC; ++j) {
        const double a = F.st.p00 * x0[j] + F.st.p01 * x1[j], b = F.st.p10 * x0[j] + F.st.p11 * x1[j];
        x0[j] = a;
        x1[j] = b;
      }
    }
    const double P00 = F.P00, P01 = F.P01;
    const double S = F.update();
    const double rs = 1.0 / sqrt(S);
    logdet += log(S);
    double w[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) {
      const double y = j < M1 ? Ac[(int64_t)j * n + i] : fc[i];
      const double e = y - x0[j];
      w[j] = e * rs;
      x0[j] += P00 / S * e;
      x1[j] += P01 / S * e;
    }
#pragma unroll
    for (int a = 0; a < KC; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) G[a * (a + 1) / 2 + b] = fma(w[a], w[b], G[a * (a + 1) / 2 + b]);
  }
  // trend coefficients from the Gram: G_AA w = G_Af (Cholesky)
  double Lc[M1 > 0 ? M1 * M1 : 1], wt[M1 > 0 ? M1 : 1];
  bool ok = true;
#pragma unroll
  for (int a = 0; a < M1; ++a) {
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      double v = G[a * (a + 1) / 2 + b];
#pragma unroll
      for (int k = 0; k < b; ++k) v -= Lc[a * M1 + k] * Lc[b * M1 + k];
      if (a == b) {
        ok = ok && v > 0.0;
        Lc[a * M1 + a] = sqrt(fmax(v, 1e-300));
      } else {
        Lc[a * M1 + b] = v / Lc[b * M1 + b];
      }
    }
  }
#pragma unroll
  for (int a = 0; a < M1; ++a) {
    double v = G[M1 * (M1 + 1) / 2 + a];
#pragma unroll
    for (int k = 0; k < a; ++k) v -= Lc[a * M1 + k] * wt[k];
    wt[a] = v / Lc[a * M1 + a];
  }
#pragma unroll
  for (int a = M1 - 1; a >= 0; --a) {
    double v = wt[a];
#pragma unroll
    for (int k = a + 1; k < M1; ++k) v -= Lc[k * M1 + a] * wt[k];
    wt[a] = v / Lc[a * M1 + a];
  }
  // pass 2: chi^2 of the residual r = f - A w, whitened by the same filter
  F.start(th);
  double r0 = 0.0, r1 = 0.0, chi2 = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (i > 0) {
      F.predict(tc[i] - tc[i - 1]);
      const double a = F.st.p00 * r0 + F.st.p01 * r1, b = F.st.p10 * r0 + F.st.p11 * r1;
      r0 = a;
      r1 = b;
    }
    double y = fc[i];
#pragma unroll
    for (int j = 0; j < M1; ++j) y -= Ac[(int64_t)j * n + i] * wt[j];
    const double P00 = F.P00, P01 = F.P01;
    const double S = F.update();
    const double e = y - r0;
    chi2 += e * e / S;
    r0 += P00 / S * e;
    r1 += P01 / S * e;
  }
  nll[idx] = ok ? 0.5 * chi2 + 0.5 * logdet + 0.5 * (double)n * log(2.0 * M_PI) : INFINITY;
}

hipError_t launch_kalman_nll(hipStream_t s, const double* t, const double* f, const double* A, int m1,
                             const int64_t* off, int n_curves, const nu_sho* theta, int n_eval, double* nll) {
  const int total = n_curves * n_eval;
  const dim3 g((unsigned)((total + 63) / 64)), b(64);
  switch (m1) {
    case 0: hipLaunchKernelGGL(kalman_nll_kernel<0>, g, b, 0, s, t, f, A, off, n_curves, theta, n_eval, nll); break;
    case 1: hipLaunchKernelGGL(kalman_nll_kernel<1>, g, b, 0, s, t, f, A, off, n_curves, theta, n_eval, nll); break;
    case 2: hipLaunchKernelGGL(kalman_nll_kernel<2>, g, b, 0, s, t, f, A, off, n_curves, theta, n_eval, nll); break;
    case 3: hipLaunchKernelGGL(kalman_nll_kernel<3>, g, b, 0, s, t, f, A, off, n_curves, theta, n_eval, nll); break;
    case 4: hipLaunchKernelGGL(kalman_nll_kernel<4>, g, b, 0, s, t, f, A, off, n_curves, theta, n_eval, nll); break;
    case 5: hipLaunchKernelGGL(kalman_nll_kernel<5>, g, b, 0, s, t, f, A, off, n_curves, theta, n_eval, nll); break;
    case 6: hipLaunchKernelGGL(kalman_nll_kernel<6>, g, b, 0, s, t, f, A, off, n_curves, theta, n_eval, nll); break;
    case 7: hipLaunchKernelGGL(kalman_nll_kernel<7>, g, b, 0, s, t, f, A, off, n_curves, theta, n_eval, nll); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The plain start: moments, Lomb-Scargle power, first argmax over the grid.

// one workgroup per curve: mean, std (population), rms of second differences
__global__ __launch_bounds__(256) void moments_kernel(const double* __restrict__ f, const int64_t* __restrict__ off,
                                                      double* __restrict__ mom) {
  __shared__ double red[256];
  const int c = blockIdx.x, tid = threadIdx.x;
  const int64_t s0 = off[c], n = off[c + 1] - s0;
  const double* fc = f + s0;
  auto block_sum = [&](double v) {
    red[tid] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) red[tid] += red[tid + o];
      __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
  };
  double a = 0.0;
  for (int64_t i = tid; i < n; i += 256) a += fc[i];
  const double mean = block_sum(a) / (double)n;
  double v = 0.0, d = 0.0;
  for (int64_t i = tid; i < n; i += 256) {
    const double e = fc[i] - mean;
    v += e * e;
    if (i >= 1 && i + 1 < n) {
      const double d2 = fc[i + 1] - 2.0 * fc[i] + fc[i - 1];
      d += d2 * d2;
    }
  }
  const double var = block_sum(v) / (double)n;
  const double dd = block_sum(d) / (double)max<int64_t>(n - 2, 1);
  if (tid == 0) {
    mom[3 * c + 0] = mean;
    mom[3 * c + 1] = sqrt(var);
    mom[3 * c + 2] = sqrt(dd / 6.0);
  }
}

// one thread per (curve, trial period): the classic Lomb-Scargle power with the
// time offset tau that decouples the sine and cosine terms, on y = f - mean
__global__ __launch_bounds__(256) void lomb_scargle_kernel(const double* __restrict__ t, const double* __restrict__ f,
                                                           const int64_t* __restrict__ off,
                                                           const double* __restrict__ mom,
                                                           const double* __restrict__ prot, int n_grid,
                                                           double* __restrict__ power) {
  const int c = blockIdx.y;
  const int g = blockIdx.x * 256 + threadIdx.x;
  if (g >= n_grid) return;
  const int64_t s0 = off[c], n = off[c + 1] - s0;
  const double* tc = t + s0;
  const double* fc = f + s0;
  const double w = 2.0 * M_PI / prot[g];
  const double mean = mom[3 * c];
  double cc = 0.0, cs = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double s, co;
    sincos(w * tc[i], &s, &co);
    cc += co * co;
    cs += co * s;
  }
  const double inv = 1.0 / (double)n;
  cc *= inv;
  cs *= inv;
  const double tau = 0.5 * atan2(2.0 * cs, cc - (1.0 - cc));
  double yc = 0.0, ys = 0.0, c2 = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double s, co;
    sincos(w * tc[i] - tau, &s, &co);
    const double y = fc[i] - mean;
    yc += y * co;
    ys += y * s;
    c2 += co * co;
  }
  yc *= inv;
  ys *= inv;
  c2 *= inv;
  const double eps = 1.1102230246251565e-16;
  const double C2 = fmax(c2, eps), S2 = fmax(1.0 - c2, eps);
  power[(int64_t)c * n_grid + g] = 2.0 * (yc * yc / C2 + ys * ys / S2) * (double)n / 4.0;
}

// one workgroup per curve: first argmax of the power -> x0 = ln(std, prot, 5, sigma_w)
__global__ __launch_bounds__(256) void plain_init_kernel(const double* __restrict__ power, int n_grid,
                                                         const double* __restrict__ prot,
                                                         const double* __restrict__ mom, double* __restrict__ x0) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  const int c = blockIdx.x, tid = threadIdx.x;
  double v = -INFINITY;
  int i0 = n_grid;
  for (int g = tid; g < n_grid; g += 256) {
    const double p = power[(int64_t)c * n_grid + g];
    if (p > v) {
      v = p;
      i0 = g;
    }
  }
  bv[tid] = v;
  bi[tid] = i0;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o && (bv[tid + o] > bv[tid] || (bv[tid + o] == bv[tid] && bi[tid + o] < bi[tid]))) {
      bv[tid] = bv[tid + o];
      bi[tid] = bi[tid + o];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int g = bi[0] < n_grid ? bi[0] : 0;
    x0[4 * c + 0] = log(mom[3 * c + 1]);
    x0[4 * c + 1] = log(prot[g]);
    x0[4 * c + 2] = log(5.0);
    x0[4 * c + 3] = log(mom[3 * c + 2]);
  }
}

hipError_t launch_plain_init(hipStream_t s, const double* t, const double* f, const int64_t* off, int n_curves,
                             const double* prot, int n_grid, double* mom, double* power, double* x0) {
  hipLaunchKernelGGL(moments_kernel, dim3((unsigned)n_curves), dim3(256), 0, s, f, off, mom);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lomb_scargle_kernel, dim3((unsigned)((n_grid + 255) / 256), (unsigned)n_curves), dim3(256), 0, s,
                     t, f, off, mom, prot, n_grid, power);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(plain_init_kernel, dim3((unsigned)n_curves), dim3(256), 0, s, power, n_grid, prot, mom, x0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CNN: convolutions as implicit GEMMs on the matrix cores.
//
// Activations are FP32 [batch][channel][position]; the weights of a layer are
// [64][c_in * 7] (output channel, then input channel and tap). A workgroup of
// 4 waves computes a 64 x 64 output tile; wave w owns rows 16w..16w+15 as four
// 16 x 16 MFMA accumulators. K runs over chunks of 16 channels x 7 taps staged
// in LDS, converted to the element type T of the products (FP16 with FP32
// accumulation, or FP32).

template <typename T>
struct CM;
template <>
struct CM<float> {
  static constexpr int KS = 4, KPL = 1;  // k per step, k per lane
  static __device__ __forceinline__ flt4 op(const float* a, const float* b, flt4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
  }
};
template <>
struct CM<_Float16> {
  static constexpr int KS = 16, KPL = 4;
  static __device__ __forceinline__ flt4 op(const _Float16* a, const _Float16* b, flt4 c) {
    const half4 av = {a[0], a[1], a[2], a[3]};
    const half4 bv = {b[0], b[1], b[2], b[3]};
    return __builtin_amdgcn_mfma_f32_16x16x16f16(av, bv, c, 0, 0, 0);
  }
};

constexpr int CW = CNN_CH;       // channels of every convolution's output
constexpr int KW = CNN_KW;       // taps
constexpr int PADW = 3;          // zero padding each side
constexpr int CCH = 16;          // input channels per K chunk
constexpr int KCP = CCH * KW;    // 112, a multiple of 16
constexpr int LT = 64;           // positions per tile
constexpr int XW = 2 * LT + 6;   // input window of a tile of outputs (134)

// y[b][co][l] = relu(bias[co] + sum_{ci,k} W[co][ci*7+k] x[b][ci][2l+k-3])
template <typename T>
__global__ __launch_bounds__(256) void conv_fwd_kernel(const float* __restrict__ x, const T* __restrict__ W,
                                                       const float* __restrict__ bias, float* __restrict__ y,
                                                       int cin, int lin, int lout) {
  typedef CM<T> M;
  __shared__ T Ws[CW][KCP + 4];
  __shared__ T Xs[CCH][XW];
  const int b = blockIdx.y, l0 = blockIdx.x * LT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  flt4 acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = flt4{0.f, 0.f, 0.f, 0.f};
  for (int c0 = 0; c0 < cin; c0 += CCH) {
    const int cc = min(CCH, cin - c0), kc = cc * KW;
    const int kp = (kc + M::KS - 1) / M::KS * M::KS;
    __syncthreads();
    for (int e = tid; e < CW * kp; e += 256) {
      const int co = e / kp, k = e - co * kp;
      Ws[co][k] = k < kc ? W[(int64_t)co * cin * KW + c0 * KW + k] : T(0);
    }
    for (int e = tid; e < cc * XW; e += 256) {
      const int ci = e / XW, p = e - ci * XW;
      const int j = 2 * l0 - PADW + p;
      Xs[ci][p] = (j >= 0 && j < lin) ? T(x[((int64_t)b * cin + c0 + ci) * lin + j]) : T(0);
    }
    __syncthreads();
    for (int ks = 0; ks < kp; ks += M::KS) {
      T a[M::KPL];
#pragma unroll
      for (int j = 0; j < M::KPL; ++j) a[j] = Ws[wave * 16 + lr][ks + lq * M::KPL + j];
#pragma unroll
      for (int lb = 0; lb < 4; ++lb) {
        T bv[M::KPL];
#pragma unroll
        for (int j = 0; j < M::KPL; ++j) {
          const int k = ks + lq * M::KPL + j;
          bv[j] = k < kc ? Xs[k / KW][2 * (lb * 16 + lr) + k % KW] : T(0);
        }
        acc[lb] = M::op(a, bv, acc[lb]);
      }
    }
  }
#pragma unroll
  for (int lb = 0; lb < 4; ++lb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = wave * 16 + 4 * lq + i, l = l0 + lb * 16 + lr;
      if (l < lout) y[((int64_t)b * CW + co) * lout + l] = fmaxf(acc[lb][i] + bias[co], 0.f);
    }
}

// dzp[b][ci][j] = [yp[b][ci][j] > 0] sum_{co,k : 2l+k-3 = j} W[co][ci*7+k] dz[b][co][l]
// (the input gradient of a layer times the mask of the previous layer's ReLU)
template <typename T>
__global__ __launch_bounds__(256) void conv_bwd_data_kernel(const float* __restrict__ dz, const T* __restrict__ W,
                                                            const float* __restrict__ yp, float* __restrict__ dzp,
                                                            int lin, int lout) {
  typedef CM<T> M;
  constexpr int cin = CW;
  constexpr int DL = 40;  // dz positions a tile of 64 inputs reaches (36 used)
  __shared__ T Wt[CW][KCP + 4];
  __shared__ T Ds[CCH][DL];
  const int b = blockIdx.y, j0 = blockIdx.x * LT;
  const int lbase = (j0 >> 1) - 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  flt4 acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = flt4{0.f, 0.f, 0.f, 0.f};
  for (int co0 = 0; co0 < CW; co0 += CCH) {
    __syncthreads();
    for (int e = tid; e < CW * KCP; e += 256) {
      const int ci = e / KCP, k = e - ci * KCP;
      const int cl = k / KW, tap = k - cl * KW;
      Wt[ci][k] = W[(int64_t)(co0 + cl) * cin * KW + ci * KW + tap];
    }
    for (int e = tid; e < CCH * DL; e += 256) {
      const int cl = e / DL, qq = e - cl * DL;
      const int l = lbase + qq;
      Ds[cl][qq] = (l >= 0 && l < lout) ? T(dz[((int64_t)b * CW + co0 + cl) * lout + l]) : T(0);
    }
    __syncthreads();
    for (int ks = 0; ks < KCP; ks += M::KS) {
      T a[M::KPL];
#pragma unroll
      for (int j = 0; j < M::KPL; ++j) a[j] = Wt[wave * 16 + lr][ks + lq * M::KPL + j];
#pragma unroll
      for (int lb = 0; lb < 4; ++lb) {
        T bv[M::KPL];
        const int jj = j0 + lb * 16 + lr;
#pragma unroll
        for (int j = 0; j < M::KPL; ++j) {
          const int k = ks + lq * M::KPL + j;
          const int cl = k / KW, tap = k - cl * KW;
          const int num = jj + PADW - tap;
          bv[j] = (num & 1) ? T(0) : Ds[cl][num / 2 - lbase];
        }
        acc[lb] = M::op(a, bv, acc[lb]);
      }
    }
  }
#pragma unroll
  for (int lb = 0; lb < 4; ++lb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ci = wave * 16 + 4 * lq + i, jj = j0 + lb * 16 + lr;
      if (jj < lin) {
        const int64_t o = ((int64_t)b * cin + ci) * lin + jj;
        dzp[o] = yp[o] > 0.f ? acc[lb][i] : 0.f;
      }
    }
}

// part[chunk][co][n] = sum over the chunk's samples and all l of dz[b][co][l] x[b][ci][2l+k-3],
// n = ci*7 + k in the workgroup's tile of 64 columns
template <typename T>
__global__ __launch_bounds__(256) void conv_bwd_weight_kernel(const float* __restrict__ dz,
                                                              const float* __restrict__ x,
                                                              float* __restrict__ part, int cin, int lin, int lout,
                                                              int batch, int per_chunk) {
  typedef CM<T> M;
  constexpr int NCI = 11;  // input channels a tile of 64 columns spans, at most
  __shared__ T Dz[CW][LT + 4];
  __shared__ T Xw[NCI][XW];
  const int ntot = cin * KW;
  const int n0 = blockIdx.x * 64, chunk = blockIdx.y;
  const int ci_lo = n0 / KW;
  const int ci_hi = min(cin, (n0 + 63) / KW + 1);
  const int nci = ci_hi - ci_lo;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  flt4 acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = flt4{0.f, 0.f, 0.f, 0.f};
  const int b_end = min(batch, (chunk + 1) * per_chunk);
  for (int b = chunk * per_chunk; b < b_end; ++b)
    for (int l0 = 0; l0 < lout; l0 += LT) {
      __syncthreads();
      for (int e = tid; e < CW * LT; e += 256) {
        const int co = e / LT, l = e - co * LT;
        Dz[co][l] = (l0 + l < lout) ? T(dz[((int64_t)b * CW + co) * lout + l0 + l]) : T(0);
      }
      for (int e = tid; e < nci * XW; e += 256) {
        const int ci = e / XW, p = e - ci * XW;
        const int j = 2 * l0 - PADW + p;
        Xw[ci][p] = (j >= 0 && j < lin) ? T(x[((int64_t)b * cin + ci_lo + ci) * lin + j]) : T(0);
      }
      __syncthreads();
      for (int ks = 0; ks < LT; ks += M::KS) {
        T a[M::KPL];
#pragma unroll
        for (int j = 0; j < M::KPL; ++j) a[j] = Dz[wave * 16 + lr][ks + lq * M::KPL + j];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          const int n = n0 + nb * 16 + lr;
          const int ci = n / KW, tap = n - ci * KW;
          T bv[M::KPL];
#pragma unroll
          for (int j = 0; j < M::KPL; ++j) {
            const int k = ks + lq * M::KPL + j;
            bv[j] = n < ntot ? Xw[ci - ci_lo][2 * k + tap] : T(0);
          }
          acc[nb] = M::op(a, bv, acc[nb]);
        }
      }
    }
#pragma unroll
  for (int nb = 0; nb < 4; ++nb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = wave * 16 + 4 * lq + i, n = n0 + nb * 16 + lr;
      if (n < ntot) part[((int64_t)chunk * CW + co) * ntot + n] = acc[nb][i];
    }
}

// dW = sum of the chunk partials in chunk order; db[co] = sum over samples and positions of dz
__global__ __launch_bounds__(256) void wgrad_reduce_kernel(const float* __restrict__ part, int nchunks, int64_t count,
                                                           float* __restrict__ dW) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  float s = 0.f;
  for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * count + i];
  dW[i] = s;
}

__global__ __launch_bounds__(256) void bgrad_kernel(const float* __restrict__ dz, int batch, int lout,
                                                    float* __restrict__ db) {
  __shared__ float red[256];
  const int co = blockIdx.x, tid = threadIdx.x;
  float s = 0.f;
  for (int64_t e = tid; e < (int64_t)batch * lout; e += 256) {
    const int64_t b = e / lout, l = e - b * lout;
    s += dz[(b * CW + co) * lout + l];
  }
  red[tid] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) db[co] = red[0];
}

// per sample: h = mean over positions, out = Wh h + bh
__global__ __launch_bounds__(64) void head_fwd_kernel(const float* __restrict__ y4, const float* __restrict__ Wh,
                                                      const float* __restrict__ bh, float* __restrict__ h,
                                                      float* __restrict__ out, int l4) {
  __shared__ float hs[CW];
  const int b = blockIdx.x, c = threadIdx.x;
  float s = 0.f;
  for (int l = 0; l < l4; ++l) s += y4[((int64_t)b * CW + c) * l4 + l];
  hs[c] = s / (float)l4;
  h[(int64_t)b * CW + c] = hs[c];
  __syncthreads();
  if (c < CNN_OUT) {
    float o = bh[c];
    for (int k = 0; k < CW; ++k) o = fmaf(Wh[c * CW + k], hs[k], o);
    out[(int64_t)b * CNN_OUT + c] = o;
  }
}

// per sample: dO = 2 (out - target) / (batch * 4), squared error, dz4 = [y4 > 0] (Wh^T dO) / l4
__global__ __launch_bounds__(64) void head_bwd_kernel(const float* __restrict__ y4, const float* __restrict__ Wh,
                                                      const float* __restrict__ out,
                                                      const float* __restrict__ target, float* __restrict__ dO,
                                                      float* __restrict__ sq, float* __restrict__ dz4, int l4,
                                                      float scale) {
  __shared__ float d[CNN_OUT];
  const int b = blockIdx.x, c = threadIdx.x;
  if (c < CNN_OUT) {
    const float e = out[(int64_t)b * CNN_OUT + c] - target[(int64_t)b * CNN_OUT + c];
    d[c] = 2.f * e * scale;
    dO[(int64_t)b * CNN_OUT + c] = d[c];
  }
  __syncthreads();
  if (c == 0) {
    float s = 0.f;
    for (int j = 0; j < CNN_OUT; ++j) {
      const float e = out[(int64_t)b * CNN_OUT + j] - target[(int64_t)b * CNN_OUT + j];
      s = fmaf(e, e, s);
    }
    sq[b] = s;
  }
  float g = 0.f;
  for (int j = 0; j < CNN_OUT; ++j) g = fmaf(Wh[j * CW + c], d[j], g);
  g /= (float)l4;
  for (int l = 0; l < l4; ++l) {
    const int64_t o = ((int64_t)b * CW + c) * l4 + l;
    dz4[o] = y4[o] > 0.f ? g : 0.f;
  }
}

// one workgroup: head weight gradients and the loss, sums in sample order
__global__ __launch_bounds__(256) void head_wgrad_kernel(const float* __restrict__ dO, const float* __restrict__ h,
                                                         const float* __restrict__ sq, int batch, float scale,
                                                         float* __restrict__ gWh, float* __restrict__ gbh,
                                                         float* __restrict__ loss) {
  const int tid = threadIdx.x;
  if (tid < CNN_OUT * CW) {  // 256 = 4 x 64 weights
    const int j = tid / CW, c = tid - j * CW;
    float s = 0.f;
    for (int b = 0; b < batch; ++b) s = fmaf(dO[(int64_t)b * CNN_OUT + j], h[(int64_t)b * CW + c], s);
    gWh[j * CW + c] = s;
  }
  if (tid < CNN_OUT) {
    float s = 0.f;
    for (int b = 0; b < batch; ++b) s += dO[(int64_t)b * CNN_OUT + tid];
    gbh[tid] = s;
  }
  if (tid == 0 && loss) {
    float s = 0.f;
    for (int b = 0; b < batch; ++b) s += sq[b];
    *loss = s * scale;
  }
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, _Float16* __restrict__ p16,
                                                   const float* __restrict__ g, float* __restrict__ m,
                                                   float* __restrict__ v, int64_t n, float lr, float b1, float b2,
                                                   float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  p[i] = pi;
  if (p16) p16[i] = (_Float16)pi;
}

// He-uniform weights, zero biases: parameter i of a weight block with fan-in F
// is U(-sqrt(6/F), sqrt(6/F)), the uniform from Philox (counter i, stream 4)
__global__ __launch_bounds__(256) void cnn_init_kernel(float* __restrict__ p, int64_t n, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  int fan = 0;
  for (int l = 0; l < CNN_LAYERS; ++l)
    if (i >= cnn_w_offset(l) && i < cnn_b_offset(l)) fan = (l == 0 ? 1 : CNN_CH) * CNN_KW;
  if (i >= cnn_head_w() && i < cnn_head_b()) fan = CNN_CH;
  if (fan == 0) {
    p[i] = 0.f;
    return;
  }
  const U4 w = draw((uint64_t)i, 0, 4, seed);
  const double u = uniform01(w.v[0], w.v[1]);
  p[i] = (float)((2.0 * u - 1.0) * sqrt(6.0 / fan));
}

hipError_t launch_cnn_init(hipStream_t s, float* p, int64_t n, uint64_t seed) {
  hipLaunchKernelGGL(cnn_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, seed);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void to_half_kernel(const float* __restrict__ p, _Float16* __restrict__ p16,
                                                      int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p16[i] = (_Float16)p[i];
}

// standardised outputs -> fit coordinates (ln amp, ln P_rot, ln Q, ln sigma_w); with x_plain,
// ln sigma_w is taken from it (the white noise is averaged out of the binned input, the
// second differences of the full curve measure it directly)
__global__ void outputs_to_log_kernel(const float* __restrict__ y, int batch, const double* __restrict__ x_plain,
                                      double* __restrict__ x) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= batch * CNN_OUT) return;
  const int k = i % CNN_OUT;
  const double lo = log(prior_lo(k)), hi = log(prior_hi(k));
  x[i] = (x_plain && k == 3) ? x_plain[i] : 0.5 * (lo + hi) + (hi - lo) / sqrt(12.0) * (double)y[i];
}

// ---------------------------------------------------------------------------
// Launchers of the network passes

template <typename T>
hipError_t conv_fwd(hipStream_t s, const float* x, const T* W, const float* bias, float* y, int batch, int cin,
                    int lin) {
  const int lout = lin / 2;
  hipLaunchKernelGGL(conv_fwd_kernel<T>, dim3((unsigned)((lout + LT - 1) / LT), (unsigned)batch), dim3(256), 0, s,
                     x, W, bias, y, cin, lin, lout);
  return hipGetLastError();
}

template <typename T>
hipError_t conv_bwd_data(hipStream_t s, const float* dz, const T* W, const float* yp, float* dzp, int batch, int lin) {
  hipLaunchKernelGGL(conv_bwd_data_kernel<T>, dim3((unsigned)((lin + LT - 1) / LT), (unsigned)batch), dim3(256), 0, s,
                     dz, W, yp, dzp, lin, lin / 2);
  return hipGetLastError();
}

template <typename T>
hipError_t conv_bwd_weight(hipStream_t s, const float* dz, const float* x, float* part, float* dW, float* db,
                           int batch, int cin, int lin) {
  const int lout = lin / 2, ntot = cin * KW;
  const int nchunks = (batch + CNN_WCHUNK - 1) / CNN_WCHUNK;
  hipLaunchKernelGGL(conv_bwd_weight_kernel<T>, dim3((unsigned)((ntot + 63) / 64), (unsigned)nchunks), dim3(256), 0,
                     s, dz, x, part, cin, lin, lout, batch, CNN_WCHUNK);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t count = (int64_t)CW * ntot;
  hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, part, nchunks, count,
                     dW);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bgrad_kernel, dim3(CW), dim3(256), 0, s, dz, batch, lout, db);
  return hipGetLastError();
}

template <typename T>
hipError_t cnn_forward_t(hipStream_t s, const CnnBuffers& B, const float* P, const T* Pw, const float* input,
                         int batch, float* out) {
  const float* x = input;
  int cin = 1, lin = CNN_IN;
  for (int l = 0; l < CNN_LAYERS; ++l) {
    hipError_t e = conv_fwd<T>(s, x, Pw + cnn_w_offset(l), P + cnn_b_offset(l), B.y[l], batch, cin, lin);
    if (e != hipSuccess) return e;
    x = B.y[l];
    cin = CW;
    lin /= 2;
  }
  hipLaunchKernelGGL(head_fwd_kernel, dim3((unsigned)batch), dim3(64), 0, s, B.y[CNN_LAYERS - 1], P + cnn_head_w(),
                     P + cnn_head_b(), B.h, out, lin);
  return hipGetLastError();
}

template <typename T>
hipError_t cnn_backward_t(hipStream_t s, const CnnBuffers& B, const float* P, const T* Pw, const float* input,
                          const float* target, int batch, float* grad, float* loss) {
  const int l4 = CNN_IN >> CNN_LAYERS;
  const float scale = 1.f / (float)(batch * CNN_OUT);
  hipLaunchKernelGGL(head_bwd_kernel, dim3((unsigned)batch), dim3(64), 0, s, B.y[CNN_LAYERS - 1], P + cnn_head_w(),
                     B.out, target, B.dO, B.sq, B.dz[CNN_LAYERS - 1], l4, scale);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(head_wgrad_kernel, dim3(1), dim3(256), 0, s, B.dO, B.h, B.sq, batch, scale,
                     grad + cnn_head_w(), grad + cnn_head_b(), loss);
  e = hipGetLastError();
  for (int l = CNN_LAYERS - 1; e == hipSuccess && l >= 0; --l) {
    const int lin = CNN_IN >> l;
    const int cin = l == 0 ? 1 : CW;
    const float* xin = l == 0 ? input : B.y[l - 1];
    e = conv_bwd_weight<T>(s, B.dz[l], xin, B.part, grad + cnn_w_offset(l), grad + cnn_b_offset(l), batch, cin, lin);
    if (e == hipSuccess && l > 0) e = conv_bwd_data<T>(s, B.dz[l], Pw + cnn_w_offset(l), B.y[l - 1], B.dz[l - 1],
                                                      batch, lin);
  }
  return e;
}

hipError_t launch_cnn_forward(hipStream_t s, const CnnBuffers& B, const float* P, const _Float16* P16, bool half,
                              const float* input, int batch, float* out) {
  return half ? cnn_forward_t<_Float16>(s, B, P, P16, input, batch, out)
              : cnn_forward_t<float>(s, B, P, P, input, batch, out);
}

hipError_t launch_cnn_backward(hipStream_t s, const CnnBuffers& B, const float* P, const _Float16* P16, bool half,
                               const float* input, const float* target, int batch, float* grad, float* loss) {
  return half ? cnn_backward_t<_Float16>(s, B, P, P16, input, target, batch, grad, loss)
              : cnn_backward_t<float>(s, B, P, P, input, target, batch, grad, loss);
}

hipError_t launch_adam(hipStream_t s, float* p, _Float16* p16, const float* g, float* m, float* v, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, p16, g, m, v, n, lr, b1, b2,
                     eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_to_half(hipStream_t s, const float* p, _Float16* p16, int64_t n) {
  hipLaunchKernelGGL(to_half_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, p16, n);
  return hipGetLastError();
}

hipError_t launch_outputs_to_log(hipStream_t s, const float* y, int batch, const double* x_plain, double* x) {
  hipLaunchKernelGGL(outputs_to_log_kernel, dim3((unsigned)((batch * CNN_OUT + 255) / 256)), dim3(256), 0, s, y,
                     batch, x_plain, x);
  return hipGetLastError();
}

}  // namespace nu
