// Linear search (Section 2.2, Eqs. 5-6) in O(N J^2) without a dense factor,
// for the sum-of-terms covariances of Appendix A (SHO) and Section 3.2 (the
// rotation kernel): the quasiseparable route of the GP package the paper
// uses, written here as the Kalman filter of the equivalent state-space model.
//
// Every SHO term is the stationary response of a damped oscillator driven by
// white noise (two states: position and velocity) and every exponential term
// a one-state Ornstein-Uhlenbeck process, so K is the covariance of
// y_n = H x(t_n) + w_n, with x the J-state Markov process (J = 2 n_sho +
// n_exp, states ordered as the SHO pairs then the exponential terms), H
// picking every position state and w white with variance sigma_w^2. Between
// samples the state moves by Phi_{n+1} = exp(F h) and gains the process
// noise Qd = Pinf - Phi Pinf Phi^T (h = t_{n+1} - t_n).
//
// The filter is the Cholesky factorisation K = L L^T taken sample by sample:
//   S_n = H P_n H^T + sigma_w^2            (the squared pivots: ln|K| = sum ln S_n)
//   k_n = P_n H^T / S_n,  P_{n+1} = Phi_{n+1} (P_n - k_n S_n k_n^T) Phi_{n+1}^T + Qd_{n+1},  P_0 = Pinf
// and L^-1 v is the scaled innovation sequence
//   z_n = (v_n - H x_n) / sqrt(S_n),  x_{n+1} = Phi_{n+1} (x_n + k_n (v_n - H x_n)),  x_0 = 0.
// Its transpose L^-T w runs backwards with an adjoint state lambda (lambda_N = 0):
//   mu = Phi_{n+1}^T lambda_{n+1},  u_n = w_n / sqrt(S_n) + k_n . mu,  lambda_n = mu - H^T u_n.
// For a box b = 1 on samples [lo, hi), L^-1 b is zero before lo, follows the
// recursion with v = 1 inside, and after hi is the free response of x_hi,
// whose energy is x_hi^T G_hi x_hi with
//   G_n = H^T H / S_n + M_n^T G_{n+1} M_n,  M_n = Phi_{n+1} (I - k_n H),  G_N = 0,
// so q = b^T K^-1 b costs O(d J + J^2) per box instead of a pass over L^-1.
//
// Kernels, in launch order (the trend/flux packing, the trend-only fit, the
// slot table and the per-cell Schur epilogue are the dense path's):
//   ss_step      per sample gap: Phi and Qd of every term              (parallel)
//   ss_riccati   S_n, k_n               (one wave; lane a keeps row a of P), then ln|K|
//   ss_forward   Y = L^-1 [A | f]       (one lane per column)
//   ss_backward  Z = L^-T [A~ | r~0]    (one lane per column) and G_n (one wave; lane a keeps row a)
//   ss_box       q of every cell, one thread per box start: the boxes of all
//                durations that start on one slot share the in-box recursion
//   ss_template  q of every cell of a template search (a shape in place of the
//                box), one thread per cell
#include "cells.hpp"
#include "internal.hpp"

namespace nu {

namespace {

// Step record of one sample gap: per SHO term 7 doubles (Phi row-major
// p00 p01 p10 p11, then Qd00 Qd01 Qd11), per exponential term 2 (phi, Qd).
// Gain record of one sample: 1/sqrt(S_n), then k_n[J].
template <int NS, int NE>
struct SsLayout {
  static constexpr int J = 2 * NS + NE;
  static constexpr int TS = 7 * NS + 2 * NE;
  static constexpr int GS = J + 1;
  static constexpr bool pos(int b) { return b >= 2 * NS || (b & 1) == 0; }
};

// e^{-a h} cos(b h) and e^{-a h} sin(b h) / b of the oscillator (and their
// limits at Q = 1/2 and their hyperbolic forms for Q < 1/2), a = omega / 2Q.
__device__ void sho_step_coeffs(double amp, double om, double q, double h, double* c) {
  const double a = om / (2.0 * q);
  double eC, eS;
  if (q == 0.5) {
    const double e = exp(-a * h);
    eC = e;
    eS = e * h;
  } else if (q > 0.5) {
    const double b = om * sqrt(1.0 - 1.0 / (4.0 * q * q));
    double sn, cs;
    sincos(b * h, &sn, &cs);
    const double e = exp(-a * h);
    eC = e * cs;
    eS = e * sn / b;
  } else {
    // b < a: e^{-ah} cosh(bh) = (e1 + e2) / 2 and e^{-ah} sinh(bh) / b =
    // e1 (1 - e^{-2bh}) / 2b with e1 = e^{-(a-b)h}, e2 = e^{-(a+b)h}, which
    // neither overflow at long gaps nor cancel at short ones
    const double b = om * sqrt(1.0 / (4.0 * q * q) - 1.0);
    const double e1 = exp(-(a - b) * h), e2 = exp(-(a + b) * h);
    eC = 0.5 * (e1 + e2);
    eS = -e1 * expm1(-2.0 * b * h) / (2.0 * b);
  }
  const double p00 = eC + a * eS, p01 = eS, p10 = -om * om * eS, p11 = eC - a * eS;
  const double v0 = amp * amp, v1 = v0 * om * om;
  c[0] = p00;
  c[1] = p01;
  c[2] = p10;
  c[3] = p11;
  c[4] = v0 - (p00 * p00 * v0 + p01 * p01 * v1);
  c[5] = -(p00 * p10 * v0 + p01 * p11 * v1);
  c[6] = v1 - (p10 * p10 * v0 + p11 * p11 * v1);
}

__global__ __launch_bounds__(256) void ss_step_kernel(const double* __restrict__ t, int64_t n, nu_kernel k,
                                                      int ts, double* __restrict__ step) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i + 1 >= n) return;
  const double h = t[i + 1] - t[i];
  double* c = step + i * ts;
  const int ns = k.n_sho, ne = k.n_exp;
  for (int s = 0; s < ns; ++s) sho_step_coeffs(k.sho_amp[s], k.sho_omega[s], k.sho_q[s], h, c + 7 * s);
  for (int e = 0; e < ne; ++e) {
    const double sg = k.exp_sigma[e], ell = k.exp_ell[e];
    c[7 * ns + 2 * e] = exp(-h / ell);
    c[7 * ns + 2 * e + 1] = -sg * sg * expm1(-2.0 * h / ell);
  }
}

// v of lane src in every lane (two readlanes; src uniform)
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// v of lane l ^ 1 (the partner row of an SHO pair): a DPP quad permutation
// [1, 0, 3, 2] of both halves, no LDS round trip
__device__ __forceinline__ double pair_swap(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, 0xb1, 0xf, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), 0xb1, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// 1 / sqrt(s) for positive normal s: the hardware estimate r with a
// third-order correction. With h = 1 - s r^2, 1/sqrt(s) = r (1 + h/2 + 3 h^2/8
// + ...); the estimate has |h| <= 2^-23.2 (measured on gfx950), so the
// truncation is below 2^-70 and the result within 1.3 ulp, as with two Newton
// steps but two operations shorter on the dependent chain.
__device__ __forceinline__ double rsqrt_nr(double s) {
  const double r = __builtin_amdgcn_rsq(s);
  const double h = fma(-s * r, r, 1.0);
  return fma(r * h, fma(h, 0.375, 0.5), r);
}

// The sequential kernels take their per-sample records from LDS, staged one
// chunk of CH samples ahead: at the start of a chunk the wave issues the
// global loads of the next chunk's records (coalesced: lane l moves words l,
// l + 64, ... of the chunk's contiguous span of W-double records) and writes
// them to the other LDS buffer at the end of the chunk, so no load latency
// sits on the recursion's critical path.
constexpr int CH = 64;

template <int W>
struct Stage {
  double r[W];
  // records [c0, c0 + CH) of an array of nrec records
  __device__ __forceinline__ void load(const double* __restrict__ src, int64_t c0, int64_t nrec, int lane) {
    const int64_t first = c0 * W, end = nrec * W;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const int64_t idx = first + k * 64 + lane;
      r[k] = idx < end ? src[idx] : 0.0;
    }
  }
  __device__ __forceinline__ void put(double* lds, int lane) const {
#pragma unroll
    for (int k = 0; k < W; ++k) lds[k * 64 + lane] = r[k];
  }
};

// x <- Phi x for the block-diagonal transition of a step record
template <int NS, int NE>
__device__ __forceinline__ void apply_phi(const double* c, double* x) {
#pragma unroll
  for (int s2 = 0; s2 < NS; ++s2) {
    const double u0 = x[2 * s2], u1 = x[2 * s2 + 1];
    x[2 * s2] = c[7 * s2] * u0 + c[7 * s2 + 1] * u1;
    x[2 * s2 + 1] = c[7 * s2 + 2] * u0 + c[7 * s2 + 3] * u1;
  }
#pragma unroll
  for (int e2 = 0; e2 < NE; ++e2) x[2 * NS + e2] = c[7 * NS + 2 * e2] * x[2 * NS + e2];
}

// x <- Phi^T x
template <int NS, int NE>
__device__ __forceinline__ void apply_phi_t(const double* c, double* x) {
#pragma unroll
  for (int s2 = 0; s2 < NS; ++s2) {
    const double l0 = x[2 * s2], l1 = x[2 * s2 + 1];
    x[2 * s2] = c[7 * s2] * l0 + c[7 * s2 + 2] * l1;
    x[2 * s2 + 1] = c[7 * s2 + 1] * l0 + c[7 * s2 + 3] * l1;
  }
#pragma unroll
  for (int e2 = 0; e2 < NE; ++e2) x[2 * NS + e2] = c[7 * NS + 2 * e2] * x[2 * NS + e2];
}

// Lane a of the wave keeps row a of the J x J state covariance (lanes past J
// shadow row 0 and store nothing). Per sample: the pivot S from the
// broadcast row sums over the position columns, the rank-one update, Phi
// from the left (the partner row of an SHO pair by a lane swap), Phi^T from
// the right and the process noise of the lane's own block. ln|K| is summed
// afterwards, in parallel, from the stored 1/sqrt(S_n).
template <int NS, int NE>
__global__ __launch_bounds__(64) void ss_riccati_kernel(const double* __restrict__ step, nu_kernel kp, int64_t n,
                                                        double* __restrict__ gain, int64_t* __restrict__ status) {
  using Lt = SsLayout<NS, NE>;
  constexpr int J = Lt::J, TS = Lt::TS, GS = Lt::GS;
  __shared__ double st[2][CH * TS];
  const int lane = threadIdx.x;
  const int a = lane < J ? lane : 0;
  const bool sho = a < 2 * NS;
  const int s = a >> 1, r = a & 1, e = a - 2 * NS;
  // own-block offsets in the step record: Phi(r, r), Phi(r, 1-r), Qd(r, 0), Qd(r, 1)
  const int o_diag = sho ? 7 * s + 3 * r : 7 * NS + 2 * e;
  const int o_off = sho ? 7 * s + 1 + r : 0;
  const int o_q0 = sho ? 7 * s + 4 + r : 7 * NS + 2 * e + 1;
  const int o_q1 = sho ? 7 * s + 5 + r : 0;
  const int c0 = sho ? 2 * s : a;  // first column of the lane's own block
  double pinf;
  if (sho) {
    const double amp = kp.sho_amp[s], om = kp.sho_omega[s];
    pinf = r == 0 ? amp * amp : amp * amp * om * om;
  } else {
    const double sg = kp.exp_sigma[e];
    pinf = sg * sg;
  }
  const double sw2 = kp.sigma_w * kp.sigma_w;
  double P[J];
#pragma unroll
  for (int b = 0; b < J; ++b) P[b] = b == a ? pinf : 0.0;
  int64_t fail = -1;
  Stage<TS> pre;
  pre.load(step, 0, n - 1, lane);
  pre.put(st[0], lane);
  wave_lds_fence();
  const int64_t nch = (n + CH - 1) / CH;
  for (int64_t ch = 0; ch < nch && fail < 0; ++ch) {
    const double* cur = st[ch & 1];
    if (ch + 1 < nch) pre.load(step, (ch + 1) * CH, n - 1, lane);
    const int iend = (int)min((int64_t)CH, n - ch * CH);
    for (int ii = 0; ii < iend; ++ii) {
      const int64_t i = ch * CH + ii;
      double ph = 0.0;
#pragma unroll
      for (int b = 0; b < J; ++b)
        if (Lt::pos(b)) ph += P[b];
      double phv[J];
#pragma unroll
      for (int b = 0; b < J; ++b) phv[b] = lane_bcast(ph, b);
      double S = sw2;
#pragma unroll
      for (int b = 0; b < J; ++b)
        if (Lt::pos(b)) S += phv[b];
      if (!(S > 0.0 && S < INFINITY)) {
        fail = i;
        break;
      }
      const double rsq = rsqrt_nr(S);
      const double rS = rsq * rsq;
      double* g = gain + i * GS;
      if (lane == 0) g[0] = rsq;
      if (lane < J) g[1 + lane] = ph * rS;
      if (i + 1 == n) break;
      // P - P H^T H P / S
      const double kr = ph * rS;
#pragma unroll
      for (int b = 0; b < J; ++b) P[b] = fma(-kr, phv[b], P[b]);
      // Phi from the left: rows of the lane's own block
      const double* c = cur + ii * TS;
      const double al = c[o_diag];
      const double be = sho ? c[o_off] : 0.0;
      double T[J];
#pragma unroll
      for (int b = 0; b < J; ++b) {
        const double other = pair_swap(P[b]);
        T[b] = al * P[b] + (sho ? be * other : 0.0);
      }
      // Phi^T from the right, then the process noise of the own block
#pragma unroll
      for (int s2 = 0; s2 < NS; ++s2) {
        const double p00 = c[7 * s2], p01 = c[7 * s2 + 1], p10 = c[7 * s2 + 2], p11 = c[7 * s2 + 3];
        const double t0 = T[2 * s2], t1 = T[2 * s2 + 1];
        P[2 * s2] = t0 * p00 + t1 * p01;
        P[2 * s2 + 1] = t0 * p10 + t1 * p11;
      }
#pragma unroll
      for (int e2 = 0; e2 < NE; ++e2) P[2 * NS + e2] = T[2 * NS + e2] * c[7 * NS + 2 * e2];
      const double q0 = c[o_q0], q1 = sho ? c[o_q1] : 0.0;
#pragma unroll
      for (int b = 0; b < J; ++b) {
        if (b == c0) P[b] += q0;
        if (sho && b == c0 + 1) P[b] += q1;
      }
    }
    if (ch + 1 < nch) pre.put(st[(ch + 1) & 1], lane);
    wave_lds_fence();
  }
  if (lane == 0) *status = fail;
}

// ln|K| = sum ln S_n = -2 sum ln(1/sqrt(S_n)) in a fixed order; NaN if the
// filter failed. With failmin (the chunked filter's smallest failing sample,
// n if none) the status is written here from it.
__global__ __launch_bounds__(256) void ss_logdet_kernel(const double* __restrict__ gain, int gs, int64_t n,
                                                        const unsigned long long* __restrict__ failmin,
                                                        int64_t* __restrict__ status, double* __restrict__ logdet) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) acc += log(gain[i * gs]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t st = *status;
    if (failmin) {
      st = *failmin < (unsigned long long)n ? (int64_t)*failmin : -1;
      *status = st;
    }
    *logdet = st >= 0 ? NAN : -2.0 * (((red[0] + red[1]) + red[2]) + red[3]);
  }
}

// Y = L^-1 V: lane c carries the filter state of column c (lanes past the
// last column repeat it and store nothing).
template <int NS, int NE>
__global__ __launch_bounds__(64) void ss_forward_kernel(const double* __restrict__ step,
                                                        const double* __restrict__ gain, int64_t n,
                                                        const double* __restrict__ V, int nv, double* __restrict__ Y) {
  using Lt = SsLayout<NS, NE>;
  constexpr int J = Lt::J, TS = Lt::TS, GS = Lt::GS;
  __shared__ double sv[2][CH * YCOLS], sg[2][CH * GS], ss[2][CH * TS];
  const int lane = threadIdx.x;
  const int col = lane < nv ? lane : nv - 1;
  double x[J];
#pragma unroll
  for (int b = 0; b < J; ++b) x[b] = 0.0;
  Stage<YCOLS> pv;
  Stage<GS> pg;
  Stage<TS> ps;
  pv.load(V, 0, n, lane);
  pg.load(gain, 0, n, lane);
  ps.load(step, 0, n - 1, lane);
  pv.put(sv[0], lane);
  pg.put(sg[0], lane);
  ps.put(ss[0], lane);
  wave_lds_fence();
  const int64_t nch = (n + CH - 1) / CH;
  for (int64_t ch = 0; ch < nch; ++ch) {
    const int buf = (int)(ch & 1);
    if (ch + 1 < nch) {
      pv.load(V, (ch + 1) * CH, n, lane);
      pg.load(gain, (ch + 1) * CH, n, lane);
      ps.load(step, (ch + 1) * CH, n - 1, lane);
    }
    const int iend = (int)min((int64_t)CH, n - ch * CH);
    for (int ii = 0; ii < iend; ++ii) {
      const int64_t i = ch * CH + ii;
      const double* g = sg[buf] + ii * GS;
      double hx = 0.0;
#pragma unroll
      for (int b = 0; b < J; ++b)
        if (Lt::pos(b)) hx += x[b];
      const double ev = sv[buf][ii * YCOLS + col] - hx;
      if (lane < nv) Y[i * YCOLS + lane] = ev * g[0];
#pragma unroll
      for (int b = 0; b < J; ++b) x[b] = fma(g[1 + b], ev, x[b]);
      apply_phi<NS, NE>(ss[buf] + ii * TS, x);  // the last sample's record is unused padding
    }
    if (ch + 1 < nch) {
      pv.put(sv[buf ^ 1], lane);
      pg.put(sg[buf ^ 1], lane);
      ps.put(ss[buf ^ 1], lane);
    }
    wave_lds_fence();
  }
}

// Workgroup 0: Z = L^-T W (lane c carries the adjoint state of column c).
// Workgroup 1: G_n for n = N .. 0 (lane a keeps row a), stored row-major
// J x J per sample. The two chains are independent and run side by side;
// both walk the chunks backwards, staging the previous chunk.
template <int NS, int NE>
__global__ __launch_bounds__(64) void ss_backward_kernel(const double* __restrict__ step,
                                                         const double* __restrict__ gain, int64_t n,
                                                         const double* __restrict__ W, int nv, double* __restrict__ Z,
                                                         double* __restrict__ Gm) {
  using Lt = SsLayout<NS, NE>;
  constexpr int J = Lt::J, TS = Lt::TS, GS = Lt::GS;
  __shared__ double sw[2][CH * YCOLS], sg[2][CH * GS], ss[2][CH * TS];
  const int lane = threadIdx.x;
  const bool adj = blockIdx.x == 0;
  const int64_t nch = (n + CH - 1) / CH;
  Stage<YCOLS> pw;
  Stage<GS> pg;
  Stage<TS> ps;
  {
    const int64_t c0 = (nch - 1) * CH;
    if (adj) pw.load(W, c0, n, lane);
    pg.load(gain, c0, n, lane);
    ps.load(step, c0, n - 1, lane);
    if (adj) pw.put(sw[(nch - 1) & 1], lane);
    pg.put(sg[(nch - 1) & 1], lane);
    ps.put(ss[(nch - 1) & 1], lane);
    wave_lds_fence();
  }
  if (adj) {
    const int col = lane < nv ? lane : nv - 1;
    double lam[J];
#pragma unroll
    for (int b = 0; b < J; ++b) lam[b] = 0.0;
    for (int64_t ch = nch - 1; ch >= 0; --ch) {
      const int buf = (int)(ch & 1);
      if (ch > 0) {
        pw.load(W, (ch - 1) * CH, n, lane);
        pg.load(gain, (ch - 1) * CH, n, lane);
        ps.load(step, (ch - 1) * CH, n - 1, lane);
      }
      const int iend = (int)min((int64_t)CH, n - ch * CH);
      for (int ii = iend - 1; ii >= 0; --ii) {
        const int64_t i = ch * CH + ii;
        double mu[J];
#pragma unroll
        for (int b = 0; b < J; ++b) mu[b] = lam[b];
        if (i + 1 < n) {
          apply_phi_t<NS, NE>(ss[buf] + ii * TS, mu);
        } else {
#pragma unroll
          for (int b = 0; b < J; ++b) mu[b] = 0.0;
        }
        const double* g = sg[buf] + ii * GS;
        double u = sw[buf][ii * YCOLS + col] * g[0];
#pragma unroll
        for (int b = 0; b < J; ++b) u = fma(g[1 + b], mu[b], u);
        if (lane < nv) Z[i * YCOLS + lane] = u;
#pragma unroll
        for (int b = 0; b < J; ++b) lam[b] = Lt::pos(b) ? mu[b] - u : mu[b];
      }
      if (ch > 0) {
        pw.put(sw[buf ^ 1], lane);
        pg.put(sg[buf ^ 1], lane);
        ps.put(ss[buf ^ 1], lane);
      }
      wave_lds_fence();
    }
    return;
  }
  const int a = lane < J ? lane : 0;
  const bool sho = a < 2 * NS;
  const int s = a >> 1, r = a & 1, e = a - 2 * NS;
  // Phi^T from the left: Phi(r, r) on the own row, Phi(1-r, r) on the partner row
  const int o_diag = sho ? 7 * s + 3 * r : 7 * NS + 2 * e;
  const int o_off = sho ? 7 * s + 2 - r : 0;
  const bool posa = Lt::pos(a);
  double G[J];
#pragma unroll
  for (int b = 0; b < J; ++b) G[b] = 0.0;
  if (lane < J) {
#pragma unroll
    for (int b = 0; b < J; ++b) Gm[(n * J + lane) * J + b] = 0.0;
  }
  for (int64_t ch = nch - 1; ch >= 0; --ch) {
    const int buf = (int)(ch & 1);
    if (ch > 0) {
      pg.load(gain, (ch - 1) * CH, n, lane);
      ps.load(step, (ch - 1) * CH, n - 1, lane);
    }
    const int iend = (int)min((int64_t)CH, n - ch * CH);
    for (int ii = iend - 1; ii >= 0; --ii) {
      const int64_t i = ch * CH + ii;
      double Wr[J];
      if (i + 1 < n) {
        const double* c = ss[buf] + ii * TS;
        const double al = c[o_diag];
        const double be = sho ? c[o_off] : 0.0;
        double T[J];
#pragma unroll
        for (int b = 0; b < J; ++b) {
          const double other = pair_swap(G[b]);
          T[b] = al * G[b] + (sho ? be * other : 0.0);
        }
#pragma unroll
        for (int s2 = 0; s2 < NS; ++s2) {
          const double p00 = c[7 * s2], p01 = c[7 * s2 + 1], p10 = c[7 * s2 + 2], p11 = c[7 * s2 + 3];
          const double t0 = T[2 * s2], t1 = T[2 * s2 + 1];
          Wr[2 * s2] = t0 * p00 + t1 * p10;
          Wr[2 * s2 + 1] = t0 * p01 + t1 * p11;
        }
#pragma unroll
        for (int e2 = 0; e2 < NE; ++e2) Wr[2 * NS + e2] = T[2 * NS + e2] * c[7 * NS + 2 * e2];
      } else {
#pragma unroll
        for (int b = 0; b < J; ++b) Wr[b] = 0.0;
      }
      const double* g = sg[buf] + ii * GS;
      const double rS = g[0] * g[0];
      double wk = 0.0;
#pragma unroll
      for (int b = 0; b < J; ++b) wk = fma(Wr[b], g[1 + b], wk);
      double wkv[J];
#pragma unroll
      for (int b = 0; b < J; ++b) wkv[b] = lane_bcast(wk, b);
      double kwk = 0.0;
#pragma unroll
      for (int b = 0; b < J; ++b) kwk = fma(g[1 + b], wkv[b], kwk);
      const double corner = kwk + rS;
#pragma unroll
      for (int b = 0; b < J; ++b) {
        double v = Wr[b];
        if (posa) v -= wkv[b];
        if (Lt::pos(b)) v -= wk;
        if (posa && Lt::pos(b)) v += corner;
        G[b] = v;
      }
      if (lane < J) {
#pragma unroll
        for (int b = 0; b < J; ++b) Gm[(i * J + lane) * J + b] = G[b];
      }
    }
    if (ch > 0) {
      pg.put(sg[buf ^ 1], lane);
      ps.put(ss[buf ^ 1], lane);
    }
    wave_lds_fence();
  }
}

// q of every cell. Thread for box start slot a (a from -floor(dmax/2)):
// the boxes [a, a + d_k) of the ascending durations share the recursion from
// lo = count_below(a); at each end hi_k the tail energy x^T G_hi x is added
// and the cell (k, a + floor(d_k/2)) written, if it is on the grid.
template <int NS, int NE>
__global__ __launch_bounds__(256) void ss_box_kernel(const double* __restrict__ step, const double* __restrict__ gain,
                                                     const double* __restrict__ Gm, int64_t n,
                                                     const int64_t* __restrict__ lattice,
                                                     const int32_t* __restrict__ T, int64_t n_epochs, DurList dl,
                                                     int half_max, double* __restrict__ qbox) {
  using Lt = SsLayout<NS, NE>;
  constexpr int J = Lt::J, TS = Lt::TS, GS = Lt::GS;
  const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x - half_max;
  if (a >= n_epochs) return;
  double x[J];
#pragma unroll
  for (int b = 0; b < J; ++b) x[b] = 0.0;
  double q = 0.0;
  int64_t m = count_below(lattice, n, T, n_epochs, a);
  for (int k = 0; k < dl.n; ++k) {
    const int64_t hk = count_below(lattice, n, T, n_epochs, a + dl.d[k]);
    for (; m < hk; ++m) {
      const double* g = gain + m * GS;
      double hx = 0.0;
#pragma unroll
      for (int b = 0; b < J; ++b)
        if (Lt::pos(b)) hx += x[b];
      const double ev = 1.0 - hx;
      const double z = ev * g[0];
      q = fma(z, z, q);
      if (m + 1 < n) {
        const double* c = step + m * TS;
        double u[J];
#pragma unroll
        for (int b = 0; b < J; ++b) u[b] = fma(g[1 + b], ev, x[b]);
#pragma unroll
        for (int s2 = 0; s2 < NS; ++s2) {
          const double u0 = u[2 * s2], u1 = u[2 * s2 + 1];
          x[2 * s2] = c[7 * s2] * u0 + c[7 * s2 + 1] * u1;
          x[2 * s2 + 1] = c[7 * s2 + 2] * u0 + c[7 * s2 + 3] * u1;
        }
#pragma unroll
        for (int e2 = 0; e2 < NE; ++e2) x[2 * NS + e2] = c[7 * NS + 2 * e2] * u[2 * NS + e2];
      } else {
#pragma unroll
        for (int b = 0; b < J; ++b) x[b] = 0.0;
      }
    }
    const double* G = Gm + hk * J * J;
    double tail = 0.0;
#pragma unroll
    for (int a2 = 0; a2 < J; ++a2) {
      double row = 0.0;
#pragma unroll
      for (int b = 0; b < J; ++b) row = fma(G[a2 * J + b], x[b], row);
      tail = fma(x[a2], row, tail);
    }
    const int64_t i = a + dl.d[k] / 2;
    if (i >= 0 && i < n_epochs) qbox[(int64_t)dl.perm[k] * n_epochs + i] = q + tail;
  }
}

// q of template cells: one thread per cell (the windows of different
// durations no longer share their recursion, the shape values differ). The
// in-window recursion takes v = the shape value of each sample's slot.
template <int NS, int NE>
__global__ __launch_bounds__(256) void ss_template_kernel(const double* __restrict__ step,
                                                          const double* __restrict__ gain,
                                                          const double* __restrict__ Gm, int64_t n,
                                                          const int64_t* __restrict__ lattice,
                                                          const int32_t* __restrict__ T, int64_t n_epochs, DurList dl,
                                                          const double* __restrict__ shapes,
                                                          double* __restrict__ qbox) {
  using Lt = SsLayout<NS, NE>;
  constexpr int J = Lt::J, TS = Lt::TS, GS = Lt::GS;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n_epochs) return;
  const int d = dl.d[j];
  const double* shp = shapes + dl.off[j];
  const int64_t a = i - d / 2;
  const int64_t lo = count_below(lattice, n, T, n_epochs, a);
  const int64_t hi = count_below(lattice, n, T, n_epochs, a + d);
  double x[J];
#pragma unroll
  for (int b = 0; b < J; ++b) x[b] = 0.0;
  double q = 0.0;
  for (int64_t m = lo; m < hi; ++m) {
    const double* g = gain + m * GS;
    double hx = 0.0;
#pragma unroll
    for (int b = 0; b < J; ++b)
      if (Lt::pos(b)) hx += x[b];
    const int64_t o = lattice[m] - a;  // in [0, d) for a lattice the searches accept
    const double ev = ((o >= 0 && o < d) ? shp[o] : 0.0) - hx;
    const double z = ev * g[0];
    q = fma(z, z, q);
    if (m + 1 < n) {
#pragma unroll
      for (int b = 0; b < J; ++b) x[b] = fma(g[1 + b], ev, x[b]);
      apply_phi<NS, NE>(step + m * TS, x);
    } else {
#pragma unroll
      for (int b = 0; b < J; ++b) x[b] = 0.0;
    }
  }
  const double* G = Gm + hi * J * J;
  double tail = 0.0;
#pragma unroll
  for (int a2 = 0; a2 < J; ++a2) {
    double rw = 0.0;
#pragma unroll
    for (int b = 0; b < J; ++b) rw = fma(G[a2 * J + b], x[b], rw);
    tail = fma(x[a2], rw, tail);
  }
  qbox[(int64_t)j * n_epochs + i] = q + tail;
}

// ---------------------------------------------------------------------------
// Chunked (parallel-in-time) form of the three recursions, for kernels of at
// most 6 states with white noise (sigma_w > 0) and every term of positive
// variance. The samples split into chunks of CL; one thread owns a chunk
// (J x J matrices in registers).
//
// Riccati. With R = sigma_w^2, one sample maps the predicted covariance as
// P -> Phi (P^-1 + h h^T / R)^-1 Phi^T + Qd, and maps of the form
// P -> A (P^-1 + Jm)^-1 A^T + C compose into the same form: applying
// (A2, C2, J2) after (A1, C1, J1) gives, with W = (I + C1 J2)^-1,
//   A = A2 W A1,  C = A2 W C1 A2^T + C2,  Jm = A1^T J2 W A1 + J1.
// For one more sample (J2 = h h^T / R, rank one) W = I - C1 h h^T / s with
// s = R + h^T C1 h, so a chunk composes in O(J^2) per sample:
//   A <- Phi (A - (C h)(h^T A) / s),  C <- Phi (C - (C h)(C h)^T / s) Phi^T + Qd,
//   Jm <- Jm + (A^T h)(A^T h)^T / s          (A^T h before the A update).
// ss_compose builds every chunk's map; ss_carry applies them in turn from
// Pinf, giving each chunk's true starting P, as
//   (P^-1 + Jm)^-1 = Z Z^T,  Z = Lp Rz^-T,  P = Lp Lp^T,  I + Lp^T Jm Lp = Rz Rz^T
// (two Cholesky factorisations, no pivoting: I + Lp^T Jm Lp has eigenvalues
// >= 1); ss_chunk_riccati then runs the per-sample filter of each chunk from
// its start, writing the same gain records as the sequential kernel.
//
// Linear recursions. With the gains known, x_{n+1} = M_n x_n + B_n v_n
// (M_n = Phi (I - k_n h^T)), the adjoint lambda_n = M_n^T lambda_{n+1} - ...
// and G_n = h h^T / S_n + M_n^T G_{n+1} M_n are affine in their state: each
// chunk runs from a zero state (its local part) and carries T_c = the
// product of its M_n (the forward pass of the unit vectors); a short
// sequential pass over chunks gives every chunk's true boundary state
// (x_s' = x_local + T_c x_s, lambda_s = lambda_local + T_c^T lambda_e,
// G_s = G_local + T_c^T G_e T_c); a final pass reruns each chunk from it.
constexpr int SS_CL = 192;       // samples per chunk
constexpr int SS_PAR_MAXJ = 6;   // largest state of the chunked path

template <int J>
struct Mat {
  double m[J][J];
};

// M <- Phi M (the rows of each block)
template <int NS, int NE>
__device__ __forceinline__ void rows_phi(const double* c, Mat<2 * NS + NE>& M) {
  constexpr int J = 2 * NS + NE;
#pragma unroll
  for (int s2 = 0; s2 < NS; ++s2)
#pragma unroll
    for (int b = 0; b < J; ++b) {
      const double r0 = M.m[2 * s2][b], r1 = M.m[2 * s2 + 1][b];
      M.m[2 * s2][b] = c[7 * s2] * r0 + c[7 * s2 + 1] * r1;
      M.m[2 * s2 + 1][b] = c[7 * s2 + 2] * r0 + c[7 * s2 + 3] * r1;
    }
#pragma unroll
  for (int e2 = 0; e2 < NE; ++e2)
#pragma unroll
    for (int b = 0; b < J; ++b) M.m[2 * NS + e2][b] *= c[7 * NS + 2 * e2];
}

// M <- Phi^T M
template <int NS, int NE>
__device__ __forceinline__ void rows_phi_t(const double* c, Mat<2 * NS + NE>& M) {
  constexpr int J = 2 * NS + NE;
#pragma unroll
  for (int s2 = 0; s2 < NS; ++s2)
#pragma unroll
    for (int b = 0; b < J; ++b) {
      const double r0 = M.m[2 * s2][b], r1 = M.m[2 * s2 + 1][b];
      M.m[2 * s2][b] = c[7 * s2] * r0 + c[7 * s2 + 2] * r1;
      M.m[2 * s2 + 1][b] = c[7 * s2 + 1] * r0 + c[7 * s2 + 3] * r1;
    }
#pragma unroll
  for (int e2 = 0; e2 < NE; ++e2)
#pragma unroll
    for (int b = 0; b < J; ++b) M.m[2 * NS + e2][b] *= c[7 * NS + 2 * e2];
}

// M <- M Phi^T
template <int NS, int NE>
__device__ __forceinline__ void cols_phi_t(const double* c, Mat<2 * NS + NE>& M) {
  constexpr int J = 2 * NS + NE;
#pragma unroll
  for (int a = 0; a < J; ++a) {
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) {
      const double m0 = M.m[a][2 * s2], m1 = M.m[a][2 * s2 + 1];
      M.m[a][2 * s2] = m0 * c[7 * s2] + m1 * c[7 * s2 + 1];
      M.m[a][2 * s2 + 1] = m0 * c[7 * s2 + 2] + m1 * c[7 * s2 + 3];
    }
#pragma unroll
    for (int e2 = 0; e2 < NE; ++e2) M.m[a][2 * NS + e2] *= c[7 * NS + 2 * e2];
  }
}

// M <- M Phi
template <int NS, int NE>
__device__ __forceinline__ void cols_phi(const double* c, Mat<2 * NS + NE>& M) {
  constexpr int J = 2 * NS + NE;
#pragma unroll
  for (int a = 0; a < J; ++a) {
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) {
      const double m0 = M.m[a][2 * s2], m1 = M.m[a][2 * s2 + 1];
      M.m[a][2 * s2] = m0 * c[7 * s2] + m1 * c[7 * s2 + 2];
      M.m[a][2 * s2 + 1] = m0 * c[7 * s2 + 1] + m1 * c[7 * s2 + 3];
    }
#pragma unroll
    for (int e2 = 0; e2 < NE; ++e2) M.m[a][2 * NS + e2] *= c[7 * NS + 2 * e2];
  }
}

// M += Qd on the block diagonal
template <int NS, int NE>
__device__ __forceinline__ void add_qd(const double* c, Mat<2 * NS + NE>& M) {
#pragma unroll
  for (int s2 = 0; s2 < NS; ++s2) {
    M.m[2 * s2][2 * s2] += c[7 * s2 + 4];
    M.m[2 * s2][2 * s2 + 1] += c[7 * s2 + 5];
    M.m[2 * s2 + 1][2 * s2] += c[7 * s2 + 5];
    M.m[2 * s2 + 1][2 * s2 + 1] += c[7 * s2 + 6];
  }
#pragma unroll
  for (int e2 = 0; e2 < NE; ++e2) M.m[2 * NS + e2][2 * NS + e2] += c[7 * NS + 2 * e2 + 1];
}

template <int J>
__device__ __forceinline__ void mat_load(const double* __restrict__ src, Mat<J>& M) {
#pragma unroll
  for (int a = 0; a < J; ++a)
#pragma unroll
    for (int b = 0; b < J; ++b) M.m[a][b] = src[a * J + b];
}

template <int J>
__device__ __forceinline__ void mat_store(const Mat<J>& M, double* __restrict__ dst) {
#pragma unroll
  for (int a = 0; a < J; ++a)
#pragma unroll
    for (int b = 0; b < J; ++b) dst[a * J + b] = M.m[a][b];
}

// lower Cholesky factor in place (the upper triangle is left as it is)
template <int J>
__device__ __forceinline__ void chol_lower(Mat<J>& M) {
#pragma unroll
  for (int j = 0; j < J; ++j) {
    double d = M.m[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) d = fma(-M.m[j][k], M.m[j][k], d);
    d = sqrt(d);
    M.m[j][j] = d;
    const double rd = 1.0 / d;
#pragma unroll
    for (int i = j + 1; i < J; ++i) {
      double v = M.m[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) v = fma(-M.m[i][k], M.m[j][k], v);
      M.m[i][j] = v * rd;
    }
  }
}

// One chunk's composed map (A, C, Jm), chunks 0 .. nch - 2 (the last one's is
// never applied).
template <int NS, int NE>
__global__ __launch_bounds__(64) void ss_compose_kernel(const double* __restrict__ step, double rr, int nch,
                                                        double* __restrict__ elems) {
  using Lt = SsLayout<NS, NE>;
  constexpr int J = Lt::J, TS = Lt::TS;
  const int c = blockIdx.x * 64 + threadIdx.x;
  if (c >= nch - 1) return;
  Mat<J> A, C, Jm;
#pragma unroll
  for (int a = 0; a < J; ++a)
#pragma unroll
    for (int b = 0; b < J; ++b) {
      A.m[a][b] = a == b ? 1.0 : 0.0;
      C.m[a][b] = 0.0;
      Jm.m[a][b] = 0.0;
    }
  const int64_t s0 = (int64_t)c * SS_CL;
  for (int64_t m = s0; m < s0 + SS_CL; ++m) {
    const double* cs = step + m * TS;
    double ch[J], ha[J];
    double sv = rr;
#pragma unroll
    for (int a = 0; a < J; ++a) {
      double v = 0.0, w = 0.0;
#pragma unroll
      for (int b = 0; b < J; ++b) {
        if (Lt::pos(b)) v += C.m[a][b];
        if (Lt::pos(b)) w += A.m[b][a];
      }
      ch[a] = v;
      ha[a] = w;
    }
#pragma unroll
    for (int a = 0; a < J; ++a)
      if (Lt::pos(a)) sv += ch[a];
    const double rs = 1.0 / sv;
#pragma unroll
    for (int a = 0; a < J; ++a) {
      const double ca = ch[a] * rs, hr = ha[a] * rs;
#pragma unroll
      for (int b = 0; b < J; ++b) {
        A.m[a][b] = fma(-ca, ha[b], A.m[a][b]);
        C.m[a][b] = fma(-ca, ch[b], C.m[a][b]);
        Jm.m[a][b] = fma(hr, ha[b], Jm.m[a][b]);
      }
    }
    rows_phi<NS, NE>(cs, A);
    rows_phi<NS, NE>(cs, C);
    cols_phi_t<NS, NE>(cs, C);
    add_qd<NS, NE>(cs, C);
  }
  double* out = elems + (int64_t)c * 3 * J * J;
  mat_store(A, out);
  mat_store(C, out + J * J);
  mat_store(Jm, out + 2 * J * J);
}

// Every chunk's starting covariance, applying the chunk maps in turn from
// Pinf (one thread); also clears the failure marker.
template <int NS, int NE>
__global__ __launch_bounds__(64) void ss_carry_kernel(const double* __restrict__ elems, nu_kernel kp, int nch,
                                                      int64_t n, double* __restrict__ pstart,
                                                      unsigned long long* __restrict__ failmin) {
  constexpr int J = 2 * NS + NE;
  if (threadIdx.x != 0) return;
  *failmin = (unsigned long long)n;
  Mat<J> P;
#pragma unroll
  for (int a = 0; a < J; ++a)
#pragma unroll
    for (int b = 0; b < J; ++b) P.m[a][b] = 0.0;
#pragma unroll
  for (int s2 = 0; s2 < NS; ++s2) {
    const double v0 = kp.sho_amp[s2] * kp.sho_amp[s2];
    P.m[2 * s2][2 * s2] = v0;
    P.m[2 * s2 + 1][2 * s2 + 1] = v0 * kp.sho_omega[s2] * kp.sho_omega[s2];
  }
#pragma unroll
  for (int e2 = 0; e2 < NE; ++e2) P.m[2 * NS + e2][2 * NS + e2] = kp.exp_sigma[e2] * kp.exp_sigma[e2];
  mat_store(P, pstart);
  for (int c = 0; c + 1 < nch; ++c) {
    const double* el = elems + (int64_t)c * 3 * J * J;
    Mat<J> L = P;
    chol_lower(L);  // P = L L^T
    // Y = I + L^T Jm L, then its lower factor R
    Mat<J> Jm, T, Y;
    mat_load(el + 2 * J * J, Jm);
#pragma unroll
    for (int a = 0; a < J; ++a)
#pragma unroll
      for (int b = 0; b < J; ++b) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < J; ++k) v = fma(Jm.m[a][k], (k >= b ? L.m[k][b] : 0.0), v);
        T.m[a][b] = v;  // Jm L
      }
#pragma unroll
    for (int a = 0; a < J; ++a)
#pragma unroll
      for (int b = 0; b < J; ++b) {
        double v = a == b ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < J; ++k) v = fma((k >= a ? L.m[k][a] : 0.0), T.m[k][b], v);
        Y.m[a][b] = v;
      }
    chol_lower(Y);
    // Z = L R^-T: row i of Z solves R z^T = (row i of L)^T
    Mat<J> Z;
#pragma unroll
    for (int i = 0; i < J; ++i)
#pragma unroll
      for (int j = 0; j < J; ++j) {
        double v = j <= i ? L.m[i][j] : 0.0;
#pragma unroll
        for (int k = 0; k < j; ++k) v = fma(-Y.m[j][k], Z.m[i][k], v);
        Z.m[i][j] = v / Y.m[j][j];
      }
    // P = (A Z)(A Z)^T + C
    Mat<J> A, AZ;
    mat_load(el, A);
#pragma unroll
    for (int a = 0; a < J; ++a)
#pragma unroll
      for (int b = 0; b < J; ++b) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < J; ++k) v = fma(A.m[a][k], Z.m[k][b], v);
        AZ.m[a][b] = v;
      }
    mat_load(el + J * J, P);
#pragma unroll
    for (int a = 0; a < J; ++a)
#pragma unroll
      for (int b = 0; b < J; ++b) {
        if (b < a) continue;
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < J; ++k) v = fma(AZ.m[a][k], AZ.m[b][k], v);
        const double cc = 0.5 * (P.m[a][b] + P.m[b][a]);
        P.m[a][b] = v + cc;
        P.m[b][a] = v + cc;
      }
    mat_store(P, pstart + (int64_t)(c + 1) * J * J);
  }
}

// The per-sample filter of each chunk from its starting covariance.
template <int NS, int NE>
__global__ __launch_bounds__(64) void ss_chunk_riccati_kernel(const double* __restrict__ step,
                                                              const double* __restrict__ pstart, int64_t n, int nch,
                                                              double rr, double* __restrict__ gain,
                                                              unsigned long long* __restrict__ failmin) {
  using Lt = SsLayout<NS, NE>;
  constexpr int J = Lt::J, TS = Lt::TS, GS = Lt::GS;
  const int c = blockIdx.x * 64 + threadIdx.x;
  if (c >= nch) return;
  Mat<J> P;
  mat_load(pstart + (int64_t)c * J * J, P);
  const int64_t s0 = (int64_t)c * SS_CL, s1 = min(n, s0 + SS_CL);
  for (int64_t m = s0; m < s1; ++m) {
    double ph[J];
    double S = rr;
#pragma unroll
    for (int a = 0; a < J; ++a) {
      double v = 0.0;
#pragma unroll
      for (int b = 0; b < J; ++b)
        if (Lt::pos(b)) v += P.m[a][b];
      ph[a] = v;
    }
#pragma unroll
    for (int a = 0; a < J; ++a)
      if (Lt::pos(a)) S += ph[a];
    if (!(S > 0.0 && S < INFINITY)) {
      atomicMin(failmin, (unsigned long long)m);
      return;
    }
    const double rsq = rsqrt_nr(S);
    const double rS = rsq * rsq;
    double* g = gain + m * GS;
    g[0] = rsq;
#pragma unroll
    for (int a = 0; a < J; ++a) g[1 + a] = ph[a] * rS;
    if (m + 1 == n) break;
    const double* cs = step + m * TS;
#pragma unroll
    for (int a = 0; a < J; ++a) {
      const double ka = ph[a] * rS;
#pragma unroll
      for (int b = 0; b < J; ++b) P.m[a][b] = fma(-ka, ph[b], P.m[a][b]);
    }
    rows_phi<NS, NE>(cs, P);
    cols_phi_t<NS, NE>(cs, P);
    add_qd<NS, NE>(cs, P);
  }
}

// x <- Phi (x + k e) with e = v - h.x; returns e
template <int NS, int NE>
__device__ __forceinline__ double filter_step(const double* g, const double* cs, double v, double* x, bool last) {
  using Lt = SsLayout<NS, NE>;
  constexpr int J = Lt::J;
  double hx = 0.0;
#pragma unroll
  for (int b = 0; b < J; ++b)
    if (Lt::pos(b)) hx += x[b];
  const double ev = v - hx;
  if (!last) {
#pragma unroll
    for (int b = 0; b < J; ++b) x[b] = fma(g[1 + b], ev, x[b]);
    apply_phi<NS, NE>(cs, x);
  }
  return ev;
}

// Forward local pass: thread (chunk c < nch - 1, column col < nv + J). Data
// columns start from 0 with v = V[., col]; column nv + j starts from the unit
// vector e_j with v = 0 and ends as column j of T_c. xe[c][col] = the state
// entering chunk c + 1.
template <int NS, int NE>
__global__ __launch_bounds__(64) void ss_fwd_local_kernel(const double* __restrict__ step,
                                                          const double* __restrict__ gain, int64_t n,
                                                          const double* __restrict__ V, int nv, int nch,
                                                          double* __restrict__ xe) {
  using Lt = SsLayout<NS, NE>;
  constexpr int J = Lt::J, TS = Lt::TS, GS = Lt::GS;
  const int cw = nv + J;
  const int t = blockIdx.x * 64 + threadIdx.x;
  const int c = t / cw, col = t - c * cw;
  if (c >= nch - 1) return;
  double x[J];
#pragma unroll
  for (int b = 0; b < J; ++b) x[b] = (col >= nv && b == col - nv) ? 1.0 : 0.0;
  const int64_t s0 = (int64_t)c * SS_CL;
  for (int64_t m = s0; m < s0 + SS_CL; ++m) {
    const double v = col < nv ? V[m * YCOLS + col] : 0.0;
    filter_step<NS, NE>(gain + m * GS, step + m * TS, v, x, false);
  }
  double* o = xe + ((int64_t)c * cw + col) * J;
#pragma unroll
  for (int b = 0; b < J; ++b) o[b] = x[b];
}

// Forward carry (one wave, lane = data column): xs[c] = the true state
// entering chunk c.
template <int NS, int NE>
__global__ __launch_bounds__(64) void ss_fwd_carry_kernel(const double* __restrict__ xe, int nv, int nch,
                                                          double* __restrict__ xs) {
  constexpr int J = 2 * NS + NE;
  const int col = threadIdx.x;
  if (col >= nv) return;
  const int cw = nv + J;
  double x[J];
#pragma unroll
  for (int b = 0; b < J; ++b) x[b] = 0.0;
  for (int c = 0; c < nch; ++c) {
    double* o = xs + ((int64_t)c * YCOLS + col) * J;
#pragma unroll
    for (int b = 0; b < J; ++b) o[b] = x[b];
    if (c + 1 == nch) break;
    const double* e = xe + (int64_t)c * cw * J;
    double y[J];
#pragma unroll
    for (int a = 0; a < J; ++a) {
      double v = e[col * J + a];
#pragma unroll
      for (int j = 0; j < J; ++j) v = fma(e[(nv + j) * J + a], x[j], v);
      y[a] = v;
    }
#pragma unroll
    for (int b = 0; b < J; ++b) x[b] = y[b];
  }
}

// Forward final pass: thread (chunk, data column) from the true entering
// state, writing Y = L^-1 V.
template <int NS, int NE>
__global__ __launch_bounds__(64) void ss_fwd_final_kernel(const double* __restrict__ step,
                                                          const double* __restrict__ gain, int64_t n,
                                                          const double* __restrict__ V, int nv, int nch,
                                                          const double* __restrict__ xs, double* __restrict__ Y) {
  using Lt = SsLayout<NS, NE>;
  constexpr int J = Lt::J, TS = Lt::TS, GS = Lt::GS;
  const int t = blockIdx.x * 64 + threadIdx.x;
  const int c = t / nv, col = t - c * nv;
  if (c >= nch) return;
  double x[J];
  const double* xi = xs + ((int64_t)c * YCOLS + col) * J;
#pragma unroll
  for (int b = 0; b < J; ++b) x[b] = xi[b];
  const int64_t s0 = (int64_t)c * SS_CL, s1 = min(n, s0 + SS_CL);
  for (int64_t m = s0; m < s1; ++m) {
    const double* g = gain + m * GS;
    const double ev = filter_step<NS, NE>(g, step + m * TS, V[m * YCOLS + col], x, m + 1 == n);
    Y[m * YCOLS + col] = ev * g[0];
  }
}

// One backward step of the adjoint: returns u_m, updates lambda.
template <int NS, int NE>
__device__ __forceinline__ double adjoint_step(const double* g, const double* cs, double w, double* lam, bool last) {
  using Lt = SsLayout<NS, NE>;
  constexpr int J = Lt::J;
  if (last) {
#pragma unroll
    for (int b = 0; b < J; ++b) lam[b] = 0.0;
  } else {
    apply_phi_t<NS, NE>(cs, lam);
  }
  double u = w * g[0];
#pragma unroll
  for (int b = 0; b < J; ++b) u = fma(g[1 + b], lam[b], u);
#pragma unroll
  for (int b = 0; b < J; ++b)
    if (Lt::pos(b)) lam[b] -= u;
  return u;
}

// G_m from G_{m+1}: h h^T / S_m + M_m^T G M_m, M_m = Phi (I - k_m h^T)
template <int NS, int NE>
__device__ __forceinline__ void gtail_step(const double* g, const double* cs, Mat<2 * NS + NE>& G, bool last) {
  using Lt = SsLayout<NS, NE>;
  constexpr int J = Lt::J;
  if (last) {
#pragma unroll
    for (int a = 0; a < J; ++a)
#pragma unroll
      for (int b = 0; b < J; ++b) G.m[a][b] = 0.0;
  } else {
    rows_phi_t<NS, NE>(cs, G);
    cols_phi<NS, NE>(cs, G);
  }
  double wk[J];
#pragma unroll
  for (int a = 0; a < J; ++a) {
    double v = 0.0;
#pragma unroll
    for (int b = 0; b < J; ++b) v = fma(G.m[a][b], g[1 + b], v);
    wk[a] = v;
  }
  double kwk = 0.0;
#pragma unroll
  for (int a = 0; a < J; ++a) kwk = fma(g[1 + a], wk[a], kwk);
  const double corner = kwk + g[0] * g[0];
#pragma unroll
  for (int a = 0; a < J; ++a)
#pragma unroll
    for (int b = 0; b < J; ++b) {
      double v = G.m[a][b];
      if (Lt::pos(a)) v -= wk[b];
      if (Lt::pos(b)) v -= wk[a];
      if (Lt::pos(a) && Lt::pos(b)) v += corner;
      G.m[a][b] = v;
    }
}

// Backward local pass: thread (chunk 1 <= c < nch, role). Roles < nv: the
// adjoint of column role from lambda = 0 after the chunk, giving
// ls[c][role] = the local lambda at the chunk's first sample; role nv: G from
// 0 after the chunk, giving Gl[c].
template <int NS, int NE>
__global__ __launch_bounds__(64) void ss_bwd_local_kernel(const double* __restrict__ step,
                                                          const double* __restrict__ gain, int64_t n,
                                                          const double* __restrict__ W, int nv, int nch,
                                                          double* __restrict__ ls, double* __restrict__ Gl) {
  using Lt = SsLayout<NS, NE>;
  constexpr int J = Lt::J, TS = Lt::TS, GS = Lt::GS;
  const int rw = nv + 1;
  const int t = blockIdx.x * 64 + threadIdx.x;
  const int c = 1 + t / rw, role = t - (c - 1) * rw;
  if (c >= nch) return;
  const int64_t s0 = (int64_t)c * SS_CL, s1 = min(n, s0 + SS_CL);
  if (role < nv) {
    double lam[J];
#pragma unroll
    for (int b = 0; b < J; ++b) lam[b] = 0.0;
    for (int64_t m = s1 - 1; m >= s0; --m) {
      const bool last = m + 1 == n;
      adjoint_step<NS, NE>(gain + m * GS, step + (last ? 0 : m) * TS, W[m * YCOLS + role], lam, last);
    }
    double* o = ls + ((int64_t)c * YCOLS + role) * J;
#pragma unroll
    for (int b = 0; b < J; ++b) o[b] = lam[b];
  } else {
    Mat<J> G;
#pragma unroll
    for (int a = 0; a < J; ++a)
#pragma unroll
      for (int b = 0; b < J; ++b) G.m[a][b] = 0.0;
    for (int64_t m = s1 - 1; m >= s0; --m) {
      const bool last = m + 1 == n;
      gtail_step<NS, NE>(gain + m * GS, step + (last ? 0 : m) * TS, G, last);
    }
    mat_store(G, Gl + (int64_t)c * J * J);
  }
}

// Backward carry, from the last chunk down. Workgroup 0, lane = column:
// le[c][col] = the true lambda entering chunk c from after its end. Workgroup
// 1, one thread: ge[c] = the true G after chunk c's end. T_c (columns
// xe[c][nv + j]) is the forward transfer of chunk c.
template <int NS, int NE>
__global__ __launch_bounds__(64) void ss_bwd_carry_kernel(const double* __restrict__ xe,
                                                          const double* __restrict__ ls,
                                                          const double* __restrict__ Gl, int nv, int nch,
                                                          double* __restrict__ le, double* __restrict__ ge) {
  constexpr int J = 2 * NS + NE;
  const int cw = nv + J;
  if (blockIdx.x == 0) {
    const int col = threadIdx.x;
    if (col >= nv) return;
    double lam[J];
#pragma unroll
    for (int b = 0; b < J; ++b) lam[b] = 0.0;
    for (int c = nch - 1; c >= 0; --c) {
      double* o = le + ((int64_t)c * YCOLS + col) * J;
#pragma unroll
      for (int b = 0; b < J; ++b) o[b] = lam[b];
      if (c == 0) break;
      // lambda at chunk c's first sample = local + T_c^T lambda_after (the
      // last chunk has nothing after it and no T)
      const double* e = xe + (int64_t)c * cw * J;
      const double* l0 = ls + ((int64_t)c * YCOLS + col) * J;
      const bool tail = c + 1 < nch;
      double y[J];
#pragma unroll
      for (int j = 0; j < J; ++j) {
        double v = l0[j];
        if (tail) {
#pragma unroll
          for (int a = 0; a < J; ++a) v = fma(e[(nv + j) * J + a], lam[a], v);
        }
        y[j] = v;
      }
#pragma unroll
      for (int b = 0; b < J; ++b) lam[b] = y[b];
    }
    return;
  }
  if (threadIdx.x != 0) return;
  Mat<J> G;
#pragma unroll
  for (int a = 0; a < J; ++a)
#pragma unroll
    for (int b = 0; b < J; ++b) G.m[a][b] = 0.0;
  for (int c = nch - 1; c >= 0; --c) {
    mat_store(G, ge + (int64_t)c * J * J);
    if (c == 0) break;
    if (c + 1 == nch) {  // nothing after the last chunk: G at its start is its local part
      mat_load(Gl + (int64_t)c * J * J, G);
      continue;
    }
    const double* e = xe + (int64_t)c * cw * J;
    Mat<J> T, GT;
#pragma unroll
    for (int a = 0; a < J; ++a)
#pragma unroll
      for (int j = 0; j < J; ++j) T.m[a][j] = e[(nv + j) * J + a];
#pragma unroll
    for (int a = 0; a < J; ++a)
#pragma unroll
      for (int b = 0; b < J; ++b) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < J; ++k) v = fma(G.m[a][k], T.m[k][b], v);
        GT.m[a][b] = v;
      }
    const double* gl = Gl + (int64_t)c * J * J;
#pragma unroll
    for (int a = 0; a < J; ++a)
#pragma unroll
      for (int b = 0; b < J; ++b) {
        if (b < a) continue;
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < J; ++k) v = fma(T.m[k][a], GT.m[k][b], v);
        const double cc = 0.5 * (gl[a * J + b] + gl[b * J + a]);
        G.m[a][b] = v + cc;
        G.m[b][a] = v + cc;
      }
  }
}

// Backward final pass: thread (chunk, role) from the true state after the
// chunk: the adjoint columns write Z, the G thread writes Gm (and G_n = 0).
template <int NS, int NE>
__global__ __launch_bounds__(64) void ss_bwd_final_kernel(const double* __restrict__ step,
                                                          const double* __restrict__ gain, int64_t n,
                                                          const double* __restrict__ W, int nv, int nch,
                                                          const double* __restrict__ le,
                                                          const double* __restrict__ ge, double* __restrict__ Z,
                                                          double* __restrict__ Gm) {
  using Lt = SsLayout<NS, NE>;
  constexpr int J = Lt::J, TS = Lt::TS, GS = Lt::GS;
  const int rw = nv + 1;
  const int t = blockIdx.x * 64 + threadIdx.x;
  const int c = t / rw, role = t - c * rw;
  if (c >= nch) return;
  const int64_t s0 = (int64_t)c * SS_CL, s1 = min(n, s0 + SS_CL);
  if (role < nv) {
    double lam[J];
    const double* li = le + ((int64_t)c * YCOLS + role) * J;
#pragma unroll
    for (int b = 0; b < J; ++b) lam[b] = li[b];
    for (int64_t m = s1 - 1; m >= s0; --m) {
      const bool last = m + 1 == n;
      Z[m * YCOLS + role] = adjoint_step<NS, NE>(gain + m * GS, step + (last ? 0 : m) * TS, W[m * YCOLS + role],
                                                 lam, last);
    }
  } else {
    Mat<J> G;
    mat_load(ge + (int64_t)c * J * J, G);
    if (s1 == n) mat_store(G, Gm + n * J * J);
    for (int64_t m = s1 - 1; m >= s0; --m) {
      const bool last = m + 1 == n;
      gtail_step<NS, NE>(gain + m * GS, step + (last ? 0 : m) * TS, G, last);
      mat_store(G, Gm + m * J * J);
    }
  }
}

// chunk buffers inside A.chunk (doubles), for nch chunks
struct ChunkWs {
  double *elems, *pstart, *xe, *xs, *ls, *le, *Gl, *ge;
  unsigned long long* failmin;
};

inline ChunkWs chunk_layout(double* base, int nch, int J) {
  ChunkWs w;
  const int64_t jj = (int64_t)J * J;
  double* p = base;
  w.elems = p;  p += (int64_t)nch * 3 * jj;
  w.pstart = p; p += (int64_t)nch * jj;
  w.xe = p;     p += (int64_t)nch * (YCOLS + J) * J;
  w.xs = p;     p += (int64_t)nch * YCOLS * J;
  w.ls = p;     p += (int64_t)nch * YCOLS * J;
  w.le = p;     p += (int64_t)nch * YCOLS * J;
  w.Gl = p;     p += (int64_t)nch * jj;
  w.ge = p;     p += (int64_t)nch * jj;
  w.failmin = reinterpret_cast<unsigned long long*>(p);
  return w;
}

template <int NS, int NE>
hipError_t launch_ss_chunked(int phase, hipStream_t s, const SsArgs& A) {
  using Lt = SsLayout<NS, NE>;
  constexpr int J = Lt::J;
  const int nch = (int)((A.n + SS_CL - 1) / SS_CL);
  const ChunkWs w = chunk_layout(A.chunk, nch, J);
  const double rr = A.kernel.sigma_w * A.kernel.sigma_w;
  auto blocks = [](int64_t threads) { return dim3((unsigned)((threads + 63) / 64)); };
  switch (phase) {
    case SS_PAR_RICCATI:
      if (nch > 1) {
        hipLaunchKernelGGL((ss_compose_kernel<NS, NE>), blocks(nch - 1), dim3(64), 0, s, A.step, rr, nch, w.elems);
        if (hipPeekAtLastError() != hipSuccess) break;
      }
      hipLaunchKernelGGL((ss_carry_kernel<NS, NE>), dim3(1), dim3(64), 0, s, w.elems, A.kernel, nch, A.n, w.pstart,
                         w.failmin);
      if (hipPeekAtLastError() != hipSuccess) break;
      hipLaunchKernelGGL((ss_chunk_riccati_kernel<NS, NE>), blocks(nch), dim3(64), 0, s, A.step, w.pstart, A.n, nch,
                         rr, A.gain, w.failmin);
      if (hipPeekAtLastError() != hipSuccess) break;
      hipLaunchKernelGGL(ss_logdet_kernel, dim3(1), dim3(256), 0, s, A.gain, Lt::GS, A.n,
                         (const unsigned long long*)w.failmin, A.status, A.logdet);
      break;
    case SS_PAR_FORWARD:
      if (nch > 1) {
        hipLaunchKernelGGL((ss_fwd_local_kernel<NS, NE>), blocks((int64_t)(nch - 1) * (A.nv + J)), dim3(64), 0, s,
                           A.step, A.gain, A.n, A.V, A.nv, nch, w.xe);
        if (hipPeekAtLastError() != hipSuccess) break;
      }
      hipLaunchKernelGGL((ss_fwd_carry_kernel<NS, NE>), dim3(1), dim3(64), 0, s, w.xe, A.nv, nch, w.xs);
      if (hipPeekAtLastError() != hipSuccess) break;
      hipLaunchKernelGGL((ss_fwd_final_kernel<NS, NE>), blocks((int64_t)nch * A.nv), dim3(64), 0, s, A.step, A.gain,
                         A.n, A.V, A.nv, nch, w.xs, A.Y);
      break;
    case SS_PAR_BACKWARD:
      if (nch > 1) {
        hipLaunchKernelGGL((ss_bwd_local_kernel<NS, NE>), blocks((int64_t)(nch - 1) * (A.nv + 1)), dim3(64), 0, s,
                           A.step, A.gain, A.n, A.Y, A.nv, nch, w.ls, w.Gl);
        if (hipPeekAtLastError() != hipSuccess) break;
      }
      hipLaunchKernelGGL((ss_bwd_carry_kernel<NS, NE>), dim3(2), dim3(64), 0, s, w.xe, w.ls, w.Gl, A.nv, nch, w.le,
                         w.ge);
      if (hipPeekAtLastError() != hipSuccess) break;
      hipLaunchKernelGGL((ss_bwd_final_kernel<NS, NE>), blocks((int64_t)nch * (A.nv + 1)), dim3(64), 0, s, A.step,
                         A.gain, A.n, A.Y, A.nv, nch, w.le, w.ge, A.Z, A.Gm);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int NS, int NE>
hipError_t launch_ss_typed(int phase, hipStream_t s, const SsArgs& A) {
  switch (phase) {
    case SS_RICCATI:
      hipLaunchKernelGGL((ss_riccati_kernel<NS, NE>), dim3(1), dim3(64), 0, s, A.step, A.kernel, A.n, A.gain,
                         A.status);
      if (hipPeekAtLastError() != hipSuccess) break;
      hipLaunchKernelGGL(ss_logdet_kernel, dim3(1), dim3(256), 0, s, A.gain, SsLayout<NS, NE>::GS, A.n,
                         (const unsigned long long*)nullptr, A.status, A.logdet);
      break;
    case SS_FORWARD:
      hipLaunchKernelGGL((ss_forward_kernel<NS, NE>), dim3(1), dim3(64), 0, s, A.step, A.gain, A.n, A.V, A.nv, A.Y);
      break;
    case SS_BACKWARD:
      hipLaunchKernelGGL((ss_backward_kernel<NS, NE>), dim3(2), dim3(64), 0, s, A.step, A.gain, A.n, A.Y, A.nv,
                         A.Z, A.Gm);
      break;
    case SS_BOX: {
      DurList dl{};
      dl.n = A.n_d;
      int dmax = 0;
      for (int k = 0; k < A.n_d; ++k) {
        dl.d[k] = A.dur_sorted[k];
        dl.perm[k] = A.dur_sorted[A.n_d + k];
        dmax = dl.d[k] > dmax ? dl.d[k] : dmax;
      }
      const int half = dmax / 2;
      const int64_t threads = A.n_epochs + half;
      hipLaunchKernelGGL((ss_box_kernel<NS, NE>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, A.step,
                         A.gain, A.Gm, A.n, A.lattice, A.slot_count, A.n_epochs, dl, half, A.qbox);
      break;
    }
    case SS_TEMPLATE: {
      DurList dl{};
      dl.n = A.n_d;
      int off = 0;
      for (int k = 0; k < A.n_d; ++k) {
        dl.d[k] = A.dur[k];
        dl.perm[k] = k;
        dl.off[k] = off;
        off += A.dur[k];
      }
      hipLaunchKernelGGL((ss_template_kernel<NS, NE>), dim3((unsigned)((A.n_epochs + 255) / 256), (unsigned)A.n_d),
                         dim3(256), 0, s, A.step, A.gain, A.Gm, A.n, A.lattice, A.slot_count, A.n_epochs, dl,
                         A.shapes, A.qbox);
      break;
    }
    case SS_PAR_RICCATI:
    case SS_PAR_FORWARD:
    case SS_PAR_BACKWARD:
      if constexpr (2 * NS + NE <= SS_PAR_MAXJ) return launch_ss_chunked<NS, NE>(phase, s, A);
      return hipErrorInvalidValue;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int NS>
hipError_t dispatch_ne(int phase, hipStream_t s, const SsArgs& A) {
  switch (A.n_exp) {
    case 0:
      if constexpr (NS > 0) return launch_ss_typed<NS, 0>(phase, s, A);
      return hipErrorInvalidValue;
    case 1: return launch_ss_typed<NS, 1>(phase, s, A);
    case 2: return launch_ss_typed<NS, 2>(phase, s, A);
    case 3: return launch_ss_typed<NS, 3>(phase, s, A);
    case 4: return launch_ss_typed<NS, 4>(phase, s, A);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_ss_step(hipStream_t s, const double* t, int64_t n, const nu_kernel& k, double* step) {
  if (n < 2) return hipSuccess;
  const int ts = 7 * k.n_sho + 2 * k.n_exp;
  hipLaunchKernelGGL(ss_step_kernel, dim3((unsigned)((n - 1 + 255) / 256)), dim3(256), 0, s, t, n, k, ts, step);
  return hipGetLastError();
}

size_t ss_chunk_ws_doubles(int64_t n, int J) {
  const int64_t nch = (n + SS_CL - 1) / SS_CL;
  const int64_t jj = (int64_t)J * J;
  return (size_t)(nch * (3 * jj + jj + (YCOLS + J) * J + 3 * YCOLS * J + 2 * jj) + 1);
}

bool ss_chunked_applies(const nu_kernel& k) {
  if (2 * k.n_sho + k.n_exp > SS_PAR_MAXJ || !(k.sigma_w > 0.0)) return false;
  for (int i = 0; i < k.n_sho; ++i)
    if (!(k.sho_amp[i] > 0.0)) return false;
  for (int i = 0; i < k.n_exp; ++i)
    if (!(k.exp_sigma[i] > 0.0)) return false;
  return true;
}

hipError_t launch_ss(int phase, hipStream_t s, const SsArgs& A) {
  switch (A.n_sho) {
    case 0: return dispatch_ne<0>(phase, s, A);
    case 1: return dispatch_ne<1>(phase, s, A);
    case 2: return dispatch_ne<2>(phase, s, A);
    case 3: return dispatch_ne<3>(phase, s, A);
    case 4: return dispatch_ne<4>(phase, s, A);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace nu
