// Periodic search (Sections 2.3-2.4): fold of the single-event grid over
// phases, common-depth combination (Eq. 8 with the estimates of Eq. B4), the
// argmax of Eq. 9 and Q(P) = depth / sigma; then the best period.
//
// One workgroup per trial period; thread = phase m, for groups of four
// durations at a time (the event positions m + k p are shared by all
// durations). Consecutive threads read consecutive epoch slots, so each
// event gather is one coalesced segment per wave. Interpolation is evaluated
// as written (this file is compiled without floating-point contraction); the
// sums run in increasing k.
#include <mutex>
#include <vector>

#include "batch_dev.hpp"
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

// 1/x for positive normal x: the hardware reciprocal estimate r with a
// third-order correction. With e = 1 - x r, 1/x = r (1 + e + e^2 + ...); the
// estimate has |e| <= 2^-24.4 (measured on gfx950 over 1e-300 .. 1e300), so
// r (1 + e + e^2) leaves a truncation below 2^-72 and is within 1 ulp: the
// accuracy of two Newton-Raphson steps with one FMA fewer.
__device__ __forceinline__ double rcp_nr(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

constexpr int FPAD = 64;  // padded slots after the grid (invalid), one wave wide
constexpr int WPH = 63;   // phases per wave: lane 63 only supplies its neighbour

// Packed copy of the single-event grid for the fold: rows of n_t + FPAD slots
// holding (depth, var) pairs and dll; var = NaN where the cell is invalid or
// past the grid, so "valid and inside the grid" is var == var.
__device__ __forceinline__ void fold_pack_at(const double* __restrict__ depth, const double* __restrict__ var,
                                             const double* __restrict__ dll, const uint8_t* __restrict__ valid,
                                             int n_d, int64_t n_t, double2* __restrict__ DV, double* __restrict__ Lp,
                                             int64_t e) {
  const int64_t ld = n_t + FPAD;
  if (e >= (int64_t)n_d * ld) return;
  const int j = (int)(e / ld);
  const int64_t i = e - (int64_t)j * ld;
  double d = 0.0, v = NAN, l = 0.0;
  if (i < n_t) {
    const int64_t o = (int64_t)j * n_t + i;
    if (valid[o]) {
      d = depth[o];
      v = var[o];
      l = dll[o];
    }
  }
  DV[e] = make_double2(d, v);
  Lp[e] = l;
}

__global__ __launch_bounds__(256) void fold_pack_kernel(const double* __restrict__ depth,
                                                        const double* __restrict__ var,
                                                        const double* __restrict__ dll,
                                                        const uint8_t* __restrict__ valid, int n_d, int64_t n_t,
                                                        double2* __restrict__ DV, double* __restrict__ Lp) {
  fold_pack_at(depth, var, dll, valid, n_d, n_t, DV, Lp, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// lane i receives lane i+1's value (DPP wave shift; lane 63 receives 0 through
// the bound control, with no old value to set up)
__device__ __forceinline__ double from_next_lane(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x130, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x130, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// (1 - w) x + w y with u = 1 - w, the second product rounded into the sum
__device__ __forceinline__ double interp(double u, double w, double x, double y) { return fma(w, y, u * x); }

// min of two doubles that are not NaN: one v_min_f64 (fmin would first quiet
// both operands, as a signalling NaN could reach it as far as the compiler knows)
__device__ __forceinline__ double min_num(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Element idx (>= 0, within 2^32 bytes of the row start: the periodic search
// accepts at most 2^27 epoch slots) of a row whose start is wave-uniform: a
// 32-bit byte offset from a scalar base, so the load takes the scalar-base
// form with no per-lane 64-bit address arithmetic.
__device__ __forceinline__ double row_at(const double* row, int idx) {
  return *(const NU_GLOBAL double*)((const NU_GLOBAL char*)row + 8u * (uint32_t)idx);
}
__device__ __forceinline__ double2 row_at(const double2* row, int idx) {
  typedef double d2v __attribute__((ext_vector_type(2)));
  const d2v v = *(const NU_GLOBAL d2v*)((const NU_GLOBAL char*)row + 16u * (uint32_t)idx);
  return make_double2(v.x, v.y);
}

// Segments of one global lattice (sectors with their own linear searches):
// segment s covers global slots [off[s], off[s] + len[s]); the packed grid
// holds each segment's slots at [pstart[s], pstart[s] + len[s]) of a row,
// with FPAD invalid slots before and after every segment, and the caller's
// grid holds segment s as an [n_d][len[s]] block at in_start[s].
struct Segs {
  int n;
  int64_t off[MAX_SEG], len[MAX_SEG], pstart[MAX_SEG], in_start[MAX_SEG];
};

// Event base b of a wave (global slot mb + b for lane 0) on a segmented grid:
// advances the segment cursor and gives the packed offset of the window in
// *delta; or, when the 64-slot window lies in the gap before segment *seg,
// returns false with the next k worth trying (one below the first k whose
// window could reach the segment, to stay clear of rounding in k p).
// Segments are at least FPAD slots apart, so a window touches one segment and
// the lanes outside it read that segment's padding.
__device__ __forceinline__ bool seg_event(const Segs& S, int64_t mb, int64_t b, int64_t k, double p, int& seg,
                                          int64_t& delta, int64_t& knext) {
  const int64_t g0 = mb + b;
  while (seg < S.n - 1 && g0 > S.off[seg] + S.len[seg] - 1) ++seg;
  if (g0 + 63 < S.off[seg]) {
    const int64_t kj = (int64_t)ceil((double)(S.off[seg] - 63 - mb) / p) - 1;
    knext = kj > k ? kj : k + 1;
    return false;
  }
  delta = S.pstart[seg] - S.off[seg];
  return true;
}

// Eq. 8 with the estimates of Eq. B4, for the durations j0 .. j0+JG-1 and the
// phases m = mb + lane of one wave. All lanes share base_k = floor(k p) and
// w_k, so an event's right-hand slot is the next lane's left-hand slot; the
// interpolation (1 - w) V_i + w V_i+1 rounds the second product into the sum
// (one FMA), within an ulp of the separately rounded form.
// The sum of log ratios is taken as one logarithm of a product:
//   sum_k [ln var_k - ln(sigma^2 + var_k)] = ln prod_k var_k / (var_k + sigma^2),
// where the product lies in [1/e, 1) because sigma^2 sum_k 1/var_k = 1; one
// reciprocal r = 1 / (var_k + sigma^2) per event gives both the factor
// var_k r and the chi^2 term (d_k - D)^2 r.
//
// Pass 2 (the chi^2 and log terms, which need the combined depth and sigma^2
// of pass 1) is skipped for a group of durations when no cell of the wave can
// reach the best lnP found so far for this period (thr, from any wave of the
// workgroup). The bound, from pass-1 sums alone: with L = -ln prod in [0, 1],
//   lnP = S_ll - (-s L + chi^2) / 2 <= S_ll + [s > 0] / 2 - chi^2 / 2,
// and, since sigma^2 <= v_min (the smallest var_k) and sum_k (d_k - D) / v_k = 0,
//   chi^2 >= sum_k (d_k - D)^2 / (v_k (1 + sigma^2 / v_min))
//         = (sum_k d_k^2 / v_k - D^2 S_w) / (1 + sigma^2 / v_min).
// A skipped cell's lnP is below a value some cell reaches, so the argmax and
// every per-period output are unchanged; a relative margin covers rounding.
template <int JG, bool SEG>  // durations per pass over the events; segmented grid
__device__ __forceinline__ void fold_cells(const double2* __restrict__ DV, const double* __restrict__ Lp, int n_d,
                                           int64_t n_t, int64_t ld, const Segs& S, int j0, int64_t mb, int lane,
                                           int64_t nph, double p, double sign, double thr, Best& best) {
  const int64_t m = mb + lane;
  const int64_t kmax_base = n_t - 1 - mb;  // events while base_k <= this (uniform)
  // the rows of the group from the wave's first phase: uniform pointers, so an
  // event's loads share one 32-bit lane offset
  const double2* dvr[JG];
  const double* lpr[JG];
#pragma unroll
  for (int g = 0; g < JG; ++g) {
    const int64_t r0 = (int64_t)min(j0 + g, n_d - 1) * ld + mb;
    dvr[g] = DV + r0;
    lpr[g] = Lp + r0;
  }
  // s_w > 0 once a cell has an event (every valid var is positive and finite)
  double s_w[JG], s_wd[JG], s_ll[JG], s_dd[JG];
  double vmin = INFINITY;  // over the group's durations: a smaller v_min only loosens the bound
#pragma unroll
  for (int g = 0; g < JG; ++g) s_w[g] = s_wd[g] = s_ll[g] = s_dd[g] = 0.0;
  // one event of pass 1 for every duration of the group, from its loaded slots
  auto event1 = [&](const double2 (&dv)[JG], const double (&l)[JG], double w) {
    const double u = 1.0 - w;
#pragma unroll
    for (int g = 0; g < JG; ++g) {
      double d = dv[g].x, v = dv[g].y, ll = l[g];
      if (w != 0.0) {
        d = interp(u, w, d, from_next_lane(d));
        v = interp(u, w, v, from_next_lane(v));
        ll = interp(u, w, ll, from_next_lane(ll));
      }
      if (v == v && j0 + g < n_d) {
        const double iv = rcp_nr(v);
        const double dw = d * iv;
        s_w[g] = s_w[g] + iv;
        s_wd[g] = s_wd[g] + dw;
        s_dd[g] = fma(d, dw, s_dd[g]);  // enters only the skipping bound, which has a margin
        s_ll[g] = s_ll[g] + ll;
        vmin = min_num(vmin, v);
      }
    }
  };
  // pass 1 (k counts events as an int64 and, exactly, as a double for k p)
  int seg = 0;
  double kd = 0.0;
  for (int64_t k = 0;; ++k, kd += 1.0) {
    const double kp = kd * p;
    const double base = floor(kp);
    if (base > (double)kmax_base) break;
    int b = (int)base;
    if constexpr (SEG) {
      int64_t delta, knext;
      if (!seg_event(S, mb, b, k, p, seg, delta, knext)) {
        k = knext - 1;
        kd = (double)k;
        continue;
      }
      b += (int)delta;
    }
    const int idx = lane + b;
    double2 dv[JG];
    double l[JG];
#pragma unroll
    for (int g = 0; g < JG; ++g) {
      if constexpr (SEG) {  // idx may be negative there (the window's packed offset)
        dv[g] = dvr[g][idx];
        l[g] = lpr[g][idx];
      } else {
        dv[g] = row_at(dvr[g], idx);
        l[g] = row_at(lpr[g], idx);
      }
    }
    event1(dv, l, kp - base);
  }
  double s2[JG], dc[JG], prod[JG], chi[JG];
  bool need[JG];
  bool any_need = false;
#pragma unroll
  for (int g = 0; g < JG; ++g) {
    s2[g] = rcp_nr(s_w[g]);  // used only where s_w > 0
    dc[g] = s2[g] * s_wd[g];
    prod[g] = 1.0;
    chi[g] = 0.0;
    bool mine = false;
    if (j0 + g < n_d && s_w[g] > 0.0 && m < nph && lane < WPH) {
      // ub + margin < thr with chi_lb = chi_ub v_min / (v_min + sigma^2), multiplied
      // out by v_min + sigma^2 > 0 (no division)
      const double chi_ub = fmax(s_dd[g] - dc[g] * dc[g] * s_w[g], 0.0);
      const double margin = 1e-9 * (1.0 + fabs(s_ll[g]) + s_dd[g]);
      const double x = s_ll[g] + (sign > 0.0 ? 0.5 : 0.0) + margin - thr;
      mine = !(x * (vmin + s2[g]) < 0.5 * chi_ub * vmin);  // NaN: evaluated
    }
    need[g] = __ballot(mine) != 0;
    any_need = any_need || need[g];
  }
  if (!any_need) return;
  // one event of pass 2 for the durations that need it
  auto event2 = [&](const double2 (&dv)[JG], double w) {
    const double u = 1.0 - w;
#pragma unroll
    for (int g = 0; g < JG; ++g) {
      if (!need[g]) continue;
      double d = dv[g].x, v = dv[g].y;
      if (w != 0.0) {
        d = interp(u, w, d, from_next_lane(d));
        v = interp(u, w, v, from_next_lane(v));
      }
      if (v == v && s_w[g] > 0.0) {
        const double r = rcp_nr(v + s2[g]);  // 1 / (var_k + sigma^2)
        prod[g] = prod[g] * (v * r);
        const double dd = d - dc[g];
        chi[g] = fma(dd * dd, r, chi[g]);  // (d_k - d)^2 / (var_k + sigma^2)
      }
    }
  };
  // pass 2
  seg = 0;
  kd = 0.0;
  for (int64_t k = 0;; ++k, kd += 1.0) {
    const double kp = kd * p;
    const double base = floor(kp);
    if (base > (double)kmax_base) break;
    int b = (int)base;
    if constexpr (SEG) {
      int64_t delta, knext;
      if (!seg_event(S, mb, b, k, p, seg, delta, knext)) {
        k = knext - 1;
        kd = (double)k;
        continue;
      }
      b += (int)delta;
    }
    const int idx = lane + b;
    // every group's slots, needed or not: conditional loads made the compiler
    // wait for each one before issuing the next
    double2 dv[JG];
#pragma unroll
    for (int g = 0; g < JG; ++g) {
      if constexpr (SEG) {
        dv[g] = dvr[g][idx];
      } else {
        dv[g] = row_at(dvr[g], idx);
      }
    }
    event2(dv, kp - base);
  }
#pragma unroll
  for (int g = 0; g < JG; ++g) {
    const int j = j0 + g;
    if (need[g] && j < n_d && s_w[g] > 0.0 && m < nph && lane < WPH) {
      // ln prod lies in [-1, 0): a cell whose bound stays below the lane's best
      // (with a margin for rounding) cannot win, and skips the logarithm
      const double ubx = s_ll[g] - 0.5 * chi[g] + (sign > 0.0 ? 0.5 : 0.0);
      if (!(ubx + 1e-9 * (1.0 + fabs(s_ll[g]) + chi[g]) < best.val)) {
        const double corr = sign * log(prod[g]) + chi[g];
        const double lnp = s_ll[g] - 0.5 * corr;
        Best cand{lnp, m * (int64_t)n_d + j, dc[g], s2[g]};
        if (lnp == lnp && lnp > -INFINITY && beats(cand, best)) best = cand;
      }
    }
  }
}

template <int JG, bool SEG>
__device__ __forceinline__ void fold_period_block(const double2* __restrict__ DV, const double* __restrict__ Lp,
                                                  int n_d, int64_t n_t, int64_t ld, const Segs& S, double dt,
                                                  const double* __restrict__ periods, double sign,
                                                  double* __restrict__ q_snr, int64_t* __restrict__ best_phase,
                                                  int32_t* __restrict__ best_dur, double* __restrict__ best_depth,
                                                  double* __restrict__ best_sigma, double* __restrict__ best_lnp,
                                                  int64_t ip) {
  __shared__ Best red[256];
  __shared__ double wave_best[4];  // best lnP found so far by each wave (only rises)
  // the wave index is uniform within a wave: read it into a scalar register, so
  // that the phase base and the per-duration row pointers derived from it stay
  // scalar and each event's loads share one 32-bit lane offset
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (tid < 4) wave_best[tid] = -INFINITY;
  __syncthreads();
  // the waves' best values are read and written as relaxed workgroup-scope
  // atomics on the LDS array: plain ds operations (a volatile generic pointer
  // made each read a serialised flat access)
  auto wb_get = [&](int w) { return __hip_atomic_load(&wave_best[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); };
  const double P = periods[ip];
  const double p = P / dt;
  Best best{-INFINITY, -1, 0.0, 0.0};
  // a period below one cadence (p < 1), or not finite, has no event: the
  // phase grid steps by one cadence (Section 2.3)
  if (p >= 1.0 && p < INFINITY) {
    const double nph_d = ceil(p);
    const int64_t nph = nph_d < (double)n_t ? (int64_t)nph_d : n_t;  // phases >= n_t hold no event
    for (int64_t mb = (int64_t)wave * WPH; mb < nph; mb += 4 * WPH)
      for (int j0 = 0; j0 < n_d; j0 += JG) {
        // read without synchronisation: a stale value only prunes less
        const double thr = fmax(fmax(wb_get(0), wb_get(1)), fmax(wb_get(2), wb_get(3)));
        const double before = best.val;
        fold_cells<JG, SEG>(DV, Lp, n_d, n_t, ld, S, j0, mb, lane, nph, p, sign, thr, best);
        // the wave's best, published for the other waves' skipping, only when
        // some lane found a better cell in this call
        if (__ballot(best.val != before) != 0) {
          double v = best.flat >= 0 ? best.val : -INFINITY;
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
          if (lane == 0 && v > wb_get(wave))
            __hip_atomic_store(&wave_best[wave], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
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

template <int JG, bool SEG>
__global__ __launch_bounds__(256, 3) void fold_kernel(const double2* __restrict__ DV, const double* __restrict__ Lp,
                                                   int n_d, int64_t n_t, int64_t ld, const Segs S, double dt,
                                                   const double* __restrict__ periods, double sign,
                                                   double* __restrict__ q_snr, int64_t* __restrict__ best_phase,
                                                   int32_t* __restrict__ best_dur, double* __restrict__ best_depth,
                                                   double* __restrict__ best_sigma, double* __restrict__ best_lnp) {
  fold_period_block<JG, SEG>(DV, Lp, n_d, n_t, ld, S, dt, periods, sign, q_snr, best_phase, best_dur, best_depth,
                             best_sigma, best_lnp, (int64_t)blockIdx.x);
}

// durations per pass: 5 when that pads fewer cells than 4 (10 durations: 10 rather than 12)
template <bool SEG>
static hipError_t launch_fold_kernel(hipStream_t s, const double2* DV, const double* Lp, int n_d, int64_t n_t,
                                     int64_t ld, const Segs& S, double dt, const double* periods, int64_t n_p,
                                     int sign, double* q_snr, int64_t* best_phase, int32_t* best_dur,
                                     double* best_depth, double* best_sigma, double* best_lnp) {
  const int pad4 = (n_d + 3) / 4 * 4, pad5 = (n_d + 4) / 5 * 5;
  if (pad5 < pad4)
    hipLaunchKernelGGL((fold_kernel<5, SEG>), dim3((unsigned)n_p), dim3(256), 0, s, DV, Lp, n_d, n_t, ld, S, dt,
                       periods, (double)sign, q_snr, best_phase, best_dur, best_depth, best_sigma, best_lnp);
  else
    hipLaunchKernelGGL((fold_kernel<4, SEG>), dim3((unsigned)n_p), dim3(256), 0, s, DV, Lp, n_d, n_t, ld, S, dt,
                       periods, (double)sign, q_snr, best_phase, best_dur, best_depth, best_sigma, best_lnp);
  return hipGetLastError();
}

hipError_t launch_fold(hipStream_t s, const double* depth, const double* var, const double* dll,
                       const uint8_t* valid, int n_d, int64_t n_epochs, double dt, const double* periods, int64_t n_p,
                       int sign, double* q_snr, int64_t* best_phase, int32_t* best_dur, double* best_depth,
                       double* best_sigma, double* best_lnp, double* packed) {
  const int64_t ld = n_epochs + FPAD;
  double2* DV = reinterpret_cast<double2*>(packed);
  double* Lp = packed + 2 * (int64_t)n_d * ld;
  const int64_t tot = (int64_t)n_d * ld;
  hipLaunchKernelGGL(fold_pack_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, depth, var, dll, valid,
                     n_d, n_epochs, DV, Lp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_fold_kernel<false>(s, DV, Lp, n_d, n_epochs, ld, Segs{}, dt, periods, n_p, sign, q_snr, best_phase,
                                   best_dur, best_depth, best_sigma, best_lnp);
}

// Packed grid of a segmented search (layout in Segs).
__global__ __launch_bounds__(256) void fold_pack_segments_kernel(const double* __restrict__ depth,
                                                                 const double* __restrict__ var,
                                                                 const double* __restrict__ dll,
                                                                 const uint8_t* __restrict__ valid, int n_d,
                                                                 const Segs S, int64_t ld, double2* __restrict__ DV,
                                                                 double* __restrict__ Lp) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n_d * ld) return;
  const int j = (int)(e / ld);
  const int64_t pos = e - (int64_t)j * ld;
  double d = 0.0, v = NAN, l = 0.0;
  for (int s = 0; s < S.n; ++s)
    if (pos >= S.pstart[s] && pos < S.pstart[s] + S.len[s]) {
      const int64_t o = S.in_start[s] + (int64_t)j * S.len[s] + (pos - S.pstart[s]);
      if (valid[o]) {
        d = depth[o];
        v = var[o];
        l = dll[o];
      }
      break;
    }
  DV[e] = make_double2(d, v);
  Lp[e] = l;
}

// row length of the packed grid of a segmented search
static int64_t seg_row(const int64_t* len, int n_seg) {
  int64_t t = FPAD;
  for (int s = 0; s < n_seg; ++s) t += len[s] + FPAD;
  return t;
}

size_t fold_segments_workspace_doubles(int n_d, const int64_t* len, int n_seg) {
  return (size_t)3 * n_d * (size_t)seg_row(len, n_seg);
}

hipError_t launch_fold_segments(hipStream_t s, const double* depth, const double* var, const double* dll,
                                const uint8_t* valid, int n_d, int n_seg, const int64_t* seg_len,
                                const int64_t* seg_off, double dt, const double* periods, int64_t n_p, int sign,
                                double* q_snr, int64_t* best_phase, int32_t* best_dur, double* best_depth,
                                double* best_sigma, double* best_lnp, double* packed) {
  if (n_seg < 1 || n_seg > MAX_SEG) return hipErrorInvalidValue;
  Segs S{};
  S.n = n_seg;
  int64_t pstart = FPAD, in_start = 0;
  for (int i = 0; i < n_seg; ++i) {
    S.off[i] = seg_off[i];
    S.len[i] = seg_len[i];
    S.pstart[i] = pstart;
    S.in_start[i] = in_start;
    pstart += seg_len[i] + FPAD;
    in_start += (int64_t)n_d * seg_len[i];
  }
  const int64_t ld = seg_row(seg_len, n_seg);
  const int64_t n_t = seg_off[n_seg - 1] + seg_len[n_seg - 1];  // global extent
  double2* DV = reinterpret_cast<double2*>(packed);
  double* Lp = packed + 2 * (int64_t)n_d * ld;
  const int64_t tot = (int64_t)n_d * ld;
  hipLaunchKernelGGL(fold_pack_segments_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, depth, var, dll,
                     valid, n_d, S, ld, DV, Lp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_fold_kernel<true>(s, DV, Lp, n_d, n_t, ld, S, dt, periods, n_p, sign, q_snr, best_phase, best_dur,
                                  best_depth, best_sigma, best_lnp);
}

size_t fold_workspace_doubles(int n_d, int64_t n_epochs) { return (size_t)3 * n_d * (size_t)(n_epochs + FPAD); }

// ---------------------------------------------------------------------------
// The allocation-free periodic search keeps its packed grid in a fixed device
// array instead of the context's workspace. Each GPU the library runs on holds
// its own copy of the array until the process ends; in host code its name
// stands for no device address, so the host takes each device's address once
// (hipGetSymbolAddress with that device current) and passes that pointer to
// the kernels. Every call on a device shares its array: calls that overlap on
// one device race. The fold's pack kernel writes every element of the part a
// call uses, so nothing needs clearing between calls.
static __device__ __align__(256) double scratch[FOLD_SCRATCH_DOUBLES];

namespace {
std::mutex scratch_mu;
std::vector<double*> scratch_dev;  // per device; nullptr until looked up
}  // namespace

hipError_t fold_scratch_ptr(int device, double** out) {
  *out = nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (device < 0) return hipErrorInvalidDevice;
  if ((size_t)device >= scratch_dev.size()) scratch_dev.resize((size_t)device + 1, nullptr);
  if (!scratch_dev[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current
    double* p = nullptr;
    e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    scratch_dev[device] = p;
  }
  *out = scratch_dev[device];
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Search for further candidates (Section 3.3, the search of TOI-540): the trial
// epochs in windows of width 2 D centred on a found candidate's transits are
// masked in the linear-search products, which the next periodic search then
// skips. Transit k of the candidate sits at slot m + k p (any integer k), the
// position the fold combines; slot i is masked, for every duration, when
// |(i - m) - k p| < h for some k, evaluated with one rounding for k p (this
// file is compiled without floating-point contraction). One thread per slot;
// the k range covers [(i - m - h) / p, (i - m + h) / p] with a margin of one.
__global__ __launch_bounds__(256) void mask_transit_kernel(double* __restrict__ depth, double* __restrict__ var,
                                                           double* __restrict__ dll, uint8_t* __restrict__ valid,
                                                           int n_d, int64_t n_t, double p, int64_t m, int h) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n_t) return;
  const double x = (double)(i - m), hd = (double)h;
  const int64_t k_lo = (int64_t)floor((x - hd) / p) - 1, k_hi = (int64_t)ceil((x + hd) / p) + 1;
  bool hit = false;
  for (int64_t k = k_lo; k <= k_hi && !hit; ++k) hit = fabs(x - (double)k * p) < hd;
  if (!hit) return;
  for (int j = 0; j < n_d; ++j) {
    const int64_t o = (int64_t)j * n_t + i;
    depth[o] = 0.0;
    var[o] = INFINITY;
    dll[o] = 0.0;
    valid[o] = 0;
  }
}

hipError_t launch_mask_transit(hipStream_t s, double* depth, double* var, double* dll, uint8_t* valid, int n_d,
                               int64_t n_t, double p, int64_t m, int h) {
  hipLaunchKernelGGL(mask_transit_kernel, dim3((unsigned)((n_t + 255) / 256)), dim3(256), 0, s, depth, var, dll,
                     valid, n_d, n_t, p, m, h);
  return hipGetLastError();
}

// First period of largest Q (NaN never wins).
__device__ __forceinline__ void best_period_block(const double* __restrict__ q, int64_t n_p,
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

__global__ __launch_bounds__(1024) void best_period_kernel(const double* __restrict__ q, int64_t n_p,
                                                           int64_t* __restrict__ out) {
  best_period_block(q, n_p, out);
}

hipError_t launch_best_period(hipStream_t s, const double* q_snr, int64_t n_p, int64_t* out) {
  hipLaunchKernelGGL(best_period_kernel, dim3(1), dim3(1024), 0, s, q_snr, n_p, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched forms of the periodic search: the packed grids of every curve, the
// fold over (period, curve) and the best period of every curve, one launch
// each (workgroups of the pack numbered curve after curve, see CurveJob).

__global__ __launch_bounds__(256) void batch_fold_pack_kernel(const CurveJob* __restrict__ jobs,
                                                              const int* __restrict__ begin, int n_curves, int n_d) {
  int u;
  const CurveJob& J = jobs[batch_find(begin, n_curves, (int)blockIdx.x, u)];
  const int64_t ld = J.n_epochs + FPAD;
  fold_pack_at(J.depth, J.var, J.dll, J.valid, n_d, J.n_epochs, reinterpret_cast<double2*>(J.packed),
               J.packed + 2 * (int64_t)n_d * ld, (int64_t)u * 256 + threadIdx.x);
}

template <int JG>
__global__ __launch_bounds__(256, 3) void batch_fold_kernel(const CurveJob* __restrict__ jobs, int n_d,
                                                         const double* __restrict__ periods, double sign) {
  const CurveJob& J = jobs[blockIdx.y];
  const int64_t ld = J.n_epochs + FPAD;
  fold_period_block<JG, false>(reinterpret_cast<const double2*>(J.packed), J.packed + 2 * (int64_t)n_d * ld, n_d,
                               J.n_epochs, ld, Segs{}, J.dt, periods, sign, J.q_snr, J.best_phase, J.best_dur,
                               J.best_depth, J.best_sigma, J.best_lnp, (int64_t)blockIdx.x);
}

// the best period of every curve; -1 for a curve whose factorisation failed
// (status_out: the statuses collected by curve index, see launch_batch_collect)
__global__ __launch_bounds__(1024) void batch_best_kernel(const CurveJob* __restrict__ jobs, int64_t n_p,
                                                          const int64_t* __restrict__ status_out) {
  const CurveJob& J = jobs[blockIdx.x];
  if (!J.best_index) return;
  if (status_out[J.curve] >= 0) {
    if (threadIdx.x == 0) *J.best_index = -1;
    return;
  }
  best_period_block(J.q_snr, n_p, J.best_index);
}

hipError_t launch_batch_fold(hipStream_t s, const CurveJob* jobs, const int* begin_pack, int n_curves,
                             int total_pack, int n_d, const double* periods, int64_t n_p, int sign) {
  if (total_pack > 0) {
    hipLaunchKernelGGL(batch_fold_pack_kernel, dim3((unsigned)total_pack), dim3(256), 0, s, jobs, begin_pack,
                       n_curves, n_d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int pad4 = (n_d + 3) / 4 * 4, pad5 = (n_d + 4) / 5 * 5;
  const dim3 g((unsigned)n_p, (unsigned)n_curves);
  if (pad5 < pad4)
    hipLaunchKernelGGL(batch_fold_kernel<5>, g, dim3(256), 0, s, jobs, n_d, periods, (double)sign);
  else
    hipLaunchKernelGGL(batch_fold_kernel<4>, g, dim3(256), 0, s, jobs, n_d, periods, (double)sign);
  return hipGetLastError();
}

hipError_t launch_batch_best(hipStream_t s, const CurveJob* jobs, int n_curves, int64_t n_p,
                             const int64_t* status_out) {
  hipLaunchKernelGGL(batch_best_kernel, dim3((unsigned)n_curves), dim3(1024), 0, s, jobs, n_p, status_out);
  return hipGetLastError();
}

}  // namespace nu
