/*
 * nuance_mi355x.h -- C ABI of the MI355X (gfx950) transit-search hot path.
 *
 * The method is nuance (Garcia et al., arXiv:2402.06835): a linear search
 * that fits, at every trial epoch and duration, a box transit plus a linear
 * trend by generalised least squares under a fixed Gaussian-process
 * covariance (Section 2.2, Eqs. 5-6), followed by a periodic search that
 * combines those single events over a period x phase grid with a common
 * depth (Section 2.3, Eq. 8 with the estimates of Eq. B4) and reports the
 * periodogram Q(P) = depth/sigma at the best phase and duration (Section
 * 2.4, Eq. 9).
 *
 * Conventions for every entry point:
 *  - No C++ exception crosses this boundary. Every call returns a nu_status;
 *    nu_ctx_last_error() gives a message for the last non-OK status.
 *  - Pointers named *_host are host memory; every other array pointer is
 *    DEVICE memory on the context's device, owned by the caller, and must
 *    stay valid until the enqueued work has finished.
 *  - All device work is enqueued on the context's stream (the caller's, e.g.
 *    torch.cuda.current_stream().cuda_stream). Only nu_gp_factor synchronises
 *    that stream (once, to report a non-positive-definite covariance).
 *  - Argument errors are detected on the host before any launch and return
 *    NU_ERR_ARG with nothing enqueued.
 *  - One context per host thread; calls that share a context are not
 *    thread-safe.
 */
#ifndef NUANCE_MI355X_H
#define NUANCE_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NU_OK = 0,
  NU_ERR_ARG = 1,         /* invalid argument; nothing was enqueued */
  NU_ERR_NOT_PD = 2,      /* covariance not positive definite (pivot reported) */
  NU_ERR_OOM = 3,         /* device allocation failed */
  NU_ERR_DEVICE = 4,      /* a HIP call or kernel launch failed */
  NU_ERR_UNSUPPORTED = 5  /* valid request the library does not implement */
} nu_status;

/* Arithmetic of the bulk whitening solve of the linear search (the triangular
 * inverse W = L^-1). The Cholesky factor, the trend fit, the cell normal
 * equations and the periodic search are FP64 in every mode.
 *  NU_FP64          all FP64.
 *  NU_FP32_REFINE   the doubling products of the inverse in FP32 on the matrix
 *                   cores, then one FP64 Newton step W += W (I - L W) on the
 *                   block band next to the diagonal, and one step of iterative
 *                   refinement against L of the whitened trend and flux and of
 *                   their back-substitution. Outputs within ~1e-9 of FP64 on
 *                   the test workloads (the bar is 1e-6 on dll).
 *  NU_BF16X3_REFINE the doubling products as split BF16 products on the
 *                   matrix cores: each FP32 operand held as hi + lo BF16
 *                   halves, three products (lo*hi, hi*lo, hi*hi) with FP32
 *                   accumulation; the same FP64 Newton step on a band of 8
 *                   block diagonals (FP32_REFINE: 2) and two steps of the
 *                   refinement of the small solves (FP32_REFINE: one). The
 *                   factor then holds wider band buffers: 2 x 9 x 128 n
 *                   doubles (FP32_REFINE: 2 x 3 x 128 n). Outputs within
 *                   ~1e-8 of FP64 on a TESS-sector curve, but up to a few
 *                   1e-6 on dll for curves whose L^-1 decays slowly (strong,
 *                   long-period variability over white noise). */
typedef enum {
  NU_FP64 = 0,
  NU_FP32_REFINE = 1,
  NU_BF16X3_REFINE = 2
} nu_precision;

/* SHO covariance of Appendix A plus white noise on the diagonal (Section 1.1):
 *   k(tau) = amp^2 exp(-omega tau / 2Q) * { 1 + omega tau                 (Q = 1/2)
 *                                           cosh(f x) + sinh(f x) / f     (Q < 1/2)
 *                                           cos(g x) + sin(g x) / g       (Q > 1/2) }
 * with x = omega tau / 2Q, f = sqrt(1 - 4Q^2), g = sqrt(4Q^2 - 1), and
 *   K[n][m] = k(|t_n - t_m|) + sigma_w^2 delta_nm.
 * Units: omega in radians per time unit of t. Requires amp >= 0, omega > 0,
 * q > 0, sigma_w >= 0, all finite. */
typedef struct {
  double amp;
  double omega;
  double q;
  double sigma_w;
} nu_sho;

/* A GP covariance as a sum of terms: the stellar-variability kernel of
 * Section 3.2 is k = k1 + k2 + k3 + k4 with two SHO terms (at the rotation
 * period and half of it) and two exponential terms.
 *   k(tau) = sum_{s < n_sho} SHO(tau; sho_amp[s], sho_omega[s], sho_q[s])   (as nu_sho)
 *          + sum_{e < n_exp} exp_sigma[e]^2 exp(-tau / exp_ell[e]),
 *   K[n][m] = k(|t_n - t_m|) + sigma_w^2 delta_nm.
 * Requires 0 <= n_sho, n_exp <= 4; amp >= 0, omega > 0, q > 0, sigma >= 0,
 * ell > 0, sigma_w >= 0, all finite. */
typedef struct {
  int32_t n_sho;
  int32_t n_exp;
  double sho_amp[4];
  double sho_omega[4];
  double sho_q[4];
  double exp_sigma[4];
  double exp_ell[4];
  double sigma_w;
} nu_kernel;

/* The stellar-variability kernel of Section 3.2 (the "rotation kernel"),
 * k = k1 + k2 + k3 + k4, as a nu_kernel (host only; no device work):
 *   k1: SHO with Q1 = 1/2 + q0 + dq, omega1 = 4 pi Q1 / (period sqrt(4 Q1^2 - 1)),
 *       power S1 = sigma^2 / ((1 + f) omega1 Q1);
 *   k2: SHO with Q2 = 1/2 + q0, omega2 = 2 omega1, power S2 = f sigma^2 / ((1 + f) omega2 Q2);
 *   k3, k4: sigma_short^2 exp(-tau / ell_short), sigma_long^2 exp(-tau / ell_long);
 * plus sigma_w^2 on the diagonal. An SHO term of power S0 has k(0) = S0 omega Q,
 * so the amplitudes are sqrt(S1 omega1 Q1) and sqrt(S2 omega2 Q2), and
 * k1(0) + k2(0) = sigma^2. Requires every argument finite, sigma >= 0,
 * period > 0, q0 > 0, dq >= 0, f >= 0, sigma_short, sigma_long, sigma_w >= 0,
 * ell_short, ell_long > 0; NU_ERR_ARG otherwise (out_host untouched). */
nu_status nu_rotation_kernel(double sigma, double period, double q0, double dq, double f, double sigma_short,
                             double ell_short, double sigma_long, double ell_long, double sigma_w,
                             nu_kernel* out_host);

typedef struct nu_ctx nu_ctx;
typedef struct nu_factor nu_factor;

/* Context: device, stream, growable workspace, optional kernel timing.
 * stream == NULL means the device's null stream. workspace_limit_bytes (0: no
 * limit) caps the device memory the library allocates on this context: the
 * search workspace, the batch arena (4) and per-call fold grids and records,
 * and the buffers of the factors, graphs and networks made on it, counted
 * while they live (the small launch schedules are not counted). A call that
 * would exceed it allocates nothing more and returns NU_ERR_OOM (the caller
 * may retry with a smaller problem or batch); the batch (4, 4b) plans its
 * waves within it. */
nu_status nu_ctx_create(int device, void* stream, size_t workspace_limit_bytes, nu_ctx** out);
void nu_ctx_destroy(nu_ctx* ctx);
nu_status nu_ctx_set_stream(nu_ctx* ctx, void* stream);
/* Frees the device memory the context keeps between calls: the search
 * workspace and the arena of the batch factors (4). Synchronises the stream. */
nu_status nu_ctx_release_memory(nu_ctx* ctx);
/* Device bytes counted against the workspace limit right now (0 for NULL). */
size_t nu_ctx_device_bytes(const nu_ctx* ctx);
const char* nu_ctx_last_error(const nu_ctx* ctx);
/* Inverse prefetch. prec = NU_FP32_REFINE or NU_BF16X3_REFINE: every later
 * nu_gp_factor / nu_gp_factor_kernel on this context also computes the
 * factor's triangular inverse L^-1 at that precision (the one the linear
 * search of Section 2.2 applies to f and the design columns), starting the
 * parts that read only finished columns of L (the inverse of its top-left
 * half and that half's product with the block below, then the same one level
 * down in the bottom-right half) while the Cholesky factors the rest, on
 * compute_units of the device's compute units (0: three quarters of them;
 * rounded to whole XCDs of 32), which the late, latency-bound steps leave
 * idle. A linear search at prec then finds
 * the inverse made; at another precision it makes its own as without
 * prefetch. Results are bit-identical to those without prefetch. prec = -1
 * (the default) turns it off. NU_ERR_ARG for other precisions or
 * compute_units < 0. */
nu_status nu_ctx_set_inverse_prefetch(nu_ctx* ctx, int prec, int compute_units);

/* Kernel timing with HIP events recorded on the context's stream around
 * every launch of the library's kernels, accumulated per kernel name.
 * work_units is the algorithmic work the library attributes to the
 * launches (flops for the dense kernels, bytes for the fold). Reading the
 * entries synchronises the stream. */
nu_status nu_ctx_enable_timing(nu_ctx* ctx, int enable);
/* Restricts the timing to the launches whose kernel name starts with prefix
 * (NULL or "": every launch), so that the events of a measurement do not
 * delay the other launches. The prefix is copied. */
nu_status nu_ctx_set_timing_filter(nu_ctx* ctx, const char* prefix);
nu_status nu_ctx_timing_reset(nu_ctx* ctx);
int nu_ctx_timing_count(nu_ctx* ctx);
nu_status nu_ctx_timing_entry(nu_ctx* ctx, int index, const char** name_host, int64_t* launches_host,
                              double* total_ms_host, double* work_units_host);

/* (1) GP factor (Appendix A covariance; Eq. 5's ln|Sigma|).
 * t: device, n doubles, strictly increasing. Builds K on the device, factors
 * it as K = L L^T in FP64 (blocked, right-looking), and returns a factor
 * object owning L and the workspace of the later solves (about 2 n^2 + n^2/4
 * doubles of device memory, n rounded up to 128, plus 2 n^2 floats once a
 * reduced-precision search has run on it). Synchronises the stream
 * once. On NU_ERR_NOT_PD, *fail_pivot_host is the first failing pivot and
 * no factor is returned. logdet_host (ln|K|) and fail_pivot_host may be NULL. */
nu_status nu_gp_factor(nu_ctx* ctx, const double* t, int64_t n, const nu_sho* theta, nu_factor** out,
                       double* logdet_host, int64_t* fail_pivot_host);

/* (1b) GP factor of a sum-of-terms covariance (nu_kernel, e.g. the rotation
 * kernel of Section 3.2): as (1), with K built from kernel_host. The factor
 * then serves (2) like any other; nu_gp_factor_into with a nu_sho turns it
 * back into a single-SHO factor. */
nu_status nu_gp_factor_kernel(nu_ctx* ctx, const double* t, int64_t n, const nu_kernel* kernel_host,
                              nu_factor** out, double* logdet_host, int64_t* fail_pivot_host);
/* (1b) Same as (1) into an existing factor of the same n (its device buffers
 * are reused; no allocation). On NU_ERR_NOT_PD the factor's contents are
 * undefined until the next successful call. */
nu_status nu_gp_factor_into(nu_ctx* ctx, nu_factor* factor, const double* t, int64_t n, const nu_sho* theta,
                            double* logdet_host, int64_t* fail_pivot_host);
void nu_factor_destroy(nu_factor* factor);
int64_t nu_factor_n(const nu_factor* factor);

/* (2) Linear search (Section 2.2, Eqs. 5-6).
 * f: device, n doubles (n = nu_factor_n). A: device, n x m1 column-major
 * (column c at A + c*n), 0 <= m1 <= 7; may be NULL when m1 == 0.
 * lattice: device, n int64, lattice[0] == 0 and strictly increasing: sample
 * s sits at epoch slot lattice[s] (time t_first + lattice[s] * dt).
 * n_epochs == lattice[n-1] + 1 epoch slots are searched. The lattice is
 * checked on the device (no synchronisation): one that breaks these rules
 * leaves every cell invalid and ln L_0 = NaN in null_out. dur_samples_host:
 * host, n_d box lengths in slots, 1 <= value <= 1024, 1 <= n_d <= 16.
 * The box of cell (j, i) is -1 on samples whose slot lies in
 * [i - floor(d_j/2), i - floor(d_j/2) + d_j) and 0 elsewhere.
 * Outputs (device, row-major [n_d][n_epochs]): depth (GLS depth of the box),
 * var (its variance, the MM element of (X^T K^-1 X)^-1), dll (log-likelihood
 * gain over the trend-only fit, 0.5 depth^2 / var), valid (1/0). Invalid
 * cells (empty box, or box collinear with the trend): depth = 0,
 * var = +inf, dll = 0, valid = 0.
 * null_out: device, 3 doubles or NULL: ln L_0 (Eq. 5 of the trend-only
 * fit), chi2_0 and ln|K|.
 * prec selects the arithmetic of the bulk whitening solve. */
nu_status nu_linear_search(nu_ctx* ctx, nu_factor* factor, const double* f, const double* A, int m1,
                           const int64_t* lattice, int64_t n_epochs, const int32_t* dur_samples_host, int n_d,
                           nu_precision prec, double* depth, double* var, double* dll, uint8_t* valid,
                           double* null_out);

/* (2b) Linear search of (2) without a dense factor, for a sum-of-terms
 * covariance (Appendix A's SHO, Section 3.2's rotation kernel): the O(N J^2)
 * quasiseparable route of the GP package the paper uses (Section 3.2,
 * Appendix A), as the Kalman filter of the equivalent state-space model
 * (J = 2 n_sho + n_exp states; at least one term). The filter's innovations
 * are the Cholesky factorisation of K sample by sample, so every output is
 * the one (2) gives with the factor of (1b) of the same kernel, up to
 * rounding, in FP64.
 * t: device, n doubles, non-decreasing (the sample times of K). f, A,
 * lattice, n_epochs, dur_samples_host, the outputs and null_out as in (2).
 * shapes_host: NULL for boxes, or template shapes as in (2c).
 * The kernel is passed by value to the device (no upload, no allocation
 * beyond the context's workspace: about n (3 YCOLS + 8 J + J^2) doubles plus
 * one double per cell).
 * fail_index_host: host or NULL. Non-NULL: the call synchronises the stream
 * once and, if an innovation variance is not positive (K not positive
 * definite in floating point), stores the first failing sample there and
 * returns NU_ERR_NOT_PD (else stores -1). NULL: no synchronisation; a failure
 * then shows as ln L_0 = NaN and ln|K| = NaN in null_out and every cell
 * invalid. */
nu_status nu_linear_search_ss(nu_ctx* ctx, const double* t, int64_t n, const nu_kernel* kernel_host, const double* f,
                              const double* A, int m1, const int64_t* lattice, int64_t n_epochs,
                              const int32_t* dur_samples_host, int n_d, const double* shapes_host, double* depth,
                              double* var, double* dll, uint8_t* valid, double* null_out, int64_t* fail_index_host);

/* (2c) Linear search with a non-box base model in the last column of the
 * design (Section 4.4, prospects: limb-darkened transits, exocomets, flares):
 * as (2), with the box of duration j replaced by its shape. shapes_host:
 * host, the n_d shapes concatenated in the caller's duration order, shape j
 * holding dur_samples_host[j] finite values (one per lattice slot of the
 * window), at most 2048 values together; copied before the call returns.
 * The last column of cell (j, i) is -shape_j[l - a] on samples whose slot l
 * lies in [a, a + d_j), a = i - floor(d_j/2), and 0 elsewhere; depth is the
 * coefficient of the shape (the unit shape gives (2)'s outputs). The same
 * shapes_host argument of (2b) (NULL there means boxes) gives the
 * state-space version of this search. */
nu_status nu_linear_search_template(nu_ctx* ctx, nu_factor* factor, const double* f, const double* A, int m1,
                                    const int64_t* lattice, int64_t n_epochs, const int32_t* dur_samples_host,
                                    int n_d, const double* shapes_host, nu_precision prec, double* depth,
                                    double* var, double* dll, uint8_t* valid, double* null_out);

/* (3) Periodic search (Sections 2.3-2.4, Eqs. 8, 9, B4).
 * depth/var/dll/valid: device, [n_d][n_epochs] as produced by (2).
 * periods: device, n_p doubles in the time unit of dt (dt > 0).
 * 1 <= n_epochs <= 2^27 (the global extent for (3c)).
 * For period P, p = P / dt; phases m = 0 .. ceil(p) - 1 (slot units from the
 * first sample); events k >= 0 at slot position m + k p, linearly
 * interpolated between slots floor and floor+1 (a single slot when k p is
 * an integer); an event needs its slot(s) inside the grid and valid.
 * Events are combined per (m, j) with Eq. B4's depth and sigma^2, and
 *   lnP = sum dll_k - 1/2 sum [ s (ln var_k - ln(sigma^2 + var_k))
 *                              + (depth_k - depth)^2 / (var_k + sigma^2) ]
 * with s = log_term_sign (+1: the sign printed in Eq. 8; -1: the sign of the
 * derivation in Appendix B). The first maximum over (m outer, j inner)
 * gives per period: q_snr = depth/sigma, best_phase m, best_dur j,
 * best_depth, best_sigma, best_lnp. A period without any event has
 * q_snr = 0, best_phase = best_dur = -1, best_lnp = -inf.
 * A period shorter than one cadence (p < 1) or not finite (NaN, +-inf) has
 * no event: the phase grid steps by one cadence, and several transits would
 * fall into one lattice step.
 * best_period_index: device, 1 int64 or NULL: the first period of largest
 * q_snr (period 0 when no period has an event, all q_snr being 0).
 * n_p >= 1 is required. */
nu_status nu_periodic_search(nu_ctx* ctx, const double* depth, const double* var, const double* dll,
                             const uint8_t* valid, int n_d, int64_t n_epochs, double dt, const double* periods,
                             int64_t n_p, int log_term_sign, double* q_snr, int64_t* best_phase, int32_t* best_dur,
                             double* best_depth, double* best_sigma, double* best_lnp, int64_t* best_period_index);

/* (3d) The periodic search (3) for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same arguments, kernels and outputs (bitwise equal to
 * (3)), with its one scratch buffer, the packed copy of the grid (24 n_d
 * (n_epochs + 64) bytes), in a fixed device array of NU_PERIODIC_SCRATCH_BYTES
 * per device instead of the context's workspace. The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine) and does not
 * synchronise. A grid needing more than the array returns NU_ERR_ARG before
 * any launch (e.g. 10 durations x 139 000 slots fit). Every call on one device
 * shares that device's array: calls that overlap on a device (other streams,
 * other contexts, other host threads) race, and must be ordered by the caller.
 * The library's kernel timing does not cover this call. */
#define NU_PERIODIC_SCRATCH_BYTES ((size_t)32 << 20)
nu_status nu_periodic_search_noalloc(nu_ctx* ctx, const double* depth, const double* var, const double* dll,
                                     const uint8_t* valid, int n_d, int64_t n_epochs, double dt,
                                     const double* periods, int64_t n_p, int log_term_sign, double* q_snr,
                                     int64_t* best_phase, int32_t* best_dur, double* best_depth, double* best_sigma,
                                     double* best_lnp, int64_t* best_period_index);

/* (3c) Periodic search over segments of one light curve, each with its own
 * linear search (Sections 3.3 and 4.1: sectors observed apart, one GP and one
 * linear search per sector, combined in the fold).
 * Segment s covers the global lattice slots [seg_off_host[s],
 * seg_off_host[s] + seg_len_host[s]) (host arrays, n_seg in 1 .. 32; ascending,
 * at least 64 slots apart; the global slot 0 is the phase origin). Its grid,
 * as produced by (2) for that segment, is the [n_d][seg_len_host[s]] block of
 * depth/var/dll/valid (device) that follows the blocks of segments 0 .. s-1,
 * i.e. the concatenated outputs of (2), or of (4) with one curve per segment.
 * The result equals (3) on one global grid with every slot of no segment an
 * invalid cell; phases (best_phase) are global slots. The fold skips the gaps,
 * so its work is that of the segments. Outputs as in (3). */
nu_status nu_periodic_search_segments(nu_ctx* ctx, const double* depth, const double* var, const double* dll,
                                      const uint8_t* valid, int n_d, int n_seg, const int64_t* seg_len_host,
                                      const int64_t* seg_off_host, double dt, const double* periods, int64_t n_p,
                                      int log_term_sign, double* q_snr, int64_t* best_phase, int32_t* best_dur,
                                      double* best_depth, double* best_sigma, double* best_lnp,
                                      int64_t* best_period_index);

/* (3b) Search for further candidates (Section 3.3, the search of TOI-540): mask
 * a found candidate's transits in the linear-search outputs, in place, so
 * that the next periodic search (3) on them skips those epochs; the linear
 * search is not repeated.
 * depth/var/dll/valid: device, [n_d][n_epochs] as produced by (2), modified
 * in place. period: the candidate's period (time unit of dt, p = period / dt
 * >= 1); phase: its best phase m in slots (0 <= m < n_epochs); half_width:
 * its duration in slots, n_j (1 .. 1024): windows of width 2 D.
 * Slot i is masked, for every duration, when |(i - m) - k p| < half_width for
 * some integer k (k p rounded once to FP64); masked cells take the invalid
 * encoding of (2): depth = 0, var = +inf, dll = 0, valid = 0.
 * Argument errors return NU_ERR_ARG before any launch; no synchronisation. */
nu_status nu_mask_transit(nu_ctx* ctx, double* depth, double* var, double* dll, uint8_t* valid, int n_d,
                          int64_t n_epochs, double dt, double period, int64_t phase, int half_width);

/* (4) Batch search of light curves of uneven length: (1), (2) and (3) for
 * every curve of the batch (Sections 2.2-2.4 per curve).
 * Curve c owns samples [sample_off_host[c], sample_off_host[c+1]) of t, f and
 * lattice (device; its lattice starts at 0 as in (2)), trend columns at
 * A + m1 * sample_off_host[c] (column-major n_c x m1, as in (2)), and epoch
 * slots [epoch_off_host[c], epoch_off_host[c+1]); both offset arrays are host,
 * n_curves + 1 entries, starting at 0. theta_host and dt_host: host, one per
 * curve. Durations, periods (device, n_p), precision and log_term_sign are
 * shared by all curves.
 * Outputs (device): depth/var/dll/valid of curve c at n_d * epoch_off[c],
 * laid out [n_d][n_epochs_c] as in (2); null_out (3 per curve, may be NULL);
 * the per-period arrays of (3) at c * n_p; best_period_index (one per curve,
 * may be NULL). logdet_host and fail_pivot_host (host, one per curve, may be
 * NULL): ln|K| and -1 or the failing pivot.
 * The curves are processed longest first in waves whose factors fit in
 * memory_budget_bytes of device memory (0: 90 % of the free memory counting
 * the arena the context already holds as free). Every stage of a wave is one
 * launch for all its curves: the covariance build, each Cholesky step's
 * diagonal blocks and grouped GEMMs, each level of the inverse, each pass of
 * the linear search, the fold over (period, curve) and the best periods, so
 * a call issues a number of launches set by the stages and the waves, not by
 * the curves. The factors and each curve's search workspace live in a device
 * arena of the size of the largest wave, which the context keeps for later
 * calls (released by nu_ctx_release_memory or nu_ctx_destroy); a later call
 * keeps that arena when a plan within it needs no more waves than the budget
 * allows, and grows it otherwise. The call
 * synchronises the stream once, before it returns. A curve whose covariance
 * is not positive definite gets invalid cells, no event at any period and
 * best_period_index -1; the call finishes the other curves and returns
 * NU_ERR_NOT_PD. A single curve larger than the budget gives NU_ERR_OOM
 * before any work. Each curve's outputs equal those of (1)-(3) on that curve
 * alone, bit for bit. */
nu_status nu_search_batch(nu_ctx* ctx, int n_curves, const int64_t* sample_off_host, const int64_t* epoch_off_host,
                          const double* t, const double* f, const double* A, int m1, const int64_t* lattice,
                          const nu_sho* theta_host, const double* dt_host, const int32_t* dur_samples_host, int n_d,
                          const double* periods, int64_t n_p, nu_precision prec, int log_term_sign,
                          size_t memory_budget_bytes, double* depth, double* var, double* dll, uint8_t* valid,
                          double* null_out, double* q_snr, int64_t* best_phase, int32_t* best_dur,
                          double* best_depth, double* best_sigma, double* best_lnp, int64_t* best_period_index,
                          double* logdet_host, int64_t* fail_pivot_host);

/* (4b) Captured graph of the batch search (4): every stage of every wave of
 * (4), recorded once into a HIP graph bound to these device buffers, with its
 * own device arena (allocated here, before the capture; memory_budget_bytes
 * as in (4), 0: 90 % of the free memory). Each nu_batch_graph_launch replays
 * the whole batch on the context's stream in one graph launch and reads the
 * current contents of t, f, A, lattice, periods and theta_dev (device,
 * n_curves nu_sho: the caller may rewrite them between launches, in stream
 * order). Nothing synchronises: status_dev (device, n_curves int64) receives
 * -1 or the failing pivot of each curve, logdet_dev (device, n_curves, may be
 * NULL) its ln|K|. Other arguments and outputs as in (4); the outputs of a
 * launch equal those of (4) on the same inputs, bit for bit. Launches of one
 * graph must not overlap. theta_dev is not validated: it must satisfy (1)'s
 * bounds. */
typedef struct nu_batch_graph nu_batch_graph;
nu_status nu_batch_graph_create(nu_ctx* ctx, int n_curves, const int64_t* sample_off_host,
                                const int64_t* epoch_off_host, const double* t, const double* f, const double* A,
                                int m1, const int64_t* lattice, const nu_sho* theta_dev, const double* dt_host,
                                const int32_t* dur_samples_host, int n_d, const double* periods, int64_t n_p,
                                nu_precision prec, int log_term_sign, size_t memory_budget_bytes, double* depth,
                                double* var, double* dll, uint8_t* valid, double* null_out, double* q_snr,
                                int64_t* best_phase, int32_t* best_dur, double* best_depth, double* best_sigma,
                                double* best_lnp, int64_t* best_period_index, int64_t* status_dev,
                                double* logdet_dev, nu_batch_graph** out);
nu_status nu_batch_graph_launch(nu_ctx* ctx, nu_batch_graph* graph);
void nu_batch_graph_destroy(nu_batch_graph* graph);

/* (5) Captured graph of the whole search of one light curve: K build,
 * Cholesky, inverse, linear search, periodic search and best period, as
 * (1)-(3) with the same arguments, recorded once into a HIP graph bound to
 * these device buffers. Each nu_graph_launch replays it on the context's
 * stream and reads the current contents of t, f, A, lattice, periods and
 * theta_dev (device, one nu_sho: the caller may rewrite it between launches,
 * in stream order). No synchronisation: status_dev (device, one int64)
 * receives -1 or the failing pivot of that launch; after a failing pivot the
 * outputs of that launch are meaningless. The graph owns its factor and
 * workspace (created here, before the capture); launches of one graph must
 * not overlap. theta_dev is not validated: it must satisfy (1)'s bounds. */
typedef struct nu_graph nu_graph;
nu_status nu_graph_create(nu_ctx* ctx, const double* t, int64_t n, const nu_sho* theta_dev, const double* f,
                          const double* A, int m1, const int64_t* lattice, int64_t n_epochs,
                          const int32_t* dur_samples_host, int n_d, nu_precision prec, double dt,
                          const double* periods, int64_t n_p, int log_term_sign, double* depth, double* var,
                          double* dll, uint8_t* valid, double* null_out, double* q_snr, int64_t* best_phase,
                          int32_t* best_dur, double* best_depth, double* best_sigma, double* best_lnp,
                          int64_t* best_period_index, int64_t* status_dev, nu_graph** out);
nu_status nu_graph_launch(nu_ctx* ctx, nu_graph* graph);
void nu_graph_destroy(nu_graph* graph);

/* (6) Tile policy of the dense launches. Launch classes: 0 Cholesky panel,
 * 1 panel update, 2 trailing update, 3 FP64 inverse levels, 4 FP32 inverse
 * levels, 5 band Newton step, 6 split-BF16 inverse levels. A launch of a
 * class takes 64 x 64 output tiles when it has fewer 128 x 128 tiles than the
 * class threshold (default 512),
 * else 128 x 128. The choice changes speed only: every output element sums
 * the same products in the same order either way, so results are bitwise
 * identical. nu_ctx_autotune times the factorisation and inverse of a
 * synthetic covariance of size n (128 <= n <= 131072) under six thresholds
 * per class, keeps the fastest per class in the context, and restores the
 * caller's timing state; schedules built afterwards (new factors, batches,
 * graphs) use it. It synchronises the stream and allocates about 2.5 n^2
 * doubles while it runs. */
nu_status nu_ctx_autotune(nu_ctx* ctx, int64_t n, nu_precision prec);
nu_status nu_ctx_get_tuning(const nu_ctx* ctx, int launch_class, int* small_below_host);
nu_status nu_ctx_set_tuning(nu_ctx* ctx, int launch_class, int small_below);

/* ---------------------------------------------------------------------------
 * (7) The hyperparameter fit the search needs first, and its learned warm
 * start. The paper fits the GP hyperparameters of each curve by maximum
 * likelihood with the trend solved linearly (Section 3.2); the likelihood is
 * Eq. 5 of the trend-only model. Here the fit runs in the coordinates
 * x = (ln amp, ln P_rot, ln Q, ln sigma_w), with omega = 4 pi Q / (P_rot
 * sqrt(4Q^2 - 1)) for Q > 1/2 (2 pi / P_rot otherwise). The warm start is a 1D
 * CNN trained on curves drawn from the GP itself.
 * --------------------------------------------------------------------------- */

/* (7a) Training curves from the SHO process plus white noise on a unit
 * baseline: f_n = 1 + g(t_n) + sigma_w e_n, g by the exact discretisation of
 * the oscillator's state-space model, random numbers from Philox-4x32-10
 * (Salmon et al. 2011) keyed by seed, counter (sample index, curve index low,
 * high word, stream: 0 process noise, 1 white noise, 2 initial state, 3
 * hyperparameters), uniforms (k + 1/2) 2^-52 from the top 26 bits of two words,
 * Box-Muller normals. Curve c has index curve_base + c. t: device, n >= 2,
 * strictly increasing, shared by all curves. theta: device, n_curves, or NULL
 * to draw each curve's hyperparameters from the training prior (log-uniform:
 * amp [0.005, 0.03], P_rot [0.3, 2] time units, Q [1, 100], sigma_w [3e-4,
 * 3e-3]). Outputs (device, each may be NULL): flux [n_curves][n]; input
 * [n_curves][n_bins] (n_bins <= 512): 100 (m_b / median - 1) of the bin means
 * m_b over n_bins equal time bins (bin floor((t - t_0)/(t_{n-1} - t_0) n_bins),
 * the last sample in the last bin; median over non-empty bins; empty bins 0);
 * target [n_curves][4]: the standardised logs of (amp, P_rot, Q, sigma_w)
 * under the prior; theta_out [n_curves]. */
nu_status nu_gp_sample(nu_ctx* ctx, const double* t, int64_t n, int n_curves, const nu_sho* theta, uint64_t seed,
                       uint64_t curve_base, int n_bins, double* flux, float* input, float* target,
                       nu_sho* theta_out);

/* (7b) -ln L_0 (Eq. 5 of the trend-only model, the trend profiled) for
 * n_curves x n_eval (curve, theta) pairs, by the Kalman filter of the SHO
 * state-space model: its innovations whiten [A | f] and ln|K| is the sum of
 * their log variances (exact, O(N) per pair). sample_off: DEVICE, n_curves + 1
 * offsets; t, f: device; A: device, curve c's n_c x m1 column-major block at
 * A + m1 * sample_off[c] (as in (4)); theta: device [n_curves][n_eval]; nll:
 * device [n_curves][n_eval] (+inf when the trend Gram is singular). */
nu_status nu_gp_nll(nu_ctx* ctx, int n_curves, const int64_t* sample_off, const double* t, const double* f,
                    const double* A, int m1, const nu_sho* theta, int n_eval, double* nll);

/* (7c) The plain start (fallback of the learned one): P_rot = the first
 * maximum of the Lomb-Scargle power of f - mean(f) over prot_grid (device,
 * n_grid trial periods), amp = std(f), Q = 5, sigma_w = rms of the second
 * differences / sqrt(6). sample_off: DEVICE, n_curves + 1. x0: device
 * [n_curves][4] in fit coordinates. */
nu_status nu_plain_init(nu_ctx* ctx, int n_curves, const int64_t* sample_off, const double* t, const double* f,
                        const double* prot_grid, int n_grid, double* x0);

/* (7d) Maximum-likelihood fit by BFGS of all curves in lockstep: gradients by
 * central differences (step 1e-4 in x), Armijo backtracking, coordinates
 * clamped to wide bounds; one likelihood launch (7b) per gradient or line-
 * search trial for all curves. sample_off_host: HOST, n_curves + 1. x0_host,
 * x_host: host [n_curves][4]. Stops per curve when every |gradient| <= gtol,
 * the step no longer decreases the likelihood, or after max_iter iterations.
 * nll_host, n_eval_host (likelihood evaluations used), iters_host: host, may
 * be NULL. Synchronises the stream at every step. */
nu_status nu_fit_hyper(nu_ctx* ctx, int n_curves, const int64_t* sample_off_host, const double* t, const double* f,
                       const double* A, int m1, const double* x0_host, int max_iter, double gtol, double* x_host,
                       double* nll_host, int32_t* n_eval_host, int32_t* iters_host);

/* (7e) The CNN: input 512 values; four convolutions of width 7, stride 2,
 * zero padding 3, 64 channels, ReLU; global average pool; linear head to 4
 * outputs (the standardised logs of amp, P_rot, Q, sigma_w). Parameters flat,
 * FP32: (W1 [64][1][7], b1, W2..W4 [64][64][7], b2..b4, Wh [4][64], bh),
 * nu_cnn_param_count() values. half_precision != 0: the convolutions run on
 * the matrix cores in FP16 (weights and activations rounded to FP16, FP32
 * accumulation, FP32 master weights); 0: FP32 products. Adam (beta 0.9,
 * 0.999, eps 1e-8) on the mean squared error. All arrays device except
 * params_host; input [batch][512], target and out [batch][4], grad
 * [param_count], loss one float; x_log (may be NULL) [batch][4] receives the
 * outputs in fit coordinates. */
typedef struct nu_cnn nu_cnn;
int64_t nu_cnn_param_count(void);
nu_status nu_cnn_create(nu_ctx* ctx, int half_precision, int max_batch, nu_cnn** out);
void nu_cnn_destroy(nu_cnn* model);
nu_status nu_cnn_set_params(nu_ctx* ctx, nu_cnn* model, const float* params_host);
/* He-uniform weights (U(-sqrt(6/fan_in), sqrt(6/fan_in)), uniforms from
 * Philox with counter = parameter index, stream 4), zero biases, fresh Adam. */
nu_status nu_cnn_init(nu_ctx* ctx, nu_cnn* model, uint64_t seed);
nu_status nu_cnn_get_params(nu_ctx* ctx, nu_cnn* model, float* params_host);
nu_status nu_cnn_forward(nu_ctx* ctx, nu_cnn* model, const float* input, int batch, float* out, double* x_log);
/* (7f) The learned warm start of the fit (7d): the network's amp, P_rot and Q
 * with sigma_w from the plain start x_plain (device [batch][4], from (7c)): the
 * binned input averages the white noise away, the second differences of the
 * full curve measure it. x_out: device [batch][4] fit coordinates. */
nu_status nu_warm_start(nu_ctx* ctx, nu_cnn* model, const float* input, int batch, const double* x_plain,
                        double* x_out);
nu_status nu_cnn_gradient(nu_ctx* ctx, nu_cnn* model, const float* input, const float* target, int batch,
                          float* grad, float* loss);
nu_status nu_cnn_train_step(nu_ctx* ctx, nu_cnn* model, const float* input, const float* target, int batch, float lr,
                            float* loss);

#ifdef __cplusplus
}
#endif

#endif /* NUANCE_MI355X_H */
