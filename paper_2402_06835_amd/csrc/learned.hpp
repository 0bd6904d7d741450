// Shared declarations of the learned warm start (sampler, likelihood, CNN).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "nuance_mi355x.h"

namespace nu {

// Philox streams of the sampler (fourth counter word)
constexpr uint32_t STREAM_PROCESS = 0, STREAM_WHITE = 1, STREAM_INITIAL = 2, STREAM_THETA = 3;

// training prior, log-uniform: amp, P_rot (time unit of t), Q, sigma_w
__host__ __device__ inline double prior_lo(int i) {
  return i == 0 ? 0.005 : (i == 1 ? 0.3 : (i == 2 ? 1.0 : 3e-4));
}
__host__ __device__ inline double prior_hi(int i) {
  return i == 0 ? 0.03 : (i == 1 ? 2.0 : (i == 2 ? 100.0 : 3e-3));
}

// network shape: 4 stride-2 convolutions of width 7, 64 channels, ReLU,
// global average pool, linear head; input 512 bins
constexpr int CNN_IN = 512, CNN_CH = 64, CNN_KW = 7, CNN_LAYERS = 4, CNN_OUT = 4;
constexpr int CNN_WCHUNK = 8;  // samples per partial of the weight gradient

// flat parameter layout: (W1, b1, ..., W4, b4, Wh, bh), W of layer l is [64][c_in * 7]
__host__ __device__ inline int64_t cnn_w_offset(int l) {
  return l == 0 ? 0 : (int64_t)CNN_CH * CNN_KW + CNN_CH + (int64_t)(l - 1) * (CNN_CH * CNN_CH * CNN_KW + CNN_CH);
}
__host__ __device__ inline int64_t cnn_b_offset(int l) {
  return cnn_w_offset(l) + (int64_t)CNN_CH * (l == 0 ? 1 : CNN_CH) * CNN_KW;
}
__host__ __device__ inline int64_t cnn_head_w() { return cnn_b_offset(CNN_LAYERS - 1) + CNN_CH; }
__host__ __device__ inline int64_t cnn_head_b() { return cnn_head_w() + (int64_t)CNN_OUT * CNN_CH; }
__host__ __device__ inline int64_t cnn_param_count() { return cnn_head_b() + CNN_OUT; }

// activations and scratch of one batch
struct CnnBuffers {
  float* y[CNN_LAYERS];   // post-ReLU outputs, [batch][64][512 >> (l+1)]
  float* dz[CNN_LAYERS];  // gradients of the pre-activations, same shapes
  float* h;               // pooled features [batch][64]
  float* out;             // outputs [batch][4]
  float* dO;              // output gradients [batch][4]
  float* sq;              // per-sample squared error [batch]
  float* part;            // weight-gradient partials [chunks][64][448]
};

hipError_t launch_gp_sample(hipStream_t s, const double* t, int64_t n, int n_curves, const nu_sho* theta_in,
                            uint64_t seed, uint64_t curve_base, int n_bins, double* flux, double* bin_mean,
                            nu_sho* theta_out, float* target, float* input);
hipError_t launch_kalman_nll(hipStream_t s, const double* t, const double* f, const double* A, int m1,
                             const int64_t* off, int n_curves, const nu_sho* theta, int n_eval, double* nll);
hipError_t launch_plain_init(hipStream_t s, const double* t, const double* f, const int64_t* off, int n_curves,
                             const double* prot, int n_grid, double* mom, double* power, double* x0);
hipError_t launch_cnn_forward(hipStream_t s, const CnnBuffers& B, const float* P, const _Float16* P16, bool half,
                              const float* input, int batch, float* out);
hipError_t launch_cnn_backward(hipStream_t s, const CnnBuffers& B, const float* P, const _Float16* P16, bool half,
                               const float* input, const float* target, int batch, float* grad, float* loss);
hipError_t launch_adam(hipStream_t s, float* p, _Float16* p16, const float* g, float* m, float* v, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2);
hipError_t launch_to_half(hipStream_t s, const float* p, _Float16* p16, int64_t n);
hipError_t launch_cnn_init(hipStream_t s, float* p, int64_t n, uint64_t seed);
hipError_t launch_outputs_to_log(hipStream_t s, const float* y, int batch, const double* x_plain, double* x);

}  // namespace nu
