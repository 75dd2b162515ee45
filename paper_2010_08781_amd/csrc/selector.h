// selector.h -- the exchange selector's network, shared by the training
// kernels and the superstep engine (inference on the device).
#pragma once

#include "common.h"

namespace ipg {

constexpr int kSelD = 4, kSelH = 16, kSelK = 3;
// Outputs: predicted log2 microseconds of the superstep's exchange variants.
enum : int { kSelPushList = 0, kSelPushDense = 1, kSelPull = 2 };
constexpr int kSelParams = kSelH * kSelD + kSelH + kSelH * kSelH + kSelH + kSelK * kSelH + kSelK;

// Inputs of the network for one superstep.
__host__ __device__ inline void sel_features(uint64_t frontier, uint64_t frontier_deg, uint32_t superstep, uint64_t e,
                                             double* x) {
  x[0] = log2(1.0 + static_cast<double>(frontier)) / 32.0;
  x[1] = log2(1.0 + static_cast<double>(frontier_deg)) / 32.0;
  x[2] = static_cast<double>(superstep < 128u ? superstep : 128u) / 64.0;
  x[3] = log2(1.0 + static_cast<double>(e)) / 32.0;
}

__host__ __device__ inline void sel_forward1(const double* p, const double* x, double* h1, double* h2, double* y) {
  const double* W1 = p;
  const double* b1 = W1 + kSelH * kSelD;
  const double* W2 = b1 + kSelH;
  const double* b2 = W2 + kSelH * kSelH;
  const double* W3 = b2 + kSelH;
  const double* b3 = W3 + kSelK * kSelH;
  for (int j = 0; j < kSelH; ++j) {
    double z = b1[j];
    for (int d = 0; d < kSelD; ++d) z += W1[j * kSelD + d] * x[d];
    h1[j] = tanh(z);
  }
  for (int j = 0; j < kSelH; ++j) {
    double z = b2[j];
    for (int l = 0; l < kSelH; ++l) z += W2[j * kSelH + l] * h1[l];
    h2[j] = tanh(z);
  }
  for (int k = 0; k < kSelK; ++k) {
    double z = b3[k];
    for (int j = 0; j < kSelH; ++j) z += W3[k * kSelH + j] * h2[j];
    y[k] = z;
  }
}

// The variant of the smallest prediction among those available: a push that
// visits the frontier as a list (only when `list_ok`: the previous superstep
// pushed and left a complete list), a push that sweeps every vertex's
// mailbox, a pull.  Returns the predicted log2 time of the push minus that
// of the pull; *use_list tells which push.
__host__ __device__ inline double sel_pick(const double* y, bool list_ok, int* mode, bool* use_list) {
  const bool list = list_ok && y[kSelPushList] <= y[kSelPushDense];
  const double push = list ? y[kSelPushList] : y[kSelPushDense];
  *mode = y[kSelPull] < push ? IPG_MODE_PULL : IPG_MODE_PUSH;
  *use_list = list;
  return push - y[kSelPull];
}

__host__ __device__ inline double sel_predict_mode(const double* p, uint64_t frontier, uint64_t frontier_deg, uint32_t superstep,
                                   uint64_t e, bool list_ok, int* mode, bool* use_list) {
  double x[kSelD], h1[kSelH], h2[kSelH], y[kSelK];
  sel_features(frontier, frontier_deg, superstep, e, x);
  sel_forward1(p, x, h1, h2, y);
  return sel_pick(y, list_ok, mode, use_list);
}

// The same prediction by a whole wavefront (every lane calls it and gets the
// result): lane j < 16 computes hidden unit j of each layer, reading the
// previous layer from the other lanes, and lanes 0 .. kSelK-1 the outputs.
// Every unit is summed in the order of sel_forward1, so the result is the
// same; the latency is that of one unit per layer instead of all of them.
__device__ inline double sel_predict_mode_wave(const double* p, uint64_t frontier, uint64_t frontier_deg,
                                               uint32_t superstep, uint64_t e, bool list_ok, int* mode,
                                               bool* use_list) {
  const double* W1 = p;
  const double* b1 = W1 + kSelH * kSelD;
  const double* W2 = b1 + kSelH;
  const double* b2 = W2 + kSelH * kSelH;
  const double* W3 = b2 + kSelH;
  const double* b3 = W3 + kSelK * kSelH;
  double x[kSelD];
  sel_features(frontier, frontier_deg, superstep, e, x);
  const int lane = static_cast<int>(lane_id());
  const int j = lane < kSelH ? lane : 0;
  double z = b1[j];
  for (int d = 0; d < kSelD; ++d) z += W1[j * kSelD + d] * x[d];
  const double h1 = tanh(z);
  double z2 = b2[j];
  for (int l = 0; l < kSelH; ++l) z2 += W2[j * kSelH + l] * __shfl(h1, l);
  const double h2 = tanh(z2);
  const int k = lane < kSelK ? lane : 0;
  double y = b3[k];
  for (int l = 0; l < kSelH; ++l) y += W3[k * kSelH + l] * __shfl(h2, l);
  double ys[kSelK];
  for (int q = 0; q < kSelK; ++q) ys[q] = __shfl(y, q);
  return sel_pick(ys, list_ok, mode, use_list);
}

}  // namespace ipg
