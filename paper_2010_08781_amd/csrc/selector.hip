// selector.hip -- the learned per-superstep exchange selector.
//
// The paper fixes push or pull per program at compile time and leaves the
// choice to the user's experiments (Section 4.3.2); Ligra switches at run
// time on a user threshold.  Here a small MLP predicts, from the state of a
// superstep, the log2 of the time a push and a pull exchange would take, and
// the engine runs the cheaper one.  The exchange never changes results.
//
// Network: 4 inputs -> 16 tanh -> 16 tanh -> 2 linear outputs, FP64,
// parameters packed as W1[16][4], b1[16], W2[16][16], b2[16], W3[2][16],
// b3[2].  Inputs (sel_features): log2(1+|F|)/32, log2(1+sum outdeg F)/32,
// min(superstep, 128)/64, log2(1+E)/32.  Loss: half the mean squared error
// of the predicted log2-times.  Training is full-batch gradient descent by a
// single workgroup in a fixed reduction order (bitwise reproducible).
#include <mutex>

#include "common.h"
#include "engine.h"
#include "selector.h"

namespace ipg {

__global__ void sel_forward_kernel(const double* p, const double* X, uint32_t n, double* Y) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double h1[kSelH], h2[kSelH];
  sel_forward1(p, X + (size_t)i * kSelD, h1, h2, Y + (size_t)i * kSelK);
}

// Scratch of one batch gradient: h1, h2, dz2, dz1 [n][H] and dY [n][K].
static size_t sel_scratch_doubles(uint32_t n) { return (size_t)n * (4 * kSelH + kSelK); }

// Full-batch gradient, one workgroup, every reduction over samples in
// ascending sample order.
__device__ void sel_grad_block(const double* p, const double* X, const double* T, uint32_t n, double* g, double* scr) {
  const double* W2 = p + kSelH * kSelD + kSelH;
  const double* W3 = W2 + kSelH * kSelH + kSelH;
  double* h1 = scr;
  double* h2 = h1 + (size_t)n * kSelH;
  double* dz2 = h2 + (size_t)n * kSelH;
  double* dz1 = dz2 + (size_t)n * kSelH;
  double* dY = dz1 + (size_t)n * kSelH;
  double* gW1 = g;
  double* gb1 = gW1 + kSelH * kSelD;
  double* gW2 = gb1 + kSelH;
  double* gb2 = gW2 + kSelH * kSelH;
  double* gW3 = gb2 + kSelH;
  double* gb3 = gW3 + kSelK * kSelH;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const double inv_n = 1.0 / static_cast<double>(n);
  for (uint32_t i = tid; i < n; i += nt) {
    double y[kSelK];
    sel_forward1(p, X + (size_t)i * kSelD, h1 + (size_t)i * kSelH, h2 + (size_t)i * kSelH, y);
    for (int k = 0; k < kSelK; ++k) dY[(size_t)i * kSelK + k] = (y[k] - T[(size_t)i * kSelK + k]) * inv_n;
  }
  __syncthreads();
  // output layer, and the error of the second hidden layer
  for (uint32_t q = tid; q < kSelK * kSelH + kSelK; q += nt) {
    double s = 0.0;
    if (q < kSelK * kSelH) {
      const uint32_t k = q / kSelH, j = q % kSelH;
      for (uint32_t i = 0; i < n; ++i) s += dY[(size_t)i * kSelK + k] * h2[(size_t)i * kSelH + j];
      gW3[q] = s;
    } else {
      const uint32_t k = q - kSelK * kSelH;
      for (uint32_t i = 0; i < n; ++i) s += dY[(size_t)i * kSelK + k];
      gb3[k] = s;
    }
  }
  for (uint64_t q = tid; q < (uint64_t)n * kSelH; q += nt) {
    const uint64_t i = q / kSelH;
    const uint32_t j = static_cast<uint32_t>(q % kSelH);
    double s = 0.0;
    for (int k = 0; k < kSelK; ++k) s += dY[i * kSelK + k] * W3[k * kSelH + j];
    const double h = h2[q];
    dz2[q] = s * (1.0 - h * h);
  }
  __syncthreads();
  for (uint32_t q = tid; q < kSelH * kSelH + kSelH; q += nt) {
    double s = 0.0;
    if (q < kSelH * kSelH) {
      const uint32_t j = q / kSelH, l = q % kSelH;
      for (uint32_t i = 0; i < n; ++i) s += dz2[(size_t)i * kSelH + j] * h1[(size_t)i * kSelH + l];
      gW2[q] = s;
    } else {
      const uint32_t j = q - kSelH * kSelH;
      for (uint32_t i = 0; i < n; ++i) s += dz2[(size_t)i * kSelH + j];
      gb2[j] = s;
    }
  }
  for (uint64_t q = tid; q < (uint64_t)n * kSelH; q += nt) {
    const uint64_t i = q / kSelH;
    const uint32_t l = static_cast<uint32_t>(q % kSelH);
    double s = 0.0;
    for (int j = 0; j < kSelH; ++j) s += dz2[i * kSelH + j] * W2[j * kSelH + l];
    const double h = h1[q];
    dz1[q] = s * (1.0 - h * h);
  }
  __syncthreads();
  for (uint32_t q = tid; q < kSelH * kSelD + kSelH; q += nt) {
    double s = 0.0;
    if (q < kSelH * kSelD) {
      const uint32_t j = q / kSelD, d = q % kSelD;
      for (uint32_t i = 0; i < n; ++i) s += dz1[(size_t)i * kSelH + j] * X[(size_t)i * kSelD + d];
      gW1[q] = s;
    } else {
      const uint32_t j = q - kSelH * kSelD;
      for (uint32_t i = 0; i < n; ++i) s += dz1[(size_t)i * kSelH + j];
      gb1[j] = s;
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kBlock) void sel_grad_kernel(const double* p, const double* X, const double* T, uint32_t n,
                                                          double* g, double* scr) {
  sel_grad_block(p, X, T, n, g, scr);
}

// `epochs` steps of full-batch gradient descent: p <- p - lr * grad.
__global__ __launch_bounds__(kBlock) void sel_train_kernel(double* p, const double* X, const double* T, uint32_t n,
                                                           uint32_t epochs, double lr, double* g, double* scr) {
  for (uint32_t ep = 0; ep < epochs; ++ep) {
    sel_grad_block(p, X, T, n, g, scr);
    for (uint32_t q = threadIdx.x; q < kSelParams; q += blockDim.x) p[q] -= lr * g[q];
    __syncthreads();
  }
}

// Scratch of the allocation-free training entry point: the gradient
// followed by the batch scratch of up to IPG_SELECTOR_NOALLOC_MAX_SAMPLES
// samples, in a device array the library owns (one copy per GPU, held until
// the process ends).  Host code never passes `scratch` itself to a kernel:
// on the host the name stands for a host-side shadow, not for the device
// copy, so every use goes through the per-device address below.
constexpr size_t kNoAllocDoubles = kSelParams + (size_t)IPG_SELECTOR_NOALLOC_MAX_SAMPLES * (4 * kSelH + kSelK);
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_dev[kMaxDevices];  // device address of `scratch` on each GPU, looked up once

// Device address of the current GPU's copy of `scratch`, found with
// hipGetSymbolAddress on the first call made with that GPU current.
static ipg_status noalloc_scratch(double** out) {
  int dev = -1;
  IPG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(IPG_EDEVICE, "ipg_selector_train_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    IPG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(IPG_EDEVICE, "ipg_selector_train_noalloc: no device address for the scratch array");
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return IPG_OK;
}

}  // namespace ipg

using namespace ipg;

extern "C" size_t ipg_selector_workspace_bytes(uint32_t n_samples) {
  return align_up((kSelParams + sel_scratch_doubles(n_samples)) * sizeof(double), 256);
}

extern "C" ipg_status ipg_selector_forward(const double* params, const double* x, uint32_t n, double* y,
                                           void* hip_stream) {
  if (!params || (n && (!x || !y))) return fail(IPG_EINVAL, "ipg_selector_forward: NULL argument");
  if (n == 0) return IPG_OK;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(sel_forward_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, params, x, n, y);
  IPG_HIP(hipGetLastError());
  return IPG_OK;
}

extern "C" ipg_status ipg_selector_grad(const double* params, const double* x, const double* t, uint32_t n,
                                        double* grad, void* ws, size_t ws_bytes, void* hip_stream) {
  if (!params || !x || !t || !grad || n == 0) return fail(IPG_EINVAL, "ipg_selector_grad: NULL argument or n == 0");
  if (!ws || ws_bytes < ipg_selector_workspace_bytes(n)) return fail(IPG_EWORKSPACE, "ipg_selector_grad: workspace too small");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  double* scr = static_cast<double*>(ws) + kSelParams;
  hipLaunchKernelGGL(sel_grad_kernel, dim3(1), dim3(kBlock), 0, s, params, x, t, n, grad, scr);
  IPG_HIP(hipGetLastError());
  return IPG_OK;
}

extern "C" ipg_status ipg_selector_train(double* params, const double* x, const double* t, uint32_t n,
                                         uint32_t epochs, double lr, void* ws, size_t ws_bytes, void* hip_stream) {
  if (!params || !x || !t || n == 0) return fail(IPG_EINVAL, "ipg_selector_train: NULL argument or n == 0");
  if (!ws || ws_bytes < ipg_selector_workspace_bytes(n)) return fail(IPG_EWORKSPACE, "ipg_selector_train: workspace too small");
  if (!(lr > 0.0)) return fail(IPG_EINVAL, "ipg_selector_train: lr must be > 0");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  double* g = static_cast<double*>(ws);
  double* scr = g + kSelParams;
  hipLaunchKernelGGL(sel_train_kernel, dim3(1), dim3(kBlock), 0, s, params, x, t, n, epochs, lr, g, scr);
  IPG_HIP(hipGetLastError());
  return IPG_OK;
}

extern "C" ipg_status ipg_selector_train_noalloc(double* params, const double* x, const double* t, uint32_t n,
                                                 uint32_t epochs, double lr, void* hip_stream) {
  if (!params || !x || !t || n == 0) return fail(IPG_EINVAL, "ipg_selector_train_noalloc: NULL argument or n == 0");
  if (n > IPG_SELECTOR_NOALLOC_MAX_SAMPLES)
    return fail(IPG_EINVAL, "ipg_selector_train_noalloc: n exceeds IPG_SELECTOR_NOALLOC_MAX_SAMPLES (" +
                                std::to_string(IPG_SELECTOR_NOALLOC_MAX_SAMPLES) + ")");
  if (!(lr > 0.0)) return fail(IPG_EINVAL, "ipg_selector_train_noalloc: lr must be > 0");
  double* ws = nullptr;
  const ipg_status rc = noalloc_scratch(&ws);
  if (rc != IPG_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // every gradient entry and every scratch entry the kernel reads is written
  // by it first in each epoch, so nothing left by an earlier call is read
  hipLaunchKernelGGL(sel_train_kernel, dim3(1), dim3(kBlock), 0, s, params, x, t, n, epochs, lr, ws, ws + kSelParams);
  IPG_HIP(hipGetLastError());
  return IPG_OK;
}
