// Test and validation use (Sec. 4): one chromosome applied to a pattern set.
//
//   prediction: z = sum_i sum_k g[i*K+k] phi_k(x_i) (+ bias gene), output z
//               (regression) or sigmoid(z) (classification); in the
//               shared-coefficient model (M == K) feature i uses g[k];
//   metrics:    squared error summed over the patterns, and for
//               classification the confusion counts (class 1 positive,
//               predicted 1 iff z >= 0, label [t >= 0.5]).
//
// Every pattern is computed in double from the float32 genes, whatever the
// training dtype.  Metric partials are summed per thread in row order, per
// workgroup in a fixed tree, then across workgroups in order, so repeated
// calls give identical results.  Bound: the basis recurrences (VALU), one
// pass over X.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "expand.hpp"
#include "game_internal.hpp"

namespace game {
namespace {

constexpr int kThreads = 256;

template <typename T>
__device__ __forceinline__ double pattern_z(const T* __restrict__ X, int64_t n, const PredictArgs& a) {
  double z = a.bias ? (double)a.genes[a.M] : 0.0;
  for (int i = 0; i < a.F; ++i) {
    const float* g = a.genes + (a.M == a.K ? 0 : (int64_t)i * a.K);
    expand_feature(a.basis, a.D, (double)X[n * a.F + i],
                   [&](int k, double v) { z = fma(v, (double)g[k], z); });
  }
  return z;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void predict_kernel(PredictArgs a) {
  const T* X = static_cast<const T*>(a.X);
  T* out = static_cast<T*>(a.out);
  for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < a.n;
       n += (int64_t)gridDim.x * kThreads) {
    const double z = pattern_z(X, n, a);
    out[n] = (T)(a.task == GAME_CLASSIFICATION ? 1.0 / (1.0 + exp(-z)) : z);
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void metrics_kernel(PredictArgs a) {
  const T* X = static_cast<const T*>(a.X);
  const T* t = static_cast<const T*>(a.t);
  double sse = 0.0;
  uint64_t cnt[4] = {0, 0, 0, 0};  // TP, FP, TN, FN
  for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < a.n;
       n += (int64_t)gridDim.x * kThreads) {
    const double z = pattern_z(X, n, a);
    const double tn = (double)t[n];
    if (a.task == GAME_CLASSIFICATION) {
      const bool lab = tn >= 0.5, pred = z >= 0.0;
      const double e = (lab ? 1.0 : 0.0) - 1.0 / (1.0 + exp(-z));
      sse = fma(e, e, sse);
      cnt[pred ? (lab ? 0 : 1) : (lab ? 3 : 2)] += 1;
    } else {
      const double e = tn - z;
      sse = fma(e, e, sse);
    }
  }
  __shared__ double s_sse[kThreads];
  __shared__ uint64_t s_cnt[4][kThreads];
  s_sse[threadIdx.x] = sse;
  for (int q = 0; q < 4; ++q) s_cnt[q][threadIdx.x] = cnt[q];
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s_sse[threadIdx.x] += s_sse[threadIdx.x + h];
      for (int q = 0; q < 4; ++q) s_cnt[q][threadIdx.x] += s_cnt[q][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* p = a.part + 5 * (int64_t)blockIdx.x;
    p[0] = s_sse[0];
    for (int q = 0; q < 4; ++q) p[1 + q] = (double)s_cnt[q][0];
  }
}

// Adds the workgroup partials in order: result = {sse, TP, FP, TN, FN}.
__global__ void metrics_final_kernel(const double* __restrict__ part, int parts, double* result) {
  if (threadIdx.x != 0) return;
  double r[5] = {0, 0, 0, 0, 0};
  for (int b = 0; b < parts; ++b)
    for (int q = 0; q < 5; ++q) r[q] += part[5 * b + q];
  for (int q = 0; q < 5; ++q) result[q] = r[q];
}

int grid_for(int64_t n) {
  const int64_t g = (n + kThreads - 1) / kThreads;
  return (int)(g < kPredictParts ? (g > 0 ? g : 1) : kPredictParts);
}

}  // namespace

hipError_t launch_predict(bool f64, const PredictArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (f64)
    hipLaunchKernelGGL(predict_kernel<double>, dim3((unsigned)grid_for(a.n)), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(predict_kernel<float>, dim3((unsigned)grid_for(a.n)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_metrics(bool f64, const PredictArgs& a, double* result, hipStream_t s) {
  const int g = grid_for(a.n);
  if (f64)
    hipLaunchKernelGGL(metrics_kernel<double>, dim3((unsigned)g), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(metrics_kernel<float>, dim3((unsigned)g), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(metrics_final_kernel, dim3(1), dim3(64), 0, s, a.part, g, result);
  return hipGetLastError();
}

}  // namespace game
