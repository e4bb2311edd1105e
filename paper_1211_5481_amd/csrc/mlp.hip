// Fitness-surrogate MLP: y = w3 . gelu(W2 gelu(W1 g + b1) + b2) + b3, trained
// online with Adam (Kingma and Ba) on (chromosome, standardised log MSE)
// pairs.  GELU is the exact form a * Phi(a) = a (1 + erf(a / sqrt 2)) / 2.
//
// All products go through one float32 GEMM kernel, C = op(A) op(B), with
// arbitrary element strides (so the transposed products of the backward pass
// need no copies) and a fused epilogue.  Products too small to fill the chip
// split K into S slices whose partial tiles a second kernel adds in slice
// order before the epilogue; every output element is a fixed-order sum, so
// results are bit-reproducible.
//
// Parameters are one flat float32 array: W1 (H1 x L), b1 (H1), W2 (H2 x H1),
// b2 (H2), w3 (H2), b3 (1); gradients and Adam moments use the same layout.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "game_internal.hpp"

namespace game {
namespace {

constexpr int kTile = 64, kKStep = 16, kGemmThreads = 256;

enum Epi : int {
  kEpiStore = 0,      // C = acc
  kEpiBiasGelu = 1,   // pre = acc + bias[n] -> P (if given); C = gelu(pre)
  kEpiGeluGrad = 2,   // C = acc * gelu'(P[m, n])
  kEpiPartial = 3,    // split K: slice z of the sum to part[z][m][n]
};

__device__ __forceinline__ float gelu(float a) { return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float a) {
  const float cdf = 0.5f * (1.0f + erff(a * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * a * a);
  return cdf + a * pdf;
}

struct GemmArgs {
  int M, N, K;
  const float* A;
  int64_t as0, as1;  // A(m, k) = A[m * as0 + k * as1]
  const float* B;
  int64_t bs0, bs1;  // B(k, n) = B[k * bs0 + n * bs1]
  float* C;
  int64_t ldc;       // C(m, n) = C[m * ldc + n]
  const float* bias; // kEpiBiasGelu
  float* P;          // pre-activation store / read, row stride ldc
  float* part;       // split K: S slices of M x N partial sums
  int S;             // K slices (1: no split)
};

template <int EPI>
__device__ __forceinline__ void epilogue(const GemmArgs& g, int m, int n, float acc) {
  const int64_t o = (int64_t)m * g.ldc + n;
  if constexpr (EPI == kEpiStore) {
    g.C[o] = acc;
  } else if constexpr (EPI == kEpiBiasGelu) {
    const float pre = acc + g.bias[n];
    if (g.P) g.P[o] = pre;
    g.C[o] = gelu(pre);
  } else {
    g.C[o] = acc * gelu_grad(g.P[o]);
  }
}

template <int EPI>
__global__ __launch_bounds__(kGemmThreads) void gemm_kernel(GemmArgs g, const DevState* halt) {
  if (run_halted(halt)) return;
  __shared__ float As[kKStep][kTile + 1];
  __shared__ float Bs[kKStep][kTile + 1];
  const int tid = threadIdx.x;
  const int tm = tid / 16, tn = tid % 16;  // 16 x 16 threads, 4 x 4 outputs each
  const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
  // K slice of this workgroup (whole K without a split)
  const int kc = (g.K + g.S - 1) / g.S;
  const int kbeg = blockIdx.z * kc, kend = min(g.K, kbeg + kc);
  float acc[4][4] = {};
  for (int k0 = kbeg; k0 < kend; k0 += kKStep) {
    for (int e = tid; e < kTile * kKStep; e += kGemmThreads) {
      const int r = e / kKStep, kk = e % kKStep;  // A tile: 64 rows x 16 k
      const int m = m0 + r, k = k0 + kk;
      As[kk][r] = (m < g.M && k < kend) ? g.A[m * g.as0 + k * g.as1] : 0.0f;
      const int c = e % kTile, kb = e / kTile;    // B tile: 16 k x 64 cols
      const int n = n0 + c, k2 = k0 + kb;
      Bs[kb][c] = (n < g.N && k2 < kend) ? g.B[k2 * g.bs0 + n * g.bs1] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kKStep; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tm * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tn * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + tm * 4 + i;
    if (m >= g.M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tn * 4 + j;
      if (n >= g.N) continue;
      if constexpr (EPI == kEpiPartial)
        g.part[((int64_t)blockIdx.z * g.M + m) * g.N + n] = acc[i][j];
      else
        epilogue<EPI>(g, m, n, acc[i][j]);
    }
  }
}

// Split K, second pass: add the S slices in order, then the epilogue.
template <int EPI>
__global__ void splitk_sum_kernel(GemmArgs g, const DevState* halt) {
  if (run_halted(halt)) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t mn = (int64_t)g.M * g.N;
  if (e >= mn) return;
  float acc = 0.0f;
  for (int z = 0; z < g.S; ++z) acc += g.part[z * mn + e];
  epilogue<EPI>(g, (int)(e / g.N), (int)(e % g.N), acc);
}

constexpr int kFillWgs = 256;  // workgroups that fill the chip once

template <int EPI>
hipError_t gemm(GemmArgs g, const float* part, int64_t part_cap, const DevState* halt, hipStream_t s) {
  if (g.M == 0 || g.N == 0) return hipSuccess;
  const int tiles = ((g.N + kTile - 1) / kTile) * ((g.M + kTile - 1) / kTile);
  int S = 1;
  if (part && tiles < kFillWgs) {
    S = (kFillWgs + tiles - 1) / tiles;
    S = std::min(S, std::max(1, g.K / (4 * kKStep)));           // slices of >= 64 k
    S = (int)std::min<int64_t>(S, part_cap / ((int64_t)g.M * g.N));
    if (S < 1) S = 1;
  }
  g.S = S;
  g.part = const_cast<float*>(part);
  const dim3 grid((unsigned)((g.N + kTile - 1) / kTile), (unsigned)((g.M + kTile - 1) / kTile), (unsigned)S);
  if (S == 1) {
    hipLaunchKernelGGL(gemm_kernel<EPI>, grid, dim3(kGemmThreads), 0, s, g, halt);
  } else {
    hipLaunchKernelGGL(gemm_kernel<kEpiPartial>, grid, dim3(kGemmThreads), 0, s, g, halt);
    const int64_t mn = (int64_t)g.M * g.N;
    hipLaunchKernelGGL(splitk_sum_kernel<EPI>, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, g,
                       halt);
  }
  return hipGetLastError();
}

// y[b] = h2[b, :] . w3 + b3 (one wave per row, lanes over the hidden units,
// fixed shuffle tree)
__global__ void head_kernel(const float* __restrict__ h2, int B, int H2, const float* __restrict__ w3,
                            const float* __restrict__ b3, float* __restrict__ y, const DevState* halt) {
  if (run_halted(halt)) return;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= B) return;
  float s = 0.0f;
  for (int k = lane; k < H2; k += 64) s = fmaf(h2[(int64_t)row * H2 + k], w3[k], s);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) y[row] = s + b3[0];
}

// Loss and output gradient: r = y - target, dy = 2 r / B; loss = sum r^2 / B
// (one workgroup, fixed order).
__global__ void loss_kernel(const float* __restrict__ y, const float* __restrict__ target, int B,
                            float* __restrict__ dy, float* __restrict__ loss, const DevState* halt) {
  if (run_halted(halt)) return;
  __shared__ float part[256];
  float s = 0.0f;
  for (int b = threadIdx.x; b < B; b += 256) {
    const float r = y[b] - target[b];
    dy[b] = 2.0f * r / (float)B;
    s = fmaf(r, r, s);
  }
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int i = 0; i < 256; ++i) t += part[i];
    if (loss) *loss = t / (float)B;
  }
}

// dA2[b, n] = dy[b] * w3[n] * gelu'(A2[b, n])
__global__ void head_back_kernel(const float* __restrict__ dy, const float* __restrict__ w3,
                                 const float* __restrict__ a2, int B, int H2, float* __restrict__ da2,
                                 const DevState* halt) {
  if (run_halted(halt)) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * H2) return;
  const int b = (int)(i / H2), n = (int)(i % H2);
  da2[i] = dy[b] * w3[n] * gelu_grad(a2[i]);
}

// Column sums (bias gradients) and the head weight gradient: out[n] = sum_b
// X[b, n] * (w ? w[b] : 1).  A workgroup takes 64 columns; its 16 row slices
// (rows b = slice mod 16, in order) are added in slice order.
__global__ __launch_bounds__(1024) void colsum_kernel(const float* __restrict__ X,
                                                      const float* __restrict__ w, int B, int N,
                                                      float* __restrict__ out, const DevState* halt) {
  if (run_halted(halt)) return;
  __shared__ float part[16][64];
  const int c = threadIdx.x & 63, slice = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  float s = 0.0f;
  if (n < N)
    for (int b = slice; b < B; b += 16) s = fmaf(X[(int64_t)b * N + n], w ? w[b] : 1.0f, s);
  part[slice][c] = s;
  __syncthreads();
  if (slice == 0 && n < N) {
    float t = 0.0f;
    for (int q = 0; q < 16; ++q) t += part[q][c];
    out[n] = t;
  }
}

// Adam over the flat parameter array; t is the step number after increment.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                            const int32_t* __restrict__ step, const DevState* halt) {
  if (run_halted(halt)) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int t = *step;
  const float mi = b1 * m[i] + (1.0f - b1) * g[i];
  const float vi = b2 * v[i] + (1.0f - b2) * g[i] * g[i];
  m[i] = mi;
  v[i] = vi;
  const float mhat = mi / (1.0f - powf(b1, (float)t));
  const float vhat = vi / (1.0f - powf(b2, (float)t));
  p[i] -= lr * mhat / (sqrtf(vhat) + eps);
}

__global__ void step_inc_kernel(int32_t* step, const DevState* halt) {
  if (run_halted(halt)) return;
  *step += 1;
}

// He-uniform init: block (layer, row, col, MLP_INIT) word 0 -> u in (0, 1),
// w = sqrt(6 / fan_in) (2u - 1); biases and moments zero.
__global__ void init_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            int L, int H1, int H2, uint32_t k0, uint32_t k1) {
  const int64_t n1 = (int64_t)H1 * L, n2 = (int64_t)H2 * H1;
  const int64_t total = n1 + H1 + n2 + H2 + H2 + 1;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  m[i] = 0.0f;
  v[i] = 0.0f;
  int layer = 0, rows = 0, cols = 1;
  int64_t j = i;
  if (j < n1) {
    layer = 1; cols = L;
  } else if ((j -= n1) < H1) {
    p[i] = 0.0f; return;
  } else if ((j -= H1) < n2) {
    layer = 2; cols = H1;
  } else if ((j -= n2) < H2) {
    p[i] = 0.0f; return;
  } else if ((j -= H2) < H2) {
    layer = 3; cols = H2;
  } else {
    p[i] = 0.0f; return;
  }
  (void)rows;
  const uint32_t r = (uint32_t)(j / cols), c = (uint32_t)(j % cols);
  const u32x4 b = philox((uint32_t)layer, r, c, kTagMlpInit, k0, k1);
  const double u = ((double)(b.x >> 8) + 0.5) * 0x1p-24;
  p[i] = (float)(sqrt(6.0 / (double)cols) * (2.0 * u - 1.0));
}

}  // namespace

MlpLayout mlp_layout(int L, int H1, int H2) {
  MlpLayout o;
  o.W1 = 0;
  o.b1 = o.W1 + (int64_t)H1 * L;
  o.W2 = o.b1 + H1;
  o.b2 = o.W2 + (int64_t)H2 * H1;
  o.w3 = o.b2 + H2;
  o.b3 = o.w3 + H2;
  o.total = o.b3 + 1;
  return o;
}

hipError_t mlp_init(const MlpDims& d, float* params, float* m, float* v, uint64_t seed,
                    hipStream_t s) {
  const int64_t n = mlp_layout(d.L, d.H1, d.H2).total;
  hipLaunchKernelGGL(init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, params, m, v,
                     d.L, d.H1, d.H2, (uint32_t)seed, (uint32_t)(seed >> 32));
  return hipGetLastError();
}

// Forward for B rows of X (B x L, row stride L).  a1/a2 (pre-activations) may
// be null when no backward pass follows.
hipError_t mlp_forward(const MlpDims& d, const float* params, const float* X, int B, float* a1,
                       float* h1, float* a2, float* h2, float* y, float* part, int64_t part_cap,
                       const DevState* halt, hipStream_t s) {
  const MlpLayout o = mlp_layout(d.L, d.H1, d.H2);
  hipError_t e;
  e = gemm<kEpiBiasGelu>({B, d.H1, d.L, X, d.L, 1, params + o.W1, 1, d.L, h1, d.H1, params + o.b1, a1},
                         part, part_cap, halt, s);
  if (e != hipSuccess) return e;
  e = gemm<kEpiBiasGelu>({B, d.H2, d.H1, h1, d.H1, 1, params + o.W2, 1, d.H1, h2, d.H2, params + o.b2, a2},
                         part, part_cap, halt, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(head_kernel, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, s, h2, B, d.H2,
                     params + o.w3, params + o.b3, y, halt);
  return hipGetLastError();
}

// Gradients of the mean squared error for one batch (forward included).
hipError_t mlp_grads(const MlpDims& d, const float* params, const float* X, const float* target,
                     int B, const MlpScratch& w, float* grads, float* loss, const DevState* halt,
                     hipStream_t s) {
  const MlpLayout o = mlp_layout(d.L, d.H1, d.H2);
  hipError_t e = mlp_forward(d, params, X, B, w.a1, w.h1, w.a2, w.h2, w.y, w.part, w.part_cap, halt, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, s, w.y, target, B, w.dy, loss, halt);
  // head: gw3 = h2^T dy, gb3 = sum dy
  hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((d.H2 + 63) / 64)), dim3(1024), 0, s, w.h2,
                     w.dy, B, d.H2, grads + o.w3, halt);
  hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(1024), 0, s, w.dy, nullptr, B, 1, grads + o.b3, halt);
  const int64_t n2 = (int64_t)B * d.H2;
  hipLaunchKernelGGL(head_back_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, w.dy,
                     params + o.w3, w.a2, B, d.H2, w.da2, halt);
  // layer 2: gW2 = dA2^T h1, gb2 = colsum dA2, dA1 = (dA2 W2) * gelu'(A1)
  e = gemm<kEpiStore>({d.H2, d.H1, B, w.da2, 1, d.H2, w.h1, d.H1, 1, grads + o.W2, d.H1, nullptr, nullptr},
                      w.part, w.part_cap, halt, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((d.H2 + 63) / 64)), dim3(1024), 0, s, w.da2,
                     nullptr, B, d.H2, grads + o.b2, halt);
  e = gemm<kEpiGeluGrad>({B, d.H1, d.H2, w.da2, d.H2, 1, params + o.W2, d.H1, 1, w.da1, d.H1, nullptr, w.a1},
                         w.part, w.part_cap, halt, s);
  if (e != hipSuccess) return e;
  // layer 1: gW1 = dA1^T X, gb1 = colsum dA1
  e = gemm<kEpiStore>({d.H1, d.L, B, w.da1, 1, d.H1, X, d.L, 1, grads + o.W1, d.L, nullptr, nullptr},
                      w.part, w.part_cap, halt, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((d.H1 + 63) / 64)), dim3(1024), 0, s, w.da1,
                     nullptr, B, d.H1, grads + o.b1, halt);
  return hipGetLastError();
}

hipError_t mlp_adam(const MlpDims& d, float* params, const float* grads, float* m, float* v,
                    int32_t* step, float lr, const DevState* halt, hipStream_t s) {
  const int64_t n = mlp_layout(d.L, d.H1, d.H2).total;
  hipLaunchKernelGGL(step_inc_kernel, dim3(1), dim3(1), 0, s, step, halt);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, params, grads,
                     m, v, n, lr, 0.9f, 0.999f, 1e-8f, step, halt);
  return hipGetLastError();
}

}  // namespace game
