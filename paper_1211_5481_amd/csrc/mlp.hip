// Fitness-surrogate MLP: y = w3 . gelu(W2 gelu(W1 g + b1) + b2) + b3, trained
// online with Adam (Kingma and Ba) on (chromosome, standardised log MSE)
// pairs.  GELU is the exact form a * Phi(a) = a (1 + erf(a / sqrt 2)) / 2.
//
// The network is small (L = 128 inputs, H = 256 hidden at the surrogate
// workload) and trained in many short steps, so a training step is two
// launches instead of one per product:
//   * rows kernel: a workgroup takes R minibatch rows at a time, draws them
//     from the replay ring (or reads given rows), runs the forward pass and
//     the whole backward pass for them in LDS and registers, and adds the
//     rows' gradient contributions to its own slab of partial sums (the
//     parameter layout plus the loss);
//   * reduce kernel: one thread per parameter adds the slabs in workgroup
//     order and applies Adam (or writes the gradient); the last workgroup to
//     finish advances the step counter.
// Every sum has a fixed order, so results are bit-reproducible.  Forward
// products read transposed copies of W1 and W2 (kept in step with every
// parameter update) so that lanes over output units load contiguous memory;
// the backward product through W2 reads W2 itself for the same reason.
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

constexpr int kThreads = 1024;
constexpr int kMaxR = 8;            // rows per workgroup pass (registers)
constexpr size_t kRowsLds = 98304;  // LDS budget of the rows kernel

__device__ __forceinline__ float gelu(float a) { return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float a) {
  const float cdf = 0.5f * (1.0f + erff(a * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * a * a);
  return cdf + a * pdf;
}

struct RowsArgs {
  const float* params;
  const float* WT;  // W1^T (L x H1) then W2^T (H1 x H2)
  int L, H1, H2, B, R, W;
  // rows: explicit (X, target) or drawn from the replay ring
  const float* X;
  const float* target;
  const float* buf;
  const float* bufy;
  const SurState* ss;
  const int32_t* step;
  uint32_t k0, k1;
  int n_recent, cap;
  float* y;       // forward only: scores of the B rows
  float* slab;    // training: W slabs of (parameters + 1) floats
  int64_t total;  // parameters
};

// Thread layout of the rows kernel: 1024 threads = 4 groups (ks) of 256
// column lanes (c).  A product over K is split into 4 contiguous K quarters,
// one per group; the quarters' partial sums are added in group order.
constexpr int kLanes = 256, kGroups = kThreads / kLanes;

// Partial dot products of column j (lane stride kLanes) over K quarter ks:
// acc[r] = sum_{k in quarter} W[k * ldw + j] * V[r * ldv + k], r < R.
__device__ __forceinline__ void quarter_dot(const float* __restrict__ W, int64_t ldw, int j,
                                            const float* V, int ldv, int K, int ks, int R,
                                            float (&acc)[kMaxR]) {
#pragma unroll
  for (int r = 0; r < kMaxR; ++r) acc[r] = 0.0f;
  const int q = (K + kGroups - 1) / kGroups;
  const int k0 = ks * q, k1 = min(K, k0 + q);
  int k = k0;
  if (((k0 | q | ldv) & 3) == 0 && (reinterpret_cast<uintptr_t>(V) & 15) == 0) {
    for (; k + 4 <= k1; k += 4) {
      float w[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) w[u] = W[(int64_t)(k + u) * ldw + j];
#pragma unroll
      for (int r = 0; r < kMaxR; ++r)
        if (r < R) {
          const float4 v = *reinterpret_cast<const float4*>(&V[r * ldv + k]);
          acc[r] = fmaf(w[0], v.x, acc[r]);
          acc[r] = fmaf(w[1], v.y, acc[r]);
          acc[r] = fmaf(w[2], v.z, acc[r]);
          acc[r] = fmaf(w[3], v.w, acc[r]);
        }
    }
  }
  for (; k < k1; ++k) {
    const float w = W[(int64_t)k * ldw + j];
#pragma unroll
    for (int r = 0; r < kMaxR; ++r)
      if (r < R) acc[r] = fmaf(w, V[r * ldv + k], acc[r]);
  }
}

template <bool kTrain>
__global__ __launch_bounds__(kThreads) void rows_kernel(RowsArgs a, const DevState* halt) {
  if (run_halted(halt)) return;
  extern __shared__ __align__(16) float sm[];
  const int L = a.L, H1 = a.H1, H2 = a.H2, R = a.R;
  const int Hm = H1 > H2 ? H1 : H2;
  float* X = sm;              // R x L
  float* A1 = X + R * L;      // R x H1 pre-activations
  float* Hd1 = A1 + R * H1;   // R x H1 activations
  float* D1 = Hd1 + R * H1;   // R x H1: dLoss/dA1
  float* A2 = D1 + R * H1;    // R x H2
  float* Hd2 = A2 + R * H2;   // R x H2
  float* D2 = Hd2 + R * H2;   // R x H2: dLoss/dA2
  float* red = D2 + R * H2;   // kGroups x R x Hm quarter sums
  __shared__ float s_t[kMaxR], s_y[kMaxR], s_dy[kMaxR];
  __shared__ int s_slot[kMaxR];
  const int tid = threadIdx.x, c = tid % kLanes, ks = tid / kLanes;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t oW1 = 0, ob1 = (int64_t)H1 * L, oW2 = ob1 + H1, ob2 = oW2 + (int64_t)H2 * H1,
                ow3 = ob2 + H2, ob3 = ow3 + H2;
  const float* P = a.params;
  const float* W1T = a.WT;
  const float* W2T = a.WT + (int64_t)L * H1;
  float* slab = kTrain ? a.slab + (int64_t)blockIdx.x * (a.total + 1) : nullptr;
  bool first = true;
  auto put = [&](int64_t o, float v) { slab[o] = first ? v : slab[o] + v; };
  // quarter sums of the columns this thread owns -> red[ks][r][j]
  auto to_red = [&](int j, const float (&acc)[kMaxR]) {
#pragma unroll
    for (int r = 0; r < kMaxR; ++r)
      if (r < R) red[(ks * R + r) * Hm + j] = acc[r];
  };
  auto quarters = [&](int r, int j) {
    float t = 0.0f;
    for (int g = 0; g < kGroups; ++g) t += red[(g * R + r) * Hm + j];
    return t;
  };

  for (int r0 = blockIdx.x * R; r0 < a.B; r0 += a.W * R) {
    const int nr = min(R, a.B - r0);
    // ---- rows and targets
    if (tid < nr) {
      if (a.X == nullptr) {
        const int i = r0 + tid;
        const uint32_t w = philox((uint32_t)*a.step, (uint32_t)i, 0u, kTagMinibatch, a.k0, a.k1).x;
        int slot;
        if (i < a.B - a.n_recent) {
          slot = (int)__umulhi(w, (uint32_t)a.ss->count);
        } else {
          const int back = (int)__umulhi(w, (uint32_t)a.ss->last);
          slot = (int)(((int64_t)a.ss->head - 1 - back + a.cap) % a.cap);
        }
        s_slot[tid] = slot;
        if (kTrain) s_t[tid] = (a.bufy[slot] - a.ss->mu) / a.ss->sigma;
      } else if (kTrain) {
        s_t[tid] = a.target[r0 + tid];
      }
    }
    __syncthreads();
    for (int r = 0; r < R; ++r)
      for (int l = tid; l < L; l += kThreads) {
        float v = 0.0f;
        if (r < nr) v = a.X ? a.X[(int64_t)(r0 + r) * L + l] : a.buf[(int64_t)s_slot[r] * L + l];
        X[r * L + l] = v;
      }
    __syncthreads();
    // ---- layer 1: A1 = X W1^T + b1
    for (int j = c; j < H1; j += kLanes) {
      float acc[kMaxR];
      quarter_dot(W1T, H1, j, X, L, L, ks, R, acc);
      to_red(j, acc);
    }
    __syncthreads();
    for (int e = tid; e < R * H1; e += kThreads) {
      const int r = e / H1, j = e - r * H1;
      const float pre = P[ob1 + j] + quarters(r, j);
      A1[e] = pre;
      Hd1[e] = gelu(pre);
    }
    __syncthreads();
    // ---- layer 2: A2 = H1 W2^T + b2
    for (int j = c; j < H2; j += kLanes) {
      float acc[kMaxR];
      quarter_dot(W2T, H2, j, Hd1, H1, H1, ks, R, acc);
      to_red(j, acc);
    }
    __syncthreads();
    for (int e = tid; e < R * H2; e += kThreads) {
      const int r = e / H2, j = e - r * H2;
      const float pre = P[ob2 + j] + quarters(r, j);
      A2[e] = pre;
      Hd2[e] = gelu(pre);
    }
    __syncthreads();
    // ---- head: y = H2 w3 + b3, wave r sums row r (fixed order)
    if (wave < R) {
      float y = 0.0f;
      for (int j = lane; j < H2; j += 64) y = fmaf(Hd2[wave * H2 + j], P[ow3 + j], y);
      for (int off = 32; off > 0; off >>= 1) y += __shfl_xor(y, off);
      if (lane == 0) s_y[wave] = y + P[ob3];
    }
    __syncthreads();
    if (!kTrain) {
      if (tid < nr) a.y[r0 + tid] = s_y[tid];
      __syncthreads();
      continue;
    }
    // ---- loss and output gradient: residual = y - t, dy = 2 residual / B
    if (tid < kMaxR) {
      const float res = tid < nr ? s_y[tid] - s_t[tid] : 0.0f;
      s_dy[tid] = 2.0f * res / (float)a.B;
      s_y[tid] = res * res;
    }
    __syncthreads();
    if (tid == 0) {
      float dsum = 0.0f, lsum = 0.0f;
      for (int r = 0; r < nr; ++r) {
        dsum += s_dy[r];
        lsum += s_y[r];
      }
      put(ob3, dsum);
      put(a.total, lsum);
    }
    // ---- dA2 = dy w3 gelu'(A2)
    for (int e = tid; e < R * H2; e += kThreads) {
      const int r = e / H2, j = e - r * H2;
      D2[e] = s_dy[r] * P[ow3 + j] * gelu_grad(A2[e]);  // zero for rows past the batch
    }
    __syncthreads();
    // ---- gradients of w3 and b2
    for (int j = tid; j < H2; j += kThreads) {
      float gw3 = 0.0f, gb2 = 0.0f;
      for (int r = 0; r < R; ++r) {
        gw3 = fmaf(Hd2[r * H2 + j], s_dy[r], gw3);
        gb2 += D2[r * H2 + j];
      }
      put(ow3 + j, gw3);
      put(ob2 + j, gb2);
    }
    // ---- gradient of W2: dA2^T H1 (rows j by group, columns i by lane)
    for (int j = ks; j < H2; j += kGroups)
      for (int i = c; i < H1; i += kLanes) {
        float g = 0.0f;
        for (int r = 0; r < R; ++r) g = fmaf(D2[r * H2 + j], Hd1[r * H1 + i], g);
        put(oW2 + (int64_t)j * H1 + i, g);
      }
    // ---- dA1 = (dA2 W2) gelu'(A1): quarter sums over j
    for (int i = c; i < H1; i += kLanes) {
      float acc[kMaxR];
      quarter_dot(P + oW2, H1, i, D2, H2, H2, ks, R, acc);
      to_red(i, acc);
    }
    __syncthreads();
    for (int e = tid; e < R * H1; e += kThreads) {
      const int r = e / H1, i = e - r * H1;
      D1[e] = quarters(r, i) * gelu_grad(A1[e]);
    }
    __syncthreads();
    // ---- gradient of b1, and of W1: dA1^T X
    for (int i = tid; i < H1; i += kThreads) {
      float gb1 = 0.0f;
      for (int r = 0; r < R; ++r) gb1 += D1[r * H1 + i];
      put(ob1 + i, gb1);
    }
    for (int i = ks; i < H1; i += kGroups)
      for (int l = c; l < L; l += kLanes) {
        float g = 0.0f;
        for (int r = 0; r < R; ++r) g = fmaf(D1[r * H1 + i], X[r * L + l], g);
        put(oW1 + (int64_t)i * L + l, g);
      }
    first = false;
    __syncthreads();
  }
  // a workgroup without rows contributes zeros
  if (kTrain && first)
    for (int64_t e = tid; e <= a.total; e += kThreads) slab[e] = 0.0f;
}

struct ReduceArgs {
  const float* slab;  // W slabs, `stride` floats apart
  int W;
  int64_t stride, total;
  int B;          // rows behind the sums (loss = sum / B)
  float* grads;   // gradient output (null: Adam)
  float* loss;    // loss output (null: none; the slabs then have no loss entry)
  float* params;  // Adam
  float* WT;
  float* m;
  float* v;
  int32_t* step;  // step counter, then an arrival counter (zero between launches)
  float lr;
  int L, H1, H2;
};

// Adds the slabs in order; writes the gradient, or applies one Adam step with
// t = step + 1 and refreshes the transposed weights; the last workgroup
// stores t.
__global__ void reduce_kernel(ReduceArgs a, const DevState* halt) {
  if (run_halted(halt)) return;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int t = a.grads ? 0 : *a.step + 1;
  if (p < a.total || (p == a.total && a.loss)) {
    float g = 0.0f;
    for (int w = 0; w < a.W; ++w) g += a.slab[(int64_t)w * a.stride + p];
    if (p == a.total) {
      *a.loss = g / (float)a.B;
    } else if (a.grads) {
      a.grads[p] = g;
    } else {
      const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
      const float mi = b1 * a.m[p] + (1.0f - b1) * g;
      const float vi = b2 * a.v[p] + (1.0f - b2) * g * g;
      a.m[p] = mi;
      a.v[p] = vi;
      const float mhat = mi / (1.0f - powf(b1, (float)t));
      const float vhat = vi / (1.0f - powf(b2, (float)t));
      const float nv = a.params[p] - a.lr * mhat / (sqrtf(vhat) + eps);
      a.params[p] = nv;
      const int64_t n1 = (int64_t)a.H1 * a.L, o2 = n1 + a.H1, n2 = (int64_t)a.H2 * a.H1;
      if (p < n1) {
        const int64_t j = p / a.L, l = p - j * a.L;
        a.WT[l * a.H1 + j] = nv;
      } else if (p >= o2 && p < o2 + n2) {
        const int64_t q = p - o2, j = q / a.H1, i = q - j * a.H1;
        a.WT[n1 + i * a.H2 + j] = nv;
      }
    }
  }
  if (a.grads) return;
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0)
    s_last = atomicAdd(reinterpret_cast<uint32_t*>(a.step + 1), 1u) == gridDim.x - 1;
  __syncthreads();
  if (s_last && threadIdx.x == 0) {
    *a.step = t;
    a.step[1] = 0;
  }
}

// Transposed copies of W1 and W2 from the parameters.
__global__ void transpose_kernel(const float* __restrict__ P, float* __restrict__ WT, int L, int H1,
                                 int H2) {
  const int64_t n1 = (int64_t)H1 * L, n2 = (int64_t)H2 * H1;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n1) {
    const int64_t j = e / L, l = e - j * L;
    WT[l * H1 + j] = P[e];
  } else if (e < n1 + n2) {
    const int64_t q = e - n1, j = q / H1, i = q - j * H1;
    WT[n1 + i * H2 + j] = P[n1 + H1 + q];
  }
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
  int layer = 0, cols = 1;
  int64_t j = i;
  if (j < n1) {
    layer = 1;
    cols = L;
  } else if ((j -= n1) < H1) {
    p[i] = 0.0f;
    return;
  } else if ((j -= H1) < n2) {
    layer = 2;
    cols = H1;
  } else if ((j -= n2) < H2) {
    p[i] = 0.0f;
    return;
  } else if ((j -= H2) < H2) {
    layer = 3;
    cols = H2;
  } else {
    p[i] = 0.0f;
    return;
  }
  const uint32_t r = (uint32_t)(j / cols), c = (uint32_t)(j % cols);
  const u32x4 b = philox((uint32_t)layer, r, c, kTagMlpInit, k0, k1);
  const double u = ((double)(b.x >> 8) + 0.5) * 0x1p-24;
  p[i] = (float)(sqrt(6.0 / (double)cols) * (2.0 * u - 1.0));
}

size_t rows_lds(const MlpDims& d, int R) {
  const size_t Hm = (size_t)std::max(d.H1, d.H2);
  return (size_t)R * ((size_t)d.L + 3 * (size_t)d.H1 + 3 * (size_t)d.H2 + 4 * Hm) * sizeof(float);
}

hipError_t rows_prepare() {
  static bool done = false;
  if (done) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(rows_kernel<true>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRowsLds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(rows_kernel<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRowsLds);
  if (e == hipSuccess) done = true;
  return e;
}

hipError_t launch_rows(bool train, const RowsArgs& a, const MlpDims& d, const DevState* halt,
                       hipStream_t s) {
  const hipError_t e = rows_prepare();
  if (e != hipSuccess) return e;
  const size_t lds = rows_lds(d, a.R);
  if (train)
    hipLaunchKernelGGL(rows_kernel<true>, dim3((unsigned)a.W), dim3(kThreads), lds, s, a, halt);
  else
    hipLaunchKernelGGL(rows_kernel<false>, dim3((unsigned)a.W), dim3(kThreads), lds, s, a, halt);
  return hipGetLastError();
}

int64_t slab_stride(const MlpDims& d) { return mlp_layout(d.L, d.H1, d.H2).total + 1; }

RowsArgs rows_args(const MlpDims& d, const float* params, const float* WT, int B) {
  RowsArgs a{};
  a.params = params;
  a.WT = WT;
  a.L = d.L;
  a.H1 = d.H1;
  a.H2 = d.H2;
  a.B = B;
  a.R = mlp_rows_per_pass(d);
  a.total = mlp_layout(d.L, d.H1, d.H2).total;
  return a;
}

// Workgroups of a training launch: one per R rows, as many slabs as fit.
int train_wgs(const MlpDims& d, int B, int R, int64_t slab_cap) {
  int64_t W = (B + R - 1) / R;
  W = std::min<int64_t>(W, slab_cap / slab_stride(d));
  return (int)std::max<int64_t>(W, 1);
}

hipError_t launch_reduce(const ReduceArgs& a, const DevState* halt, hipStream_t s) {
  const int64_t n = a.total + 1;
  hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, halt);
  return hipGetLastError();
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

int mlp_rows_per_pass(const MlpDims& d) {
  int R = kMaxR;
  while (R > 1 && rows_lds(d, R) > kRowsLds) R /= 2;
  return R;
}

bool mlp_fits(const MlpDims& d) { return rows_lds(d, 1) <= kRowsLds; }

int64_t mlp_slab_floats(const MlpDims& d, int rows) {
  const int64_t per = slab_stride(d);
  const int R = mlp_rows_per_pass(d);
  int64_t W = std::min<int64_t>((rows + R - 1) / R, kMlpSlabFloats / per);
  return std::max<int64_t>(W, 1) * per;
}

hipError_t mlp_transpose(const MlpDims& d, const float* params, float* WT, hipStream_t s) {
  const int64_t n = (int64_t)d.H1 * d.L + (int64_t)d.H2 * d.H1;
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, params, WT,
                     d.L, d.H1, d.H2);
  return hipGetLastError();
}

hipError_t mlp_init(const MlpDims& d, float* params, float* m, float* v, float* WT, uint64_t seed,
                    hipStream_t s) {
  const int64_t n = mlp_layout(d.L, d.H1, d.H2).total;
  hipLaunchKernelGGL(init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, params, m, v,
                     d.L, d.H1, d.H2, (uint32_t)seed, (uint32_t)(seed >> 32));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return mlp_transpose(d, params, WT, s);
}

hipError_t mlp_forward(const MlpDims& d, const float* params, const float* WT, const float* X, int B,
                       float* y, const DevState* halt, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  RowsArgs a = rows_args(d, params, WT, B);
  a.W = (B + a.R - 1) / a.R;
  a.X = X;
  a.y = y;
  return launch_rows(false, a, d, halt, s);
}

hipError_t mlp_grads(const MlpDims& d, const float* params, const float* WT, const float* X,
                     const float* target, int B, float* slab, int64_t slab_cap, float* grads,
                     float* loss, const DevState* halt, hipStream_t s) {
  RowsArgs a = rows_args(d, params, WT, B);
  a.W = train_wgs(d, B, a.R, slab_cap);
  a.X = X;
  a.target = target;
  a.slab = slab;
  hipError_t e = launch_rows(true, a, d, halt, s);
  if (e != hipSuccess) return e;
  ReduceArgs r{};
  r.slab = slab;
  r.W = a.W;
  r.stride = a.total + 1;
  r.total = a.total;
  r.B = B;
  r.grads = grads;
  r.loss = loss;
  return launch_reduce(r, halt, s);
}

hipError_t mlp_train_step(const MlpDims& d, float* params, float* WT, float* m, float* v,
                          int32_t* step, float lr, const float* buf, const float* bufy,
                          const SurState* ss, uint64_t seed, int B, int n_recent, int cap,
                          float* slab, int64_t slab_cap, float* loss, const DevState* halt,
                          hipStream_t s) {
  RowsArgs a = rows_args(d, params, WT, B);
  a.W = train_wgs(d, B, a.R, slab_cap);
  a.buf = buf;
  a.bufy = bufy;
  a.ss = ss;
  a.step = step;
  a.k0 = (uint32_t)seed;
  a.k1 = (uint32_t)(seed >> 32);
  a.n_recent = n_recent;
  a.cap = cap;
  a.slab = slab;
  hipError_t e = launch_rows(true, a, d, halt, s);
  if (e != hipSuccess) return e;
  ReduceArgs r{};
  r.slab = slab;
  r.W = a.W;
  r.stride = a.total + 1;
  r.total = a.total;
  r.B = B;
  r.loss = loss;
  r.params = params;
  r.WT = WT;
  r.m = m;
  r.v = v;
  r.step = step;
  r.lr = lr;
  r.L = d.L;
  r.H1 = d.H1;
  r.H2 = d.H2;
  return launch_reduce(r, halt, s);
}

hipError_t mlp_adam(const MlpDims& d, float* params, float* WT, const float* grads, float* m, float* v,
                    int32_t* step, float lr, const DevState* halt, hipStream_t s) {
  ReduceArgs r{};
  r.slab = grads;  // one slab: the gradient itself (no loss entry)
  r.W = 1;
  r.total = mlp_layout(d.L, d.H1, d.H2).total;
  r.stride = r.total;
  r.B = 1;
  r.params = params;
  r.WT = WT;
  r.m = m;
  r.v = v;
  r.step = step;
  r.lr = lr;
  r.L = d.L;
  r.H1 = d.H1;
  r.H2 = d.H2;
  return launch_reduce(r, halt, s);
}

}  // namespace game
