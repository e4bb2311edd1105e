// Float32 re-score of a few chromosomes (the elites of a 16-bit run).
//
// The BF16/FP16 forms rank the population with 16-bit Phi and genes; the
// chromosomes that matter (the elites, and in the end the best one) are
// scored again here with float32 basis values and float32 arithmetic: each
// thread walks patterns, recomputes the pattern's basis row from x (double
// recurrence rounded to float32, as the FP32 path stores Phi), forms
// z = sum_m phi_m g_m in float32 for every chromosome, and adds the error
// (eq. 3; classification against the class label) in double.  In the
// shared-coefficient model (M == K) a pattern's basis value k is the sum over
// its features in double, rounded to float32 once, as the FP32 path stores
// it; each column re-runs the features' recurrences (K times the work of the
// per-feature model, but no per-column array).  Block sums
// are combined in a fixed order by the last workgroup to arrive, so results
// are bit-reproducible.  For a population evaluation the same workgroup then
// tracks the best chromosome by the float32 MSE and applies the stop test.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "expand.hpp"
#include "game_internal.hpp"
#include "select.hpp"

namespace game {
namespace {

constexpr int kThreads = 256;

struct RescoreArgs {
  const float* X;        // N x F, float32 copy of the patterns
  const float* t;        // N_pad targets (float32)
  int64_t N;
  int F, D, K, basis, M, L, bias, task;
  const float* genes;    // n x L chromosomes (explicit set), or null: population elites
  int n;                 // chromosomes to score (<= kMaxRescore)
  const float* pop0;     // population buffers (generation parity) when genes is null
  const float* pop1;
  const int* top;        // ranking of the population when genes is null
  double* part;          // [grid][2 * kMaxRescore] block partials (sse, misses)
  uint32_t* counter;     // zero between launches
  double* mse;           // n results (device) or null
  double* miscls;
  const DevState* sel;   // generation parity for the population buffers (never null)
  DevState* st;          // tracking mode: best tracking + stop test; else null
  float* best;           // best genes (tracking mode)
};

// NS = a.n chromosomes (1..kMaxRescore) as a template parameter: the
// per-basis-value loop over chromosomes then has no runtime guards, which
// cost more than the arithmetic they guarded.
template <int NS>
__global__ __launch_bounds__(kThreads) void rescore_kernel(RescoreArgs a) {
  if (run_halted(a.st)) return;
  extern __shared__ float g_lds[];  // n x L genes
  __shared__ double s_red[kThreads / 64][2 * kMaxRescore];
  __shared__ int s_flag;
  __shared__ int s_rows[kMaxRescore];
  const int tid = threadIdx.x;
  const float* src = a.genes;
  if (!src) src = (a.sel->generation & 1) ? a.pop1 : a.pop0;
  if (tid < a.n) s_rows[tid] = a.genes ? tid : a.top[tid];
  __syncthreads();
  for (int i = tid; i < a.n * a.L; i += kThreads) {
    const int e = i / a.L, l = i - e * a.L;
    g_lds[i] = src[(int64_t)s_rows[e] * a.L + l];
  }
  __syncthreads();

  double sse[NS];
  double mis[NS];
#pragma unroll
  for (int e = 0; e < NS; ++e) {
    sse[e] = 0.0;
    mis[e] = 0.0;
  }
  // shared-coefficient model; with one feature both forms are the same
  const bool shared = a.M == a.K && a.F > 1;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t nrow = (int64_t)blockIdx.x * kThreads + tid; nrow < a.N; nrow += stride) {
    float z[NS];
#pragma unroll
    for (int e = 0; e < NS; ++e) z[e] = 0.0f;
    for (int k = 0; shared && k < a.K; ++k) {
      double sum = 0.0;
      for (int i = 0; i < a.F; ++i) {
        double v = 0.0;
        expand_feature(a.basis, a.D, (double)a.X[nrow * a.F + i], [&](int kk, double val) {
          if (kk == k) v = val;
        });
        sum += v;
      }
      const float vf = (float)sum;
#pragma unroll
      for (int e = 0; e < NS; ++e) z[e] = fmaf(vf, g_lds[e * a.L + k], z[e]);
    }
    for (int i = 0; !shared && i < a.F; ++i) {
      const float* gi = g_lds + i * a.K;
      expand_feature(a.basis, a.D, (double)a.X[nrow * a.F + i], [&](int k, double val) {
        const float vf = (float)val;
#pragma unroll
        for (int e = 0; e < NS; ++e) z[e] = fmaf(vf, gi[e * a.L + k], z[e]);
      });
    }
    const float tn = a.t[nrow];
    const float lab = tn >= 0.5f ? 1.0f : 0.0f;
#pragma unroll
    for (int e = 0; e < NS; ++e) {
      const float ze = a.bias ? z[e] + g_lds[e * a.L + a.M] : z[e];
      float d;
      if (a.task == GAME_CLASSIFICATION) {
        d = lab - 1.0f / (1.0f + expf(-ze));
        mis[e] += ((ze >= 0.0f) != (lab > 0.5f)) ? 1.0 : 0.0;
      } else {
        d = tn - ze;
      }
      sse[e] += (double)(d * d);
    }
  }
  // fixed-order block reduction: wave shuffle tree, then waves in order
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int e = 0; e < NS; ++e) {
    for (int off = 32; off > 0; off >>= 1) {
      sse[e] += __shfl_xor(sse[e], off);
      mis[e] += __shfl_xor(mis[e], off);
    }
    if (lane == 0) {
      s_red[wave][e] = sse[e];
      s_red[wave][kMaxRescore + e] = mis[e];
    }
  }
  __syncthreads();
  // value v of a block: sse of chromosome v (v < kMaxRescore), misses of
  // chromosome v - kMaxRescore; only the first NS of each are used
  const int v_me = tid < NS ? tid : kMaxRescore + tid - NS;
  if (tid < 2 * NS) {
    double s = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) s += s_red[w][v_me];
    st_agent(a.part + (int64_t)blockIdx.x * 2 * kMaxRescore + v_me, s);
  }
  agent_stores_done();
  __syncthreads();
  if (tid == 0) s_flag = atomicAdd(a.counter, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!s_flag) return;
  // last workgroup: thread t adds blocks t, t + 256, ... (in that order), then
  // thread v adds the 256 thread sums of value v in thread order
  __shared__ double s_all[kThreads][2 * kMaxRescore];
  __shared__ double s_mse[kMaxRescore], s_mis[kMaxRescore];
  {
    double acc[2 * NS];
#pragma unroll
    for (int v = 0; v < 2 * NS; ++v) acc[v] = 0.0;
    for (unsigned b = tid; b < gridDim.x; b += kThreads) {
#pragma unroll
      for (int v = 0; v < 2 * NS; ++v)
        acc[v] += ld_agent(a.part + (int64_t)b * 2 * kMaxRescore + (v < NS ? v : kMaxRescore + v - NS));
    }
#pragma unroll
    for (int v = 0; v < 2 * NS; ++v) s_all[tid][v < NS ? v : kMaxRescore + v - NS] = acc[v];
  }
  __syncthreads();
  if (tid < 2 * NS) {
    double s = 0.0;
    for (int q = 0; q < kThreads; ++q) s += s_all[q][v_me];
    if (tid < NS)
      s_mse[tid] = s / (double)a.N;
    else
      s_mis[tid - NS] = s / (double)a.N;
  }
  __syncthreads();
  if (tid < a.n) {
    if (a.mse) a.mse[tid] = s_mse[tid];
    if (a.miscls) a.miscls[tid] = s_mis[tid];
  }
  if (tid == 0) *a.counter = 0u;
  if (!a.st || a.genes) return;
  // population mode: best of the re-scored elites (lowest float32 MSE, ties
  // to the better-ranked one) becomes the tracked best; then the stop test
  __shared__ int s_b, s_improve;
  if (tid == 0) {
    int b = 0;
    for (int e = 1; e < a.n; ++e)
      if (s_mse[e] < s_mse[b]) b = e;
    s_b = b;
    s_improve = (!a.st->have_best || s_mse[b] < a.st->best_mse) ? 1 : 0;
  }
  __syncthreads();
  if (s_improve)
    for (int l = tid; l < a.L; l += kThreads) a.best[l] = g_lds[s_b * a.L + l];
  if (tid == 0) {
    DevState* st = a.st;
    st->best_index = s_rows[s_b];
    if (s_improve) {
      st->have_best = 1;
      st->best_mse = s_mse[s_b];
      st->best_fitness = 1.0 - s_mse[s_b];
      st->best_miscls = s_mis[s_b];
    }
    if (st->run_active) {
      if (st->best_mse <= st->mse_threshold) {
        st->stopped = 1;
        st->stop_reason = GAME_STOP_THRESHOLD;
      } else if (st->generation + 1 >= st->end_generation) {
        st->stopped = 1;
        st->stop_reason = GAME_STOP_MAX_GEN;
      }
    }
  }
}

constexpr int kGrid = 1024;  // workgroups of every re-score launch

// Scratch of the allocation-free entry point (game_rescore_noalloc): the
// kGrid x 2 kMaxRescore block partials, then the arrival counter (a uint32 in
// the first word of the last 256 bytes).  One copy per GPU, held until the
// process ends; every call on a GPU shares it.  The partials are written in
// full by each launch before they are read; the counter is zero when the code
// object is loaded, is cleared once more by a small kernel at the first call
// on each device, and every launch returns it to zero.
constexpr size_t kScratchPartDoubles = (size_t)kGrid * 2 * kMaxRescore;
static __device__ __align__(256) double scratch[kScratchPartDoubles + 32];

__global__ void clear_counter_kernel(uint32_t* counter) { *counter = 0u; }

}  // namespace

int rescore_grid() { return kGrid; }

size_t rescore_scratch_bytes() { return sizeof(double) * (kScratchPartDoubles + 32); }

hipError_t rescore_scratch(hipStream_t s, double** part, uint32_t** counter) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  static std::mutex mu;
  static std::vector<double*> ptrs;  // per device: the array's device address
  std::lock_guard<std::mutex> lock(mu);
  if (dev < 0) return hipErrorInvalidDevice;
  if ((size_t)dev >= ptrs.size()) ptrs.resize((size_t)dev + 1, nullptr);
  if (!ptrs[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    hipLaunchKernelGGL(clear_counter_kernel, dim3(1), dim3(1), 0, s,
                       reinterpret_cast<uint32_t*>(static_cast<double*>(p) + kScratchPartDoubles));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    ptrs[dev] = static_cast<double*>(p);
  }
  *part = ptrs[dev];
  *counter = reinterpret_cast<uint32_t*>(ptrs[dev] + kScratchPartDoubles);
  return hipSuccess;
}

hipError_t launch_rescore(const float* X, const float* t, int64_t N, int F, int D, int K, int basis,
                          int M, int L, int bias, int task, const float* genes, int n,
                          const float* pop0, const float* pop1, const int* top, double* part,
                          uint32_t* counter, double* mse, double* miscls, const DevState* sel,
                          DevState* st, float* best, hipStream_t s) {
  RescoreArgs a{X, t, N, F, D, K, basis, M, L, bias, task, genes, n, pop0, pop1, top,
                part, counter, mse, miscls, sel, st, best};
  if (!genes && !sel) return hipErrorInvalidValue;
  if (n < 1 || n > kMaxRescore) return hipErrorInvalidValue;
  const size_t lds = (size_t)n * L * sizeof(float);
  if (lds > 65536) return hipErrorInvalidValue;
  switch (n) {
#define GAME_RESCORE_N(NS)                                                                   \
  case NS:                                                                                   \
    hipLaunchKernelGGL(rescore_kernel<NS>, dim3(rescore_grid()), dim3(kThreads), lds, s, a); \
    break;
    GAME_RESCORE_N(1)
    GAME_RESCORE_N(2)
    GAME_RESCORE_N(3)
    GAME_RESCORE_N(4)
    GAME_RESCORE_N(5)
    GAME_RESCORE_N(6)
    GAME_RESCORE_N(7)
    GAME_RESCORE_N(8)
#undef GAME_RESCORE_N
  }
  return hipGetLastError();
}

}  // namespace game
