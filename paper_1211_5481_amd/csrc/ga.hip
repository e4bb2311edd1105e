// Genetic operators on the device (Sec. 3 operator list, Sec. 5 rates), and
// the small kernels that move genes between the population and the tiles the
// fitness kernel reads.
//
// Every random decision comes from one Philox4x32-10 block addressed by a
// counter (a, b, generation, tag) under key = seed:
//   init      gene (p, l):              (p, l, 0, INIT) word 0
//   selection pair j, parent s, draw i: (j, 4 s + i / 4, g, SEL) word i % 4
//   crossover pair j:                   (j, 8, g, SEL) words 0 (decision), 1 (cut)
//   mutation  child c, gene l:          (c, l, g, MUT) word 0 (decision), Gaussian
//             from (c,l,g,MUT) words 1..3, MUT1 words 0..3, MUT2 words 0..3,
//             MUT3 word 0
// Decisions compare a word with floor(p * 2^32); indices are
// floor(word * n / 2^32).  The mutation step is float32 with every operation
// rounded separately (no fused multiply-add), so the result depends only on
// the counter values and the input genes, not on the launch shape.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "game_internal.hpp"

// Every float operation in this file is rounded on its own: a fused
// multiply-add would change the mutated genes.
#pragma clang fp contract(off)

namespace game {
namespace {

__device__ __forceinline__ uint32_t key_lo(uint64_t seed) { return (uint32_t)seed; }
__device__ __forceinline__ uint32_t key_hi(uint64_t seed) { return (uint32_t)(seed >> 32); }

// ---------------------------------------------------------------- init
__global__ void init_population_kernel(float* __restrict__ pop, int P, int L, uint64_t seed) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)P * L) return;
  const uint32_t p = (uint32_t)(idx / L), l = (uint32_t)(idx % L);
  const u32x4 b = philox(p, l, 0u, kTagInit, key_lo(seed), key_hi(seed));
  const float u = (float)(b.x >> 8);  // exact: 24-bit integer
  pop[idx] = u * 0x1p-23f - 1.0f;
}

// ------------------------------------------------------------ ranking
// Order: higher fitness first, ties to the lower index, NaN ranks last.
struct Ranked {
  double key;
  int idx;
};
__device__ __forceinline__ bool better(const Ranked& a, const Ranked& b) {
  return a.key > b.key || (a.key == b.key && a.idx < b.idx);
}
__device__ __forceinline__ double rank_key(double f) { return isnan(f) ? -INFINITY : f; }

constexpr int kRankThreads = 1024;

// Top n_top indices by repeated arg-max (n_top <= kMaxElite); one workgroup.
__global__ __launch_bounds__(kRankThreads) void rank_kernel(const double* __restrict__ fit, int P,
                                                            int n_top, int* __restrict__ top,
                                                            const DevState* st) {
  if (run_halted(st)) return;
  __shared__ int chosen[kMaxElite];
  __shared__ double wkey[kRankThreads / 64];
  __shared__ int widx[kRankThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = 0; e < n_top; ++e) {
    Ranked best{-INFINITY, 0x7fffffff};
    for (int i = tid; i < P; i += kRankThreads) {
      bool taken = false;
      for (int q = 0; q < e; ++q) taken |= (chosen[q] == i);
      if (taken) continue;
      const Ranked c{rank_key(fit[i]), i};
      if (better(c, best)) best = c;
    }
    for (int off = 32; off > 0; off >>= 1) {
      Ranked o{__shfl_xor(best.key, off), __shfl_xor(best.idx, off)};
      if (better(o, best)) best = o;
    }
    if (lane == 0) {
      wkey[wave] = best.key;
      widx[wave] = best.idx;
    }
    __syncthreads();
    if (tid == 0) {
      Ranked b{wkey[0], widx[0]};
      for (int q = 1; q < kRankThreads / 64; ++q) {
        const Ranked o{wkey[q], widx[q]};
        if (better(o, b)) b = o;
      }
      chosen[e] = b.idx;
      top[e] = b.idx;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------- best tracking
// Keeps the best chromosome seen (strictly lower MSE replaces it) and, while
// a run is active, decides whether the run stops after this generation.
__global__ void track_kernel(DevState* st, const int* __restrict__ top,
                             const double* __restrict__ mse, const double* __restrict__ miscls,
                             const float* __restrict__ pop, int L, float* __restrict__ best) {
  if (run_halted(st)) return;
  const int b = top[0];
  const double m = mse[b];
  const bool improve = !st->have_best || m < st->best_mse;
  __syncthreads();
  if (improve)
    for (int l = threadIdx.x; l < L; l += blockDim.x) best[l] = pop[(int64_t)b * L + l];
  __syncthreads();
  if (threadIdx.x == 0) {
    st->best_index = b;
    if (improve) {
      st->have_best = 1;
      st->best_mse = m;
      st->best_fitness = 1.0 - m;
      st->best_miscls = miscls[b];
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

// --------------------------------------------------------------- breed
// One wave per output slot group: waves 0..E-1 copy the elites, wave E + j
// builds the children of pair j (tournaments, crossover, mutation).
struct BreedArgs {
  const float* pop;
  const double* fit;
  const int* elite;
  float* next;
  int P, L, E, n_children, k;
  uint64_t thr_c, thr_m;
  float sigma;
  uint32_t k0, k1;
};

__device__ __forceinline__ int tournament(const BreedArgs& a, uint32_t j, uint32_t s, uint32_t g) {
  Ranked win{0.0, -1};
  u32x4 blk{0, 0, 0, 0};
  for (int i = 0; i < a.k; ++i) {
    if ((i & 3) == 0) blk = philox(j, 4u * s + (uint32_t)(i >> 2), g, kTagSel, a.k0, a.k1);
    const int cand = (int)__umulhi(word_of(blk, i & 3), (uint32_t)a.P);
    const Ranked c{rank_key(a.fit[cand]), cand};
    if (win.idx < 0 || better(c, win)) win = c;
  }
  return win.idx;
}

__device__ __forceinline__ float mutate_gene(float gene, uint32_t c, uint32_t l, uint32_t g,
                                             const BreedArgs& a) {
  const u32x4 b0 = philox(c, l, g, kTagMut, a.k0, a.k1);
  if ((uint64_t)b0.x >= a.thr_m) return gene;
  const u32x4 b1 = philox(c, l, g, kTagMut1, a.k0, a.k1);
  const u32x4 b2 = philox(c, l, g, kTagMut2, a.k0, a.k1);
  const u32x4 b3 = philox(c, l, g, kTagMut3, a.k0, a.k1);
  const uint32_t w[12] = {b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w, b2.x, b2.y, b2.z, b2.w, b3.x};
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < 12; ++i) s += (int32_t)(2u * (w[i] >> 8) + 1u);
  s -= 12 * (1 << 24);
  const float z = (float)s * 0x1p-25f;
  const float delta = a.sigma * z;
  const float v = gene + delta;
  return fminf(fmaxf(v, -1.0f), 1.0f);
}

__global__ __launch_bounds__(256) void breed_kernel(BreedArgs a, const DevState* st) {
  if (run_halted(st)) return;
  const int wave = (int)((blockIdx.x * 256u + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const uint32_t g = (uint32_t)st->generation;
  if (wave < a.E) {
    const float* src = a.pop + (int64_t)a.elite[wave] * a.L;
    float* dst = a.next + (int64_t)wave * a.L;
    for (int l = lane; l < a.L; l += 64) dst[l] = src[l];
    return;
  }
  const int j = wave - a.E;
  if (2 * j >= a.n_children) return;
  const int pa = tournament(a, (uint32_t)j, 0u, g);
  const int pb = tournament(a, (uint32_t)j, 1u, g);
  const u32x4 xb = philox((uint32_t)j, 8u, g, kTagSel, a.k0, a.k1);
  int cut = a.L;  // no crossover: child0 = a, child1 = b
  if ((uint64_t)xb.x < a.thr_c && a.L >= 2) cut = 1 + (int)__umulhi(xb.y, (uint32_t)(a.L - 1));
  const float* ra = a.pop + (int64_t)pa * a.L;
  const float* rb = a.pop + (int64_t)pb * a.L;
  const uint32_t c0 = 2u * (uint32_t)j, c1 = c0 + 1u;
  const bool has1 = (int)c1 < a.n_children;
  float* d0 = a.next + (int64_t)(a.E + (int)c0) * a.L;
  float* d1 = a.next + (int64_t)(a.E + (int)c1) * a.L;
  for (int l = lane; l < a.L; l += 64) {
    const float ga = ra[l], gb = rb[l];
    const float x0 = l < cut ? ga : gb;
    const float x1 = l < cut ? gb : ga;
    d0[l] = mutate_gene(x0, c0, (uint32_t)l, g, a);
    if (has1) d1[l] = mutate_gene(x1, c1, (uint32_t)l, g, a);
  }
}

// ------------------------------------------------------------- commit
__global__ void commit_kernel(const float4* __restrict__ next, float4* __restrict__ pop,
                              int64_t n4, const float* __restrict__ next_s,
                              float* __restrict__ pop_s, int64_t count, DevState* st) {
  if (run_halted(st)) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n4) pop[i] = next[i];
  const int64_t tail = n4 * 4 + i;
  if (i < 4 && tail < count) pop_s[tail] = next_s[tail];
  if (i == 0) st->generation += 1;
}

// --------------------------------------------------------------- pack
template <typename O>
__device__ __forceinline__ O cvt_gene(float g);
template <>
__device__ __forceinline__ double cvt_gene<double>(float g) {
  return (double)g;
}
template <>
__device__ __forceinline__ float cvt_gene<float>(float g) {
  return g;
}
template <>
__device__ __forceinline__ _Float16 cvt_gene<_Float16>(float g) {
  return (_Float16)g;
}
template <>
__device__ __forceinline__ uint16_t cvt_gene<uint16_t>(float g) {  // bf16, nearest even
  const uint32_t u = __float_as_uint(g);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

template <typename O, typename B>
__global__ void pack_kernel(const float* __restrict__ genes, int P, int L, int M, int bias,
                            int M_pad, int P_pad, O* __restrict__ tile, B* __restrict__ biasv,
                            const DevState* st) {
  if (run_halted(st)) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)P_pad * M_pad;
  if (idx < total) {
    const int p = (int)(idx / M_pad), m = (int)(idx % M_pad);
    tile[idx] = (p < P && m < M) ? cvt_gene<O>(genes[(int64_t)p * L + m]) : cvt_gene<O>(0.0f);
  }
  if (idx < P_pad) biasv[idx] = (bias && idx < P) ? (B)genes[idx * L + M] : (B)0;
}

template <typename T>
__global__ void copy_targets_kernel(const T* __restrict__ t, int64_t N, int64_t N_pad,
                                    T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N_pad) out[i] = i < N ? t[i] : (T)0;
}

__global__ void state_init_kernel(DevState* st) {
  st->generation = 0;
  st->stopped = 0;
  st->best_index = 0;
  st->stop_reason = GAME_STOP_NONE;
  st->run_active = 0;
  st->end_generation = 0;
  st->have_best = 0;
  st->pad = 0;
  st->best_mse = INFINITY;
  st->best_fitness = -INFINITY;
  st->best_miscls = 0.0;
  st->mse_threshold = -INFINITY;
}

__global__ void run_arm_kernel(DevState* st, int max_generations, double threshold) {
  st->run_active = 1;
  st->stopped = 0;
  st->stop_reason = GAME_STOP_NONE;
  st->end_generation = st->generation + max_generations;
  st->mse_threshold = threshold;
}

__global__ void run_disarm_kernel(DevState* st) { st->run_active = 0; }

}  // namespace

hipError_t launch_init_population(float* pop, int P, int L, uint64_t seed, hipStream_t s) {
  const int64_t n = (int64_t)P * L;
  hipLaunchKernelGGL(init_population_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     pop, P, L, seed);
  return hipGetLastError();
}

hipError_t launch_rank(const double* fit, int P, int n_top, int* top_idx, const DevState* st,
                       hipStream_t s) {
  hipLaunchKernelGGL(rank_kernel, dim3(1), dim3(kRankThreads), 0, s, fit, P, n_top, top_idx, st);
  return hipGetLastError();
}

hipError_t launch_track(DevState* st, const int* top_idx, const double* mse, const double* miscls,
                        const float* pop, int L, float* best_genes, hipStream_t s) {
  hipLaunchKernelGGL(track_kernel, dim3(1), dim3(256), 0, s, st, top_idx, mse, miscls, pop, L,
                     best_genes);
  return hipGetLastError();
}

hipError_t launch_breed(const float* pop, const double* fit, const int* elite_idx, float* next,
                        int P, int L, int E, int n_children, int k, uint64_t thr_c,
                        uint64_t thr_m, float sigma, uint64_t seed, const DevState* st,
                        hipStream_t s) {
  BreedArgs a{pop, fit, elite_idx, next, P, L, E, n_children, k, thr_c, thr_m, sigma,
              (uint32_t)seed, (uint32_t)(seed >> 32)};
  const int waves = E + (n_children + 1) / 2;
  if (waves == 0) return hipSuccess;
  hipLaunchKernelGGL(breed_kernel, dim3((waves + 3) / 4), dim3(256), 0, s, a, st);
  return hipGetLastError();
}

hipError_t launch_commit(const float* next, float* pop, int64_t count, DevState* st,
                         hipStream_t s) {
  const int64_t n4 = count / 4;
  const int64_t threads = n4 > 4 ? n4 : 4;
  hipLaunchKernelGGL(commit_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(next), reinterpret_cast<float4*>(pop), n4,
                     next, pop, count, st);
  return hipGetLastError();
}

hipError_t launch_pack(int dtype, const float* genes, int P, int L, int M, int bias, int M_pad,
                       int P_pad, void* tile, void* biasv, const DevState* st, hipStream_t s) {
  const int64_t total = (int64_t)P_pad * M_pad;
  const dim3 grid((unsigned)((total + 255) / 256)), block(256);
  switch (dtype) {
    case GAME_F64:
      hipLaunchKernelGGL((pack_kernel<double, double>), grid, block, 0, s, genes, P, L, M, bias,
                         M_pad, P_pad, (double*)tile, (double*)biasv, st);
      break;
    case GAME_F32:
      hipLaunchKernelGGL((pack_kernel<float, float>), grid, block, 0, s, genes, P, L, M, bias,
                         M_pad, P_pad, (float*)tile, (float*)biasv, st);
      break;
    case GAME_BF16:
      hipLaunchKernelGGL((pack_kernel<uint16_t, float>), grid, block, 0, s, genes, P, L, M, bias,
                         M_pad, P_pad, (uint16_t*)tile, (float*)biasv, st);
      break;
    case GAME_F16:
      hipLaunchKernelGGL((pack_kernel<_Float16, float>), grid, block, 0, s, genes, P, L, M, bias,
                         M_pad, P_pad, (_Float16*)tile, (float*)biasv, st);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_copy_targets(int dtype, const void* t, int64_t N, int64_t N_pad, void* tvec,
                               hipStream_t s) {
  const dim3 grid((unsigned)((N_pad + 255) / 256)), block(256);
  if (dtype == GAME_F64)
    hipLaunchKernelGGL(copy_targets_kernel<double>, grid, block, 0, s, (const double*)t, N, N_pad,
                       (double*)tvec);
  else
    hipLaunchKernelGGL(copy_targets_kernel<float>, grid, block, 0, s, (const float*)t, N, N_pad,
                       (float*)tvec);
  return hipGetLastError();
}

hipError_t launch_state_init(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(1), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_run_arm(DevState* st, int max_generations, double threshold, hipStream_t s) {
  hipLaunchKernelGGL(run_arm_kernel, dim3(1), dim3(1), 0, s, st, max_generations, threshold);
  return hipGetLastError();
}

hipError_t launch_run_disarm(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(run_disarm_kernel, dim3(1), dim3(1), 0, s, st);
  return hipGetLastError();
}

}  // namespace game
