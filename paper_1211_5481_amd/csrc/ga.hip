// Kernels of the genetic operators (Sec. 3 operator list, Sec. 5 rates): the
// random initial population, the per-generation breed launch, the roulette
// wheel and full ranking for the wheel selections, and the small kernels that
// move genes between the population and the tiles the fitness kernel reads.
// The operators themselves, and the Philox counter layout of every random
// decision, are in breed.hpp.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "breed.hpp"
#include "game_internal.hpp"
#include "select.hpp"

// Every float operation in this file is rounded on its own: a fused
// multiply-add would change the mutated genes.
#pragma clang fp contract(off)

namespace game {
namespace {

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
constexpr int kRankThreads = 1024;

__global__ __launch_bounds__(kRankThreads) void rank_kernel(const double* __restrict__ fit, int P,
                                                            int n_top, int* __restrict__ top) {
  block_topk<kRankThreads>(fit, P, n_top, top);
}

// --------------------------------------------------------------- breed
// One launch per generation: one wave per elite or child pair (breed_work in
// breed.hpp); the last workgroup advances the generation counter.
template <typename O, typename B>
__global__ __launch_bounds__(256) void breed_kernel(BreedArgs a, DevState* st) {
  breed_block<O, B>(a, st, (int)blockIdx.x, (int)gridDim.x);
}

__global__ void pop_copy_kernel(float* __restrict__ pop0, float* __restrict__ pop1,
                                const DevState* __restrict__ st, float* __restrict__ ext,
                                int64_t n, int dir) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float* cur = (st->generation & 1) ? pop1 : pop0;
  if (dir == 0)
    ext[i] = cur[i];
  else
    cur[i] = ext[i];
}

// --------------------------------------------------------------- pack
template <typename O, typename B>
__global__ void pack_kernel(const float* __restrict__ genes0, const float* __restrict__ genes1,
                            const DevState* sel, int P, int L, int M, int bias, int M_pad,
                            int P_pad, O* __restrict__ tile, B* __restrict__ biasv) {
  const float* genes = (sel && (sel->generation & 1)) ? genes1 : genes0;
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

__global__ void zero_counters_kernel(uint32_t* c, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = 0u;
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

// The per-generation inputs of the roulette and ranking selections, one
// workgroup of 1024 threads (wheel_block / rank_block in breed.hpp).
__global__ __launch_bounds__(1024) void wheel_kernel(const double* __restrict__ fit, int P,
                                                     uint64_t* __restrict__ wheel, const DevState* st) {
  if (run_halted(st)) return;
  wheel_block<1024, false>(fit, P, wheel);
}

__global__ __launch_bounds__(1024) void rank_all_kernel(const double* __restrict__ fit, int P, int n_pow2,
                                                        int* __restrict__ order, const DevState* st) {
  if (run_halted(st)) return;
  extern __shared__ __align__(16) unsigned char smem[];
  rank_block<1024, false>(fit, P, n_pow2, order, smem);
}

}  // namespace

hipError_t select_prepare(int sel) {
  static bool prepared = false;
  if (sel != GAME_SEL_RANKING || prepared) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(rank_all_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 98304);
  if (e == hipSuccess) prepared = true;
  return e;
}

hipError_t launch_select_prep(int sel, const double* fit, int P, uint64_t* wheel, int* order,
                              const DevState* st, hipStream_t s) {
  if (sel == GAME_SEL_ROULETTE) {
    hipLaunchKernelGGL(wheel_kernel, dim3(1), dim3(1024), 0, s, fit, P, wheel, st);
    return hipGetLastError();
  }
  if (sel == GAME_SEL_RANKING) {
    const hipError_t e = select_prepare(sel);
    if (e != hipSuccess) return e;
    int n = 1;
    while (n < P) n <<= 1;
    if ((size_t)n * 12 > 98304) return hipErrorInvalidValue;
    hipLaunchKernelGGL(rank_all_kernel, dim3(1), dim3(1024), (size_t)n * 12, s, fit, P, n, order, st);
    return hipGetLastError();
  }
  return hipSuccess;
}

hipError_t launch_init_population(float* pop, int P, int L, uint64_t seed, hipStream_t s) {
  const int64_t n = (int64_t)P * L;
  hipLaunchKernelGGL(init_population_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     pop, P, L, seed);
  return hipGetLastError();
}

hipError_t launch_rank(const double* fit, int P, int n_top, int* top_idx, const DevState* st,
                       hipStream_t s) {
  (void)st;
  hipLaunchKernelGGL(rank_kernel, dim3(1), dim3(kRankThreads), 0, s, fit, P, n_top, top_idx);
  return hipGetLastError();
}

hipError_t launch_breed(int dtype, const BreedArgs& a, DevState* st, hipStream_t s) {
  const dim3 grid((unsigned)breed_blocks(a)), block(256);
  switch (dtype) {
    case GAME_F64:
      hipLaunchKernelGGL((breed_kernel<double, double>), grid, block, 0, s, a, st);
      break;
    case GAME_F32:
      hipLaunchKernelGGL((breed_kernel<float, float>), grid, block, 0, s, a, st);
      break;
    case GAME_BF16:
      hipLaunchKernelGGL((breed_kernel<uint16_t, float>), grid, block, 0, s, a, st);
      break;
    case GAME_F16:
      hipLaunchKernelGGL((breed_kernel<_Float16, float>), grid, block, 0, s, a, st);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int breed_blocks(const BreedArgs& a) {
  const int waves = a.E + (a.n_children + 1) / 2;
  return (waves + 3) / 4 > 0 ? (waves + 3) / 4 : 1;
}

hipError_t launch_pop_copy(float* pop0, float* pop1, const DevState* st, float* ext, int64_t n,
                           int dir, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(pop_copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pop0,
                     pop1, st, ext, n, dir);
  return hipGetLastError();
}

hipError_t launch_pack(int dtype, const float* genes0, const float* genes1, const DevState* sel,
                       int P, int L, int M, int bias, int M_pad, int P_pad, void* tile, void* biasv,
                       hipStream_t s) {
  const int64_t total = (int64_t)P_pad * M_pad;
  const dim3 grid((unsigned)((total + 255) / 256)), block(256);
  switch (dtype) {
    case GAME_F64:
      hipLaunchKernelGGL((pack_kernel<double, double>), grid, block, 0, s, genes0, genes1, sel, P,
                         L, M, bias, M_pad, P_pad, (double*)tile, (double*)biasv);
      break;
    case GAME_F32:
      hipLaunchKernelGGL((pack_kernel<float, float>), grid, block, 0, s, genes0, genes1, sel, P, L,
                         M, bias, M_pad, P_pad, (float*)tile, (float*)biasv);
      break;
    case GAME_BF16:
      hipLaunchKernelGGL((pack_kernel<uint16_t, float>), grid, block, 0, s, genes0, genes1, sel, P,
                         L, M, bias, M_pad, P_pad, (uint16_t*)tile, (float*)biasv);
      break;
    case GAME_F16:
      hipLaunchKernelGGL((pack_kernel<_Float16, float>), grid, block, 0, s, genes0, genes1, sel, P,
                         L, M, bias, M_pad, P_pad, (_Float16*)tile, (float*)biasv);
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

hipError_t launch_state_init(DevState* st, uint32_t* counters, int n_counters, hipStream_t s) {
  hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(1), 0, s, st);
  hipLaunchKernelGGL(zero_counters_kernel, dim3((unsigned)((n_counters + 255) / 256)), dim3(256), 0,
                     s, counters, n_counters);
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
