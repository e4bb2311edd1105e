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
#include "select.hpp"

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
constexpr int kRankThreads = 1024;

__global__ __launch_bounds__(kRankThreads) void rank_kernel(const double* __restrict__ fit, int P,
                                                            int n_top, int* __restrict__ top) {
  block_topk<kRankThreads>(fit, P, n_top, top);
}

// --------------------------------------------------------------- breed
// One wave per output row group: waves 0..E-1 copy the elites, wave E + j
// builds the children of pair j (tournaments, crossover, mutation).  Each
// new gene goes to the next population buffer (float32 master) and, rounded
// to the contraction type, to the gene tile the fitness kernel reads next.
// The last workgroup to finish advances the generation counter.

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

// Both tournaments of pair j with every candidate's fitness load in flight
// at once (the loop above waits for each load before drawing the next), for
// k <= kTourMax; the same candidates, compared in the same order.
constexpr int kTourMax = 8;
__device__ __forceinline__ void tournament_pair(const BreedArgs& a, uint32_t j, uint32_t g, int* pa,
                                                int* pb) {
  int cand[2][kTourMax];
  double key[2][kTourMax];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int q = 0; q < kTourMax / 4; ++q) {
      if (4 * q >= a.k) continue;
      const u32x4 blk = philox(j, 4u * (uint32_t)s + (uint32_t)q, g, kTagSel, a.k0, a.k1);
#pragma unroll
      for (int w = 0; w < 4; ++w) cand[s][4 * q + w] = (int)__umulhi(word_of(blk, w), (uint32_t)a.P);
    }
  }
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int i = 0; i < kTourMax; ++i)
      if (i < a.k) key[s][i] = a.fit[cand[s][i]];
  int out[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    Ranked win{0.0, -1};
#pragma unroll
    for (int i = 0; i < kTourMax; ++i) {
      if (i >= a.k) continue;
      const Ranked c{rank_key(key[s][i]), cand[s][i]};
      if (win.idx < 0 || better(c, win)) win = c;
    }
    out[s] = win.idx;
  }
  *pa = out[0];
  *pb = out[1];
}

// Parent s of pair j: a tournament, or a 64-bit draw r from block
// (j, s, g, ROULETTE) (word 1 high, word 0 low) scaled to the wheel's integer
// total, t = floor(r T / 2^64), and the first slot whose cumulative weight
// exceeds t.  Rank wheel: rank q (0 = best) weighs P - q, so its cumulative
// weight is (q + 1) P - q (q + 1) / 2 and T = P (P + 1) / 2.
__device__ __forceinline__ int select_parent(const BreedArgs& a, uint32_t j, uint32_t s, uint32_t g) {
  if (a.sel == GAME_SEL_TOURNAMENT) return tournament(a, j, s, g);
  const u32x4 b = philox(j, s, g, kTagRoulette, a.k0, a.k1);
  const uint64_t r = ((uint64_t)b.y << 32) | (uint64_t)b.x;
  int lo = 0, hi = a.P - 1;
  if (a.sel == GAME_SEL_ROULETTE) {
    const uint64_t t = __umul64hi(r, a.wheel[a.P - 1]);
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (a.wheel[mid] > t) hi = mid;
      else lo = mid + 1;
    }
    return lo;
  }
  const uint64_t P = (uint64_t)a.P;
  const uint64_t t = __umul64hi(r, P * (P + 1) / 2);
  while (lo < hi) {
    const uint64_t mid = (uint64_t)((lo + hi) >> 1);
    if ((mid + 1) * P - mid * (mid + 1) / 2 > t) hi = (int)mid;
    else lo = (int)mid + 1;
  }
  return a.order[lo];
}

// Random immigrant gene: as at init, from block (c, l, g, IMMIGRANT) word 0.
__device__ __forceinline__ float immigrant_gene(uint32_t c, uint32_t l, uint32_t g, const BreedArgs& a) {
  const uint32_t w = philox(c, l, g, kTagImmigrant, a.k0, a.k1).x;
  return (float)(w >> 8) * 0x1p-23f - 1.0f;
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

template <typename O, typename B>
__device__ __forceinline__ void put_gene(const BreedArgs& a, float* dst, int row, int l, float v) {
  dst[(int64_t)row * a.L + l] = v;
  if (!a.tile) return;
  if (l < a.M)
    static_cast<O*>(a.tile)[(int64_t)row * a.M_pad + l] = cvt_gene<O>(v);
  else
    static_cast<B*>(a.biasv)[row] = (B)v;
}

// Workgroup `blk` of the n_blocks a context's breed takes (4 waves each: the
// first E waves copy elites, then one wave per child pair).  The last of them
// to finish advances the context's generation and, when t_done is given,
// stamps the time in slot generation - t_gen0.
template <typename O, typename B>
__device__ __forceinline__ void breed_block(const BreedArgs& a, DevState* st, int blk, int n_blocks,
                                            uint64_t* t_done, int t_cap, int t_gen0) {
  if (run_halted(st)) return;
  const int wave = (int)(((unsigned)blk * 256u + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const uint32_t g = (uint32_t)st->generation;
  const float* src = (g & 1u) ? a.pop1 : a.pop0;
  float* dst = a.out ? a.out : ((g & 1u) ? a.pop0 : a.pop1);
  if (wave < a.E) {
    const float* row = src + (int64_t)a.elite[wave] * a.L;
    for (int l = lane; l < a.L; l += 64) put_gene<O, B>(a, dst, wave, l, row[l]);
  } else if (2 * (wave - a.E) < a.n_children) {
    const int j = wave - a.E;
    int pa, pb;
    if (a.sel == GAME_SEL_TOURNAMENT && a.k <= kTourMax) {
      tournament_pair(a, (uint32_t)j, g, &pa, &pb);
    } else {
      pa = select_parent(a, (uint32_t)j, 0u, g);
      pb = select_parent(a, (uint32_t)j, 1u, g);
    }
    const u32x4 xb = philox((uint32_t)j, 8u, g, kTagSel, a.k0, a.k1);
    int cut = a.L;  // no crossover: child0 = a, child1 = b
    if ((uint64_t)xb.x < a.thr_c && a.L >= 2) cut = 1 + (int)__umulhi(xb.y, (uint32_t)(a.L - 1));
    const float* __restrict__ ra = src + (int64_t)pa * a.L;
    const float* __restrict__ rb = src + (int64_t)pb * a.L;
    const uint32_t c0 = 2u * (uint32_t)j, c1 = c0 + 1u;
    const bool has1 = (int)c1 < a.n_children;
    const int first_imm = a.n_children - a.n_imm;  // children from here on are immigrants
    const bool imm0 = (int)c0 >= first_imm, imm1 = (int)c1 >= first_imm;
    auto child_genes = [&](int l, float ga, float gb) {
      const float x0 = l < cut ? ga : gb;
      const float x1 = l < cut ? gb : ga;
      const uint32_t ul = (uint32_t)l;
      put_gene<O, B>(a, dst, a.E + (int)c0, l,
                     imm0 ? immigrant_gene(c0, ul, g, a) : mutate_gene(x0, c0, ul, g, a));
      if (has1)
        put_gene<O, B>(a, dst, a.E + (int)c1, l,
                       imm1 ? immigrant_gene(c1, ul, g, a) : mutate_gene(x1, c1, ul, g, a));
    };
    // two strides of parent genes loaded before the first child gene is stored
    for (int l = lane; l < a.L; l += 128) {
      const bool two = l + 64 < a.L;
      const float ga = ra[l], gb = rb[l];
      const float ga2 = two ? ra[l + 64] : 0.0f, gb2 = two ? rb[l + 64] : 0.0f;
      child_genes(l, ga, gb);
      if (two) child_genes(l + 64, ga2, gb2);
    }
  }
  // The last workgroup to arrive advances the generation.  The barrier waits
  // for this workgroup's loads (its read of the generation included) before
  // the arrival; the new genes are read only by later launches.
  if (!a.counter) return;
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0) s_last = atomicAdd(a.counter, 1u) == (uint32_t)(n_blocks - 1);
  __syncthreads();
  if (s_last && threadIdx.x == 0) {
    if (t_done) {
      const int rel = (int)g - t_gen0;
      if (rel >= 0 && rel < t_cap) t_done[rel] = (uint64_t)wall_clock64();
    }
    st->generation += 1;
    *a.counter = 0u;
  }
}

template <typename O, typename B>
__global__ __launch_bounds__(256) void breed_kernel(BreedArgs a, DevState* st) {
  breed_block<O, B>(a, st, (int)blockIdx.x, (int)gridDim.x, nullptr, 0, 0);
}

// Batched form: workgroup b serves the context whose range of workgroups
// holds b; the last workgroup of the launch advances the batch generation.
template <typename O, typename B>
__global__ __launch_bounds__(256) void breed_batch_kernel(const BatchBreedRun* __restrict__ runs,
                                                          int n_runs, BatchQueue* q, int t_cap) {
  const int b = (int)blockIdx.x;
  int lo = 0, hi = n_runs - 1;  // last context whose first workgroup is <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (runs[mid].block0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const BatchBreedRun& r = runs[lo];
  breed_block<O, B>(r.a, r.st, b - r.block0, r.n_blocks, r.t_done, t_cap, r.gen0);
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0) s_last = atomicAdd(&q->bred, 1u) == gridDim.x - 1;
  __syncthreads();
  if (s_last && threadIdx.x == 0) {
    q->gen += 1;
    q->bred = 0u;
  }
}

// After a chunk of batched generations: count the contexts still running;
// with arm set, also note the starting generations for the timestamps.
__global__ void batch_status_kernel(DevState* const* __restrict__ states, BatchBreedRun* runs,
                                    int n_runs, BatchQueue* q, int arm) {
  __shared__ int s_active[256];
  int act = 0;
  for (int i = threadIdx.x; i < n_runs; i += 256) {
    const DevState* st = states[i];
    act += run_halted(st) ? 0 : 1;
    if (arm) runs[i].gen0 = st->generation;
  }
  s_active[threadIdx.x] = act;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int i = 0; i < 256; ++i) tot += s_active[i];
    q->active = tot;
    if (arm) q->base = q->gen;
  }
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

// Roulette wheel of fit[0..P): integer weights (see select_parent) and their
// inclusive prefix sums, one workgroup.  Integer sums are exact, so the wheel
// does not depend on the order of the additions.
__global__ __launch_bounds__(1024) void wheel_kernel(const double* __restrict__ fit, int P,
                                                     uint64_t* __restrict__ wheel, const DevState* st) {
  if (run_halted(st)) return;
  __shared__ double s_lo[16], s_hi[16];
  __shared__ uint64_t s_scan[1024];
  __shared__ uint64_t s_carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double mn = INFINITY, mx = -INFINITY;
  for (int i = tid; i < P; i += 1024) {
    const double f = fit[i];
    if (!isnan(f)) {
      mn = fmin(mn, f);
      mx = fmax(mx, f);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, off));
    mx = fmax(mx, __shfl_xor(mx, off));
  }
  if (lane == 0) {
    s_lo[wave] = mn;
    s_hi[wave] = mx;
  }
  if (tid == 0) s_carry = 0;
  __syncthreads();
  double lo = s_lo[0], hi = s_hi[0];
  for (int w = 1; w < 16; ++w) {
    lo = fmin(lo, s_lo[w]);
    hi = fmax(hi, s_hi[w]);
  }
  const bool any = lo <= hi;  // some finite fitness
  const double span = hi - lo;
  for (int base = 0; base < P; base += 1024) {
    const int i = base + tid;
    uint64_t w = 0;
    if (i < P) {
      const double f = fit[i];
      if (!any) w = 1;
      else if (isnan(f)) w = 0;
      else if (!(hi > lo)) w = 1;
      else w = (uint64_t)floor((f - lo) / span * 4294967296.0);
    }
    s_scan[tid] = w;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan (Hillis-Steele)
      const uint64_t add = tid >= off ? s_scan[tid - off] : 0;
      __syncthreads();
      s_scan[tid] += add;
      __syncthreads();
    }
    if (i < P) wheel[i] = s_carry + s_scan[tid];
    __syncthreads();
    if (tid == 0) s_carry += s_scan[1023];
    __syncthreads();
  }
}

// Full ranking of fit[0..P) (fitness descending, index ascending, NaN last)
// by a bitonic sort in LDS, one workgroup; order[q] = chromosome of rank q.
__global__ __launch_bounds__(1024) void rank_all_kernel(const double* __restrict__ fit, int P, int n_pow2,
                                                        int* __restrict__ order, const DevState* st) {
  if (run_halted(st)) return;
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* sk = reinterpret_cast<uint64_t*>(smem);
  int* si = reinterpret_cast<int*>(smem + (size_t)n_pow2 * 8);
  for (int i = threadIdx.x; i < n_pow2; i += 1024) {
    sk[i] = i < P ? ord_desc_f64(fit[i]) : ~0ull;
    si[i] = i < P ? i : 0x7fffffff;
  }
  __syncthreads();
  block_sort_pairs<1024>(sk, si, n_pow2);
  for (int q = threadIdx.x; q < P; q += 1024) order[q] = si[q];
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

hipError_t launch_breed_batch(int dtype, const BatchBreedRun* runs, int n_runs, int n_blocks,
                              BatchQueue* q, int t_cap, hipStream_t s) {
  const dim3 grid((unsigned)n_blocks), block(256);
  switch (dtype) {
    case GAME_F32:
      hipLaunchKernelGGL((breed_batch_kernel<float, float>), grid, block, 0, s, runs, n_runs, q, t_cap);
      break;
    case GAME_BF16:
      hipLaunchKernelGGL((breed_batch_kernel<uint16_t, float>), grid, block, 0, s, runs, n_runs, q, t_cap);
      break;
    case GAME_F16:
      hipLaunchKernelGGL((breed_batch_kernel<_Float16, float>), grid, block, 0, s, runs, n_runs, q, t_cap);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_status(DevState* const* states, BatchBreedRun* runs, int n_runs, BatchQueue* q,
                               int arm, hipStream_t s) {
  hipLaunchKernelGGL(batch_status_kernel, dim3(1), dim3(256), 0, s, states, runs, n_runs, q, arm);
  return hipGetLastError();
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
