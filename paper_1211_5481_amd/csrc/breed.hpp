// Genetic operators as device functions (Sec. 3 operator list, Sec. 5
// rates): parent selection (tournament, roulette, ranking), one-point
// crossover, Gaussian mutation with clamping, random immigrants, elitism,
// and the per-generation roulette wheel and full ranking.  Used by the breed
// kernels (one launch per generation) and by the batched scheduler (every
// phase of a run inside one persistent launch); the kA template flag selects
// device-scope loads and stores for the latter.
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
// rounded separately (no fused multiply-add: the functions with floating-
// point arithmetic switch contraction off), so the result depends only on
// the counter values and the input genes, not on the launch shape.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "game_internal.hpp"
#include "select.hpp"

namespace game {
namespace {

__device__ __forceinline__ uint32_t key_lo(uint64_t seed) { return (uint32_t)seed; }
__device__ __forceinline__ uint32_t key_hi(uint64_t seed) { return (uint32_t)(seed >> 32); }

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

template <bool kA>
__device__ __forceinline__ int tournament(const BreedArgs& a, uint32_t j, uint32_t s, uint32_t g) {
  Ranked win{0.0, -1};
  u32x4 blk{0, 0, 0, 0};
  for (int i = 0; i < a.k; ++i) {
    if ((i & 3) == 0) blk = philox(j, 4u * s + (uint32_t)(i >> 2), g, kTagSel, a.k0, a.k1);
    const int cand = (int)__umulhi(word_of(blk, i & 3), (uint32_t)a.P);
    const Ranked c{rank_key(ldc<kA>(a.fit + cand)), cand};
    if (win.idx < 0 || better(c, win)) win = c;
  }
  return win.idx;
}

// Both tournaments of pair j with every candidate's fitness load in flight
// at once (the loop above waits for each load before drawing the next), for
// k <= kTourMax; the same candidates, compared in the same order.
constexpr int kTourMax = 8;
template <bool kA>
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
      if (i < a.k) key[s][i] = ldc<kA>(a.fit + cand[s][i]);
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
template <bool kA>
__device__ __forceinline__ int select_parent(const BreedArgs& a, uint32_t j, uint32_t s, uint32_t g) {
  if (a.sel == GAME_SEL_TOURNAMENT) return tournament<kA>(a, j, s, g);
  const u32x4 b = philox(j, s, g, kTagRoulette, a.k0, a.k1);
  const uint64_t r = ((uint64_t)b.y << 32) | (uint64_t)b.x;
  int lo = 0, hi = a.P - 1;
  if (a.sel == GAME_SEL_ROULETTE) {
    const uint64_t t = __umul64hi(r, ldc<kA>(a.wheel + (a.P - 1)));
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (ldc<kA>(a.wheel + mid) > t) hi = mid;
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
  return ldc<kA>(a.order + lo);
}

// Random immigrant gene: as at init, from block (c, l, g, IMMIGRANT) word 0.
__device__ __forceinline__ float immigrant_gene(uint32_t c, uint32_t l, uint32_t g, const BreedArgs& a) {
#pragma clang fp contract(off)
  const uint32_t w = philox(c, l, g, kTagImmigrant, a.k0, a.k1).x;
  return (float)(w >> 8) * 0x1p-23f - 1.0f;
}

__device__ __forceinline__ float mutate_gene(float gene, uint32_t c, uint32_t l, uint32_t g,
                                             const BreedArgs& a) {
#pragma clang fp contract(off)
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

template <typename O, typename B, bool kA>
__device__ __forceinline__ void put_gene(const BreedArgs& a, float* dst, int row, int l, float v) {
  stc<kA>(dst + (int64_t)row * a.L + l, v);
  if (!a.tile) return;
  if (l < a.M)
    stc<kA>(static_cast<O*>(a.tile) + (int64_t)row * a.M_pad + l, cvt_gene<O>(v));
  else
    stc<kA>(static_cast<B*>(a.biasv) + row, (B)v);
}

// Workgroup `blk` of the workgroups a context's breed of generation g takes
// (4 waves each: the first E waves copy elites, then one wave per child
// pair).  kA: the population, the ranking, the fitness and the wheel were
// written in the same launch by other workgroups, and the new genes are read
// there too (batched scheduler), so every access is at device scope.
template <typename O, typename B, bool kA>
__device__ __forceinline__ void breed_work(const BreedArgs& a, int blk, uint32_t g) {
  const int wave = (int)(((unsigned)blk * 256u + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const float* src = (g & 1u) ? a.pop1 : a.pop0;
  float* dst = a.out ? a.out : ((g & 1u) ? a.pop0 : a.pop1);
  if (wave < a.E) {
    const float* row = src + (int64_t)ldc<kA>(a.elite + wave) * a.L;
    for (int l = lane; l < a.L; l += 64) put_gene<O, B, kA>(a, dst, wave, l, ldc<kA>(row + l));
  } else if (2 * (wave - a.E) < a.n_children) {
    const int j = wave - a.E;
    int pa, pb;
    if (a.sel == GAME_SEL_TOURNAMENT && a.k <= kTourMax) {
      tournament_pair<kA>(a, (uint32_t)j, g, &pa, &pb);
    } else {
      pa = select_parent<kA>(a, (uint32_t)j, 0u, g);
      pb = select_parent<kA>(a, (uint32_t)j, 1u, g);
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
      put_gene<O, B, kA>(a, dst, a.E + (int)c0, l,
                     imm0 ? immigrant_gene(c0, ul, g, a) : mutate_gene(x0, c0, ul, g, a));
      if (has1)
        put_gene<O, B, kA>(a, dst, a.E + (int)c1, l,
                       imm1 ? immigrant_gene(c1, ul, g, a) : mutate_gene(x1, c1, ul, g, a));
    };
    // two strides of parent genes loaded before the first child gene is
    // stored, without a branch (the second from a clamped index when it is
    // past the row, unused): a load under a branch is waited for where the
    // paths join
    for (int l = lane; l < a.L; l += 128) {
      const bool two = l + 64 < a.L;
      const int l2 = two ? l + 64 : l;
      const float ga = ldc<kA>(ra + l), gb = ldc<kA>(rb + l);
      const float ga2 = ldc<kA>(ra + l2), gb2 = ldc<kA>(rb + l2);
      child_genes(l, ga, gb);
      if (two) child_genes(l + 64, ga2, gb2);
    }
  }
}

// One breed launch's workgroup: the work above for the context's current
// generation; the last workgroup to arrive advances the generation.  The
// barrier waits for this workgroup's loads (its read of the generation
// included) before the arrival; the new genes are read only by later
// launches.
template <typename O, typename B>
__device__ __forceinline__ void breed_block(const BreedArgs& a, DevState* st, int blk, int n_blocks) {
  if (run_halted(st)) return;
  const uint32_t g = (uint32_t)st->generation;
  breed_work<O, B, false>(a, blk, g);
  if (!a.counter) return;
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0) s_last = atomicAdd(a.counter, 1u) == (uint32_t)(n_blocks - 1);
  __syncthreads();
  if (s_last && threadIdx.x == 0) {
    st->generation = (int32_t)g + 1;
    *a.counter = 0u;
  }
}

// Roulette wheel of fit[0..P): integer weights (see select_parent) and their
// inclusive prefix sums, computed by one workgroup of kThreads threads (all
// of which call this).  Integer sums are exact, so the wheel does not depend
// on the order of the additions.  kA: fit was written and the wheel is read
// by other workgroups of the same launch.
template <int kThreads, bool kA>
__device__ void wheel_block(const double* __restrict__ fit, int P, uint64_t* __restrict__ wheel) {
#pragma clang fp contract(off)
  constexpr int kWaves = kThreads / 64;
  __shared__ double s_lo[kWaves], s_hi[kWaves];
  __shared__ uint64_t s_scan[kThreads];
  __shared__ uint64_t s_carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double mn = INFINITY, mx = -INFINITY;
  for (int i = tid; i < P; i += kThreads) {
    const double f = ldc<kA>(fit + i);
    if (!isnan(f)) {
      mn = fmin(mn, f);
      mx = fmax(mx, f);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, off));
    mx = fmax(mx, __shfl_xor(mx, off));
  }
  __syncthreads();  // the caller's earlier use of these arrays is over
  if (lane == 0) {
    s_lo[wave] = mn;
    s_hi[wave] = mx;
  }
  if (tid == 0) s_carry = 0;
  __syncthreads();
  double lo = s_lo[0], hi = s_hi[0];
  for (int w = 1; w < kWaves; ++w) {
    lo = fmin(lo, s_lo[w]);
    hi = fmax(hi, s_hi[w]);
  }
  const bool any = lo <= hi;  // some finite fitness
  const double span = hi - lo;
  for (int base = 0; base < P; base += kThreads) {
    const int i = base + tid;
    uint64_t w = 0;
    if (i < P) {
      const double f = ldc<kA>(fit + i);
      if (!any) w = 1;
      else if (isnan(f)) w = 0;
      else if (!(hi > lo)) w = 1;
      else w = (uint64_t)floor((f - lo) / span * 4294967296.0);
    }
    s_scan[tid] = w;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {  // inclusive scan (Hillis-Steele)
      const uint64_t add = tid >= off ? s_scan[tid - off] : 0;
      __syncthreads();
      s_scan[tid] += add;
      __syncthreads();
    }
    if (i < P) stc<kA>(wheel + i, s_carry + s_scan[tid]);
    __syncthreads();
    if (tid == 0) s_carry += s_scan[kThreads - 1];
    __syncthreads();
  }
}

// Full ranking of fit[0..P) (fitness descending, index ascending, NaN last)
// by a bitonic sort of n_pow2 >= P keys in smem (n_pow2 x 12 bytes), one
// workgroup of kThreads threads; order[q] = chromosome of rank q.
template <int kThreads, bool kA>
__device__ void rank_block(const double* __restrict__ fit, int P, int n_pow2, int* __restrict__ order,
                           unsigned char* smem) {
  uint64_t* sk = reinterpret_cast<uint64_t*>(smem);
  int* si = reinterpret_cast<int*>(smem + (size_t)n_pow2 * 8);
  for (int i = threadIdx.x; i < n_pow2; i += kThreads) {
    sk[i] = i < P ? ord_desc_f64(ldc<kA>(fit + i)) : ~0ull;
    si[i] = i < P ? i : 0x7fffffff;
  }
  __syncthreads();
  block_sort_pairs<kThreads>(sk, si, n_pow2);
  for (int q = threadIdx.x; q < P; q += kThreads) stc<kA>(order + q, si[q]);
}

}  // namespace
}  // namespace game
