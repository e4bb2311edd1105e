// Block-level ranking and best tracking, shared by the standalone rank kernel
// and the tail of the fitness kernels.
//
// Order (Sec. 3 elitism with a total order): higher fitness first, ties to
// the lower index, NaN ranks last.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "game_internal.hpp"

namespace game {

struct Ranked {
  double key;
  int idx;
};
__device__ __forceinline__ bool better(const Ranked& a, const Ranked& b) {
  return a.key > b.key || (a.key == b.key && a.idx < b.idx);
}
__device__ __forceinline__ double rank_key(double f) { return isnan(f) ? -INFINITY : f; }

// Order-preserving maps to unsigned integers: ascending float; descending
// double with NaN ranked like -inf (the order above).
__device__ __forceinline__ uint64_t ord_f32(float f) {
  if (isnan(f)) return 0xFFFFFFFFull;
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? (uint64_t)(~u) : (uint64_t)(u | 0x80000000u);
}
__device__ __forceinline__ uint64_t ord_desc_f64(double f) {
  if (isnan(f)) f = -INFINITY;
  const uint64_t u = (uint64_t)__double_as_longlong(f);
  const uint64_t asc = (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
  return ~asc;
}

// Bitonic sort of n_pow2 (key, index) pairs in LDS by one workgroup of
// kThreads threads (all of which call this), ascending by key then index.
template <int kThreads>
__device__ void block_sort_pairs(uint64_t* sk, int* si, int n_pow2) {
  for (int size = 2; size <= n_pow2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < n_pow2 / 2; t += kThreads) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint64_t ka = sk[lo], kb = sk[hi];
        const int ia = si[lo], ib = si[hi];
        const bool a_gt_b = ka > kb || (ka == kb && ia > ib);
        if (a_gt_b == up) {
          sk[lo] = kb;
          sk[hi] = ka;
          si[lo] = ib;
          si[hi] = ia;
        }
      }
      __syncthreads();
    }
  }
}

// Loads and stores of values another workgroup of the same launch produces or
// consumes: agent-scope atomics, which go through to the device-coherent
// level instead of an XCD's L2 (no cache invalidation needed).  They always
// address global memory, and say so: a pointer read from memory (the
// batched scheduler's table) would otherwise be accessed with flat
// instructions, whose completions the LDS counter waits for too.
template <class T>
using agent_ptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ T ld_agent_g(const T* p) {
  return __hip_atomic_load((agent_ptr<const T>)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_agent_g(T* p, T v) {
  __hip_atomic_store((agent_ptr<T>)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) { return ld_agent_g(p); }
__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p) { return ld_agent_g(p); }
__device__ __forceinline__ int32_t ld_agent(const int32_t* p) { return ld_agent_g(p); }
__device__ __forceinline__ float ld_agent(const float* p) { return ld_agent_g(p); }
__device__ __forceinline__ uint64_t ld_agent(const uint64_t* p) { return ld_agent_g(p); }
__device__ __forceinline__ void st_agent(double* p, double v) { st_agent_g(p, v); }
__device__ __forceinline__ void st_agent(uint32_t* p, uint32_t v) { st_agent_g(p, v); }
__device__ __forceinline__ void st_agent(int32_t* p, int32_t v) { st_agent_g(p, v); }
__device__ __forceinline__ void st_agent(float* p, float v) { st_agent_g(p, v); }
__device__ __forceinline__ void st_agent(uint64_t* p, uint64_t v) { st_agent_g(p, v); }
__device__ __forceinline__ void st_agent(uint16_t* p, uint16_t v) { st_agent_g(p, v); }
__device__ __forceinline__ void st_agent(_Float16* p, _Float16 v) { st_agent_g(p, v); }

// Loads and stores whose flavour a kernel picks at compile time: kAgent for
// data that other workgroups of the same launch write or read (the batched
// scheduler hands a run's population, gene tile, ranking and state from one
// phase to the next inside one launch), plain otherwise.
template <bool kAgent, class T>
__device__ __forceinline__ T ldc(const T* p) {
  if constexpr (kAgent) return ld_agent(p);
  else return *p;
}
template <bool kAgent, class T>
__device__ __forceinline__ void stc(T* p, T v) {
  if constexpr (kAgent) st_agent(p, v);
  else *p = v;
}

// Order this thread's earlier st_agent stores before an arrival count that
// follows a barrier.  Every value one workgroup of a launch hands to another
// is written with st_agent (device-scope stores, acknowledged once visible
// at device scope) and read with ld_agent, so waiting for the stores'
// acknowledgements is the ordering the consumer needs.  A device-scope
// release fence would in addition write back the XCD's whole L2 for plain
// stores, which no workgroup of these launches reads from another; with one
// such write-back per workgroup it cost 10-13 us of a fitness launch.
__device__ __forceinline__ void agent_stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Top n_top indices of fit[0..P) by repeated arg-max, computed by one
// workgroup of kThreads threads (all of which must call this).  kAgent: fit
// was written earlier in the same launch by other workgroups, and top is
// stored for them too.  Up to
// kCache values per thread are read once into registers (all loads in
// flight together), so the n_top passes cost no further memory round trips;
// larger P re-reads fit on every pass.
template <int kThreads, bool kAgent = false>
__device__ void block_topk(const double* __restrict__ fit, int P, int n_top, int* __restrict__ top) {
  constexpr int kCache = 8;
  __shared__ int chosen[kMaxElite];
  __shared__ double wkey[kThreads / 64];
  __shared__ int widx[kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto pick = [&](Ranked best, int e) {  // workgroup arg-max of the threads' candidates
    for (int off = 32; off > 0; off >>= 1) {
      const Ranked o{__shfl_xor(best.key, off), __shfl_xor(best.idx, off)};
      if (better(o, best)) best = o;
    }
    if (lane == 0) {
      wkey[wave] = best.key;
      widx[wave] = best.idx;
    }
    __syncthreads();
    if (tid == 0) {
      Ranked b{wkey[0], widx[0]};
      for (int q = 1; q < kThreads / 64; ++q) {
        const Ranked o{wkey[q], widx[q]};
        if (better(o, b)) b = o;
      }
      chosen[e] = b.idx;
      stc<kAgent>(top + e, b.idx);
    }
    __syncthreads();
  };
  if (P <= kThreads * kCache) {
    double key[kCache];
    // unconditional loads (index clamped into fit, keys past P replaced): a
    // load under a bounds branch is waited for where the paths join, which
    // would make these one memory round trip each
#pragma unroll
    for (int q = 0; q < kCache; ++q) {
      const int i = tid + q * kThreads;
      const int ic = i < P ? i : P - 1;
      const double f = kAgent ? ld_agent(fit + ic) : fit[ic];
      key[q] = i < P ? rank_key(f) : -INFINITY;
    }
    uint32_t taken = 0u;  // bit q: value q of this thread already chosen
    for (int e = 0; e < n_top; ++e) {
      Ranked best{-INFINITY, 0x7fffffff};
#pragma unroll
      for (int q = 0; q < kCache; ++q) {
        const int i = tid + q * kThreads;
        const Ranked c{key[q], i};
        if (i < P && !((taken >> q) & 1u) && better(c, best)) best = c;
      }
      pick(best, e);
      const int w = chosen[e];
      if (w < P && w % kThreads == tid) taken |= 1u << (w / kThreads);
    }
    return;
  }
  for (int e = 0; e < n_top; ++e) {
    Ranked best{-INFINITY, 0x7fffffff};
    for (int i = tid; i < P; i += kThreads) {
      bool taken = false;
      for (int q = 0; q < e; ++q) taken |= (chosen[q] == i);
      if (taken) continue;
      const Ranked c{rank_key(kAgent ? ld_agent(fit + i) : fit[i]), i};
      if (better(c, best)) best = c;
    }
    pick(best, e);
  }
}

// Keep the best chromosome seen (strictly lower MSE replaces it) and, while a
// run is active, decide whether the run stops after this generation.  `top`
// holds the generation's ranking (written by this workgroup); mse and miscls
// were written by other workgroups of the same launch.  Every thread of the
// workgroup calls this.  kAgent: the state, the population and the best
// genes are also handed between workgroups of one launch (batched
// scheduler), so they are read and written at device scope.
template <bool kAgent = false>
__device__ inline void track_best(DevState* st, const int* __restrict__ top,
                                  const double* __restrict__ mse, const double* __restrict__ miscls,
                                  const float* __restrict__ pop, int L, float* __restrict__ best) {
  __shared__ int s_improve, s_b;
  __syncthreads();
  // thread 0 reads everything the decision needs at once (one memory round
  // trip after the index; nothing else writes these values meanwhile)
  double m = 0.0, mc = 0.0, best_mse = 0.0, thr = 0.0;
  int active = 0, gen = 0, end_gen = 0;
  if (threadIdx.x == 0) {
    const int b = ldc<kAgent>(top);
    m = ld_agent(mse + b);
    mc = ld_agent(miscls + b);
    const int have = ldc<kAgent>(&st->have_best);
    best_mse = ldc<kAgent>(&st->best_mse);
    active = ldc<kAgent>(&st->run_active);
    thr = ldc<kAgent>(&st->mse_threshold);
    gen = ldc<kAgent>(&st->generation);
    end_gen = ldc<kAgent>(&st->end_generation);
    s_b = b;
    s_improve = (!have || m < best_mse) ? 1 : 0;
  }
  __syncthreads();
  const int b = s_b;
  if (s_improve)
    for (int l = threadIdx.x; l < L; l += blockDim.x) stc<kAgent>(best + l, ldc<kAgent>(pop + (int64_t)b * L + l));
  if (threadIdx.x == 0) {
    stc<kAgent>(&st->best_index, b);
    if (s_improve) {
      best_mse = m;
      stc<kAgent>(&st->have_best, 1);
      stc<kAgent>(&st->best_mse, m);
      stc<kAgent>(&st->best_fitness, 1.0 - m);
      stc<kAgent>(&st->best_miscls, mc);
    }
    if (active) {
      if (best_mse <= thr) {
        stc<kAgent>(&st->stopped, 1);
        stc<kAgent>(&st->stop_reason, (int32_t)GAME_STOP_THRESHOLD);
      } else if (gen + 1 >= end_gen) {
        stc<kAgent>(&st->stopped, 1);
        stc<kAgent>(&st->stop_reason, (int32_t)GAME_STOP_MAX_GEN);
      }
    }
  }
}

}  // namespace game
