// Population fitness: z = Phi . G^T on MFMA with the error reduction fused in.
//
// For every chromosome p and pattern n (eq. 2 and 3):
//   z[n,p]  = sum_m Phi[n,m] G[p,m] (+ a_0 of p)
//   e[n,p]  = (t_n - z)^2                    (regression)
//           = (l_n - 1/(1+exp(-z)))^2        (classification, label l_n = [t_n >= 0.5])
//   miss    = [(z >= 0) != l_n]              (classification)
// and per chromosome sse = sum_n e, misses = sum_n miss, reduced to
// mse = sse / N and fitness = 1 - mse by the kernels' tail (fitness_tail).
//
// Two kernels share that definition: fitness_lds_kernel (the gene tile
// staged in LDS, persistent; described with lds_item below) and the
// streaming fitness_kernel (FP64, and gene counts whose tile does not fit
// in LDS), whose decomposition is this (one workgroup = 4 waves of 64
// lanes, 2 x 2):
//   * a workgroup owns one tile of tile_p chromosomes and a group of
//     consecutive row tiles of tile_n patterns; Z never leaves registers;
//   * each wave computes a (16*WM) x (16*WN) block of Z with 16x16 MFMAs,
//     streaming Phi rows and gene rows straight from global memory into the
//     MFMA operand registers (each lane loads 8 or 16 contiguous bytes of one
//     row per K-block; the same k permutation is applied to both operands, so
//     the contraction is unchanged), double-buffered one K-block ahead;
//   * the epilogue maps every accumulator element to its error, sums a row
//     tile in the accumulation type, adds that into a double per column, and
//     after the last row tile reduces the four 16-lane groups by shuffles and
//     the two row-waves through LDS in a fixed order.  Partial sums go to
//     part_sse[row_group][p] (double) and part_miss (uint32); no floating-
//     point atomics (only arrival counts), so every run is bit-reproducible;
//   * workgroups sharing a row group run back to back on one XCD (the
//     dispatcher deals workgroups round-robin over the 8 XCDs; the logical
//     tile index is remapped so each XCD gets a contiguous range), so the
//     Phi rows they share hit that XCD's L2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "breed.hpp"
#include "game_internal.hpp"
#include "select.hpp"

namespace game {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

// Accumulator layout of the 16x16 MFMA outputs: lane l, element r holds
// column l % 16 and row 4 (l / 16) + r, except for the double-precision
// instruction, whose rows are interleaved: row (l / 16) + 4 r.
struct F32Tr {
  static constexpr bool kRowInterleave = false;
  using T = float;
  using Acc = float;
  using AccV = v4f;
  using Ld = float2;                  // 2 k-steps of 16x16x4
  static constexpr int kBlk = 8;      // Phi columns per K-block
  static constexpr int kPerLane = 2;  // contiguous elements a lane loads per K-block
  static constexpr int kSteps = 2;    // MFMAs per K-block
  template <int S>
  __device__ static AccV mma(const Ld& a, const Ld& b, AccV c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(S == 0 ? a.x : a.y, S == 0 ? b.x : b.y, c, 0, 0, 0);
  }
};

struct F64Tr {
  static constexpr bool kRowInterleave = true;
  using T = double;
  using Acc = double;
  using AccV = v4d;
  using Ld = double2;
  static constexpr int kBlk = 8;
  static constexpr int kPerLane = 2;
  static constexpr int kSteps = 2;
  template <int S>
  __device__ static AccV mma(const Ld& a, const Ld& b, AccV c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(S == 0 ? a.x : a.y, S == 0 ? b.x : b.y, c, 0, 0, 0);
  }
};

struct BF16Tr {
  static constexpr bool kRowInterleave = false;
  using T = uint16_t;  // bf16 bit patterns
  using Acc = float;
  using AccV = v4f;
  using Ld = uint4;    // 8 x bf16
  static constexpr int kBlk = 32;
  static constexpr int kPerLane = 8;
  static constexpr int kSteps = 1;
  template <int S>
  __device__ static AccV mma(const Ld& a, const Ld& b, AccV c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                   __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
  }
};

struct F16Tr {
  static constexpr bool kRowInterleave = false;
  using T = _Float16;
  using Acc = float;
  using AccV = v4f;
  using Ld = uint4;    // 8 x f16
  static constexpr int kBlk = 32;
  static constexpr int kPerLane = 8;
  static constexpr int kSteps = 1;
  template <int S>
  __device__ static AccV mma(const Ld& a, const Ld& b, AccV c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8h, a),
                                                  __builtin_bit_cast(v8h, b), c, 0, 0, 0);
  }
};

// Classification error of one pattern, (l - sigmoid(z))^2 with the class label
// l in {0, 1}, written as sigmoid(s z)^2 with s = +1 for l = 0 and -1 for
// l = 1:  r = 1 / (1 + 2^(c z)),  c = -s log2(e),  error = r^2.  One exp and
// one reciprocal (v_exp_f32 / v_rcp_f32, about 1 ulp each).
constexpr double kLog2e = 1.4426950408889634;
__device__ __forceinline__ float sig_pos(float cz) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(cz));
}
__device__ __forceinline__ double sig_pos(double cz) { return 1.0 / (1.0 + exp2(cz)); }

// loc + q^2 as one fused multiply-add: written out, so that every kernel
// that shares the error arithmetic rounds it the same way (left to the
// compiler, a sum of two squares may be fused around either product).
__device__ __forceinline__ float sq_acc(float q, float loc) { return __builtin_fmaf(q, q, loc); }

// Misclassification test by floating-point class: for label 0 a pattern is
// missed when z >= 0 (+-0, positive denormal/normal/inf), for label 1 when
// z < 0 or z is NaN; padding rows use an empty class mask.
constexpr int kMissIfLabel0 = 0x3E0;  // -0, +0, +denorm, +normal, +inf
constexpr int kMissIfLabel1 = 0x01F;  // sNaN, qNaN, -inf, -normal, -denorm
__device__ __forceinline__ bool in_class(float z, int mask) { return __builtin_amdgcn_classf(z, mask); }
__device__ __forceinline__ bool in_class(double z, int mask) { return __builtin_amdgcn_class(z, mask); }

// Tail shared by both fitness kernels (all 256 threads call it after their
// partial row is written).  The last workgroup of chromosome tile pt (atomic
// arrival count) adds that tile's partial rows in a fixed order: 256 / TP
// contiguous segments of row groups, each summed in row order, then the
// segments in order.  For a population evaluation the last tile to finish
// ranks the population and tracks the best chromosome.  Counters return to
// zero, so the kernel can be replayed from a graph.
// One copy of the tail's LDS per kernel, whatever tile widths it serves.
struct TailLds {
  double red[256];
  uint64_t redm[256];
  int flag;
};
__device__ __forceinline__ TailLds& tail_lds() {
  __shared__ TailLds s;
  return s;
}

// An arrival count: the counter's previous value (device scope, in global memory).
__device__ __forceinline__ uint32_t arrive(uint32_t* c) {
  return __hip_atomic_fetch_add((agent_ptr<uint32_t>)c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// kFlow: the batched scheduler runs every phase of a run inside one launch,
// so the counters, the ranking and the state are also written at device scope.
template <int TP, bool kFlow = false>
__device__ __forceinline__ void fitness_tail(const FitTail& t, int pt, int n_pt, int64_t n_rg, int part_ld,
                             const double* psse, const uint32_t* pmiss) {
  constexpr int S = 256 / TP;
  TailLds& sh = tail_lds();
  int& s_flag = sh.flag;
  double* s_red = sh.red;
  uint64_t* s_redm = sh.redm;
  // the partial row was stored at agent scope; order it before the arrival
  agent_stores_done();
  __syncthreads();
  if (threadIdx.x == 0) s_flag = arrive(&t.counters[pt]) == (uint32_t)(n_rg - 1);
  __syncthreads();
  if (!s_flag) return;
  const int c = threadIdx.x % TP, seg = threadIdx.x / TP;
  const int p = pt * TP + c;
  const int64_t chunk = (n_rg + S - 1) / S;
  const int64_t b = seg * chunk, e = min(n_rg, b + chunk);
  double sum = 0.0;
  uint64_t cnt = 0;
  // 16 rows in flight per thread, the rest of a segment 4 at a time: these
  // device-scope loads go past the XCD's L2, so each batch is a full memory
  // round trip
  int64_t r = b;
  for (; r + 16 <= e; r += 16) {
    double v[16];
    uint32_t m[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      v[q] = ld_agent(psse + (r + q) * part_ld + p);
      m[q] = ld_agent(pmiss + (r + q) * part_ld + p);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      sum += v[q];
      cnt += m[q];
    }
  }
  for (; r < e; r += 4) {
    double v[4];
    uint32_t m[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q] = r + q < e ? ld_agent(psse + (r + q) * part_ld + p) : 0.0;
      m[q] = r + q < e ? ld_agent(pmiss + (r + q) * part_ld + p) : 0u;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (r + q < e) {
        sum += v[q];
        cnt += m[q];
      }
  }
  s_red[threadIdx.x] = sum;
  s_redm[threadIdx.x] = cnt;
  __syncthreads();
  if (seg == 0 && p < t.P) {
    double tot = 0.0;
    uint64_t mt = 0;
#pragma unroll
    for (int q = 0; q < S; ++q) {
      tot += s_red[q * TP + c];
      mt += s_redm[q * TP + c];
    }
    const double ms = tot * t.invN, mc = (double)mt * t.invN, f = 1.0 - ms;
    if (t.mse) st_agent(t.mse + p, ms);
    if (t.miscls) st_agent(t.miscls + p, mc);
    if (t.fit) st_agent(t.fit + p, f);
    if (t.mse2) t.mse2[p] = ms;
    if (t.miscls2) t.miscls2[p] = mc;
    if (t.fit2) t.fit2[p] = f;
  }
  agent_stores_done();
  __syncthreads();
  if (threadIdx.x == 0) {
    stc<kFlow>(&t.counters[pt], 0u);
    s_flag = t.n_top > 0 && arrive(&t.counters[t.n_pt_cap]) == (uint32_t)(n_pt - 1);
  }
  __syncthreads();
  if (!s_flag) return;
  block_topk<256, true>(t.fit, t.P, t.n_top, t.top);
  __syncthreads();
  if (t.track) {
    const float* pop = (ldc<kFlow>(&t.st->generation) & 1) ? t.pop1 : t.pop0;
    track_best<kFlow>(t.st, t.top, t.mse, t.miscls, pop, t.L, t.best);
  }
  if (threadIdx.x == 0) stc<kFlow>(&t.counters[t.n_pt_cap], 0u);
}

template <class Tr, int WM, int WN, bool kCls>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void fitness_kernel(
    const typename Tr::T* __restrict__ phi, const typename Tr::T* __restrict__ tile,
    const typename Tr::Acc* __restrict__ biasv, const typename Tr::Acc* __restrict__ tvec,
    int64_t N, int M_pad, int64_t n_rt, int n_pt, int rt_per_wg, int64_t n_items, int part_ld,
    double* __restrict__ part_sse, uint32_t* __restrict__ part_miss, const DevState* st,
    const FitTail tail) {
  using T = typename Tr::T;
  using Acc = typename Tr::Acc;
  using AccV = typename Tr::AccV;
  using Ld = typename Tr::Ld;
  constexpr int TN = 32 * WM, TP = 32 * WN;

  if (run_halted(st)) return;
  const int64_t nwg = gridDim.x;
  const int64_t w = blockIdx.x;
  const int64_t lt = (w & 7) * (nwg >> 3) + (w >> 3);
  if (lt >= n_items) return;
  const int pt = (int)(lt % n_pt);
  const int64_t rg = lt / n_pt;

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int lrow = lane & 15, lgrp = lane >> 4;
  const int KB = M_pad / Tr::kBlk;

  const int pw0 = pt * TP + wc * 16 * WN;  // first chromosome of this wave
  const T* bptr[WN];
#pragma unroll
  for (int j = 0; j < WN; ++j)
    bptr[j] = tile + (int64_t)(pw0 + j * 16 + lrow) * M_pad + lgrp * Tr::kPerLane;

  Acc bias_j[WN];
#pragma unroll
  for (int j = 0; j < WN; ++j) bias_j[j] = biasv ? biasv[pw0 + j * 16 + lrow] : Acc(0);

  double sse[WN];
  uint32_t miss[WN];
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    sse[j] = 0.0;
    miss[j] = 0u;
  }

  const int64_t rt_begin = rg * rt_per_wg;
  const int64_t rt_end = min(n_rt, rt_begin + rt_per_wg);
  for (int64_t rt = rt_begin; rt < rt_end; ++rt) {
    const int64_t nw0 = rt * TN + wr * 16 * WM;  // first pattern of this wave
    const T* aptr[WM];
#pragma unroll
    for (int i = 0; i < WM; ++i)
      aptr[i] = phi + (nw0 + i * 16 + lrow) * (int64_t)M_pad + lgrp * Tr::kPerLane;

    AccV acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) acc[i][j] = AccV{};

    Ld a0[WM], b0[WN], a1[WM], b1[WN];
    auto load = [&](Ld* a, Ld* b, int kb) {
#pragma unroll
      for (int i = 0; i < WM; ++i) a[i] = *reinterpret_cast<const Ld*>(aptr[i] + kb * Tr::kBlk);
#pragma unroll
      for (int j = 0; j < WN; ++j) b[j] = *reinterpret_cast<const Ld*>(bptr[j] + kb * Tr::kBlk);
    };
    auto mma_all = [&](const Ld* a, const Ld* b) {
      // one k-step across all accumulators before the next, so consecutive
      // MFMAs never depend on each other
      auto step = [&](auto s_tag) {
        constexpr int S = decltype(s_tag)::value;
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) acc[i][j] = Tr::template mma<S>(a[i], b[j], acc[i][j]);
      };
      step(std::integral_constant<int, 0>{});
      if constexpr (Tr::kSteps > 1) step(std::integral_constant<int, 1>{});
    };
    // loads unconditional (K-block index clamped), so only the needed one is waited for
    auto kc = [&](int k) { return k < KB ? k : KB - 1; };
    load(a0, b0, 0);
    for (int kb = 0; kb < KB; kb += 2) {
      load(a1, b1, kc(kb + 1));
      mma_all(a0, b0);
      load(a0, b0, kc(kb + 2));
      if (kb + 1 < KB) mma_all(a1, b1);
    }

    // epilogue: accumulator element r of block (i, j) is pattern
    // nw0 + 16 i + row_in_block(r) and chromosome pw0 + 16 j + lrow
    auto row_in_block = [&](int r) { return Tr::kRowInterleave ? lgrp + 4 * r : 4 * lgrp + r; };
    Acc tv[WM][4], cz[WM][4], wgt[WM][4];
    int cmask[WM][4];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool valid = nw0 + i * 16 + row_in_block(r) < N;
        tv[i][r] = tvec[nw0 + i * 16 + row_in_block(r)];
        const bool lab = tv[i][r] >= Acc(0.5);
        cz[i][r] = lab ? Acc(kLog2e) : Acc(-kLog2e);
        cmask[i][r] = valid ? (lab ? kMissIfLabel1 : kMissIfLabel0) : 0;
        wgt[i][r] = valid ? Acc(1) : Acc(0);
      }
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      Acc loc = Acc(0);
      uint32_t ms = 0u;
#pragma unroll
      for (int i = 0; i < WM; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const Acc z = acc[i][j][r] + bias_j[j];
          if constexpr (kCls) {
            const Acc q = sig_pos(cz[i][r] * z) * wgt[i][r];
            loc += q * q;
            ms += in_class(z, cmask[i][r]) ? 1u : 0u;
          } else {
            const Acc d = (tv[i][r] - z) * wgt[i][r];
            loc += d * d;
          }
        }
      }
      sse[j] += (double)loc;
      miss[j] += ms;
    }
  }

  // reduce the four 16-lane groups (lanes l, l^16, l^32, l^48 share a column)
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    sse[j] += __shfl_xor(sse[j], 16);
    sse[j] += __shfl_xor(sse[j], 32);
    miss[j] += __shfl_xor(miss[j], 16);
    miss[j] += __shfl_xor(miss[j], 32);
  }
  __shared__ double s_sse[2][TP];
  __shared__ uint32_t s_miss[2][TP];
  if (lgrp == 0) {
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      s_sse[wr][wc * 16 * WN + j * 16 + lrow] = sse[j];
      s_miss[wr][wc * 16 * WN + j * 16 + lrow] = miss[j];
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < TP; c += 256) {
    const int64_t o = rg * part_ld + pt * TP + c;
    st_agent(part_sse + o, s_sse[0][c] + s_sse[1][c]);
    st_agent(part_miss + o, s_miss[0][c] + s_miss[1][c]);
  }
  const int64_t n_rg = (n_rt + rt_per_wg - 1) / rt_per_wg;
  fitness_tail<TP>(tail, pt, n_pt, n_rg, part_ld, part_sse, part_miss);
}

// Persistent decomposition, used when the gene tile fits in LDS.  The grid
// holds as many workgroups as can be resident; a work item (row range wr,
// chromosome tile pt) stages its gene tile in LDS once (K-block-major, in
// the order the MFMA operand fragments are read) and walks its
// contiguous range of 32-pattern row units.  The four waves of an item take
// the range's units round-robin, each computing 32 patterns x TP chromosomes
// (2 x WN blocks of 16 x 16) per unit, so every Phi row is read by exactly
// one wave.  Range boundaries fall on blocks of ub units: with ub = 4
// (128-pattern row tiles) the four waves of a range do equal work; with
// ub = 1 a range of U units gives U mod 4 of its waves one unit more, and
// which waves those are is rotated by two (item_rot below) between the two
// workgroups that share a CU, whose waves w run on the same SIMD, so their
// extra units do not stack on one SIMD.  The host picks the ub whose busiest
// SIMD carries fewer units (fitness_range_block).  The next unit's targets
// and first Phi K-blocks are fetched before the current epilogue.
//
// One work item of the LDS-staged kernels: chromosome tile pt (TP = 16 WN
// chromosomes, staged in LDS) against row range wr of n_ranges; writes the
// range's partial sums part_sse / part_miss[wr][pt * TP ..].  The
// single-context and the batched kernels run exactly this code, so a
// chromosome's sums do not depend on which of them evaluated it.  kDepth is
// how many K-blocks ahead the Phi fragments are loaded (1 or 2): it moves
// loads, not arithmetic.
//
// Rotation of item lt of a launch of n_items items (grid rounded up to a
// multiple of 8, remapped so each XCD runs a contiguous block of per items).
// An XCD's dispatcher gives each of its cpx CUs one workgroup before any
// second, so the k-th and (k + cpx)-th of its items share a CU: with ub = 1
// they get opposite rotations.  Placement only moves time; the sums of an
// item depend on (lt, n_items, cpx, ub) alone, which the batched kernel
// reproduces.
__device__ __forceinline__ int item_rot(int64_t lt, int64_t n_items, int cpx, int ub) {
  const int64_t per = (n_items + 7) / 8;
  return ub == 1 ? 2 * (int)(((lt % per) / cpx) & 1) : 0;
}

// Loads through the global address space.  The item's pointers are global
// memory; said so explicitly, the loads are global ones even where the
// pointer came from memory (the batched scheduler's table) rather than a
// kernel argument: a flat load would count against the LDS counter too, so
// each LDS wait of the K loop would also wait for the Phi loads in flight.
template <class T>
using gptr = const __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ T gload(const T* p) {
  typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, *(gptr<uint32_t>)p);
  else if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, *(gptr<uint64_t>)p);
  else {
    static_assert(sizeof(T) == 16, "4, 8 or 16-byte loads");
    return __builtin_bit_cast(T, *(gptr<u32x4v>)p);
  }
}
__device__ __forceinline__ uint64_t gload_agent(const uint64_t* p) {
  return __hip_atomic_load((gptr<uint64_t>)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A gene-tile load unit: plain, or at device scope (kAgent: the tile was
// written by the breed phase of the same launch).
template <bool kAgent, class Ld>
__device__ __forceinline__ Ld ld_unit(const Ld* p) {
  if constexpr (!kAgent) {
    return gload(p);
  } else if constexpr (sizeof(Ld) == 8) {
    return __builtin_bit_cast(Ld, gload_agent(reinterpret_cast<const uint64_t*>(p)));
  } else {
    static_assert(sizeof(Ld) == 16, "gene-tile units are 8 or 16 bytes");
    const uint64_t* q = reinterpret_cast<const uint64_t*>(p);
    struct Pair {
      uint64_t lo, hi;
    };
    return __builtin_bit_cast(Ld, Pair{gload_agent(q), gload_agent(q + 1)});
  }
}

template <class Tr, bool kCls, int WN, int kDepth, bool kFlow = false>
__device__ __forceinline__ void lds_item(const typename Tr::T* __restrict__ phi,
                                         const typename Tr::T* __restrict__ tile,
                                         const typename Tr::Acc* __restrict__ biasv,
                                         const typename Tr::Acc* __restrict__ tvec, int64_t N,
                                         int M_pad, int ldsw, int n_ranges, int pt, int wr,
                                         int ub, int rot, int part_ld,
                                         double* __restrict__ part_sse,
                                         uint32_t* __restrict__ part_miss, uint32_t* lds) {
  using T = typename Tr::T;
  using Acc = typename Tr::Acc;
  using AccV = typename Tr::AccV;
  using Ld = typename Tr::Ld;
  constexpr int WM = 2, TU = 32, TP = 16 * WN;
  constexpr int kLdWords = (int)(sizeof(Ld) / 4);
  static_assert(Tr::kBlk / Tr::kPerLane == 4, "a K-block is four lane groups of one Ld unit");
  // LDS: the gene tile (TP x M_pad elements = TP ldsw words), then the
  // per-wave column sums.  The tile is stored K-block-major in MFMA operand
  // order: the fragment lane l of block column j reads for K-block kb sits at
  // Ld unit (kb WN + j) 64 + l, so a wave's read of a fragment is 64
  // consecutive Ld units (no bank conflicts) and every address is one
  // lane-constant base plus a compile-time or per-K-block offset.
  double (*s_sse)[TP] = reinterpret_cast<double (*)[TP]>(lds + TP * ldsw);
  uint32_t (*s_miss)[TP] = reinterpret_cast<uint32_t (*)[TP]>(lds + TP * ldsw + 8 * TP);

  // the wave index is uniform in a wave; saying so keeps the unit loop and
  // the full/ragged test on scalar registers and branches
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lrow = lane & 15, lgrp = lane >> 4;
  const int KB = M_pad / Tr::kBlk;
  const int64_t n_units = (N + TU - 1) / TU;
  const int64_t n_blk = (n_units + ub - 1) / ub;
  const int64_t u_begin = (int64_t)wr * n_blk / n_ranges * ub;
  const int64_t u_end = min(n_units, (int64_t)(wr + 1) * n_blk / n_ranges * ub);
  const int64_t u_first = u_begin + ((wave + rot) & 3);  // this wave's units: u_first, +4, ...

  const int p0 = pt * TP;
  Acc bias_j[WN];
#pragma unroll
  for (int j = 0; j < WN; ++j) bias_j[j] = biasv ? ldc<kFlow>(biasv + p0 + j * 16 + lrow) : Acc(0);
  const int bofs0 = lane * kLdWords;  // + ((kb WN + j) 64) kLdWords

  auto row_in_block = [&](int r) { return Tr::kRowInterleave ? lgrp + 4 * r : 4 * lgrp + r; };

  double sse[WN];
  uint32_t miss[WN];
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    sse[j] = 0.0;
    miss[j] = 0u;
  }

  Ld a0[WM], a1[WM], b0[WN], b1[WN];
  Acc tv[WM][4];
  auto load_t = [&](int64_t u) {
    const int64_t nw0 = u * TU;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) tv[i][r] = gload(tvec + nw0 + i * 16 + row_in_block(r));
  };
  auto loadA = [&](Ld* a, int64_t u, int kb) {
    const int64_t nw0 = u * TU;
#pragma unroll
    for (int i = 0; i < WM; ++i)
      a[i] = gload(reinterpret_cast<const Ld*>(phi + (nw0 + i * 16 + lrow) * (int64_t)M_pad +
                                               lgrp * Tr::kPerLane + kb * Tr::kBlk));
  };
  auto loadB = [&](Ld* b, int kb) {
#pragma unroll
    for (int j = 0; j < WN; ++j)
      b[j] = *reinterpret_cast<const Ld*>(&lds[bofs0 + (kb * WN + j) * 64 * kLdWords]);
  };

  if (u_first < u_end) {
    load_t(u_first);
    loadA(a0, u_first, 0);
    if (kDepth == 2) loadA(a1, u_first, KB > 1 ? 1 : 0);
  }
  // stage the gene tile (rows pt*TP .. +TP) into LDS with 64 bytes of loads
  // in flight per thread before their stores (a load-store loop waits out
  // the full memory latency once per element); the first unit's Phi loads
  // above are already on their way.  Named registers, not an array, so
  // nothing is placed in scratch memory.
  {
    const int units = M_pad / Tr::kPerLane;  // Ld units per gene row
    const int total = TP * units;
    const Ld* src = reinterpret_cast<const Ld*>(tile + (int64_t)pt * TP * M_pad);
    // unconditional loads (the index clamped into the tile; st skips the
    // extra ones): a load under a branch makes the compiler wait for it at
    // the join, and the batch's loads would go one memory latency at a time
    auto ld = [&](int v) { return ld_unit<kFlow>(src + min(v, total - 1)); };
    auto st = [&](int v, const Ld& x) {
      if (v < total) {
        // global unit c of gene row r: K-block c / 4, lane group c % 4;
        // block column r / 16, lane row r % 16
        const int r = v / units, c = v - r * units;
        const int slot = ((c >> 2) * WN + (r >> 4)) * 64 + (c & 3) * 16 + (r & 15);
        *reinterpret_cast<Ld*>(&lds[slot * kLdWords]) = x;
      }
    };
    // 128 bytes of loads in flight per thread, all issued before the stores
    constexpr int kBatch = 128 / (int)sizeof(Ld);
    for (int v = tid; v < total; v += 256 * kBatch) {
      Ld g[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) g[q] = ld(v + 256 * q);
#pragma unroll
      for (int q = 0; q < kBatch; ++q) st(v + 256 * q, g[q]);
    }
  }
  __syncthreads();

  // Wave priorities of the two phases.  Where the matrix cores bind (FP32,
  // regression), a wave in its K loop issues ahead of the other wave on the
  // SIMD in its epilogue, whose VALU work then fills the MFMA gaps (workload
  // 2 FP32 1 % faster); where the classification epilogue's VALU work binds
  // (16-bit tiles), the epilogue goes first and the MFMAs fill its gaps
  // (BF16 10 % faster at 100 000 x 1000, 17 % at 10^6 x 2048).
  constexpr bool kValuBound = kCls && sizeof(T) == 2;
  constexpr int kPrioK = kValuBound ? 0 : 1, kPrioEpi = kValuBound ? 1 : 0;
  for (int64_t u = u_first; u < u_end; u += 4) {
    __builtin_amdgcn_s_setprio(kPrioK);
    AccV acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) acc[i][j] = AccV{};
    auto mma_all = [&](const Ld* a, const Ld* b) {
      // one k-step across all accumulators before the next, so consecutive
      // MFMAs never depend on each other
      auto step = [&](auto s_tag) {
        constexpr int S = decltype(s_tag)::value;
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) acc[i][j] = Tr::template mma<S>(a[i], b[j], acc[i][j]);
      };
      step(std::integral_constant<int, 0>{});
      if constexpr (Tr::kSteps > 1) step(std::integral_constant<int, 1>{});
    };
    // Loads are issued unconditionally (block indices clamped to the last
    // K-block; a clamped load is simply not used), so the compiler can count
    // the loads in flight and wait only for the one an MFMA needs: a load
    // under a branch makes it wait for all of them.  16-bit operands: the
    // gene fragments are 16 bytes per lane, so only Phi is double-buffered
    // (LDS reads are issued right before their MFMAs).
    constexpr bool kDoubleB = sizeof(Ld) == 8;
    auto kc = [&](int k) { return k < KB ? k : KB - 1; };
    if constexpr (kDepth == 2) {
      // Phi fragments two K-blocks ahead: a0..a3 hold blocks kb..kb+3
      Ld a2[WM], a3[WM];
      if constexpr (kDoubleB) loadB(b0, 0);
      for (int kb = 0; kb < KB; kb += 4) {
        loadA(a2, u, kc(kb + 2));
        if constexpr (kDoubleB) loadB(b1, kc(kb + 1));
        else loadB(b0, kb);
        mma_all(a0, b0);
        loadA(a3, u, kc(kb + 3));
        if constexpr (kDoubleB) {
          loadB(b0, kc(kb + 2));
          if (kb + 1 < KB) mma_all(a1, b1);
        } else {
          loadB(b0, kc(kb + 1));
          if (kb + 1 < KB) mma_all(a1, b0);
        }
        loadA(a0, u, kc(kb + 4));
        if constexpr (kDoubleB) loadB(b1, kc(kb + 3));
        else loadB(b0, kc(kb + 2));
        if (kb + 2 < KB) mma_all(a2, b0);
        loadA(a1, u, kc(kb + 5));
        if constexpr (kDoubleB) {
          loadB(b0, kc(kb + 4));
          if (kb + 3 < KB) mma_all(a3, b1);
        } else {
          loadB(b0, kc(kb + 3));
          if (kb + 3 < KB) mma_all(a3, b0);
        }
      }
    } else {
      // one K-block ahead, loads under their bounds: in the batched kernel,
      // whose registers also hold the other tile widths' variants, this
      // schedules better than the clamped form
      int kb = 0;
      if constexpr (kDoubleB) {
        loadB(b0, 0);
        for (; kb + 1 < KB; kb += 2) {
          loadA(a1, u, kb + 1);
          loadB(b1, kb + 1);
          mma_all(a0, b0);
          if (kb + 2 < KB) {
            loadA(a0, u, kb + 2);
            loadB(b0, kb + 2);
          }
          mma_all(a1, b1);
        }
        if (kb < KB) mma_all(a0, b0);
      } else {
        for (; kb + 1 < KB; kb += 2) {
          loadA(a1, u, kb + 1);
          loadB(b0, kb);
          mma_all(a0, b0);
          if (kb + 2 < KB) loadA(a0, u, kb + 2);
          loadB(b0, kb + 1);
          mma_all(a1, b0);
        }
        if (kb < KB) {
          loadB(b0, kb);
          mma_all(a0, b0);
        }
      }
    }
    (void)b1;

    // this unit's targets -> per-pattern coefficients, then prefetch the next unit
    const int64_t nw0 = u * TU;
    const bool full = (u + 1) * TU <= N;
    Acc tcur[WM][4];   // regression: target; classification: -s log2(e)
    int cmask[WM][4];  // classification: class mask of missed outputs
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool valid = full || nw0 + i * 16 + row_in_block(r) < N;
        const bool lab = tv[i][r] >= Acc(0.5);
        tcur[i][r] = kCls ? (lab ? Acc(kLog2e) : Acc(-kLog2e)) : tv[i][r];
        cmask[i][r] = valid ? (lab ? kMissIfLabel1 : kMissIfLabel0) : 0;
      }
    if constexpr (kDepth == 2) {  // next unit (the last unit reloads itself, unused)
      const int64_t un = u + 4 < u_end ? u + 4 : u;
      load_t(un);
      loadA(a0, un, 0);
      loadA(a1, un, kc(1));
    } else if (u + 4 < u_end) {
      load_t(u + 4);
      loadA(a0, u + 4, 0);
    }

    __builtin_amdgcn_s_setprio(kPrioEpi);
    // epilogue: element r of block (i, j) is pattern nw0 + 16 i + row_in_block(r),
    // chromosome p0 + 16 j + lrow
    auto epilogue = [&](auto full_tag) {
      constexpr bool kFull = decltype(full_tag)::value;
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        Acc loc = Acc(0);
        uint32_t ms = 0u;
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const Acc z = acc[i][j][r] + bias_j[j];
            Acc q;
            if constexpr (kCls) {
              q = sig_pos(tcur[i][r] * z);
              ms += in_class(z, cmask[i][r]) ? 1u : 0u;
            } else {
              q = tcur[i][r] - z;
            }
            if constexpr (!kFull) q = (nw0 + i * 16 + row_in_block(r) < N) ? q : Acc(0);
            loc = sq_acc(q, loc);
          }
        sse[j] += (double)loc;
        miss[j] += ms;
      }
    };
    // the bias is added as 0 without a bias gene (z = +-0 give the same
    // error and miss); a separate no-bias variant measured slower
    if (full) epilogue(std::true_type{});
    else epilogue(std::false_type{});
  }

  __builtin_amdgcn_s_setprio(0);
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    sse[j] += __shfl_xor(sse[j], 16);
    sse[j] += __shfl_xor(sse[j], 32);
    miss[j] += __shfl_xor(miss[j], 16);
    miss[j] += __shfl_xor(miss[j], 32);
  }
  if (lgrp == 0) {
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      s_sse[wave][j * 16 + lrow] = sse[j];
      s_miss[wave][j * 16 + lrow] = miss[j];
    }
  }
  __syncthreads();
  if (tid < TP) {
    const int64_t o = (int64_t)wr * part_ld + p0 + tid;
    st_agent(part_sse + o, ((s_sse[0][tid] + s_sse[1][tid]) + s_sse[2][tid]) + s_sse[3][tid]);
    st_agent(part_miss + o, s_miss[0][tid] + s_miss[1][tid] + s_miss[2][tid] + s_miss[3][tid]);
  }
}

template <class Tr, bool kCls, int WN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void fitness_lds_kernel(
    const typename Tr::T* __restrict__ phi, const typename Tr::T* __restrict__ tile,
    const typename Tr::Acc* __restrict__ biasv, const typename Tr::Acc* __restrict__ tvec,
    int64_t N, int M_pad, int ldsw, int n_pt, int n_ranges, int64_t n_items, int cpx, int ub,
    int part_ld, double* __restrict__ part_sse, uint32_t* __restrict__ part_miss,
    const DevState* st, const FitTail tail) {
  extern __shared__ __align__(16) uint32_t lds[];
  if (run_halted(st)) return;
  const int64_t nwg = gridDim.x;
  const int64_t w = blockIdx.x;
  const int64_t lt = (w & 7) * (nwg >> 3) + (w >> 3);
  if (lt >= n_items) return;
  const int pt = (int)(lt % n_pt);
  const int wr = (int)(lt / n_pt);
  lds_item<Tr, kCls, WN, 2>(phi, tile, biasv, tvec, N, M_pad, ldsw, n_ranges, pt, wr,
                            ub, item_rot(lt, n_items, cpx, ub), part_ld, part_sse, part_miss,
                            lds);
  fitness_tail<16 * WN>(tail, pt, n_pt, n_ranges, part_ld, part_sse, part_miss);
}

// Batched form: one persistent launch advances many independent runs, each
// at its own pace.  A run moves through three phases per generation:
// fitness (its chromosome tile x row range items, each with the tail above,
// so the last item ranks the population, tracks the best and applies the
// stop rule), the roulette wheel or full ranking (one item, wheel selections
// only) and the breed (its breed workgroups).  Per run, a 64-bit word holds
// the phase epoch and the count of items claimed in it; a workgroup claims
// an item by an atomic add on the word and takes the epoch the add returns,
// so a claim is always for the phase it names.  Items of a phase never wait
// for anything: the workgroup that finishes a phase's last item opens the
// run's next phase (or parks the run: stopped, evaluation only, or its
// generations for this launch bred).  A workgroup takes an item of the run
// with the earliest deadline among those with open items; a generation's
// deadline is the time it opened plus the time the run's generation would
// take with 1/n of the device (earliest-deadline-first on fair-share
// deadlines: runs share the device in proportion to their work, so a run's
// generation takes about its own work times the runs in flight, and no run
// starves).  Every value
// one phase hands to the next (population, gene tile, fitness, ranking,
// wheel, state, counters) is written and read at device scope, since the
// phases of a run land on workgroups of different XCDs.  An item is the
// single-context kernels' work, so a run's results equal its results alone
// with the same tile width and row ranges.  Exit: every run parked, or no
// open item for idle_ticks of the wall clock (error flag; bounds a lost
// hand-off).
constexpr uint32_t kParked = 0xFFFFFFFFu;


// Items of run r in epoch e: all of them (completion count), and those
// claimed through the run's word (wheel and breed phases) or through XCD
// slice x (fitness phase: slice x holds the row ranges
// [x n_ranges / 8, (x + 1) n_ranges / 8), every chromosome tile of each, so
// the tiles that share a range's Phi rows run on one XCD and share its L2).
__device__ __forceinline__ uint32_t flow_count(const FlowRun& r, uint32_t e) {
  if (e == kParked) return 0u;
  const uint32_t ph = e % 3u;
  return ph == 0u ? (uint32_t)r.n_fit : ph == 1u ? 1u : (uint32_t)r.n_breed;
}
__device__ __forceinline__ uint32_t flow_word_count(const FlowRun& r, uint32_t e) {
  return e == kParked || e % 3u == 0u ? 0u : flow_count(r, e);
}
__device__ __forceinline__ int slice_lo(const FlowRun& r, int x) { return x * r.n_ranges / kXcds; }
__device__ __forceinline__ uint32_t flow_slice_count(const FlowRun& r, uint32_t e, int x) {
  if (e == kParked || e % 3u != 0u) return 0u;
  return (uint32_t)((slice_lo(r, x + 1) - slice_lo(r, x)) * r.n_pt);
}

// Run r finished epoch e: open its next phase or park it (thread 0 of the
// workgroup that finished the epoch's last item).
__device__ __forceinline__ void flow_advance(const FlowRun& r, FlowCtl* c, FlowQueue* q, uint32_t e, int eval_only) {
  const uint32_t ph = e % 3u;
  // every item of epoch e is claimed and finished: the count restarts before
  // any item of the next phase can be claimed (and counted)
  st_agent(&c->done, 0u);
  agent_stores_done();
  uint32_t next;
  if (ph == 0u) {
    const bool halted = ld_agent(&r.st->run_active) != 0 && ld_agent(&r.st->stopped) != 0;
    next = (eval_only || halted) ? kParked : e + (r.sel != GAME_SEL_TOURNAMENT ? 1u : 2u);
  } else if (ph == 1u) {
    next = e + 1u;
  } else {
    const int32_t g = ld_agent(&c->gen) + 1, rel = ld_agent(&c->rel), left = ld_agent(&c->left) - 1;
    st_agent(&r.st->generation, g);
    st_agent(&c->gen, g);
    st_agent(&c->rel, rel + 1);
    st_agent(&c->left, left);
    const uint64_t now = wall_clock64();
    if (rel < r.t_cap) st_agent(r.t_done + rel, now);
    if (left > 0) {
      next = e + 1u;
      st_agent(&c->deadline, now + r.span);
      if (rel + 1 < r.t_cap) st_agent(r.t_start + rel + 1, now);
    } else {
      next = kParked;  // this launch's generations are bred; the next launch resumes
    }
  }
  // Everything above is visible before the next phase's items can be
  // claimed.  Opening them is this thread's last action on the run: once
  // they are open, the phase may finish and the next transition begin at
  // any moment, so the word must already name the phase (the fitness
  // phase's items are claimed through the slices, opened after the word).
  agent_stores_done();
  __hip_atomic_exchange(&c->word, (uint64_t)next << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (next == kParked) {
    atomicSub(&q->active, 1u);
  } else if (next % 3u == 0u) {
    agent_stores_done();
    for (int x = 0; x < kXcds; ++x) st_agent(&c->xw[x], (uint64_t)next << 32);
  }
}

// Wave 0's search for an item (lane 0 returns the claim): the run with the
// earliest deadline among those with an open item in this XCD's slice or in
// the run's word; failing that, any open slice of the earliest-deadline run
// (an idle XCD takes over another XCD's ranges).  Claims are atomic adds on
// the slice or word, valid for the epoch the add returns.
struct Claim {
  int run, slice;  // slice -1: the run's word
  uint32_t epoch, item;
};
__device__ __forceinline__ void min_deadline(uint64_t& dl, int& idx, int& sl) {
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t odl = __shfl_xor(dl, off);
    const int oidx = __shfl_xor(idx, off), osl = __shfl_xor(sl, off);
    if (oidx >= 0 && (idx < 0 || odl < dl || (odl == dl && (oidx < idx || (oidx == idx && osl < sl))))) {
      dl = odl;
      idx = oidx;
      sl = osl;
    }
  }
}

__device__ __forceinline__ bool flow_claim(const FlowRun* __restrict__ runs, int n_runs, FlowCtl* ctl, int xcd,
                                           Claim* out) {
  const int lane = threadIdx.x & 63;
  uint64_t best_dl = ~0ull;
  int found = -1, fslice = -1;
  for (int base = 0; base < n_runs; base += 64) {
    const int r = base + lane;
    uint64_t dl = ~0ull;
    int idx = -1, sl = -1;
    if (r < n_runs) {
      const uint64_t w = ld_agent(&ctl[r].word);
      const uint32_t e = (uint32_t)(w >> 32);
      bool open = (uint32_t)w < flow_word_count(runs[r], e);
      if (!open && e != kParked && e % 3u == 0u) {
        const uint64_t xw = ld_agent(&ctl[r].xw[xcd]);
        open = (uint32_t)xw < flow_slice_count(runs[r], (uint32_t)(xw >> 32), xcd);
        sl = xcd;
      }
      if (open) {
        dl = ld_agent(&ctl[r].deadline);
        idx = r;
      }
    }
    min_deadline(dl, idx, sl);
    if (idx >= 0 && (found < 0 || dl < best_dl)) {
      best_dl = dl;
      found = idx;
      fslice = sl;
    }
  }
  if (found < 0) {
    // steal: every (run, slice) pair of runs in a fitness phase
    for (int base = 0; base < n_runs * kXcds; base += 64) {
      const int pidx = base + lane, r = pidx / kXcds, x = pidx % kXcds;
      uint64_t dl = ~0ull;
      int idx = -1, sl = -1;
      if (r < n_runs) {
        const uint64_t xw = ld_agent(&ctl[r].xw[x]);
        if ((uint32_t)xw < flow_slice_count(runs[r], (uint32_t)(xw >> 32), x)) {
          dl = ld_agent(&ctl[r].deadline);
          idx = r;
          sl = x;
        }
      }
      min_deadline(dl, idx, sl);
      if (idx >= 0 && (found < 0 || dl < best_dl)) {
        best_dl = dl;
        found = idx;
        fslice = sl;
      }
    }
  }
  if (found < 0 || lane != 0) return false;
  const FlowRun& r = runs[found];
  if (fslice < 0) {
    const uint64_t old = __hip_atomic_fetch_add(&ctl[found].word, 1ull, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t e = (uint32_t)(old >> 32), i = (uint32_t)old;
    if (i >= flow_word_count(r, e)) return false;
    *out = Claim{found, -1, e, i};
    return true;
  }
  const uint64_t old = __hip_atomic_fetch_add(&ctl[found].xw[fslice], 1ull, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t e = (uint32_t)(old >> 32), i = (uint32_t)old;
  if (i >= flow_slice_count(r, e, fslice)) return false;
  // slice-local item -> the run's item number (chromosome tile fastest)
  *out = Claim{found, fslice, e, (uint32_t)(slice_lo(r, fslice) * r.n_pt) + i};
  return true;
}

template <class Tr, class O>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void flow_kernel(
    const FlowRun* __restrict__ runs, int n_runs, FlowCtl* ctl, FlowQueue* q, int eval_only, int cpx,
    uint64_t idle_ticks) {
  using T = typename Tr::T;
  using Acc = typename Tr::Acc;
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ int s_state, s_run, s_gen;  // s_state: 0 item claimed, 1 none open, 2 leave
  __shared__ uint32_t s_epoch, s_idx;
  __shared__ int s_last;
  const int xcd = (int)(blockIdx.x % kXcds);
  uint64_t idle_since = 0;
  for (;;) {
    __syncthreads();  // the previous item's LDS is no longer read
    if (threadIdx.x < 64) {
      Claim cl{};
      const bool got = flow_claim(runs, n_runs, ctl, xcd, &cl);
      if (threadIdx.x == 0) {
        int state = 1;
        if (got) {
          state = 0;
          s_run = cl.run;
          s_epoch = cl.epoch;
          s_idx = cl.item;
          s_gen = ld_agent(&ctl[cl.run].gen);
        } else if (ld_agent(&q->active) == 0u || ld_agent(&q->error) != 0u) {
          state = 2;
        }
        // the idle clock is thread 0's alone, so the whole workgroup leaves together
        if (state == 1) {
          const uint64_t now = wall_clock64();
          if (idle_since == 0) {
            idle_since = now;
          } else if (now - idle_since > idle_ticks) {
            atomicOr(&q->error, 1u);
            state = 2;
          }
        } else {
          idle_since = 0;
        }
        s_state = state;
      }
    }
    __syncthreads();
    const int state = s_state;
    if (state == 2) break;
    if (state == 1) {
      __builtin_amdgcn_s_sleep(8);
      continue;
    }
    // the claim is the same for every lane; saying so keeps the run's
    // parameters, and the item's loop bounds, in scalar registers
    const int ri = __builtin_amdgcn_readfirstlane(s_run);
    const uint32_t e = __builtin_amdgcn_readfirstlane(s_epoch);
    const uint32_t item = __builtin_amdgcn_readfirstlane(s_idx);
    const FlowRun& r = runs[ri];
    const uint32_t ph = e % 3u;
    if (ph == 0u) {
      const int pt = (int)(item % (uint32_t)r.n_pt);
      const int wr = (int)(item / (uint32_t)r.n_pt);
      const T* phi = static_cast<const T*>(r.phi);
      const T* tile = static_cast<const T*>(r.tile);
      const Acc* biasv = static_cast<const Acc*>(r.biasv);
      const Acc* tvec = static_cast<const Acc*>(r.tvec);
      double* psse = r.psse;
      uint32_t* pmiss = r.pmiss;
#define GAME_FLOW_ITEM(CLS, WN)                                                                   \
  do {                                                                                            \
    lds_item<Tr, CLS, WN, 2, true>(phi, tile, biasv, tvec, r.N, r.M_pad, r.ldsw, r.n_ranges, pt,  \
                                   wr, r.ub, item_rot(item, r.n_fit, cpx, r.ub), r.part_ld,       \
                                   psse, pmiss, lds);                                             \
    fitness_tail<16 * WN, true>(r.tail, pt, r.n_pt, r.n_ranges, r.part_ld, psse, pmiss);          \
  } while (0)
      if (r.task == GAME_CLASSIFICATION) {
        if (r.tile_p == 128) GAME_FLOW_ITEM(true, 8);
        else if (r.tile_p == 64) GAME_FLOW_ITEM(true, 4);
        else GAME_FLOW_ITEM(true, 2);
      } else {
        if (r.tile_p == 128) GAME_FLOW_ITEM(false, 8);
        else if (r.tile_p == 64) GAME_FLOW_ITEM(false, 4);
        else GAME_FLOW_ITEM(false, 2);
      }
#undef GAME_FLOW_ITEM
    } else if (ph == 1u) {
      if (r.sel == GAME_SEL_ROULETTE)
        wheel_block<256, true>(r.tail.fit, r.tail.P, r.wheel);
      else
        rank_block<256, true>(r.tail.fit, r.tail.P, r.rank_pow2, reinterpret_cast<int*>(r.wheel),
                              reinterpret_cast<unsigned char*>(lds));
    } else {
      breed_work<O, float, true>(r.breed, (int)item, (uint32_t)__builtin_amdgcn_readfirstlane(s_gen));
    }
    // every store of the item is acknowledged before its completion counts
    agent_stores_done();
    __syncthreads();
    if (threadIdx.x == 0)
      s_last = atomicAdd(&ctl[ri].done, 1u) + 1u == flow_count(r, e);
    __syncthreads();
    if (s_last && threadIdx.x == 0) flow_advance(r, &ctl[ri], q, e, eval_only);
  }
}

// Before a launch: open the fitness phase of every run that has not stopped
// (park the others), note the generation and the start time, count the runs
// with work.  first: the start of a batch run (timestamp slots restart).
__global__ void flow_arm_kernel(const FlowRun* __restrict__ runs, int n_runs, FlowCtl* ctl, FlowQueue* q,
                                int chunk, int first, int eval_only) {
  __shared__ uint32_t s_active[256];
  uint32_t act = 0;
  const uint64_t now = wall_clock64();
  for (int i = threadIdx.x; i < n_runs; i += 256) {
    const FlowRun& r = runs[i];
    const bool halted = run_halted(r.st);
    FlowCtl& c = ctl[i];
    // epoch 0 (the fitness phase) opens in the word and the slices; a
    // stopped run stays closed in both
    const uint64_t open = halted ? (uint64_t)kParked << 32 : 0ull;
    c.word = open;
    for (int x = 0; x < kXcds; ++x) c.xw[x] = open;
    c.deadline = now + r.span;
    c.done = 0u;
    c.gen = r.st->generation;
    c.left = chunk;
    if (first) c.rel = 0;
    if (!halted && !eval_only && c.rel < r.t_cap) r.t_start[c.rel] = now;
    act += halted ? 0u : 1u;
  }
  s_active[threadIdx.x] = act;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int i = 0; i < 256; ++i) tot += s_active[i];
    q->active = tot;
    q->error = 0u;
  }
}

// After a launch: how many runs have not stopped.
__global__ void flow_status_kernel(const FlowRun* __restrict__ runs, int n_runs, FlowQueue* q) {
  __shared__ uint32_t s_run[256];
  uint32_t n = 0;
  for (int i = threadIdx.x; i < n_runs; i += 256) n += run_halted(runs[i].st) ? 0u : 1u;
  s_run[threadIdx.x] = n;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int i = 0; i < 256; ++i) tot += s_run[i];
    q->running = tot;
  }
}

template <class Tr, int WM, int WN>
hipError_t launch_tr(int task, const FitnessGeom& g, const Plan& p, const void* phi,
                     const void* tile, const void* biasv, const void* tvec, double* psse,
                     uint32_t* pmiss, const DevState* st, const FitTail& tail, hipStream_t s) {
  using T = typename Tr::T;
  using Acc = typename Tr::Acc;
  if (task == GAME_CLASSIFICATION)
    hipLaunchKernelGGL((fitness_kernel<Tr, WM, WN, true>), dim3((unsigned)g.grid), dim3(256), 0, s,
                       (const T*)phi, (const T*)tile, (const Acc*)biasv, (const Acc*)tvec, p.N,
                       p.M_pad, p.n_rt, g.n_pt, g.rt_per_wg, g.n_items, p.P_max_pad, psse, pmiss,
                       st, tail);
  else
    hipLaunchKernelGGL((fitness_kernel<Tr, WM, WN, false>), dim3((unsigned)g.grid), dim3(256), 0,
                       s, (const T*)phi, (const T*)tile, (const Acc*)biasv, (const Acc*)tvec, p.N,
                       p.M_pad, p.n_rt, g.n_pt, g.rt_per_wg, g.n_items, p.P_max_pad, psse, pmiss,
                       st, tail);
  return hipGetLastError();
}

// LDS words per staged gene row: the tile is stored dense (K-block-major,
// see lds_item), so a row is its M_pad elements.
template <class Tr>
int lds_stride_words(int M_pad) {
  return M_pad * (int)sizeof(typename Tr::T) / 4;
}

// Dynamic LDS of one LDS-kernel workgroup: gene tile plus column sums.
template <class Tr>
size_t lds_bytes(int M_pad, int tp) {
  return (size_t)tp * lds_stride_words<Tr>(M_pad) * 4 + (size_t)tp * 48;
}
constexpr size_t kLdsMax = 98304;  // dynamic LDS one workgroup may take

template <class Tr, int WN>
auto lds_kernel_wn(int task) {
  return task == GAME_CLASSIFICATION ? fitness_lds_kernel<Tr, true, WN> : fitness_lds_kernel<Tr, false, WN>;
}
template <class Tr>
const void* lds_kernel_for(int task, int tp) {
  if (tp == 128) return reinterpret_cast<const void*>(lds_kernel_wn<Tr, 8>(task));
  if (tp == 64) return reinterpret_cast<const void*>(lds_kernel_wn<Tr, 4>(task));
  return reinterpret_cast<const void*>(lds_kernel_wn<Tr, 2>(task));
}
int tp_index(int tp) { return tp == 128 ? 0 : tp == 64 ? 1 : 2; }

// Dynamic LDS above 64 KiB has to be enabled per kernel once.
template <class Tr>
hipError_t lds_prepare(int task, int tp) {
  static bool done[2][3] = {};
  const int ai = task == GAME_CLASSIFICATION ? 1 : 0, ti = tp_index(tp);
  if (done[ai][ti]) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(lds_kernel_for<Tr>(task, tp),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
  if (e == hipSuccess) done[ai][ti] = true;
  return e;
}

int device_cus();
int cus_per_xcd();

template <class Tr, int WN>
hipError_t launch_lds_wn(int task, const FitnessGeom& g, const Plan& p, const void* phi,
                         const void* tile, const void* biasv, const void* tvec, double* psse,
                         uint32_t* pmiss, const DevState* st, const FitTail& tail, hipStream_t s) {
  using T = typename Tr::T;
  using Acc = typename Tr::Acc;
  const int ldsw = lds_stride_words<Tr>(p.M_pad);
  const size_t lds = lds_bytes<Tr>(p.M_pad, 16 * WN);
  const hipError_t e = lds_prepare<Tr>(task, 16 * WN);
  if (e != hipSuccess) return e;
  if (task == GAME_CLASSIFICATION)
    hipLaunchKernelGGL((fitness_lds_kernel<Tr, true, WN>), dim3((unsigned)g.grid), dim3(256), lds, s,
                       (const T*)phi, (const T*)tile, (const Acc*)biasv, (const Acc*)tvec, p.N,
                       p.M_pad, ldsw, g.n_pt, (int)g.n_rg, g.n_items, cus_per_xcd(), g.ub, p.P_max_pad, psse,
                       pmiss, st, tail);
  else
    hipLaunchKernelGGL((fitness_lds_kernel<Tr, false, WN>), dim3((unsigned)g.grid), dim3(256), lds,
                       s, (const T*)phi, (const T*)tile, (const Acc*)biasv, (const Acc*)tvec, p.N,
                       p.M_pad, ldsw, g.n_pt, (int)g.n_rg, g.n_items, cus_per_xcd(), g.ub, p.P_max_pad, psse,
                       pmiss, st, tail);
  return hipGetLastError();
}

template <class Tr>
hipError_t launch_lds(int task, const FitnessGeom& g, const Plan& p, const void* phi,
                      const void* tile, const void* biasv, const void* tvec, double* psse,
                      uint32_t* pmiss, const DevState* st, const FitTail& tail, hipStream_t s) {
  switch (p.tile_p) {
    case 128:
      return launch_lds_wn<Tr, 8>(task, g, p, phi, tile, biasv, tvec, psse, pmiss, st, tail, s);
    case 64:
      return launch_lds_wn<Tr, 4>(task, g, p, phi, tile, biasv, tvec, psse, pmiss, st, tail, s);
    case 32:
      return launch_lds_wn<Tr, 2>(task, g, p, phi, tile, biasv, tvec, psse, pmiss, st, tail, s);
  }
  return hipErrorInvalidValue;
}

int device_cus() {
  static int cus = 0;
  if (cus) return cus;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
  return cus;
}

// CUs of one of the 8 XCDs (the dispatcher's unit of workgroup placement).
int cus_per_xcd() {
  const int c = device_cus() / 8;
  return c > 0 ? c : 1;
}

// Workgroups of an LDS kernel that are resident at once on the device.
template <class Tr>
int lds_resident(int task, int M_pad, int tp) {
  static int cache[2][3][8192 / 8 + 1] = {};
  const int ai = task == GAME_CLASSIFICATION ? 1 : 0, ti = tp_index(tp);
  const int ci = M_pad / 8 < 1024 ? M_pad / 8 : 1024;
  if (cache[ai][ti][ci]) return cache[ai][ti][ci];
  if (lds_prepare<Tr>(task, tp) != hipSuccess) return 0;
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, lds_kernel_for<Tr>(task, tp), 256,
                                                   lds_bytes<Tr>(M_pad, tp)) != hipSuccess)
    return 0;
  cache[ai][ti][ci] = blocks * device_cus();
  return cache[ai][ti][ci];
}

template <class Tr>
bool lds_fits(int M_pad, int tp) {
  return lds_bytes<Tr>(M_pad, tp) <= kLdsMax;
}

}  // namespace

size_t fitness_lds_bytes(int dtype, int M_pad, int tp) {
  switch (dtype) {
    case GAME_F32: return lds_bytes<F32Tr>(M_pad, tp);
    case GAME_BF16: return lds_bytes<BF16Tr>(M_pad, tp);
    case GAME_F16: return lds_bytes<F16Tr>(M_pad, tp);
  }
  return 0;
}

int fitness_lds_stride(int dtype, int M_pad) {
  switch (dtype) {
    case GAME_F32: return lds_stride_words<F32Tr>(M_pad);
    case GAME_BF16: return lds_stride_words<BF16Tr>(M_pad);
    case GAME_F16: return lds_stride_words<F16Tr>(M_pad);
  }
  return 0;
}

int fitness_lds_fits(int dtype, int M_pad, int tp) {
  if (tp != 128 && tp != 64 && tp != 32) return 0;
  switch (dtype) {
    case GAME_F32: return lds_fits<F32Tr>(M_pad, tp);
    case GAME_BF16: return lds_fits<BF16Tr>(M_pad, tp);
    case GAME_F16: return lds_fits<F16Tr>(M_pad, tp);
  }
  return 0;
}

namespace {
template <class Tr, class O>
hipError_t flow_prepare() {
  static bool done = false;
  if (done) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(flow_kernel<Tr, O>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
  if (e == hipSuccess) done = true;
  return e;
}

template <class Tr, class O>
int flow_slots_tr(size_t lds) {
  if (flow_prepare<Tr, O>() != hipSuccess) return 0;
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &blocks, reinterpret_cast<const void*>(flow_kernel<Tr, O>), 256, lds) != hipSuccess)
    return 0;
  return blocks * device_cus();
}

template <class Tr, class O>
hipError_t flow_launch(const FlowRun* runs, int n_runs, FlowCtl* ctl, FlowQueue* q, int grid, size_t lds,
                       int chunk, int first, int eval_only, uint64_t idle_ticks, hipStream_t s) {
  const hipError_t e = flow_prepare<Tr, O>();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(flow_arm_kernel, dim3(1), dim3(256), 0, s, runs, n_runs, ctl, q, chunk, first,
                     eval_only);
  hipLaunchKernelGGL((flow_kernel<Tr, O>), dim3((unsigned)grid), dim3(256), lds, s, runs, n_runs, ctl, q,
                     eval_only, cus_per_xcd(), idle_ticks);
  hipLaunchKernelGGL(flow_status_kernel, dim3(1), dim3(256), 0, s, runs, n_runs, q);
  return hipGetLastError();
}
}  // namespace

int flow_slots(int dtype, size_t lds) {
  if (lds > kLdsMax) return 0;
  switch (dtype) {
    case GAME_F32: return flow_slots_tr<F32Tr, float>(lds);
    case GAME_BF16: return flow_slots_tr<BF16Tr, uint16_t>(lds);
    case GAME_F16: return flow_slots_tr<F16Tr, _Float16>(lds);
  }
  return 0;
}

hipError_t launch_flow(int dtype, const FlowRun* runs, int n_runs, FlowCtl* ctl, FlowQueue* q,
                       int grid, size_t lds, int chunk, int first, int eval_only, uint64_t idle_ticks,
                       hipStream_t s) {
  switch (dtype) {
    case GAME_F32:
      return flow_launch<F32Tr, float>(runs, n_runs, ctl, q, grid, lds, chunk, first, eval_only, idle_ticks, s);
    case GAME_BF16:
      return flow_launch<BF16Tr, uint16_t>(runs, n_runs, ctl, q, grid, lds, chunk, first, eval_only,
                                           idle_ticks, s);
    case GAME_F16:
      return flow_launch<F16Tr, _Float16>(runs, n_runs, ctl, q, grid, lds, chunk, first, eval_only,
                                          idle_ticks, s);
  }
  return hipErrorInvalidValue;
}

// Range boundary block for the LDS kernels (see lds_item): 1 when 32-row
// units with rotated extra units leave the busiest SIMD fewer units than
// whole 128-row tiles, else 4.  Placement model: all items resident at once,
// item lt on XCD lt / per and CU (lt % per) % cpx of it, wave w of every item
// on SIMD w.  With more items than resident workgroups there is no fixed
// placement, and tiles are kept.
int fitness_range_block(int64_t N, int64_t n_rg, int n_pt, int slots) {
  const int64_t n_items = n_rg * n_pt;
  if (slots <= 0 || n_items > slots || n_rg < 1) return 4;
  // a context asks again for every launch it enqueues: keep the last answer
  struct Memo {
    int64_t N, n_rg;
    int n_pt, slots, ub;
  };
  static thread_local Memo memo{-1, -1, -1, -1, 4};
  if (memo.N == N && memo.n_rg == n_rg && memo.n_pt == n_pt && memo.slots == slots) return memo.ub;
  const int cpx = cus_per_xcd();
  const int64_t n_units = (N + 31) / 32, per = (n_items + 7) / 8;
  int64_t worst[2] = {0, 0};
  std::vector<int64_t> load((size_t)8 * cpx * 4);
  for (int m = 0; m < 2; ++m) {
    const int ub = m == 0 ? 4 : 1;
    const int64_t n_blk = (n_units + ub - 1) / ub;
    std::fill(load.begin(), load.end(), 0);
    for (int64_t lt = 0; lt < n_items; ++lt) {
      const int64_t wr = lt / n_pt, k = lt % per;
      const int rot = ub == 1 ? 2 * (int)((k / cpx) & 1) : 0;
      const int64_t b = wr * n_blk / n_rg * ub, e = std::min(n_units, (wr + 1) * n_blk / n_rg * ub);
      const size_t cu = (size_t)(lt / per) * cpx + (size_t)(k % cpx);
      for (int w = 0; w < 4; ++w) {
        const int64_t f = b + ((w + rot) & 3);
        load[cu * 4 + w] += f < e ? (e - f + 3) / 4 : 0;
      }
    }
    worst[m] = *std::max_element(load.begin(), load.end());
  }
  memo = Memo{N, n_rg, n_pt, slots, worst[1] < worst[0] ? 1 : 4};
  return memo.ub;
}

int fitness_persistent_slots(const Plan& p, int task, int dtype) {
  if (!p.lds) return 0;
  switch (dtype) {
    case GAME_F32: return lds_resident<F32Tr>(task, p.M_pad, p.tile_p);
    case GAME_BF16: return lds_resident<BF16Tr>(task, p.M_pad, p.tile_p);
    case GAME_F16: return lds_resident<F16Tr>(task, p.M_pad, p.tile_p);
  }
  return 0;
}

hipError_t launch_fitness(const Plan& p, int task, int dtype, const FitnessGeom& g, const void* phi,
                          const void* tile, const void* biasv, const void* tvec, double* psse,
                          uint32_t* pmiss, const DevState* st, const FitTail& tail,
                          hipStream_t s) {
  switch (dtype) {
    case GAME_F64:
      return launch_tr<F64Tr, 2, 2>(task, g, p, phi, tile, biasv, tvec, psse, pmiss, st, tail, s);
    case GAME_F32:
      if (p.lds)
        return launch_lds<F32Tr>(task, g, p, phi, tile, biasv, tvec, psse, pmiss, st, tail, s);
      return launch_tr<F32Tr, 4, 4>(task, g, p, phi, tile, biasv, tvec, psse, pmiss, st, tail, s);
    case GAME_BF16:
      if (p.lds)
        return launch_lds<BF16Tr>(task, g, p, phi, tile, biasv, tvec, psse, pmiss, st, tail, s);
      return launch_tr<BF16Tr, 4, 4>(task, g, p, phi, tile, biasv, tvec, psse, pmiss, st, tail, s);
    case GAME_F16:
      if (p.lds)
        return launch_lds<F16Tr>(task, g, p, phi, tile, biasv, tvec, psse, pmiss, st, tail, s);
      return launch_tr<F16Tr, 4, 4>(task, g, p, phi, tile, biasv, tvec, psse, pmiss, st, tail, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace game
