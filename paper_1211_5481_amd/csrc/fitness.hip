// Population fitness: z = Phi . G^T on MFMA with the error reduction fused in.
//
// For every chromosome p and pattern n (eq. 2 and 3):
//   z[n,p]  = sum_m Phi[n,m] G[p,m] (+ a_0 of p)
//   e[n,p]  = (t_n - out)^2,  out = z (regression) or 1/(1+exp(-z)) (classification)
//   miss    = [(z >= 0) != (t_n >= 0.5)]            (classification)
// and per chromosome sse = sum_n e, misses = sum_n miss, reduced to
// mse = sse / N and fitness = 1 - mse by reduce_kernel.
//
// Work decomposition (one workgroup = 4 waves of 64 lanes, 2 x 2):
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
//     part_sse[row_group][p] (double) and part_miss (uint32); no atomics, so
//     every run is bit-reproducible;
//   * workgroups sharing a row group run back to back on one XCD (the
//     dispatcher deals workgroups round-robin over the 8 XCDs; the logical
//     tile index is remapped so each XCD gets a contiguous range), so the
//     Phi rows they share hit that XCD's L2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "game_internal.hpp"

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
  __device__ static AccV mma(const Ld& a, const Ld& b, AccV c) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, c, 0, 0, 0);
    return c;
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
  __device__ static AccV mma(const Ld& a, const Ld& b, AccV c) {
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, c, 0, 0, 0);
    return c;
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
  __device__ static AccV mma(const Ld& a, const Ld& b, AccV c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8h, a),
                                                  __builtin_bit_cast(v8h, b), c, 0, 0, 0);
  }
};

__device__ __forceinline__ float sigmoid_acc(float z) {
  // 1 / (1 + 2^(-z log2 e)); v_exp_f32 and v_rcp_f32 (about 1 ulp each)
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-z * 1.4426950408889634f));
}
__device__ __forceinline__ double sigmoid_acc(double z) { return 1.0 / (1.0 + exp(-z)); }

template <class Tr, int WM, int WN, bool kCls>
__global__ __launch_bounds__(256) void fitness_kernel(
    const typename Tr::T* __restrict__ phi, const typename Tr::T* __restrict__ tile,
    const typename Tr::Acc* __restrict__ biasv, const typename Tr::Acc* __restrict__ tvec,
    int64_t N, int M_pad, int64_t n_rt, int n_pt, int rt_per_wg, int64_t n_items, int part_ld,
    double* __restrict__ part_sse, uint32_t* __restrict__ part_miss, const DevState* st) {
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
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = Tr::mma(a[i], b[j], acc[i][j]);
    };
    load(a0, b0, 0);
    int kb = 0;
    for (; kb + 1 < KB; kb += 2) {
      load(a1, b1, kb + 1);
      mma_all(a0, b0);
      if (kb + 2 < KB) load(a0, b0, kb + 2);
      mma_all(a1, b1);
    }
    if (kb < KB) mma_all(a0, b0);

    // epilogue: accumulator element r of block (i, j) is pattern
    // nw0 + 16 i + row_in_block(r) and chromosome pw0 + 16 j + lrow
    auto row_in_block = [&](int r) { return Tr::kRowInterleave ? lgrp + 4 * r : 4 * lgrp + r; };
    const bool full = (rt + 1) * TN <= N;
    Acc tv[WM][4];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) tv[i][r] = tvec[nw0 + i * 16 + row_in_block(r)];
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      Acc loc = Acc(0);
      uint32_t ms = 0u;
#pragma unroll
      for (int i = 0; i < WM; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const Acc z = acc[i][j][r] + bias_j[j];
          const Acc t = tv[i][r];
          Acc e;
          bool m = false;
          if constexpr (kCls) {
            const Acc d = t - sigmoid_acc(z);
            e = d * d;
            m = (z >= Acc(0)) != (t >= Acc(0.5));
          } else {
            const Acc d = t - z;
            e = d * d;
          }
          if (!full) {
            const bool valid = nw0 + i * 16 + row_in_block(r) < N;
            e = valid ? e : Acc(0);
            m = m && valid;
          }
          loc += e;
          ms += m ? 1u : 0u;
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
    part_sse[o] = s_sse[0][c] + s_sse[1][c];
    part_miss[o] = s_miss[0][c] + s_miss[1][c];
  }
}

// Fixed-order sum of the row-group partials: 16 chromosomes x 16 segments per
// workgroup; segments are contiguous row-group ranges added in index order.
__global__ __launch_bounds__(256) void reduce_kernel(int64_t n_rg, int part_ld, int P, double invN,
                                                     const double* __restrict__ psse,
                                                     const uint32_t* __restrict__ pmiss,
                                                     double* mse, double* miscls, double* fit,
                                                     double* mse2, double* miscls2, double* fit2,
                                                     const DevState* st) {
  if (run_halted(st)) return;
  const int c = threadIdx.x & 15, seg = threadIdx.x >> 4;
  const int p = blockIdx.x * 16 + c;
  const int64_t chunk = (n_rg + 15) / 16;
  const int64_t b = seg * chunk, e = min(n_rg, b + chunk);
  double s = 0.0;
  uint64_t m = 0;
  if (p < P) {
    for (int64_t r = b; r < e; ++r) {
      s += psse[r * part_ld + p];
      m += pmiss[r * part_ld + p];
    }
  }
  __shared__ double ss[16][16];
  __shared__ uint64_t sm[16][16];
  ss[seg][c] = s;
  sm[seg][c] = m;
  __syncthreads();
  if (seg == 0 && p < P) {
    double tot = 0.0;
    uint64_t mt = 0;
    for (int q = 0; q < 16; ++q) {
      tot += ss[q][c];
      mt += sm[q][c];
    }
    const double ms = tot * invN;
    const double mc = (double)mt * invN;
    const double f = 1.0 - ms;
    if (mse) mse[p] = ms;
    if (miscls) miscls[p] = mc;
    if (fit) fit[p] = f;
    if (mse2) mse2[p] = ms;
    if (miscls2) miscls2[p] = mc;
    if (fit2) fit2[p] = f;
  }
}

template <class Tr, int WM, int WN>
hipError_t launch_tr(int task, const FitnessGeom& g, const Plan& p, const void* phi,
                     const void* tile, const void* biasv, const void* tvec, double* psse,
                     uint32_t* pmiss, const DevState* st, hipStream_t s) {
  using T = typename Tr::T;
  using Acc = typename Tr::Acc;
  if (task == GAME_CLASSIFICATION)
    hipLaunchKernelGGL((fitness_kernel<Tr, WM, WN, true>), dim3((unsigned)g.grid), dim3(256), 0, s,
                       (const T*)phi, (const T*)tile, (const Acc*)biasv, (const Acc*)tvec, p.N,
                       p.M_pad, p.n_rt, g.n_pt, g.rt_per_wg, g.n_items, p.P_max_pad, psse, pmiss,
                       st);
  else
    hipLaunchKernelGGL((fitness_kernel<Tr, WM, WN, false>), dim3((unsigned)g.grid), dim3(256), 0,
                       s, (const T*)phi, (const T*)tile, (const Acc*)biasv, (const Acc*)tvec, p.N,
                       p.M_pad, p.n_rt, g.n_pt, g.rt_per_wg, g.n_items, p.P_max_pad, psse, pmiss,
                       st);
  return hipGetLastError();
}

}  // namespace

// Workgroup tile per dtype: rows x chromosomes = (32 WM) x (32 WN).
void fitness_tile(int dtype, int* tile_n, int* tile_p) {
  if (dtype == GAME_F64) {
    *tile_n = 64;
    *tile_p = 64;
  } else {
    *tile_n = 128;
    *tile_p = 128;
  }
}

hipError_t launch_fitness(const Plan& p, int task, int dtype, const FitnessGeom& g, const void* phi,
                          const void* tile, const void* biasv, const void* tvec, double* psse,
                          uint32_t* pmiss, const DevState* st, hipStream_t s) {
  switch (dtype) {
    case GAME_F64:
      return launch_tr<F64Tr, 2, 2>(task, g, p, phi, tile, biasv, tvec, psse, pmiss, st, s);
    case GAME_F32:
      return launch_tr<F32Tr, 4, 4>(task, g, p, phi, tile, biasv, tvec, psse, pmiss, st, s);
    case GAME_BF16:
      return launch_tr<BF16Tr, 4, 4>(task, g, p, phi, tile, biasv, tvec, psse, pmiss, st, s);
    case GAME_F16:
      return launch_tr<F16Tr, 4, 4>(task, g, p, phi, tile, biasv, tvec, psse, pmiss, st, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_reduce(const Plan& p, const FitnessGeom& g, int P, const double* psse,
                         const uint32_t* pmiss, double* mse, double* miscls, double* fit,
                         double* mse2, double* miscls2, double* fit2, const DevState* st,
                         hipStream_t s) {
  const int grid = (P + 15) / 16;
  hipLaunchKernelGGL(reduce_kernel, dim3(grid), dim3(256), 0, s, g.n_rg, p.P_max_pad, P,
                     1.0 / (double)p.N, psse, pmiss, mse, miscls, fit, mse2, miscls2, fit2, st);
  return hipGetLastError();
}

}  // namespace game
