// Basis expansion Phi[n, i*K + k] = phi_{k+1}(x[n, i])  (eq. 1; eq. 6 for trig).
// In the shared-coefficient model (one coefficient per basis function for all
// features, eq. 2 and eq. 7) the row holds K values instead,
// Phi[n, k] = sum_i phi_{k+1}(x[n, i]), summed in double in feature order.
//
// The values are computed once per dataset, as the paper does with its sin/cos
// tables (Sec. 4): inputs never change during training, so only the genes are
// re-read every generation.  Each value is evaluated in double by the
// three-term recurrences (Chebyshev, Legendre, the cos/sin multiple-angle
// recurrence seeded by one sincos) and rounded once to the storage type
// (bf16/f16 round the float32-rounded value).
//
// Layout: Phi is row-major N x ld.  Where a feature's K values fill whole
// 16-byte stores (per-feature layout), one thread per (row, feature) writes
// them directly (basis_direct_kernel); otherwise a workgroup builds a block
// of rows in LDS in any order, then the block, which is contiguous in HBM,
// is written with 16-byte stores by consecutive lanes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "expand.hpp"
#include "game_internal.hpp"

namespace game {
namespace {

constexpr int kBasisThreads = 256;
constexpr int kBasisLdsBytes = 32768;

template <typename O>
__device__ __forceinline__ O to_storage(double v);
template <>
__device__ __forceinline__ double to_storage<double>(double v) {
  return v;
}
template <>
__device__ __forceinline__ float to_storage<float>(double v) {
  return (float)v;
}
template <>
__device__ __forceinline__ _Float16 to_storage<_Float16>(double v) {
  return (_Float16)(float)v;  // v_cvt_f16_f32 rounds to nearest even
}
// bf16 kept as its bit pattern; round to nearest even from the float32 value.
struct bf16_bits {
  uint16_t b;
};
template <>
__device__ __forceinline__ bf16_bits to_storage<bf16_bits>(double v) {
  const uint32_t u = __float_as_uint((float)v);
  const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
  return bf16_bits{(uint16_t)(r >> 16)};
}

// byte offset of the shared model's accumulators: after the block, 16-aligned
__host__ __device__ inline size_t acc_offset(int rows, int64_t ld, size_t elem) {
  return ((size_t)rows * (size_t)ld * elem + 15) & ~(size_t)15;
}

template <typename XT, typename O>
__global__ __launch_bounds__(kBasisThreads) void basis_kernel(const XT* __restrict__ X,
                                                              int64_t rows_in, int64_t rows_out,
                                                              int F, int D, int K, int basis,
                                                              int M, int64_t ld, int rows_per_wg,
                                                              int shared, O* __restrict__ phi) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  O* lds = reinterpret_cast<O*>(lds_raw);
  const int64_t row0 = (int64_t)blockIdx.x * rows_per_wg;
  if (row0 >= rows_out) return;
  const int rows = (int)min((int64_t)rows_per_wg, rows_out - row0);
  const int tid = threadIdx.x;

  // 1) every (row, feature) pair expands into its K columns in LDS; in the
  //    shared model a thread owns a row and adds its features' expansions
  //    into double accumulators placed after the block
  if (shared) {
    double* acc = reinterpret_cast<double*>(lds_raw + acc_offset(rows_per_wg, ld, sizeof(O)));
    for (int r = tid; r < rows; r += kBasisThreads) {
      const int64_t n = row0 + r;
      double* a = acc + (int64_t)r * K;
      for (int k = 0; k < K; ++k) a[k] = 0.0;
      if (n < rows_in)
        for (int i = 0; i < F; ++i)
          expand_feature(basis, D, (double)X[n * F + i], [&](int k, double v) { a[k] += v; });
      O* dst = lds + (int64_t)r * ld;
      for (int k = 0; k < K; ++k) dst[k] = to_storage<O>(a[k]);
    }
  }
  for (int idx = tid; !shared && idx < rows * F; idx += kBasisThreads) {
    const int r = idx / F, i = idx - r * F;
    const int64_t n = row0 + r;
    O* dst = lds + (int64_t)r * ld + (int64_t)i * K;
    if (n < rows_in) {
      const double x = (double)X[n * F + i];
      expand_feature(basis, D, x, [&](int k, double v) { dst[k] = to_storage<O>(v); });
    } else {
      for (int k = 0; k < K; ++k) dst[k] = to_storage<O>(0.0);
    }
  }
  // pad columns M..ld-1
  const int padw = (int)(ld - M);
  for (int idx = tid; idx < rows * padw; idx += kBasisThreads) {
    const int r = idx / padw, c = idx - r * padw;
    lds[(int64_t)r * ld + M + c] = to_storage<O>(0.0);
  }
  __syncthreads();

  // 2) the block is contiguous in global memory: coalesced stores
  const int64_t bytes = (int64_t)rows * ld * (int64_t)sizeof(O);
  unsigned char* gdst = reinterpret_cast<unsigned char*>(phi + row0 * ld);
  if ((bytes & 15) == 0 && (reinterpret_cast<uintptr_t>(gdst) & 15) == 0) {
    const int64_t n16 = bytes >> 4;
    const uint4* s = reinterpret_cast<const uint4*>(lds_raw);
    uint4* d = reinterpret_cast<uint4*>(gdst);
    for (int64_t v = tid; v < n16; v += kBasisThreads) d[v] = s[v];
  } else {
    const int64_t n = (int64_t)rows * ld;
    for (int64_t v = tid; v < n; v += kBasisThreads) phi[row0 * ld + v] = lds[v];
  }
}

// Direct form, for the per-feature layout when a feature's K values fill
// whole 16-byte stores: each thread takes kPairs (row, feature) pairs a
// workgroup-width apart, loads their inputs together (the loads' latency
// binds otherwise), then expands each in column order and stores its K
// values with 16-byte stores; the thread of a row's last feature also
// zeroes the row's pad columns.  No LDS, no barrier.
constexpr int kPairs = 4;
template <typename XT, typename O, int kBasis>
__global__ __launch_bounds__(kBasisThreads) void basis_direct_kernel(const XT* __restrict__ X,
                                                                     int64_t rows_in, int64_t rows_out,
                                                                     int F, int D, int K, int M,
                                                                     int64_t ld, O* __restrict__ phi) {
  constexpr int kPer = 16 / (int)sizeof(O);  // values per 16-byte store
  const int64_t total = rows_out * F, in_total = rows_in * F;
  const int64_t base = (int64_t)blockIdx.x * kBasisThreads * kPairs + threadIdx.x;
  XT xs[kPairs];
#pragma unroll
  for (int p = 0; p < kPairs; ++p) {
    const int64_t idx = base + (int64_t)p * kBasisThreads;
    // the load address is clamped, its value unused past the input rows
    xs[p] = X[idx < in_total ? idx : 0];
  }
#pragma unroll
  for (int p = 0; p < kPairs; ++p) {
    const int64_t idx = base + (int64_t)p * kBasisThreads;
    if (idx >= total) break;
    // (row, feature) by a 32-bit division where the pair count allows
    int64_t n;
    if (total <= 0xFFFFFFFFll) n = (int64_t)((uint32_t)idx / (uint32_t)F);
    else n = idx / F;
    const int i = (int)(idx - n * F);
    const bool valid = idx < in_total;
    BasisSeq<kBasis> g(D, valid ? (double)xs[p] : 0.0);
    O* dst = phi + n * ld + (int64_t)i * K;
    for (int k = 0; k < K; k += kPer) {
      O v[kPer];
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const double val = g.next();
        v[j] = to_storage<O>(valid ? val : 0.0);
      }
      *reinterpret_cast<uint4*>(dst + k) = __builtin_bit_cast(uint4, v);
    }
    if (i == F - 1)
      for (int64_t c = M; c < ld; ++c) phi[n * ld + c] = to_storage<O>(0.0);
  }
}

template <typename XT, typename O>
hipError_t launch_typed(const game_config* cfg, const void* X, int64_t rows_in, int64_t rows_out,
                        void* phi, int64_t ld, hipStream_t s) {
  const int F = cfg->n_features, D = cfg->degree;
  const int K = (cfg->basis == GAME_BASIS_TRIG ? 2 : 1) * D;
  const int shared = cfg->shared;
  const int M = shared ? K : F * K;
  if (!shared && ((int64_t)K * (int64_t)sizeof(O)) % 16 == 0 && (ld * (int64_t)sizeof(O)) % 16 == 0 &&
      (reinterpret_cast<uintptr_t>(phi) & 15) == 0) {
    const int64_t pairs = rows_out * F;
    if (pairs == 0) return hipSuccess;
    const int64_t per_wg = (int64_t)kBasisThreads * kPairs;
    const int64_t grid = (pairs + per_wg - 1) / per_wg;
    if (grid > 0x7FFFFFFFll) return hipErrorInvalidValue;
    const dim3 g((unsigned)grid), b(kBasisThreads);
    const XT* x = static_cast<const XT*>(X);
    O* out = static_cast<O*>(phi);
    switch (cfg->basis) {
      case GAME_BASIS_POWER:
        hipLaunchKernelGGL((basis_direct_kernel<XT, O, GAME_BASIS_POWER>), g, b, 0, s, x, rows_in, rows_out, F, D, K, M, ld, out);
        break;
      case GAME_BASIS_CHEBYSHEV:
        hipLaunchKernelGGL((basis_direct_kernel<XT, O, GAME_BASIS_CHEBYSHEV>), g, b, 0, s, x, rows_in, rows_out, F, D, K, M, ld, out);
        break;
      case GAME_BASIS_LEGENDRE:
        hipLaunchKernelGGL((basis_direct_kernel<XT, O, GAME_BASIS_LEGENDRE>), g, b, 0, s, x, rows_in, rows_out, F, D, K, M, ld, out);
        break;
      default:
        hipLaunchKernelGGL((basis_direct_kernel<XT, O, GAME_BASIS_TRIG>), g, b, 0, s, x, rows_in, rows_out, F, D, K, M, ld, out);
        break;
    }
    return hipGetLastError();
  }
  const int64_t row_bytes = ld * (int64_t)sizeof(O);
  // the shared model keeps K double accumulators per row (one thread per row)
  const int64_t acc_bytes = shared ? (int64_t)K * 8 : 0;
  int rows_per_wg = (int)(kBasisLdsBytes / (row_bytes + acc_bytes));
  if (rows_per_wg < 1) rows_per_wg = 1;
  if (rows_per_wg > (shared ? kBasisThreads : 64)) rows_per_wg = shared ? kBasisThreads : 64;
  const size_t lds = shared ? acc_offset(rows_per_wg, ld, sizeof(O)) + (size_t)rows_per_wg * acc_bytes
                            : (size_t)rows_per_wg * (size_t)row_bytes;
  const int64_t grid = (rows_out + rows_per_wg - 1) / rows_per_wg;
  if (grid == 0) return hipSuccess;
  if (lds > 65536) return hipErrorInvalidValue;  // a single row larger than LDS allows
  hipLaunchKernelGGL((basis_kernel<XT, O>), dim3((unsigned)grid), dim3(kBasisThreads), lds, s,
                     static_cast<const XT*>(X), rows_in, rows_out, F, D, K, cfg->basis, M, ld,
                     rows_per_wg, shared, static_cast<O*>(phi));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_basis(const game_config* cfg, const void* X, int64_t rows_in, int64_t rows_out,
                        void* phi, int64_t ld, hipStream_t s) {
  switch (cfg->dtype) {
    case GAME_F64:
      return launch_typed<double, double>(cfg, X, rows_in, rows_out, phi, ld, s);
    case GAME_F32:
      return launch_typed<float, float>(cfg, X, rows_in, rows_out, phi, ld, s);
    case GAME_BF16:
      return launch_typed<float, bf16_bits>(cfg, X, rows_in, rows_out, phi, ld, s);
    case GAME_F16:
      return launch_typed<float, _Float16>(cfg, X, rows_in, rows_out, phi, ld, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace game
