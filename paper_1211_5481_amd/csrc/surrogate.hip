// Offspring form of a generation, with an optional learned prescreen.
//
// Each generation breeds n_off offspring from the current population
// (tournaments on its exact fitness), scores them with the surrogate MLP (or
// with random keys for the control run), evaluates exactly only the k best by
// that score plus a random audit sample, stores every exactly evaluated
// (chromosome, log MSE) pair in a ring buffer the MLP trains on, and builds
// the next population from the E elites and the best P - E of the k
// evaluated offspring.  The audit sample measures the surrogate's rank error
// (Spearman's rho with average ranks for ties).
//
// The small kernels here are selections and rank statistics over at most a
// few thousand values (by counting, see below), plus row gathers; every sum
// is in a fixed order and every selection breaks ties by the lower index, so
// a run is bit-reproducible and each selection matches the CPU rule exactly.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "game_internal.hpp"
#include "select.hpp"

namespace game {
namespace {


// keys for the selections: 0 = float ascending (scores), 1 = random u32 word
// of block (i, 0, g, tag), 2 = double descending (fitness)
__global__ void keys_kernel(int mode, const float* __restrict__ fsrc, const double* __restrict__ dsrc,
                            int n, uint32_t tag, const DevState* st, uint32_t k0, uint32_t k1,
                            uint64_t* __restrict__ keys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (mode == 0) {
    keys[i] = ord_f32(fsrc[i]);
  } else if (mode == 1) {
    keys[i] = philox((uint32_t)i, 0u, (uint32_t)st->generation, tag, k0, k1).x;
  } else {
    keys[i] = ord_desc_f64(dsrc[i]);
  }
}

// Selections and rank statistics count instead of sorting: the rank of value
// i is the number of values before it in the order (key, index), counted in
// kRankSplits slices of the values by separate workgroups and added in slice
// order (integers, so exact).  n <= kRankSplits * kRankChunk.
constexpr int kRankThreads = 256;
constexpr int kRankSplits = 16;
constexpr int kRankChunk = 512;

struct KeySrc {
  const uint64_t* keys;  // explicit keys, or: side 0 orders x[xi[i]] ascending,
  const float* x;        // side 1 orders y[i] ascending
  const int* xi;
  const double* y;
};
__device__ __forceinline__ uint64_t key_of(const KeySrc& k, int side, int i) {
  if (k.keys) return k.keys[i];
  if (side == 0) return ord_f32(k.x[k.xi ? k.xi[i] : i]);
  return ~ord_desc_f64(k.y[i]);
}

// Slice s = blockIdx.y of side blockIdx.z; counts for value i:
//   kTies = false: c0 = #{j in slice : (key_j, j) < (key_i, i)}
//   kTies = true:  c0 = #{j in slice : key_j < key_i}, c1 = #{j in slice : key_j == key_i}
// at cnt[((side * 2 + c) * S + s) * n + i].
template <bool kTies>
__global__ __launch_bounds__(kRankThreads) void rank_part_kernel(KeySrc src, int n, int chunk,
                                                                 int* __restrict__ cnt,
                                                                 const DevState* st) {
  if (run_halted(st)) return;
  __shared__ uint64_t sk[kRankChunk];
  const int side = blockIdx.z, sl = blockIdx.y, S = gridDim.y;
  const int j0 = sl * chunk, j1 = min(n, j0 + chunk);
  for (int j = j0 + (int)threadIdx.x; j < j1; j += kRankThreads) sk[j - j0] = key_of(src, side, j);
  __syncthreads();
  const int i = blockIdx.x * kRankThreads + threadIdx.x;
  if (i >= n) return;
  const uint64_t ki = key_of(src, side, i);
  int c0 = 0, c1 = 0;
  for (int j = j0; j < j1; ++j) {
    const uint64_t kj = sk[j - j0];
    if (kTies) {
      c0 += kj < ki;
      c1 += kj == ki;
    } else {
      c0 += kj < ki || (kj == ki && j < i);
    }
  }
  cnt[((int64_t)(side * 2) * S + sl) * n + i] = c0;
  if (kTies) cnt[((int64_t)(side * 2 + 1) * S + sl) * n + i] = c1;
}

// out[rank] = i for the k values of lowest rank: the indices of the k
// smallest keys (ties to the lower index), in order.
__global__ void select_scatter_kernel(const int* __restrict__ cnt, int n, int S, int k,
                                      int* __restrict__ out, const DevState* st) {
  if (run_halted(st)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int r = 0;
  for (int s = 0; s < S; ++s) r += cnt[(int64_t)s * n + i];
  if (r < k) out[r] = i;
}

// Spearman's rho of (x[xi[i]], y[i]), i < n, average ranks for ties: value i
// of a side ranks lt + (eq + 1) / 2 (1-based; lt values below it, eq equal
// to it, itself included); then the Pearson correlation of the ranks with
// fixed-order sums (thread-strided, wave tree, waves in order).
constexpr int kRhoThreads = 1024;
__global__ __launch_bounds__(kRhoThreads) void spearman_final_kernel(const int* __restrict__ cnt, int n,
                                                                     int S, float* __restrict__ out,
                                                                     const DevState* st) {
  if (run_halted(st)) return;
  __shared__ double red[kRhoThreads / 64][3];
  auto rank = [&](int side, int i) {
    int lt = 0, eq = 0;
    for (int s = 0; s < S; ++s) {
      lt += cnt[((int64_t)(side * 2) * S + s) * n + i];
      eq += cnt[((int64_t)(side * 2 + 1) * S + s) * n + i];
    }
    return 0.5f * (float)(2 * lt + eq - 1) + 1.0f;
  };
  const double mean = 0.5 * (double)(n + 1);
  double sxy = 0.0, sxx = 0.0, syy = 0.0;
  for (int i = threadIdx.x; i < n; i += kRhoThreads) {
    const double a = rank(0, i) - mean, b = rank(1, i) - mean;
    sxy += a * b;
    sxx += a * a;
    syy += b * b;
  }
  for (int off = 32; off > 0; off >>= 1) {
    sxy += __shfl_xor(sxy, off);
    sxx += __shfl_xor(sxx, off);
    syy += __shfl_xor(syy, off);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[wave][0] = sxy;
    red[wave][1] = sxx;
    red[wave][2] = syy;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0, c = 0;
    for (int w = 0; w < kRhoThreads / 64; ++w) {
      a += red[w][0];
      b += red[w][1];
      c += red[w][2];
    }
    const double den = sqrt(b * c);
    *out = den > 0.0 ? (float)(a / den) : 0.0f;
  }
}

// dst row i = src row idx[i] (or row i when idx is null), L floats per row
__global__ void gather_kernel(const float* __restrict__ src, const int* __restrict__ idx, int n, int L,
                              float* __restrict__ dst, const DevState* st) {
  if (run_halted(st)) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * L) return;
  const int i = (int)(e / L), l = (int)(e % L);
  dst[e] = src[(int64_t)(idx ? idx[i] : i) * L + l];
}

// ---------------------------------------------------------- replay buffer
__global__ void append_kernel(const float* __restrict__ genes, const double* __restrict__ mse, int n,
                              int L, float* __restrict__ buf, float* __restrict__ buf_y, int cap,
                              const SurState* ss, const DevState* st) {
  if (run_halted(st)) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * L) return;
  const int i = (int)(e / L), l = (int)(e % L);
  const int slot = (int)(((int64_t)ss->head + i) % cap);
  buf[(int64_t)slot * L + l] = genes[e];
  if (l == 0) buf_y[slot] = (float)log(fmax(mse[i], 1e-300));
}

// advance the ring, then mean / std of the stored targets (fixed order)
__global__ __launch_bounds__(1024) void buffer_stats_kernel(const float* __restrict__ buf_y, int cap,
                                                            int n_new, SurState* ss,
                                                            const DevState* st) {
  if (run_halted(st)) return;
  __shared__ double red[16][2];
  __shared__ int s_count;
  if (threadIdx.x == 0) {
    const int count = min(cap, ss->count + n_new);
    ss->head = (int)(((int64_t)ss->head + n_new) % cap);
    ss->count = count;
    ss->last = n_new;
    s_count = count;
  }
  __syncthreads();
  const int count = s_count;
  double s = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < count; i += 1024) {
    const double v = buf_y[i];
    s += v;
    s2 += v * v;
  }
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off);
    s2 += __shfl_xor(s2, off);
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = s;
    red[threadIdx.x >> 6][1] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < 16; ++w) {
      a += red[w][0];
      b += red[w][1];
    }
    const double mu = count > 0 ? a / count : 0.0;
    const double var = count > 0 ? fmax(b / count - mu * mu, 0.0) : 0.0;
    ss->mu = (float)mu;
    ss->sigma = var > 0.0 ? (float)sqrt(var) : 1.0f;
  }
}

// ----------------------------------------------------------- population
// Snapshot the current elites' exact values before the merge overwrites them.
__global__ void snapshot_kernel(const int* __restrict__ elite, int E, const double* __restrict__ fit,
                                const double* __restrict__ mse, const double* __restrict__ miscls,
                                double* __restrict__ snap, const DevState* st) {
  if (run_halted(st)) return;
  const int e = threadIdx.x;
  if (e >= E) return;
  const int b = elite[e];
  snap[3 * e] = fit[b];
  snap[3 * e + 1] = mse[b];
  snap[3 * e + 2] = miscls[b];
}

// Next population: rows < E are the elites (pop[g & 1][elite[r]]), the rest
// the survivors among the evaluated offspring; fitness values follow.
__global__ void merge_kernel(const float* __restrict__ pop0, const float* __restrict__ pop1,
                             float* __restrict__ out0, float* __restrict__ out1,
                             const int* __restrict__ elite, const double* __restrict__ snap, int E,
                             const float* __restrict__ cand, const int* __restrict__ surv,
                             const double* __restrict__ cfit, const double* __restrict__ cmse,
                             const double* __restrict__ cmis, int P, int L, double* __restrict__ fit,
                             double* __restrict__ mse, double* __restrict__ miscls, const DevState* st) {
  if (run_halted(st)) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)P * L) return;
  const uint32_t g = (uint32_t)st->generation;
  const float* src = (g & 1u) ? pop1 : pop0;
  float* dst = (g & 1u) ? out0 : out1;
  const int r = (int)(e / L), l = (int)(e % L);
  if (r < E) {
    dst[e] = src[(int64_t)elite[r] * L + l];
    if (l == 0) {
      fit[r] = snap[3 * r];
      mse[r] = snap[3 * r + 1];
      miscls[r] = snap[3 * r + 2];
    }
  } else {
    const int c = surv[r - E];
    dst[e] = cand[(int64_t)c * L + l];
    if (l == 0) {
      fit[r] = cfit[c];
      mse[r] = cmse[c];
      miscls[r] = cmis[c];
    }
  }
}

// Rank the new population, track the best, apply the stop rule and advance
// the generation (one workgroup).
__global__ __launch_bounds__(1024) void rank_track_kernel(const double* __restrict__ fit, const double* __restrict__ mse,
                                                          const double* __restrict__ miscls, int P, int n_top,
                                                          int* __restrict__ top, const float* __restrict__ pop0,
                                                          const float* __restrict__ pop1, int L,
                                                          float* __restrict__ best, DevState* st,
                                                          int advance) {
  if (run_halted(st)) return;
  block_topk<1024>(fit, P, n_top, top);
  __syncthreads();
  // the population being ranked is generation g + advance; the stop rule is
  // tested with the generation counter still at g (g + 1 offspring
  // generations done), then the counter advances
  const uint32_t g = (uint32_t)st->generation + (uint32_t)advance;
  const float* pop = (g & 1u) ? pop1 : pop0;
  track_best(st, top, mse, miscls, pop, L, best);
  __syncthreads();
  if (advance && threadIdx.x == 0) st->generation += 1;
}

__global__ void log_kernel(const float* __restrict__ rho, const float* __restrict__ loss,
                           float* __restrict__ log, int cap, SurState* ss, const DevState* st) {
  if (run_halted(st)) return;
  const int slot = ss->n_logged % cap;
  log[4 * slot + 0] = rho[0];
  log[4 * slot + 1] = rho[1];
  log[4 * slot + 2] = loss ? *loss : 0.0f;
  log[4 * slot + 3] = 1.0f;
  ss->n_logged += 1;
}

}  // namespace

hipError_t sur_keys(int mode, const float* fsrc, const double* dsrc, int n, uint32_t tag,
                    const DevState* st, uint64_t seed, uint64_t* keys, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(keys_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, mode, fsrc, dsrc,
                     n, tag, st, (uint32_t)seed, (uint32_t)(seed >> 32), keys);
  return hipGetLastError();
}

hipError_t sur_select(const uint64_t* keys, int n, int k, int* out, int* rank_ws, const DevState* st,
                      hipStream_t s) {
  if (n <= 0 || k <= 0) return hipSuccess;
  if (n > kRankSplits * kRankChunk || k > n) return hipErrorInvalidValue;
  const int chunk = (n + kRankSplits - 1) / kRankSplits;
  const unsigned g = (unsigned)((n + kRankThreads - 1) / kRankThreads);
  const KeySrc src{keys, nullptr, nullptr, nullptr};
  hipLaunchKernelGGL(rank_part_kernel<false>, dim3(g, kRankSplits, 1), dim3(kRankThreads), 0, s, src, n,
                     chunk, rank_ws, st);
  hipLaunchKernelGGL(select_scatter_kernel, dim3(g), dim3(kRankThreads), 0, s, rank_ws, n, kRankSplits, k,
                     out, st);
  return hipGetLastError();
}

hipError_t sur_spearman(const float* x, const int* xi, const double* y, int n, float* out, int* rank_ws,
                        const DevState* st, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > kRankSplits * kRankChunk) return hipErrorInvalidValue;
  const int chunk = (n + kRankSplits - 1) / kRankSplits;
  const unsigned g = (unsigned)((n + kRankThreads - 1) / kRankThreads);
  const KeySrc src{nullptr, x, xi, y};
  hipLaunchKernelGGL(rank_part_kernel<true>, dim3(g, kRankSplits, 2), dim3(kRankThreads), 0, s, src, n,
                     chunk, rank_ws, st);
  hipLaunchKernelGGL(spearman_final_kernel, dim3(1), dim3(kRhoThreads), 0, s, rank_ws, n, kRankSplits, out,
                     st);
  return hipGetLastError();
}

hipError_t sur_gather(const float* src, const int* idx, int n, int L, float* dst, const DevState* st,
                      hipStream_t s) {
  const int64_t t = (int64_t)n * L;
  if (t == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, src, idx, n, L,
                     dst, st);
  return hipGetLastError();
}

hipError_t sur_append(const float* genes, const double* mse, int n, int L, float* buf, float* buf_y,
                      int cap, SurState* ss, const DevState* st, hipStream_t s) {
  const int64_t t = (int64_t)n * L;
  hipLaunchKernelGGL(append_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, genes, mse, n,
                     L, buf, buf_y, cap, ss, st);
  hipLaunchKernelGGL(buffer_stats_kernel, dim3(1), dim3(1024), 0, s, buf_y, cap, n, ss, st);
  return hipGetLastError();
}

hipError_t sur_snapshot(const int* elite, int E, const double* fit, const double* mse,
                        const double* miscls, double* snap, const DevState* st, hipStream_t s) {
  if (E == 0) return hipSuccess;
  hipLaunchKernelGGL(snapshot_kernel, dim3(1), dim3(64), 0, s, elite, E, fit, mse, miscls, snap, st);
  return hipGetLastError();
}

hipError_t sur_merge(float* pop0, float* pop1, const int* elite, const double* snap, int E,
                     const float* cand, const int* surv, const double* cfit, const double* cmse,
                     const double* cmis, int P, int L, double* fit, double* mse, double* miscls,
                     const DevState* st, hipStream_t s) {
  const int64_t t = (int64_t)P * L;
  hipLaunchKernelGGL(merge_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, pop0, pop1, pop0,
                     pop1, elite, snap, E, cand, surv, cfit, cmse, cmis, P, L, fit, mse, miscls, st);
  return hipGetLastError();
}

hipError_t sur_rank_track(const double* fit, const double* mse, const double* miscls, int P, int n_top,
                          int* top, const float* pop0, const float* pop1, int L, float* best,
                          DevState* st, int advance, hipStream_t s) {
  hipLaunchKernelGGL(rank_track_kernel, dim3(1), dim3(1024), 0, s, fit, mse, miscls, P, n_top, top,
                     pop0, pop1, L, best, st, advance);
  return hipGetLastError();
}

hipError_t sur_log(const float* rho, const float* loss, float* log, int cap, SurState* ss,
                   const DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(log_kernel, dim3(1), dim3(1), 0, s, rho, loss, log, cap, ss, st);
  return hipGetLastError();
}

int64_t sur_rank_ints(int n) { return (int64_t)4 * kRankSplits * n; }


}  // namespace game
