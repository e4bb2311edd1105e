// Fitness-surrogate MLP: y = w3 . gelu(W2 gelu(W1 g + b1) + b2) + b3, trained
// online with Adam (Kingma and Ba) on (chromosome, standardised log MSE)
// pairs.  GELU is the exact form a * Phi(a) = a (1 + erf(a / sqrt 2)) / 2.
//
// Every product of a forward pass or of a training step is a dense
// contraction and runs on the matrix cores (v_mfma_f32_16x16x4f32: float32
// operands and accumulation).  A training step on B minibatch rows is four
// launches:
//   layer 1: A1 = X W1^T + b1, H1 = gelu(A1), in tiles of 32 rows x 32 units;
//            the rows are drawn from the replay ring by the counter-based
//            generator, or read from a given matrix;
//   layer 2: A2 = H1 W2^T + b2, and every tile's share of the head gelu(A2) w3;
//   back:    y = head + b3, dy = 2 (y - t) / B, dA2 = dy w3 gelu'(A2),
//            dA1 = (dA2 W2) gelu'(A1) (the layers store gelu' of their
//            pre-activations, so each is evaluated once);
//   grads:   dW1 = dA1^T X, dW2 = dA2^T H1, db1, db2, dw3 = H2^T dy, db3 and the
//            loss, all products over the B rows.  Each workgroup owns a tile
//            of parameters and applies Adam to it (or writes the gradient):
//            no partial-sum slabs, no atomics on values; the last workgroup
//            to finish advances the step counter.
// A forward pass alone is layer 1, layer 2 and a head sum.
//
// Every operand is read with the contraction index contiguous, as 16-byte
// vectors: the layers store activations row-major and also transposed (batch
// rows contiguous) for the parameter-gradient products, which contract over
// rows; W2 is kept transposed as well (W2T, H1 x H2) for the product dA2 W2.
// Where every row holds whole 16-byte groups (activation rows are padded;
// weight rows when the widths are multiples of 4) the groups are read
// without branches, four groups per wave at once (tile_product_v).
// A workgroup's waves (4; 16 for the gradient products, which contract over
// all B rows) take interleaved 16-wide slices of the contraction and add
// their 32 x 32 partial tiles in wave order, so every result has a fixed
// summation order and is bit-reproducible.
//
// Parameters are one flat float32 array: W1 (H1 x L), b1 (H1), W2 (H2 x H1),
// b2 (H2), w3 (H2), b3 (1); gradients and Adam moments use the same layout.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "game_internal.hpp"

namespace game {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;  // four waves
constexpr int kT = 32;         // tile edge
constexpr int kMaxHidden = 1024;  // widest hidden layer a context accepts

__device__ __forceinline__ float gelu(float a) { return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float a) {
  const float cdf = 0.5f * (1.0f + erff(a * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * a * a);
  return cdf + a * pdf;
}

constexpr int64_t round4(int64_t n) { return (n + 3) & ~int64_t(3); }

// Activations of one step (floats; B4 = B rounded up to 4, ld1/ld2 the hidden
// widths rounded up to 4).  Row-major: Hd1 (B x ld1), G2 = gelu'(A2)
// (B x ld2), ypart (B x nT2 head shares).  Transposed, batch rows contiguous
// (ld B4): XT (L), G1T = gelu'(A1), Hd1T, D1T (H1), Hd2T, D2T (H2), dyres (dy
// then squared residuals).  tv: standardised targets; ones: 1 for rows < B.
struct Scratch {
  uint32_t* gcnt;  // per parameter tile: arrival count of its split products (zero between launches)
  float* gpart;    // per parameter tile and split: the 32 x 32 partial product
  float *Hd1, *ypart, *XT, *tv, *ones, *G1T, *Hd1T, *G2, *Hd2T, *dyres, *D2T, *D1T;
  int B4, ld1, ld2, nT2;
};
int grad_tiles(const MlpDims& d);
constexpr int kSplit = 4;  // row ranges each parameter tile's product is split into

// Lays the scratch out from `base` (null: sizes only); returns the floats
// used.  A forward pass needs only Hd1 and ypart, which come first.
int64_t scratch_layout(const MlpDims& d, int B, bool train, float* base, Scratch* s) {
  Scratch z{};
  z.B4 = (int)round4(B);
  z.ld1 = (int)round4(d.H1);
  z.ld2 = (int)round4(d.H2);
  z.nT2 = (d.H2 + kT - 1) / kT;
  int64_t o = 0;
  auto take = [&](int64_t n) {
    float* p = base ? base + o : nullptr;
    o += round4(n);
    return p;
  };
  const int64_t B4 = z.B4;
  // the gradient products' counters and partials come first in every layout,
  // so that no other scratch use overwrites the counters
  const int64_t nt = grad_tiles(d);
  z.gcnt = reinterpret_cast<uint32_t*>(take(nt));
  z.gpart = take(nt * kSplit * kT * kT);
  z.Hd1 = take(B4 * z.ld1);
  z.ypart = take(B4 * z.nT2);
  if (train) {
    z.XT = take((int64_t)d.L * B4);
    z.tv = take(B4);
    z.ones = take(B4);
    z.G1T = take((int64_t)d.H1 * B4);
    z.Hd1T = take((int64_t)d.H1 * B4);
    z.G2 = take(B4 * z.ld2);
    z.Hd2T = take((int64_t)d.H2 * B4);
    z.dyres = take(2 * B4);
    z.D2T = take((int64_t)d.H2 * B4);
    z.D1T = take((int64_t)d.H1 * B4);
  }
  if (s) *s = z;
  return o;
}

__device__ __forceinline__ void st_agent(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_agent(const float* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until this thread's device-scope stores are acknowledged (they are
// then visible to the workgroup that counts the arrival after them).
__device__ __forceinline__ void stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Four consecutive k of one operand row, zero past K or for a missing row.
__device__ __forceinline__ v4f load4(const float* row, int k, int K, bool vec) {
  v4f v = {0.0f, 0.0f, 0.0f, 0.0f};
  if (!row) return v;
  if (vec && k + 3 < K) return *reinterpret_cast<const v4f*>(row + k);
#pragma unroll
  for (int s = 0; s < 4; ++s)
    if (k + s < K) v[s] = row[k + s];
  return v;
}

__device__ __forceinline__ bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// The same four k read without a branch, in two parts: raw4 loads 16 bytes
// from a row with at least K rounded up to 4 readable floats (16-byte
// aligned; k clamped into the row, so any k is in bounds), and mask4 keeps
// the elements below K of a row that exists (ok) and zeroes the rest.
__device__ __forceinline__ v4f raw4(const float* row, int k, int K) {
  return *reinterpret_cast<const v4f*>(row + min(k, ((K + 3) & ~3) - 4));
}
__device__ __forceinline__ v4f mask4(v4f v, bool ok, int k, int K) {
  v4f r;
#pragma unroll
  for (int s = 0; s < 4; ++s) r[s] = (ok && k + s < K) ? v[s] : 0.0f;
  return r;
}

// C (32 x 32) = sum_{k < K} A(m, k) B(n, k) with NW waves.  Wave w takes the
// 16-wide k groups w, w + NW, ...; in a group, lane (i, q) supplies rows i and
// 16 + i of both operands at k = 4q .. 4q + 3 (fa / fb return those four
// values), one MFMA per k of the four, so every k of the group is used
// exactly once.  The next group's operands are loaded before the current
// group's MFMAs, so two groups' loads are in flight.  The waves' partial
// tiles go to `red` (NW x 4 x 64 v4f, 4 KiB per wave).
template <int NW, class FA, class FB>
__device__ __forceinline__ void tile_product(int K, FA fa, FB fb, v4f* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  v4f acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  int k0 = wave * 16;
  v4f a0, a1, b0, b1;
  if (k0 < K) {
    const int k = k0 + 4 * q;
    a0 = fa(i, k);
    a1 = fa(16 + i, k);
    b0 = fb(i, k);
    b1 = fb(16 + i, k);
  }
  for (; k0 < K; k0 += 16 * NW) {
    const v4f c0 = a0, c1 = a1, d0 = b0, d1 = b1;
    const int kn = k0 + 16 * NW;
    if (kn < K) {
      const int k = kn + 4 * q;
      a0 = fa(i, k);
      a1 = fa(16 + i, k);
      b0 = fb(i, k);
      b1 = fb(16 + i, k);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(c0[s], d0[s], acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(c0[s], d1[s], acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(c1[s], d0[s], acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(c1[s], d1[s], acc[1][1], 0, 0, 0);
    }
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) red[(wave * 4 + bi * 2 + bj) * 64 + lane] = acc[bi][bj];
  __syncthreads();
}

// tile_product with branch-free operand reads: la / lb return a group's raw
// 16 bytes (any k in bounds), ma / mb turn them into the operand where the
// group is used (masking, and any per-element work).  Each wave issues the
// loads of kDepth of its groups at once, then runs their MFMAs in the same
// order as tile_product.  A group past K is all zeros and its products are
// added too (a branch around them would let the compiler sink each group's
// loads to their use, one memory latency per group again), so a sum that
// is exactly -0 in tile_product can come out +0 here; otherwise the result
// is the same, bit for bit.  A load under a branch, or its value masked as
// soon as it arrives, makes the compiler wait for it there; here one memory
// latency is paid per kDepth groups.
template <int NW, int kDepth, class LA, class MA, class LB, class MB>
__device__ __forceinline__ void tile_product_v(int K, LA la, MA ma, LB lb, MB mb, v4f* red) {
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int i = lane & 15, q = lane >> 4;
  v4f acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = wave * 16; k0 < K; k0 += kDepth * 16 * NW) {
    v4f ra[kDepth][2], rb[kDepth][2];
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
      const int k = k0 + d * 16 * NW + 4 * q;
      ra[d][0] = la(i, k);
      ra[d][1] = la(16 + i, k);
      rb[d][0] = lb(i, k);
      rb[d][1] = lb(16 + i, k);
    }
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
      const int k = k0 + d * 16 * NW + 4 * q;
      const v4f c0 = ma(i, k, ra[d][0]), c1 = ma(16 + i, k, ra[d][1]);
      const v4f d0 = mb(i, k, rb[d][0]), d1 = mb(16 + i, k, rb[d][1]);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(c0[s], d0[s], acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(c0[s], d1[s], acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(c1[s], d0[s], acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(c1[s], d1[s], acc[1][1], 0, 0, 0);
      }
    }
    // the chunk's order: every group's loads ahead of the products (left
    // alone, the scheduler reuses one group's registers and so waits for
    // each group in turn)
    __builtin_amdgcn_sched_group_barrier(0x0020, 4 * kDepth, 0);   // vector memory reads
    __builtin_amdgcn_sched_group_barrier(0x0008, 16 * kDepth, 0);  // MFMAs
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) red[(wave * 4 + bi * 2 + bj) * 64 + lane] = acc[bi][bj];
  __syncthreads();
}

// Thread t < 256's share of the tile after tile_product: block t / 64 =
// (bi, bj), accumulator lane t % 64, i.e. rows m0 .. m0 + 3 (m0 = 16 bi +
// 4 (lane / 16)) of column n = 16 bj + lane % 16, the waves' partials added in
// wave order.  Threads from 256 on hold nothing (n = kT).
struct TileOut {
  int m0, n;
  v4f v;
};
template <int NW>
__device__ __forceinline__ TileOut tile_sum(const v4f* red) {
  if (threadIdx.x >= 256) return TileOut{0, kT, v4f{0.0f, 0.0f, 0.0f, 0.0f}};
  const int blk = threadIdx.x >> 6, lane = threadIdx.x & 63;
  v4f v = red[blk * 64 + lane];
#pragma unroll
  for (int w = 1; w < NW; ++w) v += red[(w * 4 + blk) * 64 + lane];
  return TileOut{16 * (blk >> 1) + 4 * (lane >> 4), 16 * (blk & 1) + (lane & 15), v};
}

struct Args {
  const float* P;    // parameters
  const float* W2T;  // H1 x H2
  int L, H1, H2, B;
  // rows: explicit (X, target) or drawn from the replay ring
  const float* X;
  const float* target;
  const float* buf;
  const float* bufy;
  const SurState* ss;
  const int32_t* step;
  uint32_t k0, k1;
  int n_recent, cap;
  Scratch s;
  float* y;  // forward: scores of the B rows
};

struct Offs {
  int64_t W1, b1, W2, b2, w3, b3;
};
__host__ __device__ __forceinline__ Offs offs(int L, int H1, int H2) {
  Offs o;
  o.W1 = 0;
  o.b1 = (int64_t)H1 * L;
  o.W2 = o.b1 + H1;
  o.b2 = o.W2 + (int64_t)H2 * H1;
  o.w3 = o.b2 + H2;
  o.b3 = o.w3 + H2;
  return o;
}

// Layer 1: tile (row tile blockIdx.y, unit tile blockIdx.x).  The row
// tile's unit tiles also store its rows' inputs transposed (a slice of the
// genes each); the first one stores the targets and ones.
template <bool kTrain, bool kV>
__global__ __launch_bounds__(kThreads) void layer1_kernel(Args a, const DevState* halt) {
  if (run_halted(halt)) return;
  __shared__ v4f red[16 * 64];
  __shared__ int s_slot[kT];
  const Scratch& S = a.s;
  const int c0 = blockIdx.x * kT, r0 = blockIdx.y * kT, tid = threadIdx.x, L = a.L;
  const bool lead = kTrain && blockIdx.x == 0;
  if (tid < kT) {
    const int r = r0 + tid;
    int slot = -1;
    if (r < a.B) {
      if (a.X) {
        slot = r;
      } else {
        const uint32_t w = philox((uint32_t)*a.step, (uint32_t)r, 0u, kTagMinibatch, a.k0, a.k1).x;
        if (r < a.B - a.n_recent) {
          slot = (int)__umulhi(w, (uint32_t)a.ss->count);
        } else {
          const int back = (int)__umulhi(w, (uint32_t)a.ss->last);
          slot = (int)(((int64_t)a.ss->head - 1 - back + a.cap) % a.cap);
        }
      }
    }
    s_slot[tid] = slot;
    if (lead && r < S.B4) {
      float t = 0.0f, one = 0.0f;
      if (r < a.B) {
        t = a.X ? a.target[r] : (a.bufy[slot] - a.ss->mu) / a.ss->sigma;
        one = 1.0f;
      }
      S.tv[r] = t;
      S.ones[r] = one;
    }
  }
  __syncthreads();
  const float* src = a.X ? a.X : a.buf;
  // the row tile's unit tiles keep the inputs transposed, each its own slice
  // of k (every element stored once, the work shared)
  const int xs = (L + gridDim.x - 1) / gridDim.x, xk0 = blockIdx.x * xs, xk1 = min(L, xk0 + xs);
  auto xt = [&](int m, int k, v4f v) {
    if (kTrain && s_slot[m] >= 0) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (k + s >= xk0 && k + s < xk1) S.XT[(int64_t)(k + s) * S.B4 + r0 + m] = v[s];
    }
    return v;
  };
  if constexpr (kV) {  // rows of L floats, L a multiple of 4, 16-byte aligned
    auto la = [&](int m, int k) { return raw4(src + (int64_t)max(s_slot[m], 0) * L, k, L); };
    auto ma = [&](int m, int k, v4f v) { return xt(m, k, mask4(v, s_slot[m] >= 0, k, L)); };
    auto lb = [&](int n, int k) { return raw4(a.P + (int64_t)(c0 + n < a.H1 ? c0 + n : 0) * L, k, L); };
    auto mb = [&](int n, int k, v4f v) { return mask4(v, c0 + n < a.H1, k, L); };
    tile_product_v<4, 2>(L, la, ma, lb, mb, red);
  } else {
    const bool vx = (L & 3) == 0 && aligned16(src);
    auto fa = [&](int m, int k) {
      const int slot = s_slot[m];
      return xt(m, k, load4(slot >= 0 ? src + (int64_t)slot * L : nullptr, k, L, vx));
    };
    const bool vw = (L & 3) == 0;  // W1 starts the parameter array
    auto fb = [&](int n, int k) {
      const int h = c0 + n;
      return load4(h < a.H1 ? a.P + (int64_t)h * L : nullptr, k, L, vw);
    };
    tile_product<4>(L, fa, fb, red);
  }
  const TileOut o = tile_sum<4>(red);
  const int h = c0 + o.n, r = r0 + o.m0;
  if (h < a.H1 && r < S.B4) {
    const float b1 = a.P[(int64_t)a.H1 * L + h];
    v4f act, der;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool ok = r + q < a.B;
      const float pre = o.v[q] + b1;
      act[q] = ok ? gelu(pre) : 0.0f;
      der[q] = ok && kTrain ? gelu_grad(pre) : 0.0f;
      if (ok) S.Hd1[(int64_t)(r + q) * S.ld1 + h] = act[q];
    }
    if (kTrain) {
      *reinterpret_cast<v4f*>(S.G1T + (int64_t)h * S.B4 + r) = der;
      *reinterpret_cast<v4f*>(S.Hd1T + (int64_t)h * S.B4 + r) = act;
    }
  }
}

// Layer 2 and the tile's share of the head: ypart[r][unit tile] = sum over
// the tile's units j (in order) of gelu(A2[r][j]) w3[j].
template <bool kTrain, bool kV>
__global__ __launch_bounds__(kThreads) void layer2_kernel(Args a, const DevState* halt) {
  if (run_halted(halt)) return;
  __shared__ v4f red[16 * 64];
  __shared__ float s_h[kT][kT + 1];
  const Scratch& S = a.s;
  const int c0 = blockIdx.x * kT, r0 = blockIdx.y * kT, tid = threadIdx.x, H1 = a.H1;
  const Offs po = offs(a.L, H1, a.H2);
  const float* W2 = a.P + po.W2;
  // rows of Hd1: ld1 >= H1 rounded up to 4 floats
  auto la = [&](int m, int k) { return raw4(S.Hd1 + (int64_t)(r0 + m < a.B ? r0 + m : 0) * S.ld1, k, H1); };
  auto ma = [&](int m, int k, v4f v) { return mask4(v, r0 + m < a.B, k, H1); };
  if constexpr (kV) {  // W2 rows of H1 floats, H1 a multiple of 4
    auto lb = [&](int n, int k) { return raw4(W2 + (int64_t)(c0 + n < a.H2 ? c0 + n : 0) * H1, k, H1); };
    auto mb = [&](int n, int k, v4f v) { return mask4(v, c0 + n < a.H2, k, H1); };
    tile_product_v<4, 4>(H1, la, ma, lb, mb, red);
  } else {
    auto fa = [&](int m, int k) {
      const int r = r0 + m;
      return load4(r < a.B ? S.Hd1 + (int64_t)r * S.ld1 : nullptr, k, H1, true);
    };
    const bool vw = ((po.W2 | H1) & 3) == 0;
    auto fb = [&](int n, int k) {
      const int j = c0 + n;
      return load4(j < a.H2 ? W2 + (int64_t)j * H1 : nullptr, k, H1, vw);
    };
    tile_product<4>(H1, fa, fb, red);
  }
  const TileOut o = tile_sum<4>(red);
  const int j = c0 + o.n, r = r0 + o.m0;
  const bool jok = j < a.H2;
  const float b2 = jok ? a.P[po.b2 + j] : 0.0f, w3 = jok ? a.P[po.w3 + j] : 0.0f;
  v4f act;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const bool ok = jok && r + q < a.B;
    const float pre = o.v[q] + b2;
    act[q] = ok ? gelu(pre) : 0.0f;
    s_h[o.m0 + q][o.n] = act[q] * w3;
    if (kTrain && ok) S.G2[(int64_t)(r + q) * S.ld2 + j] = gelu_grad(pre);
  }
  if (kTrain && jok && r < S.B4) *reinterpret_cast<v4f*>(S.Hd2T + (int64_t)j * S.B4 + r) = act;
  __syncthreads();
  if (tid < kT && r0 + tid < a.B) {
    float sum = 0.0f;
    for (int n = 0; n < kT; ++n) sum += s_h[tid][n];
    S.ypart[(int64_t)(r0 + tid) * S.nT2 + blockIdx.x] = sum;
  }
}

// y = sum of the head shares in tile order + b3.
__device__ __forceinline__ float head_sum(const Args& a, int r) {
  const float* yp = a.s.ypart + (int64_t)r * a.s.nT2;
  const int n = a.s.nT2;
  const float b3 = a.P[offs(a.L, a.H1, a.H2).b3];
  float y = 0.0f;
  // eight shares loaded before they are added (a load per addition would be
  // a memory round trip each)
  for (int t0 = 0; t0 < n; t0 += 8) {
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = yp[min(t0 + q, n - 1)];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (t0 + q < n) y += v[q];
  }
  return y + b3;
}

__global__ __launch_bounds__(kThreads) void head_kernel(Args a, const DevState* halt) {
  if (run_halted(halt)) return;
  const int r = blockIdx.x * kThreads + threadIdx.x;
  if (r < a.B) a.y[r] = head_sum(a, r);
}

// Backward through the head and W2: tile (row tile blockIdx.y, layer-1 unit
// tile blockIdx.x) of dA1 = (dA2 W2) gelu'(A1), with dA2 formed as the left
// operand is read; the row tile's unit tiles also store dA2 transposed (a
// slice of the H2 units each), the first one dy and the squared residuals.
template <bool kV>
__global__ __launch_bounds__(kThreads) void back_kernel(Args a, const DevState* halt) {
  if (run_halted(halt)) return;
  __shared__ v4f red[16 * 64];
  __shared__ float s_dy[kT];
  __shared__ float s_w3[kV ? kMaxHidden : 1];
  const Scratch& S = a.s;
  const int c0 = blockIdx.x * kT, r0 = blockIdx.y * kT, tid = threadIdx.x, H2 = a.H2;
  const bool lead = blockIdx.x == 0;
  // dA2 is stored transposed by the row tile's unit tiles, each its own
  // slice of the H2 units (every element once, the work shared)
  const int ds = (H2 + gridDim.x - 1) / gridDim.x, dk0 = blockIdx.x * ds, dk1 = min(H2, dk0 + ds);
  if (tid < kT) {
    const int r = r0 + tid;
    float dy = 0.0f;
    if (r < a.B) {
      const float res = head_sum(a, r) - S.tv[r];
      dy = 2.0f * res / (float)a.B;
      if (lead) {
        S.dyres[r] = dy;
        S.dyres[S.B4 + r] = res * res;
      }
    }
    s_dy[tid] = dy;
  }
  const float* w3 = a.P + offs(a.L, a.H1, H2).w3;
  if constexpr (kV) {
    // w3 in LDS (read per element where a group is used); G2 rows of ld2 >=
    // H2 rounded up to 4 floats, W2T rows of H2 floats (a multiple of 4)
    for (int j = tid; j < H2; j += kThreads) s_w3[j] = w3[j];
    __syncthreads();
    auto la = [&](int m, int k) { return raw4(S.G2 + (int64_t)(r0 + m < a.B ? r0 + m : 0) * S.ld2, k, H2); };
    auto ma = [&](int m, int k, v4f g2) {
      const int r = r0 + m;
      v4f d;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const bool in = r < a.B && k + s < H2;
        const float v = s_dy[m] * s_w3[in ? k + s : 0] * g2[s];
        d[s] = in ? v : 0.0f;
        if (in && k + s >= dk0 && k + s < dk1) S.D2T[(int64_t)(k + s) * S.B4 + r] = v;
      }
      return d;
    };
    auto lb = [&](int n, int k) { return raw4(a.W2T + (int64_t)(c0 + n < a.H1 ? c0 + n : 0) * H2, k, H2); };
    auto mb = [&](int n, int k, v4f v) { return mask4(v, c0 + n < a.H1, k, H2); };
    tile_product_v<4, 4>(H2, la, ma, lb, mb, red);
  } else {
    __syncthreads();
    auto fa = [&](int m, int k) {
      const int r = r0 + m;
      v4f d = {0.0f, 0.0f, 0.0f, 0.0f};
      if (r >= a.B) return d;
      const v4f g2 = load4(S.G2 + (int64_t)r * S.ld2, k, H2, true);
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (k + s < H2) {
          d[s] = s_dy[m] * w3[k + s] * g2[s];
          if (k + s >= dk0 && k + s < dk1) S.D2T[(int64_t)(k + s) * S.B4 + r] = d[s];
        }
      return d;
    };
    const bool vw = (H2 & 3) == 0;
    auto fb = [&](int n, int k) {
      const int i = c0 + n;
      return load4(i < a.H1 ? a.W2T + (int64_t)i * H2 : nullptr, k, H2, vw);
    };
    tile_product<4>(H2, fa, fb, red);
  }
  const TileOut o = tile_sum<4>(red);
  const int i = c0 + o.n, r = r0 + o.m0;
  if (i < a.H1 && r < S.B4) {
    const v4f g1 = *reinterpret_cast<const v4f*>(S.G1T + (int64_t)i * S.B4 + r);
    v4f d;
#pragma unroll
    for (int q = 0; q < 4; ++q) d[q] = r + q < a.B ? o.v[q] * g1[q] : 0.0f;
    *reinterpret_cast<v4f*>(S.D1T + (int64_t)i * S.B4 + r) = d;
  }
}

struct GradArgs {
  int L, H1, H2, B;
  Scratch s;
  float* params;  // Adam: updated in place
  float* W2T;
  float* m;
  float* v;
  int32_t* step;  // step counter, then an arrival counter (zero between launches)
  float lr;
  float* grads;   // gradient output instead of Adam (null: Adam)
  float* loss;    // mean squared error of the rows (may be null)
};

// One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on parameter p with
// gradient g at step t; refreshes W2T for an element of W2.
__device__ __forceinline__ void adam_update(float* params, float* m, float* v, float* W2T, int64_t p,
                                            float g, int t, float lr, int L, int H1, int H2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mi = b1 * m[p] + (1.0f - b1) * g;
  const float vi = b2 * v[p] + (1.0f - b2) * g * g;
  m[p] = mi;
  v[p] = vi;
  const float mhat = mi / (1.0f - powf(b1, (float)t));
  const float vhat = vi / (1.0f - powf(b2, (float)t));
  const float nv = params[p] - lr * mhat / (sqrtf(vhat) + eps);
  params[p] = nv;
  const int64_t o2 = (int64_t)H1 * L + H1, n2 = (int64_t)H2 * H1;
  if (p >= o2 && p < o2 + n2) {
    const int64_t q = p - o2, j = q / H1, i = q - j * H1;
    W2T[i * H2 + j] = nv;
  }
}

// The parameter-gradient products, as a list of jobs C (M x N) = A Bt^T over
// the B rows; the element (m, n) of a job is parameter p0 + m * ldp + n.
struct Job {
  const float* A;
  const float* Bt;
  int M, N;
  int64_t p0, ldp;
  int scalars;  // the (db3, loss) job
};

__device__ bool find_job(const GradArgs& g, int wg, Job& job, int& tm, int& tn) {
  const Scratch& S = g.s;
  const Offs o = offs(g.L, g.H1, g.H2);
  const Job list[6] = {
      {S.D1T, S.XT, g.H1, g.L, o.W1, g.L, 0},      // dW1 = dA1^T X
      {S.D2T, S.Hd1T, g.H2, g.H1, o.W2, g.H1, 0},  // dW2 = dA2^T H1
      {S.D1T, S.ones, g.H1, 1, o.b1, 1, 0},        // db1 = dA1^T 1
      {S.D2T, S.ones, g.H2, 1, o.b2, 1, 0},        // db2 = dA2^T 1
      {S.Hd2T, S.dyres, g.H2, 1, o.w3, 1, 0},      // dw3 = H2^T dy
      {S.dyres, S.ones, 2, 1, o.b3, 0, 1},         // db3 = dy^T 1, loss sum
  };
  for (int q = 0; q < 6; ++q) {
    const int nm = (list[q].M + kT - 1) / kT, nn = (list[q].N + kT - 1) / kT;
    if (wg < nm * nn) {
      job = list[q];
      tm = wg / nn;
      tn = wg - tm * nn;
      return true;
    }
    wg -= nm * nn;
  }
  return false;
}

// The gradient products contract over all B rows.  Each parameter tile's
// product is split into kSplit consecutive row ranges, one workgroup each
// (4 waves interleaving 16-row groups), so that the products cover the whole
// device; a workgroup stores its 32 x 32 partial at device scope, and the
// last of a tile's workgroups to arrive adds the partials in range order and
// applies Adam to the tile (or writes the gradient).
constexpr int kGradWaves = 4;

int grad_tiles(const MlpDims& d) {
  auto t = [](int M, int N) { return ((M + kT - 1) / kT) * ((N + kT - 1) / kT); };
  return t(d.H1, d.L) + t(d.H2, d.H1) + t(d.H1, 1) + t(d.H2, 1) + t(d.H2, 1) + t(2, 1);
}

__global__ __launch_bounds__(64 * kGradWaves) void grads_kernel(GradArgs g, const DevState* halt) {
  if (run_halted(halt)) return;
  __shared__ v4f red[kGradWaves * 4 * 64];
  __shared__ int s_last;
  const int B4 = g.s.B4;
  const int t = g.grads ? 0 : *g.step + 1;
  const int tile = (int)blockIdx.x / kSplit, split = (int)blockIdx.x - tile * kSplit;
  Job job{};
  int tm = 0, tn = 0;
  const bool have = find_job(g, tile, job, tm, tn);
  // rows of this split: [k0, k1), ranges of a multiple of 16 rows
  const int kc = ((g.B + kSplit - 1) / kSplit + 15) & ~15;
  const int k0 = min(split * kc, g.B), k1 = min(g.B, k0 + kc);
  const int m0 = tm * kT, n0 = tn * kT;
  // rows of B4 floats (B rounded up to 4) from k0; a missing row reads the
  // ones row
  const int K = k1 - k0;
  auto la = [&](int m, int k) {
    const bool ok = have && m0 + m < job.M;
    return raw4((ok ? job.A + (int64_t)(m0 + m) * B4 : g.s.ones) + k0, k, K);
  };
  auto ma = [&](int m, int k, v4f v) { return mask4(v, have && m0 + m < job.M, k, K); };
  auto lb = [&](int n, int k) {
    const bool ok = have && n0 + n < job.N;
    return raw4((ok ? job.Bt + (int64_t)(n0 + n) * B4 : g.s.ones) + k0, k, K);
  };
  auto mb = [&](int n, int k, v4f v) { return mask4(v, have && n0 + n < job.N, k, K); };
  tile_product_v<kGradWaves, 4>(K, la, ma, lb, mb, red);
  const TileOut o = tile_sum<kGradWaves>(red);
  const int64_t tsz = kT * kT;
  float* part = g.s.gpart + ((int64_t)tile * kSplit + split) * tsz;
  if (have) {
#pragma unroll
    for (int q = 0; q < 4; ++q) st_agent(part + (o.m0 + q) * kT + o.n, o.v[q]);
  }
  stores_done();
  __syncthreads();
  if (threadIdx.x == 0) s_last = atomicAdd(&g.s.gcnt[tile], 1u) == (uint32_t)(kSplit - 1);
  __syncthreads();
  if (s_last) {
    const int n = n0 + o.n;
    if (have && n < job.N) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + o.m0 + q;
        if (m >= job.M) continue;
        const float* pt = g.s.gpart + (int64_t)tile * kSplit * tsz + (o.m0 + q) * kT + o.n;
        float val = 0.0f;
        for (int sp = 0; sp < kSplit; ++sp) val += ld_agent(pt + sp * tsz);
        if (job.scalars && m == 1) {
          if (g.loss) *g.loss = val / (float)g.B;
          continue;
        }
        const int64_t p = job.p0 + (int64_t)m * job.ldp + n;
        if (g.grads)
          g.grads[p] = val;
        else
          adam_update(g.params, g.m, g.v, g.W2T, p, val, t, g.lr, g.L, g.H1, g.H2);
      }
    }
    if (threadIdx.x == 0) g.s.gcnt[tile] = 0u;
  }
  if (g.grads) return;
  __syncthreads();
  if (threadIdx.x == 0)
    s_last = atomicAdd(reinterpret_cast<uint32_t*>(g.step + 1), 1u) == gridDim.x - 1;
  __syncthreads();
  if (s_last && threadIdx.x == 0) {
    *g.step = t;
    g.step[1] = 0;
  }
}

// One Adam step from a given gradient (every parameter); the last workgroup
// stores the step count.
__global__ void adam_kernel(float* params, float* W2T, const float* grads, float* m, float* v,
                            int32_t* step, float lr, int L, int H1, int H2, int64_t total,
                            const DevState* halt) {
  if (run_halted(halt)) return;
  __shared__ int s_last;
  const int t = *step + 1;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < total) adam_update(params, m, v, W2T, p, grads[p], t, lr, L, H1, H2);
  __syncthreads();
  if (threadIdx.x == 0) s_last = atomicAdd(reinterpret_cast<uint32_t*>(step + 1), 1u) == gridDim.x - 1;
  __syncthreads();
  if (s_last && threadIdx.x == 0) {
    *step = t;
    step[1] = 0;
  }
}

// W2T from the parameters.
__global__ void transpose_kernel(const float* __restrict__ P, float* __restrict__ W2T, int L, int H1,
                                 int H2) {
  const int64_t n2 = (int64_t)H2 * H1;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n2) {
    const int64_t j = e / H1, i = e - j * H1;
    W2T[i * H2 + j] = P[(int64_t)H1 * L + H1 + e];
  }
}

// He-uniform init: block (layer, row, col, MLP_INIT) word 0 -> u in (0, 1),
// w = sqrt(6 / fan_in) (2u - 1); biases and moments zero.
__global__ void init_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            int L, int H1, int H2, uint32_t k0, uint32_t k1) {
  const int64_t n1 = (int64_t)H1 * L, n2 = (int64_t)H2 * H1;
  const int64_t total = n1 + H1 + n2 + H2 + H2 + 1;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  m[i] = 0.0f;
  v[i] = 0.0f;
  int layer = 0, cols = 1;
  int64_t j = i;
  if (j < n1) {
    layer = 1;
    cols = L;
  } else if ((j -= n1) < H1) {
    p[i] = 0.0f;
    return;
  } else if ((j -= H1) < n2) {
    layer = 2;
    cols = H1;
  } else if ((j -= n2) < H2) {
    p[i] = 0.0f;
    return;
  } else if ((j -= H2) < H2) {
    layer = 3;
    cols = H2;
  } else {
    p[i] = 0.0f;
    return;
  }
  const uint32_t r = (uint32_t)(j / cols), c = (uint32_t)(j % cols);
  const u32x4 b = philox((uint32_t)layer, r, c, kTagMlpInit, k0, k1);
  const double u = ((double)(b.x >> 8) + 0.5) * 0x1p-24;
  p[i] = (float)(sqrt(6.0 / (double)cols) * (2.0 * u - 1.0));
}

Args base_args(const MlpDims& d, const float* params, const float* W2T, int B, float* scratch,
               bool train) {
  Args a{};
  a.P = params;
  a.W2T = W2T;
  a.L = d.L;
  a.H1 = d.H1;
  a.H2 = d.H2;
  a.B = B;
  scratch_layout(d, B, train, scratch, &a.s);
  return a;
}

dim3 grid_of(int units, int rows) {
  return dim3((unsigned)((units + kT - 1) / kT), (unsigned)((rows + kT - 1) / kT));
}

// Whether every operand row of the layer products can be read as whole
// 16-byte groups: widths that are multiples of 4 and 16-byte aligned rows
// (inputs, parameters, transposed W2).
bool vec_rows(const Args& a) {
  auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  return (a.L & 3) == 0 && (a.H1 & 3) == 0 && (a.H2 & 3) == 0 && al(a.X ? a.X : a.buf) && al(a.P) &&
         al(a.W2T);
}

// The three training launches before the gradient products.
template <bool kV>
void launch_train_rows_v(const Args& a, const DevState* halt, hipStream_t s) {
  hipLaunchKernelGGL((layer1_kernel<true, kV>), grid_of(a.H1, a.B), dim3(kThreads), 0, s, a, halt);
  hipLaunchKernelGGL((layer2_kernel<true, kV>), grid_of(a.H2, a.B), dim3(kThreads), 0, s, a, halt);
  hipLaunchKernelGGL(back_kernel<kV>, grid_of(a.H1, a.B), dim3(kThreads), 0, s, a, halt);
}
hipError_t launch_train_rows(const Args& a, const DevState* halt, hipStream_t s) {
  if (vec_rows(a))
    launch_train_rows_v<true>(a, halt, s);
  else
    launch_train_rows_v<false>(a, halt, s);
  return hipGetLastError();
}

GradArgs grad_args(const MlpDims& d, const Args& a) {
  GradArgs g{};
  g.L = d.L;
  g.H1 = d.H1;
  g.H2 = d.H2;
  g.B = a.B;
  g.s = a.s;
  return g;
}

hipError_t launch_grads(const MlpDims& d, const GradArgs& g, const DevState* halt, hipStream_t s) {
  hipLaunchKernelGGL(grads_kernel, dim3((unsigned)(grad_tiles(d) * kSplit)), dim3(64 * kGradWaves), 0, s,
                     g, halt);
  return hipGetLastError();
}

__global__ void clear_counts_kernel(uint32_t* c, int n) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) c[i] = 0u;
}

}  // namespace

MlpLayout mlp_layout(int L, int H1, int H2) {
  MlpLayout o;
  o.W1 = 0;
  o.b1 = o.W1 + (int64_t)H1 * L;
  o.W2 = o.b1 + H1;
  o.b2 = o.W2 + (int64_t)H2 * H1;
  o.w3 = o.b2 + H2;
  o.b3 = o.w3 + H2;
  o.total = o.b3 + 1;
  return o;
}

int64_t mlp_scratch_floats(const MlpDims& d, int batch, int rows_max) {
  return std::max(scratch_layout(d, batch, true, nullptr, nullptr),
                  scratch_layout(d, rows_max, false, nullptr, nullptr));
}

hipError_t mlp_transpose(const MlpDims& d, const float* params, float* W2T, hipStream_t s) {
  const int64_t n = (int64_t)d.H2 * d.H1;
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, params, W2T,
                     d.L, d.H1, d.H2);
  return hipGetLastError();
}

hipError_t mlp_scratch_init(const MlpDims& d, float* scratch, hipStream_t s) {
  Scratch z{};
  scratch_layout(d, 4, true, scratch, &z);
  const int n = grad_tiles(d);
  hipLaunchKernelGGL(clear_counts_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, z.gcnt, n);
  return hipGetLastError();
}

hipError_t mlp_init(const MlpDims& d, float* params, float* m, float* v, float* W2T, uint64_t seed,
                    hipStream_t s) {
  const int64_t n = mlp_layout(d.L, d.H1, d.H2).total;
  hipLaunchKernelGGL(init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, params, m, v,
                     d.L, d.H1, d.H2, (uint32_t)seed, (uint32_t)(seed >> 32));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return mlp_transpose(d, params, W2T, s);
}

hipError_t mlp_forward(const MlpDims& d, const float* params, const float* W2T, const float* X, int B,
                       float* y, float* scratch, const DevState* halt, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  Args a = base_args(d, params, W2T, B, scratch, false);
  a.X = X;
  a.y = y;
  if (vec_rows(a)) {
    hipLaunchKernelGGL((layer1_kernel<false, true>), grid_of(d.H1, B), dim3(kThreads), 0, s, a, halt);
    hipLaunchKernelGGL((layer2_kernel<false, true>), grid_of(d.H2, B), dim3(kThreads), 0, s, a, halt);
  } else {
    hipLaunchKernelGGL((layer1_kernel<false, false>), grid_of(d.H1, B), dim3(kThreads), 0, s, a, halt);
    hipLaunchKernelGGL((layer2_kernel<false, false>), grid_of(d.H2, B), dim3(kThreads), 0, s, a, halt);
  }
  hipLaunchKernelGGL(head_kernel, dim3((unsigned)((B + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                     a, halt);
  return hipGetLastError();
}

hipError_t mlp_grads(const MlpDims& d, const float* params, const float* W2T, const float* X,
                     const float* target, int B, float* scratch, float* grads, float* loss,
                     const DevState* halt, hipStream_t s) {
  Args a = base_args(d, params, W2T, B, scratch, true);
  a.X = X;
  a.target = target;
  hipError_t e = launch_train_rows(a, halt, s);
  if (e != hipSuccess) return e;
  GradArgs g = grad_args(d, a);
  g.grads = grads;
  g.loss = loss;
  return launch_grads(d, g, halt, s);
}

hipError_t mlp_train_step(const MlpDims& d, float* params, float* W2T, float* m, float* v,
                          int32_t* step, float lr, const float* buf, const float* bufy,
                          const SurState* ss, uint64_t seed, int B, int n_recent, int cap,
                          float* scratch, float* loss, const DevState* halt, hipStream_t s) {
  Args a = base_args(d, params, W2T, B, scratch, true);
  a.buf = buf;
  a.bufy = bufy;
  a.ss = ss;
  a.step = step;
  a.k0 = (uint32_t)seed;
  a.k1 = (uint32_t)(seed >> 32);
  a.n_recent = n_recent;
  a.cap = cap;
  hipError_t e = launch_train_rows(a, halt, s);
  if (e != hipSuccess) return e;
  GradArgs g = grad_args(d, a);
  g.params = params;
  g.W2T = W2T;
  g.m = m;
  g.v = v;
  g.step = step;
  g.lr = lr;
  g.loss = loss;
  return launch_grads(d, g, halt, s);
}

hipError_t mlp_adam(const MlpDims& d, float* params, float* W2T, const float* grads, float* m, float* v,
                    int32_t* step, float lr, const DevState* halt, hipStream_t s) {
  const int64_t total = mlp_layout(d.L, d.H1, d.H2).total;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, params, W2T,
                     grads, m, v, step, lr, d.L, d.H1, d.H2, total, halt);
  return hipGetLastError();
}

}  // namespace game
