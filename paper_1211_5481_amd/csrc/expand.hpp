// Basis values of one feature value (eq. 1; eq. 6 for trig), shared by the
// basis, re-score and prediction kernels.  Evaluated in double by the
// three-term recurrences (Chebyshev, Legendre, the cos/sin multiple-angle
// recurrence seeded by one sincos); power by repeated products.  The K values
// are handed to put(k, value) in column order: phi_1..phi_D, or for trig
// cos(1x)..cos(Dx) then sin(1x)..sin(Dx).
#pragma once

#include <hip/hip_runtime.h>

#include "game.h"

namespace game {

// 1/(j+1), j = 1..kLegInv, correctly rounded at compile time: the Legendre
// recurrence multiplies by it instead of dividing by j+1 (a double division
// is a dozen FP64 instructions; the product differs from the quotient by at
// most about an ulp of double).  Higher degrees divide.
constexpr int kLegInv = 64;
struct LegInvTable {
  double v[kLegInv];
};
constexpr LegInvTable make_leg_inv() {
  LegInvTable t{};
  for (int i = 0; i < kLegInv; ++i) t.v[i] = 1.0 / (double)(i + 2);
  return t;
}
__device__ constexpr LegInvTable kLegInvTab = make_leg_inv();

template <typename Put>
__device__ __forceinline__ void expand_feature(int basis, int D, double x, Put put) {
  if (basis == GAME_BASIS_POWER) {
    double p = x;
    for (int k = 0; k < D; ++k) {
      put(k, p);
      p *= x;
    }
  } else if (basis == GAME_BASIS_CHEBYSHEV) {
    double prev = 1.0, cur = x;
    for (int k = 0; k < D; ++k) {
      put(k, cur);
      const double nxt = 2.0 * x * cur - prev;
      prev = cur;
      cur = nxt;
    }
  } else if (basis == GAME_BASIS_LEGENDRE) {
    double prev = 1.0, cur = x;
    for (int k = 0; k < D; ++k) {
      put(k, cur);
      const double j = (double)(k + 1);
      const double num = (2.0 * j + 1.0) * x * cur - j * prev;
      const double nxt = k < kLegInv ? num * kLegInvTab.v[k] : num / (j + 1.0);
      prev = cur;
      cur = nxt;
    }
  } else {
    double s1, c1;
    sincos(x, &s1, &c1);
    double cp = 1.0, cc = c1, sp = 0.0, sc = s1;
    for (int k = 0; k < D; ++k) {
      put(k, cc);
      put(D + k, sc);
      const double cn = 2.0 * c1 * cc - cp;
      const double sn = 2.0 * c1 * sc - sp;
      cp = cc;
      cc = cn;
      sp = sc;
      sc = sn;
    }
  }
}

// The same K values, one at a time in column order (for trig: every cosine,
// then every sine, each sequence its own recurrence), by the same operations
// as expand_feature, so each value is the same double.  The basis is a
// template parameter, so the sequence is branch-free per value.
template <int kBasis>
struct BasisSeq {
  int D, k;
  double x, prev, cur;  // power / Chebyshev / Legendre state; trig: cosines
  double c1, sp, sc;    // trig: cos(x), and the sine recurrence
  __device__ __forceinline__ BasisSeq(int d, double xv) : D(d), k(0), x(xv) {
    prev = 1.0;
    cur = x;
    c1 = sp = sc = 0.0;
    if constexpr (kBasis == GAME_BASIS_TRIG) {
      double s1;
      sincos(x, &s1, &c1);
      cur = c1;
      sc = s1;
    }
  }
  __device__ __forceinline__ double next() {
    double v;
    if constexpr (kBasis == GAME_BASIS_POWER) {
      v = cur;
      cur *= x;
    } else if constexpr (kBasis == GAME_BASIS_CHEBYSHEV) {
      v = cur;
      const double nxt = 2.0 * x * cur - prev;
      prev = cur;
      cur = nxt;
    } else if constexpr (kBasis == GAME_BASIS_LEGENDRE) {
      v = cur;
      const double j = (double)(k + 1);
      const double num = (2.0 * j + 1.0) * x * cur - j * prev;
      const double nxt = k < kLegInv ? num * kLegInvTab.v[k] : num / (j + 1.0);
      prev = cur;
      cur = nxt;
    } else if (k < D) {
      v = cur;
      const double cn = 2.0 * c1 * cur - prev;
      prev = cur;
      cur = cn;
    } else {
      v = sc;
      const double sn = 2.0 * c1 * sc - sp;
      sp = sc;
      sc = sn;
    }
    ++k;
    return v;
  }
};

}  // namespace game
