// Block projector applied inside kernels (Sec. 3.1 / 3.2: Pi_B is block
// diagonal, one block per row of P).  Row i's values are spread over a group
// of G lanes, L per lane; `oc` holds each value's column (-1: not a slot of
// the row).  Pi_i x = x - G_i W_i G_i^T x with G_i = B_c(J_i, :) gathered on
// the fly and W_i the pseudo-inverse of G_i^T G_i (for m = 1, W_i = 1/g^T g,
// recomputed here).  All G lanes of the group must call it (shuffles).
#pragma once

#include "common.hpp"

namespace emin {

__device__ __forceinline__ int packed_idx(int a, int b, int m) {
  return a * m - (a * (a - 1)) / 2 + (b - a);
}

// M1: compile only the m = 1 path (fewer registers in the hot kernels).
template <int G, int L, bool M1 = false>
__device__ __forceinline__ void project_row(double* v, const int* oc,
                                            const double* __restrict__ bc,
                                            const double* __restrict__ w, int m, bool valid) {
  if (M1 || m == 1) {
    double g[L];
    double gx = 0.0, gg = 0.0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
      g[t] = (oc[t] >= 0) ? bc[oc[t]] : 0.0;
      gx += g[t] * v[t];
      gg += g[t] * g[t];
    }
    gx = group_sum<G>(gx);
    gg = group_sum<G>(gg);
    if (gg > 0.0) {
      const double c = gx / gg;
#pragma unroll
      for (int t = 0; t < L; ++t) v[t] -= g[t] * c;
    }
    return;
  }
  if constexpr (!M1) {
    double cs[kMaxM];
#pragma unroll
    for (int x = 0; x < kMaxM; ++x) cs[x] = 0.0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
      if (oc[t] < 0) continue;
#pragma unroll
      for (int x = 0; x < kMaxM; ++x)
        if (x < m) cs[x] += bc[(long)oc[t] * m + x] * v[t];
    }
#pragma unroll
    for (int x = 0; x < kMaxM; ++x)
      if (x < m) cs[x] = group_sum<G>(cs[x]);
    double d[kMaxM];
#pragma unroll
    for (int x = 0; x < kMaxM; ++x) {
      double s = 0.0;
      if (valid && x < m) {
#pragma unroll
        for (int y = 0; y < kMaxM; ++y) {
          if (y >= m) continue;
          const int pi = (x <= y) ? packed_idx(x, y, m) : packed_idx(y, x, m);
          s += w[pi] * cs[y];
        }
      }
      d[x] = s;
    }
#pragma unroll
    for (int t = 0; t < L; ++t) {
      if (oc[t] < 0) continue;
      double s = 0.0;
#pragma unroll
      for (int x = 0; x < kMaxM; ++x)
        if (x < m) s += bc[(long)oc[t] * m + x] * d[x];
      v[t] -= s;
    }
  }
}

// Re-projection onto the constraint (the correction step of Alg. 2):
// v += G_i W_i (b_i - G_i^T v).
template <int G, int L, bool M1 = false>
__device__ __forceinline__ void correct_row(double* v, const int* oc,
                                            const double* __restrict__ bc,
                                            const double* __restrict__ w,
                                            const double* __restrict__ b, int m, bool valid) {
  if (M1 || m == 1) {
    double g[L];
    double gx = 0.0, gg = 0.0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
      g[t] = (oc[t] >= 0) ? bc[oc[t]] : 0.0;
      gx += g[t] * v[t];
      gg += g[t] * g[t];
    }
    gx = group_sum<G>(gx);
    gg = group_sum<G>(gg);
    if (valid && gg > 0.0) {
      const double c = (b[0] - gx) / gg;
#pragma unroll
      for (int t = 0; t < L; ++t) v[t] += g[t] * c;
    }
    return;
  }
  if constexpr (!M1) {
    double cs[kMaxM];
#pragma unroll
    for (int x = 0; x < kMaxM; ++x) cs[x] = 0.0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
      if (oc[t] < 0) continue;
#pragma unroll
      for (int x = 0; x < kMaxM; ++x)
        if (x < m) cs[x] += bc[(long)oc[t] * m + x] * v[t];
    }
#pragma unroll
    for (int x = 0; x < kMaxM; ++x)
      if (x < m) cs[x] = group_sum<G>(cs[x]);
    double d[kMaxM];
#pragma unroll
    for (int x = 0; x < kMaxM; ++x) {
      double s = 0.0;
      if (valid && x < m) {
#pragma unroll
        for (int y = 0; y < kMaxM; ++y) {
          if (y >= m) continue;
          const int pi = (x <= y) ? packed_idx(x, y, m) : packed_idx(y, x, m);
          s += w[pi] * (b[y] - cs[y]);
        }
      }
      d[x] = s;
    }
#pragma unroll
    for (int t = 0; t < L; ++t) {
      if (oc[t] < 0) continue;
      double s = 0.0;
#pragma unroll
      for (int x = 0; x < kMaxM; ++x)
        if (x < m) s += bc[(long)oc[t] * m + x] * d[x];
      v[t] += s;
    }
  }
}

}  // namespace emin
