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

// Wave-wide totals of N per-lane partial sums, returned to every lane as
// uniform values.  Folds the wave down to P = the next power of two >= N
// lanes, reduce-scatters over those P lanes by recursive halving (lane j ends
// up with total j), then reads total j from lane j.  About N + P shuffles
// instead of the N * log2(64) of N separate butterflies.
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int N>
__device__ __forceinline__ void wave_sums(const double (&acc)[N], double (&tot)[N], int lane) {
  static_assert(N >= 1 && N <= kWave, "wave_sums: 1..64 sums");
  constexpr int P = N <= 1 ? 1 : N <= 2 ? 2 : N <= 4 ? 4 : N <= 8 ? 8 : N <= 16 ? 16 : N <= 32 ? 32 : 64;
  double a[P];
#pragma unroll
  for (int j = 0; j < P; ++j) a[j] = j < N ? acc[j] : 0.0;
#pragma unroll
  for (int d = kWave / 2; d >= P; d >>= 1)
#pragma unroll
    for (int j = 0; j < N; ++j) a[j] += __shfl_xor(a[j], d, kWave);
  ReduceScatter<P, P, double>::run(a, lane);
#pragma unroll
  for (int j = 0; j < N; ++j) tot[j] = readlane_d(a[0], j);
}

// As wave_sums, without the broadcast: lane j (j < N) returns total j.
template <int N>
__device__ __forceinline__ double wave_scatter_sums(const double (&acc)[N], int lane) {
  static_assert(N >= 1 && N <= kWave, "wave_scatter_sums: 1..64 sums");
  constexpr int P = N <= 1 ? 1 : N <= 2 ? 2 : N <= 4 ? 4 : N <= 8 ? 8 : N <= 16 ? 16 : N <= 32 ? 32 : 64;
  double a[P];
#pragma unroll
  for (int j = 0; j < P; ++j) a[j] = j < N ? acc[j] : 0.0;
#pragma unroll
  for (int d = kWave / 2; d >= P; d >>= 1)
#pragma unroll
    for (int j = 0; j < N; ++j) a[j] += __shfl_xor(a[j], d, kWave);
  ReduceScatter<P, P, double>::run(a, lane);
  return a[0];
}

// One slot's row of B_c (M entries), 16-byte loads when M is even (rows
// then start on 16-byte boundaries: the array is 256-byte aligned).
template <int M>
__device__ __forceinline__ void load_bc_row(const double* __restrict__ bc, int c, double (&g)[M]) {
  const double* p = bc + (long)c * M;
  if constexpr (M % 2 == 0) {
    using V2 = double __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int x = 0; x < M; x += 2) {
      const V2 q = *reinterpret_cast<const V2*>(p + x);
      g[x] = q.x;
      g[x + 1] = q.y;
    }
  } else {
#pragma unroll
    for (int x = 0; x < M; ++x) g[x] = p[x];
  }
}

// Pi_i for the NR rows of a node (Sec. 3.1), or with CORRECT the
// correction step of Alg. 2 (v += G_i W_i (b_i - G_i^T v)).  The rows share
// one pattern row, so they share G_i = B_c(J_i, :) and W_i (the set-up
// computes W_i from J_i and B_c alone, so the rows' copies are identical).
// Each slot's row of B_c is loaded once for all of them, the NR * M inner
// products G_i^T v are reduced together, and W (packed, of the node's first
// row) is read once with scalar loads; b (CORRECT) holds the NR rows of B,
// row r at b + r * M.
// One wave per node: lane-slot s = lane + 64 t holds v[r][t] with column
// oc[t].  Every oc[t] must be a valid column of B_c, also for slots beyond
// the row (any column of the row will do), and those slots must hold
// v = 0: they then add nothing, and what is left in them on return is
// meaningless.  Every lane of the wave must call it.  M is the constraint
// count.
template <int L, int M, int NR, bool CORRECT = false>
__device__ __forceinline__ void node_apply(double (&v)[NR][L], const int (&oc)[L],
                                           const double* __restrict__ bc, const double* w0,
                                           const double* b, int lane) {
  double cs[NR * M];
#pragma unroll
  for (int j = 0; j < NR * M; ++j) cs[j] = 0.0;
#pragma unroll
  for (int t = 0; t < L; ++t) {
    double g[M];
    load_bc_row<M>(bc, oc[t], g);
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int x = 0; x < M; ++x) cs[r * M + x] += g[x] * v[r][t];
  }
  double tot[NR * M];
  wave_sums<NR * M>(cs, tot, lane);
  if constexpr (CORRECT) {
    Uniform<double>* ub = (Uniform<double>*)b;
#pragma unroll
    for (int j = 0; j < NR * M; ++j) tot[j] = ub[j] - tot[j];
  }
  Uniform<double>* uw = (Uniform<double>*)w0;
  double w[M * (M + 1) / 2];
#pragma unroll
  for (int j = 0; j < M * (M + 1) / 2; ++j) w[j] = uw[j];
  double d[NR][M];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
#pragma unroll
    for (int x = 0; x < M; ++x) {
      double s = 0.0;
#pragma unroll
      for (int y = 0; y < M; ++y)
        s += w[(x <= y) ? packed_idx(x, y, M) : packed_idx(y, x, M)] * tot[r * M + y];
      d[r][x] = CORRECT ? s : -s;
    }
  }
  // reload the B_c rows (cache hits) rather than keep them live across the
  // reduction: fewer registers
  const double* bc2 = bc;
  asm volatile("" : "+s"(bc2));
#pragma unroll
  for (int t = 0; t < L; ++t) {
    double g[M];
    load_bc_row<M>(bc2, oc[t], g);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      double s = 0.0;
#pragma unroll
      for (int x = 0; x < M; ++x) s += g[x] * d[r][x];
      v[r][t] += s;
    }
  }
}

template <int L, int M, int NR>
__device__ __forceinline__ void project_node(double (&v)[NR][L], const int (&oc)[L],
                                             const double* __restrict__ bc, const double* w0,
                                             int lane) {
  node_apply<L, M, NR, false>(v, oc, bc, w0, nullptr, lane);
}

}  // namespace emin
