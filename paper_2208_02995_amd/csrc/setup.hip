// Numeric set-up (Sec. 3.2, Alg. 2) and the preconditioner data.
//
// Row i of P carries the local constraint G_i^T p_i = b_i with
// G_i = B_c(J_i, :) (l_i x m).  Instead of storing an orthonormal Q_i per row
// (l_i * m values, as many bytes as m extra copies of P), the GPU keeps the
// m x m pseudo-inverse W_i of the Gram matrix G_i^T G_i (m(m+1)/2 values) and
// re-gathers G_i from B_c, which stays cache resident.  Then
//   Pi_i x = x - G_i W_i G_i^T x           (= x - Q_i Q_i^T x)
//   delta_i = G_i W_i r_i,  r_i = b_i - G_i^T p_hat_i   (min-norm correction)
// Full-rank rows factor the Gram matrix by Cholesky; rows whose pivots fall
// below max(l_i, m) * 1e3 * eps of the largest diagonal (rank deficient, or
// l_i < m) go to a fallback that diagonalizes the Gram matrix (cyclic Jacobi)
// and keeps the eigenvalues above that tolerance -- the pseudo-inverse
// counterpart of the SVD branch of Alg. 2.
#include <float.h>

#include "common.hpp"
#include "launch.hpp"
#include "project.hpp"

namespace emin {

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------------ structure --

// The stored diagonal must exist in every row of A.
__global__ __launch_bounds__(kBlock) void k_diag_has(const int* __restrict__ arp,
                                                    const int* __restrict__ aci, int n,
                                                    int* flags) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int lo = arp[i], hi = arp[i + 1] - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int c = aci[mid];
    if (c == i) return;
    if (c < i) lo = mid + 1; else hi = mid - 1;
  }
  atomicOr(flags, 1 << kFlagNoDiag);
}

// Node a = rows bs*a .. bs*a+bs-1.  what & 1 -> kFlagNodePattern: the rows do
// not share one pattern row.  what & 2 -> kFlagNodeA: A's rows of the node
// differ, or are not made of complete aligned bs-blocks (needed by the node
// masked product and by node-level pattern growth).
__global__ __launch_bounds__(kBlock) void k_check_nodes(const int* __restrict__ arp,
                                                       const int* __restrict__ aci,
                                                       const int* __restrict__ prp,
                                                       const int* __restrict__ pci, int nnodes,
                                                       int bs, int what, int* flags) {
  // one wave per node, lanes over the entries of the node's first row
  const int lane = threadIdx.x % kWave;
  const int a = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  if (a >= nnodes) return;
  const int r0 = a * bs;
  if (what & 1) {
    const int pl = prp[r0 + 1] - prp[r0];
    bool ok = true;
    for (int r = 1; r < bs; ++r) ok = ok && (prp[r0 + r + 1] - prp[r0 + r] == pl);
    for (int t = lane; ok && t < pl; t += kWave) {
      const int c = pci[prp[r0] + t];
      for (int r = 1; r < bs; ++r) ok = ok && (pci[prp[r0 + r] + t] == c);
    }
    if (!ok) atomicOr(flags, 1 << kFlagNodePattern);
  }
  if (what & 2) {
    const int al = arp[r0 + 1] - arp[r0];
    bool ok = (al % bs) == 0;
    for (int r = 1; r < bs; ++r) ok = ok && (arp[r0 + r + 1] - arp[r0 + r] == al);
    for (int t = lane; ok && t < al; t += kWave) {
      const int j = t % bs;
      const int c0 = aci[arp[r0] + t - j];
      ok = (c0 % bs) == 0;
      for (int r = 0; r < bs; ++r) ok = ok && (aci[arp[r0 + r] + t] == c0 + j);
    }
    if (!ok) atomicOr(flags, 1 << kFlagNodeA);
  }
}

// -------------------------------------------------------------- numeric --

__device__ __forceinline__ int packed_index(int a, int b, int m) {
  // upper triangle, row-major: (a, b) with a <= b
  return a * m - (a * (a - 1)) / 2 + (b - a);
}

__device__ __forceinline__ double lookup_p0(const int* __restrict__ qci,
                                            const double* __restrict__ qv, int q0, int q1,
                                            int c) {
  int lo = q0, hi = q1 - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int v = qci[mid];
    if (v == c) return qv[mid];
    if (v < c) lo = mid + 1; else hi = mid - 1;
  }
  return 0.0;
}

// A row whose G_i has rank below m: counted for the problem and, in the
// batched form, for the matrix holding the row.
__device__ __forceinline__ void count_rank_deficient(const SetupArgs& a, int i) {
  if (a.fixed && a.fixed[i] >= 0) return;  // a fixed COARSE row of P = [W; I]
  atomicAdd(&a.st->rank_def, 1);
  if (a.segs) atomicAdd(&a.segs[a.row_seg[i]].rank_def, 1);
}

__device__ __forceinline__ double rank_tol(int l, int m) {
  return (double)(l > m ? l : m) * 1e3 * DBL_EPSILON;
}

// One group of G lanes per row; lane owns slots lane + G*t (t < L).
template <int G, int L, bool M1>
__global__ __launch_bounds__(kBlock) void k_setup(SetupArgs a) {
  constexpr int ROWS = kBlock / G;
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  const int m = M1 ? 1 : a.m;
  const int ntiles = (a.n + ROWS - 1) / ROWS;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int i = w.t * ROWS + grp;
    if (i >= a.n) continue;  // no group-wide sync below besides shuffles within the group
    const int p0 = a.prp[i];
    const int l = a.prp[i + 1] - p0;
    const int q0 = a.qrp[i], q1 = a.qrp[i + 1];
    // diagonal of A (lane 0 searches, all lanes of the group get it)
    if (lane == 0) {
      int lo = a.arp[i], hi = a.arp[i + 1] - 1;
      double d = 0.0;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int c = a.aci[mid];
        if (c == i) { d = a.av[mid]; break; }
        if (c < i) lo = mid + 1; else hi = mid - 1;
      }
      if (!(d > 0.0)) {
        a.st->done = 4;  // bad diagonal: every later kernel skips
        a.dinv[i] = 0.0;
      } else {
        a.dinv[i] = 1.0 / d;
      }
    }
    double phat[L];
    int col[L];
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int s = lane + G * t;
      col[t] = (s < l) ? a.pci[p0 + s] : -1;
      phat[t] = (s < l) ? lookup_p0(a.qci, a.qv, q0, q1, col[t]) : 0.0;
    }
    if constexpr (M1) {
      double gg = 0.0, gp = 0.0;
#pragma unroll
      for (int t = 0; t < L; ++t) {
        if (col[t] >= 0) {
          const double g = a.bc[col[t]];
          gg += g * g;
          gp += g * phat[t];
        }
      }
      gg = group_sum<G>(gg);
      gp = group_sum<G>(gp);
      const double r = a.B[i] - gp;
      const double coef = (gg > 0.0) ? r / gg : 0.0;
      if (!(gg > 0.0) && lane == 0) count_rank_deficient(a, i);
#pragma unroll
      for (int t = 0; t < L; ++t)
        if (col[t] >= 0) a.p0p[p0 + lane + G * t] = phat[t] + a.bc[col[t]] * coef;
    } else {
      double gram[kMaxM][kMaxM];
      double u[kMaxM];
#pragma unroll
      for (int x = 0; x < kMaxM; ++x) {
        u[x] = 0.0;
#pragma unroll
        for (int y = 0; y < kMaxM; ++y) gram[x][y] = 0.0;
      }
#pragma unroll
      for (int t = 0; t < L; ++t) {
        if (col[t] < 0) continue;
        double g[kMaxM];
#pragma unroll
        for (int x = 0; x < kMaxM; ++x) g[x] = (x < m) ? a.bc[(long)col[t] * m + x] : 0.0;
#pragma unroll
        for (int x = 0; x < kMaxM; ++x) {
          u[x] += g[x] * phat[t];
#pragma unroll
          for (int y = x; y < kMaxM; ++y) gram[x][y] += g[x] * g[y];
        }
      }
#pragma unroll
      for (int x = 0; x < kMaxM; ++x) {
        if (x >= m) continue;
        u[x] = group_sum<G>(u[x]);
#pragma unroll
        for (int y = x; y < kMaxM; ++y)
          if (y < m) gram[x][y] = group_sum<G>(gram[x][y]);
      }
      // Cholesky of the Gram matrix with a relative pivot test
      double maxdiag = 0.0;
#pragma unroll
      for (int x = 0; x < kMaxM; ++x)
        if (x < m) maxdiag = fmax(maxdiag, gram[x][x]);
      const double tol = rank_tol(l, m) * maxdiag;
      double Lc[kMaxM][kMaxM];
      bool ok = (l >= m) && (maxdiag > 0.0);
#pragma unroll
      for (int j = 0; j < kMaxM; ++j) {
        if (j >= m) continue;
        double d = gram[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= Lc[j][k] * Lc[j][k];
        if (!(d > tol)) ok = false;
        const double ljj = sqrt(fmax(d, DBL_MIN));
        Lc[j][j] = ljj;
#pragma unroll
        for (int i2 = j + 1; i2 < kMaxM; ++i2) {
          if (i2 >= m) continue;
          double s = gram[j][i2];
#pragma unroll
          for (int k = 0; k < j; ++k) s -= Lc[i2][k] * Lc[j][k];
          Lc[i2][j] = s / ljj;
        }
      }
      if (!ok) {
        if (lane == 0) {
          const int pos = atomicAdd(a.fb_count, 1);
          a.fb_list[pos] = i;
        }
        continue;
      }
      // inverse of the Cholesky factor, then W = Linv^T Linv
      double Li[kMaxM][kMaxM];
#pragma unroll
      for (int j = 0; j < kMaxM; ++j) {
        if (j >= m) continue;
        Li[j][j] = 1.0 / Lc[j][j];
#pragma unroll
        for (int i2 = j + 1; i2 < kMaxM; ++i2) {
          if (i2 >= m) continue;
          double s = 0.0;
#pragma unroll
          for (int k = j; k < i2; ++k) s += Lc[i2][k] * Li[k][j];
          Li[i2][j] = -s / Lc[i2][i2];
        }
      }
      double W[kMaxM][kMaxM];
#pragma unroll
      for (int x = 0; x < kMaxM; ++x) {
#pragma unroll
        for (int y = x; y < kMaxM; ++y) {
          double s = 0.0;
          if (x < m && y < m) {
#pragma unroll
            for (int k = y; k < kMaxM; ++k)
              if (k < m) s += Li[k][x] * Li[k][y];
          }
          W[x][y] = s;
          W[y][x] = s;
        }
      }
      double coef[kMaxM];
#pragma unroll
      for (int x = 0; x < kMaxM; ++x) {
        double s = 0.0;
#pragma unroll
        for (int y = 0; y < kMaxM; ++y)
          if (x < m && y < m) s += W[x][y] * (a.B[(long)i * m + y] - u[y]);
        coef[x] = s;
      }
#pragma unroll
      for (int t = 0; t < L; ++t) {
        if (col[t] < 0) continue;
        double dl = 0.0;
#pragma unroll
        for (int x = 0; x < kMaxM; ++x)
          if (x < m) dl += a.bc[(long)col[t] * m + x] * coef[x];
        a.p0p[p0 + lane + G * t] = phat[t] + dl;
      }
      // lane x of the group stores row x of the packed W (G >= 1 lanes)
      const int mp = m * (m + 1) / 2;
      double* wr = a.wpk + (long)i * mp;
#pragma unroll
      for (int x = 0; x < kMaxM; ++x) {
        if (x >= m || (x % G) != lane) continue;
#pragma unroll
        for (int y = x; y < kMaxM; ++y)
          if (y < m) wr[packed_index(x, y, m)] = W[x][y];
      }
    }
  }
}

// Inverse of an N x N block (the first bs rows and columns are used) by
// Gauss-Jordan elimination with partial pivoting on [M | I]; false when a
// pivot is not above 1e-14 times the largest diagonal magnitude.  Rows are
// swapped through compile-time indices only (no dynamic register indexing).
template <int N>
__device__ __forceinline__ bool gj_inverse(double (&M)[N][N], double (&Inv)[N][N], int bs) {
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int c = 0; c < N; ++c) Inv[r][c] = (r == c) ? 1.0 : 0.0;
  double scale = 0.0;
#pragma unroll
  for (int r = 0; r < N; ++r)
    if (r < bs) scale = fmax(scale, fabs(M[r][r]));
  bool ok = scale > 0.0;
#pragma unroll
  for (int c = 0; c < N; ++c) {
    if (c >= bs || !ok) break;
    int piv = c;
    double best = fabs(M[c][c]);
#pragma unroll
    for (int r = c + 1; r < N; ++r)
      if (r < bs && fabs(M[r][c]) > best) { piv = r; best = fabs(M[r][c]); }
    if (!(best > 1e-14 * scale)) { ok = false; break; }
#pragma unroll
    for (int r = c + 1; r < N; ++r) {
      if (r != piv) continue;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        double t = M[c][k]; M[c][k] = M[r][k]; M[r][k] = t;
        t = Inv[c][k]; Inv[c][k] = Inv[r][k]; Inv[r][k] = t;
      }
    }
    const double d = 1.0 / M[c][c];
#pragma unroll
    for (int k = 0; k < N; ++k) { M[c][k] *= d; Inv[c][k] *= d; }
#pragma unroll
    for (int r = 0; r < N; ++r) {
      if (r == c || r >= bs) continue;
      const double f = M[r][c];
#pragma unroll
      for (int k = 0; k < N; ++k) { M[r][k] -= f * M[c][k]; Inv[r][k] -= f * Inv[c][k]; }
    }
  }
  return ok;
}

// Alg. 2 for the rows of a node (bs rows sharing one pattern row, checked
// when the problem is created).  They share G = B_c(J, :), hence the Gram
// matrix, its Cholesky factor and W; only p_hat_i and b_i differ.  Three
// kernels over a per-node record in device memory:
//  * sums (one wave per node): the node's diagonal block of A, and the Gram
//    matrix with the bs vectors G^T p_hat_i, reduced over the node's slots
//    (each slot's row of B_c loaded once, 16-byte loads when M is even);
//  * solve (one thread per node): 1 / A_ii, the block inverse (block
//    Jacobi), the Cholesky factorization of the Gram matrix, W and the
//    correction coefficients W (b_i - G^T p_hat_i) -- the small dense
//    algebra once per node rather than once per lane;
//  * apply (one wave per node): p0' = p_hat + G coef on every slot.
// A node that fails the pivot test (or has l < M) sends all its rows to the
// fallback, which handles them one by one.
//
// Record of a node: diagonal block (BS*BS), Gram (packed) and G^T p_hat
// (NS), coefficients (BS*M), status (1: factored, 0: fallback).
template <int BS, int M>
struct NodeRec {
  static constexpr int MP = M * (M + 1) / 2;
  static constexpr int NS = MP + BS * M;
  static constexpr int BLK = 0, SUM = BS * BS, COEF = SUM + NS, OK = COEF + BS * M;
  static constexpr int SIZE = OK + 1;
};

// Sums of the node set-up: the Gram matrix G^T G over the node's slots, and
// G^T p_hat_i = sum over the entries (i, c) of P0's row of P0(i, c) B_c(c, :)
// (P0's row lies inside J, so this is the same sum without locating P0's
// entries among the slots).
template <int BS, int M, int L>
__global__ __launch_bounds__(kBlock) void k_setup_node_sums(SetupArgs a) {
  using R = NodeRec<BS, M>;
  constexpr int WPB = kBlock / kWave;
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  const int nnodes = a.n / BS;
  __shared__ double sblk[WPB][BS * BS];
  Uniform<int>* uarp = (Uniform<int>*)a.arp;
  Uniform<int>* uprp = (Uniform<int>*)a.prp;
  Uniform<int>* uqrp = (Uniform<int>*)a.qrp;
  const int ntiles = (nnodes + WPB - 1) / WPB;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int node = __builtin_amdgcn_readfirstlane(w.t * WPB + wid);
    if (node >= nnodes) continue;
    const int r0 = node * BS;
    double* rec = a.nrec + (long)node * R::SIZE;
    // the node's diagonal block A(r0.., r0..): lanes over the entries of
    // each row (coalesced), the matching ones write their value to LDS (the
    // wave's own LDS writes are seen by its later reads, in order)
    if (a.ablk) {
      // A in full aligned BS x BS blocks: find the node's own block among the
      // blocks of its first row (by their first columns), then read it
      const int e0 = uarp[r0];
      const int nbk = (uarp[r0 + 1] - e0) / BS;
      int k = -1;
      for (int n0 = 0; n0 < nbk && k < 0; n0 += kWave) {
        const int n = n0 + lane;
        const unsigned long long hit = __ballot(n < nbk && a.aci[e0 + n * BS] == r0);
        if (hit) k = n0 + __ffsll((long long)hit) - 1;
      }
      if (lane < BS * BS) {
        const int x = lane / BS, c = lane - x * BS;
        rec[R::BLK + lane] = k >= 0 ? a.av[uarp[r0 + x] + k * BS + c] : 0.0;
      }
    } else {
      if (lane < BS * BS) sblk[wid][lane] = 0.0;
#pragma unroll
      for (int x = 0; x < BS; ++x) {
        const int e1 = uarp[r0 + x + 1];
        for (int e = uarp[r0 + x] + lane; e < e1; e += kWave) {
          const int c = a.aci[e] - r0;
          if (c >= 0 && c < BS) sblk[wid][x * BS + c] = a.av[e];
        }
      }
      if (lane < BS * BS) rec[R::BLK + lane] = sblk[wid][lane];
    }
    const int p0 = uprp[r0];
    const int l = uprp[r0 + 1] - p0;
    double acc[R::NS];
#pragma unroll
    for (int j = 0; j < R::NS; ++j) acc[j] = 0.0;
    // the slot passes this node's row needs (L is the longest row's)
    const int nt = (l + kWave - 1) / kWave;
#pragma unroll
    for (int t = 0; t < L; ++t) {
      if (t >= nt) break;  // uniform over the wave
      const int st = lane + kWave * t;
      const bool on = st < l;
      double g[M];
      load_bc_row<M>(a.bc, a.pci[p0 + (on ? st : 0)], g);
#pragma unroll
      for (int x = 0; x < M; ++x) g[x] = on ? g[x] : 0.0;
#pragma unroll
      for (int x = 0; x < M; ++x)
#pragma unroll
        for (int y = x; y < M; ++y) acc[packed_idx(x, y, M)] += g[x] * g[y];
    }
    // P0's entries of the node's rows (contiguous, rows in order), one a lane
    int qb[BS + 1];
#pragma unroll
    for (int x = 0; x <= BS; ++x) qb[x] = uqrp[r0 + x];
    for (int e = qb[0] + lane; e < qb[BS]; e += kWave) {
      double g[M];
      load_bc_row<M>(a.bc, a.qci[e], g);
      const double v = a.qv[e];
#pragma unroll
      for (int r = 0; r < BS; ++r) {
        const double vr = (e >= qb[r] && e < qb[r + 1]) ? v : 0.0;
#pragma unroll
        for (int x = 0; x < M; ++x) acc[R::MP + r * M + x] += g[x] * vr;
      }
    }
    const double mine = wave_scatter_sums<R::NS>(acc, lane);
    if (lane < R::NS) rec[R::SUM + lane] = mine;
  }
}

template <int BS, int M>
__global__ __launch_bounds__(kBlock) void k_setup_node_solve(SetupArgs a) {
  using R = NodeRec<BS, M>;
  constexpr int MP = R::MP;
  const int node = blockIdx.x * kBlock + threadIdx.x;
  if (node >= a.n / BS) return;
  const int r0 = node * BS;
  double* rec = a.nrec + (long)node * R::SIZE;
  double D[BS][BS];
#pragma unroll
  for (int r = 0; r < BS; ++r)
#pragma unroll
    for (int c = 0; c < BS; ++c) D[r][c] = rec[R::BLK + r * BS + c];
#pragma unroll
  for (int r = 0; r < BS; ++r) {
    const double d = D[r][r];
    if (!(d > 0.0)) {
      a.st->done = 4;  // bad diagonal: every later kernel skips
      a.dinv[r0 + r] = 0.0;
    } else {
      a.dinv[r0 + r] = 1.0 / d;
    }
  }
  if (a.binv && a.bs == BS) {  // block Jacobi: the block's inverse
    double Inv[BS][BS];
    const bool okb = gj_inverse<BS>(D, Inv, BS);
    if (!okb) a.st->done = 4;
#pragma unroll
    for (int r = 0; r < BS; ++r)
#pragma unroll
      for (int c = 0; c < BS; ++c) a.binv[(long)node * BS * BS + r * BS + c] = okb ? Inv[r][c] : 0.0;
  }
  const int l = a.prp[r0 + 1] - a.prp[r0];
  double tot[R::NS];
#pragma unroll
  for (int j = 0; j < R::NS; ++j) tot[j] = rec[R::SUM + j];
  // Cholesky of the Gram matrix with the relative pivot test of the
  // row-wise kernel (G^T G is singular when l < M)
  double maxdiag = 0.0;
#pragma unroll
  for (int x = 0; x < M; ++x) maxdiag = fmax(maxdiag, tot[packed_idx(x, x, M)]);
  const double tol = rank_tol(l, M) * maxdiag;
  bool ok = l >= M && maxdiag > 0.0;
  double Lc[M][M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    double d = tot[packed_idx(j, j, M)];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= Lc[j][k] * Lc[j][k];
    if (!(d > tol)) ok = false;
    const double ljj = sqrt(fmax(d, DBL_MIN));
    Lc[j][j] = ljj;
#pragma unroll
    for (int i2 = j + 1; i2 < M; ++i2) {
      double s = tot[packed_idx(j, i2, M)];
#pragma unroll
      for (int k = 0; k < j; ++k) s -= Lc[i2][k] * Lc[j][k];
      Lc[i2][j] = s / ljj;
    }
  }
  if (!ok) {
#pragma unroll
    for (int r = 0; r < BS; ++r) a.fb_list[atomicAdd(a.fb_count, 1)] = r0 + r;
    rec[R::OK] = 0.0;
    return;
  }
  double Li[M][M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    Li[j][j] = 1.0 / Lc[j][j];
#pragma unroll
    for (int i2 = j + 1; i2 < M; ++i2) {
      double s = 0.0;
#pragma unroll
      for (int k = j; k < i2; ++k) s += Lc[i2][k] * Li[k][j];
      Li[i2][j] = -s / Lc[i2][i2];
    }
  }
  double W[MP];
#pragma unroll
  for (int x = 0; x < M; ++x)
#pragma unroll
    for (int y = x; y < M; ++y) {
      double s = 0.0;
#pragma unroll
      for (int k = y; k < M; ++k) s += Li[k][x] * Li[k][y];
      W[packed_idx(x, y, M)] = s;
    }
#pragma unroll
  for (int r = 0; r < BS; ++r) {
    double bres[M];
#pragma unroll
    for (int y = 0; y < M; ++y) bres[y] = a.B[(long)(r0 + r) * M + y] - tot[MP + r * M + y];
#pragma unroll
    for (int x = 0; x < M; ++x) {
      double s = 0.0;
#pragma unroll
      for (int y = 0; y < M; ++y) s += W[x <= y ? packed_idx(x, y, M) : packed_idx(y, x, M)] * bres[y];
      rec[R::COEF + r * M + x] = s;
    }
    double* wr = a.wpk + (long)(r0 + r) * MP;
#pragma unroll
    for (int j = 0; j < MP; ++j) wr[j] = W[j];
  }
  rec[R::OK] = 1.0;
}

// p0' = p_hat + G coef on the node's slots.  p_hat is zero except at P0's
// entries: the slots' columns go to LDS, each of P0's entries (one a lane)
// finds its slot there by bisection and writes its value into a zeroed LDS
// row, which the slots then read.
template <int BS, int M, int L>
__global__ __launch_bounds__(kBlock) void k_setup_node_apply(SetupArgs a) {
  using R = NodeRec<BS, M>;
  constexpr int WPB = kBlock / kWave;
  constexpr int LM = L * kWave;
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  const int nnodes = a.n / BS;
  __shared__ int scol[WPB][LM];
  __shared__ double sph[WPB][BS][LM];
  Uniform<int>* uprp = (Uniform<int>*)a.prp;
  Uniform<int>* uqrp = (Uniform<int>*)a.qrp;
  const int ntiles = (nnodes + WPB - 1) / WPB;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int node = __builtin_amdgcn_readfirstlane(w.t * WPB + wid);
    if (node >= nnodes) continue;
    Uniform<double>* urec = (Uniform<double>*)(a.nrec + (long)node * R::SIZE);
    if (urec[R::OK] == 0.0) continue;  // the fallback writes these rows
    const int r0 = node * BS;
    int pr[BS], qb[BS + 1];
#pragma unroll
    for (int x = 0; x < BS; ++x) pr[x] = uprp[r0 + x];
#pragma unroll
    for (int x = 0; x <= BS; ++x) qb[x] = uqrp[r0 + x];
    const int l = uprp[r0 + 1] - pr[0];
    const int nt = (l + kWave - 1) / kWave;  // the slot passes this row needs
    bool on[L];
    int so[L], col[L];
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int st = lane + kWave * t;
      on[t] = st < l;
      so[t] = on[t] ? st : 0;
      col[t] = t < nt ? a.pci[pr[0] + so[t]] : 0;
    }
#pragma unroll
    for (int t = 0; t < L; ++t) {
      if (t >= nt) break;  // uniform over the wave
      scol[wid][lane + kWave * t] = col[t];
#pragma unroll
      for (int x = 0; x < BS; ++x) sph[wid][x][lane + kWave * t] = 0.0;
    }
    // (the wave's own LDS writes are seen by its later reads, in order)
    for (int e = qb[0] + lane; e < qb[BS]; e += kWave) {
      const int c = a.qci[e];
      const double v = a.qv[e];
      int lo = 0, hi = l - 1;
      while (lo < hi) {  // first slot with column >= c (c is in J)
        const int mid = (lo + hi) >> 1;
        if (scol[wid][mid] < c) lo = mid + 1; else hi = mid;
      }
#pragma unroll
      for (int x = 0; x < BS; ++x)
        if (e >= qb[x] && e < qb[x + 1]) sph[wid][x][lo] = v;
    }
    double coef[BS][M];
#pragma unroll
    for (int r = 0; r < BS; ++r)
#pragma unroll
      for (int x = 0; x < M; ++x) coef[r][x] = urec[R::COEF + r * M + x];
#pragma unroll
    for (int t = 0; t < L; ++t) {
      if (t >= nt) break;  // uniform over the wave
      double g[M];
      load_bc_row<M>(a.bc, col[t], g);
#pragma unroll
      for (int r = 0; r < BS; ++r) {
        double dl = 0.0;
#pragma unroll
        for (int x = 0; x < M; ++x) dl += g[x] * coef[r][x];
        if (on[t]) a.p0p[pr[r] + so[t]] = sph[wid][r][lane + kWave * t] + dl;
      }
    }
  }
}

// Rank-deficient rows: one thread per listed row; symmetric eigen-solve of
// the m x m Gram matrix by cyclic Jacobi rotations, pseudo-inverse on the
// eigenvalues above the rank tolerance.
__global__ __launch_bounds__(kBlock) void k_setup_fallback(SetupArgs a) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= *a.fb_count) return;
  const int i = a.fb_list[t];
  const int m = a.m;
  const int p0 = a.prp[i], p1 = a.prp[i + 1];
  const int l = p1 - p0;
  const int q0 = a.qrp[i], q1 = a.qrp[i + 1];
  double M[kMaxM][kMaxM], V[kMaxM][kMaxM], u[kMaxM];
  for (int x = 0; x < m; ++x) {
    u[x] = 0.0;
    for (int y = 0; y < m; ++y) { M[x][y] = 0.0; V[x][y] = (x == y) ? 1.0 : 0.0; }
  }
  for (int s = p0; s < p1; ++s) {
    const int c = a.pci[s];
    const double ph = lookup_p0(a.qci, a.qv, q0, q1, c);
    for (int x = 0; x < m; ++x) {
      const double gx = a.bc[(long)c * m + x];
      u[x] += gx * ph;
      for (int y = 0; y < m; ++y) M[x][y] += gx * a.bc[(long)c * m + y];
    }
  }
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int x = 0; x < m; ++x) {
      dia += M[x][x] * M[x][x];
      for (int y = x + 1; y < m; ++y) off += M[x][y] * M[x][y];
    }
    if (off <= 1e-32 * dia || off == 0.0) break;
    for (int p = 0; p < m; ++p) {
      for (int q = p + 1; q < m; ++q) {
        const double apq = M[p][q];
        if (apq == 0.0) continue;
        const double theta = (M[q][q] - M[p][p]) / (2.0 * apq);
        const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(tt * tt + 1.0);
        const double s = tt * c;
        for (int k = 0; k < m; ++k) {
          const double mkp = M[k][p], mkq = M[k][q];
          M[k][p] = c * mkp - s * mkq;
          M[k][q] = s * mkp + c * mkq;
        }
        for (int k = 0; k < m; ++k) {
          const double mpk = M[p][k], mqk = M[q][k];
          M[p][k] = c * mpk - s * mqk;
          M[q][k] = s * mpk + c * mqk;
        }
        for (int k = 0; k < m; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
    }
  }
  double lmax = 0.0;
  for (int x = 0; x < m; ++x) lmax = fmax(lmax, M[x][x]);
  const double tol = rank_tol(l, m) * lmax;
  int rank = 0;
  double W[kMaxM][kMaxM];
  for (int x = 0; x < m; ++x)
    for (int y = 0; y < m; ++y) W[x][y] = 0.0;
  for (int j = 0; j < m; ++j) {
    const double lj = M[j][j];
    if (!(lj > tol) || !(lmax > 0.0)) continue;
    ++rank;
    for (int x = 0; x < m; ++x)
      for (int y = 0; y < m; ++y) W[x][y] += V[x][j] * V[y][j] / lj;
  }
  if (rank < m) count_rank_deficient(a, i);
  double coef[kMaxM];
  for (int x = 0; x < m; ++x) {
    double s = 0.0;
    for (int y = 0; y < m; ++y) s += W[x][y] * (a.B[(long)i * m + y] - u[y]);
    coef[x] = s;
  }
  for (int s = p0; s < p1; ++s) {
    const int c = a.pci[s];
    double dl = 0.0;
    for (int x = 0; x < m; ++x) dl += a.bc[(long)c * m + x] * coef[x];
    a.p0p[s] = lookup_p0(a.qci, a.qv, q0, q1, c) + dl;
  }
  const int mp = m * (m + 1) / 2;
  for (int x = 0; x < m; ++x)
    for (int y = x; y < m; ++y) a.wpk[(long)i * mp + packed_index(x, y, m)] = W[x][y];
}

// Inverse of each node's diagonal block A(rows, rows) (a pivot at or below
// the threshold marks the problem as having a bad diagonal).  One thread per
// node; the node set-up kernel does the same when it runs.
__global__ __launch_bounds__(kBlock) void k_block_inverse(SetupArgs a) {
  const int node = blockIdx.x * kBlock + threadIdx.x;
  const int bs = a.bs;
  if (node >= a.n / bs) return;
  const int r0 = node * bs;
  double M[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) M[r][c] = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (r >= bs) break;
    const int e0 = a.arp[r0 + r], e1 = a.arp[r0 + r + 1];
    for (int e = e0; e < e1; ++e) {
      const int c = a.aci[e] - r0;
      const double v = a.av[e];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (c == k && k < bs) M[r][k] = v;
    }
  }
  double Inv[4][4];
  const bool ok = gj_inverse<4>(M, Inv, bs);
  if (!ok) a.st->done = 4;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (r < bs && c < bs) a.binv[(long)node * bs * bs + r * bs + c] = ok ? Inv[r][c] : 0.0;
}

__global__ __launch_bounds__(kBlock) void k_to_float(const double* __restrict__ x,
                                                    float* __restrict__ y, int n) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

__global__ void k_zero_ints(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_state_init(DevState* st, double tau) {
  if (threadIdx.x != 0) return;
  st->gamma = st->gamma_old = st->gamma1 = 0.0;
  st->delta = st->alpha = st->beta = st->dE1 = 0.0;
  st->energy = st->aux = 0.0;
  st->tau = tau;
  st->k = 0;
  st->iterations = 0;
  st->done = 0;
  st->rank_def = 0;

}

// ------------------------------------------------------------- launchers --

void launch_diag_has(const int* arp, const int* aci, int n, int* flags, hipStream_t s) {
  if (n > 0) k_diag_has<<<cdiv(n, kBlock), kBlock, 0, s>>>(arp, aci, n, flags);
}

void launch_check_nodes(const int* arp, const int* aci, const int* prp, const int* pci,
                        int nnodes, int bs, int what, int* flags, hipStream_t s) {
  if (nnodes > 0)
    k_check_nodes<<<cdiv(nnodes, kBlock / kWave), kBlock, 0, s>>>(arp, aci, prp, pci, nnodes, bs,
                                                                  what, flags);
}

void launch_state_init(DevState* st, double tau, hipStream_t s) {
  k_state_init<<<1, kWave, 0, s>>>(st, tau);
}

template <int G, int L>
static void setup_go(const SetupArgs& a, int grid_cap, hipStream_t s) {
  constexpr int ROWS = kBlock / G;
  int ntiles = cdiv(a.n, ROWS);
  int g = ntiles < grid_cap ? ntiles : grid_cap;
  g = ((g + kNumXcd - 1) / kNumXcd) * kNumXcd;
  if (a.m == 1)
    k_setup<G, L, true><<<g, kBlock, 0, s>>>(a);
  else
    k_setup<G, L, false><<<g, kBlock, 0, s>>>(a);
}

template <int BS, int M, int L>
static void setup_node_l(const SetupArgs& a, int g, hipStream_t s) {
  k_setup_node_sums<BS, M, L><<<g, kBlock, 0, s>>>(a);
  k_setup_node_solve<BS, M><<<cdiv(a.n / BS, kBlock), kBlock, 0, s>>>(a);
  k_setup_node_apply<BS, M, L><<<g, kBlock, 0, s>>>(a);
}

template <int BS, int M>
static bool setup_node_go(const SetupArgs& a, int lmax, int grid_cap, hipStream_t s) {
  int ntiles = cdiv(a.n / BS, kBlock / kWave);
  int g = ntiles < grid_cap ? ntiles : grid_cap;
  g = ((g + kNumXcd - 1) / kNumXcd) * kNumXcd;
  if (lmax <= 64) setup_node_l<BS, M, 1>(a, g, s);
  else if (lmax <= 128) setup_node_l<BS, M, 2>(a, g, s);
  else if (lmax <= 192) setup_node_l<BS, M, 3>(a, g, s);
  else if (lmax <= 256) setup_node_l<BS, M, 4>(a, g, s);
  else return false;
  return true;
}

int setup_node_record(int bs, int m) {
  if (bs == 3 && m == 6) return NodeRec<3, 6>::SIZE;
  if (bs == 3 && m == 3) return NodeRec<3, 3>::SIZE;
  if (bs == 2 && m == 3) return NodeRec<2, 3>::SIZE;
  return 0;
}

// Node set-up for nodes of 2 or 3 rows with m = 3 or 6 (B_c 16-byte aligned
// for m = 6) when the caller gave the node records; false: use the row-wise
// kernel.
static bool setup_node(const SetupArgs& a, int lmax, int grid_cap, hipStream_t s) {
  if (a.nbs < 2 || a.n % a.nbs || !a.nrec) return false;
  const bool al16 = ((unsigned long long)a.bc & 15) == 0;
  if (a.nbs == 3 && a.m == 6 && al16) return setup_node_go<3, 6>(a, lmax, grid_cap, s);
  if (a.nbs == 3 && a.m == 3) return setup_node_go<3, 3>(a, lmax, grid_cap, s);
  if (a.nbs == 2 && a.m == 3) return setup_node_go<2, 3>(a, lmax, grid_cap, s);
  return false;
}

void launch_setup(const SetupArgs& a, int lmax, int grid_cap, hipStream_t s) {
  if (a.n <= 0) return;
  k_zero_ints<<<1, kWave, 0, s>>>(a.fb_count, 1);
  const bool node = setup_node(a, lmax, grid_cap, s);
  // short rows on average but a few long ones: four lanes per row with up to
  // four slots each, instead of lanes sized for the longest row
  const bool narrow = a.lavg > 0 && a.lavg <= 4 && lmax > 4 && lmax <= 16;
  if (node) {
  } else if (narrow && lmax <= 8) setup_go<4, 2>(a, grid_cap, s);
  else if (narrow) setup_go<4, 4>(a, grid_cap, s);
  else if (lmax <= 2) setup_go<2, 1>(a, grid_cap, s);
  else if (lmax <= 4) setup_go<4, 1>(a, grid_cap, s);
  else if (lmax <= 8) setup_go<8, 1>(a, grid_cap, s);
  else if (lmax <= 16) setup_go<16, 1>(a, grid_cap, s);
  else if (lmax <= 32) setup_go<32, 1>(a, grid_cap, s);
  else if (lmax <= 64) setup_go<64, 1>(a, grid_cap, s);
  else if (lmax <= 128) setup_go<64, 2>(a, grid_cap, s);
  else if (lmax <= 192) setup_go<64, 3>(a, grid_cap, s);
  else setup_go<64, 4>(a, grid_cap, s);
  if (a.m > 1) k_setup_fallback<<<cdiv(a.n, kBlock), kBlock, 0, s>>>(a);
  if (a.binv && a.bs > 0 && !(node && a.bs == a.nbs))
    k_block_inverse<<<cdiv(a.n / a.bs, kBlock), kBlock, 0, s>>>(a);
  if (a.avf) k_to_float<<<cdiv(a.nnzA, kBlock), kBlock, 0, s>>>(a.av, a.avf, a.nnzA);
}

}  // namespace emin
