// Tentative prolongation set-up (Alg. 1, Sec. 3.2) for a C/F splitting, on
// the device.  One wave per FINE node i:
//   for l = 1 .. l_max: add the nodes at distance l from i in the strength
//   graph S (breadth-first rings, an LDS hash set of visited nodes); the
//   COARSE ones, ordered by coarse index, are the candidates N_i; max vol
//   picks (up to) m of them on the rows of V(N_i, :); w solves B w = v_i
//   for B = V(J, :)^T; the row is kept at the first l where v_i - B w
//   vanishes (relative 2-norm at most 1e-10).
// COARSE rows are the identity (P = [W; I]).
//
// Max vol: Gaussian elimination with partial (row) pivoting over the
// candidate rows (a column whose remaining entries are all below 1e-12 of
// the largest entry gives no row); with m rows, the coefficients C of every
// row in the basis of the selected ones (M_sel^T C^T = M^T by Gaussian
// elimination with partial pivoting) and, while some |C| exceeds 1.05, the
// first such maximum's row replaces the selected row of its column
// (Goreinov et al.); ties go to the first row in order.  The fit: the
// square system by the same elimination, a smaller set through its normal
// equations.  The selection is an integer decision made from floating-point
// comparisons, so this file keeps every product and sum separately rounded
// (no contraction into fused multiply-adds) and every reduction in a fixed
// sequential order.
#include "common.hpp"
#include "launch.hpp"

#pragma clang fp contract(off)

namespace emin {

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

constexpr int kPtHash = 2048;   // visited-node hash slots
constexpr int kPtNodes = 1024;  // nodes within distance l_max of a row
constexpr int kPtCand = 128;    // COARSE candidates (two per lane)
constexpr int kPtT = kPtCand / kWave;
constexpr double kMaxvolTol = 1.05;
constexpr int kMaxvolSwaps = 64;
constexpr double kPivotTol = 1e-12;
constexpr double kFitTol = 1e-10;

struct PtArgs {
  const int* srp; const int* sci;  // S
  const int* cf;                    // coarse index, -1 FINE
  const double* V; int n, m, lmax;
  int* cnt; int* cols; double* vals; int* level;  // per row: up to m (col, val)
  int* flags;                       // bit 0: a neighbourhood exceeded the LDS limits
};

// Gaussian elimination with partial pivoting on the s x s leading block of
// a (first row on ties), applied to one right-hand side; false on a zero
// pivot.  Sequential, uniform across the wave.
template <int M>
__device__ __forceinline__ bool ge_solve1(double (&a)[M][M], double (&b)[M], int s) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    if (j < s && ok) {
      int p = j;
      double best = fabs(a[j][j]);
#pragma unroll
      for (int r = j + 1; r < M; ++r)
        if (r < s && fabs(a[r][j]) > best) { p = r; best = fabs(a[r][j]); }
      double pv = 0.0;
#pragma unroll
      for (int r = 0; r < M; ++r)
        if (r == p) pv = a[r][j];
      ok = pv != 0.0;
#pragma unroll
      for (int r = j + 1; r < M; ++r) {  // swap rows j and p
        if (r != p) continue;
#pragma unroll
        for (int c = 0; c < M; ++c) {
          const double t = a[j][c]; a[j][c] = a[r][c]; a[r][c] = t;
        }
        const double t = b[j]; b[j] = b[r]; b[r] = t;
      }
      if (ok) {
#pragma unroll
        for (int r = j + 1; r < M; ++r) {
          if (r >= s) continue;
          const double f = a[r][j] / a[j][j];
#pragma unroll
          for (int c = j; c < M; ++c)
            if (c < s) a[r][c] = a[r][c] - f * a[j][c];
          b[r] = b[r] - f * b[j];
        }
      }
    }
  }
  if (!ok) return false;
#pragma unroll
  for (int j = M - 1; j >= 0; --j) {
    if (j >= s) continue;
    double v = b[j];
#pragma unroll
    for (int k = j + 1; k < M; ++k)
      if (k < s) v = v - a[j][k] * b[k];
    b[j] = v / a[j][j];
  }
  return true;
}

// wave argmax of (value, first index): the lane holding the smallest index
// among the largest values wins
__device__ __forceinline__ void wave_argmax(double& v, int& idx, int& aux) {
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) {
    const double ov = __shfl_xor(v, d, kWave);
    const int oi = __shfl_xor(idx, d, kWave);
    const int oa = __shfl_xor(aux, d, kWave);
    const bool take = ov > v || (ov == v && (oi < idx || (oi == idx && oa < aux)));
    if (take) { v = ov; idx = oi; aux = oa; }
  }
}

template <int M>
__global__ __launch_bounds__(kWave) void k_ptent_rows(PtArgs a) {
  __shared__ int tab[kPtHash];
  __shared__ int nodes[kPtNodes];
  __shared__ int cand[kPtCand];
  __shared__ int sorted_c[kPtCand];
  __shared__ int nvis, ncand, over;
  const int lane = threadIdx.x;
  for (int i = blockIdx.x; i < a.n; i += gridDim.x) {
    const int ci = a.cf[i];
    if (ci >= 0) {  // COARSE: the identity row
      if (lane == 0) {
        a.cnt[i] = 1;
        a.cols[(long)i * M] = ci;
        a.vals[(long)i * M] = 1.0;
        if (a.level) a.level[i] = 0;
      }
      continue;
    }
    double v[M];
#pragma unroll
    for (int x = 0; x < M; ++x) v[x] = a.V[(long)i * M + x];
    for (int h = lane; h < kPtHash; h += kWave) tab[h] = -1;
    if (lane == 0) {
      nodes[0] = i;
      nvis = 1;
      ncand = 0;
      over = 0;
      tab[((unsigned)i * 2654435761u) & (kPtHash - 1)] = i;
    }
    __syncthreads();
    int lo = 0, hi = 1, found = -1, nsel = 0;
    int sel[M];
    double wv[M];
    for (int l = 1; l <= a.lmax && found < 0; ++l) {
      // ring l: unvisited neighbours of ring l - 1
      for (int f = lo; f < hi; ++f) {
        const int u = nodes[f];
        for (int e = a.srp[u] + lane; e < a.srp[u + 1]; e += kWave) {
          const int w = a.sci[e];
          unsigned h = ((unsigned)w * 2654435761u) & (kPtHash - 1);
          // the table holds twice the node limit, so a free slot exists while
          // the limit holds; the probe count is bounded regardless
          for (int probe = 0; probe < kPtHash; ++probe) {
            const int old = atomicCAS(&tab[h], -1, w);
            if (old == -1) {
              const int pos = atomicAdd(&nvis, 1);
              if (pos < kPtNodes) nodes[pos] = w; else over = 1;
              if (a.cf[w] >= 0) {
                const int q = atomicAdd(&ncand, 1);
                if (q < kPtCand) cand[q] = w; else over = 1;
              }
              break;
            }
            if (old == w) break;
            h = (h + 1) & (kPtHash - 1);
            if (probe == kPtHash - 1) over = 1;
          }
        }
      }
      __syncthreads();
      if (over) break;
      lo = hi;
      hi = nvis;
      const int K = ncand;
      if (K == 0) continue;
      // candidates in coarse-index order (rank sort: coarse indices differ)
      for (int q = lane; q < K; q += kWave) {
        const int cq = a.cf[cand[q]];
        int rank = 0;
        for (int y = 0; y < K; ++y) rank += a.cf[cand[y]] < cq ? 1 : 0;
        sorted_c[rank] = cand[q];
      }
      __syncthreads();
      // rows of M = V(N_i, :), row q = lane + 64 t held by its lane
      double Mr[kPtT][M], U[kPtT][M];
      bool live[kPtT];
      double amax = 0.0;
#pragma unroll
      for (int t = 0; t < kPtT; ++t) {
        const int q = lane + kWave * t;
        live[t] = q < K;
#pragma unroll
        for (int x = 0; x < M; ++x) {
          Mr[t][x] = live[t] ? a.V[(long)sorted_c[q] * M + x] : 0.0;
          U[t][x] = Mr[t][x];
          amax = fmax(amax, fabs(Mr[t][x]));
        }
      }
#pragma unroll
      for (int d = kWave / 2; d >= 1; d >>= 1) amax = fmax(amax, __shfl_xor(amax, d, kWave));
      const double floor_v = kPivotTol * amax;
      // elimination with partial pivoting: rows in order, first on ties
      bool avail[kPtT];
#pragma unroll
      for (int t = 0; t < kPtT; ++t) avail[t] = live[t];
      nsel = 0;
#pragma unroll
      for (int j = 0; j < M; ++j) {
        double bv = floor_v;
        int bq = 0x7fffffff, dummy = 0;
#pragma unroll
        for (int t = 0; t < kPtT; ++t)
          if (avail[t] && fabs(U[t][j]) > bv) { bv = fabs(U[t][j]); bq = lane + kWave * t; }
        if (bq == 0x7fffffff) bv = -1.0;  // no candidate on this lane
        wave_argmax(bv, bq, dummy);
        if (bv < 0.0) continue;  // no pivot: the column adds no direction
        const int bl = bq % kWave, bt = bq / kWave;
        double prow[M];
#pragma unroll
        for (int x = 0; x < M; ++x) {
          double mine = 0.0;
#pragma unroll
          for (int t = 0; t < kPtT; ++t)
            if (t == bt) mine = U[t][x];
          prow[x] = __shfl(mine, bl, kWave);
        }
#pragma unroll
        for (int s2 = 0; s2 < M; ++s2)
          if (s2 == nsel) sel[s2] = bq;
        ++nsel;
#pragma unroll
        for (int t = 0; t < kPtT; ++t) {
          if (lane + kWave * t == bq) avail[t] = false;
          if (!avail[t]) continue;
          const double f = U[t][j] / prow[j];
#pragma unroll
          for (int c = 0; c < M; ++c)
            if (c >= j) U[t][c] = U[t][c] - f * prow[c];
        }
      }
      if (nsel == M) {
        for (int it = 0; it < kMaxvolSwaps; ++it) {
          // M_sel^T (uniform): column c is the selected row sel[c]
          double Ms[M][M];
#pragma unroll
          for (int c = 0; c < M; ++c) {
            const int sq = sel[c];
            const int sl = sq % kWave, st = sq / kWave;
#pragma unroll
            for (int x = 0; x < M; ++x) {
              double mine = 0.0;
#pragma unroll
              for (int t = 0; t < kPtT; ++t)
                if (t == st) mine = Mr[t][x];
              Ms[x][c] = __shfl(mine, sl, kWave);
            }
          }
          // coefficients of the lane's rows; the largest |C| over rows not
          // selected, first (row, column) in order on ties
          double bv = kMaxvolTol;
          int bq = 0x7fffffff, bc = 0x7fffffff;
          bool ok = true;
#pragma unroll
          for (int t = 0; t < kPtT; ++t) {
            const int q = lane + kWave * t;
            bool chosen = false;
#pragma unroll
            for (int c = 0; c < M; ++c) chosen = chosen || sel[c] == q;
            double A2[M][M], rhs[M];
#pragma unroll
            for (int x = 0; x < M; ++x) {
              rhs[x] = Mr[t][x];
#pragma unroll
              for (int c = 0; c < M; ++c) A2[x][c] = Ms[x][c];
            }
            ok = ge_solve1<M>(A2, rhs, M) && ok;
            if (!live[t] || chosen) continue;
#pragma unroll
            for (int c = 0; c < M; ++c)
              if (fabs(rhs[c]) > bv) { bv = fabs(rhs[c]); bq = q; bc = c; }
          }
          if (bq == 0x7fffffff) bv = -1.0;
          wave_argmax(bv, bq, bc);
          if (!ok || bv < 0.0) break;
#pragma unroll
          for (int c = 0; c < M; ++c)
            if (c == bc) sel[c] = bq;
        }
      }
      // the selected rows in candidate order
#pragma unroll
      for (int x = 1; x < M; ++x)
#pragma unroll
        for (int y = M - 1; y >= x; --y)
          if (y < nsel && sel[y - 1] > sel[y]) {
            const int t = sel[y - 1]; sel[y - 1] = sel[y]; sel[y] = t;
          }
      // B = V(J, :)^T (M x nsel): column c is candidate row sel[c]
      double B[M][M];
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const int sq = c < nsel ? sel[c] : 0;
        const int sl = sq % kWave, st = sq / kWave;
#pragma unroll
        for (int x = 0; x < M; ++x) {
          double mine = 0.0;
#pragma unroll
          for (int t = 0; t < kPtT; ++t)
            if (t == st) mine = Mr[t][x];
          B[x][c] = c < nsel ? __shfl(mine, sl, kWave) : 0.0;
        }
      }
      double w[M];
      bool solved;
      if (nsel == M) {
        double A2[M][M];
#pragma unroll
        for (int x = 0; x < M; ++x) {
          w[x] = v[x];
#pragma unroll
          for (int c = 0; c < M; ++c) A2[x][c] = B[x][c];
        }
        solved = ge_solve1<M>(A2, w, M);
      } else {  // normal equations B^T B w = B^T v, sums in order
        double A2[M][M];
#pragma unroll
        for (int p = 0; p < M; ++p) {
#pragma unroll
          for (int q = 0; q < M; ++q) {
            double s = 0.0;
#pragma unroll
            for (int x = 0; x < M; ++x) s = s + B[x][p] * B[x][q];
            A2[p][q] = s;
          }
          double s = 0.0;
#pragma unroll
          for (int x = 0; x < M; ++x) s = s + B[x][p] * v[x];
          w[p] = s;
        }
        solved = ge_solve1<M>(A2, w, nsel);
      }
      if (!solved) continue;
      double nv = 0.0, nr = 0.0;
#pragma unroll
      for (int x = 0; x < M; ++x) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c)
          if (c < nsel) s = s + B[x][c] * w[c];
        const double r = v[x] - s;
        nv = nv + v[x] * v[x];
        nr = nr + r * r;
      }
      nv = sqrt(nv);
      nr = sqrt(nr);
      const double rel = nv > 0.0 ? nr / nv : nr;
      if (rel <= kFitTol) {
        found = l;
#pragma unroll
        for (int c = 0; c < M; ++c) {
          wv[c] = w[c];
          if (c < nsel) sel[c] = a.cf[sorted_c[sel[c]]];
        }
      }
    }
    if (lane == 0) {
      if (over) atomicOr(a.flags, 1);
      const int cnt = found > 0 ? nsel : 0;
      a.cnt[i] = cnt;
#pragma unroll
      for (int c = 0; c < M; ++c)
        if (c < cnt) {
          a.cols[(long)i * M + c] = sel[c];
          a.vals[(long)i * M + c] = wv[c];
        }
      if (a.level) a.level[i] = found > 0 ? found : -1;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_ptent_compact(const int* __restrict__ cnt,
                                                         const int* __restrict__ cols,
                                                         const double* __restrict__ vals,
                                                         const int* __restrict__ rp, int n, int m,
                                                         int* __restrict__ colind,
                                                         double* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < cnt[i]; ++c) {
    colind[rp[i] + c] = cols[(long)i * m + c];
    out[rp[i] + c] = vals[(long)i * m + c];
  }
}

// ------------------------------------------------------------- C/F form --

// cf: every value in [-1, nc), every coarse index held by exactly one node
__global__ __launch_bounds__(kBlock) void k_cf_range(const int* __restrict__ cf, int n, int nc,
                                                    int* __restrict__ seen, int* flags) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int c = cf[i];
  if (c < -1 || c >= nc) atomicOr(flags, 1 << kFlagCF);
  else if (c >= 0) atomicAdd(&seen[c], 1);
}

__global__ __launch_bounds__(kBlock) void k_cf_unique(const int* __restrict__ seen, int nc,
                                                     int* flags) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c < nc && seen[c] != 1) atomicOr(flags, 1 << kFlagCF);
}

// P0's COARSE rows must be the identity: one entry, at cf[i], equal to 1
__global__ __launch_bounds__(kBlock) void k_cf_p0(const int* __restrict__ qrp,
                                                 const int* __restrict__ qci,
                                                 const double* __restrict__ qv,
                                                 const int* __restrict__ cf, int n, int* flags) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n || cf[i] < 0) return;
  const int q = qrp[i];
  if (qrp[i + 1] - q != 1 || qci[q] != cf[i] || qv[q] != 1.0) atomicOr(flags, 1 << kFlagCFP0);
}

// pattern of P = [W; I]: COARSE rows keep only their identity column
__global__ __launch_bounds__(kBlock) void k_cf_count(const int* __restrict__ prp,
                                                    const int* __restrict__ cf, int n,
                                                    int* __restrict__ cnt) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) cnt[i] = cf[i] >= 0 ? 1 : prp[i + 1] - prp[i];
}

__global__ __launch_bounds__(kBlock) void k_cf_fill(const int* __restrict__ prp,
                                                   const int* __restrict__ pci,
                                                   const int* __restrict__ cf, int n,
                                                   const int* __restrict__ rp2,
                                                   int* __restrict__ ci2) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  if (cf[i] >= 0) {
    ci2[rp2[i]] = cf[i];
    return;
  }
  for (int e = prp[i]; e < prp[i + 1]; ++e) ci2[rp2[i] + e - prp[i]] = pci[e];
}

// a given pattern: COARSE rows must be exactly their identity column
__global__ __launch_bounds__(kBlock) void k_cf_pattern_check(const int* __restrict__ prp,
                                                            const int* __restrict__ pci,
                                                            const int* __restrict__ cf, int n,
                                                            int* flags) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n || cf[i] < 0) return;
  if (prp[i + 1] - prp[i] != 1 || pci[prp[i]] != cf[i]) atomicOr(flags, 1 << kFlagCFPattern);
}

// COARSE rows of the assembled P: their identity entry, exactly (with m > 1
// their projector is formed from a rank-one Gram pseudo-inverse, so the
// iteration leaves them at 1 only to rounding)
__global__ __launch_bounds__(kBlock) void k_cf_identity(const int* __restrict__ prp,
                                                       const int* __restrict__ cf, int n,
                                                       double* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n && cf[i] >= 0) out[prp[i]] = 1.0;
}

void launch_cf_identity(const int* prp, const int* cf, int n, double* out, hipStream_t s) {
  if (n > 0) k_cf_identity<<<cdiv(n, kBlock), kBlock, 0, s>>>(prp, cf, n, out);
}

void launch_cf_check(const int* cf, int n, int nc, int* seen, const int* qrp, const int* qci,
                     const double* qv, int* flags, hipStream_t s) {
  if (n <= 0) return;
  k_cf_range<<<cdiv(n, kBlock), kBlock, 0, s>>>(cf, n, nc, seen, flags);
  if (nc > 0) k_cf_unique<<<cdiv(nc, kBlock), kBlock, 0, s>>>(seen, nc, flags);
  if (qrp) k_cf_p0<<<cdiv(n, kBlock), kBlock, 0, s>>>(qrp, qci, qv, cf, n, flags);
}

void launch_cf_count(const int* prp, const int* cf, int n, int* cnt, hipStream_t s) {
  if (n > 0) k_cf_count<<<cdiv(n, kBlock), kBlock, 0, s>>>(prp, cf, n, cnt);
}

void launch_cf_fill(const int* prp, const int* pci, const int* cf, int n, const int* rp2,
                    int* ci2, hipStream_t s) {
  if (n > 0) k_cf_fill<<<cdiv(n, kBlock), kBlock, 0, s>>>(prp, pci, cf, n, rp2, ci2);
}

void launch_cf_pattern_check(const int* prp, const int* pci, const int* cf, int n, int* flags,
                             hipStream_t s) {
  if (n > 0) k_cf_pattern_check<<<cdiv(n, kBlock), kBlock, 0, s>>>(prp, pci, cf, n, flags);
}

int launch_ptent_rows(const int* srp, const int* sci, const int* cf, const double* V, int n,
                      int m, int lmax, int* cnt, int* cols, double* vals, int* level, int* flags,
                      hipStream_t s) {
  if (n <= 0) return 0;
  PtArgs a{srp, sci, cf, V, n, m, lmax, cnt, cols, vals, level, flags};
  const int grid = n < 65536 ? n : 65536;
  switch (m) {
    case 1: k_ptent_rows<1><<<grid, kWave, 0, s>>>(a); break;
    case 2: k_ptent_rows<2><<<grid, kWave, 0, s>>>(a); break;
    case 3: k_ptent_rows<3><<<grid, kWave, 0, s>>>(a); break;
    case 4: k_ptent_rows<4><<<grid, kWave, 0, s>>>(a); break;
    case 5: k_ptent_rows<5><<<grid, kWave, 0, s>>>(a); break;
    case 6: k_ptent_rows<6><<<grid, kWave, 0, s>>>(a); break;
    case 7: k_ptent_rows<7><<<grid, kWave, 0, s>>>(a); break;
    case 8: k_ptent_rows<8><<<grid, kWave, 0, s>>>(a); break;
    default: return -1;
  }
  return 0;
}

void launch_ptent_compact(const int* cnt, const int* cols, const double* vals, const int* rp,
                          int n, int m, int* colind, double* out, hipStream_t s) {
  if (n > 0)
    k_ptent_compact<<<cdiv(n, kBlock), kBlock, 0, s>>>(cnt, cols, vals, rp, n, m, colind, out);
}

}  // namespace emin
