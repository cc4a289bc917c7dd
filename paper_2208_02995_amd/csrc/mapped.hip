// Masked product with the intersection structure precomputed (the pattern of
// P is fixed for the whole iteration, Sec. 4, so its adjacency with A's
// pattern is worked out once, in the symbolic phase).
//
// For row i with neighbours k_0..k_{a-1} (A's row) and pattern row J_i of
// length l, the byte map holds, for every (neighbour n, slot s), the position
// of J_i[s] inside J_{k_n}, or 0xFF when J_{k_n} lacks it:
//     amap[mrp[i] + n * l + s]
// and aoff[e] = rowptr of the neighbour's pattern row.  Then
//     Y_hat(i, s) = sum_n A(i, k_n) * Y[aoff[e_n] + amap[..n..s]]
// with no column comparisons at all: one predicated gather and one FMA per
// (neighbour, slot).  A group of G lanes owns row i, lane g the slots
// g, g + G, ... (L of them); A's entries are read once per group (same
// address across the group), the map bytes of one neighbour step are
// contiguous across the group.
#include "common.hpp"
#include "launch.hpp"
#include "project.hpp"

namespace emin {

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

__global__ __launch_bounds__(kBlock) void k_map_count(const int* __restrict__ arp,
                                                     const int* __restrict__ prp, int n,
                                                     int* __restrict__ cnt) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) cnt[i] = (arp[i + 1] - arp[i]) * (prp[i + 1] - prp[i]);
}

__global__ __launch_bounds__(kBlock) void k_map_fill(const int* __restrict__ arp,
                                                    const int* __restrict__ aci,
                                                    const int* __restrict__ prp,
                                                    const int* __restrict__ pci,
                                                    const int* __restrict__ mrp, int n,
                                                    unsigned char* __restrict__ amap,
                                                    int* __restrict__ aoff) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int p0 = prp[i], l = prp[i + 1] - p0;
  const int e0 = arp[i], e1 = arp[i + 1];
  const int base = mrp[i];
  for (int e = e0; e < e1; ++e) {
    const int k = aci[e];
    const int q0 = prp[k], q1 = prp[k + 1];
    aoff[e] = q0;
    const int nn = e - e0;
    for (int s = 0; s < l; ++s) {
      const int c = pci[p0 + s];
      int lo = q0, hi = q1 - 1, pos = 0xFF;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = pci[mid];
        if (v == c) { pos = mid - q0; break; }
        if (v < c) lo = mid + 1; else hi = mid - 1;
      }
      amap[base + nn * l + s] = (unsigned char)pos;
    }
  }
}

template <class TA, class TI, class TO, int G, int L, int MODE, bool M1, bool SEG>
__global__ __launch_bounds__(kBlock) void k1_mapped(K1Args a) {
  using TAcc = TI;
  constexpr int ROWS = kBlock / G;
  constexpr int U = 4;  // neighbours per step (independent gathers in flight)
  if (!SEG && (MODE == kModeIter || MODE == kModeInit) && a.st->done) return;
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  const TA* __restrict__ av = (const TA*)a.av;
  const TI* __restrict__ y = (const TI*)a.y;
  const int* __restrict__ pci = a.pci;
  const double* __restrict__ bc = a.bc;
  const unsigned char* __restrict__ amap = a.amap;
  const int* __restrict__ aoff = a.aoff;
  TO* __restrict__ out = (TO*)a.out;
  const int mp = a.m * (a.m + 1) / 2;
  double dot = 0.0;
  const int ntiles = (a.n + ROWS - 1) / ROWS;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int li = w.t * ROWS + grp;
    const bool valid = li < a.n;
    const int i = (valid && a.rows) ? a.rows[li] : li;
    int p0 = 0, l = 0, e0 = 0, na = 0, mb = 0;
    if (valid) {
      p0 = a.prp[i];
      l = a.prp[i + 1] - p0;
      e0 = a.arp[i];
      na = a.arp[i + 1] - e0;
      mb = a.mrp[i];
    }
    int oc[L];
    double yo[L], g[L];
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int s = lane + G * t;
      const int is = (s < l) ? p0 + s : 0;
      oc[t] = pci[is];
      yo[t] = (double)y[is];
      if (s >= l) oc[t] = -1;
      if (M1) g[t] = (oc[t] >= 0) ? bc[oc[t]] : 0.0;
    }
    TAcc acc[L];
#pragma unroll
    for (int t = 0; t < L; ++t) acc[t] = TAcc(0);
    for (int n0 = 0; n0 < na; n0 += U) {
      int off[U];
      TAcc va[U];
      int q[U][L];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int nn = n0 + u;
        const bool hn = nn < na;
        const int e = e0 + (hn ? nn : 0);
        off[u] = aoff[e];
        va[u] = hn ? (TAcc)av[e] : TAcc(0);
#pragma unroll
        for (int t = 0; t < L; ++t) {
          const int s = lane + G * t;
          const bool ok = hn && s < l;
          const int qq = amap[ok ? mb + nn * l + s : 0];
          q[u][t] = ok ? qq : 0xFF;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int t = 0; t < L; ++t) {
          const bool hit = q[u][t] != 0xFF;
          const TAcc yv = (TAcc)y[hit ? off[u] + q[u][t] : 0];
          acc[t] = fma(hit ? va[u] : TAcc(0), yv, acc[t]);
        }
      }
    }
    double v[L];
#pragma unroll
    for (int t = 0; t < L; ++t) v[t] = (double)acc[t];
    if (MODE != kModeEnergy && MODE != kModeRaw) {
      if (M1) {
        double gx = 0.0, gg = 0.0;
#pragma unroll
        for (int t = 0; t < L; ++t) {
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
      } else {
        project_row<G, L, false>(v, oc, bc, valid ? a.wpk + (long)i * mp : nullptr, a.m, valid);
      }
    }
    double rdot = 0.0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
      if (oc[t] < 0) continue;
      const int idx = p0 + lane + G * t;
      if (MODE == kModeIter) {
        const TO o = (TO)v[t];
        out[idx] = o;
        rdot += yo[t] * (double)o;
      } else if (MODE == kModeInit) {
        out[idx] = (TO)(-v[t]);
      } else if (MODE == kModePlain || MODE == kModeRaw) {
        out[idx] = (TO)v[t];
      } else {
        rdot += yo[t] * v[t];
      }
    }
    if (SEG && (MODE == kModeIter || MODE == kModeEnergy)) {
      rdot = group_sum<G>(rdot);
      if (lane == 0 && valid) a.rowdot[i] = rdot;
    } else {
      dot += rdot;
    }
  }
  if (!SEG && (MODE == kModeIter || MODE == kModeEnergy)) store_partial(dot, a.part_out);
}

// ------------------------------------------------------------- launchers --

void launch_map_count(const int* arp, const int* prp, int n, int* cnt, hipStream_t s) {
  if (n > 0) k_map_count<<<cdiv(n, kBlock), kBlock, 0, s>>>(arp, prp, n, cnt);
}

void launch_map_fill(const int* arp, const int* aci, const int* prp, const int* pci,
                     const int* mrp, int n, unsigned char* amap, int* aoff, hipStream_t s) {
  if (n > 0)
    k_map_fill<<<cdiv(n, kBlock), kBlock, 0, s>>>(arp, aci, prp, pci, mrp, n, amap, aoff);
}

template <class TA, class TI, class TO, int MODE, bool M1>
static int mapped_go(const K1Shape& sh, const K1Args& a, int grid, hipStream_t s) {
#define EMIN_K1M(GG, LL)                                                           \
  if (sh.G == GG && sh.L == LL) {                                                  \
    if (a.seg)                                                                     \
      k1_mapped<TA, TI, TO, GG, LL, MODE, M1, true><<<grid, kBlock, 0, s>>>(a);    \
    else                                                                           \
      k1_mapped<TA, TI, TO, GG, LL, MODE, M1, false><<<grid, kBlock, 0, s>>>(a);   \
    return 0;                                                                      \
  }
  EMIN_K1M(1, 1) EMIN_K1M(2, 1) EMIN_K1M(4, 1) EMIN_K1M(8, 1) EMIN_K1M(16, 1)
  EMIN_K1M(32, 1) EMIN_K1M(64, 1) EMIN_K1M(4, 2) EMIN_K1M(8, 2) EMIN_K1M(16, 2)
  EMIN_K1M(4, 4)
#undef EMIN_K1M
  return -1;
}

template <class TA, class TI, class TO, int MODE>
int k1_mapped_go(const K1Shape& sh, const K1Args& a, int grid, hipStream_t s) {
  return a.m == 1 ? mapped_go<TA, TI, TO, MODE, true>(sh, a, grid, s)
                  : mapped_go<TA, TI, TO, MODE, false>(sh, a, grid, s);
}

int launch_k1_mapped(int mode, int precision, const K1Shape& sh, const K1Args& a, int grid,
                     hipStream_t s) {
  if (precision == 0) {
    switch (mode) {
      case kModeIter: return k1_mapped_go<double, double, double, kModeIter>(sh, a, grid, s);
      case kModeInit: return k1_mapped_go<double, double, double, kModeInit>(sh, a, grid, s);
      case kModeEnergy: return k1_mapped_go<double, double, double, kModeEnergy>(sh, a, grid, s);
      case kModePlain: return k1_mapped_go<double, double, double, kModePlain>(sh, a, grid, s);
      case kModeRaw: return k1_mapped_go<double, double, double, kModeRaw>(sh, a, grid, s);
    }
  } else if (precision == 1) {
    if (mode == kModeIter) return k1_mapped_go<float, float, float, kModeIter>(sh, a, grid, s);
  } else if (precision == 2) {
    if (mode == kModeInit) return k1_mapped_go<double, double, float, kModeInit>(sh, a, grid, s);
  }
  return -1;
}

}  // namespace emin
