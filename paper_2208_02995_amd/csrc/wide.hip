// Masked product for short pattern rows with one lane per row and whole rows
// moved in 16-byte vector loads (Sec. 4: Y_hat = mask(A Y) on the fixed
// pattern, then the block projector of Sec. 3.1 and the partial <Y, Y_hat>
// of Alg. 3).
//
// The gather kernels with several lanes per row issue one narrow load per
// (lane, column) and per (lane, value); on this GPU the address unit
// processes a fixed number of lanes per clock whatever the width, so the
// cost is the count of lane-loads, not the bytes.  Here a lane owns row i
// and reads
//   * its own pattern row (S column indices, S values of Y) in S/4 and
//     S*sizeof(T)/16 vector loads,
//   * A's row U entries at a time: the packed neighbour descriptors
//     (offset << 4 | length) in 16-byte loads, the values in pairs,
//   * the pattern rows of those U neighbours the same way as its own, all
//     issued before any is used (the next chunk's descriptors are fetched
//     while this chunk is matched, so a tile waits on about two round trips
//     per chunk of U neighbours rather than two per neighbour pair),
// then matches columns in registers.  Loads may run past the end of a row
// (never past the end of an allocation: every library buffer carries at
// least 64 bytes of slack); the surplus entries are masked out by the row
// lengths before they can match.  A's values are the caller's array, so the
// second value of a pair is loaded only when it belongs to the row.
#include "common.hpp"
#include "launch.hpp"
#include "project.hpp"

namespace emin {

template <class T>
struct __attribute__((aligned(sizeof(T)))) Vec16 {
  T v[16 / sizeof(T)];
};
template <class T>
struct __attribute__((aligned(sizeof(T)))) Pair {
  T v[2];
};

// out[0..N) = p[0..N) in 16-byte loads (p aligned to sizeof(T) only)
template <class T, int N>
__device__ __forceinline__ void load_row(const T* __restrict__ p, T (&out)[N]) {
  constexpr int E = 16 / sizeof(T);
  static_assert(N % E == 0, "row capacity must fill whole 16-byte loads");
#pragma unroll
  for (int c = 0; c < N / E; ++c) {
    const Vec16<T> w = *reinterpret_cast<const Vec16<T>*>(p + c * E);
#pragma unroll
    for (int k = 0; k < E; ++k) out[c * E + k] = w.v[k];
  }
}

// A's values of entries e .. e+3 of a row ending at e1 (the caller's array:
// nothing past e1 - 1 is read); missing entries are 0.
template <class TA, class TAcc>
__device__ __forceinline__ void load_vals4(const TA* __restrict__ av, int e, int e1, TAcc (&v)[4]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int f = e + 2 * h;
    if (f + 1 < e1) {
      const Pair<TA> t = *reinterpret_cast<const Pair<TA>*>(av + f);
      v[2 * h] = (TAcc)t.v[0];
      v[2 * h + 1] = (TAcc)t.v[1];
    } else {
      v[2 * h] = (f < e1) ? (TAcc)av[f] : TAcc(0);
      v[2 * h + 1] = TAcc(0);
    }
  }
}

// S = capacity of the row's own pattern row, SN = of its neighbours' rows
// (every neighbour row must be at most SN long), U = neighbours whose rows
// are in flight together (a multiple of 4)
template <class TA, class TI, class TO, int S, int SN, int U, int MODE, bool M1, bool SEG>
__global__ __launch_bounds__(kBlock) void k1_wide(K1Args a) {
  using TAcc = TI;
  constexpr int SY = (S * sizeof(TI) < 16) ? 16 / sizeof(TI) : S;     // own Y slots loaded
  constexpr int SNY = (SN * sizeof(TI) < 16) ? 16 / sizeof(TI) : SN;  // neighbour Y slots
  static_assert(U % 4 == 0, "neighbour chunk must fill whole 16-byte loads");
  if (!SEG && (MODE == kModeIter || MODE == kModeInit) && a.st->done) return;
  const TA* __restrict__ av = (const TA*)a.av;
  const TI* __restrict__ y = (const TI*)a.y;
  const int* __restrict__ pci = a.pci;
  const int* __restrict__ anb = a.anb;
  const double* __restrict__ bc = a.bc;
  TO* __restrict__ out = (TO*)a.out;
  const int mp = a.m * (a.m + 1) / 2;
  double dot = 0.0;
  const int ntiles = (a.n + kBlock - 1) / kBlock;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int li = w.t * kBlock + threadIdx.x;
    const bool valid = li < a.n;
    const int i = valid ? (a.rows ? a.rows[li] : li) : 0;
    int p0 = 0, l = 0, e0 = 0, e1 = 0;
    if (valid) {
      const Pair<int> pp = *reinterpret_cast<const Pair<int>*>(a.prp + i);
      const Pair<int> ee = *reinterpret_cast<const Pair<int>*>(a.arp + i);
      p0 = pp.v[0];
      l = pp.v[1] - p0;
      e0 = ee.v[0];
      e1 = ee.v[1];
    }
    // own row and the first chunk's descriptors and values: one round trip
    int col[S];
    TI yo[SY];
    load_row<int, S>(pci + p0, col);
    load_row<TI, SY>(y + p0, yo);
    int d[U];
    TAcc va[U];
    load_row<int, U>(anb + e0, d);
#pragma unroll
    for (int c = 0; c < U / 4; ++c) {
      TAcc t[4];
      load_vals4<TA, TAcc>(av, e0 + 4 * c, e1, t);
#pragma unroll
      for (int k = 0; k < 4; ++k) va[4 * c + k] = t[k];
    }
#pragma unroll
    for (int j = 0; j < S; ++j)
      if (j >= l) col[j] = -1;
    TAcc acc[S];
#pragma unroll
    for (int j = 0; j < S; ++j) acc[j] = TAcc(0);
    for (int e = e0; e < e1; e += U) {
      // every neighbour row of the chunk in flight at once
      int cn[U][SN];
      TI yn[U][SNY];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool has = e + u < e1;
        const int q = has ? (d[u] >> 4) : p0;
        load_row<int, SN>(pci + q, cn[u]);
        load_row<TI, SNY>(y + q, yn[u]);
        const int ln = has ? (d[u] & 15) : 0;
#pragma unroll
        for (int j = 0; j < SN; ++j)
          if (j >= ln) cn[u][j] = -2;
      }
      TAcc vc[U];
#pragma unroll
      for (int u = 0; u < U; ++u) vc[u] = va[u];
      // next chunk's descriptors and values while this one is matched
      const int en = e + U;
      if (en < e1) {
        load_row<int, U>(anb + en, d);
#pragma unroll
        for (int c = 0; c < U / 4; ++c) {
          TAcc t[4];
          load_vals4<TA, TAcc>(av, en + 4 * c, e1, t);
#pragma unroll
          for (int k = 0; k < 4; ++k) va[4 * c + k] = t[k];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int j = 0; j < SN; ++j) {
#pragma unroll
          for (int s = 0; s < S; ++s)
            if (col[s] == cn[u][j]) acc[s] = fma(vc[u], (TAcc)yn[u][j], acc[s]);
        }
      }
    }
    double v[S];
#pragma unroll
    for (int j = 0; j < S; ++j) v[j] = (double)acc[j];
    if (MODE != kModeEnergy && MODE != kModeRaw) {
      if (M1) {
        double g[S], gx = 0.0, gg = 0.0;
#pragma unroll
        for (int j = 0; j < S; ++j) {
          g[j] = (col[j] >= 0) ? bc[col[j]] : 0.0;
          gx += g[j] * v[j];
          gg += g[j] * g[j];
        }
        if (gg > 0.0) {
          const double c = gx / gg;
#pragma unroll
          for (int j = 0; j < S; ++j) v[j] -= g[j] * c;
        }
      } else {
        project_row<1, S, false>(v, col, bc, valid ? a.wpk + (long)i * mp : nullptr, a.m, valid);
      }
    }
    double rdot = 0.0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      if (col[j] < 0) continue;
      const int idx = p0 + j;
      if (MODE == kModeIter) {
        const TO o = (TO)v[j];
        out[idx] = o;
        rdot += (double)yo[j] * (double)o;
      } else if (MODE == kModeInit) {
        out[idx] = (TO)(-v[j]);
      } else if (MODE == kModePlain || MODE == kModeRaw) {
        out[idx] = (TO)v[j];
      } else {
        rdot += (double)yo[j] * v[j];
      }
    }
    if (SEG && (MODE == kModeIter || MODE == kModeEnergy)) {
      if (valid) a.rowdot[i] = rdot;
    } else {
      dot += rdot;
    }
  }
  if (!SEG && (MODE == kModeIter || MODE == kModeEnergy)) store_partial(dot, a.part_out);
}

template <class TA, class TI, class TO, int MODE, bool M1>
static int wide_go(const K1Shape& sh, const K1Args& a, int grid, hipStream_t s) {
#define EMIN_K1W(SS, NN, UU)                                                           \
  if (sh.S == SS && sh.G == NN && sh.L == UU) {                                        \
    if (a.seg)                                                                         \
      k1_wide<TA, TI, TO, SS, NN, UU, MODE, M1, true><<<grid, kBlock, 0, s>>>(a);      \
    else                                                                               \
      k1_wide<TA, TI, TO, SS, NN, UU, MODE, M1, false><<<grid, kBlock, 0, s>>>(a);     \
    return 0;                                                                          \
  }
  EMIN_K1W(4, 4, 4) EMIN_K1W(4, 8, 4) EMIN_K1W(8, 8, 4) EMIN_K1W(4, 4, 8) EMIN_K1W(8, 8, 8)
#undef EMIN_K1W
  return -1;
}

template <class TA, class TI, class TO, int MODE>
static int wide_m(const K1Shape& sh, const K1Args& a, int grid, hipStream_t s) {
  return a.m == 1 ? wide_go<TA, TI, TO, MODE, true>(sh, a, grid, s)
                  : wide_go<TA, TI, TO, MODE, false>(sh, a, grid, s);
}

// out[i] = longest pattern row among row i's neighbours in A (bucket plans)
__global__ __launch_bounds__(kBlock) void k_nb_maxlen(const int* __restrict__ arp,
                                                     const int* __restrict__ aci,
                                                     const int* __restrict__ prp, int n,
                                                     int* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int mx = 0;
  for (int e = arp[i]; e < arp[i + 1]; ++e) {
    const int k = aci[e];
    const int len = prp[k + 1] - prp[k];
    mx = len > mx ? len : mx;
  }
  out[i] = mx;
}

void launch_nb_maxlen(const int* arp, const int* aci, const int* prp, int n, int* out,
                      hipStream_t s) {
  if (n > 0) k_nb_maxlen<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(arp, aci, prp, n, out);
}

bool k1_wide_supported(int S, int SN, int U) {
  if (U == 4) return (S == 4 && (SN == 4 || SN == 8)) || (S == 8 && SN == 8);
  if (U == 8) return (S == 4 && SN == 4) || (S == 8 && SN == 8);
  return false;
}

int launch_k1_wide(int mode, int precision, const K1Shape& sh, const K1Args& a, int grid,
                   hipStream_t s) {
  if (!a.anb) return -1;
  if (precision == 0) {
    switch (mode) {
      case kModeIter: return wide_m<double, double, double, kModeIter>(sh, a, grid, s);
      case kModeInit: return wide_m<double, double, double, kModeInit>(sh, a, grid, s);
      case kModeEnergy: return wide_m<double, double, double, kModeEnergy>(sh, a, grid, s);
      case kModePlain: return wide_m<double, double, double, kModePlain>(sh, a, grid, s);
      case kModeRaw: return wide_m<double, double, double, kModeRaw>(sh, a, grid, s);
    }
  } else if (precision == 1) {
    if (mode == kModeIter) return wide_m<float, float, float, kModeIter>(sh, a, grid, s);
  } else if (precision == 2) {
    if (mode == kModeInit) return wide_m<double, double, float, kModeInit>(sh, a, grid, s);
  }
  return -1;
}

}  // namespace emin
