// Masked product for node-blocked problems whose pattern rows are made of
// whole coarse-column groups (the K y product of Sec. 4 on systems such as
// elasticity, with aggregation P0: every aggregate contributes G consecutive
// coarse columns, and a pattern grown from P0 (eq. enlPatt) holds either all
// or none of an aggregate's columns).
//
// For node a, its n-th neighbour node b (the n-th BS x BS block of A's node
// row) and group q of J_a, the intersection J_a cap J_b is recorded once per
// pattern as one byte,
//     gmap[gmrp[a] + n * (l_a / G) + q] = position of that group in J_b, or 0xFF,
// a G-th of the size of a slot-level map.  Because groups are aligned and G
// is even, a lane can own two consecutive slots (s, s + 1) of J_a: they lie in
// one group and map to two consecutive positions of J_b, and every row starts
// at an even pattern offset, so both values of a row come in one 16-byte (FP64)
// or 8-byte (FP32) load.  One wave owns a node; for every neighbour block the
// wave reads the BS x BS block of A and the neighbour's row offsets with
// scalar loads, each lane one map byte, then per row c of b one paired load
// of Y, and accumulates BS x 2 products per row.  The neighbour's row offset
// and row stride ride in the buffer instruction's scalar offset; a missing
// group sends the lane's vector offset past the buffer end, which reads as
// zero, so the FMAs need no select.  The Y loads of block n + 1 are issued
// before block n is accumulated.
#include "common.hpp"
#include "launch.hpp"

namespace emin {

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------------ structure --

// Rows whose pattern row is not a sequence of whole aligned groups of G
// columns set bit kFlagGroups of flags.
__global__ __launch_bounds__(kBlock) void k_group_check(const int* __restrict__ prp,
                                                       const int* __restrict__ pci, int n, int G,
                                                       int* flags) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int p0 = prp[i], l = prp[i + 1] - p0;
  bool ok = (l % G) == 0 && (l / G) < 255;
  for (int q = 0; ok && q < l / G; ++q) {
    const int c0 = pci[p0 + q * G];
    ok = (c0 % G) == 0;
    for (int j = 1; ok && j < G; ++j) ok = pci[p0 + q * G + j] == c0 + j;
  }
  if (!ok) atomicOr(flags, 1 << kFlagGroups);
}

__global__ __launch_bounds__(kBlock) void k_gmap_count(const int* __restrict__ arp,
                                                      const int* __restrict__ prp, int nnodes,
                                                      int bs, int G, long* __restrict__ cnt) {
  const int a = blockIdx.x * kBlock + threadIdx.x;
  if (a >= nnodes) return;
  const int r0 = a * bs;
  cnt[a] = (long)((arp[r0 + 1] - arp[r0]) / bs) * ((prp[r0 + 1] - prp[r0]) / G);
}

// One wave per node: for every neighbour block, lanes over the node's groups,
// each group located in the neighbour's (sorted) group list by bisection.
__global__ __launch_bounds__(kBlock) void k_gmap_fill(const int* __restrict__ arp,
                                                     const int* __restrict__ aci,
                                                     const int* __restrict__ prp,
                                                     const int* __restrict__ pci,
                                                     const long* __restrict__ gmrp,
                                                     const int* __restrict__ nqrp, int nnodes,
                                                     int bs, int G, unsigned char* __restrict__ gmap,
                                                     int2* __restrict__ nq) {
  const int lane = threadIdx.x % kWave;
  const int a = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  if (a >= nnodes) return;
  const int r0 = a * bs;
  const int p0 = prp[r0], ng = (prp[r0 + 1] - p0) / G;
  const int e0 = arp[r0], nb = (arp[r0 + 1] - e0) / bs;
  unsigned char* out = gmap + gmrp[a];
  for (int n = 0; n < nb; ++n) {
    const int kc = aci[e0 + n * bs];  // first row of the neighbour node
    const int q0 = prp[kc], lb = prp[kc + 1] - q0;
    if (lane == 0) nq[nqrp[a] + n] = make_int2(q0, lb);
    const int ngb = lb / G;
    for (int q = lane; q < ng; q += kWave) {
      const int c = pci[p0 + q * G];
      int lo = 0, hi = ngb - 1, pos = 0xFF;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = pci[q0 + mid * G];
        if (v == c) { pos = mid; break; }
        if (v < c) lo = mid + 1; else hi = mid - 1;
      }
      out[(long)n * ng + q] = (unsigned char)pos;
    }
  }
}

// ------------------------------------------------------------- product --

constexpr int kRawWord3 = 0x00020000;   // word 3 of a raw buffer resource (32-bit format)
constexpr unsigned kMissOff = 0x80000000u;  // beyond any buffer below 2 GiB

template <class T> struct Two { T x, y; };

// Two consecutive values at byte offset voff + soff of the buffer (zeros when
// voff is past its end).
template <class T>
__device__ __forceinline__ Two<T> load_two(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ Two<double> load_two<double>(__amdgpu_buffer_rsrc_t r, unsigned voff,
                                                        unsigned soff) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  const u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
  Two<double> o;
  o.x = __builtin_bit_cast(double, (unsigned long long)v.x | ((unsigned long long)v.y << 32));
  o.y = __builtin_bit_cast(double, (unsigned long long)v.z | ((unsigned long long)v.w << 32));
  return o;
}
// The halves are split from one 64-bit integer: extracting the elements of
// the builtin's 2 x 32-bit vector directly is narrowed by this compiler to a
// single 32-bit load whose value lands in both halves.
template <>
__device__ __forceinline__ Two<float> load_two<float>(__amdgpu_buffer_rsrc_t r, unsigned voff,
                                                      unsigned soff) {
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
  const unsigned long long w = __builtin_bit_cast(unsigned long long, v);
  Two<float> o;
  o.x = __builtin_bit_cast(float, (unsigned)(w & 0xffffffffull));
  o.y = __builtin_bit_cast(float, (unsigned)(w >> 32));
  return o;
}

template <class T>
__device__ __forceinline__ Two<T> ld_two(const T* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 q = *reinterpret_cast<const v2*>(p);
  return Two<T>{q.x, q.y};
}
template <class T>
__device__ __forceinline__ void st_two(T* p, T x, T y) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 q;
  q.x = x;
  q.y = y;
  *reinterpret_cast<v2*>(p) = q;
}

// Where one neighbour block's values are: its first row's pattern offset
// and row length (uniform) and the lane's map byte.
struct NbAddr {
  int q0, ql, pos;
};

// A node whose row holds more than 128 slots is done in passes of 64 slot
// pairs (one chunk per pass, re-reading A's blocks and the map): registers
// stay those of one chunk, so occupancy does not follow the longest row.
// Modes: kModeIterRaw (Y_hat = mask(A Y) and the partial <Y, Y_hat>),
// kModeRaw (mask(A Y) only), kModeEnergy (the partial <Y, mask(A Y)>); the
// projector is applied by the consumer.
template <class TA, class TV, class TO, int BS, int MODE>
__global__ __launch_bounds__(kBlock) void k1_nodepair(K1Args a) {
  constexpr int WPB = kBlock / kWave;
  using TAcc = TV;
  static_assert(MODE == kModeIterRaw || MODE == kModeRaw || MODE == kModeEnergy,
                "the node-pair product returns K y without the projector");
  if (MODE == kModeIterRaw && a.st->done) return;
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  const TV* __restrict__ y = (const TV*)a.y;
  TO* __restrict__ out = (TO*)a.out;
  const __amdgpu_buffer_rsrc_t ybuf = __builtin_amdgcn_make_buffer_rsrc(
      (void*)a.y, (short)0, (int)((long)a.nnz_p * (long)sizeof(TV)), kRawWord3);
  const int G = a.grp;
  const int nnodes = a.n / BS;
  double dot = 0.0;
  const int ntiles = (nnodes + WPB - 1) / WPB;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int node = __builtin_amdgcn_readfirstlane(w.t * WPB + wid);
    if (node >= nnodes) continue;  // uniform over the wave
    const int r0 = node * BS;
    Uniform<int>* uprp = (Uniform<int>*)a.prp;
    const int p0 = uprp[r0];
    const int l = uprp[r0 + 1] - p0;
    const int ng = l / G;
    const int nch = (l / 2 + kWave - 1) / kWave;  // pair chunks (0 for an empty row)
    Uniform<int>* uarp = (Uniform<int>*)a.arp;
    Uniform<TA>* uav = (Uniform<TA>*)a.av;
    int ea[BS];
#pragma unroll
    for (int r = 0; r < BS; ++r) ea[r] = uarp[r0 + r];
    const int nb = (uarp[r0 + 1] - ea[0]) / BS;
    const unsigned char* __restrict__ mrow = a.amap + a.mrp64[node];
    Uniform<int>* unq = (Uniform<int>*)(a.nq + a.nqrp[node]);
    for (int ch = 0; ch < nch; ++ch) {
      // the lane's pair: slots s, s + 1 of J_a; its group and offset in it
      const int s = 2 * (lane + kWave * ch);
      const bool on = s < l;
      const int gq = on ? s / G : 0;
      const unsigned go = (unsigned)(s - gq * G) * (unsigned)sizeof(TV);
      TAcc acc[BS][2];
#pragma unroll
      for (int r = 0; r < BS; ++r) acc[r][0] = acc[r][1] = TAcc(0);
      auto fetch_addr = [&](int n, NbAddr& d) {
        d.q0 = unq[2 * n];
        d.ql = unq[2 * n + 1];
        d.pos = on ? (int)mrow[(long)n * ng + gq] : 0xFF;
      };
      auto fetch_blk = [&](int n, TAcc (&blk)[BS][BS]) {
#pragma unroll
        for (int r = 0; r < BS; ++r)
#pragma unroll
          for (int c = 0; c < BS; ++c) blk[r][c] = (TAcc)uav[ea[r] + n * BS + c];
      };
      auto gather = [&](const NbAddr& d, Two<TV> (&yv)[BS]) {
        const unsigned vo =
            d.pos == 0xFF ? kMissOff : (unsigned)(d.pos * G) * (unsigned)sizeof(TV) + go;
#pragma unroll
        for (int c = 0; c < BS; ++c)
          yv[c] = load_two<TV>(ybuf, vo, (unsigned)(d.q0 + c * d.ql) * (unsigned)sizeof(TV));
      };
      auto accumulate = [&](const TAcc (&blk)[BS][BS], const Two<TV> (&yv)[BS]) {
#pragma unroll
        for (int c = 0; c < BS; ++c)
#pragma unroll
          for (int r = 0; r < BS; ++r) {
            acc[r][0] = fma(blk[r][c], (TAcc)yv[c].x, acc[r][0]);
            acc[r][1] = fma(blk[r][c], (TAcc)yv[c].y, acc[r][1]);
          }
      };
      // Pipeline: the map byte and offsets of block n + 2 are fetched and the
      // Y values of block n + 1 are in flight while block n is accumulated.
      // Unrolled by two so the buffers swap roles without copies.
      NbAddr ad;
      TAcc b0[BS][BS], b1[BS][BS];
      Two<TV> y0[BS], y1[BS];
      if (nb > 0) {
        fetch_addr(0, ad);
        gather(ad, y0);
        fetch_blk(0, b0);
        if (nb > 1) fetch_addr(1, ad);
      }
      for (int n = 0; n < nb; n += 2) {
        if (n + 1 < nb) {
          gather(ad, y1);
          fetch_blk(n + 1, b1);
          if (n + 2 < nb) fetch_addr(n + 2, ad);
        }
        accumulate(b0, y0);
        if (n + 1 < nb) {
          if (n + 2 < nb) {
            gather(ad, y0);
            fetch_blk(n + 2, b0);
            if (n + 3 < nb) fetch_addr(n + 3, ad);
          }
          accumulate(b1, y1);
        }
      }
      // epilogue: the node's rows at this pass's two slots per lane
#pragma unroll
      for (int r = 0; r < BS; ++r) {
        const int pr = uprp[r0 + r];
        const double v[2] = {(double)acc[r][0], (double)acc[r][1]};
        if (!on) continue;
        const int idx = pr + s;
        if constexpr (MODE == kModeIterRaw) {
          const TO o0 = (TO)v[0], o1 = (TO)v[1];
          st_two<TO>(out + idx, o0, o1);
          const Two<TV> yo = ld_two<TV>(y + idx);
          dot += (double)yo.x * (double)o0 + (double)yo.y * (double)o1;
        } else if constexpr (MODE == kModeRaw) {
          st_two<TO>(out + idx, (TO)v[0], (TO)v[1]);
        } else {  // kModeEnergy
          const Two<TV> yo = ld_two<TV>(y + idx);
          dot += (double)yo.x * v[0] + (double)yo.y * v[1];
        }
      }
    }
  }
  if (MODE == kModeIterRaw || MODE == kModeEnergy) store_partial(dot, a.part_out);
}

// ------------------------------------------------------------- launchers --

void launch_group_check(const int* prp, const int* pci, int n, int G, int* flags,
                        hipStream_t s) {
  if (n > 0) k_group_check<<<cdiv(n, kBlock), kBlock, 0, s>>>(prp, pci, n, G, flags);
}

void launch_gmap_count(const int* arp, const int* prp, int nnodes, int bs, int G, long* cnt,
                       hipStream_t s) {
  if (nnodes > 0)
    k_gmap_count<<<cdiv(nnodes, kBlock), kBlock, 0, s>>>(arp, prp, nnodes, bs, G, cnt);
}

void launch_gmap_fill(const int* arp, const int* aci, const int* prp, const int* pci,
                      const long* gmrp, const int* nqrp, int nnodes, int bs, int G,
                      unsigned char* gmap, int2* nq, hipStream_t s) {
  if (nnodes > 0)
    k_gmap_fill<<<cdiv(nnodes, kBlock / kWave), kBlock, 0, s>>>(arp, aci, prp, pci, gmrp, nqrp,
                                                                nnodes, bs, G, gmap, nq);
}

template <class TA, class TV, class TO, int MODE>
static int nodepair_go(const K1Shape& sh, const K1Args& a, int grid, hipStream_t s) {
  if (sh.bs == 3) {
    k1_nodepair<TA, TV, TO, 3, MODE><<<grid, kBlock, 0, s>>>(a);
    return 0;
  }
  if (sh.bs == 2) {
    k1_nodepair<TA, TV, TO, 2, MODE><<<grid, kBlock, 0, s>>>(a);
    return 0;
  }
  return -1;
}

int launch_k1_nodepair(int mode, int precision, const K1Shape& sh, const K1Args& a, int grid,
                       hipStream_t s) {
  if (!a.amap || !a.mrp64 || !a.nq || !a.nqrp || a.grp < 2 || (a.grp & 1)) return -1;
  if ((long)a.nnz_p * 8 >= (1L << 31)) return -1;  // the buffer offsets are 31-bit
  if (precision == 0) {
    switch (mode) {
      case kModeIterRaw: return nodepair_go<double, double, double, kModeIterRaw>(sh, a, grid, s);
      case kModeRaw: return nodepair_go<double, double, double, kModeRaw>(sh, a, grid, s);
      case kModeEnergy: return nodepair_go<double, double, double, kModeEnergy>(sh, a, grid, s);
    }
  } else if (precision == 1) {
    if (mode == kModeIterRaw) return nodepair_go<float, float, float, kModeIterRaw>(sh, a, grid, s);
  }
  return -1;
}

}  // namespace emin
