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
// or 8-byte (FP32) load.  A wave owns a window of 64 such pairs from up to
// three consecutive nodes; for every neighbour block n of its node a lane
// reads the BS x BS block of A, the neighbour's row offsets and its map byte
// from LDS, then per row c of b one paired load of Y, and accumulates BS x 2
// products per row.  A missing group sends the lane's buffer offset past the
// buffer end, which reads as zero, so the FMAs need no select.  The Y loads
// of the next blocks are issued before block n is accumulated (two to four
// blocks in flight).
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "launch.hpp"

namespace emin {

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------------ structure --

// Rows that are not a sequence of whole aligned groups of G columns (or hold
// more than maxg groups) set flag `bit`.
__global__ __launch_bounds__(kBlock) void k_group_check(const int* __restrict__ prp,
                                                       const int* __restrict__ pci, int n, int G,
                                                       int maxg, int bit, int* flags) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int p0 = prp[i], l = prp[i + 1] - p0;
  bool ok = (l % G) == 0 && (l / G) <= maxg;
  for (int q = 0; ok && q < l / G; ++q) {
    const int c0 = pci[p0 + q * G];
    ok = (c0 % G) == 0;
    for (int j = 1; ok && j < G; ++j) ok = pci[p0 + q * G + j] == c0 + j;
  }
  if (!ok) atomicOr(flags, 1 << bit);
}

// Map bytes per node (padded to 16, so every node's map starts on a 16-byte
// boundary), and {slot pairs, neighbour blocks} per node.
__global__ __launch_bounds__(kBlock) void k_gmap_count(const int* __restrict__ arp,
                                                      const int* __restrict__ prp, int nnodes,
                                                      int bs, int G, long* __restrict__ cnt,
                                                      int2* __restrict__ shape) {
  const int a = blockIdx.x * kBlock + threadIdx.x;
  if (a >= nnodes) return;
  const int r0 = a * bs;
  const int nb = (arp[r0 + 1] - arp[r0]) / bs, l = prp[r0 + 1] - prp[r0];
  const long bytes = (long)nb * (l / G);
  cnt[a] = (bytes + 15) & ~15L;
  shape[a] = make_int2(l / 2, nb);
}

// One wave per node, lanes over the (neighbour block, group) pairs of the
// node: each group located in the neighbour's (sorted) group list by
// bisection.
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
  for (int n = lane; n < nb; n += kWave) {
    const int kc = aci[e0 + n * bs];  // first row of the neighbour node
    nq[nqrp[a] + n] = make_int2(prp[kc], prp[kc + 1] - prp[kc]);
  }
  unsigned char* out = gmap + gmrp[a];
  const int total = nb * ng;
  for (int x = lane; x < total; x += kWave) {
    const int n = x / ng, q = x - n * ng;
    const int kc = aci[e0 + n * bs];
    const int q0 = prp[kc], ngb = (prp[kc + 1] - q0) / G;
    const int c = pci[p0 + q * G];
    int lo = 0, hi = ngb - 1, pos = 0xFF;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int v = pci[q0 + mid * G];
      if (v == c) { pos = mid; break; }
      if (v < c) lo = mid + 1; else hi = mid - 1;
    }
    out[x] = (unsigned char)pos;  // = out[n * ng + q]
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

// Largest node row the staged kernel takes: neighbour blocks per node and
// map bytes per node (the launcher checks both; larger rows take the
// slot-level node kernel).
constexpr int kPairMaxNb = 32;
constexpr int kPairMaxMap = 2048;


// Modes: kModeIterRaw (Y_hat = mask(A Y) and the partial <Y, Y_hat>),
// kModeRaw (mask(A Y) only), kModeEnergy (the partial <Y, mask(A Y)>); the
// projector is applied by the consumer.
//
// Work comes as windows of 64 slot pairs (built once per pattern): the pairs
// of all node rows are taken in node order, and window w holds the next 64
// of them, from at most kWinNodes consecutive nodes (a node may start in one
// window and end in the next).  The cost of a load in the texture units is
// the same for every lane of the wave, active or not, and those units bound
// this kernel, so a wave whose lanes all hold a pair does the most work per
// load.
//
// Per window, the wave first copies its nodes' rows of A (BS rows of BS nb
// values each, two values per lane and load), neighbour descriptors and map
// bytes into a region of LDS of its own.  The neighbour loop then reads them
// from LDS, so the only memory loads left in it are the gathers of Y.
// (Scalar loads would do for the uniform values, but they complete out of
// order: a wait on one drains all in flight, which serialises a pipelined
// loop.)
template <class TA, class TV, class TO, int BS, int MODE, int DEPTH>
__global__ __launch_bounds__(kBlock) void k1_nodepair(K1Args a) {
  constexpr int WPB = kBlock / kWave;
  constexpr int K = kWinNodes;
  using TAcc = TV;
  static_assert(MODE == kModeIterRaw || MODE == kModeRaw || MODE == kModeEnergy,
                "the node-pair product returns K y without the projector");
  static_assert(DEPTH >= 2 && DEPTH <= 4, "two to four neighbour blocks in flight");
  __shared__ TA sA[WPB][BS][K * BS * kPairMaxNb];
  __shared__ int2 sQ[WPB][K * kPairMaxNb];
  __shared__ __attribute__((aligned(16))) unsigned char sM[WPB][kPairMaxMap];
  if (MODE == kModeIterRaw && a.st->done) return;
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  const TV* __restrict__ y = (const TV*)a.y;
  TO* __restrict__ out = (TO*)a.out;
  const TA* __restrict__ av = (const TA*)a.av;
  const __amdgpu_buffer_rsrc_t ybuf = __builtin_amdgcn_make_buffer_rsrc(
      (void*)a.y, (short)0, (int)((long)a.nnz_p * (long)sizeof(TV)), kRawWord3);
  const int G = a.grp;
  const int nnodes = a.n / BS;
  Uniform<int>* uprp = (Uniform<int>*)a.prp;
  Uniform<int>* uarp = (Uniform<int>*)a.arp;
  const __amdgpu_buffer_rsrc_t abuf = __builtin_amdgcn_make_buffer_rsrc(
      (void*)av, (short)0, (int)((long)uarp[a.n] * (long)sizeof(TA)), kRawWord3);
  Uniform<int>* uwin = (Uniform<int>*)a.win;  // {first node, first pair, nodes} per window
  double dot = 0.0;
  const int ntiles = (a.nwin + WPB - 1) / WPB;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int t = __builtin_amdgcn_readfirstlane(w.t * WPB + wid);
    if (t >= a.nwin) continue;  // uniform over the wave
    const int node0 = uwin[3 * t], p0 = uwin[3 * t + 1], nn = uwin[3 * t + 2];
    // the window's nodes (uniform): pattern rows, A rows, block and map
    // offsets in LDS, and the first lane of each
    int pr[K][BS], l[K], ng[K], nb[K], boff[K], moff[K], lane0[K + 1];
    lane0[0] = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int r0 = min(node0 + j, nnodes - 1) * BS;
#pragma unroll
      for (int r = 0; r < BS; ++r) pr[j][r] = uprp[r0 + r];
      l[j] = uprp[r0 + 1] - pr[j][0];
      ng[j] = l[j] / G;
      nb[j] = (uarp[r0 + 1] - uarp[r0]) / BS;
      boff[j] = j == 0 ? 0 : boff[j - 1] + nb[j - 1];
      moff[j] = j == 0 ? 0 : moff[j - 1] + ((nb[j - 1] * ng[j - 1] + 15) & ~15);
      lane0[j + 1] = j < nn ? min(kWave, lane0[j] + l[j] / 2 - (j == 0 ? p0 : 0)) : lane0[j];
    }
    // stage the window's A rows, neighbour descriptors and map bytes: for
    // consecutive nodes each is one contiguous range (the maps start on
    // 16-byte boundaries and are padded to them), copied in one sweep
    {
      int gA[K + 1], rl[K];  // first A entry of each node in the range; row length
      float rinv[K];
      gA[0] = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        rl[j] = BS * nb[j];
        rinv[j] = 1.0f / (float)max(rl[j], 1);
        gA[j + 1] = gA[j] + (j < nn ? BS * rl[j] : 0);
      }
      const int ea0 = uarp[node0 * BS];
      const int na = gA[K];
      for (int g = 2 * lane; g < na; g += 2 * kWave) {
        const Two<TA> v = load_two<TA>(abuf, (unsigned)(ea0 + g) * (unsigned)sizeof(TA), 0u);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int gg = g + h;
          if (gg >= na) break;
          int j = 0;
#pragma unroll
          for (int jj = 1; jj < K; ++jj) j += gg >= gA[jj] ? 1 : 0;
          int g0 = 0, len = 1, bo = 0;
          float ri = 1.0f;
#pragma unroll
          for (int jj = 0; jj < K; ++jj)
            if (j == jj) {
              g0 = gA[jj];
              len = rl[jj];
              ri = rinv[jj];
              bo = BS * boff[jj];
            }
          // row and entry of gg in its node (entries < 2^12: the float
          // quotient is exact after truncation)
          const int loc = gg - g0;
          const int r = (int)(((float)loc + 0.5f) * ri);
          sA[wid][r][bo + loc - r * len] = h ? v.y : v.x;
        }
      }
      const int nqa = a.nqrp[node0];
      int nbs = 0;  // descriptors of the window's nodes
#pragma unroll
      for (int j = 0; j < K; ++j) nbs += j < nn ? nb[j] : 0;
      for (int e = lane; e < nbs; e += kWave) sQ[wid][e] = a.nq[nqa + e];
      int mbs = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) mbs += j < nn ? ((nb[j] * ng[j] + 15) & ~15) : 0;
      typedef unsigned int u4 __attribute__((ext_vector_type(4)));
      const u4* msrc = reinterpret_cast<const u4*>(a.amap + a.mrp64[node0]);
      u4* mdst = reinterpret_cast<u4*>(&sM[wid][0]);
      for (int e = lane; e < mbs / 16; e += kWave) mdst[e] = msrc[e];
    }
    // the lane's node (per lane from here on); lanes past the window's last
    // pair are off
    int jl = 0;
#pragma unroll
    for (int j = 1; j < K; ++j) jl += (j < nn && lane >= lane0[j]) ? 1 : 0;
    int ll = 0, lng = 1, lnb = 0, lbo = 0, lmo = 0, first = 0, lp[BS];
#pragma unroll
    for (int r = 0; r < BS; ++r) lp[r] = 0;
#pragma unroll
    for (int j = 0; j < K; ++j)
      if (jl == j) {
        ll = l[j];
        lng = ng[j];
        lnb = nb[j];
        lbo = boff[j];
        lmo = moff[j];
        first = lane0[j] - (j == 0 ? p0 : 0);  // lane of the node's pair 0
#pragma unroll
        for (int r = 0; r < BS; ++r) lp[r] = pr[j][r];
      }
    int nbmax = 0, lend = 0;  // uniform: most blocks of a node, lanes in use
#pragma unroll
    for (int j = 0; j < K; ++j) {
      nbmax = j < nn ? max(nbmax, nb[j]) : nbmax;
      lend = j + 1 == nn ? lane0[j + 1] : lend;
    }
    // the wave's own LDS writes are seen by its later reads (in order)
    {
      // the lane's pair: slots s, s + 1 of its row; its group and offset in it
      const int s = 2 * (lane - first);
      const bool on = lane < lend && s < ll && lnb > 0;
      const int gq = on ? s / G : 0;
      const unsigned go = (unsigned)(s - gq * G) * (unsigned)sizeof(TV);
      TAcc acc[BS][2];
#pragma unroll
      for (int r = 0; r < BS; ++r) acc[r][0] = acc[r][1] = TAcc(0);
      // block n of the lane's node from LDS; indices past its last block are
      // clamped (valid entries, results discarded), so the loop body has no
      // branches.  The raw descriptor of block n (neighbour offsets, map
      // byte) is read a step before it is used.
      struct Desc { int2 q; int byte; };
      auto get_desc = [&](int n) -> Desc {
        const int k = n < lnb ? n : lnb - 1;
        Desc d;
        d.q = sQ[wid][lbo + k];
        d.byte = (int)sM[wid][lmo + k * lng + gq];
        return d;
      };
      auto get_blk = [&](int n, TAcc (&blk)[BS][BS]) {
        const int k = lbo + (n < lnb ? n : lnb - 1);
#pragma unroll
        for (int r = 0; r < BS; ++r)
#pragma unroll
          for (int c = 0; c < BS; ++c) blk[r][c] = (TAcc)sA[wid][r][k * BS + c];
      };
      // block n's Y values; a lane off the row, a group missing from the
      // neighbour's row and a block past the node's last read zeros
      // (bitwise conditions: no branch inside the loop)
      auto gather = [&](int n, const Desc& d, Two<TV> (&yv)[BS]) {
        const bool hit = on & (n < lnb) & (d.byte != 0xFF);
        const unsigned base =
            (unsigned)(d.byte * G + d.q.x) * (unsigned)sizeof(TV) + go;
        const unsigned stride = (unsigned)d.q.y * (unsigned)sizeof(TV);
#pragma unroll
        for (int c = 0; c < BS; ++c)
          yv[c] = load_two<TV>(ybuf, hit ? base + (unsigned)c * stride : kMissOff, 0u);
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
      // Pipeline over the neighbour blocks: the Y of blocks n + 1 .. n + D - 1
      // is in flight while block n is accumulated (D register buffers); the
      // A block and the descriptor of the next step are read from LDS one
      // step ahead.  The inner loop is unrolled so every buffer index is a
      // constant (U steps: D for even D, 2D for odd D, so the two A buffers
      // also keep their roles across passes).  A scheduling barrier keeps
      // each step's loads issued before its accumulation.  Lanes without a
      // pair sit the loop out (the branch is taken once per window, so every
      // load in the loop is issued unconditionally).
      if (on) {
        constexpr int U = (DEPTH % 2 == 0) ? DEPTH : 2 * DEPTH;
        Two<TV> yb[DEPTH][BS];
        TAcc bk[2][BS][BS];
        Desc dn = get_desc(0);
#pragma unroll
        for (int j = 0; j < DEPTH - 1; ++j) {
          gather(j, dn, yb[j]);
          dn = get_desc(j + 1);
          __builtin_amdgcn_sched_barrier(0);  // blocks issued in order
        }
        get_blk(0, bk[0]);
        for (int n = 0; n < nbmax; n += U) {
#pragma unroll
          for (int j = 0; j < U; ++j) {
            gather(n + j + DEPTH - 1, dn, yb[(j + DEPTH - 1) % DEPTH]);
            dn = get_desc(n + j + DEPTH);
            get_blk(n + j + 1, bk[(j + 1) % 2]);
            // keep the scheduler from sinking the loads above below the
            // accumulation (which would drain the pipeline every step)
            __builtin_amdgcn_sched_barrier(0);
            accumulate(bk[j % 2], yb[j % DEPTH]);
          }
        }
      }
      // epilogue: the node's rows at the lane's two slots (zeros for a node
      // without neighbour blocks)
      const bool own = lane < lend && s < ll;
#pragma unroll
      for (int r = 0; r < BS; ++r) {
        const int prow = lp[r];
        const double v[2] = {(double)acc[r][0], (double)acc[r][1]};
        if (!own) continue;
        const int idx = prow + s;
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

void launch_group_check(const int* prp, const int* pci, int n, int G, int maxg, int bit,
                        int* flags, hipStream_t s) {
  if (n > 0) k_group_check<<<cdiv(n, kBlock), kBlock, 0, s>>>(prp, pci, n, G, maxg, bit, flags);
}

void launch_gmap_count(const int* arp, const int* prp, int nnodes, int bs, int G, long* cnt,
                       int2* shape, hipStream_t s) {
  if (nnodes > 0)
    k_gmap_count<<<cdiv(nnodes, kBlock), kBlock, 0, s>>>(arp, prp, nnodes, bs, G, cnt, shape);
}

void launch_gmap_fill(const int* arp, const int* aci, const int* prp, const int* pci,
                      const long* gmrp, const int* nqrp, int nnodes, int bs, int G,
                      unsigned char* gmap, int2* nq, hipStream_t s) {
  if (nnodes > 0)
    k_gmap_fill<<<cdiv(nnodes, kBlock / kWave), kBlock, 0, s>>>(arp, aci, prp, pci, gmrp, nqrp,
                                                                nnodes, bs, G, gmap, nq);
}

template <class TA, class TV, class TO, int MODE, int DEPTH>
static int nodepair_go(const K1Shape& sh, const K1Args& a, int grid, hipStream_t s) {
  // sh.S > 0: at most sh.S blocks per CU, by padding each block's LDS
  constexpr int WPB = kBlock / kWave;
  const size_t stat = sizeof(TA) * WPB * 3 * kWinNodes * 3 * kPairMaxNb +
                      sizeof(int2) * WPB * kWinNodes * kPairMaxNb + (size_t)WPB * kPairMaxMap;
  const size_t want = sh.S > 0 ? (size_t)(160 * 1024) / sh.S + 64 : 0;
  const size_t dyn = want > stat ? want - stat : 0;
  if (sh.bs == 3) {
    k1_nodepair<TA, TV, TO, 3, MODE, DEPTH><<<grid, kBlock, dyn, s>>>(a);
    return 0;
  }
  if (sh.bs == 2) {
    k1_nodepair<TA, TV, TO, 2, MODE, DEPTH><<<grid, kBlock, dyn, s>>>(a);
    return 0;
  }
  return -1;
}

// The per-iteration product at the shape's pipeline depth (sh.G: neighbour
// blocks in flight, 0 = two); the once-per-solve forms run two deep.
template <class T>
static int nodepair_iter(const K1Shape& sh, const K1Args& a, int grid, hipStream_t s) {
  switch (sh.G) {
    case 0:
    case 2: return nodepair_go<T, T, T, kModeIterRaw, 2>(sh, a, grid, s);
    case 3: return nodepair_go<T, T, T, kModeIterRaw, 3>(sh, a, grid, s);
    case 4: return nodepair_go<T, T, T, kModeIterRaw, 4>(sh, a, grid, s);
  }
  return -1;
}

bool nodepair_fits(int max_nb, long max_map) {
  return max_nb <= kPairMaxNb && max_map <= kPairMaxMap;
}

// Windows of 64 slot pairs over the nodes in order: {first node, first pair
// of it, nodes} per window.  A window closes at 64 pairs, at kWinNodes
// nodes, or before a node whose map bytes would overflow the wave's map
// region; a node cut at 64 pairs continues in the next window.
void nodepair_windows(int nnodes, const int2* shape, const long* mapbytes, std::vector<int>& win) {
  win.clear();
  int node = 0, p = 0;
  while (node < nnodes) {
    const int node0 = node, p0 = p;
    int lanes = 0, nn = 0;
    long map = 0;
    while (node < nnodes && nn < kWinNodes) {
      if (nn > 0 && map + mapbytes[node] > kPairMaxMap) break;
      const int left = shape[node].x - p;
      const int take = std::min(left, kWave - lanes);
      lanes += take;
      map += mapbytes[node];
      ++nn;
      if (take < left) {  // the node continues in the next window
        p += take;
        break;
      }
      ++node;
      p = 0;
      if (lanes == kWave) break;
    }
    win.push_back(node0);
    win.push_back(p0);
    win.push_back(nn);
  }
}

int launch_k1_nodepair(int mode, int precision, const K1Shape& sh, const K1Args& a, int grid,
                       hipStream_t s) {
  if (!a.amap || !a.mrp64 || !a.nq || !a.nqrp || !a.win || a.grp < 2 || (a.grp & 1)) return -1;
  if ((long)a.nnz_p * 8 >= (1L << 31)) return -1;  // the buffer offsets are 31-bit
  if (precision == 0) {
    switch (mode) {
      case kModeIterRaw: return nodepair_iter<double>(sh, a, grid, s);
      case kModeRaw: return nodepair_go<double, double, double, kModeRaw, 2>(sh, a, grid, s);
      case kModeEnergy: return nodepair_go<double, double, double, kModeEnergy, 2>(sh, a, grid, s);
    }
  } else if (precision == 1) {
    if (mode == kModeIterRaw) return nodepair_iter<float>(sh, a, grid, s);
  }
  return -1;
}

}  // namespace emin
