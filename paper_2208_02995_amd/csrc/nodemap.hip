// Masked product for node-blocked problems with long pattern rows (systems
// such as elasticity: BS unknowns per mesh node, A stored as full BS x BS
// node blocks, the BS rows of a node sharing one pattern row J_a; Sec. 4's
// K y product with the block projector of Sec. 3.1 in the epilogue).
//
// The intersection of J_a with each neighbour node's J_b is fixed for the
// whole iteration, so it is worked out once per pattern, at node level: for
// node a, neighbour n (the n-th node block of A's row) and slot s of J_a,
//     nmap[nmrp[a] + n * l_a + s] = position of J_a[s] inside J_b, or 0xFF,
// and nq[nqrp[a] + n] = (start of node b's first row in the pattern, its
// length): b's rows are consecutive rows of equal length.
// One wave owns node a; lane g owns slots g, g + 64, ...  For every
// neighbour block the wave reads the BS x BS block of A (the same for all
// lanes), one map byte per slot and the BS values Y(b rows, position), and
// accumulates BS x BS products per slot in registers.  No hashing, no LDS,
// no barriers.  U neighbour blocks are handled together so that all their
// loads are in flight at once (the kernel is bound by gather latency).
// Y is gathered with raw buffer loads: 32-bit byte offsets (no 64-bit
// address arithmetic per lane), and a slot missing from J_b gets an offset
// past the buffer's end, which the hardware reads as 0 -- no select.  This
// needs nnz(pattern) * sizeof(value) < 2^31.
#include "common.hpp"
#include "launch.hpp"
#include "project.hpp"

namespace emin {

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

__global__ __launch_bounds__(kBlock) void k_nmap_count(const int* __restrict__ arp,
                                                      const int* __restrict__ prp, int nnodes,
                                                      int bs, long* __restrict__ cnt) {
  const int a = blockIdx.x * kBlock + threadIdx.x;
  if (a >= nnodes) return;
  const int r0 = a * bs;
  const long nb = (arp[r0 + 1] - arp[r0]) / bs;
  cnt[a] = nb * (prp[r0 + 1] - prp[r0]);
}

__global__ __launch_bounds__(kBlock) void k_nmap_fill(const int* __restrict__ arp,
                                                     const int* __restrict__ aci,
                                                     const int* __restrict__ prp,
                                                     const int* __restrict__ pci,
                                                     const long* __restrict__ nmrp,
                                                     const int* __restrict__ nqrp, int nnodes,
                                                     int bs, unsigned char* __restrict__ nmap,
                                                     int2* __restrict__ nq) {
  const int a = blockIdx.x * kBlock + threadIdx.x;
  if (a >= nnodes) return;
  const int r0 = a * bs;
  const int p0 = prp[r0], l = prp[r0 + 1] - p0;
  const int e0 = arp[r0], nb = (arp[r0 + 1] - e0) / bs;
  unsigned char* out = nmap + nmrp[a];
  for (int n = 0; n < nb; ++n) {
    const int kc = aci[e0 + n * bs];
    const int q0 = prp[kc], q1 = prp[kc + 1];
    nq[nqrp[a] + n] = make_int2(q0, q1 - q0);  // the neighbour node's rows: q0 + c (q1 - q0)
    int lo0 = q0;  // J_a and J_b are sorted: the search window only moves right
    for (int s = 0; s < l; ++s) {
      const int c = pci[p0 + s];
      int lo = lo0, hi = q1 - 1, pos = 0xFF;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = pci[mid];
        if (v == c) { pos = mid - q0; break; }
        if (v < c) lo = mid + 1; else hi = mid - 1;
      }
      if (pos != 0xFF) lo0 = q0 + pos + 1;
      else lo0 = lo;
      out[(long)n * l + s] = (unsigned char)pos;
    }
  }
}

template <class T>
__device__ __forceinline__ T buffer_load(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ __forceinline__ double buffer_load<double>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  return __builtin_bit_cast(double, v);
}
template <>
__device__ __forceinline__ float buffer_load<float>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// word 3 of a raw buffer resource on this GPU family (32-bit data format)
constexpr int kRawBufferWord3 = 0x00020000;
constexpr unsigned kMissOffset = 0x80000000u;  // beyond any buffer below 2 GiB

// U > 0: U neighbour blocks per step, the next step's descriptors fetched
// during this step's gathers.  U == 0: one block per step, three deep: the
// gathers of block n+1 and the descriptors of block n+2 are in flight while
// block n is accumulated.
template <class TA, class TI, class TO, int BS, int L, int U, int MODE, bool M1>
__global__ __launch_bounds__(kBlock) void k1_nodemap(K1Args a) {
  using TAcc = TI;
  constexpr int WPB = kBlock / kWave;
  if ((MODE == kModeIter || MODE == kModeIterRaw || MODE == kModeInit) && a.st->done) return;
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  const TI* __restrict__ y = (const TI*)a.y;
  const unsigned char* __restrict__ nmap = a.amap;
  TO* __restrict__ out = (TO*)a.out;
  const __amdgpu_buffer_rsrc_t ybuf = __builtin_amdgcn_make_buffer_rsrc(
      (void*)a.y, (short)0, (int)((long)a.nnz_p * (long)sizeof(TI)), kRawBufferWord3);
  const int mp = a.m * (a.m + 1) / 2;
  const int nnodes = a.n / BS;
  double dot = 0.0;
  const int ntiles = (nnodes + WPB - 1) / WPB;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    // node-level quantities are the same on every lane: keep them scalar
    const int node = __builtin_amdgcn_readfirstlane(w.t * WPB + wid);
    const bool valid = node < nnodes;
    const int r0 = node * BS;
    int p0 = 0, l = 0;
    if (valid) {
      p0 = __builtin_amdgcn_readfirstlane(a.prp[r0]);
      l = __builtin_amdgcn_readfirstlane(a.prp[r0 + 1]) - p0;
    }
    TAcc acc[BS][L];
#pragma unroll
    for (int r = 0; r < BS; ++r)
#pragma unroll
      for (int t = 0; t < L; ++t) acc[r][t] = TAcc(0);
    if (valid) {
      Uniform<int>* uarp = (Uniform<int>*)a.arp;
      Uniform<TA>* uav = (Uniform<TA>*)a.av;
      int ea[BS];
#pragma unroll
      for (int r = 0; r < BS; ++r) ea[r] = uarp[r0 + r];
      const int nb = (uarp[r0 + 1] - ea[0]) / BS;
      const long mb = a.mrp64[node];
      Uniform<int>* unq = (Uniform<int>*)(a.nq + a.nqrp[node]);  // (start, length) pairs
      const int nch = (l + kWave - 1) / kWave;  // slot chunks in use (<= L)
      if constexpr (U == 0) {
        // fetched (block n+2 while block n is accumulated), gathered (n+1), current (n)
        int f0 = 0, fl = 0, fq[L];
        TAcc fblk[BS][BS];
        TAcc gy[L][BS], gblk[BS][BS];
#define EMIN_NM_FETCH(NN)                                                              \
  {                                                                                    \
    const int n_ = (NN);                                                               \
    f0 = unq[2 * n_];                                                                  \
    fl = unq[2 * n_ + 1];                                                              \
    _Pragma("unroll") for (int r = 0; r < BS; ++r)                                     \
      _Pragma("unroll") for (int c = 0; c < BS; ++c)                                   \
        fblk[r][c] = (TAcc)uav[ea[r] + n_ * BS + c];                                   \
    const unsigned char* __restrict__ mrow = nmap + mb + (long)n_ * l;                 \
    _Pragma("unroll") for (int t = 0; t < L; ++t) {                                    \
      const int s = lane + kWave * t;                                                  \
      fq[t] = (t < nch && s < l) ? (int)mrow[s] : 0xFF;                                \
    }                                                                                  \
  }
#define EMIN_NM_GATHER(YY)                                                             \
  _Pragma("unroll") for (int t = 0; t < L; ++t) {                                      \
    if (t >= nch) break;                                                               \
    const unsigned qo = fq[t] == 0xFF ? kMissOffset : (unsigned)fq[t] * (unsigned)sizeof(TI); \
    _Pragma("unroll") for (int c = 0; c < BS; ++c)                                     \
      YY[t][c] = buffer_load<TI>(ybuf, qo + (unsigned)(f0 + c * fl) * (unsigned)sizeof(TI)); \
  }
        if (nb > 0) {
          EMIN_NM_FETCH(0)
          EMIN_NM_GATHER(gy)
#pragma unroll
          for (int r = 0; r < BS; ++r)
#pragma unroll
            for (int c = 0; c < BS; ++c) gblk[r][c] = fblk[r][c];
          if (nb > 1) EMIN_NM_FETCH(1)
        }
        for (int n = 0; n < nb; ++n) {
          const bool more = n + 1 < nb;
          TAcc ny[L][BS], nblk[BS][BS];
          if (more) {
            EMIN_NM_GATHER(ny)
#pragma unroll
            for (int r = 0; r < BS; ++r)
#pragma unroll
              for (int c = 0; c < BS; ++c) nblk[r][c] = fblk[r][c];
          }
          if (n + 2 < nb) EMIN_NM_FETCH(n + 2)
#pragma unroll
          for (int t = 0; t < L; ++t) {
            if (t >= nch) break;
#pragma unroll
            for (int c = 0; c < BS; ++c)
#pragma unroll
              for (int r = 0; r < BS; ++r) acc[r][t] = fma(gblk[r][c], gy[t][c], acc[r][t]);
          }
          if (more) {
#pragma unroll
            for (int t = 0; t < L; ++t)
#pragma unroll
              for (int c = 0; c < BS; ++c) gy[t][c] = ny[t][c];
#pragma unroll
            for (int r = 0; r < BS; ++r)
#pragma unroll
              for (int c = 0; c < BS; ++c) gblk[r][c] = nblk[r][c];
          }
        }
#undef EMIN_NM_FETCH
#undef EMIN_NM_GATHER
      } else {
        // U neighbour blocks per step; the next step's descriptors, A blocks
        // and map bytes are fetched while this step's gathers of Y are in flight
        int dq0[U], dql[U];
        TAcc blk[U][BS][BS];
        int q[U][L];
        auto fetch = [&](int n0) {
  #pragma unroll
          for (int u = 0; u < U; ++u) {
            const int n = (n0 + u < nb) ? n0 + u : nb - 1;  // repeat the last block
            dq0[u] = unq[2 * n];
            dql[u] = unq[2 * n + 1];
  #pragma unroll
            for (int r = 0; r < BS; ++r)
  #pragma unroll
              for (int c = 0; c < BS; ++c)
                blk[u][r][c] = (n0 + u < nb) ? (TAcc)uav[ea[r] + n * BS + c] : TAcc(0);
            const unsigned char* __restrict__ mrow = nmap + mb + (long)n * l;
  #pragma unroll
            for (int t = 0; t < L; ++t) {
              const int s = lane + kWave * t;
              q[u][t] = (t < nch && s < l) ? (int)mrow[s] : 0xFF;
            }
          }
        };
        if (nb > 0) fetch(0);
        for (int n0 = 0; n0 < nb; n0 += U) {
          TAcc yv[U][L][BS];
          TAcc bc_[U][BS][BS];
  #pragma unroll
          for (int u = 0; u < U; ++u) {
  #pragma unroll
            for (int r = 0; r < BS; ++r)
  #pragma unroll
              for (int c = 0; c < BS; ++c) bc_[u][r][c] = blk[u][r][c];
  #pragma unroll
            for (int t = 0; t < L; ++t) {
              if (t >= nch) break;  // the same on every lane
              const unsigned qo =
                  q[u][t] == 0xFF ? kMissOffset : (unsigned)q[u][t] * (unsigned)sizeof(TI);
  #pragma unroll
              for (int c = 0; c < BS; ++c)
                yv[u][t][c] = buffer_load<TI>(
                    ybuf, qo + (unsigned)(dq0[u] + c * dql[u]) * (unsigned)sizeof(TI));
            }
          }
          if (n0 + U < nb) fetch(n0 + U);
  #pragma unroll
          for (int u = 0; u < U; ++u)
  #pragma unroll
            for (int t = 0; t < L; ++t) {
              if (t >= nch) break;
  #pragma unroll
              for (int c = 0; c < BS; ++c)
  #pragma unroll
                for (int r = 0; r < BS; ++r) acc[r][t] = fma(bc_[u][r][c], yv[u][t][c], acc[r][t]);
            }
        }
      }
    }
    int oc[L];
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int s = lane + kWave * t;
      oc[t] = (valid && s < l) ? a.pci[p0 + s] : -1;
    }
#pragma unroll
    for (int r = 0; r < BS; ++r) {
      double v[L];
#pragma unroll
      for (int t = 0; t < L; ++t) v[t] = (double)acc[r][t];
      const int row = r0 + r;
      if (MODE != kModeEnergy && MODE != kModeRaw && MODE != kModeIterRaw)
        project_row<kWave, L, M1>(v, oc, a.bc, valid ? a.wpk + (long)row * mp : nullptr, a.m,
                                  valid);
      const int pr = valid ? a.prp[row] : 0;
#pragma unroll
      for (int t = 0; t < L; ++t) {
        if (oc[t] < 0) continue;
        const int idx = pr + lane + kWave * t;
        if (MODE == kModeIter || MODE == kModeIterRaw) {
          const TO o = (TO)v[t];
          out[idx] = o;
          dot += (double)y[idx] * (double)o;
        } else if (MODE == kModeInit) {
          out[idx] = (TO)(-v[t]);
        } else if (MODE == kModePlain || MODE == kModeRaw) {
          out[idx] = (TO)v[t];
        } else {
          dot += (double)y[idx] * v[t];
        }
      }
    }
  }
  if (MODE == kModeIter || MODE == kModeIterRaw || MODE == kModeEnergy)
    store_partial(dot, a.part_out);
}

// ------------------------------------------------------------- launchers --

void launch_nmap_count(const int* arp, const int* prp, int nnodes, int bs, long* cnt,
                       hipStream_t s) {
  if (nnodes > 0) k_nmap_count<<<cdiv(nnodes, kBlock), kBlock, 0, s>>>(arp, prp, nnodes, bs, cnt);
}

void launch_nmap_fill(const int* arp, const int* aci, const int* prp, const int* pci,
                      const long* nmrp, const int* nqrp, int nnodes, int bs, unsigned char* nmap,
                      int2* nq, hipStream_t s) {
  if (nnodes > 0)
    k_nmap_fill<<<cdiv(nnodes, kBlock), kBlock, 0, s>>>(arp, aci, prp, pci, nmrp, nqrp, nnodes,
                                                        bs, nmap, nq);
}

template <class TA, class TI, class TO, int MODE>
static int nodemap_go(const K1Shape& sh, const K1Args& a, int grid, hipStream_t s) {
#define EMIN_K1NM(BB, LL, UU)                                                          \
  if (sh.bs == BB && sh.L == LL && sh.G == UU) {                                       \
    if (a.m == 1)                                                                      \
      k1_nodemap<TA, TI, TO, BB, LL, UU, MODE, true><<<grid, kBlock, 0, s>>>(a);       \
    else                                                                               \
      k1_nodemap<TA, TI, TO, BB, LL, UU, MODE, false><<<grid, kBlock, 0, s>>>(a);      \
    return 0;                                                                          \
  }
  EMIN_K1NM(2, 1, 2) EMIN_K1NM(2, 2, 2) EMIN_K1NM(2, 3, 2) EMIN_K1NM(2, 4, 2)
  EMIN_K1NM(3, 1, 2) EMIN_K1NM(3, 2, 2) EMIN_K1NM(3, 3, 2) EMIN_K1NM(3, 4, 2)
  EMIN_K1NM(3, 1, 4) EMIN_K1NM(3, 2, 4) EMIN_K1NM(3, 3, 4) EMIN_K1NM(3, 4, 4)
  EMIN_K1NM(3, 1, 1) EMIN_K1NM(3, 2, 1) EMIN_K1NM(3, 3, 1) EMIN_K1NM(3, 4, 1)
  EMIN_K1NM(3, 1, 0) EMIN_K1NM(3, 2, 0) EMIN_K1NM(3, 3, 0) EMIN_K1NM(3, 4, 0)
  EMIN_K1NM(2, 1, 0) EMIN_K1NM(2, 2, 0) EMIN_K1NM(2, 3, 0) EMIN_K1NM(2, 4, 0)
#undef EMIN_K1NM
  return -1;
}

int launch_k1_nodemap(int mode, int precision, const K1Shape& sh, const K1Args& a, int grid,
                      hipStream_t s) {
  if (!a.amap || !a.mrp64 || !a.nq || !a.nqrp) return -1;
  if ((long)a.nnz_p * 8 >= (1L << 31)) return -1;  // the buffer offsets are 31-bit
  if (precision == 0) {
    switch (mode) {
      case kModeIter: return nodemap_go<double, double, double, kModeIter>(sh, a, grid, s);
      case kModeInit: return nodemap_go<double, double, double, kModeInit>(sh, a, grid, s);
      case kModeEnergy: return nodemap_go<double, double, double, kModeEnergy>(sh, a, grid, s);
      case kModePlain: return nodemap_go<double, double, double, kModePlain>(sh, a, grid, s);
      case kModeRaw: return nodemap_go<double, double, double, kModeRaw>(sh, a, grid, s);
      case kModeIterRaw: return nodemap_go<double, double, double, kModeIterRaw>(sh, a, grid, s);
    }
  } else if (precision == 1) {
    if (mode == kModeIter) return nodemap_go<float, float, float, kModeIter>(sh, a, grid, s);
    if (mode == kModeIterRaw) return nodemap_go<float, float, float, kModeIterRaw>(sh, a, grid, s);
  } else if (precision == 2) {
    if (mode == kModeInit) return nodemap_go<double, double, float, kModeInit>(sh, a, grid, s);
  }
  return -1;
}

}  // namespace emin
