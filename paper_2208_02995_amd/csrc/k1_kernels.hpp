// Kernel templates of the two general masked-product shapes (see spgemm.hip
// for what they compute); instantiated, by precision and mode, in
// k1short_a.hip, k1short_b.hip and k1hash.hip so they compile in parallel.
#pragma once

#include "common.hpp"
#include "launch.hpp"
#include "project.hpp"

namespace emin {


template <class TA, class TI, class TO, int G, int S, int MODE, bool M1, bool PACKED>
__global__ __launch_bounds__(kBlock) void k1_short(K1Args a) {
  using TAcc = TI;
  constexpr int L = S / G;
  constexpr int ROWS = kBlock / G;
  if ((MODE == kModeIter || MODE == kModeInit) && a.st->done) return;
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  const TA* __restrict__ av = (const TA*)a.av;
  const TI* __restrict__ y = (const TI*)a.y;
  const int* __restrict__ pci = a.pci;
  const double* __restrict__ bc = a.bc;
  TO* __restrict__ out = (TO*)a.out;
  const int mp = a.m * (a.m + 1) / 2;
  double dot = 0.0;
  const int ntiles = (a.n + ROWS - 1) / ROWS;
  TileWalk w(ntiles);
  // row pointers of the first tile; the loop prefetches the next tile's
  int i = w.t * ROWS + grp;
  int np0 = 0, np1 = 0, ne0 = 0, ne1 = 0;
  if (w.t < w.end && i < a.n) {
    np0 = a.prp[i]; np1 = a.prp[i + 1]; ne0 = a.arp[i]; ne1 = a.arp[i + 1];
  }
  for (; w.t < w.end; w.t += w.step) {
    const bool valid = i < a.n;
    const int p0 = np0, l = valid ? np1 - np0 : 0, e0 = ne0, e1 = valid ? ne1 : ne0;
    {
      const int tn = w.t + w.step;
      const int inext = tn * ROWS + grp;
      if (tn < w.end && inext < a.n) {
        np0 = a.prp[inext]; np1 = a.prp[inext + 1]; ne0 = a.arp[inext]; ne1 = a.arp[inext + 1];
      }
      i = inext;
    }
    // own row: all S columns (for matching), plus this lane's owned slots'
    // columns, Y values and B_c entries -- independent of the neighbour
    // gathers below, so they are in flight together
    int col[S];
#pragma unroll
    for (int j = 0; j < S; ++j) {
      col[j] = pci[(j < l) ? p0 + j : 0];
      if (j >= l) col[j] = -1;
    }
    int oc[L];
    double yo[L], g[L];
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int s = lane * L + t;
      const int is = (s < l) ? p0 + s : 0;
      oc[t] = pci[is];
      yo[t] = (double)y[is];
      if (s >= l) oc[t] = -1;
      if (M1) g[t] = (oc[t] >= 0) ? bc[oc[t]] : 0.0;
    }
    TAcc acc[S];
#pragma unroll
    for (int j = 0; j < S; ++j) acc[j] = TAcc(0);
    for (int e = e0 + lane; e < e1; e += 2 * G) {
      const int eb = e + G;
      const bool hb = eb < e1;
      int qa, la, qb, lb;
      if (PACKED) {
        const int wa = a.anb[e];
        const int wb = hb ? a.anb[eb] : 0;
        qa = wa >> 4;
        la = wa & 15;
        qb = wb >> 4;
        lb = wb & 15;
      } else {
        const int ka = a.aci[e];
        const int kb = hb ? a.aci[eb] : ka;
        qa = a.prp[ka];
        la = a.prp[ka + 1] - qa;
        qb = a.prp[kb];
        lb = hb ? a.prp[kb + 1] - qb : 0;
      }
      const TAcc va = (TAcc)av[e];
      const TAcc vb = hb ? (TAcc)av[eb] : TAcc(0);
      int ca[S], cb[S];
      TAcc ya[S], yb[S];
#pragma unroll
      for (int j = 0; j < S; ++j) {
        const int ia = (j < la) ? qa + j : 0;
        const int ib = (j < lb) ? qb + j : 0;
        ca[j] = pci[ia];
        ya[j] = (TAcc)y[ia];
        cb[j] = pci[ib];
        yb[j] = (TAcc)y[ib];
        if (j >= la) ca[j] = -2;
        if (j >= lb) cb[j] = -2;
      }
#pragma unroll
      for (int j = 0; j < S; ++j) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
          if (col[s] == ca[j]) acc[s] = fma(va, ya[j], acc[s]);
          if (col[s] == cb[j]) acc[s] = fma(vb, yb[j], acc[s]);
        }
      }
    }
    ReduceScatter<G, S, TAcc>::run(acc, lane);
    double v[L];
#pragma unroll
    for (int t = 0; t < L; ++t) v[t] = (double)acc[t];
    if (MODE != kModeEnergy) {
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
        project_row<G, L, false>(v, oc, bc, valid ? a.wpk + (long)(w.t * ROWS + grp) * mp : nullptr,
                                 a.m, valid);
      }
    }
#pragma unroll
    for (int t = 0; t < L; ++t) {
      if (oc[t] < 0) continue;
      const int idx = p0 + lane * L + t;
      if (MODE == kModeIter) {
        const TO o = (TO)v[t];
        out[idx] = o;
        dot += yo[t] * (double)o;
      } else if (MODE == kModeInit) {
        out[idx] = (TO)(-v[t]);
      } else if (MODE == kModePlain) {
        out[idx] = (TO)v[t];
      } else {
        dot += yo[t] * v[t];
      }
    }
  }
  if (MODE == kModeIter || MODE == kModeEnergy) store_partial(dot, a.part_out);
}

template <int SL>
struct HashSize {
  static constexpr int v = (2 * SL <= 128) ? 128 : (2 * SL <= 256) ? 256 : (2 * SL <= 512) ? 512 : 1024;
};

__device__ __forceinline__ unsigned int hash_col(int c) { return (unsigned int)c * 2654435761u; }

template <class TA, class TI, class TO, int BS, int L, int MODE, bool M1>
__global__ __launch_bounds__(kBlock) void k1_node(K1Args a) {
  using TAcc = TI;
  constexpr int WPB = kBlock / kWave;
  constexpr int SL = kWave * L;
  constexpr int HS = HashSize<SL>::v;
  __shared__ int hkey[WPB][HS];
  __shared__ short hval[WPB][HS];
  __shared__ TAcc sacc[WPB][BS][SL];
  if ((MODE == kModeIter || MODE == kModeInit) && a.st->done) return;
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  const TA* __restrict__ av = (const TA*)a.av;
  const TI* __restrict__ y = (const TI*)a.y;
  TO* __restrict__ out = (TO*)a.out;
  const int mp = a.m * (a.m + 1) / 2;
  const int nnodes = a.n / BS;
  double dot = 0.0;
  const int ntiles = (nnodes + WPB - 1) / WPB;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int node = w.t * WPB + wid;
    const bool valid = node < nnodes;
    const int r0 = node * BS;
    int p0 = 0, l = 0;
    if (valid) {
      p0 = a.prp[r0];
      l = a.prp[r0 + 1] - p0;
    }
    for (int h = lane; h < HS; h += kWave) hkey[wid][h] = -1;
#pragma unroll
    for (int r = 0; r < BS; ++r)
#pragma unroll
      for (int t = 0; t < L; ++t) sacc[wid][r][lane + kWave * t] = TAcc(0);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int s = lane + kWave * t;
      if (s < l) {
        const int c = a.pci[p0 + s];
        unsigned int h = hash_col(c) & (HS - 1);
        while (atomicCAS(&hkey[wid][h], -1, c) != -1) h = (h + 1) & (HS - 1);
        hval[wid][h] = (short)s;
      }
    }
    __syncthreads();
    if (valid) {
      const int ea0 = a.arp[r0], ea1 = a.arp[r0 + 1];
      for (int e = ea0; e < ea1; e += BS) {
        const int kc = a.aci[e];  // first row of the neighbour node
        TAcc blk[BS][BS];
#pragma unroll
        for (int r = 0; r < BS; ++r)
#pragma unroll
          for (int c = 0; c < BS; ++c) blk[r][c] = (TAcc)av[a.arp[r0 + r] + (e - ea0) + c];
        int qb[BS];
#pragma unroll
        for (int c = 0; c < BS; ++c) qb[c] = a.prp[kc + c];
        const int lb = a.prp[kc + 1] - qb[0];
        for (int q = lane; q < lb; q += kWave) {
          const int c = a.pci[qb[0] + q];
          unsigned int h = hash_col(c) & (HS - 1);
          int s = -1;
          while (true) {
            const int key = hkey[wid][h];
            if (key == c) { s = hval[wid][h]; break; }
            if (key == -1) break;
            h = (h + 1) & (HS - 1);
          }
          if (s >= 0) {
            TAcc yv[BS];
#pragma unroll
            for (int cc = 0; cc < BS; ++cc) yv[cc] = (TAcc)y[qb[cc] + q];
#pragma unroll
            for (int r = 0; r < BS; ++r) {
              TAcc t = sacc[wid][r][s];
#pragma unroll
              for (int cc = 0; cc < BS; ++cc) t = fma(blk[r][cc], yv[cc], t);
              sacc[wid][r][s] = t;
            }
          }
        }
      }
    }
    __syncthreads();
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
      for (int t = 0; t < L; ++t) v[t] = (double)sacc[wid][r][lane + kWave * t];
      const int row = r0 + r;
      if (MODE != kModeEnergy)
        project_row<kWave, L, M1>(v, oc, a.bc, valid ? a.wpk + (long)row * mp : nullptr, a.m,
                                  valid);
      const int pr = valid ? a.prp[row] : 0;
#pragma unroll
      for (int t = 0; t < L; ++t) {
        if (oc[t] < 0) continue;
        const int idx = pr + lane + kWave * t;
        if (MODE == kModeIter) {
          const TO o = (TO)v[t];
          out[idx] = o;
          dot += (double)y[idx] * (double)o;
        } else if (MODE == kModeInit) {
          out[idx] = (TO)(-v[t]);
        } else if (MODE == kModePlain) {
          out[idx] = (TO)v[t];
        } else {
          dot += (double)y[idx] * v[t];
        }
      }
    }
    __syncthreads();
  }
  if (MODE == kModeIter || MODE == kModeEnergy) store_partial(dot, a.part_out);
}


}  // namespace emin
