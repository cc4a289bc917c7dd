// Symbolic phase: CSR validation and the pattern growth struct(A * T)
// (Sec. 3, eq. enlPatt, applied k times starting from T = struct(P0)).  The
// product is 0/1, so a row of the result is the set union of the rows of T
// selected by the stored columns of A's row.  Two passes over the same
// dedup: count (row sizes) then fill (sorted columns), with a device scan in
// between.
//
// Growth can run in a compressed space and be expanded once at the end:
//  * groups: when every row of P0 is made of whole aligned groups of G
//    columns (aggregation with G modes per aggregate), T is stored as group
//    ids; a union of whole groups is whole groups, so every grown row is too.
//  * nodes: when A is stored as full aligned bs x bs blocks, all bs rows of a
//    node select the same columns, so after one step all rows of a node are
//    equal; one row per node is grown, and from the second step on only the
//    first column of each neighbour block is visited (T row k is node k/bs).
// SymMap carries this: output row o reads A's row o*os, visits every ns-th
// stored entry, and the entry's column k names row k/td of T.
#include "common.hpp"
#include "launch.hpp"

namespace emin {

// ---------------------------------------------------------------- checks --

// G lanes per row: the row's bounds by its first lane, the entries (range,
// strictly increasing) over all G
template <int G>
__global__ __launch_bounds__(kBlock) void k_check_csr(const int* __restrict__ rp,
                                                     const int* __restrict__ ci, int nrows,
                                                     int ncols, int nnz, int* flags, int bit) {
  const int g = threadIdx.x % G;
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  if (i >= nrows) return;
  const int a = rp[i], b = rp[i + 1];
  bool bad = (a < 0) || (b < a) || (b > nnz);
  if (i == 0 && a != 0) bad = true;
  if (i == nrows - 1 && b != nnz) bad = true;
  if (!bad) {
    for (int e = a + g; e < b; e += G) {
      const int c = ci[e];
      if (c < 0 || c >= ncols || (e > a && ci[e - 1] >= c)) { bad = true; break; }
    }
  }
  if (bad) atomicOr(flags, 1 << bit);
}

// every entry of P0 must be present in the pattern (both rows sorted: merge)
__global__ __launch_bounds__(kBlock) void k_check_contains(const int* __restrict__ qrp,
                                                          const int* __restrict__ qci,
                                                          const int* __restrict__ prp,
                                                          const int* __restrict__ pci, int n,
                                                          int* flags, int bit) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int p = prp[i];
  const int pe = prp[i + 1];
  for (int q = qrp[i]; q < qrp[i + 1]; ++q) {
    const int c = qci[q];
    while (p < pe && pci[p] < c) ++p;
    if (p == pe || pci[p] != c) { atomicOr(flags, 1 << bit); return; }
  }
}

// block maximum, then one atomic per block
__device__ __forceinline__ void block_max_atomic(int v, int* out) {
  __shared__ int red[kBlock / kWave];
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = red[0];
#pragma unroll
    for (int w = 1; w < kBlock / kWave; ++w) t = max(t, red[w]);
    atomicMax(out, t);
  }
}

// longest row of a CSR structure (grid-stride: few blocks, few atomics)
__global__ __launch_bounds__(kBlock) void k_row_maxlen(const int* __restrict__ rp, int n,
                                                      int* out) {
  int v = 0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    v = max(v, rp[i + 1] - rp[i]);
  block_max_atomic(v, out);
}

// largest value of an int array (grid-stride)
__global__ __launch_bounds__(kBlock) void k_max_int(const int* __restrict__ p, int n, int* out) {
  int v = 0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) v = max(v, p[i]);
  block_max_atomic(v, out);
}

// ------------------------------------------------------------- symbolic --

// Upper bound on the size of row i of struct(A T): sum of the lengths of the
// rows of T that A's row selects.
__global__ __launch_bounds__(kBlock) void k_sym_ub(const int* __restrict__ arp,
                                                  const int* __restrict__ aci,
                                                  const int* __restrict__ trp, int n,
                                                  SymMap sm, int* __restrict__ maxub) {
  int best = 0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    int s = 0;
    const int ar = i * sm.os;
    for (int e = arp[ar]; e < arp[ar + 1]; e += sm.ns) {
      const int k = aci[e] / sm.td;
      s += trp[k + 1] - trp[k];
    }
    best = max(best, s);
  }
  block_max_atomic(best, maxub);
}

// Small rows: a group of G lanes per row gathers the candidate columns into
// LDS (CAP >= upper bound), marks first occurrences, and ranks the distinct
// values (rank = number of distinct smaller values).  Count pass writes the
// distinct count; fill pass writes the sorted row.
template <int G, int CAP>
__global__ __launch_bounds__(kBlock) void k_sym_small(const int* __restrict__ arp,
                                                     const int* __restrict__ aci,
                                                     const int* __restrict__ trp,
                                                     const int* __restrict__ tci, int n,
                                                     SymMap sm, int* __restrict__ cnt,
                                                     const int* __restrict__ prp,
                                                     int* __restrict__ pci, int fill) {
  constexpr int GROUPS = kBlock / G;
  __shared__ int cand[GROUPS][CAP];
  __shared__ unsigned char first[GROUPS][CAP];
  __shared__ int ncand[GROUPS];
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  const int ntiles = (n + GROUPS - 1) / GROUPS;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int i = w.t * GROUPS + grp;
    const bool valid = i < n;
    if (lane == 0) ncand[grp] = 0;
    __syncthreads();
    if (valid) {
      const int ar = i * sm.os;
      for (int e = arp[ar] + lane * sm.ns; e < arp[ar + 1]; e += G * sm.ns) {
        const int k = aci[e] / sm.td;
        for (int q = trp[k]; q < trp[k + 1]; ++q) {
          const int pos = atomicAdd(&ncand[grp], 1);
          cand[grp][pos] = tci[q];
        }
      }
    }
    __syncthreads();
    const int c = valid ? ncand[grp] : 0;
    int mine = 0;
    for (int x = lane; x < c; x += G) {
      const int v = cand[grp][x];
      unsigned char f = 1;
      for (int y = 0; y < x; ++y)
        if (cand[grp][y] == v) { f = 0; break; }
      first[grp][x] = f;
      mine += f;
    }
    __syncthreads();
    if (fill) {
      if (valid) {
        const int base = prp[i];
        for (int x = lane; x < c; x += G) {
          if (!first[grp][x]) continue;
          const int v = cand[grp][x];
          int rank = 0;
          for (int y = 0; y < c; ++y) rank += (first[grp][y] && cand[grp][y] < v) ? 1 : 0;
          pci[base + rank] = v;
        }
      }
    } else {
      mine = group_sum<G>(mine);
      if (valid && lane == 0) cnt[i] = mine;
    }
    __syncthreads();
  }
}

// Large rows: one wave per row, an open-addressing hash set in LDS (HCAP
// slots, HCAP >= 2 * upper bound), then compaction and a rank sort.  The
// wave takes 64 / W neighbours at a time, W lanes over each one's row of T
// (W a power of two, about the longest row of T).
template <int HCAP>
__global__ __launch_bounds__(kWave) void k_sym_hash(const int* __restrict__ arp,
                                                   const int* __restrict__ aci,
                                                   const int* __restrict__ trp,
                                                   const int* __restrict__ tci, int n,
                                                   SymMap sm, int W, int* __restrict__ cnt,
                                                   const int* __restrict__ prp,
                                                   int* __restrict__ pci, int fill) {
  __shared__ int tab[HCAP];
  __shared__ int uniq[HCAP / 2];
  __shared__ int nuniq;
  const int lane = threadIdx.x;
  const int sub = lane / W, t = lane % W, per = kWave / W;
  for (TileWalk w(n); w.t < w.end; w.t += w.step) {
    const int i = w.t;
    for (int h = lane; h < HCAP; h += kWave) tab[h] = -1;
    if (lane == 0) nuniq = 0;
    __syncthreads();
    const int ar = i * sm.os;
    const int a0 = arp[ar], a1 = arp[ar + 1];
    for (int e = a0 + sub * sm.ns; e < a1; e += per * sm.ns) {
      const int k = aci[e] / sm.td;
      const int q0 = trp[k], q1 = trp[k + 1];
      for (int q = q0 + t; q < q1; q += W) {
        const int v = tci[q];
        unsigned int h = ((unsigned int)v * 2654435761u) & (HCAP - 1);
        while (true) {
          const int old = atomicCAS(&tab[h], -1, v);
          if (old == -1) {
            const int pos = atomicAdd(&nuniq, 1);
            uniq[pos] = v;
            break;
          }
          if (old == v) break;
          h = (h + 1) & (HCAP - 1);
        }
      }
    }
    __syncthreads();
    const int u = nuniq;
    if (fill) {
      const int base = prp[i];
      for (int x = lane; x < u; x += kWave) {
        const int v = uniq[x];
        int rank = 0;
        for (int y = 0; y < u; ++y) rank += (uniq[y] < v) ? 1 : 0;
        pci[base + rank] = v;
      }
    } else if (lane == 0) {
      cnt[i] = u;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ compression --

// P0 in group form: row i keeps every G-th column, divided by G (valid when
// every row is made of whole aligned groups of G columns).
__global__ __launch_bounds__(kBlock) void k_compress_groups(const int* __restrict__ qrp,
                                                           const int* __restrict__ qci, int n,
                                                           int nnzc, int G,
                                                           int* __restrict__ crp,
                                                           int* __restrict__ cci) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e <= n) crp[e] = qrp[e] / G;
  if (e < nnzc) cci[e] = qci[(long)e * G] / G;
}

// Compressed pattern (rows = nodes of R rows when R > 1; entries = groups of
// G columns when G > 1) to the full row pattern.  Node a of length L starts
// at G * R * nrp[a] and each of its R rows holds the same G * L columns.
// One wave per compressed row.
__global__ __launch_bounds__(kBlock) void k_expand_pattern(const int* __restrict__ nrp,
                                                          const int* __restrict__ nci, int nrows,
                                                          int R, int G, int* __restrict__ prp,
                                                          int* __restrict__ pci) {
  const int lane = threadIdx.x % kWave;
  const int a = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  if (a >= nrows) return;
  const int c0 = nrp[a], L = nrp[a + 1] - c0;
  const long base = (long)G * R * c0;
  if (lane < R) prp[(long)a * R + lane] = (int)(base + (long)lane * L * G);
  if (a == nrows - 1 && lane == 0) prp[(long)nrows * R] = (int)(base + (long)R * L * G);
  const int row = L * G;
  for (int x = lane; x < R * row; x += kWave) {
    const int r = x / row, y = x % row;
    pci[base + (long)r * row + y] = nci[c0 + y / G] * G + y % G;
  }
}

// ------------------------------------------------------------------ scan --

constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

// exclusive scan inside each tile of kScanTile counts; tile totals to bsum
__global__ __launch_bounds__(kBlock) void k_scan_tiles(const int* __restrict__ in, int n,
                                                      int* __restrict__ out,
                                                      int* __restrict__ bsum) {
  __shared__ int s[kBlock];
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems];
  int t = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = (base + j < n) ? in[base + j] : 0;
    t += v[j];
  }
  s[threadIdx.x] = t;
  __syncthreads();
  for (int d = 1; d < kBlock; d <<= 1) {
    const int x = (threadIdx.x >= d) ? s[threadIdx.x - d] : 0;
    __syncthreads();
    s[threadIdx.x] += x;
    __syncthreads();
  }
  int run = s[threadIdx.x] - t;  // exclusive prefix of this thread
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == kBlock - 1) bsum[blockIdx.x] = s[kBlock - 1];
}

// exclusive scan of the tile totals (one block, chunked with a carry);
// writes the grand total to *total
__global__ __launch_bounds__(kBlock) void k_scan_top(int* __restrict__ bsum, int nb,
                                                    int* __restrict__ total) {
  __shared__ int s[kBlock];
  int carry = 0;
  for (int c0 = 0; c0 < nb; c0 += kBlock) {
    const int idx = c0 + threadIdx.x;
    const int v = (idx < nb) ? bsum[idx] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < kBlock; d <<= 1) {
      const int x = (threadIdx.x >= d) ? s[threadIdx.x - d] : 0;
      __syncthreads();
      s[threadIdx.x] += x;
      __syncthreads();
    }
    if (idx < nb) bsum[idx] = carry + s[threadIdx.x] - v;
    const int chunk_total = s[kBlock - 1];
    __syncthreads();
    carry += chunk_total;
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_add(int* __restrict__ out, int n,
                                                    const int* __restrict__ bsum,
                                                    const int* __restrict__ total) {
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j)
    if (base + j < n) out[base + j] += bsum[blockIdx.x];
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = *total;
}

// ------------------------------------------------------------- launchers --

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

void launch_check_csr(const int* rp, const int* ci, int nrows, int ncols, int nnz, int* flags,
                      int bit, hipStream_t s) {
  if (nrows <= 0) return;
  // lanes per row from the average row length
  const long avg = (long)nnz / nrows;
  if (avg >= 32)
    k_check_csr<64><<<cdiv((long)nrows * 64, kBlock), kBlock, 0, s>>>(rp, ci, nrows, ncols, nnz,
                                                                      flags, bit);
  else if (avg >= 8)
    k_check_csr<16><<<cdiv((long)nrows * 16, kBlock), kBlock, 0, s>>>(rp, ci, nrows, ncols, nnz,
                                                                      flags, bit);
  else if (avg >= 2)
    k_check_csr<4><<<cdiv((long)nrows * 4, kBlock), kBlock, 0, s>>>(rp, ci, nrows, ncols, nnz,
                                                                    flags, bit);
  else
    k_check_csr<1><<<cdiv(nrows, kBlock), kBlock, 0, s>>>(rp, ci, nrows, ncols, nnz, flags, bit);
}

void launch_check_contains(const int* qrp, const int* qci, const int* prp, const int* pci, int n,
                           int* flags, int bit, hipStream_t s) {
  if (n <= 0) return;
  k_check_contains<<<cdiv(n, kBlock), kBlock, 0, s>>>(qrp, qci, prp, pci, n, flags, bit);
}

static int small_grid(int n) { const int b = cdiv(n, kBlock); return b < 256 ? b : 256; }

void launch_max_int(const int* p, int n, int* out, hipStream_t s) {
  if (n <= 0) return;
  k_max_int<<<small_grid(n), kBlock, 0, s>>>(p, n, out);
}

void launch_row_maxlen(const int* rp, int n, int* out, hipStream_t s) {
  if (n <= 0) return;
  k_row_maxlen<<<small_grid(n), kBlock, 0, s>>>(rp, n, out);
}

void launch_sym_ub(const int* arp, const int* aci, const int* trp, int n, SymMap sm,
                   int* maxub, hipStream_t s) {
  if (n <= 0) return;
  k_sym_ub<<<small_grid(n), kBlock, 0, s>>>(arp, aci, trp, n, sm, maxub);
}

void launch_compress_groups(const int* qrp, const int* qci, int n, int nnzc, int G, int* crp,
                            int* cci, hipStream_t s) {
  const int m = (n + 1 > nnzc ? n + 1 : nnzc);
  k_compress_groups<<<cdiv(m, kBlock), kBlock, 0, s>>>(qrp, qci, n, nnzc, G, crp, cci);
}

void launch_expand_pattern(const int* nrp, const int* nci, int nrows, int R, int G, int* prp,
                           int* pci, hipStream_t s) {
  if (nrows <= 0) return;
  k_expand_pattern<<<cdiv(nrows, kBlock / kWave), kBlock, 0, s>>>(nrp, nci, nrows, R, G, prp,
                                                                  pci);
}

static int grid_for(int ntiles, int cap) {
  int g = ntiles < cap ? ntiles : cap;
  g = ((g + kNumXcd - 1) / kNumXcd) * kNumXcd;
  return g < kNumXcd ? kNumXcd : g;
}

int launch_sym_rows(const int* arp, const int* aci, const int* trp, const int* tci, int n,
                    SymMap sm, int maxub, int tmax, int* cnt, const int* prp, int* pci,
                    int fill, int grid_cap, hipStream_t s) {
  if (n <= 0) return 0;
  // lanes per neighbour in the hash kernel: about the longest row of T
  int W = 1;
  while (W < tmax && W < kWave) W <<= 1;
  if (maxub <= 32) {
    constexpr int G = 8;
    k_sym_small<G, 32><<<grid_for(cdiv(n, kBlock / G), grid_cap), kBlock, 0, s>>>(
        arp, aci, trp, tci, n, sm, cnt, prp, pci, fill);
  } else if (maxub <= 128) {
    constexpr int G = 16;
    k_sym_small<G, 128><<<grid_for(cdiv(n, kBlock / G), grid_cap), kBlock, 0, s>>>(
        arp, aci, trp, tci, n, sm, cnt, prp, pci, fill);
  } else if (maxub <= 512) {
    k_sym_hash<1024><<<grid_for(n, grid_cap * 4), kWave, 0, s>>>(arp, aci, trp, tci, n, sm, W,
                                                                 cnt, prp, pci, fill);
  } else if (maxub <= 2048) {
    k_sym_hash<4096><<<grid_for(n, grid_cap * 4), kWave, 0, s>>>(arp, aci, trp, tci, n, sm, W,
                                                                 cnt, prp, pci, fill);
  } else if (maxub <= 4096) {
    k_sym_hash<8192><<<grid_for(n, grid_cap * 4), kWave, 0, s>>>(arp, aci, trp, tci, n, sm, W,
                                                                 cnt, prp, pci, fill);
  } else {
    return -1;  // row of the grown pattern may exceed the LDS hash capacity
  }
  return 0;
}

int scan_tmp_ints(int n) { return cdiv(n, kScanTile) + 1; }

void launch_exclusive_scan(const int* cnt, int n, int* out, int* tmp, hipStream_t s) {
  const int nb = cdiv(n, kScanTile);
  int* bsum = tmp;
  int* total = tmp + nb;
  if (n > 0) k_scan_tiles<<<nb, kBlock, 0, s>>>(cnt, n, out, bsum);
  k_scan_top<<<1, kBlock, 0, s>>>(bsum, nb, total);
  k_scan_add<<<nb > 0 ? nb : 1, kBlock, 0, s>>>(out, n, bsum, total);
}

}  // namespace emin
