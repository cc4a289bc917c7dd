// Projected symmetric Gauss-Seidel preconditioner M_2 (Sec. 3.4.1, eq.
// SGS_prec without its second term): Z = Pi (L + D)^{-T} D (L + D)^{-1} R on
// K (Sec. 3, eq. 11blk).  K is block diagonal by columns of P and its block j
// is A(I_j, I_j), so SGS on K is, for every column j at once, a forward and a
// backward Gauss-Seidel sweep over the rows holding j -- matrix-free, with the
// same (row, neighbour, slot) triples as the masked product (Sec. 4).
//
// The sweep order is the rows by colour, then index, with the colours of
// Jones-Plassmann rounds on A's graph (priority of row i: (h(i), i), h the
// 32-bit finalizer of MurmurHash3; a row picked in a round takes the smallest
// colour its earlier-picked neighbours leave free).  Rows of one colour are
// not coupled, so each colour is one launch over all its rows and all their
// columns:
//   forward,  colours 0 .. C-1:  u_i = (r_i - sum_{k: c(k) < c(i)} A_ik u_k) / A_ii
//   backward, colours C-1 .. 0:  z_i = u_i - (sum_{k: c(k) > c(i)} A_ik z_k) / A_ii
// (slot by slot, the neighbour's value at the same column found through the
// masked product's intersection map), then Z = Pi z with <R, Z> partials.
#include "common.hpp"
#include "launch.hpp"
#include "project.hpp"
#include "scalars.hpp"

namespace emin {

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }
static int grid_round(int ntiles, int cap) {
  int g = ntiles < cap ? ntiles : cap;
  g = ((g + kNumXcd - 1) / kNumXcd) * kNumXcd;
  return g < kNumXcd ? kNumXcd : g;
}

// ------------------------------------------------------------- colouring --

// Priority of row i: the MurmurHash3 32-bit finalizer of i in the high half,
// i in the low half (no ties).
__device__ __forceinline__ unsigned long long jp_key(int i) {
  unsigned h = (unsigned)i;
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return ((unsigned long long)h << 32) | (unsigned)i;
}

// Round r: an unpicked row is picked when its priority exceeds that of every
// neighbour unpicked at the start of the round, and takes the smallest
// colour (first fit, below kMaxColours) not held by a neighbour picked in an
// earlier round.  A neighbour picked during this round reads as round -1 or
// r; both count as unpicked, so the outcome does not depend on timing (and a
// picked row has no neighbour picked in the same round).
constexpr int kMaxColours = 256;

__global__ __launch_bounds__(kBlock) void k_jp_round(const int* __restrict__ arp,
                                                    const int* __restrict__ aci, int n, int r,
                                                    int* rnd, int* colour, int* picked) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n || rnd[i] != -1) return;
  const unsigned long long ki = jp_key(i);
  unsigned long long used[kMaxColours / 64] = {};
  bool top = true;
  for (int e = arp[i]; e < arp[i + 1] && top; ++e) {
    const int k = aci[e];
    if (k == i) continue;
    const int rk = rnd[k];
    if ((rk == -1 || rk == r) && jp_key(k) > ki) top = false;
    if (rk >= 0 && rk < r) {
      const int c = colour[k];
#pragma unroll
      for (int w = 0; w < kMaxColours / 64; ++w)
        if ((c >> 6) == w) used[w] |= 1ull << (c & 63);
    }
  }
  if (!top) return;
  int c = kMaxColours;  // kMaxColours: no colour free (reported by the host)
#pragma unroll
  for (int w = kMaxColours / 64 - 1; w >= 0; --w)
    if (~used[w]) c = w * 64 + __builtin_ctzll(~used[w]);
  colour[i] = c;
  rnd[i] = r;
  atomicAdd(picked, 1);
}

// Relation of every entry of A to its row in the sweep order: 1 when the
// neighbour's colour is lower (forward sweep), 2 when higher (backward), 0 on
// the diagonal.
__global__ __launch_bounds__(kBlock) void k_entry_rel(const int* __restrict__ arp,
                                                     const int* __restrict__ aci,
                                                     const int* __restrict__ colour, int n,
                                                     unsigned char* __restrict__ rel) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int ci = colour[i];
  for (int e = arp[i]; e < arp[i + 1]; ++e) {
    const int ck = colour[aci[e]];
    rel[e] = ck < ci ? 1 : ck > ci ? 2 : 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_fill_int(int* p, int n, int v) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_colour_flags(const int* __restrict__ colour, int n,
                                                        int c, int* __restrict__ flags) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) flags[i] = colour[i] == c ? 1 : 0;
}

// rows of colour c, in index order, from the exclusive scan of the flags
__global__ __launch_bounds__(kBlock) void k_colour_scatter(const int* __restrict__ colour, int n,
                                                          int c, const int* __restrict__ pos,
                                                          int base, int* __restrict__ rows) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n && colour[i] == c) rows[base + pos[i]] = i;
}

// ----------------------------------------------------------------- sweeps --

// One colour of a sweep; G lanes per row, lane g owns slots g, g + G, ...
// The row's neighbours are taken U at a time with every load issued
// together (indices past the row clamped, their terms discarded).
template <class T, int G, int L, bool FWD>
__global__ __launch_bounds__(kBlock) void k_sgs_sweep(SgsArgs a) {
  constexpr int ROWS = kBlock / G;
  constexpr int U = 4;
  constexpr unsigned char WANT = FWD ? 1 : 2;
  if (a.st->done) return;
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  const T* __restrict__ av = (const T*)a.av;
  const T* __restrict__ base = FWD ? (const T*)a.x : (const T*)a.u;
  const T* src = FWD ? (const T*)a.u : (const T*)a.z;  // neighbours' new values
  T* out = FWD ? (T*)a.u : (T*)a.z;
  for (int t0 = blockIdx.x; t0 * ROWS < a.nrows; t0 += gridDim.x) {
    const int q = t0 * ROWS + grp;
    if (q >= a.nrows) continue;
    const int i = a.rows[a.row0 + q];
    const int p0 = a.prp[i], l = a.prp[i + 1] - p0;
    const int e0 = a.arp[i], e1 = a.arp[i + 1];
    const unsigned char* __restrict__ mp = a.amap + a.mrp[i];
    T acc[L];
#pragma unroll
    for (int t = 0; t < L; ++t) acc[t] = T(0);
    for (int e = e0; e < e1; e += U) {
      bool use[U];
      T ae[U];
      int q0[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int ee = e + u < e1 ? e + u : e0;
        use[u] = e + u < e1 && a.erel[ee] == WANT;
        ae[u] = av[ee];
        q0[u] = a.aoff[ee];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int nb = (e + u < e1 ? e + u : e0) - e0;
#pragma unroll
        for (int t = 0; t < L; ++t) {
          const int s = lane + G * t;
          const int pos = s < l ? mp[nb * l + s] : 0xFF;
          if (use[u] && pos != 0xFF) acc[t] += ae[u] * src[q0[u] + pos];
        }
      }
    }
    const T d = (T)a.dinv[i];
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int s = lane + G * t;
      if (s >= l) continue;
      const T b = base[p0 + s];
      out[p0 + s] = FWD ? (b - acc[t]) * d : b - acc[t] * d;
    }
  }
}

// Z = Pi z, row by row, and the partials of <R, Z>.
template <class T, int G, int L, bool M1>
__global__ __launch_bounds__(kBlock) void k_sgs_finish(SgsArgs a) {
  constexpr int ROWS = kBlock / G;
  if (a.st->done) return;
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  const T* __restrict__ z = (const T*)a.z;
  const T* __restrict__ R = (const T*)a.x;
  T* __restrict__ Z = (T*)a.Z;
  const int mp = a.m * (a.m + 1) / 2;
  double dot = 0.0;
  for (int t0 = blockIdx.x; t0 * ROWS < a.n; t0 += gridDim.x) {
    const int i = t0 * ROWS + grp;
    const bool valid = i < a.n;
    const int p0 = valid ? a.prp[i] : 0;
    const int l = valid ? a.prp[i + 1] - p0 : 0;
    double v[L];
    int oc[L];
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int s = lane + G * t;
      oc[t] = (s < l) ? a.pci[p0 + s] : -1;
      v[t] = (s < l) ? (double)z[p0 + s] : 0.0;
    }
    project_row<G, L, M1>(v, oc, a.bc, a.wpk + (long)(valid ? i : 0) * mp, a.m, valid);
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int s = lane + G * t;
      if (s >= l) continue;
      const T zv = (T)v[t];
      Z[p0 + s] = zv;
      dot += (double)R[p0 + s] * (double)zv;
    }
  }
  store_partial(dot, a.part_out);
}

// R -= alpha Y_hat, dP += alpha Y (alpha from the masked product's partials);
// the first update only clears dP.  Elementwise over the pattern.
template <class T, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_sgs_update(UpdArgs a, int nnz) {
  if (a.st->done) return;
  double alpha_d = 0.0;
  if (!FIRST && scalars_after_delta(a, &alpha_d)) return;
  const T alpha = (T)alpha_d;
  T* __restrict__ R = (T*)a.R;
  T* __restrict__ dP = (T*)a.dP;
  const T* __restrict__ Y = (const T*)a.Y;
  const T* __restrict__ Yh = (const T*)a.Yh;
  for (int e = blockIdx.x * kBlock + threadIdx.x; e < nnz; e += gridDim.x * kBlock) {
    if (FIRST) {
      dP[e] = T(0);
    } else {
      R[e] = R[e] - alpha * Yh[e];
      dP[e] = dP[e] + alpha * Y[e];
    }
  }
}

// Y = Z + beta Y (beta from <R, Z>; the first direction is Z).
template <class T, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_sgs_direction(UpdArgs a, const void* Zv, int nnz) {
  if (a.st->done) return;
  double beta_d = 0.0;
  if (scalars_after_gamma(a, FIRST, &beta_d)) return;
  const T beta = (T)beta_d;
  const T* __restrict__ Z = (const T*)Zv;
  T* __restrict__ Y = (T*)a.Y;
  for (int e = blockIdx.x * kBlock + threadIdx.x; e < nnz; e += gridDim.x * kBlock)
    Y[e] = FIRST ? Z[e] : Z[e] + beta * Y[e];
}

// ------------------------------------------------------------- launchers --

void launch_fill_int(int* p, int n, int v, hipStream_t s) {
  if (n > 0) k_fill_int<<<cdiv(n, kBlock), kBlock, 0, s>>>(p, n, v);
}

void launch_jp_round(const int* arp, const int* aci, int n, int r, int* rnd, int* colour,
                     int* picked, hipStream_t s) {
  if (n > 0) k_jp_round<<<cdiv(n, kBlock), kBlock, 0, s>>>(arp, aci, n, r, rnd, colour, picked);
}

int sgs_max_colours() { return kMaxColours; }

void launch_entry_rel(const int* arp, const int* aci, const int* colour, int n,
                      unsigned char* rel, hipStream_t s) {
  if (n > 0) k_entry_rel<<<cdiv(n, kBlock), kBlock, 0, s>>>(arp, aci, colour, n, rel);
}

void launch_colour_rows(const int* colour, int n, int c, int* flags, int* pos, int* scan_tmp,
                        int base, int* rows, hipStream_t s) {
  if (n <= 0) return;
  k_colour_flags<<<cdiv(n, kBlock), kBlock, 0, s>>>(colour, n, c, flags);
  launch_exclusive_scan(flags, n, pos, scan_tmp, s);
  k_colour_scatter<<<cdiv(n, kBlock), kBlock, 0, s>>>(colour, n, c, pos, base, rows);
}

template <class T, bool FWD>
static int sweep_go(int G, int L, const SgsArgs& a, int grid_cap, hipStream_t s) {
#define EMIN_SWEEP(GG, LL)                                                                \
  if (G == GG && L == LL) {                                                               \
    k_sgs_sweep<T, GG, LL, FWD><<<grid_round(cdiv(a.nrows, kBlock / GG), grid_cap), kBlock, \
                                  0, s>>>(a);                                             \
    return 0;                                                                             \
  }
  EMIN_SWEEP(1, 1) EMIN_SWEEP(2, 1) EMIN_SWEEP(4, 1) EMIN_SWEEP(8, 1) EMIN_SWEEP(16, 1)
  EMIN_SWEEP(32, 1) EMIN_SWEEP(64, 1) EMIN_SWEEP(64, 2) EMIN_SWEEP(64, 3) EMIN_SWEEP(64, 4)
#undef EMIN_SWEEP
  return -1;
}

int launch_sgs_sweep(int forward, int mixed, int G, int L, const SgsArgs& a, int grid_cap,
                     hipStream_t s) {
  if (a.nrows <= 0) return 0;
  if (mixed) return forward ? sweep_go<float, true>(G, L, a, grid_cap, s)
                            : sweep_go<float, false>(G, L, a, grid_cap, s);
  return forward ? sweep_go<double, true>(G, L, a, grid_cap, s)
                 : sweep_go<double, false>(G, L, a, grid_cap, s);
}

int sgs_finish_grid(int G, int n, int grid_cap) { return grid_round(cdiv(n, kBlock / G), grid_cap); }

template <class T>
static int finish_go(int G, int L, const SgsArgs& a, int grid, hipStream_t s) {
#define EMIN_FINISH(GG, LL)                                                           \
  if (G == GG && L == LL) {                                                           \
    if (a.m == 1) k_sgs_finish<T, GG, LL, true><<<grid, kBlock, 0, s>>>(a);           \
    else k_sgs_finish<T, GG, LL, false><<<grid, kBlock, 0, s>>>(a);                   \
    return 0;                                                                         \
  }
  EMIN_FINISH(1, 1) EMIN_FINISH(2, 1) EMIN_FINISH(4, 1) EMIN_FINISH(8, 1) EMIN_FINISH(16, 1)
  EMIN_FINISH(32, 1) EMIN_FINISH(64, 1) EMIN_FINISH(64, 2) EMIN_FINISH(64, 3)
  EMIN_FINISH(64, 4)
#undef EMIN_FINISH
  return -1;
}

int launch_sgs_finish(int mixed, int G, int L, const SgsArgs& a, int grid_cap, hipStream_t s) {
  if (a.n <= 0) return 0;
  const int grid = sgs_finish_grid(G, a.n, grid_cap);
  return mixed ? finish_go<float>(G, L, a, grid, s) : finish_go<double>(G, L, a, grid, s);
}

int sgs_flat_grid(int nnz, int grid_cap) { return grid_round(cdiv(nnz, kBlock), grid_cap); }

void launch_sgs_update(int first, int mixed, const UpdArgs& a, int nnz, int grid_cap,
                       hipStream_t s) {
  const int g = sgs_flat_grid(nnz, grid_cap);
  if (mixed) {
    if (first) k_sgs_update<float, true><<<g, kBlock, 0, s>>>(a, nnz);
    else k_sgs_update<float, false><<<g, kBlock, 0, s>>>(a, nnz);
  } else {
    if (first) k_sgs_update<double, true><<<g, kBlock, 0, s>>>(a, nnz);
    else k_sgs_update<double, false><<<g, kBlock, 0, s>>>(a, nnz);
  }
}

void launch_sgs_direction(int first, int mixed, const UpdArgs& a, const void* Z, int nnz,
                          int grid_cap, hipStream_t s) {
  const int g = sgs_flat_grid(nnz, grid_cap);
  if (mixed) {
    if (first) k_sgs_direction<float, true><<<g, kBlock, 0, s>>>(a, Z, nnz);
    else k_sgs_direction<float, false><<<g, kBlock, 0, s>>>(a, Z, nnz);
  } else {
    if (first) k_sgs_direction<double, true><<<g, kBlock, 0, s>>>(a, Z, nnz);
    else k_sgs_direction<double, false><<<g, kBlock, 0, s>>>(a, Z, nnz);
  }
}

}  // namespace emin
