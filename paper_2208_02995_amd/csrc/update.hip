// Vector phases of Alg. 3 around the masked product.
//
//  update    (after <Y, Y_hat>):  dP += alpha Y,  R -= alpha Y_hat,
//            Z = Pi M^{-1} R,  partial <R, Z>   -> gamma, beta, stop tests
//  direction (after gamma):       Y = Z + beta Y  (Z recomputed from R, so it
//            is never stored: one P-sized stream fewer per iteration)
//
// Jacobi (Sec. 3.4.1, M_1): Z = R / A(i,i) row by row; the Pi after M^{-1}
// is dropped because the row scaling keeps R inside the range of Pi
// (Corollary 3.2).  Block-Jacobi: per node of bs rows sharing a pattern row,
// Z(node, j) = A_aa^{-1} R(node, j).  The Pi after it is dropped as well:
// the bs rows of a node share one pattern row, hence one projector Pi_J, so
// on the node's bs x l block Pi acts as I (x) Pi_J while the block inverse
// acts as A_aa^{-1} (x) I; the two commute and R is already in range(Pi).
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

// ---------------------------------------------------------- Jacobi rows --

template <class T, int G, int L, bool FIRST, bool SEG>
__global__ __launch_bounds__(kBlock) void k_update_jac(UpdArgs a) {
  constexpr int ROWS = kBlock / G;
  if (!SEG && a.st->done) return;
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  T* __restrict__ R = (T*)a.R;
  T* __restrict__ dP = (T*)a.dP;
  const T* __restrict__ Y = (const T*)a.Y;
  const T* __restrict__ Yh = (const T*)a.Yh;
  double alpha_d = 0.0;
  if (!SEG && !FIRST && scalars_after_delta(a, &alpha_d)) return;
  T alpha = (T)alpha_d;
  double dot = 0.0;
  const int ntiles = (a.n + ROWS - 1) / ROWS;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int i = w.t * ROWS + grp;
    if (i >= a.n) continue;
    if (SEG) {
      const SegState& sg = a.segs[a.row_seg ? a.row_seg[i] : find_seg(a.seg_row, a.nseg, i)];
      if (sg.stop) continue;
      alpha = (T)sg.alpha;
    }
    const int p0 = a.prp[i];
    const int l = a.prp[i + 1] - p0;
    const T d = (T)a.dinv[i];
    double rdot = 0.0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int s = lane + G * t;
      if (s >= l) continue;
      const int idx = p0 + s;
      T r;
      if (FIRST) {
        r = R[idx];
        dP[idx] = T(0);
      } else {
        r = R[idx] - alpha * Yh[idx];
        dP[idx] = dP[idx] + alpha * Y[idx];
        R[idx] = r;
      }
      const T z = r * d;
      rdot += (double)r * (double)z;
    }
    if (SEG) {
      rdot = group_sum<G>(rdot);
      if (lane == 0) a.rowdot[i] = rdot;
    } else {
      dot += rdot;
    }
  }
  if (!SEG) store_partial(dot, a.part_out);
}

template <class T, int G, int L, bool FIRST, bool SEG>
__global__ __launch_bounds__(kBlock) void k_direction_jac(UpdArgs a) {
  constexpr int ROWS = kBlock / G;
  if (!SEG && a.st->done) return;
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  const T* __restrict__ R = (const T*)a.R;
  T* __restrict__ Y = (T*)a.Y;
  double beta_d = 0.0;
  if (!SEG && scalars_after_gamma(a, FIRST, &beta_d)) return;
  T beta = (T)beta_d;
  const int ntiles = (a.n + ROWS - 1) / ROWS;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int i = w.t * ROWS + grp;
    if (i >= a.n) continue;
    if (SEG) {
      const SegState& sg = a.segs[a.row_seg ? a.row_seg[i] : find_seg(a.seg_row, a.nseg, i)];
      if (sg.stop) continue;
      beta = (T)sg.beta;
    }
    const int p0 = a.prp[i];
    const int l = a.prp[i + 1] - p0;
    const T d = (T)a.dinv[i];
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int s = lane + G * t;
      if (s >= l) continue;
      const int idx = p0 + s;
      const T z = R[idx] * d;
      Y[idx] = FIRST ? z : z + beta * Y[idx];
    }
  }
}

// ------------------------------------------------- Jacobi, lane per row --
// Short, uneven rows: one lane owns a row and walks it in chunks of four
// entries, each chunk of each stream read in 16-byte loads (reads may run
// up to three entries past the row; every library buffer has slack for it)
// and written in at most two stores (a whole chunk, else a pair and a
// single, never past the row's end).  Consecutive lanes hold consecutive rows, so the
// loads of a wave cover one contiguous stretch of each stream.

template <class T>
struct __attribute__((aligned(sizeof(T)))) Chunk4 {
  T v[4];
};

template <class T>
__device__ __forceinline__ Chunk4<T> ld4(const T* p) {
  return *reinterpret_cast<const Chunk4<T>*>(p);
}

template <class T>
struct __attribute__((aligned(sizeof(T)))) Chunk2 {
  T v[2];
};

// The first rem (>= 1) entries of v to p: a whole chunk in one store, else
// a pair and a single (nothing past p[rem - 1] is written: the entries after
// a row's end belong to the next row's lane).
template <class T>
__device__ __forceinline__ void st_part(T* p, const T (&v)[4], int rem) {
  if (rem >= 4) {
    Chunk4<T> c;
#pragma unroll
    for (int k = 0; k < 4; ++k) c.v[k] = v[k];
    *reinterpret_cast<Chunk4<T>*>(p) = c;
    return;
  }
  if (rem & 2) {
    Chunk2<T> c;
    c.v[0] = v[0];
    c.v[1] = v[1];
    *reinterpret_cast<Chunk2<T>*>(p) = c;
  }
  if (rem & 1) p[rem - 1] = rem == 3 ? v[2] : v[0];
}

template <class T, bool FIRST, bool SEG>
__global__ __launch_bounds__(kBlock) void k_update_row(UpdArgs a) {
  if (!SEG && a.st->done) return;
  T* __restrict__ R = (T*)a.R;
  T* __restrict__ dP = (T*)a.dP;
  const T* __restrict__ Y = (const T*)a.Y;
  const T* __restrict__ Yh = (const T*)a.Yh;
  double alpha_d = 0.0;
  if (!SEG && !FIRST && scalars_after_delta(a, &alpha_d)) return;
  T alpha = (T)alpha_d;
  double dot = 0.0;
  const int ntiles = (a.n + kBlock - 1) / kBlock;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int i = w.t * kBlock + threadIdx.x;
    if (i >= a.n) continue;
    if (SEG) {
      const SegState& sg = a.segs[a.row_seg[i]];
      if (sg.stop) continue;
      alpha = (T)sg.alpha;
    }
    const int p0 = a.prp[i];
    const int l = a.prp[i + 1] - p0;
    const T d = (T)a.dinv[i];
    double rdot = 0.0;
    for (int j = 0; j < l; j += 4) {
      const Chunk4<T> r4 = ld4(R + p0 + j);
      Chunk4<T> h4, y4, q4;
      if (!FIRST) {
        h4 = ld4(Yh + p0 + j);
        y4 = ld4(Y + p0 + j);
        q4 = ld4(dP + p0 + j);
      }
      const int rem = l - j;
      T rn[4], pn[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        T r = r4.v[k];
        if (FIRST) {
          pn[k] = T(0);
        } else {
          r = r - alpha * h4.v[k];
          pn[k] = q4.v[k] + alpha * y4.v[k];
        }
        rn[k] = r;
        const T z = r * d;
        if (k < rem) rdot += (double)r * (double)z;
      }
      st_part(dP + p0 + j, pn, rem);
      if (!FIRST) st_part(R + p0 + j, rn, rem);
    }
    if (SEG) a.rowdot[i] = rdot;
    else dot += rdot;
  }
  if (!SEG) store_partial(dot, a.part_out);
}

template <class T, bool FIRST, bool SEG>
__global__ __launch_bounds__(kBlock) void k_direction_row(UpdArgs a) {
  if (!SEG && a.st->done) return;
  const T* __restrict__ R = (const T*)a.R;
  T* __restrict__ Y = (T*)a.Y;
  double beta_d = 0.0;
  if (!SEG && scalars_after_gamma(a, FIRST, &beta_d)) return;
  T beta = (T)beta_d;
  const int ntiles = (a.n + kBlock - 1) / kBlock;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int i = w.t * kBlock + threadIdx.x;
    if (i >= a.n) continue;
    if (SEG) {
      const SegState& sg = a.segs[a.row_seg[i]];
      if (sg.stop) continue;
      beta = (T)sg.beta;
    }
    const int p0 = a.prp[i];
    const int l = a.prp[i + 1] - p0;
    const T d = (T)a.dinv[i];
    for (int j = 0; j < l; j += 4) {
      const Chunk4<T> r4 = ld4(R + p0 + j);
      Chunk4<T> y4;
      if (!FIRST) y4 = ld4(Y + p0 + j);
      T yn[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const T z = r4.v[k] * d;
        yn[k] = FIRST ? z : z + beta * y4.v[k];
      }
      st_part(Y + p0 + j, yn, l - j);
    }
  }
}

// ------------------------------------------------------ block-Jacobi nodes --

// Z for one node: the block inverse applied per pattern column (no Pi: it
// commutes with the block inverse, see the top of this file).
template <class T, int BS, int L>
__device__ __forceinline__ void node_precond(const UpdArgs& a, int node,
                                             const double (&r)[BS][L], double (&z)[BS][L]) {
  Uniform<double>* binv = (Uniform<double>*)(a.binv + (long)node * BS * BS);
  double inv[BS][BS];
#pragma unroll
  for (int x = 0; x < BS; ++x)
#pragma unroll
    for (int c = 0; c < BS; ++c) inv[x][c] = binv[x * BS + c];
#pragma unroll
  for (int t = 0; t < L; ++t)
#pragma unroll
    for (int x = 0; x < BS; ++x) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < BS; ++c) s += inv[x][c] * r[c][t];
      z[x][t] = s;
    }
}

// V consecutive values of one row at p (V = 1, or 2 with p 2V-element aligned:
// one 16-byte FP64 / 8-byte FP32 access).
template <class T, int V>
__device__ __forceinline__ void ldv(const T* p, T* v) {
  if constexpr (V == 1) {
    v[0] = p[0];
  } else {
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 q = *reinterpret_cast<const v2*>(p);
    v[0] = q.x;
    v[1] = q.y;
  }
}
template <class T, int V>
__device__ __forceinline__ void stv(T* p, const T* v) {
  if constexpr (V == 1) {
    p[0] = v[0];
  } else {
    typedef T v2 __attribute__((ext_vector_type(2)));
    v2 q;
    q.x = v[0];
    q.y = v[1];
    *reinterpret_cast<v2*>(p) = q;
  }
}

// One node per wave.  A lane owns V consecutive slots per chunk: slots
// s = V (lane + 64 t) .. + V - 1 of every row of the node, held in register
// slots u = t V + j (V = 2 needs even pattern rows, so a pair never straddles
// a row end).  Lanes beyond the row read slot 0 of each row (every load is
// issued before any is used) and only the stores are masked; a node with an
// empty pattern row is skipped whole.
//
// PM != 0: Y_hat (or, in the first update, the initial residual's K P0')
// arrives without the projector (the node product leaves it out) and is
// projected here as it is read.  PM = 3 or 6: the node's rows
// are projected together with m = PM (B_c 16-byte aligned when PM is even);
// PM = -1: row by row for any m.
template <class T, int BS, int L, bool FIRST, int PM, int V>
__global__ __launch_bounds__(kBlock) void k_update_node(UpdArgs a) {
  constexpr int WPB = kBlock / kWave;
  constexpr int LV = L * V;
  if (a.st->done) return;
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  T* __restrict__ R = (T*)a.R;
  T* __restrict__ dP = (T*)a.dP;
  const T* __restrict__ Y = (const T*)a.Y;
  const T* __restrict__ Yh = (const T*)a.Yh;
  Uniform<int>* uprp = (Uniform<int>*)a.prp;
  double alpha_d = 0.0;
  if (!FIRST && scalars_after_delta(a, &alpha_d)) return;
  const T alpha = (T)alpha_d;
  const int nnodes = a.n / BS;
  double dot = 0.0;
  const int ntiles = (nnodes + WPB - 1) / WPB;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int node = __builtin_amdgcn_readfirstlane(w.t * WPB + wid);
    if (node >= nnodes) continue;
    const int r0 = node * BS;
    int pr[BS];
#pragma unroll
    for (int x = 0; x < BS; ++x) pr[x] = uprp[r0 + x];
    const int l = uprp[r0 + 1] - pr[0];
    if (l == 0) continue;
    bool on[LV];
    int so[LV];
#pragma unroll
    for (int t = 0; t < L; ++t)
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const int s0 = V * (lane + kWave * t);
        on[t * V + j] = s0 < l;
        so[t * V + j] = (s0 < l ? s0 : 0) + j;
      }
    T rv[BS][LV], hv[BS][LV], yv[BS][LV], pv[BS][LV];
    if constexpr (PM != 0 && FIRST) {
      // the raw mask(A P0') arrives in R (or, FP64, in r0raw for the mixed
      // form): R = -Pi of it, rounded once; dP = 0, Z, <R, Z>
      const int mp = a.m * (a.m + 1) / 2;
      int oc[LV];
#pragma unroll
      for (int u = 0; u < LV; ++u) oc[u] = a.pci[pr[0] + so[u]];
      double v[BS][LV];
#pragma unroll
      for (int x = 0; x < BS; ++x)
#pragma unroll
        for (int u = 0; u < LV; u += V) {
          if (a.r0raw) {
            double h[V];
            ldv<double, V>(a.r0raw + pr[x] + so[u], h);
#pragma unroll
            for (int j = 0; j < V; ++j) v[x][u + j] = on[u] ? h[j] : 0.0;
          } else {
            T h[V];
            ldv<T, V>(R + pr[x] + so[u], h);
#pragma unroll
            for (int j = 0; j < V; ++j) v[x][u + j] = on[u] ? (double)h[j] : 0.0;
          }
        }
      if constexpr (PM > 0) {
        project_node<LV, (PM > 0 ? PM : 1), BS>(v, oc, a.bc, a.wpk + (long)r0 * mp, lane);
      } else {
        int ocm[LV];
#pragma unroll
        for (int u = 0; u < LV; ++u) ocm[u] = on[u] ? oc[u] : -1;
#pragma unroll
        for (int x = 0; x < BS; ++x)
          project_row<kWave, LV>(v[x], ocm, a.bc, a.wpk + (long)(r0 + x) * mp, a.m, true);
      }
      double r[BS][LV], z[BS][LV];
#pragma unroll
      for (int x = 0; x < BS; ++x)
#pragma unroll
        for (int u = 0; u < LV; u += V) {
          T rn[V], zero[V];
#pragma unroll
          for (int j = 0; j < V; ++j) {
            rn[j] = (T)(-v[x][u + j]);
            zero[j] = T(0);
            r[x][u + j] = on[u] ? (double)rn[j] : 0.0;
          }
          if (on[u]) {
            const int idx = pr[x] + so[u];
            stv<T, V>(R + idx, rn);
            stv<T, V>(dP + idx, zero);
          }
        }
      node_precond<T, BS, LV>(a, node, r, z);
#pragma unroll
      for (int x = 0; x < BS; ++x)
#pragma unroll
        for (int u = 0; u < LV; ++u)
          if (on[u]) dot += r[x][u] * (double)(T)z[x][u];
      continue;
    }
    if constexpr (PM != 0 && !FIRST) {
      // Y_hat = Pi mask(A Y); the node's rows share the pattern row.  Y_hat
      // is projected before the other streams are read (fewer registers).
      const int mp = a.m * (a.m + 1) / 2;
      int oc[LV];
#pragma unroll
      for (int u = 0; u < LV; ++u) oc[u] = a.pci[pr[0] + so[u]];
      double yh[BS][LV];
#pragma unroll
      for (int x = 0; x < BS; ++x)
#pragma unroll
        for (int u = 0; u < LV; u += V) {
          T h[V];
          ldv<T, V>(Yh + pr[x] + so[u], h);
#pragma unroll
          for (int j = 0; j < V; ++j) yh[x][u + j] = on[u] ? (double)h[j] : 0.0;
        }
      if constexpr (PM > 0) {
        project_node<LV, (PM > 0 ? PM : 1), BS>(yh, oc, a.bc, a.wpk + (long)r0 * mp, lane);
      } else {
        int ocm[LV];
#pragma unroll
        for (int u = 0; u < LV; ++u) ocm[u] = on[u] ? oc[u] : -1;
#pragma unroll
        for (int x = 0; x < BS; ++x)
          project_row<kWave, LV>(yh[x], ocm, a.bc, a.wpk + (long)(r0 + x) * mp, a.m, true);
      }
#pragma unroll
      for (int x = 0; x < BS; ++x)
#pragma unroll
        for (int u = 0; u < LV; ++u) hv[x][u] = (T)yh[x][u];
      // keep the loads below from being hoisted into the projection
      __builtin_amdgcn_sched_barrier(0);
      // R -= alpha Pi Y_hat, Z, <R, Z>; then, as a phase of its own (fewer
      // registers live at once), dP += alpha Y
      double r[BS][LV], z[BS][LV];
#pragma unroll
      for (int x = 0; x < BS; ++x)
#pragma unroll
        for (int u = 0; u < LV; u += V) {
          const int idx = pr[x] + so[u];
          T ro[V], rn[V];
          ldv<T, V>(R + idx, ro);
#pragma unroll
          for (int j = 0; j < V; ++j) {
            rn[j] = ro[j] - alpha * hv[x][u + j];
            r[x][u + j] = on[u] ? (double)rn[j] : 0.0;
          }
          if (on[u]) stv<T, V>(R + idx, rn);
        }
      node_precond<T, BS, LV>(a, node, r, z);
#pragma unroll
      for (int x = 0; x < BS; ++x)
#pragma unroll
        for (int u = 0; u < LV; ++u)
          if (on[u]) dot += r[x][u] * (double)(T)z[x][u];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int x = 0; x < BS; ++x)
#pragma unroll
        for (int u = 0; u < LV; u += V) {
          const int idx = pr[x] + so[u];
          T po[V], yo[V], nv[V];
          ldv<T, V>(dP + idx, po);
          ldv<T, V>(Y + idx, yo);
#pragma unroll
          for (int j = 0; j < V; ++j) nv[j] = po[j] + alpha * yo[j];
          if (on[u]) stv<T, V>(dP + idx, nv);
        }
      continue;
    }
#pragma unroll
    for (int x = 0; x < BS; ++x)
#pragma unroll
      for (int u = 0; u < LV; u += V) {
        const int idx = pr[x] + so[u];
        ldv<T, V>(R + idx, &rv[x][u]);
        if (!FIRST) {
          if (PM == 0) ldv<T, V>(Yh + idx, &hv[x][u]);
          ldv<T, V>(Y + idx, &yv[x][u]);
          ldv<T, V>(dP + idx, &pv[x][u]);
        }
      }
    double r[BS][LV], z[BS][LV];
#pragma unroll
    for (int x = 0; x < BS; ++x)
#pragma unroll
      for (int u = 0; u < LV; u += V) {
        T rn[V], nd[V];
#pragma unroll
        for (int j = 0; j < V; ++j) {
          rn[j] = FIRST ? rv[x][u + j] : rv[x][u + j] - alpha * hv[x][u + j];
          nd[j] = FIRST ? T(0) : pv[x][u + j] + alpha * yv[x][u + j];
          r[x][u + j] = on[u] ? (double)rn[j] : 0.0;
        }
        if (on[u]) {
          const int idx = pr[x] + so[u];
          stv<T, V>(dP + idx, nd);
          if (!FIRST) stv<T, V>(R + idx, rn);
        }
      }
    node_precond<T, BS, LV>(a, node, r, z);
#pragma unroll
    for (int x = 0; x < BS; ++x)
#pragma unroll
      for (int u = 0; u < LV; ++u)
        if (on[u]) dot += r[x][u] * (double)(T)z[x][u];
  }
  store_partial(dot, a.part_out);
}

template <class T, int BS, int L, bool FIRST, int V>
__global__ __launch_bounds__(kBlock) void k_direction_node(UpdArgs a) {
  constexpr int WPB = kBlock / kWave;
  constexpr int LV = L * V;
  if (a.st->done) return;
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  const T* __restrict__ R = (const T*)a.R;
  T* __restrict__ Y = (T*)a.Y;
  Uniform<int>* uprp = (Uniform<int>*)a.prp;
  double beta_d = 0.0;
  if (scalars_after_gamma(a, FIRST, &beta_d)) return;
  const T beta = (T)beta_d;
  const int nnodes = a.n / BS;
  const int ntiles = (nnodes + WPB - 1) / WPB;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int node = __builtin_amdgcn_readfirstlane(w.t * WPB + wid);
    if (node >= nnodes) continue;
    const int r0 = node * BS;
    int pr[BS];
#pragma unroll
    for (int x = 0; x < BS; ++x) pr[x] = uprp[r0 + x];
    const int l = uprp[r0 + 1] - pr[0];
    if (l == 0) continue;
    bool on[LV];
    int so[LV];
#pragma unroll
    for (int t = 0; t < L; ++t)
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const int s0 = V * (lane + kWave * t);
        on[t * V + j] = s0 < l;
        so[t * V + j] = (s0 < l ? s0 : 0) + j;
      }
    double r[BS][LV], z[BS][LV];
    T yo[BS][LV];
#pragma unroll
    for (int x = 0; x < BS; ++x)
#pragma unroll
      for (int u = 0; u < LV; u += V) {
        const int idx = pr[x] + so[u];
        T rv[V];
        ldv<T, V>(R + idx, rv);
#pragma unroll
        for (int j = 0; j < V; ++j) r[x][u + j] = on[u] ? (double)rv[j] : 0.0;
        if (!FIRST) ldv<T, V>(Y + idx, &yo[x][u]);
      }
    node_precond<T, BS, LV>(a, node, r, z);
#pragma unroll
    for (int x = 0; x < BS; ++x)
#pragma unroll
      for (int u = 0; u < LV; u += V) {
        if (!on[u]) continue;
        T nv[V];
#pragma unroll
        for (int j = 0; j < V; ++j) {
          const T zv = (T)z[x][u + j];
          nv[j] = FIRST ? zv : zv + beta * yo[x][u + j];
        }
        stv<T, V>(Y + pr[x] + so[u], nv);
      }
  }
}

// ------------------------------------------------ slot-pair node kernels --
//
// For patterns of whole even-sized column groups (the node-pair product): a
// lane owns the slot pair s = 2 (lane + 64 t), s + 1 of every row of the
// node, accessed with one 16-byte (FP64) or 8-byte (FP32) load per row, and
// the chunks t run in a loop, so registers do not grow with the row length.
// The projector (Y_hat arrives without it) needs sums over the whole row:
// first G^T y_hat for all BS rows, one wave reduction, then y_hat - G W G^T
// y_hat.  A node of one chunk does it in one round trip (its update streams
// requested with Y_hat, Y_hat kept in registers, the B_c rows in LDS);
// longer rows take two passes over the chunks, the second reloading the
// (cache-resident) chunk.  PM = 3 or 6: the rows share G and W (m = PM);
// PM = -1: any m, each row with its own W.  The direction step runs over the
// product's windows of 64 slot pairs (it needs no row sums).

// B_c's rows of the pair's two columns c, c + 1 (consecutive in a group).
template <int M>
__device__ __forceinline__ void load_bc_pair(const double* __restrict__ bc, int c, int m,
                                             double (&g0)[M], double (&g1)[M]) {
  if constexpr (M == 3 || M == 6) {
    load_bc_row<M>(bc, c, g0);
    load_bc_row<M>(bc, c + 1, g1);
  } else {
#pragma unroll
    for (int x = 0; x < M; ++x) {
      g0[x] = x < m ? bc[(long)c * m + x] : 0.0;
      g1[x] = x < m ? bc[(long)(c + 1) * m + x] : 0.0;
    }
  }
}

template <class T, int BS, bool FIRST, int PM>
__global__ __launch_bounds__(kBlock) void k_update_pair(UpdArgs a) {
  static_assert(PM != 0, "the pair update projects Y_hat");
  constexpr int WPB = kBlock / kWave;
  constexpr int M = PM > 0 ? PM : kMaxM;  // register width of the constraint
  // a one-chunk node keeps each lane's B_c rows from pass 1 for pass 2 here
  // (their reload cost as many loads as the update's own data streams)
  __shared__ double sG[WPB][kWave][2 * M];
  if (a.st->done) return;
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  T* __restrict__ R = (T*)a.R;
  T* __restrict__ dP = (T*)a.dP;
  const T* __restrict__ Y = (const T*)a.Y;
  const T* __restrict__ Yh = (const T*)a.Yh;
  Uniform<int>* uprp = (Uniform<int>*)a.prp;
  double alpha_d = 0.0;
  if (!FIRST && scalars_after_delta(a, &alpha_d)) return;
  const T alpha = (T)alpha_d;
  const int m = PM > 0 ? PM : a.m;
  const int mp = m * (m + 1) / 2;
  const int nnodes = a.n / BS;
  double dot = 0.0;
  const int ntiles = (nnodes + WPB - 1) / WPB;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int node = __builtin_amdgcn_readfirstlane(w.t * WPB + wid);
    if (node >= nnodes) continue;
    const int r0 = node * BS;
    int pr[BS];
#pragma unroll
    for (int x = 0; x < BS; ++x) pr[x] = uprp[r0 + x];
    const int l = uprp[r0 + 1] - pr[0];
    if (l == 0) continue;
    const int nch = (l / 2 + kWave - 1) / kWave;
    // the chunk's projected-from values: Y_hat, or in the first update the
    // raw K P0' (FP64 in r0raw for the mixed form, else in R); zeros off the row
    auto load_h = [&](int s, bool on, double (&v)[BS][2]) {
#pragma unroll
      for (int x = 0; x < BS; ++x) {
        const int idx = pr[x] + (on ? s : 0);
        if (FIRST && a.r0raw) {
          double h[2];
          ldv<double, 2>(a.r0raw + idx, h);
          v[x][0] = on ? h[0] : 0.0;
          v[x][1] = on ? h[1] : 0.0;
        } else {
          T h[2];
          ldv<T, 2>((FIRST ? (const T*)R : Yh) + idx, h);
          v[x][0] = on ? (double)h[0] : 0.0;
          v[x][1] = on ? (double)h[1] : 0.0;
        }
      }
    };
    // One chunk: one round trip per node.  The update's own streams (R, dP,
    // Y; none in the first update) do not depend on the row sums, so they are
    // requested with Y_hat and the B_c rows, and arrive while the wave
    // reduces; Y_hat stays in registers and the B_c rows in LDS.
    if (nch == 1) {
      const int s = 2 * lane;
      const bool on = s < l;
      const int so = on ? s : 0;
      double v[BS][2];
      load_h(s, on, v);
      double g0[M], g1[M];
      load_bc_pair<M>(a.bc, a.pci[pr[0] + so], m, g0, g1);
      T ro[BS][2], po[BS][2], yo[BS][2];
      if constexpr (!FIRST) {
#pragma unroll
        for (int x = 0; x < BS; ++x) {
          ldv<T, 2>(R + pr[x] + so, ro[x]);
          ldv<T, 2>(dP + pr[x] + so, po[x]);
          ldv<T, 2>(Y + pr[x] + so, yo[x]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);  // all of the node's loads in flight
      double cs[BS * M];
#pragma unroll
      for (int x = 0; x < BS; ++x)
#pragma unroll
        for (int c = 0; c < M; ++c) cs[x * M + c] = g0[c] * v[x][0] + g1[c] * v[x][1];
#pragma unroll
      for (int c = 0; c < M; ++c) {
        sG[wid][lane][c] = g0[c];
        sG[wid][lane][M + c] = g1[c];
      }
      double tot[BS * M];
      wave_sums<BS * M>(cs, tot, lane);
      double d[BS][M];
#pragma unroll
      for (int x = 0; x < BS; ++x) {
        Uniform<double>* uw = (Uniform<double>*)(a.wpk + (long)(PM > 0 ? r0 : r0 + x) * mp);
#pragma unroll
        for (int c = 0; c < M; ++c) {
          double t = 0.0;
#pragma unroll
          for (int e = 0; e < M; ++e)
            if (c < m && e < m)
              t += uw[(c <= e) ? packed_idx(c, e, m) : packed_idx(e, c, m)] * tot[x * M + e];
          d[x][c] = -t;
        }
      }
      Uniform<double>* binv1 = (Uniform<double>*)(a.binv + (long)node * BS * BS);
#pragma unroll
      for (int c = 0; c < M; ++c) {  // the lane's own LDS writes (in order)
        g0[c] = sG[wid][lane][c];
        g1[c] = sG[wid][lane][M + c];
      }
      double r[BS][2];
#pragma unroll
      for (int x = 0; x < BS; ++x) {
#pragma unroll
        for (int c = 0; c < M; ++c) {
          v[x][0] += g0[c] * d[x][c];
          v[x][1] += g1[c] * d[x][c];
        }
        T rn[2];
        if constexpr (FIRST) {
          rn[0] = (T)(-v[x][0]);
          rn[1] = (T)(-v[x][1]);
        } else {
          rn[0] = ro[x][0] - alpha * (T)v[x][0];
          rn[1] = ro[x][1] - alpha * (T)v[x][1];
        }
        r[x][0] = on ? (double)rn[0] : 0.0;
        r[x][1] = on ? (double)rn[1] : 0.0;
        if (on) stv<T, 2>(R + pr[x] + s, rn);
      }
#pragma unroll
      for (int x = 0; x < BS; ++x)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          double z = 0.0;
#pragma unroll
          for (int c = 0; c < BS; ++c) z += binv1[x * BS + c] * r[c][j];
          dot += r[x][j] * (double)(T)z;
        }
#pragma unroll
      for (int x = 0; x < BS; ++x) {
        T nv[2];
        if constexpr (FIRST) {
          nv[0] = nv[1] = T(0);
        } else {
          nv[0] = po[x][0] + alpha * yo[x][0];
          nv[1] = po[x][1] + alpha * yo[x][1];
        }
        if (on) stv<T, 2>(dP + pr[x] + s, nv);
      }
      continue;
    }
    // pass 1: G^T y for every row of the node
    double cs[BS * M];
#pragma unroll
    for (int j = 0; j < BS * M; ++j) cs[j] = 0.0;
    for (int ch = 0; ch < nch; ++ch) {
      const int s = 2 * (lane + kWave * ch);
      const bool on = s < l;
      double v[BS][2];
      load_h(s, on, v);
      double g0[M], g1[M];
      load_bc_pair<M>(a.bc, a.pci[pr[0] + (on ? s : 0)], m, g0, g1);
#pragma unroll
      for (int x = 0; x < BS; ++x)
#pragma unroll
        for (int c = 0; c < M; ++c) cs[x * M + c] += g0[c] * v[x][0] + g1[c] * v[x][1];
      if (nch == 1) {
#pragma unroll
        for (int c = 0; c < M; ++c) {
          sG[wid][lane][c] = g0[c];
          sG[wid][lane][M + c] = g1[c];
        }
      }
    }
    double tot[BS * M];
    wave_sums<BS * M>(cs, tot, lane);
    // d = -W G^T y per row (W of the node's first row when shared)
    double d[BS][M];
#pragma unroll
    for (int x = 0; x < BS; ++x) {
      Uniform<double>* uw = (Uniform<double>*)(a.wpk + (long)(PM > 0 ? r0 : r0 + x) * mp);
#pragma unroll
      for (int c = 0; c < M; ++c) {
        double t = 0.0;
#pragma unroll
        for (int e = 0; e < M; ++e)
          if (c < m && e < m)
            t += uw[(c <= e) ? packed_idx(c, e, m) : packed_idx(e, c, m)] * tot[x * M + e];
        d[x][c] = -t;
      }
    }
    Uniform<double>* binv = (Uniform<double>*)(a.binv + (long)node * BS * BS);
    double inv[BS][BS];
#pragma unroll
    for (int x = 0; x < BS; ++x)
#pragma unroll
      for (int c = 0; c < BS; ++c) inv[x][c] = binv[x * BS + c];
    // pass 2: project the chunk, then the RCG update on it
    for (int ch = 0; ch < nch; ++ch) {
      const int s = 2 * (lane + kWave * ch);
      const bool on = s < l;
      double v[BS][2];
      load_h(s, on, v);
      double g0[M], g1[M];
      if (nch == 1) {  // the lane's own LDS writes of pass 1 (in order)
#pragma unroll
        for (int c = 0; c < M; ++c) {
          g0[c] = sG[wid][lane][c];
          g1[c] = sG[wid][lane][M + c];
        }
      } else {
        load_bc_pair<M>(a.bc, a.pci[pr[0] + (on ? s : 0)], m, g0, g1);
      }
#pragma unroll
      for (int x = 0; x < BS; ++x)
#pragma unroll
        for (int c = 0; c < M; ++c) {
          v[x][0] += g0[c] * d[x][c];
          v[x][1] += g1[c] * d[x][c];
        }
      double r[BS][2];
#pragma unroll
      for (int x = 0; x < BS; ++x) {
        const int idx = pr[x] + (on ? s : 0);
        T rn[2];
        if (FIRST) {
          rn[0] = (T)(-v[x][0]);
          rn[1] = (T)(-v[x][1]);
        } else {
          T ro[2];
          ldv<T, 2>(R + idx, ro);
          rn[0] = ro[0] - alpha * (T)v[x][0];
          rn[1] = ro[1] - alpha * (T)v[x][1];
        }
        r[x][0] = on ? (double)rn[0] : 0.0;
        r[x][1] = on ? (double)rn[1] : 0.0;
        if (on) stv<T, 2>(R + idx, rn);
      }
#pragma unroll
      for (int x = 0; x < BS; ++x)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          double z = 0.0;
#pragma unroll
          for (int c = 0; c < BS; ++c) z += inv[x][c] * r[c][j];
          dot += r[x][j] * (double)(T)z;
        }
      // dP += alpha Y (the first update: dP = 0)
#pragma unroll
      for (int x = 0; x < BS; ++x) {
        const int idx = pr[x] + (on ? s : 0);
        T nv[2];
        if (FIRST) {
          nv[0] = nv[1] = T(0);
        } else {
          T po[2], yo[2];
          ldv<T, 2>(dP + idx, po);
          ldv<T, 2>(Y + idx, yo);
          nv[0] = po[0] + alpha * yo[0];
          nv[1] = po[1] + alpha * yo[1];
        }
        if (on) stv<T, 2>(dP + idx, nv);
      }
    }
  }
  store_partial(dot, a.part_out);
}

// The same over the product's windows of 64 slot pairs (up to kWinNodes
// consecutive nodes per wave, a node may span two windows): every lane of a
// load holds a pair.  The window's block inverses are staged in LDS.
template <class T, int BS, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_direction_win(UpdArgs a) {
  constexpr int WPB = kBlock / kWave;
  constexpr int K = kWinNodes;
  __shared__ double sB[WPB][K * BS * BS];
  if (a.st->done) return;
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  const T* __restrict__ R = (const T*)a.R;
  T* __restrict__ Y = (T*)a.Y;
  Uniform<int>* uprp = (Uniform<int>*)a.prp;
  Uniform<int>* uwin = (Uniform<int>*)a.win;
  double beta_d = 0.0;
  if (scalars_after_gamma(a, FIRST, &beta_d)) return;
  const T beta = (T)beta_d;
  const int nnodes = a.n / BS;
  const int ntiles = (a.nwin + WPB - 1) / WPB;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int t = __builtin_amdgcn_readfirstlane(w.t * WPB + wid);
    if (t >= a.nwin) continue;
    const int node0 = uwin[3 * t], p0 = uwin[3 * t + 1], nn = uwin[3 * t + 2];
    // the window's nodes: pattern rows and the first lane of each
    int pr[K][BS], l[K], lane0[K + 1];
    lane0[0] = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int r0 = min(node0 + j, nnodes - 1) * BS;
#pragma unroll
      for (int r = 0; r < BS; ++r) pr[j][r] = uprp[r0 + r];
      l[j] = uprp[r0 + 1] - pr[j][0];
      lane0[j + 1] = j < nn ? min(kWave, lane0[j] + l[j] / 2 - (j == 0 ? p0 : 0)) : lane0[j];
    }
    for (int e = lane; e < nn * BS * BS; e += kWave)
      sB[wid][e] = a.binv[(long)node0 * BS * BS + e];
    int jl = 0, lend = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      jl += (j > 0 && j < nn && lane >= lane0[j]) ? 1 : 0;
      lend = j + 1 == nn ? lane0[j + 1] : lend;
    }
    int ll = 0, first = 0, lp[BS];
#pragma unroll
    for (int r = 0; r < BS; ++r) lp[r] = 0;
#pragma unroll
    for (int j = 0; j < K; ++j)
      if (jl == j) {
        ll = l[j];
        first = lane0[j] - (j == 0 ? p0 : 0);
#pragma unroll
        for (int r = 0; r < BS; ++r) lp[r] = pr[j][r];
      }
    const int s = 2 * (lane - first);
    const bool on = lane < lend && s < ll;
    // a lane without a pair reads entry 0 (its node may have an empty row
    // that ends the pattern)
#pragma unroll
    for (int r = 0; r < BS; ++r) lp[r] = on ? lp[r] : 0;
    // the wave's own LDS writes are seen by its later reads (in order)
    double inv[BS][BS];
#pragma unroll
    for (int x = 0; x < BS; ++x)
#pragma unroll
      for (int c = 0; c < BS; ++c) inv[x][c] = sB[wid][jl * BS * BS + x * BS + c];
    double r[BS][2];
    T yo[BS][2];
#pragma unroll
    for (int x = 0; x < BS; ++x) {
      const int idx = lp[x] + (on ? s : 0);  // 0 for a lane without a pair
      T rv[2];
      ldv<T, 2>(R + idx, rv);
      r[x][0] = (double)rv[0];
      r[x][1] = (double)rv[1];
      if (!FIRST) ldv<T, 2>(Y + idx, yo[x]);
    }
#pragma unroll
    for (int x = 0; x < BS; ++x) {
      T nv[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        double z = 0.0;
#pragma unroll
        for (int c = 0; c < BS; ++c) z += inv[x][c] * r[c][j];
        nv[j] = FIRST ? (T)z : (T)z + beta * yo[x][j];
      }
      if (on) stv<T, 2>(Y + lp[x] + s, nv);
    }
  }
}

template <class T, int BS, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_direction_pair(UpdArgs a) {
  constexpr int WPB = kBlock / kWave;
  if (a.st->done) return;
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  const T* __restrict__ R = (const T*)a.R;
  T* __restrict__ Y = (T*)a.Y;
  Uniform<int>* uprp = (Uniform<int>*)a.prp;
  double beta_d = 0.0;
  if (scalars_after_gamma(a, FIRST, &beta_d)) return;
  const T beta = (T)beta_d;
  const int nnodes = a.n / BS;
  const int ntiles = (nnodes + WPB - 1) / WPB;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int node = __builtin_amdgcn_readfirstlane(w.t * WPB + wid);
    if (node >= nnodes) continue;
    const int r0 = node * BS;
    int pr[BS];
#pragma unroll
    for (int x = 0; x < BS; ++x) pr[x] = uprp[r0 + x];
    const int l = uprp[r0 + 1] - pr[0];
    const int nch = (l / 2 + kWave - 1) / kWave;
    Uniform<double>* binv = (Uniform<double>*)(a.binv + (long)node * BS * BS);
    double inv[BS][BS];
#pragma unroll
    for (int x = 0; x < BS; ++x)
#pragma unroll
      for (int c = 0; c < BS; ++c) inv[x][c] = binv[x * BS + c];
    for (int ch = 0; ch < nch; ++ch) {
      const int s = 2 * (lane + kWave * ch);
      const bool on = s < l;
      double r[BS][2];
      T yo[BS][2];
#pragma unroll
      for (int x = 0; x < BS; ++x) {
        const int idx = pr[x] + (on ? s : 0);
        T rv[2];
        ldv<T, 2>(R + idx, rv);
        r[x][0] = (double)rv[0];
        r[x][1] = (double)rv[1];
        if (!FIRST) ldv<T, 2>(Y + idx, yo[x]);
      }
#pragma unroll
      for (int x = 0; x < BS; ++x) {
        T nv[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          double z = 0.0;
#pragma unroll
          for (int c = 0; c < BS; ++c) z += inv[x][c] * r[c][j];
          nv[j] = FIRST ? (T)z : (T)z + beta * yo[x][j];
        }
        if (on) stv<T, 2>(Y + pr[x] + s, nv);
      }
    }
  }
}

// --------------------------------------------------------- final, checks --

// P = P0' + dP (Alg. 3 final assembly); with REPROJ the row is corrected back
// onto G_i^T p_i = b_i in FP64 (the correction step of Alg. 2).
template <class TD, int G, int L, bool REPROJ>
__global__ __launch_bounds__(kBlock) void k_final(FinalArgs a) {
  constexpr int ROWS = kBlock / G;
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  const TD* __restrict__ dP = (const TD*)a.dP;
  const int mp = a.m * (a.m + 1) / 2;
  const int ntiles = (a.n + ROWS - 1) / ROWS;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int i = w.t * ROWS + grp;
    const bool valid = i < a.n;
    const int p0 = valid ? a.prp[i] : 0;
    const int l = valid ? a.prp[i + 1] - p0 : 0;
    double v[L];
    int oc[L];
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int s = lane + G * t;
      oc[t] = (s < l) ? a.pci[p0 + s] : -1;
      v[t] = (oc[t] >= 0) ? a.p0p[p0 + s] + (double)dP[p0 + s] : 0.0;
    }
    if (REPROJ)
      correct_row<G, L>(v, oc, a.bc, valid ? a.wpk + (long)i * mp : nullptr,
                        valid ? a.B + (long)i * a.m : nullptr, a.m, valid);
#pragma unroll
    for (int t = 0; t < L; ++t)
      if (oc[t] >= 0) a.out[p0 + lane + G * t] = v[t];
  }
}

// sum_i ||G_i^T p_i - b_i||^2 and sum_i ||b_i||^2
template <int G, int L>
__global__ __launch_bounds__(kBlock) void k_constraint(ConsArgs a) {
  constexpr int ROWS = kBlock / G;
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  double num = 0.0, den = 0.0;
  const int ntiles = (a.n + ROWS - 1) / ROWS;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int i = w.t * ROWS + grp;
    const bool valid = i < a.n;
    const int p0 = valid ? a.prp[i] : 0;
    const int l = valid ? a.prp[i + 1] - p0 : 0;
    double cs[kMaxM];
#pragma unroll
    for (int x = 0; x < kMaxM; ++x) cs[x] = 0.0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int s = lane + G * t;
      if (s >= l) continue;
      const int c = a.pci[p0 + s];
      const double p = a.P[p0 + s];
#pragma unroll
      for (int x = 0; x < kMaxM; ++x)
        if (x < a.m) cs[x] += a.bc[(long)c * a.m + x] * p;
    }
#pragma unroll
    for (int x = 0; x < kMaxM; ++x)
      if (x < a.m) cs[x] = group_sum<G>(cs[x]);
    if (valid && lane == 0) {
      for (int x = 0; x < a.m; ++x) {
        const double b = a.B[(long)i * a.m + x];
        num += (cs[x] - b) * (cs[x] - b);
        den += b * b;
      }
    }
  }
  store_partial(num, a.part_num);
  store_partial(den, a.part_den);
}

__global__ __launch_bounds__(kBlock) void k_reduce(const double* __restrict__ p, int np,
                                                  double* __restrict__ out) {
  const double t = sum_partials(p, np);
  if (threadIdx.x == 0) out[0] = t;
}

// ------------------------------------------------------------- dispatch --

int update_grid(const UpdShape& sh, int n, int grid_cap) {
  if (sh.node == 2) return grid_round(cdiv(n, kBlock), grid_cap);
  if (!sh.node) {
    const int rows = kBlock / sh.G;
    return grid_round(cdiv(n, rows), grid_cap);
  }
  return grid_round(cdiv(n / sh.bs, kBlock / kWave), grid_cap);
}

template <class T, bool FIRST>
static int update_go(const UpdShape& sh, const UpdArgs& a, int grid, hipStream_t s) {
  if (sh.node == 2) {
    if (a.seg && !a.row_seg) return -1;
    if (a.seg) k_update_row<T, FIRST, true><<<grid, kBlock, 0, s>>>(a);
    else k_update_row<T, FIRST, false><<<grid, kBlock, 0, s>>>(a);
    return 0;
  }
  if (!sh.node) {
#define EMIN_UJ(GG, LL)                                                            \
  if (sh.G == GG && sh.L == LL) {                                                  \
    if (a.seg)                                                                     \
      k_update_jac<T, GG, LL, FIRST, true><<<grid, kBlock, 0, s>>>(a);             \
    else                                                                           \
      k_update_jac<T, GG, LL, FIRST, false><<<grid, kBlock, 0, s>>>(a);            \
    return 0;                                                                      \
  }
    EMIN_UJ(1, 1) EMIN_UJ(2, 1) EMIN_UJ(4, 1) EMIN_UJ(8, 1) EMIN_UJ(16, 1)
    EMIN_UJ(32, 1) EMIN_UJ(64, 1) EMIN_UJ(64, 2) EMIN_UJ(64, 3) EMIN_UJ(64, 4)
    EMIN_UJ(4, 4) EMIN_UJ(4, 2)
#undef EMIN_UJ
    return -1;
  }
  const bool aligned16 = ((unsigned long long)a.bc & 15) == 0;
  if (sh.V == 2) {
    if (!a.proj_yh) return -1;
#define EMIN_UP(BB)                                                                \
  if (a.bs == BB) {                                                                \
    if (a.m == 6 && aligned16)                                                     \
      k_update_pair<T, BB, FIRST, 6><<<grid, kBlock, 0, s>>>(a);                   \
    else if (a.m == 3)                                                             \
      k_update_pair<T, BB, FIRST, 3><<<grid, kBlock, 0, s>>>(a);                   \
    else                                                                           \
      k_update_pair<T, BB, FIRST, -1><<<grid, kBlock, 0, s>>>(a);                  \
    return 0;                                                                      \
  }
    EMIN_UP(2) EMIN_UP(3)
#undef EMIN_UP
    return -1;
  }
#define EMIN_UN(BB, LL, VV)                                                        \
  if (a.bs == BB && sh.Ln == LL && sh.V == VV) {                                   \
    if (!a.proj_yh)                                                                \
      k_update_node<T, BB, LL, FIRST, 0, VV><<<grid, kBlock, 0, s>>>(a);           \
    else if (a.m == 6 && aligned16)                                                \
      k_update_node<T, BB, LL, FIRST, 6, VV><<<grid, kBlock, 0, s>>>(a);           \
    else if (a.m == 3)                                                             \
      k_update_node<T, BB, LL, FIRST, 3, VV><<<grid, kBlock, 0, s>>>(a);           \
    else                                                                           \
      k_update_node<T, BB, LL, FIRST, -1, VV><<<grid, kBlock, 0, s>>>(a);          \
    return 0;                                                                      \
  }
  EMIN_UN(1, 1, 1) EMIN_UN(2, 1, 1) EMIN_UN(3, 1, 1) EMIN_UN(4, 1, 1)
  EMIN_UN(1, 2, 1) EMIN_UN(2, 2, 1) EMIN_UN(3, 2, 1) EMIN_UN(3, 3, 1) EMIN_UN(3, 4, 1)
#undef EMIN_UN
  return -1;
}

template <class T, bool FIRST>
static int direction_go(const UpdShape& sh, const UpdArgs& a, int grid, hipStream_t s) {
  if (sh.node == 2) {
    if (a.seg && !a.row_seg) return -1;
    if (a.seg) k_direction_row<T, FIRST, true><<<grid, kBlock, 0, s>>>(a);
    else k_direction_row<T, FIRST, false><<<grid, kBlock, 0, s>>>(a);
    return 0;
  }
  if (!sh.node) {
#define EMIN_DJ(GG, LL)                                                            \
  if (sh.G == GG && sh.L == LL) {                                                  \
    if (a.seg)                                                                     \
      k_direction_jac<T, GG, LL, FIRST, true><<<grid, kBlock, 0, s>>>(a);          \
    else                                                                           \
      k_direction_jac<T, GG, LL, FIRST, false><<<grid, kBlock, 0, s>>>(a);         \
    return 0;                                                                      \
  }
    EMIN_DJ(1, 1) EMIN_DJ(2, 1) EMIN_DJ(4, 1) EMIN_DJ(8, 1) EMIN_DJ(16, 1)
    EMIN_DJ(32, 1) EMIN_DJ(64, 1) EMIN_DJ(64, 2) EMIN_DJ(64, 3) EMIN_DJ(64, 4)
    EMIN_DJ(4, 4) EMIN_DJ(4, 2)
#undef EMIN_DJ
    return -1;
  }
  if (sh.V == 2 && a.win) {  // over the product's windows (one wave each)
    if (a.bs == 2) { k_direction_win<T, 2, FIRST><<<grid, kBlock, 0, s>>>(a); return 0; }
    if (a.bs == 3) { k_direction_win<T, 3, FIRST><<<grid, kBlock, 0, s>>>(a); return 0; }
    return -1;
  }
  if (sh.V == 2) {
    if (a.bs == 2) { k_direction_pair<T, 2, FIRST><<<grid, kBlock, 0, s>>>(a); return 0; }
    if (a.bs == 3) { k_direction_pair<T, 3, FIRST><<<grid, kBlock, 0, s>>>(a); return 0; }
    return -1;
  }
#define EMIN_DN(BB, LL, VV)                                                        \
  if (a.bs == BB && sh.Ln == LL && sh.V == VV) {                                   \
    k_direction_node<T, BB, LL, FIRST, VV><<<grid, kBlock, 0, s>>>(a);             \
    return 0;                                                                      \
  }
  EMIN_DN(1, 1, 1) EMIN_DN(2, 1, 1) EMIN_DN(3, 1, 1) EMIN_DN(4, 1, 1)
  EMIN_DN(1, 2, 1) EMIN_DN(2, 2, 1) EMIN_DN(3, 2, 1) EMIN_DN(3, 3, 1) EMIN_DN(3, 4, 1)
#undef EMIN_DN
  return -1;
}

int launch_update(const UpdShape& sh, int first, int mixed, const UpdArgs& a, int grid_cap,
                  hipStream_t s) {
  if (a.n <= 0) return 0;
  const int grid = update_grid(sh, a.n, grid_cap);
  if (mixed) return first ? update_go<float, true>(sh, a, grid, s) : update_go<float, false>(sh, a, grid, s);
  return first ? update_go<double, true>(sh, a, grid, s) : update_go<double, false>(sh, a, grid, s);
}

int launch_direction(const UpdShape& sh, int first, int mixed, const UpdArgs& a, int grid_cap,
                     hipStream_t s) {
  if (a.n <= 0) return 0;
  const int grid = (sh.V == 2 && a.win) ? grid_round(cdiv(a.nwin, kBlock / kWave), grid_cap)
                                        : update_grid(sh, a.n, grid_cap);
  if (mixed)
    return first ? direction_go<float, true>(sh, a, grid, s) : direction_go<float, false>(sh, a, grid, s);
  return first ? direction_go<double, true>(sh, a, grid, s) : direction_go<double, false>(sh, a, grid, s);
}

// P = P0' + dP with the correction step applied per node (the rows of a node
// share G_i and W_i): one wave per node, as in the node update.
template <class TD, int BS, int L, int M>
__global__ __launch_bounds__(kBlock) void k_final_node(FinalArgs a) {
  constexpr int WPB = kBlock / kWave;
  constexpr int MP = M * (M + 1) / 2;
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  const TD* __restrict__ dP = (const TD*)a.dP;
  Uniform<int>* uprp = (Uniform<int>*)a.prp;
  const int nnodes = a.n / BS;
  const int ntiles = (nnodes + WPB - 1) / WPB;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int node = __builtin_amdgcn_readfirstlane(w.t * WPB + wid);
    if (node >= nnodes) continue;
    const int r0 = node * BS;
    int pr[BS];
#pragma unroll
    for (int x = 0; x < BS; ++x) pr[x] = uprp[r0 + x];
    const int l = uprp[r0 + 1] - pr[0];
    if (l == 0) continue;
    bool on[L];
    int so[L], oc[L];
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int s = lane + kWave * t;
      on[t] = s < l;
      so[t] = on[t] ? s : 0;
      oc[t] = a.pci[pr[0] + so[t]];
    }
    double v[BS][L];
#pragma unroll
    for (int x = 0; x < BS; ++x)
#pragma unroll
      for (int t = 0; t < L; ++t) {
        const int idx = pr[x] + so[t];
        const double pv = a.p0p[idx] + (double)dP[idx];
        v[x][t] = on[t] ? pv : 0.0;
      }
    node_apply<L, M, BS, true>(v, oc, a.bc, a.wpk + (long)r0 * MP, a.B + (long)r0 * M, lane);
#pragma unroll
    for (int x = 0; x < BS; ++x)
#pragma unroll
      for (int t = 0; t < L; ++t)
        if (on[t]) a.out[pr[x] + so[t]] = v[x][t];
  }
}

// The same for patterns of whole even-sized column groups (the slot-pair
// node form): a lane owns a slot pair of every row of the node, the chunks
// of 64 pairs run in a loop, and a one-chunk node keeps each lane's B_c rows
// in LDS from the first pass (the row sums) to the second (the correction).
template <class TD, int BS, int M>
__global__ __launch_bounds__(kBlock) void k_final_pair(FinalArgs a) {
  constexpr int WPB = kBlock / kWave;
  constexpr int MP = M * (M + 1) / 2;
  __shared__ double sG[WPB][kWave][2 * M];
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  const TD* __restrict__ dP = (const TD*)a.dP;
  Uniform<int>* uprp = (Uniform<int>*)a.prp;
  const int nnodes = a.n / BS;
  const int ntiles = (nnodes + WPB - 1) / WPB;
  for (TileWalk w(ntiles); w.t < w.end; w.t += w.step) {
    const int node = __builtin_amdgcn_readfirstlane(w.t * WPB + wid);
    if (node >= nnodes) continue;
    const int r0 = node * BS;
    int pr[BS];
#pragma unroll
    for (int x = 0; x < BS; ++x) pr[x] = uprp[r0 + x];
    const int l = uprp[r0 + 1] - pr[0];
    if (l == 0) continue;
    const int nch = (l / 2 + kWave - 1) / kWave;
    // p0' + dP at the chunk's pairs (zeros off the row)
    auto load_p = [&](int s, bool on, double (&v)[BS][2]) {
#pragma unroll
      for (int x = 0; x < BS; ++x) {
        const int idx = pr[x] + (on ? s : 0);
        double p0[2];
        TD d[2];
        ldv<double, 2>(a.p0p + idx, p0);
        ldv<TD, 2>(dP + idx, d);
        v[x][0] = on ? p0[0] + (double)d[0] : 0.0;
        v[x][1] = on ? p0[1] + (double)d[1] : 0.0;
      }
    };
    // pass 1: G^T p for every row of the node
    double cs[BS * M], vk[BS][2];
#pragma unroll
    for (int j = 0; j < BS * M; ++j) cs[j] = 0.0;
    for (int ch = 0; ch < nch; ++ch) {
      const int s = 2 * (lane + kWave * ch);
      const bool on = s < l;
      double v[BS][2];
      load_p(s, on, v);
#pragma unroll
      for (int x = 0; x < BS; ++x) {
        vk[x][0] = v[x][0];
        vk[x][1] = v[x][1];
      }
      double g0[M], g1[M];
      load_bc_pair<M>(a.bc, a.pci[pr[0] + (on ? s : 0)], M, g0, g1);
#pragma unroll
      for (int x = 0; x < BS; ++x)
#pragma unroll
        for (int c = 0; c < M; ++c) cs[x * M + c] += g0[c] * v[x][0] + g1[c] * v[x][1];
      if (nch == 1) {
#pragma unroll
        for (int c = 0; c < M; ++c) {
          sG[wid][lane][c] = g0[c];
          sG[wid][lane][M + c] = g1[c];
        }
      }
    }
    double tot[BS * M];
    wave_sums<BS * M>(cs, tot, lane);
    // d = W (b - G^T p) per row (the rows share the node's first row's W)
    Uniform<double>* ub = (Uniform<double>*)(a.B + (long)r0 * M);
    Uniform<double>* uw = (Uniform<double>*)(a.wpk + (long)r0 * MP);
    double d[BS][M];
#pragma unroll
    for (int x = 0; x < BS; ++x)
#pragma unroll
      for (int c = 0; c < M; ++c) {
        double t = 0.0;
#pragma unroll
        for (int e = 0; e < M; ++e)
          t += uw[(c <= e) ? packed_idx(c, e, M) : packed_idx(e, c, M)] *
               (ub[x * M + e] - tot[x * M + e]);
        d[x][c] = t;
      }
    // pass 2: p + G d, stored (a one-chunk node kept its values: vk)
    if (nch == 1) {
      const int s = 2 * lane;
      if (s < l) {
#pragma unroll
        for (int x = 0; x < BS; ++x) {
          double o[2] = {vk[x][0], vk[x][1]};
#pragma unroll
          for (int c = 0; c < M; ++c) {
            o[0] += sG[wid][lane][c] * d[x][c];
            o[1] += sG[wid][lane][M + c] * d[x][c];
          }
          stv<double, 2>(a.out + pr[x] + s, o);
        }
      }
      continue;
    }
    for (int ch = 0; ch < nch; ++ch) {
      const int s = 2 * (lane + kWave * ch);
      const bool on = s < l;
      double v[BS][2];
      load_p(s, on, v);
      double g0[M], g1[M];
      if (nch == 1) {  // the lane's own LDS writes of pass 1 (in order)
#pragma unroll
        for (int c = 0; c < M; ++c) {
          g0[c] = sG[wid][lane][c];
          g1[c] = sG[wid][lane][M + c];
        }
      } else {
        load_bc_pair<M>(a.bc, a.pci[pr[0] + (on ? s : 0)], M, g0, g1);
      }
#pragma unroll
      for (int x = 0; x < BS; ++x) {
        double o[2] = {v[x][0], v[x][1]};
#pragma unroll
        for (int c = 0; c < M; ++c) {
          o[0] += g0[c] * d[x][c];
          o[1] += g1[c] * d[x][c];
        }
        if (on) stv<double, 2>(a.out + pr[x] + s, o);
      }
    }
  }
}

template <class TD, int BS, int M>
static int final_pair_go(const FinalArgs& a, int grid_cap, hipStream_t s) {
  const int grid = grid_round(cdiv(a.n / BS, kBlock / kWave), grid_cap);
  k_final_pair<TD, BS, M><<<grid, kBlock, 0, s>>>(a);
  return 0;
}

template <class TD, int BS, int M>
static int final_node_go(const FinalArgs& a, int grid_cap, hipStream_t s) {
  const int grid = grid_round(cdiv(a.n / BS, kBlock / kWave), grid_cap);
  if (a.lmax <= 64) k_final_node<TD, BS, 1, M><<<grid, kBlock, 0, s>>>(a);
  else if (a.lmax <= 128) k_final_node<TD, BS, 2, M><<<grid, kBlock, 0, s>>>(a);
  else if (a.lmax <= 192) k_final_node<TD, BS, 3, M><<<grid, kBlock, 0, s>>>(a);
  else if (a.lmax <= 256) k_final_node<TD, BS, 4, M><<<grid, kBlock, 0, s>>>(a);
  else return -1;
  return 0;
}

// The node form of the corrected assembly: nodes of 2 or 3 rows sharing a
// pattern row, m = 3 or 6 (B_c 16-byte aligned for m = 6).  -1: not taken.
template <class TD>
static int final_node(const FinalArgs& a, int grid_cap, hipStream_t s) {
  if (a.nbs < 2 || a.n % a.nbs) return -1;
  const bool al16 = ((unsigned long long)a.bc & 15) == 0;
  // slot pairs: rows at even offsets, and 16-byte aligned arrays
  if (a.pairs && al16 && ((unsigned long long)a.out & 15) == 0 &&
      ((unsigned long long)a.p0p & 15) == 0 && ((unsigned long long)a.dP & 15) == 0) {
    if (a.nbs == 3 && a.m == 6) return final_pair_go<TD, 3, 6>(a, grid_cap, s);
    if (a.nbs == 2 && a.m == 6) return final_pair_go<TD, 2, 6>(a, grid_cap, s);
    if (a.nbs == 3 && a.m == 3) return final_pair_go<TD, 3, 3>(a, grid_cap, s);
    if (a.nbs == 2 && a.m == 3) return final_pair_go<TD, 2, 3>(a, grid_cap, s);
  }
  if (a.lmax > 256) return -1;
  if (a.nbs == 3 && a.m == 6 && al16) return final_node_go<TD, 3, 6>(a, grid_cap, s);
  if (a.nbs == 3 && a.m == 3) return final_node_go<TD, 3, 3>(a, grid_cap, s);
  if (a.nbs == 2 && a.m == 3) return final_node_go<TD, 2, 3>(a, grid_cap, s);
  return -1;
}

template <class TD, bool RP>
static int final_go(int G, int L, const FinalArgs& a, int grid_cap, hipStream_t s) {
  if (RP && final_node<TD>(a, grid_cap, s) == 0) return 0;
  const int grid = grid_round(cdiv(a.n, kBlock / G), grid_cap);
#define EMIN_FN(GG, LL)                                                            \
  if (G == GG && L == LL) {                                                        \
    k_final<TD, GG, LL, RP><<<grid, kBlock, 0, s>>>(a);                            \
    return 0;                                                                      \
  }
  EMIN_FN(1, 1) EMIN_FN(2, 1) EMIN_FN(4, 1) EMIN_FN(8, 1) EMIN_FN(16, 1)
  EMIN_FN(32, 1) EMIN_FN(64, 1) EMIN_FN(64, 2) EMIN_FN(64, 3) EMIN_FN(64, 4)
  EMIN_FN(4, 2) EMIN_FN(4, 4)
#undef EMIN_FN
  return -1;
}

int launch_final(int G, int L, int mixed, int reproject, const FinalArgs& a, int grid_cap,
                 hipStream_t s) {
  if (a.n <= 0) return 0;
  if (mixed) return final_go<float, true>(G, L, a, grid_cap, s);
  return reproject ? final_go<double, true>(G, L, a, grid_cap, s)
                   : final_go<double, false>(G, L, a, grid_cap, s);
}

int constraint_grid(int G, int n, int grid_cap) { return grid_round(cdiv(n, kBlock / G), grid_cap); }

void launch_reduce(const double* partials, int np, double* out, hipStream_t s) {
  k_reduce<<<1, kBlock, 0, s>>>(partials, np, out);
}

int launch_constraint(int G, int L, const ConsArgs& a, int grid_cap, hipStream_t s) {
  if (a.n <= 0) return 0;
  const int grid = grid_round(cdiv(a.n, kBlock / G), grid_cap);
#define EMIN_CN(GG, LL)                                                            \
  if (G == GG && L == LL) {                                                        \
    k_constraint<GG, LL><<<grid, kBlock, 0, s>>>(a);                               \
    return 0;                                                                      \
  }
  EMIN_CN(1, 1) EMIN_CN(2, 1) EMIN_CN(4, 1) EMIN_CN(8, 1) EMIN_CN(16, 1)
  EMIN_CN(32, 1) EMIN_CN(64, 1) EMIN_CN(64, 2) EMIN_CN(64, 3) EMIN_CN(64, 4)
#undef EMIN_CN
  return -1;
}

}  // namespace emin
