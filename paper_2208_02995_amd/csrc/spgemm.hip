// Masked SpGEMM: Y_hat = Pi mask(A Y), the K y product of Sec. 4 (K is block
// diagonal by columns of P, so K y is A Y restricted to the fixed pattern;
// K itself is never formed), with the block projector of Sec. 3.1 and the
// partial <Y, Y_hat> of Alg. 3 fused in the epilogue.
//
//   Y_hat(i, j) = sum_{k in A(i,:)} A(i,k) Y(k,j)   for j in J_i (and j in J_k)
//
// Two shapes, both bandwidth-oriented (no MFMA: this is a gather, not a
// dense contraction):
//  * k1_short (rows of P up to 32 long): G lanes per row of A.  Lane g takes
//    neighbours A(i, g), A(i, g+G), ... two at a time; each lane holds all S
//    columns of J_i in registers and matches every (column, value) of the
//    neighbour's row of Y against them.  With `packed`, the neighbour's row
//    of the pattern is found through one int per entry of A -- (offset << 4)
//    | length, built once per pattern -- which replaces A's column index (same
//    bytes) and removes one dependent load from the gather chain.  All S
//    candidate loads of a neighbour are issued together (clamped addresses,
//    invalid ones masked).  The group then reduce-scatters its S partial sums
//    so lane g owns slots g*S/G ..; the projector and the dot run on those.
//  * k1_node (long rows, e.g. elasticity with A^2 P0 patterns): one wave per
//    node of BS rows sharing a pattern row; J_a goes into an LDS hash
//    (column -> slot) and per-row accumulators into LDS; lanes sweep the
//    columns of each neighbour node's pattern row, look them up, and apply
//    the BS x BS block of A to the BS values of Y.
#include "common.hpp"
#include "launch.hpp"

namespace emin {

__global__ __launch_bounds__(kBlock) void k_build_anb(const int* __restrict__ aci, int nnzA,
                                                     const int* __restrict__ prp,
                                                     int* __restrict__ anb) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= nnzA) return;
  const int k = aci[e];
  const int q = prp[k];
  const int len = prp[k + 1] - q;
  anb[e] = (q << 4) | (len < 15 ? len : 15);
}

// ------------------------------------------------------------- dispatch --

static int grid_round(int ntiles, int cap) {
  int g = ntiles < cap ? ntiles : cap;
  g = ((g + kNumXcd - 1) / kNumXcd) * kNumXcd;
  return g < kNumXcd ? kNumXcd : g;
}

void launch_build_anb(const int* aci, int nnzA, const int* prp, int* anb, hipStream_t s) {
  if (nnzA > 0) k_build_anb<<<(nnzA + kBlock - 1) / kBlock, kBlock, 0, s>>>(aci, nnzA, prp, anb);
}

int k1_grid(const K1Shape& sh, int n, int grid_cap) {
  if (sh.kind == 0 || sh.kind == 2 || sh.kind == 3) {
    const int rows = sh.kind == 3 ? kBlock : kBlock / sh.G;
    return grid_round((n + rows - 1) / rows, grid_cap);
  }
  const int nodes = sh.kind == 5 ? sh.nwin : n / sh.bs;  // kind 5: one wave per window
  const int per = kBlock / kWave;
  return grid_round((nodes + per - 1) / per, grid_cap);
}

// (G, S) pairs instantiated for k1_short; keep in step with k1_short_go.
bool k1_short_supported(int G, int S) {
  static const int ok[][2] = {{1, 1}, {1, 2}, {2, 2}, {2, 4}, {4, 4}, {4, 8}, {8, 8},
                              {8, 16}, {16, 16}, {16, 32}, {32, 32}};
  for (const auto& v : ok)
    if (v[0] == G && v[1] == S) return true;
  return false;
}

int launch_k1(const K1Shape& sh, int mode, int precision, const K1Args& a, int grid_cap,
              hipStream_t s) {
  if (a.n <= 0) return 0;
  const int grid = k1_grid(sh, a.n, grid_cap);
  if (sh.kind == 2) return launch_k1_mapped(mode, precision, sh, a, grid, s);
  if (sh.kind == 3) return launch_k1_wide(mode, precision, sh, a, grid, s);
  if (sh.kind == 4) return launch_k1_nodemap(mode, precision, sh, a, grid, s);
  if (sh.kind == 5) return launch_k1_nodepair(mode, precision, sh, a, grid, s);
  int r = -2;
  if (sh.kind == 0) {
    r = launch_k1_short_a(mode, precision, sh, a, grid, s);
    if (r == -2) r = launch_k1_short_b(mode, precision, sh, a, grid, s);
  } else if (sh.kind == 1) {
    r = launch_k1_hash(mode, precision, sh, a, grid, s);
  }
  return r == -2 ? -1 : r;
}

}  // namespace emin
