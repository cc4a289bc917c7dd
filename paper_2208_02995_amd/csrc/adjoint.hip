// Kernels of the adjoint (reverse sweep of Alg. 2 + Alg. 3 with respect to
// the values of A and P0) and of the differentiation loss
//     L = w_E tr(P^T A P) + w_T ||e - P c||_A^2,  c = (P^T A P)^{-1} P^T A e.
//
// The reverse sweep needs, besides the masked product K(A) Y (and its
// transpose, equal to it for symmetric A), the sampled product
//     Abar(i, l) += sum_{j in J_i and J_l} U(i, j) V(l, j)
// on A's stored entries -- the same (i, l, j) triples as the masked product,
// read through the same precomputed intersection map.  All reductions are
// block partials summed in fixed order: results are deterministic.
#include "common.hpp"
#include "launch.hpp"
#include "project.hpp"

namespace emin {

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }
static inline int gsz(long n) { const int b = cdiv(n, kBlock); return b < 1024 ? (b < 1 ? 1 : b) : 1024; }

// y = a x + b y; with b == 0 y is not read (y may hold anything)
__global__ __launch_bounds__(kBlock) void k_axpby(int n, double a, const double* __restrict__ x,
                                                 double b, double* __restrict__ y) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const double ax = x ? a * x[i] : 0.0;
    y[i] = (b == 0.0) ? ax : ax + b * y[i];
  }
}

// y = (amul * *as) x + b y, the coefficient read on the device
__global__ __launch_bounds__(kBlock) void k_axpby_s(int n, const double* __restrict__ as,
                                                   double amul, const double* __restrict__ x,
                                                   double b, double* __restrict__ y) {
  const double a = amul * *as;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    y[i] = (b == 0.0) ? a * x[i] : a * x[i] + b * y[i];
}

// Scalars of one reverse-sweep iteration, formed on the device from the dot
// partials (sc: [gnext, gbar, abar, dbar]).  stage 0, after <Pbar, Y_k> and
// <Rbar_{k+1}, Yhat_k>: abar = their difference, gbar = gnext + abar / delta,
// dbar = -abar gamma / delta^2.  stage 1, after <Ybar, Y_{k-1}> = bbar:
// gbar += bbar / gamma_{k-1}, gnext = -bbar gamma / gamma_{k-1}^2.  stage 2
// (k = 1): gnext = 0.
__global__ __launch_bounds__(kBlock) void k_bwd_scalars(int stage, const double* __restrict__ p1,
                                                       int n1, const double* __restrict__ p2,
                                                       int n2, double g, double dl, double gprev,
                                                       double* sc) {
  const double s1 = stage < 2 ? sum_partials(p1, n1) : 0.0;
  const double s2 = stage == 0 ? sum_partials(p2, n2) : 0.0;
  if (threadIdx.x != 0) return;
  if (stage == 0) {
    const double abar = s1 - s2;
    sc[2] = abar;
    sc[1] = sc[0] + abar / dl;
    sc[3] = -abar * g / (dl * dl);
  } else if (stage == 1) {
    sc[1] = sc[1] + s1 / gprev;
    sc[0] = -s1 * g / (gprev * gprev);
  } else {
    sc[0] = 0.0;
  }
}

__global__ __launch_bounds__(kBlock) void k_dot(int n, const double* __restrict__ x,
                                               const double* __restrict__ y,
                                               double* __restrict__ partials) {
  double v = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) v += x[i] * y[i];
  store_partial(v, partials);
}

// y = x / d elementwise (coarse Jacobi)
__global__ __launch_bounds__(kBlock) void k_div(int n, const double* __restrict__ x,
                                               const double* __restrict__ d,
                                               double* __restrict__ y) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    y[i] = x[i] / d[i];
}

// y[p] = c * y[p] + x[p] * dinv[row(p)]  (thread per row; c == 0: y not read)
__global__ __launch_bounds__(kBlock) void k_rowscale(const int* __restrict__ prp,
                                                    const double* __restrict__ dinv, int n,
                                                    const double* __restrict__ x, double c,
                                                    double* __restrict__ y) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double d = dinv[i];
  for (int p = prp[i]; p < prp[i + 1]; ++p) y[p] = (c == 0.0 ? 0.0 : c * y[p]) + x[p] * d;
}

// y = Pi x, one group of G lanes per row
template <int G, int L>
__global__ __launch_bounds__(kBlock) void k_project(const int* __restrict__ prp,
                                                   const int* __restrict__ pci,
                                                   const double* __restrict__ bc,
                                                   const double* __restrict__ wpk, int m, int n,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ y) {
  constexpr int ROWS = kBlock / G;
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  const int mp = m * (m + 1) / 2;
  for (int t0 = blockIdx.x; t0 * ROWS < n; t0 += gridDim.x) {
    const int i = t0 * ROWS + grp;
    const bool valid = i < n;
    const int p0 = valid ? prp[i] : 0;
    const int l = valid ? prp[i + 1] - p0 : 0;
    double v[L];
    int oc[L];
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int s = lane + G * t;
      oc[t] = (s < l) ? pci[p0 + s] : -1;
      v[t] = (s < l) ? x[p0 + s] : 0.0;
    }
    project_row<G, L, false>(v, oc, bc, valid ? wpk + (long)i * mp : nullptr, m, valid);
#pragma unroll
    for (int t = 0; t < L; ++t)
      if (oc[t] >= 0) y[p0 + lane + G * t] = v[t];
  }
}

// Abar[e] += scale * sum_s U[p0 + s] * V[aoff[e] + amap(e, s)]  (thread per row)
__global__ __launch_bounds__(kBlock) void k_sddmm(const int* __restrict__ arp,
                                                 const int* __restrict__ prp,
                                                 const int* __restrict__ mrp,
                                                 const unsigned char* __restrict__ amap,
                                                 const int* __restrict__ aoff, int n,
                                                 const double* __restrict__ U,
                                                 const double* __restrict__ V, double scale,
                                                 double* __restrict__ Abar) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int p0 = prp[i], l = prp[i + 1] - p0;
  const int e0 = arp[i], e1 = arp[i + 1];
  const int mb = mrp[i];
  for (int e = e0; e < e1; ++e) {
    const int q0 = aoff[e];
    const unsigned char* mp = amap + mb + (long)(e - e0) * l;
    double acc = 0.0;
    for (int s = 0; s < l; ++s) {
      const int q = mp[s];
      if (q != 0xFF) acc += U[p0 + s] * V[q0 + q];
    }
    Abar[e] += scale * acc;
  }
}

// Abar(i, i) -= sum_j W(i, j) R(i, j) / A(i, i)^2   (Jacobi: Z = R / A_ii)
__global__ __launch_bounds__(kBlock) void k_diag_grad(const int* __restrict__ arp,
                                                     const int* __restrict__ aci,
                                                     const double* __restrict__ av,
                                                     const int* __restrict__ prp, int n,
                                                     const double* __restrict__ W,
                                                     const double* __restrict__ R,
                                                     double* __restrict__ Abar) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int lo = arp[i], hi = arp[i + 1] - 1, dpos = -1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int c = aci[mid];
    if (c == i) { dpos = mid; break; }
    if (c < i) lo = mid + 1; else hi = mid - 1;
  }
  if (dpos < 0) return;
  double s = 0.0;
  for (int p = prp[i]; p < prp[i + 1]; ++p) s += W[p] * R[p];
  const double d = av[dpos];
  Abar[dpos] -= s / (d * d);
}

// out[q] = x[position of P0's entry q in the pattern]
__global__ __launch_bounds__(kBlock) void k_restrict(const int* __restrict__ qrp,
                                                    const int* __restrict__ qci,
                                                    const int* __restrict__ prp,
                                                    const int* __restrict__ pci, int n,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int p = prp[i];
  const int pe = prp[i + 1];
  for (int q = qrp[i]; q < qrp[i + 1]; ++q) {
    const int c = qci[q];
    while (p < pe && pci[p] < c) ++p;
    out[q] = (p < pe && pci[p] == c) ? x[p] : 0.0;
  }
}

// y = M x for CSR M (thread per row)
__global__ __launch_bounds__(kBlock) void k_spmv(const int* __restrict__ rp,
                                                const int* __restrict__ ci,
                                                const double* __restrict__ v, int nrows,
                                                const double* __restrict__ x,
                                                double* __restrict__ y) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= nrows) return;
  double s = 0.0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) s += v[e] * x[ci[e]];
  y[i] = s;
}

// ---- column structure of the pattern (for P^T z), deterministic order
__global__ __launch_bounds__(kBlock) void k_col_count(const int* __restrict__ pci, int nnz,
                                                     int* __restrict__ cnt) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p < nnz) atomicAdd(&cnt[pci[p]], 1);
}

__global__ __launch_bounds__(kBlock) void k_col_fill(const int* __restrict__ prp,
                                                    const int* __restrict__ pci, int n,
                                                    const int* __restrict__ ccp,
                                                    int* __restrict__ fill,
                                                    int* __restrict__ cri,
                                                    int* __restrict__ cpos) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  for (int p = prp[i]; p < prp[i + 1]; ++p) {
    const int c = pci[p];
    const int slot = ccp[c] + atomicAdd(&fill[c], 1);
    cri[slot] = i;
    cpos[slot] = p;
  }
}

// sort each column's entries by row (insertion sort; columns are short)
__global__ __launch_bounds__(kBlock) void k_col_sort(const int* __restrict__ ccp, int nc,
                                                    int* __restrict__ cri,
                                                    int* __restrict__ cpos) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= nc) return;
  const int a = ccp[j], b = ccp[j + 1];
  for (int x = a + 1; x < b; ++x) {
    const int r = cri[x], q = cpos[x];
    int y = x - 1;
    while (y >= a && cri[y] > r) {
      cri[y + 1] = cri[y];
      cpos[y + 1] = cpos[y];
      --y;
    }
    cri[y + 1] = r;
    cpos[y + 1] = q;
  }
}

// y_j = sum over column j of P[cpos] * z[cri]   (z = NULL: column sums of P)
__global__ __launch_bounds__(kBlock) void k_spmv_t(const int* __restrict__ ccp,
                                                  const int* __restrict__ cri,
                                                  const int* __restrict__ cpos, int nc,
                                                  const double* __restrict__ Pv,
                                                  const double* __restrict__ z,
                                                  double* __restrict__ y) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= nc) return;
  double s = 0.0;
  for (int t = ccp[j]; t < ccp[j + 1]; ++t) s += Pv[cpos[t]] * (z ? z[cri[t]] : 1.0);
  y[j] = s;
}

// two-grid gradients: Pbar(i, j) += s Au_i c_j on the pattern; Abar(i, l) += t u_i u_l
__global__ __launch_bounds__(kBlock) void k_tg_pgrad(const int* __restrict__ prp,
                                                    const int* __restrict__ pci, int n,
                                                    const double* __restrict__ Au,
                                                    const double* __restrict__ c, double s,
                                                    double* __restrict__ Pbar) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double a = s * Au[i];
  for (int p = prp[i]; p < prp[i + 1]; ++p) Pbar[p] += a * c[pci[p]];
}

__global__ __launch_bounds__(kBlock) void k_tg_agrad(const int* __restrict__ arp,
                                                    const int* __restrict__ aci, int n,
                                                    const double* __restrict__ u, double t,
                                                    double* __restrict__ Abar) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double a = t * u[i];
  for (int e = arp[i]; e < arp[i + 1]; ++e) Abar[e] += a * u[aci[e]];
}

__global__ __launch_bounds__(kBlock) void k_mul(int n, const double* __restrict__ x,
                                               const double* __restrict__ y,
                                               double* __restrict__ z) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) z[i] = x[i] * y[i];
}

// ---- coarse CG of the two-grid loss, its scalars kept on the device ----
// q = P^T z over the column structure, and the partials of <p, q>
__global__ __launch_bounds__(kBlock) void k_spmv_t_dot(const int* __restrict__ ccp,
                                                      const int* __restrict__ cri,
                                                      const int* __restrict__ cpos, int nc,
                                                      const double* __restrict__ Pv,
                                                      const double* __restrict__ z,
                                                      const double* __restrict__ p,
                                                      double* __restrict__ q,
                                                      double* __restrict__ partials) {
  double d = 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < nc; j += gridDim.x * kBlock) {
    double s = 0.0;
    for (int t = ccp[j]; t < ccp[j + 1]; ++t) s += Pv[cpos[t]] * z[cri[t]];
    q[j] = s;
    d += p[j] * s;
  }
  store_partial(d, partials);
}

// a = <r, z> / <p, q> (0 when <p, q> <= 0); x += a p, r -= a q, z = r / dg;
// partials of the new <r, z> and <r, r>
__global__ __launch_bounds__(kBlock) void k_cg_xr(int nc, const double* __restrict__ rz,
                                                 const double* __restrict__ pq_part, int np,
                                                 const double* __restrict__ p,
                                                 const double* __restrict__ q,
                                                 const double* __restrict__ dg,
                                                 double* __restrict__ x, double* __restrict__ r,
                                                 double* __restrict__ z,
                                                 double* __restrict__ rz_part,
                                                 double* __restrict__ rr_part) {
  const double pq = sum_partials(pq_part, np);
  const double a = (pq > 0.0) ? *rz / pq : 0.0;
  double s1 = 0.0, s2 = 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < nc; j += gridDim.x * kBlock) {
    x[j] += a * p[j];
    const double rj = r[j] - a * q[j];
    r[j] = rj;
    const double zj = rj / dg[j];
    z[j] = zj;
    s1 += rj * zj;
    s2 += rj * rj;
  }
  store_partial(s1, rz_part);
  store_partial(s2, rr_part);
}

// b = <r, z>_new / <r, z>_old (0 when the old one is not positive);
// p = z + b p; block 0 records <r, z>_new
__global__ __launch_bounds__(kBlock) void k_cg_p(int nc, const double* __restrict__ rz_part,
                                                int np, const double* __restrict__ rz_old,
                                                double* __restrict__ rz_new,
                                                const double* __restrict__ z,
                                                double* __restrict__ p) {
  const double rzn = sum_partials(rz_part, np);
  const double ro = *rz_old;
  const double b = (ro > 0.0) ? rzn / ro : 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < nc; j += gridDim.x * kBlock)
    p[j] = z[j] + b * p[j];
  if (blockIdx.x == 0 && threadIdx.x == 0) *rz_new = rzn;
}

// ------------------------------------------------------------- launchers --

void launch_axpby(int n, double a, const double* x, double b, double* y, hipStream_t s) {
  if (n > 0) k_axpby<<<gsz(n), kBlock, 0, s>>>(n, a, x, b, y);
}
int dot_grid(int n) { return gsz(n); }
void launch_axpby_s(int n, const double* as, double amul, const double* x, double b, double* y,
                    hipStream_t s) {
  if (n > 0) k_axpby_s<<<gsz(n), kBlock, 0, s>>>(n, as, amul, x, b, y);
}
void launch_bwd_scalars(int stage, const double* p1, int n1, const double* p2, int n2, double g,
                        double dl, double gprev, double* sc, hipStream_t s) {
  k_bwd_scalars<<<1, kBlock, 0, s>>>(stage, p1, n1, p2, n2, g, dl, gprev, sc);
}
void launch_dot(int n, const double* x, const double* y, double* partials, hipStream_t s) {
  k_dot<<<gsz(n), kBlock, 0, s>>>(n, x, y, partials);
}
void launch_div(int n, const double* x, const double* d, double* y, hipStream_t s) {
  if (n > 0) k_div<<<gsz(n), kBlock, 0, s>>>(n, x, d, y);
}
void launch_mul(int n, const double* x, const double* y, double* z, hipStream_t s) {
  if (n > 0) k_mul<<<gsz(n), kBlock, 0, s>>>(n, x, y, z);
}
void launch_rowscale(const int* prp, const double* dinv, int n, const double* x, double c,
                     double* y, hipStream_t s) {
  if (n > 0) k_rowscale<<<cdiv(n, kBlock), kBlock, 0, s>>>(prp, dinv, n, x, c, y);
}
int launch_project(const int* prp, const int* pci, const double* bc, const double* wpk, int m,
                   int n, int lmax, const double* x, double* y, hipStream_t s) {
  if (n <= 0) return 0;
  const int G = lmax <= 4 ? 4 : lmax <= 16 ? 16 : 64;
  const int gr = cdiv(n, kBlock / G);
  const int grid = gr < 4096 ? gr : 4096;
  if (G == 4) k_project<4, 1><<<grid, kBlock, 0, s>>>(prp, pci, bc, wpk, m, n, x, y);
  else if (G == 16) k_project<16, 1><<<grid, kBlock, 0, s>>>(prp, pci, bc, wpk, m, n, x, y);
  else if (lmax <= 64) k_project<64, 1><<<grid, kBlock, 0, s>>>(prp, pci, bc, wpk, m, n, x, y);
  else if (lmax <= 128) k_project<64, 2><<<grid, kBlock, 0, s>>>(prp, pci, bc, wpk, m, n, x, y);
  else if (lmax <= 192) k_project<64, 3><<<grid, kBlock, 0, s>>>(prp, pci, bc, wpk, m, n, x, y);
  else if (lmax <= 256) k_project<64, 4><<<grid, kBlock, 0, s>>>(prp, pci, bc, wpk, m, n, x, y);
  else return -1;
  return 0;
}
void launch_sddmm(const int* arp, const int* prp, const int* mrp, const unsigned char* amap,
                  const int* aoff, int n, const double* U, const double* V, double scale,
                  double* Abar, hipStream_t s) {
  if (n > 0) k_sddmm<<<cdiv(n, kBlock), kBlock, 0, s>>>(arp, prp, mrp, amap, aoff, n, U, V, scale, Abar);
}
void launch_diag_grad(const int* arp, const int* aci, const double* av, const int* prp, int n,
                      const double* W, const double* R, double* Abar, hipStream_t s) {
  if (n > 0) k_diag_grad<<<cdiv(n, kBlock), kBlock, 0, s>>>(arp, aci, av, prp, n, W, R, Abar);
}
void launch_restrict(const int* qrp, const int* qci, const int* prp, const int* pci, int n,
                     const double* x, double* out, hipStream_t s) {
  if (n > 0) k_restrict<<<cdiv(n, kBlock), kBlock, 0, s>>>(qrp, qci, prp, pci, n, x, out);
}
void launch_spmv(const int* rp, const int* ci, const double* v, int nrows, const double* x,
                 double* y, hipStream_t s) {
  if (nrows > 0) k_spmv<<<cdiv(nrows, kBlock), kBlock, 0, s>>>(rp, ci, v, nrows, x, y);
}
void launch_col_structure(const int* prp, const int* pci, int n, int nnz, int nc, int* cnt,
                          int* ccp, int* scan_tmp, int* fill, int* cri, int* cpos, hipStream_t s) {
  if (nnz > 0) k_col_count<<<cdiv(nnz, kBlock), kBlock, 0, s>>>(pci, nnz, cnt);
  launch_exclusive_scan(cnt, nc, ccp, scan_tmp, s);
  if (n > 0) k_col_fill<<<cdiv(n, kBlock), kBlock, 0, s>>>(prp, pci, n, ccp, fill, cri, cpos);
  if (nc > 0) k_col_sort<<<cdiv(nc, kBlock), kBlock, 0, s>>>(ccp, nc, cri, cpos);
}
void launch_spmv_t(const int* ccp, const int* cri, const int* cpos, int nc, const double* Pv,
                   const double* z, double* y, hipStream_t s) {
  if (nc > 0) k_spmv_t<<<cdiv(nc, kBlock), kBlock, 0, s>>>(ccp, cri, cpos, nc, Pv, z, y);
}
void launch_spmv_t_dot(const int* ccp, const int* cri, const int* cpos, int nc, const double* Pv,
                       const double* z, const double* p, double* q, double* partials,
                       hipStream_t s) {
  k_spmv_t_dot<<<gsz(nc), kBlock, 0, s>>>(ccp, cri, cpos, nc, Pv, z, p, q, partials);
}
void launch_cg_xr(int nc, const double* rz, const double* pq_part, const double* p,
                  const double* q, const double* dg, double* x, double* r, double* z,
                  double* rz_part, double* rr_part, hipStream_t s) {
  k_cg_xr<<<gsz(nc), kBlock, 0, s>>>(nc, rz, pq_part, gsz(nc), p, q, dg, x, r, z, rz_part, rr_part);
}
void launch_cg_p(int nc, const double* rz_part, const double* rz_old, double* rz_new,
                 const double* z, double* p, hipStream_t s) {
  k_cg_p<<<gsz(nc), kBlock, 0, s>>>(nc, rz_part, gsz(nc), rz_old, rz_new, z, p);
}
void launch_tg_grads(const int* prp, const int* pci, const int* arp, const int* aci, int n,
                     const double* Au, const double* c, const double* u, double s_p, double s_a,
                     double* Pbar, double* Abar, hipStream_t s) {
  if (n <= 0) return;
  if (Pbar) k_tg_pgrad<<<cdiv(n, kBlock), kBlock, 0, s>>>(prp, pci, n, Au, c, s_p, Pbar);
  if (Abar) k_tg_agrad<<<cdiv(n, kBlock), kBlock, 0, s>>>(arp, aci, n, u, s_a, Abar);
}

}  // namespace emin
