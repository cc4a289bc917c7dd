// Host-side launch interface of the HIP kernels.  Each kernel file defines
// its launchers; the runtime (runtime.cpp) calls only these.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace emin {

// ---------------------------------------------------------------- pattern --
enum FlagBit : int {
  kFlagCsrA = 0,
  kFlagCsrP0 = 1,
  kFlagCsrPat = 2,
  kFlagContains = 3,
  kFlagNoDiag = 4,
  kFlagNodePattern = 5,  // rows of a node do not share one column set
  kFlagNodeA = 6,        // A is not stored as full aligned node blocks
};

void launch_check_csr(const int* rp, const int* ci, int nrows, int ncols, int nnz, int* flags,
                      int bit, hipStream_t s);
void launch_check_contains(const int* qrp, const int* qci, const int* prp, const int* pci, int n,
                           int* flags, int bit, hipStream_t s);
void launch_row_maxlen(const int* rp, int n, int* out, hipStream_t s);
void launch_sym_ub(const int* arp, const int* aci, const int* trp, int n, int* maxub,
                   hipStream_t s);
int launch_sym_rows(const int* arp, const int* aci, const int* trp, const int* tci, int n,
                    int maxub, int* cnt, const int* prp, int* pci, int fill, int grid_cap,
                    hipStream_t s);
int scan_tmp_ints(int n);
void launch_exclusive_scan(const int* cnt, int n, int* out, int* tmp, hipStream_t s);

// ------------------------------------------------------------------ setup --
void launch_check_nodes(const int* arp, const int* aci, const int* prp, const int* pci,
                        int nnodes, int bs, int* flags, hipStream_t s);
void launch_diag_has(const int* arp, const int* aci, int n, int* flags, hipStream_t s);

struct SetupArgs {
  const int* arp; const int* aci; const double* av;  // A
  const int* qrp; const int* qci; const double* qv;  // P0
  const int* prp; const int* pci;                    // pattern
  const double* B; const double* bc; int m; int n; int bs;
  double* p0p;     // out: corrected tentative prolongation on the pattern
  double* wpk;     // out (m > 1): packed pseudo-inverse of each row's Gram matrix
  double* dinv;    // out: 1 / A(i,i)
  double* binv;    // out (block Jacobi): inverse of each node's diagonal block
  float* avf;      // out (mixed): FP32 copy of A's values
  int nnzA;
  int* fb_list;    // scratch: rows whose Gram Cholesky failed (length n)
  int* fb_count;   // scratch: one int
  DevState* st;
};
void launch_setup(const SetupArgs& a, int lmax, int grid_cap, hipStream_t s);

// ------------------------------------------------------- masked product --
enum K1Mode : int { kModeIter = 0, kModeInit = 1, kModeEnergy = 2, kModePlain = 3 };

struct K1Shape {
  int kind;   // 0: short rows, column matching (G lanes per row, S slots)
              // 1: node/wave kernel with an LDS hash (long rows)
              // 2: short rows through the precomputed intersection map
  int G, S;   // kind 0, 2 (G lanes per row)
  int bs, L;  // kind 1: rows per node, slots per lane; kind 2: slots per lane
  int packed; // kind 0: neighbour rows read through anb (row length <= 15)
};
void launch_map_count(const int* arp, const int* prp, int n, int* cnt, hipStream_t s);
void launch_map_fill(const int* arp, const int* aci, const int* prp, const int* pci,
                     const int* mrp, int n, unsigned char* amap, int* aoff, hipStream_t s);
// (pattern-row offset << 4) | row length for every stored entry of A
void launch_build_anb(const int* aci, int nnzA, const int* prp, int* anb, hipStream_t s);

struct K1Args {
  const int* arp; const int* aci; const void* av;
  const int* anb;      // per entry of A: (pattern-row offset << 4) | length of the neighbour's row
  const int* mrp; const unsigned char* amap; const int* aoff;  // intersection map (kind 2)
  const int* prp; const int* pci;
  const void* y; void* out;
  const double* bc; const double* wpk; int m;
  int n;               // rows
  double* part_out;    // one partial per block (dot products)
  DevState* st;
};
// precision: 0 = FP64 everything; 1 = FP32 A / y / out;
// 2 = FP64 A and y, FP32 out (initial residual of the mixed form)
int launch_k1(const K1Shape& sh, int mode, int precision, const K1Args& a, int grid_cap,
              hipStream_t s);
int k1_grid(const K1Shape& sh, int n, int grid_cap);
int launch_k1_mapped(int mode, int precision, const K1Shape& sh, const K1Args& a, int grid,
                     hipStream_t s);

// ------------------------------------------------------ update / direct --
struct UpdArgs {
  const int* prp; const int* pci;
  const double* dinv; const double* binv;
  const double* bc; const double* wpk; int m; int n; int bs;
  void* R; void* dP; void* Y; const void* Yh;
  const double* part_in; int np_in;   // partials of the previous kernel
  double* part_out;                   // this kernel's partials (update only)
  DevState* st; DevHist hist; int k; int k_max; double gamma_floor;
};
struct UpdShape {
  int node;   // 0: group-per-row Jacobi kernels, 1: wave-per-node block-Jacobi kernels
  int G, L;   // node == 0
  int bs;     // node == 1: rows per node
  int Ln;     // node == 1: slots per lane
};
int launch_update(const UpdShape& sh, int first, int mixed, const UpdArgs& a, int grid_cap,
                  hipStream_t s);
int launch_direction(const UpdShape& sh, int first, int mixed, const UpdArgs& a, int grid_cap,
                     hipStream_t s);
int update_grid(const UpdShape& sh, int n, int grid_cap);

struct FinalArgs {
  const int* prp; const int* pci; const double* p0p; const void* dP;
  const double* B; const double* bc; const double* wpk; int m; int n;
  double* out;
};
int launch_final(int G, int L, int mixed, const FinalArgs& a, int grid_cap, hipStream_t s);

struct ConsArgs {
  const int* prp; const int* pci; const double* P; const double* B; const double* bc;
  int m; int n; double* part_num; double* part_den;
};
int launch_constraint(int G, int L, const ConsArgs& a, int grid_cap, hipStream_t s);
int constraint_grid(int G, int n, int grid_cap);
// out[0] = sum of partials[0..np) (one block, fixed order)
void launch_reduce(const double* partials, int np, double* out, hipStream_t s);

void launch_state_init(DevState* st, double tau, hipStream_t s);

}  // namespace emin
