// Host-side launch interface of the HIP kernels.  Each kernel file defines
// its launchers; the runtime (runtime.cpp) calls only these.
#pragma once

#include <vector>
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
  kFlagGroups = 7,       // a pattern row is not made of whole aligned column groups
  kFlagGroupsP0 = 8,     // the same, for P0
  kFlagCF = 9,           // a C/F splitting out of range or with a coarse index held twice
  kFlagCFP0 = 10,        // a COARSE row of P0 is not its identity row
  kFlagCFPattern = 11,   // a COARSE row of a given pattern is not its identity column
};

void launch_check_csr(const int* rp, const int* ci, int nrows, int ncols, int nnz, int* flags,
                      int bit, hipStream_t s);
void launch_check_contains(const int* qrp, const int* qci, const int* prp, const int* pci, int n,
                           int* flags, int bit, hipStream_t s);
void launch_row_maxlen(const int* rp, int n, int* out, hipStream_t s);
// *out = max(*out, max of p[0..n)) for non-negative values
void launch_max_int(const int* p, int n, int* out, hipStream_t s);
// Pattern growth in a compressed space: output row o reads A's row o * os,
// visits every ns-th stored entry of it, and the entry's column k names row
// k / td of T.  {1, 1, 1} is the plain row-by-row growth.
struct SymMap {
  int os{1}, ns{1}, td{1};
};
void launch_sym_ub(const int* arp, const int* aci, const int* trp, int n, SymMap sm,
                   int* maxub, hipStream_t s);
// maxub: bound from launch_sym_ub; tmax: longest row of T.  Returns -1 when
// maxub exceeds what the LDS kernels hold.
int launch_sym_rows(const int* arp, const int* aci, const int* trp, const int* tci, int n,
                    SymMap sm, int maxub, int tmax, int* cnt, const int* prp, int* pci,
                    int fill, int grid_cap, hipStream_t s);
// rows of whole aligned groups of G columns -> group ids (nnzc = nnz / G)
void launch_compress_groups(const int* qrp, const int* qci, int n, int nnzc, int G, int* crp,
                            int* cci, hipStream_t s);
// compressed pattern (nrows nodes of R rows, entries = groups of G) -> rows
void launch_expand_pattern(const int* nrp, const int* nci, int nrows, int R, int G, int* prp,
                           int* pci, hipStream_t s);
int scan_tmp_ints(int n);
void launch_exclusive_scan(const int* cnt, int n, int* out, int* tmp, hipStream_t s);

// ------------------------------------------------------------------ setup --
// what: 1 = rows of a node share one pattern row, 2 = A in full aligned blocks
void launch_check_nodes(const int* arp, const int* aci, const int* prp, const int* pci,
                        int nnodes, int bs, int what, int* flags, hipStream_t s);
void launch_diag_has(const int* arp, const int* aci, int n, int* flags, hipStream_t s);

struct SetupArgs {
  const int* arp = nullptr; const int* aci = nullptr; const double* av = nullptr;  // A
  const int* qrp = nullptr; const int* qci = nullptr; const double* qv = nullptr;  // P0
  const int* prp = nullptr; const int* pci = nullptr;                    // pattern
  const double* B = nullptr; const double* bc = nullptr; int m{}; int n{}; int bs{};
  int nbs{};                 // rows per node when a node's rows share one pattern row, else 0
  int ablk{};                // 1: A stored in full aligned nbs x nbs blocks
  double* p0p = nullptr;     // out: corrected tentative prolongation on the pattern
  double* wpk = nullptr;     // out (m > 1): packed pseudo-inverse of each row's Gram matrix
  double* dinv = nullptr;    // out: 1 / A(i,i)
  double* binv = nullptr;    // out (block Jacobi): inverse of each node's diagonal block
  float* avf = nullptr;      // out (mixed): FP32 copy of A's values
  int nnzA{};
  int* fb_list = nullptr;    // scratch: rows whose Gram Cholesky failed (length n)
  int* fb_count = nullptr;   // scratch: one int
  DevState* st = nullptr;
  // batched form: every rank-deficient row is also counted on its matrix
  const int* row_seg = nullptr;
  SegState* segs = nullptr;
  // node set-up: one record of setup_node_record(nbs, m) doubles per node
  // (NULL: the row-wise kernels)
  double* nrec = nullptr;
  // C/F form: coarse index of every row (-1 FINE); COARSE rows are fixed and
  // not counted as rank deficient (NULL: every row free)
  const int* fixed = nullptr;
  int lavg{};  // average pattern row length, rounded up (0: unknown)
};
void launch_setup(const SetupArgs& a, int lmax, int grid_cap, hipStream_t s);
// doubles per node record of the node set-up, 0 when (bs, m) has none
int setup_node_record(int bs, int m);

// ------------------------------------------------------- masked product --
enum K1Mode : int {
  kModeIter = 0, kModeInit = 1, kModeEnergy = 2, kModePlain = 3, kModeRaw = 4, kModeIterRaw = 5
};
// kModePlain: out = Pi mask(A y); kModeRaw: out = mask(A y) (no projector);
// kModeIterRaw (node kernel): kModeIter without the projector -- the update
// kernel projects Y_hat as it reads it, and <Y, mask(A Y)> = <Y, Pi mask(A Y)>
// because Y is in range(Pi)

// Nodes per window of 64 slot pairs (the slot-pair node kernels; their map
// bytes together at most the product's map region).
constexpr int kWinNodes = 3;

struct K1Shape {
  int kind{};   // 0: short rows, column matching (G lanes per row, S slots)
              // 1: node/wave kernel with an LDS hash (long rows)
              // 2: short rows through the precomputed intersection map
              // 4: node blocks, long rows: wave per node through a node-level
              //    intersection map (bs rows per node, L slots per lane)
              // 3: short rows, one lane per row, 16-byte row loads (S <= 8 own
              //    slots, G >= every neighbour row's length, L = neighbours
              //    in flight together)
              // 5: node blocks whose pattern rows are whole groups of an even
              //    number of columns: wave per node, a slot pair per lane,
              //    through a group-level intersection map (L pair chunks;
              //    S > 0: at most S blocks per CU)
  int G{}, S{};   // kind 0, 2 (G lanes per row)
  int bs{}, L{};  // kind 1: rows per node, slots per lane; kind 2: slots per lane
  int packed{}; // kind 0: neighbour rows read through anb (row length <= 15)
  int nwin{};   // kind 5: windows of 64 slot pairs (one wave each)
};
void launch_map_count(const int* arp, const int* prp, int n, int* cnt, hipStream_t s);
void launch_map_fill(const int* arp, const int* aci, const int* prp, const int* pci,
                     const int* mrp, int n, unsigned char* amap, int* aoff, hipStream_t s);
// (pattern-row offset << 4) | row length for every stored entry of A (lengths
// above 15 are stored as 15: kernels that read anb never see such rows)
void launch_build_anb(const int* aci, int nnzA, const int* prp, int* anb, hipStream_t s);

struct K1Args {
  const int* arp = nullptr; const int* aci = nullptr; const void* av = nullptr;
  const int* anb = nullptr;      // per entry of A: (pattern-row offset << 4) | length of the neighbour's row
  const int* mrp = nullptr; const unsigned char* amap{}; const int* aoff = nullptr;  // intersection map (kind 2)
  const long* mrp64 = nullptr;   // kind 4: node map offsets (amap then holds the node map)
  int nnz_p{};                   // kind 4: entries of y (buffer bound)
  const int* nqrp = nullptr; const int2* nq = nullptr;  // kind 4, 5: neighbour node rows
  int grp{};                     // kind 5: columns per group (even)
  const int* win = nullptr;      // kind 5: windows of 64 slot pairs, {first node,
  int nwin{};                    //   its first pair, nodes} each
  const int* prp = nullptr; const int* pci = nullptr;
  const void* y = nullptr; void* out = nullptr;
  const double* bc = nullptr; const double* wpk = nullptr; int m{};
  int n{};               // rows
  double* part_out = nullptr;    // one partial per block (dot products)
  DevState* st = nullptr;
  // segmented (batched) form: per-row dot contributions instead of block
  // partials; optional row list (rows bucketed by pattern length)
  int seg{};             // 1: write rowdot[i], ignore st
  double* rowdot = nullptr;
  const int* rows = nullptr;     // NULL: rows 0..n-1; else n entries of this list
};
// precision: 0 = FP64 everything; 1 = FP32 A / y / out;
// 2 = FP64 A and y, FP32 out (initial residual of the mixed form)
int launch_k1(const K1Shape& sh, int mode, int precision, const K1Args& a, int grid_cap,
              hipStream_t s);
int k1_grid(const K1Shape& sh, int n, int grid_cap);
bool k1_short_supported(int G, int S);
bool k1_wide_supported(int S, int SN, int U);
void launch_nmap_count(const int* arp, const int* prp, int nnodes, int bs, long* cnt,
                       hipStream_t s);
void launch_nmap_fill(const int* arp, const int* aci, const int* prp, const int* pci,
                      const long* nmrp, const int* nqrp, int nnodes, int bs, unsigned char* nmap,
                      int2* nq, hipStream_t s);
int launch_k1_nodemap(int mode, int precision, const K1Shape& sh, const K1Args& a, int grid,
                      hipStream_t s);
// rows made of whole aligned groups of G columns, at most maxg groups a row;
// else sets flag `bit`
void launch_group_check(const int* prp, const int* pci, int n, int G, int maxg, int bit,
                        int* flags, hipStream_t s);
void launch_gmap_count(const int* arp, const int* prp, int nnodes, int bs, int G, long* cnt,
                       int2* shape, hipStream_t s);
void launch_gmap_fill(const int* arp, const int* aci, const int* prp, const int* pci,
                      const long* gmrp, const int* nqrp, int nnodes, int bs, int G,
                      unsigned char* gmap, int2* nq, hipStream_t s);
int launch_k1_nodepair(int mode, int precision, const K1Shape& sh, const K1Args& a, int grid,
                       hipStream_t s);
// whether the node-pair kernel takes nodes with up to max_nb neighbour blocks
// and max_map bytes of (padded) group map
bool nodepair_fits(int max_nb, long max_map);
// shape: {slot pairs, neighbour blocks} per node (launch_gmap_count)
void nodepair_windows(int nnodes, const int2* shape, const long* mapbytes, std::vector<int>& win);
// shapes 0 and 1 by precision and mode (each returns -2 for a pair it does
// not instantiate)
int launch_k1_short_a(int mode, int precision, const K1Shape& sh, const K1Args& a, int grid,
                      hipStream_t s);
int launch_k1_short_b(int mode, int precision, const K1Shape& sh, const K1Args& a, int grid,
                      hipStream_t s);
int launch_k1_hash(int mode, int precision, const K1Shape& sh, const K1Args& a, int grid,
                   hipStream_t s);
void launch_nb_maxlen(const int* arp, const int* aci, const int* prp, int n, int* out,
                      hipStream_t s);
int launch_k1_wide(int mode, int precision, const K1Shape& sh, const K1Args& a, int grid,
                   hipStream_t s);
int launch_k1_mapped(int mode, int precision, const K1Shape& sh, const K1Args& a, int grid,
                     hipStream_t s);

// ------------------------------------------------------ update / direct --
struct UpdArgs {
  const int* prp = nullptr; const int* pci = nullptr;
  const double* dinv = nullptr; const double* binv = nullptr;
  const double* bc = nullptr; const double* wpk = nullptr; int m{}; int n{}; int bs{};
  void* R = nullptr; void* dP = nullptr; void* Y = nullptr; const void* Yh = nullptr;
  const double* part_in = nullptr; int np_in{};   // partials of the previous kernel
  double* part_out = nullptr;                   // this kernel's partials (update only)
  DevState* st = nullptr; DevHist hist{}; int k{}; int k_max{}; double gamma_floor{};
  // segmented (batched) form
  int seg{};             // 1: scalars per segment from segs[], dots to rowdot[]
  const int* seg_row = nullptr; int nseg{}; const SegState* segs = nullptr; double* rowdot = nullptr;
  const int* row_seg = nullptr;  // segment of every row (else found from seg_row)
  int proj_yh{};                 // node kernels: Y_hat (first update: R) arrives unprojected, apply Pi
  const double* r0raw = nullptr; // first update with proj_yh: the raw K P0' in FP64 (else read R)
  const int* win = nullptr; int nwin{};  // slot-pair node kernels: windows of 64 slot pairs
};
struct UpdShape {
  int node{};   // 0: group-per-row Jacobi kernels, 1: wave-per-node block-Jacobi kernels,
                // 2: one lane per row, rows in 4-entry chunks (Jacobi, short rows)
  int G{}, L{};   // node == 0
  int bs{};     // node == 1: rows per node
  int Ln{};     // node == 1: slot chunks per lane (of V slots each)
  int V{1};     // node == 1: consecutive slots per lane (2: pattern rows of whole
                // even-sized column groups, paired 16- / 8-byte accesses)
};
int launch_update(const UpdShape& sh, int first, int mixed, const UpdArgs& a, int grid_cap,
                  hipStream_t s);
int launch_direction(const UpdShape& sh, int first, int mixed, const UpdArgs& a, int grid_cap,
                     hipStream_t s);
int update_grid(const UpdShape& sh, int n, int grid_cap);

// --------------------------------------------- Alg. 1 and the C/F form --
// Alg. 1 on every row: cnt[i] entries (at most m) in cols / vals[i * m ..];
// level[i] (optional) the fitted distance, 0 COARSE, -1 never fitted; flags
// bit 0 when a neighbourhood exceeds the kernel's limits (1024 nodes within
// l_max, 128 COARSE candidates).  -1: m outside 1..8.
int launch_ptent_rows(const int* srp, const int* sci, const int* cf, const double* V, int n,
                      int m, int lmax, int* cnt, int* cols, double* vals, int* level, int* flags,
                      hipStream_t s);
void launch_ptent_compact(const int* cnt, const int* cols, const double* vals, const int* rp,
                          int n, int m, int* colind, double* out, hipStream_t s);
// seen: nc zeroed ints; qrp NULL skips the check of P0's COARSE rows
void launch_cf_check(const int* cf, int n, int nc, int* seen, const int* qrp, const int* qci,
                     const double* qv, int* flags, hipStream_t s);
void launch_cf_count(const int* prp, const int* cf, int n, int* cnt, hipStream_t s);
void launch_cf_fill(const int* prp, const int* pci, const int* cf, int n, const int* rp2,
                    int* ci2, hipStream_t s);
void launch_cf_pattern_check(const int* prp, const int* pci, const int* cf, int n, int* flags,
                             hipStream_t s);
// out[prp[i]] = 1 on COARSE rows (their single identity entry)
void launch_cf_identity(const int* prp, const int* cf, int n, double* out, hipStream_t s);

// ------------------------------------------------ projected SGS (M_2) --
struct SgsArgs {
  const int* arp = nullptr; const int* aci = nullptr; const void* av = nullptr;  // A (T values)
  const int* prp = nullptr; const int* pci = nullptr;                           // pattern
  const int* mrp = nullptr; const unsigned char* amap = nullptr; const int* aoff = nullptr;
  const int* colour = nullptr;  // colour of every row
  const int* rows = nullptr;    // rows sorted by colour, then index
  const unsigned char* erel = nullptr;  // per entry of A: 1 lower colour, 2 higher, 0 diagonal
  int row0{}, nrows{}, c{};     // the sweep's colour: rows[row0 .. row0 + nrows)
  const double* dinv = nullptr;
  const void* x = nullptr;      // forward: R (the residual); finish: R for <R, Z>
  void* u = nullptr;            // forward sweep output, backward base
  void* z = nullptr;            // backward sweep output, finish input
  const double* bc = nullptr; const double* wpk = nullptr; int m{}; int n{};
  void* Z = nullptr;            // finish: Pi z
  double* part_out = nullptr;   // finish: <R, Z> partials
  DevState* st = nullptr;
};
void launch_fill_int(int* p, int n, int v, hipStream_t s);
// one Jones-Plassmann round r over A's graph (rnd, colour: -1 = unpicked);
// *picked += rows picked.  A picked row's colour is sgs_max_colours() when
// every smaller colour is taken by an earlier-picked neighbour.
void launch_jp_round(const int* arp, const int* aci, int n, int r, int* rnd, int* colour,
                     int* picked, hipStream_t s);
int sgs_max_colours();
void launch_entry_rel(const int* arp, const int* aci, const int* colour, int n,
                      unsigned char* rel, hipStream_t s);
// rows of colour c (index order) to rows[base ..]; flags, pos: n ints,
// scan_tmp: scan_tmp_ints(n)
void launch_colour_rows(const int* colour, int n, int c, int* flags, int* pos, int* scan_tmp,
                        int base, int* rows, hipStream_t s);
int launch_sgs_sweep(int forward, int mixed, int G, int L, const SgsArgs& a, int grid_cap,
                     hipStream_t s);
int launch_sgs_finish(int mixed, int G, int L, const SgsArgs& a, int grid_cap, hipStream_t s);
int sgs_finish_grid(int G, int n, int grid_cap);
void launch_sgs_update(int first, int mixed, const UpdArgs& a, int nnz, int grid_cap,
                       hipStream_t s);
void launch_sgs_direction(int first, int mixed, const UpdArgs& a, const void* Z, int nnz,
                          int grid_cap, hipStream_t s);

struct FinalArgs {
  const int* prp = nullptr; const int* pci = nullptr; const double* p0p = nullptr; const void* dP = nullptr;
  const double* B = nullptr; const double* bc = nullptr; const double* wpk = nullptr; int m{}; int n{};
  double* out = nullptr;
  int nbs{};   // rows per node when a node's rows share one pattern row, else 0
  int lmax{};  // longest pattern row (the node form needs it)
  int pairs{}; // 1: pattern rows of whole even-sized column groups at even offsets
};
// reproject: correct every row back onto the constraint in FP64 (always done
// for the mixed form)
int launch_final(int G, int L, int mixed, int reproject, const FinalArgs& a, int grid_cap,
                 hipStream_t s);

struct ConsArgs {
  const int* prp = nullptr; const int* pci = nullptr; const double* P = nullptr; const double* B = nullptr; const double* bc = nullptr;
  int m{}; int n{}; double* part_num = nullptr; double* part_den = nullptr;
};
int launch_constraint(int G, int L, const ConsArgs& a, int grid_cap, hipStream_t s);
int constraint_grid(int G, int n, int grid_cap);
// out[0] = sum of partials[0..np) (one block, fixed order)
void launch_reduce(const double* partials, int np, double* out, hipStream_t s);

void launch_state_init(DevState* st, double tau, hipStream_t s);

// ---------------------------------------------------------------- adjoint --
void launch_axpby(int n, double a, const double* x, double b, double* y, hipStream_t s);
int dot_grid(int n);
// y = (amul * *as) x + b y (coefficient in device memory)
void launch_axpby_s(int n, const double* as, double amul, const double* x, double b, double* y,
                    hipStream_t s);
// reverse-sweep scalars on the device, sc = [gnext, gbar, abar, dbar] (see adjoint.hip)
void launch_bwd_scalars(int stage, const double* p1, int n1, const double* p2, int n2, double g,
                        double dl, double gprev, double* sc, hipStream_t s);
void launch_dot(int n, const double* x, const double* y, double* partials, hipStream_t s);
void launch_div(int n, const double* x, const double* d, double* y, hipStream_t s);
void launch_mul(int n, const double* x, const double* y, double* z, hipStream_t s);
void launch_rowscale(const int* prp, const double* dinv, int n, const double* x, double c,
                     double* y, hipStream_t s);
int launch_project(const int* prp, const int* pci, const double* bc, const double* wpk, int m,
                   int n, int lmax, const double* x, double* y, hipStream_t s);
void launch_sddmm(const int* arp, const int* prp, const int* mrp, const unsigned char* amap,
                  const int* aoff, int n, const double* U, const double* V, double scale,
                  double* Abar, hipStream_t s);
void launch_diag_grad(const int* arp, const int* aci, const double* av, const int* prp, int n,
                      const double* W, const double* R, double* Abar, hipStream_t s);
void launch_restrict(const int* qrp, const int* qci, const int* prp, const int* pci, int n,
                     const double* x, double* out, hipStream_t s);
void launch_spmv(const int* rp, const int* ci, const double* v, int nrows, const double* x,
                 double* y, hipStream_t s);
void launch_col_structure(const int* prp, const int* pci, int n, int nnz, int nc, int* cnt,
                          int* ccp, int* scan_tmp, int* fill, int* cri, int* cpos, hipStream_t s);
void launch_spmv_t(const int* ccp, const int* cri, const int* cpos, int nc, const double* Pv,
                   const double* z, double* y, hipStream_t s);
// coarse CG of the two-grid loss: every kernel runs on dot_grid(nc) blocks,
// so the per-block partials of one are summed in full by the next
void launch_spmv_t_dot(const int* ccp, const int* cri, const int* cpos, int nc, const double* Pv,
                       const double* z, const double* p, double* q, double* partials,
                       hipStream_t s);
void launch_cg_xr(int nc, const double* rz, const double* pq_part, const double* p,
                  const double* q, const double* dg, double* x, double* r, double* z,
                  double* rz_part, double* rr_part, hipStream_t s);
void launch_cg_p(int nc, const double* rz_part, const double* rz_old, double* rz_new,
                 const double* z, double* p, hipStream_t s);
void launch_tg_grads(const int* prp, const int* pci, const int* arp, const int* aci, int n,
                     const double* Au, const double* c, const double* u, double s_p, double s_a,
                     double* Pbar, double* Abar, hipStream_t s);

// ------------------------------------------------------------------ batch --
// rows per first-stage chunk of the per-segment reductions
constexpr int kSegChunk = 2048;
struct SegArgs {
  const int* seg_row = nullptr; int nseg{}; const double* rowdot = nullptr; SegState* segs = nullptr;
  double* hist = nullptr; int hist_len{}; int k{}; double tau{}; double gamma_floor{};
  // chunks of up to kSegChunk rows inside the segments: row bounds
  // (nchunk + 1), each segment's chunk range (nseg + 1), chunk sums (nchunk)
  const int* chunk_row = nullptr; const int* seg_chunk = nullptr; double* chunk_sum = nullptr;
  int nchunk{};
};
void launch_seg_init(SegState* segs, int nseg, hipStream_t s);
void launch_seg_delta(const SegArgs& a, hipStream_t s);
void launch_seg_gamma(const SegArgs& a, int first, hipStream_t s);
// dst[off[b] + j] = src[b][j] for j < off[b+1] - off[b], b < count (one block per b)
void launch_gather_segments(const double* const* src, const long* off, int count, double* dst,
                            hipStream_t s);
void launch_scatter_segments(const double* src, const long* off, int count, double* const* dst,
                             hipStream_t s);
// out[off_dst + j] = in[j] + add, over count ranges (structure concatenation)
void launch_shift_copy(const int* in, int len, int add, int* out, hipStream_t s);
void launch_gather_map(const double* const* src, const long* off, const int* map, int count,
                       double* dst, hipStream_t s);
void launch_scatter_map(const double* src, const long* off, const int* map, int count,
                        double* const* dst, hipStream_t s);

}  // namespace emin
