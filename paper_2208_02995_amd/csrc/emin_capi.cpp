// Host runtime and the extern "C" entry points declared in include/emin.h.
//
// A context owns a HIP stream handle (borrowed), the device properties used to
// size grids, and a caching device-memory pool so that creating and
// destroying problems of the same shape does not go back to hipMalloc.
// A problem is the symbolic phase (validated structure, grown pattern, kernel
// shapes, workspace); emin_solve is the numeric phase (Alg. 2 then Alg. 3),
// enqueued without host round trips until the final read-back of the scalars.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/emin.h"
#include "launch.hpp"

using namespace emin;

namespace {

thread_local std::string g_err;

emin_status fail(emin_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define EMIN_HIP(call)                                                                    \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? EMIN_ERR_OOM : EMIN_ERR_HIP,                \
                  std::string(#call) + ": " + hipGetErrorString(e_));                     \
  } while (0)

#define EMIN_TRY(expr)                 \
  do {                                 \
    emin_status s_ = (expr);           \
    if (s_ != EMIN_OK) return s_;      \
  } while (0)

int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Caching allocator: blocks are kept on per-size free lists and reused.
struct Pool {
  std::map<size_t, std::vector<void*>> free_;
  std::map<void*, size_t> size_;
  emin_status get(size_t bytes, void** out) {
    // at least 64 bytes of slack past every request: the row kernels may
    // read a few entries beyond a row's end (never use them)
    bytes = ((bytes + 64 + 255) / 256) * 256;
    auto it = free_.find(bytes);
    if (it != free_.end() && !it->second.empty()) {
      *out = it->second.back();
      it->second.pop_back();
      return EMIN_OK;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      // release cached blocks and retry once
      release_all();
      e = hipMalloc(&p, bytes);
      if (e != hipSuccess) return fail(EMIN_ERR_OOM, "hipMalloc failed");
    }
    size_[p] = bytes;
    *out = p;
    return EMIN_OK;
  }
  void put(void* p) {
    if (!p) return;
    auto it = size_.find(p);
    if (it == size_.end()) return;
    free_[it->second].push_back(p);
  }
  void release_all() {
    for (auto& kv : free_)
      for (void* p : kv.second) {
        size_.erase(p);
        (void)hipFree(p);
      }
    free_.clear();
  }
  ~Pool() {
    release_all();
    for (auto& kv : size_) (void)hipFree(kv.first);
  }
};

}  // namespace

struct emin_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 256;
  int grid_cap = 2048;
  Pool pool;
  // pinned host staging for the per-pattern tables the host builds (grown
  // on demand, kept until the context ends)
  void* pin = nullptr;
  size_t pin_bytes = 0;
  emin_status pinned(size_t bytes, void** out) {
    if (bytes > pin_bytes) {
      if (pin) (void)hipHostFree(pin);
      pin = nullptr;
      pin_bytes = 0;
      if (hipHostMalloc(&pin, bytes, hipHostMallocDefault) != hipSuccess)
        return fail(EMIN_ERR_HIP, "hipHostMalloc failed");
      pin_bytes = bytes;
    }
    *out = pin;
    return EMIN_OK;
  }
  ~emin_ctx() {
    if (pin) (void)hipHostFree(pin);
  }
};

struct emin_problem {
  emin_ctx* ctx = nullptr;
  int n = 0, nc = 0, m = 0, nnzA = 0, nnzP0 = 0, nnzP = 0;
  const int *arp = nullptr, *aci = nullptr;
  const double* av = nullptr;
  const int *qrp = nullptr, *qci = nullptr;
  const double* qv = nullptr;
  const double *B = nullptr, *bc = nullptr;
  emin_opts opts{};
  // owned
  std::vector<void*> owned;
  int *prp = nullptr, *pci = nullptr;
  double *p0p = nullptr, *wpk = nullptr, *dinv = nullptr, *binv = nullptr;
  float* avf = nullptr;
  void *Y = nullptr, *Yh = nullptr, *R = nullptr, *dP = nullptr;
  double* part_d = nullptr;  // masked-product partials (<Y, Y_hat>)
  double* part_g = nullptr;  // update partials (<R, Z>)
  int* anb = nullptr;        // packed neighbour-row descriptors (short rows)
  double* stage = nullptr;   // FP64 copy of a caller's array on the pattern
  double* nrec = nullptr;    // node set-up records (rows of a node share a pattern row)
  // projected SGS: colour of every row, rows sorted by colour, colour offsets
  int* colour = nullptr;
  int* crows = nullptr;
  unsigned char* erel = nullptr;  // per entry of A: neighbour's colour lower (1) / higher (2)
  std::vector<int> coff;
  void *U = nullptr, *Zs = nullptr;  // forward-sweep values; backward values, then Pi z
  int* cfix = nullptr;  // C/F form: coarse index of every row, -1 FINE (COARSE rows fixed)
  double* r0d = nullptr;     // mixed node form: the initial raw K P0' in FP64
  long* nmrp = nullptr;             // node-level intersection map (node kernel)
  unsigned char* nmap = nullptr;
  int* nqrp = nullptr;              // per node: first neighbour-block descriptor
  int2* nq = nullptr;               // per neighbour block: (pattern row start, length)
  long* gmrp = nullptr;             // group-level intersection map (node-pair kernel)
  unsigned char* gmap = nullptr;
  int* win = nullptr;               // node-pair kernel: windows of 64 slot pairs (p->k1.nwin)
  int grp = 0;                      // columns per group when every pattern row is made of
                                    // whole aligned groups of an even size (else 0)
  int* mrp = nullptr;        // intersection map: row offsets (n + 1)
  unsigned char* amap = nullptr;
  int* aoff = nullptr;       // pattern-row offset of each entry's neighbour
  // column structure of the pattern (two-grid loss), built on demand
  int *ccp = nullptr, *cri = nullptr, *cpos = nullptr;
  DevState* st = nullptr;
  double* hist = nullptr;
  int* flags = nullptr;
  int* ints = nullptr;  // small device scratch (maxima)
  int* fb_list = nullptr;
  int* fb_count = nullptr;
  int lmax = 0, amax = 0, hist_len = 1;
  bool node_ok_pattern = false, node_ok_A = false;
  bool have_factors = false;
  K1Shape k1{};
  UpdShape upd{};
  int rowG = 1, rowL = 1;  // group shape for row kernels (final, constraint)
  hipEvent_t ev[2] = {nullptr, nullptr};
  std::vector<hipEvent_t> kev;

  emin_status alloc(size_t bytes, void** p) {
    EMIN_TRY(ctx->pool.get(bytes, p));
    owned.push_back(*p);
    return EMIN_OK;
  }
  ~emin_problem() {
    for (void* p : owned) ctx->pool.put(p);
    for (hipEvent_t e : kev) (void)hipEventDestroy(e);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

// Record of one FP64 solve for the reverse sweep: Y_k and R_k of every
// applied iteration, the CG scalars, and the values the solve used (P0',
// A's values, 1/A_ii), so later solves on the same problem do not disturb
// it.  Memory (2 k + 1) nnz(P) + nnz(A) + n doubles.
struct emin_tape {
  emin_problem* p = nullptr;
  int iters = 0, slots = 0;
  double *Y = nullptr, *R = nullptr, *p0p = nullptr, *av = nullptr, *dinv = nullptr;
  std::vector<double> gamma, delta, alpha, beta;
  std::vector<void*> owned;
  // backward work arrays
  double *Ybar = nullptr, *Ynext = nullptr, *Rbar = nullptr, *Rnext = nullptr, *Yhbar = nullptr,
         *U = nullptr, *Zbar = nullptr, *Z = nullptr, *Yh = nullptr, *p0bar = nullptr,
         *part = nullptr, *res = nullptr;
  emin_status alloc(size_t bytes, double** d) {
    void* v;
    EMIN_TRY(p->ctx->pool.get(bytes, &v));
    owned.push_back(v);
    *d = (double*)v;
    return EMIN_OK;
  }
  ~emin_tape() {
    for (void* v : owned) p->ctx->pool.put(v);
  }
};

namespace {

emin_status read_flags(emin_problem* p, int* host) {
  EMIN_HIP(hipMemcpyAsync(host, p->flags, sizeof(int), hipMemcpyDeviceToHost, p->ctx->stream));
  EMIN_HIP(hipStreamSynchronize(p->ctx->stream));
  return EMIN_OK;
}

emin_status check_csr_host(const emin_csr* c, const char* name, int64_t rows, int64_t cols) {
  if (!c) return fail(EMIN_ERR_ARG, std::string(name) + " is NULL");
  if (c->n_rows != rows || c->n_cols != cols)
    return fail(EMIN_ERR_SHAPE, std::string(name) + " has the wrong shape");
  if (c->nnz < 0 || c->nnz > 0x7fffffff || c->n_rows > 0x7ffffffe || c->n_cols > 0x7ffffffe)
    return fail(EMIN_ERR_ARG, std::string(name) + ": sizes exceed int32 indexing");
  if (!c->rowptr || (c->nnz > 0 && !c->colind))
    return fail(EMIN_ERR_ARG, std::string(name) + ": NULL rowptr/colind");
  return EMIN_OK;
}

// struct(A T) in the space of `sm` (nout output rows) into freshly allocated
// (rp, ci); returns nnz and the longest output row.  tmax: longest row of T.
// ub_hint > 0: a known upper bound of the candidates per row (used as is,
// saving the bound kernel and a host round trip).
emin_status symbolic(emin_problem* p, SymMap sm, int nout, const int* trp, const int* tci,
                     int tmax, int ub_hint, int** rp_out, int** ci_out, int* nnz_out,
                     int* tmax_out) {
  emin_ctx* c = p->ctx;
  hipStream_t s = c->stream;
  int maxub = ub_hint;
  if (maxub <= 0) {
    EMIN_HIP(hipMemsetAsync(p->ints, 0, 4 * sizeof(int), s));
    launch_sym_ub(p->arp, p->aci, trp, nout, sm, p->ints, s);
    EMIN_HIP(hipMemcpyAsync(&maxub, p->ints, sizeof(int), hipMemcpyDeviceToHost, s));
    EMIN_HIP(hipStreamSynchronize(s));
  }
  if (maxub > 4096)
    return fail(EMIN_ERR_UNSUPPORTED, "pattern growth: a row collects more than 4096 candidate "
                                      "columns (" + std::to_string(maxub) + ")");
  void *cnt, *rp, *tmp;
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)std::max(nout, 1), &cnt));
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)(nout + 1), &rp));
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)scan_tmp_ints(nout), &tmp));
  if (launch_sym_rows(p->arp, p->aci, trp, tci, nout, sm, maxub, tmax, (int*)cnt, nullptr,
                      nullptr, 0, c->grid_cap, s))
    return fail(EMIN_ERR_UNSUPPORTED, "pattern growth: row too long");
  launch_exclusive_scan((int*)cnt, nout, (int*)rp, (int*)tmp, s);
  EMIN_HIP(hipMemsetAsync(p->ints + 1, 0, sizeof(int), s));
  launch_row_maxlen((int*)rp, nout, p->ints + 1, s);
  int nnz = 0, lmax = 0;
  EMIN_HIP(hipMemcpyAsync(&nnz, (int*)rp + nout, sizeof(int), hipMemcpyDeviceToHost, s));
  EMIN_HIP(hipMemcpyAsync(&lmax, p->ints + 1, sizeof(int), hipMemcpyDeviceToHost, s));
  EMIN_HIP(hipStreamSynchronize(s));
  if (nnz < 0) return fail(EMIN_ERR_UNSUPPORTED, "pattern has more than 2^31 entries");
  void* ci;
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)std::max(nnz, 1), &ci));
  launch_sym_rows(p->arp, p->aci, trp, tci, nout, sm, maxub, tmax, nullptr, (int*)rp, (int*)ci,
                  1, c->grid_cap, s);
  EMIN_HIP(hipGetLastError());
  *rp_out = (int*)rp;
  *ci_out = (int*)ci;
  *nnz_out = nnz;
  *tmax_out = lmax;
  return EMIN_OK;
}

// Pattern growth S^k P0 (Sec. 3, eq. enlPatt), in the compressed space the
// structure allows (node rows when A is stored in full aligned bs-blocks,
// group ids when every row of P0 is whole aligned groups of m columns), then
// expanded to rows.  *node_grown / *group_grown report which applied;
// *a_checked that A's block structure was checked (flag kFlagNodeA).
emin_status grow_pattern(emin_problem* p, int amax, int qmax, bool* node_grown,
                         bool* group_grown, bool* a_checked) {
  hipStream_t s = p->ctx->stream;
  const int n = p->n, m = p->m;
  const int bs = std::max(1, p->opts.block);
  bool node = bs > 1 && bs <= 64 && n % bs == 0;
  bool group = m > 1;
  *a_checked = node;
  if (node) launch_check_nodes(p->arp, p->aci, nullptr, nullptr, n / bs, bs, 2, p->flags, s);
  if (group)
    launch_group_check(p->qrp, p->qci, n, m, INT_MAX, kFlagGroupsP0, p->flags, s);
  if (node || group) {
    EMIN_HIP(hipGetLastError());
    int fl = 0;
    EMIN_TRY(read_flags(p, &fl));
    node = node && !(fl & (1 << kFlagNodeA));
    group = group && !(fl & (1 << kFlagGroupsP0));
  }
  const int G = group ? m : 1;
  const int* trp = p->qrp;
  const int* tci = p->qci;
  int tmax = qmax;
  if (group) {
    void *crp, *cci;
    const int nnzc = p->nnzP0 / G;
    EMIN_TRY(p->alloc(sizeof(int) * (size_t)(n + 1), &crp));
    EMIN_TRY(p->alloc(sizeof(int) * (size_t)std::max(nnzc, 1), &cci));
    launch_compress_groups(p->qrp, p->qci, n, nnzc, G, (int*)crp, (int*)cci, s);
    trp = (const int*)crp;
    tci = (const int*)cci;
    tmax = qmax / G;
  }
  const int nout = node ? n / bs : n;
  int *rp = nullptr, *ci = nullptr, nnz = 0;
  for (int step = 0; step < p->opts.pattern_power; ++step) {
    // from the second node-level step on, T is indexed by node: one visit
    // per neighbour block
    const int sub = (node && step > 0) ? bs : 1;
    const SymMap sm{node ? bs : 1, sub, sub};
    // candidates per row are at most (selected entries of A's row) x
    // (longest row of T); used as the bound when it is small enough
    const long loose = (long)((amax + sub - 1) / sub) * tmax;
    const int hint = (loose > 0 && loose <= (step == 0 ? 4096 : 512)) ? (int)loose : 0;
    EMIN_TRY(symbolic(p, sm, nout, trp, tci, tmax, hint, &rp, &ci, &nnz, &tmax));
    trp = rp;
    tci = ci;
  }
  if (node || group) {
    const int R = node ? bs : 1;
    const int64_t full = (int64_t)nnz * G * R;
    if (full >= (int64_t(1) << 31))
      return fail(EMIN_ERR_UNSUPPORTED, "pattern has more than 2^31 entries");
    void *prp, *pci;
    EMIN_TRY(p->alloc(sizeof(int) * (size_t)(n + 1), &prp));
    EMIN_TRY(p->alloc(sizeof(int) * (size_t)std::max<int64_t>(full, 1), &pci));
    launch_expand_pattern(rp, ci, nout, R, G, (int*)prp, (int*)pci, s);
    EMIN_HIP(hipGetLastError());
    p->prp = (int*)prp;
    p->pci = (int*)pci;
    p->nnzP = (int)full;
  } else {
    p->prp = rp;
    p->pci = ci;
    p->nnzP = nnz;
  }
  *node_grown = node;
  *group_grown = group;
  return EMIN_OK;
}

K1Shape map_shape(const emin_problem* p);
emin_status ensure_map(emin_problem* p, hipStream_t s);

// Kernel shapes from the row-length profile of the pattern and of A.
void choose_shapes(emin_problem* p) {
  const int lmax = std::max(p->lmax, 1);
  const double avgA = p->n ? (double)p->nnzA / p->n : 1.0;
  // masked product
  if (lmax <= 32 && !(p->opts.precond == EMIN_BJACOBI && p->node_ok_A && p->node_ok_pattern &&
                      p->opts.block > 1 && lmax > 8)) {
    int S = next_pow2(lmax);
    // about two neighbours per lane per pass of the unrolled-by-two loop
    int G = std::min(S, std::max(1, next_pow2((int)std::lround(avgA)) / 4));
    if (G * 4 < S) G = S / 4;
    if (p->opts.k1_group > 0) G = p->opts.k1_group;
    if (p->opts.k1_slots >= S) S = p->opts.k1_slots;
    if (!k1_short_supported(G, S)) G = S;  // (S, S) exists for every power of two <= 32
    const bool packed = lmax <= 15 && S <= 16 && (int64_t)p->nnzP < (int64_t(1) << 27);
    p->k1 = {0, G, S, 1, 1, packed ? 1 : 0};
    if (p->opts.k1_slots < 0 || lmax > 16) {
      // precomputed intersection map, one lane per slot
      int Gm = next_pow2(lmax);
      if (p->opts.k1_group > 0 && p->opts.k1_group <= 64) Gm = p->opts.k1_group;
      int Lm = (lmax + Gm - 1) / Gm;
      if (Lm > 2) { Gm = std::min(64, next_pow2(lmax)); Lm = (lmax + Gm - 1) / Gm; }
      p->k1 = {2, Gm, Gm * Lm, 1, Lm, 0};
    }
    // one lane per row with 16-byte row loads: the default for rows up to 8
    const bool hinted = p->opts.k1_group != 0 || p->opts.k1_slots != 0;
    if ((!hinted || p->opts.k1_group == -2) && lmax <= 8 &&
        (int64_t)p->nnzP < (int64_t(1) << 27)) {
      const int Sw = std::max(4, next_pow2(lmax));
      const int U = (p->opts.k1_group == -2 && p->opts.k1_slots == 8) ? 8 : 4;
      p->k1 = {3, Sw, Sw, 1, U, 1};
    }
  } else {
    const int bs = (p->node_ok_A && p->node_ok_pattern && p->opts.block > 1 &&
                    p->opts.block <= 3) ? p->opts.block : 1;
    p->k1 = {1, 0, 0, bs, (lmax + 63) / 64, 0};
    // node blocks: the node-level intersection map (positions fit a byte)
    if (bs >= 2 && lmax <= 255 && p->opts.k1_slots != -3 &&
        (int64_t)p->nnzP * 8 < (int64_t(1) << 31)) {
      int U = bs == 3 ? 1 : 2;  // neighbour blocks per pipelined step
      if (bs == 3 && (p->opts.k1_group == 2 || p->opts.k1_group == 4)) U = p->opts.k1_group;
      if (p->opts.k1_group == -4) U = 0;  // three-deep single-block pipeline
      p->k1 = {4, U, 0, bs, (lmax + 63) / 64, 0};
      // pattern rows of whole even-sized column groups: slot pairs through the
      // group-level map (block-Jacobi, whose update applies the projector)
      const bool hinted4 = p->opts.k1_group == -4 || p->opts.k1_group == -5 ||
                           p->opts.k1_group == 2 || p->opts.k1_group == 4;
      if (p->grp > 0 && p->opts.precond == EMIN_BJACOBI && !hinted4) {
        // G: neighbour blocks in flight (measured on the 40^3 elasticity
        // case: two for FP64, four for FP32); S = 0: no cap on blocks per CU
        // (registers and LDS allow four for FP64 there)
        const int depth = p->opts.k1_group <= -6 && p->opts.k1_group >= -8
                              ? -4 - p->opts.k1_group
                              : (p->opts.precision == EMIN_FP64 ? 2 : 4);
        p->k1 = {5, depth, 0, bs, (lmax / 2 + 63) / 64, 0};
      }
    }
  }
  // projected SGS: the update applies no preconditioner, and the sweeps use
  // the intersection map; the node products (which leave Pi to the node
  // update) give way to the map product
  if (p->opts.precond == EMIN_SGS && (p->k1.kind == 1 || p->k1.kind == 4 || p->k1.kind == 5))
    p->k1 = map_shape(p);
  // row-wise kernels: G lanes per row with L slots each
  p->rowG = std::min(64, next_pow2(lmax));
  p->rowL = (lmax + p->rowG - 1) / p->rowG;
  if (p->opts.precond == EMIN_JACOBI || p->opts.precond == EMIN_SGS) {
    p->upd = {0, p->rowG, p->rowL, 1, 1};
    if (lmax <= 16) p->upd = {2, 1, 1, 1, 1};  // one lane per row, 4-entry chunks
  } else if (p->k1.kind == 5) {
    p->upd = {1, 0, 0, p->opts.block, (lmax / 2 + 63) / 64, 2};
  } else {
    p->upd = {1, 0, 0, p->opts.block, (lmax + 63) / 64, 1};
  }
}

// Intersection map of the masked product (see mapped.hip): for every row,
// (A row length) x (pattern row length) bytes.  Built once per pattern.
emin_status build_map(emin_problem* p, hipStream_t s, bool* too_big) {
  void* v;
  *too_big = false;
  EMIN_TRY(p->alloc((size_t)(p->n + 1) * sizeof(int), &v));
  p->mrp = (int*)v;
  void *cnt, *tmp;
  EMIN_TRY(p->alloc((size_t)std::max(p->n, 1) * sizeof(int), &cnt));
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)scan_tmp_ints(p->n), &tmp));
  launch_map_count(p->arp, p->prp, p->n, (int*)cnt, s);
  launch_exclusive_scan((int*)cnt, p->n, p->mrp, (int*)tmp, s);
  int total = 0;
  EMIN_HIP(hipMemcpyAsync(&total, p->mrp + p->n, sizeof(int), hipMemcpyDeviceToHost, s));
  EMIN_HIP(hipStreamSynchronize(s));
  if (total < 0) {
    *too_big = true;
    return EMIN_OK;
  }
  EMIN_TRY(p->alloc((size_t)std::max(total, 1), &v));
  p->amap = (unsigned char*)v;
  EMIN_TRY(p->alloc((size_t)std::max(p->nnzA, 1) * sizeof(int), &v));
  p->aoff = (int*)v;
  launch_map_fill(p->arp, p->aci, p->prp, p->pci, p->mrp, p->n, p->amap, p->aoff, s);
  EMIN_HIP(hipGetLastError());
  return EMIN_OK;
}

// Node-level intersection map (see nodemap.hip): for every node, (node
// blocks in A's row) x (pattern row length) bytes, with 64-bit offsets.
emin_status build_nmap(emin_problem* p, hipStream_t s) {
  const int bs = p->k1.bs;
  const int nnodes = p->n / bs;
  void* v;
  EMIN_TRY(p->alloc(sizeof(long) * (size_t)(nnodes + 1), &v));
  p->nmrp = (long*)v;
  std::vector<long> cnt(std::max(nnodes, 1)), off(nnodes + 1, 0);
  std::vector<int> hrp(nnodes * bs + 1 > 0 ? (size_t)nnodes * bs + 1 : 1), qoff(nnodes + 1, 0);
  launch_nmap_count(p->arp, p->prp, nnodes, bs, p->nmrp, s);
  EMIN_HIP(hipMemcpyAsync(cnt.data(), p->nmrp, sizeof(long) * nnodes, hipMemcpyDeviceToHost, s));
  EMIN_HIP(hipMemcpyAsync(hrp.data(), p->arp, sizeof(int) * ((size_t)nnodes * bs + 1),
                          hipMemcpyDeviceToHost, s));
  EMIN_HIP(hipStreamSynchronize(s));
  for (int a = 0; a < nnodes; ++a) {
    off[a + 1] = off[a] + cnt[a];
    qoff[a + 1] = qoff[a] + (hrp[(size_t)a * bs + 1] - hrp[(size_t)a * bs]) / bs;
  }
  EMIN_HIP(hipMemcpyAsync(p->nmrp, off.data(), sizeof(long) * (nnodes + 1), hipMemcpyHostToDevice, s));
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)(nnodes + 1), &v));
  p->nqrp = (int*)v;
  EMIN_HIP(hipMemcpyAsync(p->nqrp, qoff.data(), sizeof(int) * (nnodes + 1), hipMemcpyHostToDevice, s));
  EMIN_TRY(p->alloc(sizeof(int2) * (size_t)std::max(qoff[nnodes], 1), &v));
  p->nq = (int2*)v;
  EMIN_TRY(p->alloc((size_t)std::max<long>(off[nnodes], 1), &v));
  p->nmap = (unsigned char*)v;
  launch_nmap_fill(p->arp, p->aci, p->prp, p->pci, p->nmrp, p->nqrp, nnodes, bs, p->nmap, p->nq, s);
  EMIN_HIP(hipGetLastError());
  EMIN_HIP(hipStreamSynchronize(s));  // the host offsets leave scope
  return EMIN_OK;
}

// Group-level intersection map of the node-pair product (see nodepair.hip):
// per node, neighbour block and group of the node's pattern row, one byte.
emin_status build_gmap(emin_problem* p, hipStream_t s, bool* fits) {
  const int bs = p->k1.bs;
  const int nnodes = p->n / bs;
  const size_t nn1 = (size_t)nnodes + 1;
  void* v;
  EMIN_TRY(p->alloc(sizeof(long) * nn1, &v));
  p->gmrp = (long*)v;
  EMIN_TRY(p->alloc(sizeof(int2) * nn1, &v));
  int2* dshape = (int2*)v;
  // host tables in pinned staging: map bytes and {pairs, blocks} per node in,
  // map offsets, descriptor offsets and the windows out (a window starts at
  // a node, or continues a node cut at 64 pairs: at most two per node plus
  // one per 64 pairs)
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t max_win = 2 * nn1 + (size_t)p->nnzP / 128 + 1;
  const size_t o_shape = up(sizeof(long) * nn1), o_off = o_shape + up(sizeof(int2) * nn1),
               o_qoff = o_off + up(sizeof(long) * nn1), o_win = o_qoff + up(sizeof(int) * nn1),
               total = o_win + up(sizeof(int) * 3 * max_win);
  char* pin;
  EMIN_TRY(p->ctx->pinned(total, (void**)&pin));
  long* cnt = (long*)pin;
  int2* shape = (int2*)(pin + o_shape);
  long* off = (long*)(pin + o_off);
  int* qoff = (int*)(pin + o_qoff);
  int* hwin = (int*)(pin + o_win);
  launch_gmap_count(p->arp, p->prp, nnodes, bs, p->grp, p->gmrp, dshape, s);
  EMIN_HIP(hipMemcpyAsync(cnt, p->gmrp, sizeof(long) * nnodes, hipMemcpyDeviceToHost, s));
  EMIN_HIP(hipMemcpyAsync(shape, dshape, sizeof(int2) * nnodes, hipMemcpyDeviceToHost, s));
  EMIN_HIP(hipStreamSynchronize(s));
  int max_nb = 0;
  long max_map = 0;
  off[0] = 0;
  qoff[0] = 0;
  for (int a = 0; a < nnodes; ++a) {
    off[a + 1] = off[a] + cnt[a];
    qoff[a + 1] = qoff[a] + shape[a].y;
    max_nb = std::max(max_nb, shape[a].y);
    max_map = std::max(max_map, cnt[a]);
  }
  *fits = nodepair_fits(max_nb, max_map);
  if (!*fits) return EMIN_OK;
  // windows of 64 slot pairs over the nodes in order (the product's waves)
  std::vector<int> win;
  nodepair_windows(nnodes, shape, cnt, win);
  if (win.size() > 3 * max_win) return fail(EMIN_ERR_UNSUPPORTED, "window table overflow");
  std::copy(win.begin(), win.end(), hwin);
  EMIN_TRY(p->alloc(sizeof(int) * std::max<size_t>(win.size(), 1), &v));
  p->win = (int*)v;
  EMIN_HIP(hipMemcpyAsync(p->win, hwin, sizeof(int) * win.size(), hipMemcpyHostToDevice, s));
  p->k1.nwin = (int)(win.size() / 3);
  EMIN_HIP(hipMemcpyAsync(p->gmrp, off, sizeof(long) * nn1, hipMemcpyHostToDevice, s));
  EMIN_TRY(p->alloc(sizeof(int) * nn1, &v));
  p->nqrp = (int*)v;
  EMIN_HIP(hipMemcpyAsync(p->nqrp, qoff, sizeof(int) * nn1, hipMemcpyHostToDevice, s));
  EMIN_TRY(p->alloc(sizeof(int2) * (size_t)std::max(qoff[nnodes], 1), &v));
  p->nq = (int2*)v;
  EMIN_TRY(p->alloc((size_t)std::max<long>(off[nnodes], 1), &v));
  p->gmap = (unsigned char*)v;
  launch_gmap_fill(p->arp, p->aci, p->prp, p->pci, p->gmrp, p->nqrp, nnodes, bs, p->grp, p->gmap,
                   p->nq, s);
  EMIN_HIP(hipGetLastError());
  EMIN_HIP(hipStreamSynchronize(s));  // the staging is reused by the next build
  return EMIN_OK;
}

// Sweep order of the projected SGS: Jones-Plassmann rounds on A's graph (one
// launch and one host read of the count per round) with first-fit colours,
// then the rows of each colour in index order, and every entry's relation
// (lower / higher colour) to its row.
emin_status build_colouring(emin_problem* p, hipStream_t s) {
  const int n = p->n;
  void *v, *rnd;
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)std::max(n, 1), &v));
  p->colour = (int*)v;
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)std::max(n, 1), &v));
  p->crows = (int*)v;
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)std::max(n, 1), &rnd));
  EMIN_TRY(p->alloc((size_t)std::max(p->nnzA, 1), &v));
  p->erel = (unsigned char*)v;
  launch_fill_int(p->colour, n, -1, s);
  launch_fill_int((int*)rnd, n, -1, s);
  int done = 0, rounds = 0;
  while (done < n) {
    EMIN_HIP(hipMemsetAsync(p->ints + 4, 0, sizeof(int), s));
    launch_jp_round(p->arp, p->aci, n, rounds, (int*)rnd, p->colour, p->ints + 4, s);
    int picked = 0;
    EMIN_HIP(hipMemcpyAsync(&picked, p->ints + 4, sizeof(int), hipMemcpyDeviceToHost, s));
    EMIN_HIP(hipStreamSynchronize(s));
    // the unpicked row of largest priority is always picked
    if (picked <= 0) return fail(EMIN_ERR_HIP, "SGS colouring made no progress");
    done += picked;
    ++rounds;
  }
  // number of colours: the largest colour + 1 (a row that found no free
  // colour below the limit holds the limit itself)
  EMIN_HIP(hipMemsetAsync(p->ints + 4, 0, sizeof(int), s));
  launch_max_int(p->colour, n, p->ints + 4, s);
  int cmax = 0;
  EMIN_HIP(hipMemcpyAsync(&cmax, p->ints + 4, sizeof(int), hipMemcpyDeviceToHost, s));
  EMIN_HIP(hipStreamSynchronize(s));
  if (cmax >= sgs_max_colours())
    return fail(EMIN_ERR_UNSUPPORTED, "SGS colouring needs more than " +
                                          std::to_string(sgs_max_colours()) + " colours");
  const int C = cmax + 1;
  std::vector<int> counts(C, 0);
  void *flags, *pos, *tmp;
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)std::max(n, 1), &flags));
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)(n + 1), &pos));
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)scan_tmp_ints(n), &tmp));
  p->coff.assign(C + 1, 0);
  for (int c = 0; c < C; ++c) {
    launch_colour_rows(p->colour, n, c, (int*)flags, (int*)pos, (int*)tmp, p->coff[c], p->crows,
                       s);
    int cnt = 0;
    EMIN_HIP(hipMemcpyAsync(&cnt, (int*)pos + n, sizeof(int), hipMemcpyDeviceToHost, s));
    EMIN_HIP(hipStreamSynchronize(s));
    p->coff[c + 1] = p->coff[c] + cnt;
  }
  if (p->coff[C] != n) return fail(EMIN_ERR_HIP, "SGS colouring: rows lost");
  launch_entry_rel(p->arp, p->aci, p->colour, n, p->erel, s);
  EMIN_HIP(hipGetLastError());
  return EMIN_OK;
}

emin_status validate_opts(const emin_opts* o, int64_t n) {
  if (!o) return fail(EMIN_ERR_ARG, "opts is NULL");
  if (o->precision != EMIN_FP64 && o->precision != EMIN_MIXED)
    return fail(EMIN_ERR_ARG, "opts.precision must be EMIN_FP64 or EMIN_MIXED");
  if (o->precond != EMIN_JACOBI && o->precond != EMIN_BJACOBI && o->precond != EMIN_SGS)
    return fail(EMIN_ERR_ARG, "opts.precond must be EMIN_JACOBI, EMIN_BJACOBI or EMIN_SGS");
  if (o->maxit < 0 || o->maxit > 100000) return fail(EMIN_ERR_ARG, "opts.maxit out of range");
  if (!(o->tau >= 0.0)) return fail(EMIN_ERR_ARG, "opts.tau must be >= 0");
  if (o->precond == EMIN_BJACOBI) {
    if (o->block < 1 || o->block > 4) return fail(EMIN_ERR_ARG, "opts.block must be 1..4");
    if (n % o->block) return fail(EMIN_ERR_SHAPE, "n is not a multiple of opts.block");
  }
  return EMIN_OK;
}

emin_status create_impl(emin_ctx* ctx, const emin_csr* A, const emin_csr* P0,
                        const emin_csr* pattern, int m, const double* B, const double* Bc,
                        const emin_opts* opts, emin_problem* p, const int32_t* cf = nullptr) {
  if (!A || !P0) return fail(EMIN_ERR_ARG, "A and P0 are required");
  const int64_t n = A->n_rows;
  EMIN_TRY(check_csr_host(A, "A", n, n));
  EMIN_TRY(check_csr_host(P0, "P0", n, P0->n_cols));
  if ((A->nnz > 0 && !A->vals) || (P0->nnz > 0 && !P0->vals))
    return fail(EMIN_ERR_ARG, "A/P0 values are NULL");
  if (pattern) EMIN_TRY(check_csr_host(pattern, "pattern", n, P0->n_cols));
  if (m < 1 || m > EMIN_MAX_M) return fail(EMIN_ERR_UNSUPPORTED, "m must be 1..8");
  if ((!B && n > 0) || (!Bc && P0->n_cols > 0)) return fail(EMIN_ERR_ARG, "B and B_c are required");
  EMIN_TRY(validate_opts(opts, n));
  if (!pattern && opts->pattern_power < 1)
    return fail(EMIN_ERR_ARG, "opts.pattern_power must be >= 1 when no pattern is given");
  p->ctx = ctx;
  p->n = (int)n;
  p->nc = (int)P0->n_cols;
  p->m = m;
  p->nnzA = (int)A->nnz;
  p->nnzP0 = (int)P0->nnz;
  p->arp = A->rowptr;
  p->aci = A->colind;
  p->av = A->vals;
  p->qrp = P0->rowptr;
  p->qci = P0->colind;
  p->qv = P0->vals;
  p->B = B;
  p->bc = Bc;
  p->opts = *opts;
  hipStream_t s = ctx->stream;
  bool node_grown = false, group_grown = false, a_checked = false;
  void* v;
  EMIN_TRY(p->alloc(8 * sizeof(int), &v));
  p->flags = (int*)v;
  EMIN_TRY(p->alloc(8 * sizeof(int), &v));
  p->ints = (int*)v;
  EMIN_HIP(hipMemsetAsync(p->flags, 0, 8 * sizeof(int), s));
  EMIN_HIP(hipMemsetAsync(p->ints, 0, 8 * sizeof(int), s));
  // longest rows of A and P0 (row pointers only, safe before validation)
  launch_row_maxlen(A->rowptr, p->n, p->ints + 2, s);
  launch_row_maxlen(P0->rowptr, p->n, p->ints + 3, s);
  int hmax[2] = {0, 0};
  EMIN_HIP(hipMemcpyAsync(hmax, p->ints + 2, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  launch_check_csr(A->rowptr, A->colind, p->n, p->n, p->nnzA, p->flags, kFlagCsrA, s);
  launch_check_csr(P0->rowptr, P0->colind, p->n, p->nc, p->nnzP0, p->flags, kFlagCsrP0, s);
  if (pattern)
    launch_check_csr(pattern->rowptr, pattern->colind, p->n, p->nc, (int)pattern->nnz,
                     p->flags, kFlagCsrPat, s);
  EMIN_HIP(hipGetLastError());
  int fl = 0;
  EMIN_TRY(read_flags(p, &fl));
  if (fl & (1 << kFlagCsrA)) return fail(EMIN_ERR_CSR, "A: invalid CSR (rowptr, range, order)");
  if (fl & (1 << kFlagCsrP0)) return fail(EMIN_ERR_CSR, "P0: invalid CSR (rowptr, range, order)");
  if (fl & (1 << kFlagCsrPat)) return fail(EMIN_ERR_CSR, "pattern: invalid CSR");
  if (cf) {
    // C/F form (P = [W; I]): a copy of the splitting; P0's COARSE rows must be
    // their identity rows
    if (opts->block > 1 || opts->precond == EMIN_BJACOBI)
      return fail(EMIN_ERR_UNSUPPORTED, "the C/F form takes point preconditioners (block 1)");
    EMIN_TRY(p->alloc(sizeof(int) * (size_t)std::max(p->n, 1), &v));
    p->cfix = (int*)v;
    if (p->n)
      EMIN_HIP(hipMemcpyAsync(p->cfix, cf, sizeof(int) * (size_t)p->n, hipMemcpyDeviceToDevice,
                              s));
    void* seen;
    EMIN_TRY(p->alloc(sizeof(int) * (size_t)std::max(p->nc, 1), &seen));
    EMIN_HIP(hipMemsetAsync(seen, 0, sizeof(int) * (size_t)std::max(p->nc, 1), s));
    launch_cf_check(p->cfix, p->n, p->nc, (int*)seen, P0->rowptr, P0->colind, P0->vals,
                    p->flags, s);
    EMIN_HIP(hipGetLastError());
    EMIN_TRY(read_flags(p, &fl));
    if (fl & (1 << kFlagCF))
      return fail(EMIN_ERR_ARG, "cf: an entry is outside [-1, nc) or a coarse index is not "
                                "held by exactly one node");
    if (fl & (1 << kFlagCFP0))
      return fail(EMIN_ERR_ARG, "P0: a COARSE row is not its identity row");
  }
  launch_diag_has(p->arp, p->aci, p->n, p->flags, s);
  // pattern
  if (pattern) {
    p->nnzP = (int)pattern->nnz;
    EMIN_TRY(p->alloc(sizeof(int) * (size_t)(p->n + 1), &v));
    p->prp = (int*)v;
    EMIN_TRY(p->alloc(sizeof(int) * (size_t)std::max(p->nnzP, 1), &v));
    p->pci = (int*)v;
    EMIN_HIP(hipMemcpyAsync(p->prp, pattern->rowptr, sizeof(int) * (p->n + 1),
                            hipMemcpyDeviceToDevice, s));
    if (p->nnzP)
      EMIN_HIP(hipMemcpyAsync(p->pci, pattern->colind, sizeof(int) * p->nnzP,
                              hipMemcpyDeviceToDevice, s));
  } else {
    EMIN_TRY(grow_pattern(p, hmax[0], hmax[1], &node_grown, &group_grown, &a_checked));
  }
  if (cf) {
    if (pattern) {
      launch_cf_pattern_check(p->prp, p->pci, p->cfix, p->n, p->flags, s);
    } else {
      // COARSE rows of struct(A^k P0) back to their identity column
      void *cnt, *rp2, *tmp, *ci2;
      EMIN_TRY(p->alloc(sizeof(int) * (size_t)std::max(p->n, 1), &cnt));
      EMIN_TRY(p->alloc(sizeof(int) * (size_t)(p->n + 1), &rp2));
      EMIN_TRY(p->alloc(sizeof(int) * (size_t)scan_tmp_ints(p->n), &tmp));
      launch_cf_count(p->prp, p->cfix, p->n, (int*)cnt, s);
      launch_exclusive_scan((int*)cnt, p->n, (int*)rp2, (int*)tmp, s);
      int nnz2 = 0;
      EMIN_HIP(hipMemcpyAsync(&nnz2, (int*)rp2 + p->n, sizeof(int), hipMemcpyDeviceToHost, s));
      EMIN_HIP(hipStreamSynchronize(s));
      EMIN_TRY(p->alloc(sizeof(int) * (size_t)std::max(nnz2, 1), &ci2));
      launch_cf_fill(p->prp, p->pci, p->cfix, p->n, (int*)rp2, (int*)ci2, s);
      p->prp = (int*)rp2;
      p->pci = (int*)ci2;
      p->nnzP = nnz2;
    }
  }
  // a grown pattern contains P0 when every diagonal of A is stored (checked
  // below); a given one is checked
  if (pattern)
    launch_check_contains(P0->rowptr, P0->colind, p->prp, p->pci, p->n, p->flags, kFlagContains,
                          s);
  EMIN_HIP(hipMemsetAsync(p->ints, 0, 4 * sizeof(int), s));
  launch_row_maxlen(p->prp, p->n, p->ints, s);
  if (opts->precond == EMIN_BJACOBI || opts->block > 1) {
    const int bs = std::max(1, opts->block);
    // node-level growth makes the rows of a node equal and has checked A
    const int what = (node_grown ? 0 : 1) | (a_checked ? 0 : 2);
    if (p->n % bs == 0 && what)
      launch_check_nodes(p->arp, p->aci, p->prp, p->pci, p->n / bs, bs, what, p->flags, s);
    // coarse columns in aligned groups of m (aggregation with m modes per
    // aggregate): the node-pair product applies when m is even.  Group-level
    // growth gives whole groups, at most 256 / m < 255 of them a row (rows
    // longer than 256 are refused below)
    if (p->n % bs == 0 && m % 2 == 0 && !group_grown)
      launch_group_check(p->prp, p->pci, p->n, m, 254, kFlagGroups, p->flags, s);
  }
  EMIN_HIP(hipGetLastError());
  int h[2] = {0, 0};
  EMIN_HIP(hipMemcpyAsync(h, p->ints, sizeof(int), hipMemcpyDeviceToHost, s));
  EMIN_TRY(read_flags(p, &fl));
  p->lmax = h[0];
  p->amax = hmax[0];
  if (fl & (1 << kFlagNoDiag)) return fail(EMIN_ERR_DIAG, "A: a row has no stored diagonal");
  if (fl & (1 << kFlagContains))
    return fail(EMIN_ERR_PATTERN, "the pattern does not contain P0's pattern");
  if (fl & (1 << kFlagCFPattern))
    return fail(EMIN_ERR_PATTERN, "pattern: a COARSE row is not its identity column");
  const int bs = std::max(1, opts->block);
  p->node_ok_pattern = (bs > 1) && (p->n % bs == 0) && !(fl & (1 << kFlagNodePattern));
  p->node_ok_A = (bs > 1) && (p->n % bs == 0) && !(fl & (1 << kFlagNodeA));
  p->grp = (p->node_ok_A && p->node_ok_pattern && m % 2 == 0 && !(fl & (1 << kFlagGroups)) &&
            (int64_t)p->nnzP * 8 < (int64_t(1) << 31)) ? m : 0;
  if (opts->precond == EMIN_BJACOBI && bs > 1 && !p->node_ok_pattern)
    return fail(EMIN_ERR_UNSUPPORTED,
                "block-Jacobi needs the rows of each node to share one pattern row");
  if (p->lmax > 256) return fail(EMIN_ERR_UNSUPPORTED, "a pattern row is longer than 256");
  choose_shapes(p);
  // workspace
  const size_t vs = opts->precision == EMIN_MIXED ? sizeof(float) : sizeof(double);
  const size_t np = (size_t)std::max(p->nnzP, 1);
  EMIN_TRY(p->alloc(np * sizeof(double), &v)); p->p0p = (double*)v;
  if (m > 1) { EMIN_TRY(p->alloc((size_t)p->n * m * (m + 1) / 2 * sizeof(double) + 8, &v)); p->wpk = (double*)v; }
  EMIN_TRY(p->alloc((size_t)std::max(p->n, 1) * sizeof(double), &v)); p->dinv = (double*)v;
  if (opts->precond == EMIN_BJACOBI) {
    EMIN_TRY(p->alloc((size_t)std::max(p->n, 1) * bs * sizeof(double), &v));
    p->binv = (double*)v;
  }
  if (p->node_ok_pattern) {
    const int rec = setup_node_record(bs, m);
    if (rec > 0) {
      EMIN_TRY(p->alloc((size_t)(p->n / bs) * rec * sizeof(double) + 8, &v));
      p->nrec = (double*)v;
    }
  }
  if (opts->precision == EMIN_MIXED) {
    EMIN_TRY(p->alloc((size_t)std::max(p->nnzA, 1) * sizeof(float), &v));
    p->avf = (float*)v;
  }
  EMIN_TRY(p->alloc(np * vs, &p->Y));
  EMIN_TRY(p->alloc(np * vs, &p->Yh));
  EMIN_TRY(p->alloc(np * vs, &p->R));
  EMIN_TRY(p->alloc(np * vs, &p->dP));
  EMIN_TRY(p->alloc(((size_t)ctx->grid_cap + 64) * sizeof(double), &v));
  p->part_d = (double*)v;
  EMIN_TRY(p->alloc(((size_t)ctx->grid_cap + 64) * sizeof(double), &v));
  p->part_g = (double*)v;
  if (p->k1.kind == 2) {
    bool too_big = false;
    EMIN_TRY(build_map(p, s, &too_big));
    if (too_big)  // map larger than 2^31 bytes: fall back to column matching
      p->k1 = {0, p->k1.G, next_pow2(std::max(p->lmax, 1)), 1, 1, 0};
  }
  if (p->k1.kind == 4) EMIN_TRY(build_nmap(p, s));
  if (p->k1.kind == 5) {
    bool fits = true;
    EMIN_TRY(build_gmap(p, s, &fits));
    if (!fits) {
      // more neighbour blocks or map bytes per node than the staged
      // node-pair kernel takes: the slot-level node map instead
      const int bs = p->k1.bs;
      p->k1 = {4, bs == 3 ? 1 : 2, 0, bs, (p->lmax + 63) / 64, 0};
      p->upd = {1, 0, 0, p->opts.block, (p->lmax + 63) / 64, 1};
      EMIN_TRY(build_nmap(p, s));
    }
  }
  if ((p->k1.kind == 0 || p->k1.kind == 3) && p->k1.packed) {
    EMIN_TRY(p->alloc((size_t)std::max(p->nnzA, 1) * sizeof(int), &v));
    p->anb = (int*)v;
    launch_build_anb(p->aci, p->nnzA, p->prp, p->anb, s);
  }
  if (opts->precond == EMIN_SGS) {
    EMIN_TRY(ensure_map(p, s));
    EMIN_TRY(build_colouring(p, s));
    EMIN_TRY(p->alloc(np * vs, &p->U));
    EMIN_TRY(p->alloc(np * vs, &p->Zs));
  }
  EMIN_TRY(p->alloc(sizeof(DevState), &v)); p->st = (DevState*)v;
  p->hist_len = opts->maxit + 1;
  EMIN_TRY(p->alloc(4 * (size_t)p->hist_len * sizeof(double), &v)); p->hist = (double*)v;
  EMIN_TRY(p->alloc((size_t)std::max(p->n, 1) * sizeof(int), &v)); p->fb_list = (int*)v;
  EMIN_TRY(p->alloc(sizeof(int), &v)); p->fb_count = (int*)v;
  launch_state_init(p->st, opts->tau, s);
  EMIN_HIP(hipGetLastError());
  return EMIN_OK;
}

DevHist hist_of(emin_problem* p) {
  DevHist h;
  h.gamma = p->hist;
  h.delta = p->hist + p->hist_len;
  h.alpha = p->hist + 2 * p->hist_len;
  h.beta = p->hist + 3 * p->hist_len;
  return h;
}

emin_status k1_call(emin_problem* p, int mode, int precision, const void* av, const void* y,
                    void* out) {
  K1Args a{};
  a.arp = p->arp; a.aci = p->aci; a.av = av; a.anb = p->anb;
  a.mrp = p->mrp; a.aoff = p->aoff;
  a.amap = p->k1.kind == 4 ? p->nmap : p->k1.kind == 5 ? p->gmap : p->amap;
  a.mrp64 = p->k1.kind == 5 ? p->gmrp : p->nmrp;
  a.nnz_p = p->nnzP; a.nqrp = p->nqrp; a.nq = p->nq; a.grp = p->grp;
  a.win = p->win; a.nwin = p->k1.nwin;
  a.prp = p->prp; a.pci = p->pci;
  a.y = y; a.out = out;
  a.bc = p->bc; a.wpk = p->wpk; a.m = p->m; a.n = p->n;
  a.part_out = p->part_d; a.st = p->st;
  if (launch_k1(p->k1, mode, precision, a, p->ctx->grid_cap, p->ctx->stream))
    return fail(EMIN_ERR_UNSUPPORTED, "no masked-product kernel for this shape");
  return EMIN_OK;
}

// A caller's FP64 array on the pattern as the masked product's input: the
// row-load and node-map kernels may read past row ends, so caller arrays
// (which carry no slack) are first copied into a library buffer.  Returns
// NULL on failure.
const double* staged(emin_problem* p, const double* x) {
  if (p->k1.kind != 3 && p->k1.kind != 4) return x;
  if (!p->stage) {
    void* v;
    if (p->alloc(sizeof(double) * (size_t)std::max(p->nnzP, 1), &v) != EMIN_OK) return nullptr;
    p->stage = (double*)v;
  }
  if (hipMemcpyAsync(p->stage, x, sizeof(double) * (size_t)p->nnzP, hipMemcpyDeviceToDevice,
                     p->ctx->stream) != hipSuccess)
    return nullptr;
  return p->stage;
}

UpdArgs upd_args(emin_problem* p, int k) {
  UpdArgs a{};
  a.prp = p->prp; a.pci = p->pci; a.dinv = p->dinv; a.binv = p->binv;
  a.bc = p->bc; a.wpk = p->wpk; a.m = p->m; a.n = p->n; a.bs = std::max(1, p->opts.block);
  a.R = p->R; a.dP = p->dP; a.Y = p->Y; a.Yh = p->Yh;
  a.part_in = nullptr; a.np_in = 0; a.part_out = p->part_g;
  a.st = p->st; a.hist = hist_of(p); a.k = k;
  a.k_max = p->hist_len; a.gamma_floor = 1e-26;
  if (p->k1.kind == 5) { a.win = p->win; a.nwin = p->k1.nwin; }
  return a;
}

// Z = Pi M_SGS^{-1} R: the forward sweep colour by colour, the backward sweep
// in reverse, then the projection with the <R, Z> partials (to part_g).
emin_status sgs_apply(emin_problem* p, bool mixed, hipStream_t s) {
  SgsArgs a{};
  a.arp = p->arp; a.aci = p->aci;
  a.av = mixed ? (const void*)p->avf : (const void*)p->av;
  a.prp = p->prp; a.pci = p->pci;
  a.mrp = p->mrp; a.amap = p->amap; a.aoff = p->aoff;
  a.colour = p->colour; a.rows = p->crows; a.erel = p->erel; a.dinv = p->dinv;
  a.x = p->R; a.u = p->U; a.z = p->Zs;
  a.bc = p->bc; a.wpk = p->wpk; a.m = p->m; a.n = p->n;
  a.Z = p->Zs; a.part_out = p->part_g; a.st = p->st;
  const int C = (int)p->coff.size() - 1;
  const int gc = p->ctx->grid_cap;
  for (int pass = 0; pass < 2; ++pass)
    for (int t = 0; t < C; ++t) {
      const int c = pass == 0 ? t : C - 1 - t;
      a.c = c;
      a.row0 = p->coff[c];
      a.nrows = p->coff[c + 1] - p->coff[c];
      if (launch_sgs_sweep(pass == 0, mixed, p->rowG, p->rowL, a, gc, s))
        return fail(EMIN_ERR_UNSUPPORTED, "no SGS sweep kernel for this row length");
    }
  if (launch_sgs_finish(mixed, p->rowG, p->rowL, a, gc, s))
    return fail(EMIN_ERR_UNSUPPORTED, "no SGS projection kernel for this row length");
  return EMIN_OK;
}

emin_status solve_impl(emin_problem* p, double* P_vals, double* dE_hist, emin_stats* stats,
                       const double* qv, emin_tape* tape = nullptr) {
  emin_ctx* c = p->ctx;
  hipStream_t s = c->stream;
  const bool mixed = p->opts.precision == EMIN_MIXED;
  const bool prof = p->opts.profile != 0;
  const int maxit = p->opts.maxit;
  if (prof) {
    for (int i = 0; i < 2; ++i)
      if (!p->ev[i]) EMIN_HIP(hipEventCreate(&p->ev[i]));
    while ((int)p->kev.size() < 2 * maxit) {
      hipEvent_t e;
      EMIN_HIP(hipEventCreate(&e));
      p->kev.push_back(e);
    }
    EMIN_HIP(hipEventRecord(p->ev[0], s));
  }
  launch_state_init(p->st, p->opts.tau, s);
  // Alg. 2 on every row, diagonal data, FP32 copy of A for the mixed form
  SetupArgs sa{};
  sa.arp = p->arp; sa.aci = p->aci; sa.av = p->av;
  sa.qrp = p->qrp; sa.qci = p->qci; sa.qv = qv;
  sa.prp = p->prp; sa.pci = p->pci;
  sa.B = p->B; sa.bc = p->bc; sa.m = p->m; sa.n = p->n;
  sa.bs = p->opts.precond == EMIN_BJACOBI ? std::max(1, p->opts.block) : 0;
  sa.nbs = p->node_ok_pattern ? p->opts.block : 0;
  sa.p0p = p->p0p; sa.wpk = p->wpk; sa.dinv = p->dinv; sa.binv = p->binv; sa.avf = p->avf;
  sa.nnzA = p->nnzA; sa.fb_list = p->fb_list; sa.fb_count = p->fb_count; sa.st = p->st;
  sa.nrec = p->nrec;
  sa.ablk = p->node_ok_A && p->opts.block == sa.nbs ? 1 : 0;
  sa.fixed = p->cfix;
  sa.lavg = p->n ? (int)((p->nnzP + (int64_t)p->n - 1) / p->n) : 0;
  launch_setup(sa, p->lmax, c->grid_cap, s);
  p->have_factors = true;
  if (p->nnzP == 0) {
    EMIN_HIP(hipGetLastError());
    EMIN_HIP(hipStreamSynchronize(s));
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->m = p->m;
    }
    if (dE_hist)
      for (int k = 0; k < maxit; ++k) dE_hist[k] = 0.0;
    return EMIN_OK;
  }
  // r = -Pi K w0 (Alg. 3 with f = 0), in FP64 for both forms
  const int g_k1 = k1_grid(p->k1, p->n, c->grid_cap);
  const int g_up = update_grid(p->upd, p->n, c->grid_cap);
  // node product with block-Jacobi updates: the product leaves the projector
  // to the update kernel (fewer registers in the gather-bound product), also
  // for the initial residual (the first update applies -Pi).  The mixed form
  // takes the raw product in FP64 from a buffer of its own, so it is rounded
  // to FP32 only after the projection.
  const bool raw_k1 = (p->k1.kind == 4 || p->k1.kind == 5) && p->upd.node == 1;
  if (raw_k1 && mixed && !p->r0d) {
    void* v;
    EMIN_TRY(p->alloc(sizeof(double) * (size_t)std::max(p->nnzP, 1), &v));
    p->r0d = (double*)v;
  }
  if (raw_k1)
    EMIN_TRY(k1_call(p, kModeRaw, 0, p->av, p->p0p, mixed ? (void*)p->r0d : p->R));
  else
    EMIN_TRY(k1_call(p, kModeInit, mixed ? 2 : 0, p->av, p->p0p, p->R));
  UpdArgs ua = upd_args(p, 0);
  ua.proj_yh = raw_k1 ? 1 : 0;
  ua.r0raw = raw_k1 && mixed ? p->r0d : nullptr;
  // projected SGS: the update applies no preconditioner; the sweeps form
  // Z = Pi M_SGS^{-1} R and the <R, Z> partials
  const bool sgs = p->opts.precond == EMIN_SGS;
  const int g_fin = sgs ? sgs_finish_grid(p->rowG, p->n, c->grid_cap) : 0;
  if (sgs) {
    launch_sgs_update(1, mixed, ua, p->nnzP, c->grid_cap, s);
    EMIN_TRY(sgs_apply(p, mixed, s));
    ua.part_in = p->part_g;
    ua.np_in = g_fin;
    launch_sgs_direction(1, mixed, ua, p->Zs, p->nnzP, c->grid_cap, s);
  } else {
    if (launch_update(p->upd, 1, mixed, ua, c->grid_cap, s))
      return fail(EMIN_ERR_UNSUPPORTED, "no update kernel for this shape");
    ua.part_in = p->part_g;
    ua.np_in = g_up;
    if (launch_direction(p->upd, 1, mixed, ua, c->grid_cap, s))
      return fail(EMIN_ERR_UNSUPPORTED, "no direction kernel for this shape");
  }
  const void* aiter = mixed ? (const void*)p->avf : (const void*)p->av;
  const int iter_mode = raw_k1 ? kModeIterRaw : kModeIter;
  ua.proj_yh = raw_k1 ? 1 : 0;
  ua.r0raw = nullptr;
  for (int k = 1; k <= maxit; ++k) {
    if (tape) {  // Y_k and R_k as they enter iteration k
      const size_t b = sizeof(double) * p->nnzP;
      EMIN_HIP(hipMemcpyAsync(tape->Y + (size_t)(k - 1) * p->nnzP, p->Y, b, hipMemcpyDeviceToDevice, s));
      EMIN_HIP(hipMemcpyAsync(tape->R + (size_t)(k - 1) * p->nnzP, p->R, b, hipMemcpyDeviceToDevice, s));
    }
    if (prof) EMIN_HIP(hipEventRecord(p->kev[2 * (k - 1)], s));
    EMIN_TRY(k1_call(p, iter_mode, mixed ? 1 : 0, aiter, p->Y, p->Yh));
    if (prof) EMIN_HIP(hipEventRecord(p->kev[2 * (k - 1) + 1], s));
    ua.k = k;
    ua.part_in = p->part_d;
    ua.np_in = g_k1;
    if (sgs) {
      launch_sgs_update(0, mixed, ua, p->nnzP, c->grid_cap, s);
      EMIN_TRY(sgs_apply(p, mixed, s));
      ua.part_in = p->part_g;
      ua.np_in = g_fin;
      launch_sgs_direction(0, mixed, ua, p->Zs, p->nnzP, c->grid_cap, s);
      continue;
    }
    launch_update(p->upd, 0, mixed, ua, c->grid_cap, s);
    ua.part_in = p->part_g;
    ua.np_in = g_up;
    launch_direction(p->upd, 0, mixed, ua, c->grid_cap, s);
  }
  FinalArgs fa{};
  fa.prp = p->prp; fa.pci = p->pci; fa.p0p = p->p0p; fa.dP = p->dP;
  fa.B = p->B; fa.bc = p->bc; fa.wpk = p->wpk; fa.m = p->m; fa.n = p->n; fa.out = P_vals;
  fa.nbs = p->node_ok_pattern ? p->opts.block : 0;
  fa.lmax = p->lmax;
  fa.pairs = p->upd.V == 2 ? 1 : 0;
  // block Jacobi leaves the projector out of Z (it commutes with the block
  // inverse), so rounding can drift off the constraint: re-project in FP64
  const int reproj = p->opts.precond == EMIN_BJACOBI ? 1 : 0;
  if (launch_final(p->rowG, p->rowL, mixed, reproj, fa, c->grid_cap, s))
    return fail(EMIN_ERR_UNSUPPORTED, "no final kernel for this shape");
  if (p->cfix) launch_cf_identity(p->prp, p->cfix, p->n, P_vals, s);  // P = [W; I]
  if (prof) EMIN_HIP(hipEventRecord(p->ev[1], s));
  EMIN_HIP(hipGetLastError());
  DevState hs;
  std::vector<double> hh(4 * (size_t)p->hist_len);
  EMIN_HIP(hipMemcpyAsync(&hs, p->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  EMIN_HIP(hipMemcpyAsync(hh.data(), p->hist, hh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  if (tape) {
    const size_t np = (size_t)p->nnzP;
    EMIN_HIP(hipMemcpyAsync(tape->p0p, p->p0p, np * 8, hipMemcpyDeviceToDevice, s));
    EMIN_HIP(hipMemcpyAsync(tape->av, p->av, (size_t)p->nnzA * 8, hipMemcpyDeviceToDevice, s));
    EMIN_HIP(hipMemcpyAsync(tape->dinv, p->dinv, (size_t)p->n * 8, hipMemcpyDeviceToDevice, s));
  }
  EMIN_HIP(hipStreamSynchronize(s));
  if (tape) {
    const int HL = p->hist_len;
    tape->iters = hs.iterations;
    tape->gamma.assign(hh.begin(), hh.begin() + HL);
    tape->delta.assign(hh.begin() + HL, hh.begin() + 2 * HL);
    tape->alpha.assign(hh.begin() + 2 * HL, hh.begin() + 3 * HL);
    tape->beta.assign(hh.begin() + 3 * HL, hh.begin() + 4 * HL);
  }
  if (dE_hist) {
    for (int k = 0; k < maxit; ++k)
      dE_hist[k] = (k < hs.iterations) ? hh[k] * hh[2 * p->hist_len + k] : 0.0;
  }
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->iterations = hs.iterations;
    stats->stop = (hs.done == kConverged || hs.done == kTauStop || hs.done == kBreakdown) ? hs.done : 0;
    stats->rank_deficient_rows = hs.rank_def;
    stats->m = p->m;
    stats->nnz_pattern = p->nnzP;
    stats->gamma1 = hs.gamma1;
    stats->dE_first = hs.iterations > 0 ? hh[0] * hh[2 * p->hist_len] : 0.0;
    stats->dE_last = hs.iterations > 0
                         ? hh[hs.iterations - 1] * hh[2 * p->hist_len + hs.iterations - 1] : 0.0;
    if (prof) {
      float ms = 0.f, tot = 0.f;
      int launches = 0;
      for (int k = 0; k < maxit; ++k) {
        EMIN_HIP(hipEventElapsedTime(&ms, p->kev[2 * k], p->kev[2 * k + 1]));
        tot += ms;
        ++launches;
      }
      stats->k1_ms = tot;
      stats->k1_launches = launches;
      EMIN_HIP(hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
      stats->solve_ms = ms;
    }
  }
  if (hs.done == 4) return fail(EMIN_ERR_DIAG, "A(i,i) <= 0 or a singular diagonal block");
  if (hs.done == kBreakdown)
    return fail(EMIN_ERR_BREAKDOWN, "RCG breakdown: <y, Pi K y> <= 0 or gamma < 0");
  if (hs.rank_def > 0) {
    g_err = std::to_string(hs.rank_def) + " rows have rank(G_i) < m";
    return EMIN_WARN_RANK;
  }
  return EMIN_OK;
}


// ====================================================================== batch

struct Bucket {
  K1Shape shape;
  std::vector<int> host_rows;  // empty: all rows
  int* rows = nullptr;         // device copy
  int nrows = 0;
};

struct Plan {
  std::string name;
  std::vector<Bucket> buckets;
};

}  // namespace

struct emin_batch {
  emin_ctx* ctx = nullptr;
  int count = 0;
  std::vector<emin_problem*> members;
  emin_problem* sup = nullptr;
  std::vector<void*> owned;
  int N = 0, NA = 0, NQ = 0, NC = 0, NP = 0, m = 1;
  int *Arp = nullptr, *Aci = nullptr, *Qrp = nullptr, *Qci = nullptr, *Prp = nullptr, *Pci = nullptr;
  double *Av = nullptr, *Qv = nullptr, *Bv = nullptr, *Bcv = nullptr, *Pout = nullptr;
  long *offA = nullptr, *offQ = nullptr, *offB = nullptr, *offBc = nullptr, *offP = nullptr;
  const double **srcA = nullptr, **srcQ = nullptr, **srcB = nullptr, **srcBc = nullptr;
  double** dstP = nullptr;
  int *mapA = nullptr, *mapQ = nullptr, *mapB = nullptr;  // member-local indices
  int* invP = nullptr;  // per member: layout position of each of its own P entries
  std::vector<double*> host_dst;
  int* seg_row = nullptr;
  int *chunk_row = nullptr, *seg_chunk = nullptr;  // per-member reduction chunks
  double* chunk_sum = nullptr;
  int nchunk = 0;
  int* row_seg = nullptr;  // segment (member) of every row
  SegState* segs = nullptr;
  double* shist = nullptr;
  double* rowdot = nullptr;
  int hist_len = 1;
  Plan plan;
  std::string plan_json;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  emin_status alloc(size_t bytes, void** p) {
    EMIN_TRY(ctx->pool.get(bytes, p));
    owned.push_back(*p);
    return EMIN_OK;
  }
  ~emin_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
    delete sup;
    for (void* p : owned) ctx->pool.put(p);
  }
};

namespace {

template <class T>
emin_status upload(emin_batch* b, const std::vector<T>& h, T** d) {
  void* v;
  EMIN_TRY(b->alloc(std::max<size_t>(h.size(), 1) * sizeof(T), &v));
  if (!h.empty()) EMIN_HIP(hipMemcpy(v, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  *d = (T*)v;
  return EMIN_OK;
}

// Row buckets by pattern length: (0,2], (2,4], (4,8], ... with G = bound.
Plan plan_pow2(const std::vector<int>& len, int lo_merge) {
  Plan pl;
  pl.name = lo_merge > 2 ? "buckets-merged" : "buckets-pow2";
  std::map<int, std::vector<int>> by;
  for (int i = 0; i < (int)len.size(); ++i) {
    int G = next_pow2(std::max(len[i], 1));
    if (G < lo_merge) G = lo_merge;
    by[G].push_back(i);
  }
  for (auto& kv : by) {
    Bucket bk;
    bk.shape = {2, kv.first, kv.first, 1, 1, 0};
    bk.host_rows = kv.second;
    bk.nrows = (int)kv.second.size();
    pl.buckets.push_back(bk);
  }
  return pl;
}

// Rows up to 8 long whose neighbours' rows are also up to 8 long go to the
// one-lane-per-row kernel, bucketed by (own capacity, neighbour capacity);
// the rest to the map kernel by power-of-two length.  merge 1: one wide
// bucket per own capacity, neighbour capacity 8; merge 2: all of them in one
// bucket of capacity 8 (one sweep in layout order, so rows of both lengths
// reuse the neighbour rows a cluster brought into L2).  rest1: the other rows
// in one map-kernel bucket at the longest one's power of two.
Plan plan_wide(const std::vector<int>& len, const std::vector<int>& nbmax, int merge,
               bool rest1 = false) {
  Plan pl;
  pl.name = merge == 2 ? (rest1 ? "wide-one-rest1" : "wide-one")
                       : merge == 1 ? "wide-merged" : "wide-buckets";
  std::map<std::pair<int, int>, std::vector<int>> wide;
  std::map<int, std::vector<int>> rest;
  for (int i = 0; i < (int)len.size(); ++i) {
    const int l = std::max(len[i], 1), nb = std::max(nbmax[i], 1);
    if (l <= 8 && nb <= 8) {
      int S = std::max(4, next_pow2(l));
      int SN = std::max(S, std::max(4, next_pow2(nb)));
      if (merge) SN = 8;
      if (merge == 2) S = 8;
      wide[{S, SN}].push_back(i);
    } else {
      rest[next_pow2(l)].push_back(i);
    }
  }
  for (auto& kv : wide) {
    Bucket bk;
    bk.shape = {3, kv.first.second, kv.first.first, 1, 4, 1};
    bk.host_rows = kv.second;
    bk.nrows = (int)kv.second.size();
    pl.buckets.push_back(bk);
  }
  if (rest1 && rest.size() > 1) {
    const int G = rest.rbegin()->first;
    std::vector<int> all;
    for (int i = 0; i < (int)len.size(); ++i)
      if (!(std::max(len[i], 1) <= 8 && std::max(nbmax[i], 1) <= 8)) all.push_back(i);
    rest.clear();
    rest[G] = all;
  }
  for (auto& kv : rest) {
    Bucket bk;
    bk.shape = {2, kv.first, kv.first, 1, 1, 0};
    bk.host_rows = kv.second;
    bk.nrows = (int)kv.second.size();
    pl.buckets.push_back(bk);
  }
  return pl;
}

Plan plan_single(int G, int L, int n) {
  Plan pl;
  pl.name = "single-G" + std::to_string(G) + "L" + std::to_string(L);
  Bucket bk;
  bk.shape = {2, G, G * L, 1, L, 0};
  bk.nrows = n;
  pl.buckets.push_back(bk);
  return pl;
}

emin_status plan_upload(emin_batch* b, Plan& pl) {
  for (auto& bk : pl.buckets)
    if (!bk.host_rows.empty() && !bk.rows) EMIN_TRY(upload(b, bk.host_rows, &bk.rows));
  return EMIN_OK;
}

K1Args batch_k1_args(emin_batch* b, int precision, const Bucket& bk, const void* y, void* out) {
  emin_problem* p = b->sup;
  K1Args a{};
  std::memset(&a, 0, sizeof(a));
  a.arp = p->arp; a.aci = p->aci;
  a.av = precision == 1 ? (const void*)p->avf : (const void*)p->av;
  a.anb = p->anb; a.mrp = p->mrp; a.amap = p->amap; a.aoff = p->aoff;
  a.prp = p->prp; a.pci = p->pci;
  a.y = y; a.out = out;
  a.bc = p->bc; a.wpk = p->wpk; a.m = p->m;
  a.n = bk.rows ? bk.nrows : p->n;
  a.rows = bk.rows;
  a.part_out = p->part_d; a.st = p->st;
  a.seg = 1; a.rowdot = b->rowdot;
  return a;
}

// The masked products of one plan: mode kModeIter (Y -> Y_hat, per-row dots)
// or kModeInit (P0' -> R, precision 2 in the mixed form).
emin_status enqueue_k1_plan(emin_batch* b, const Plan& pl, int mode, int precision,
                            hipStream_t s) {
  emin_problem* p = b->sup;
  const void* y = mode == kModeInit ? (const void*)p->p0p : (const void*)p->Y;
  void* out = mode == kModeInit ? (void*)p->R : (void*)p->Yh;
  for (const auto& bk : pl.buckets) {
    if (bk.nrows == 0) continue;
    const K1Args a = batch_k1_args(b, precision, bk, y, out);
    if (launch_k1(bk.shape, mode, precision, a, b->ctx->grid_cap, s))
      return fail(EMIN_ERR_UNSUPPORTED, "no masked-product kernel for a bucket shape");
  }
  return EMIN_OK;
}

// Autotuner: time each candidate plan's masked products on this batch and
// keep the fastest.  Results can be cached in a text file, one line per
// batch signature: "<signature> <plan name>".
emin_status autotune(emin_batch* b, const std::vector<int>& len, const std::vector<int>& nbmax,
                     const char* cache_path) {
  emin_problem* p = b->sup;
  const int lmax = std::max(p->lmax, 1);
  std::vector<Plan> cands;
  cands.push_back(plan_single(next_pow2(lmax), 1, p->n));
  if (lmax > 4) cands.push_back(plan_single(4, next_pow2((lmax + 3) / 4), p->n));
  cands.push_back(plan_pow2(len, 1));
  cands.push_back(plan_pow2(len, 4));
  if (p->anb) {
    cands.push_back(plan_wide(len, nbmax, 0));
    cands.push_back(plan_wide(len, nbmax, 1));
    cands.push_back(plan_wide(len, nbmax, 2));
    cands.push_back(plan_wide(len, nbmax, 2, true));
  }
  std::ostringstream sig;
  sig << "n=" << p->n << ",nnzA=" << p->nnzA << ",nnzP=" << p->nnzP << ",lmax=" << lmax
      << ",count=" << b->count << ",prec=" << p->opts.precision;
  std::string cached;
  if (cache_path && *cache_path) {
    std::ifstream f(cache_path);
    std::string key, name;
    while (f >> key >> name)
      if (key == sig.str()) cached = name;
  }
  const int precision = p->opts.precision == EMIN_MIXED ? 1 : 0;
  hipStream_t s = b->ctx->stream;
  const size_t vb = precision ? sizeof(float) : sizeof(double);
  // timing inputs: Y = 0; the FP32 copy of A (mixed form) holds whatever the
  // allocation holds until the first set-up -- values do not change the timing
  EMIN_HIP(hipMemsetAsync(p->Y, 0, (size_t)std::max(p->nnzP, 1) * vb, s));
  if (precision) EMIN_HIP(hipMemsetAsync(p->avf, 0, (size_t)std::max(p->nnzA, 1) * sizeof(float), s));
  std::ostringstream js;
  js << "{\"signature\":\"" << sig.str() << "\",\"candidates\":[";
  int best = -1;
  float best_ms = 1e30f;
  hipEvent_t e0, e1;
  EMIN_HIP(hipEventCreate(&e0));
  EMIN_HIP(hipEventCreate(&e1));
  bool first_entry = true;
  for (size_t c = 0; c < cands.size(); ++c) {
    if (!cached.empty() && cands[c].name != cached) continue;
    EMIN_TRY(plan_upload(b, cands[c]));
    float ms = 0.f;
    if (cached.empty()) {
      for (int w = 0; w < 2; ++w) EMIN_TRY(enqueue_k1_plan(b, cands[c], kModeIter, precision, s));
      EMIN_HIP(hipEventRecord(e0, s));
      const int reps = 5;
      for (int r = 0; r < reps; ++r)
        EMIN_TRY(enqueue_k1_plan(b, cands[c], kModeIter, precision, s));
      EMIN_HIP(hipEventRecord(e1, s));
      EMIN_HIP(hipEventSynchronize(e1));
      EMIN_HIP(hipEventElapsedTime(&ms, e0, e1));
      ms /= reps;
    }
    js << (first_entry ? "" : ",") << "{\"plan\":\"" << cands[c].name << "\",\"buckets\":"
       << cands[c].buckets.size() << ",\"k1_ms\":" << ms << "}";
    first_entry = false;
    if (best < 0 || ms < best_ms) {
      best = (int)c;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best < 0) {  // cached name not among candidates: tune afresh
    return autotune(b, len, nbmax, nullptr);
  }
  b->plan = cands[best];
  js << "],\"chosen\":\"" << b->plan.name << "\",\"from_cache\":" << (cached.empty() ? "false" : "true")
     << "}";
  b->plan_json = js.str();
  if (cache_path && *cache_path && cached.empty()) {
    std::ofstream f(cache_path, std::ios::app);
    f << sig.str() << " " << b->plan.name << "\n";
  }
  return EMIN_OK;
}

// The whole batched solve on stream s (captured into the graph).
emin_status enqueue_batch(emin_batch* b, hipStream_t s) {
  emin_problem* p = b->sup;
  emin_ctx* c = b->ctx;
  const bool mixed = p->opts.precision == EMIN_MIXED;
  const int maxit = p->opts.maxit;
  launch_gather_map(b->srcA, b->offA, b->mapA, b->count, b->Av, s);
  launch_gather_map(b->srcQ, b->offQ, b->mapQ, b->count, b->Qv, s);
  launch_gather_map(b->srcB, b->offB, b->mapB, b->count, b->Bv, s);
  launch_gather_segments(b->srcBc, b->offBc, b->count, b->Bcv, s);
  launch_state_init(p->st, p->opts.tau, s);
  launch_seg_init(b->segs, b->count, s);
  SetupArgs sa{};
  sa.arp = p->arp; sa.aci = p->aci; sa.av = p->av;
  sa.qrp = p->qrp; sa.qci = p->qci; sa.qv = p->qv;
  sa.prp = p->prp; sa.pci = p->pci;
  sa.B = p->B; sa.bc = p->bc; sa.m = p->m; sa.n = p->n; sa.bs = 0;
  sa.p0p = p->p0p; sa.wpk = p->wpk; sa.dinv = p->dinv; sa.binv = nullptr; sa.avf = p->avf;
  sa.nnzA = p->nnzA; sa.fb_list = p->fb_list; sa.fb_count = p->fb_count; sa.st = p->st;
  sa.row_seg = b->row_seg; sa.segs = b->segs;
  sa.lavg = p->n ? (int)((p->nnzP + (int64_t)p->n - 1) / p->n) : 0;
  launch_setup(sa, p->lmax, c->grid_cap, s);
  p->have_factors = true;
  EMIN_TRY(enqueue_k1_plan(b, b->plan, kModeInit, mixed ? 2 : 0, s));
  UpdArgs ua = upd_args(p, 0);
  ua.seg = 1; ua.seg_row = b->seg_row; ua.nseg = b->count; ua.segs = b->segs; ua.rowdot = b->rowdot;
  ua.row_seg = b->row_seg;
  SegArgs ga{};
  ga.seg_row = b->seg_row; ga.nseg = b->count; ga.rowdot = b->rowdot; ga.segs = b->segs;
  ga.chunk_row = b->chunk_row; ga.seg_chunk = b->seg_chunk; ga.chunk_sum = b->chunk_sum;
  ga.nchunk = b->nchunk;
  ga.hist = b->shist; ga.hist_len = b->hist_len; ga.k = 0; ga.tau = p->opts.tau;
  ga.gamma_floor = 1e-26;
  if (launch_update(p->upd, 1, mixed, ua, c->grid_cap, s))
    return fail(EMIN_ERR_UNSUPPORTED, "no update kernel for the batch");
  launch_seg_gamma(ga, 1, s);
  launch_direction(p->upd, 1, mixed, ua, c->grid_cap, s);
  for (int k = 1; k <= maxit; ++k) {
    EMIN_TRY(enqueue_k1_plan(b, b->plan, kModeIter, mixed ? 1 : 0, s));
    ga.k = k;
    launch_seg_delta(ga, s);
    ua.k = k;
    launch_update(p->upd, 0, mixed, ua, c->grid_cap, s);
    launch_seg_gamma(ga, 0, s);
    launch_direction(p->upd, 0, mixed, ua, c->grid_cap, s);
  }
  FinalArgs fa{};
  fa.prp = p->prp; fa.pci = p->pci; fa.p0p = p->p0p; fa.dP = p->dP;
  fa.B = p->B; fa.bc = p->bc; fa.wpk = p->wpk; fa.m = p->m; fa.n = p->n; fa.out = b->Pout;
  if (launch_final(p->rowG, p->rowL, mixed, 0, fa, c->grid_cap, s))
    return fail(EMIN_ERR_UNSUPPORTED, "no final kernel for the batch");
  launch_scatter_map(b->Pout, b->offP, b->invP, b->count, b->dstP, s);
  EMIN_HIP(hipGetLastError());
  return EMIN_OK;
}

// Breadth-first (Cuthill-McKee) order of a matrix's rows, each connected
// component started from a pseudo-peripheral row (the last row reached by a
// breadth-first sweep from its first row).  Rows adjacent in A end up close
// together, so a row's neighbours' pattern rows share cache lines; the
// batched masked product is a gather and depends on that.
void bfs_order(int n, const std::vector<int>& rp, const std::vector<int>& ci,
               std::vector<int>& order) {
  order.clear();
  order.reserve(n);
  std::vector<int> mark(n, -1), queue;
  queue.reserve(n);
  std::vector<char> placed(n, 0);
  int comp = 0;
  for (int s0 = 0; s0 < n; ++s0) {
    if (placed[s0]) continue;
    // probe sweep: the last row reached is the start of the real one
    queue.clear();
    queue.push_back(s0);
    mark[s0] = comp;
    for (size_t h = 0; h < queue.size(); ++h) {
      const int r = queue[h];
      for (int e = rp[r]; e < rp[r + 1]; ++e) {
        const int c = ci[e];
        if (mark[c] != comp) {
          mark[c] = comp;
          queue.push_back(c);
        }
      }
    }
    const int start = queue.back();
    const size_t first = order.size();
    order.push_back(start);
    placed[start] = 1;
    for (size_t h = first; h < order.size(); ++h) {
      const int r = order[h];
      for (int e = rp[r]; e < rp[r + 1]; ++e) {
        const int c = ci[e];
        if (!placed[c]) {
          placed[c] = 1;
          order.push_back(c);
        }
      }
    }
    ++comp;
  }
}

// Rows in clusters of up to `cl` rows, each grown breadth-first from a seed
// over rows not yet placed, the seeds taken in the breadth-first order
// above.  A wave of 64 consecutive rows then covers one compact piece of the
// graph (its rows share neighbour rows), where a breadth-first level of a 3D
// graph holds about n^(2/3) rows spread over the whole matrix.
void cluster_order(int n, const std::vector<int>& rp, const std::vector<int>& ci, int cl,
                   std::vector<int>& order) {
  std::vector<int> seeds;
  bfs_order(n, rp, ci, seeds);
  order.clear();
  order.reserve(n);
  std::vector<char> placed(n, 0);
  std::vector<int> seen(n, -1), queue;
  int stamp = 0;
  for (const int s0 : seeds) {
    if (placed[s0]) continue;
    queue.clear();
    queue.push_back(s0);
    seen[s0] = stamp;
    int taken = 0;
    for (size_t h = 0; h < queue.size() && taken < cl; ++h) {
      const int r = queue[h];
      order.push_back(r);
      placed[r] = 1;
      ++taken;
      for (int e = rp[r]; e < rp[r + 1]; ++e) {
        const int c = ci[e];
        if (!placed[c] && seen[c] != stamp) {
          seen[c] = stamp;
          queue.push_back(c);
        }
      }
    }
    ++stamp;
  }
}

template <class T>
emin_status to_host(const T* d, size_t len, std::vector<T>* h) {
  h->assign(std::max<size_t>(len, 1), T());
  if (len) EMIN_HIP(hipMemcpy(h->data(), d, len * sizeof(T), hipMemcpyDeviceToHost));
  return EMIN_OK;
}

emin_status batch_create_impl(emin_ctx* ctx, int count, emin_problem* const* probs,
                              const char* tune_cache, emin_batch* b) {
  if (count < 1 || !probs) return fail(EMIN_ERR_ARG, "count < 1 or probs NULL");
  const emin_problem* p0 = probs[0];
  if (!p0) return fail(EMIN_ERR_ARG, "NULL problem");
  for (int i = 0; i < count; ++i) {
    const emin_problem* q = probs[i];
    if (!q || q->ctx != ctx) return fail(EMIN_ERR_ARG, "problem NULL or from another context");
    if (q->m != p0->m || q->opts.precision != p0->opts.precision ||
        q->opts.maxit != p0->opts.maxit || q->opts.tau != p0->opts.tau)
      return fail(EMIN_ERR_ARG, "batch members must share m, precision, maxit and tau");
    if (q->opts.precond != EMIN_JACOBI)
      return fail(EMIN_ERR_UNSUPPORTED, "the batched form supports the Jacobi preconditioner");
    if (q->lmax > 32) return fail(EMIN_ERR_UNSUPPORTED, "batched form: pattern rows up to 32");
  }
  b->ctx = ctx;
  b->count = count;
  b->members.assign(probs, probs + count);
  b->m = p0->m;
  const int m = b->m;
  std::vector<long> roff(count + 1, 0), aoff(count + 1, 0), qoff(count + 1, 0),
      coff(count + 1, 0), poff(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    const emin_problem* q = probs[i];
    roff[i + 1] = roff[i] + q->n;
    aoff[i + 1] = aoff[i] + q->nnzA;
    qoff[i + 1] = qoff[i] + q->nnzP0;
    coff[i + 1] = coff[i] + q->nc;
    poff[i + 1] = poff[i] + q->nnzP;
  }
  const long lim = 0x7fffffffL;
  if (roff[count] >= lim || aoff[count] > lim || qoff[count] > lim || coff[count] >= lim ||
      poff[count] > lim)
    return fail(EMIN_ERR_UNSUPPORTED, "batch exceeds int32 indexing");
  b->N = (int)roff[count]; b->NA = (int)aoff[count]; b->NQ = (int)qoff[count];
  b->NC = (int)coff[count]; b->NP = (int)poff[count];
  void* v;
  EMIN_TRY(b->alloc(sizeof(int) * (b->N + 1), &v)); b->Arp = (int*)v;
  EMIN_TRY(b->alloc(sizeof(int) * std::max(b->NA, 1), &v)); b->Aci = (int*)v;
  EMIN_TRY(b->alloc(sizeof(double) * std::max(b->NA, 1), &v)); b->Av = (double*)v;
  EMIN_TRY(b->alloc(sizeof(int) * (b->N + 1), &v)); b->Qrp = (int*)v;
  EMIN_TRY(b->alloc(sizeof(int) * std::max(b->NQ, 1), &v)); b->Qci = (int*)v;
  EMIN_TRY(b->alloc(sizeof(double) * std::max(b->NQ, 1), &v)); b->Qv = (double*)v;
  EMIN_TRY(b->alloc(sizeof(int) * (b->N + 1), &v)); b->Prp = (int*)v;
  EMIN_TRY(b->alloc(sizeof(int) * std::max(b->NP, 1), &v)); b->Pci = (int*)v;
  EMIN_TRY(b->alloc(sizeof(double) * std::max(b->N, 1) * m, &v)); b->Bv = (double*)v;
  EMIN_TRY(b->alloc(sizeof(double) * std::max(b->NC, 1) * m, &v)); b->Bcv = (double*)v;
  EMIN_TRY(b->alloc(sizeof(double) * std::max(b->NP, 1), &v)); b->Pout = (double*)v;
  hipStream_t s = ctx->stream;
  EMIN_HIP(hipStreamSynchronize(s));
  // every member's rows in breadth-first order; the concatenated structures
  // are built in that order on the host, with member-local index maps for
  // the values (A, P0, B) and for scattering P back
  std::vector<int> hArp(b->N + 1), hAci(std::max(b->NA, 1)), hAmap(std::max(b->NA, 1));
  std::vector<int> hQrp(b->N + 1), hQci(std::max(b->NQ, 1)), hQmap(std::max(b->NQ, 1));
  std::vector<int> hPrp(b->N + 1), hPci(std::max(b->NP, 1)), hPmap(std::max(b->NP, 1));
  std::vector<int> hBmap(std::max<long>((long)b->N * m, 1));
  {
    std::vector<int> order, newidx;
    std::vector<std::pair<int, int>> rowbuf;
    long ea = 0, eq = 0, ep = 0;
    for (int i = 0; i < count; ++i) {
      const emin_problem* q = probs[i];
      const int n = q->n;
      std::vector<int> arp, aci, qrp, qci, prp, pci;
      EMIN_TRY(to_host(q->arp, (size_t)n + 1, &arp));
      EMIN_TRY(to_host(q->aci, (size_t)q->nnzA, &aci));
      EMIN_TRY(to_host(q->qrp, (size_t)n + 1, &qrp));
      EMIN_TRY(to_host(q->qci, (size_t)q->nnzP0, &qci));
      EMIN_TRY(to_host(q->prp, (size_t)n + 1, &prp));
      EMIN_TRY(to_host(q->pci, (size_t)q->nnzP, &pci));
      cluster_order(n, arp, aci, kWave, order);
      newidx.assign(n, 0);
      for (int k = 0; k < n; ++k) newidx[order[k]] = k;
      for (int k = 0; k < n; ++k) {
        const int old = order[k];
        const long row = roff[i] + k;
        hArp[row] = (int)ea;
        rowbuf.clear();
        for (int e = arp[old]; e < arp[old + 1]; ++e) rowbuf.emplace_back(newidx[aci[e]], e);
        std::sort(rowbuf.begin(), rowbuf.end());
        for (const auto& pr : rowbuf) {
          hAci[ea] = pr.first + (int)roff[i];
          hAmap[ea++] = pr.second;
        }
        hQrp[row] = (int)eq;
        for (int e = qrp[old]; e < qrp[old + 1]; ++e) {
          hQci[eq] = qci[e] + (int)coff[i];
          hQmap[eq++] = e;
        }
        hPrp[row] = (int)ep;
        for (int e = prp[old]; e < prp[old + 1]; ++e) {
          hPci[ep] = pci[e] + (int)coff[i];
          hPmap[ep++] = e;
        }
        for (int x = 0; x < m; ++x) hBmap[row * m + x] = old * m + x;
      }
    }
    hArp[b->N] = (int)ea;
    hQrp[b->N] = (int)eq;
    hPrp[b->N] = (int)ep;
  }
  EMIN_HIP(hipMemcpy(b->Arp, hArp.data(), sizeof(int) * (b->N + 1), hipMemcpyHostToDevice));
  EMIN_HIP(hipMemcpy(b->Aci, hAci.data(), sizeof(int) * std::max(b->NA, 1), hipMemcpyHostToDevice));
  EMIN_HIP(hipMemcpy(b->Qrp, hQrp.data(), sizeof(int) * (b->N + 1), hipMemcpyHostToDevice));
  EMIN_HIP(hipMemcpy(b->Qci, hQci.data(), sizeof(int) * std::max(b->NQ, 1), hipMemcpyHostToDevice));
  EMIN_HIP(hipMemcpy(b->Prp, hPrp.data(), sizeof(int) * (b->N + 1), hipMemcpyHostToDevice));
  EMIN_HIP(hipMemcpy(b->Pci, hPci.data(), sizeof(int) * std::max(b->NP, 1), hipMemcpyHostToDevice));
  EMIN_TRY(upload(b, hAmap, &b->mapA));
  EMIN_TRY(upload(b, hQmap, &b->mapQ));
  {
    // the output is written in each member's own order: invert the P map
    std::vector<int> hPinv(hPmap.size());
    for (int i = 0; i < count; ++i)
      for (long j = poff[i]; j < poff[i + 1]; ++j) hPinv[poff[i] + hPmap[j]] = (int)(j - poff[i]);
    EMIN_TRY(upload(b, hPinv, &b->invP));
  }
  EMIN_TRY(upload(b, hBmap, &b->mapB));
  // pointer and offset tables for the per-solve value gathers and output scatter
  std::vector<const double*> hA(count), hQ(count), hB(count), hBc(count);
  std::vector<long> oB(count + 1), oBc(count + 1);
  for (int i = 0; i < count; ++i) {
    hA[i] = probs[i]->av; hQ[i] = probs[i]->qv; hB[i] = probs[i]->B; hBc[i] = probs[i]->bc;
  }
  for (int i = 0; i <= count; ++i) { oB[i] = roff[i] * m; oBc[i] = coff[i] * m; }
  EMIN_TRY(upload(b, hA, (const double***)&b->srcA));
  EMIN_TRY(upload(b, hQ, (const double***)&b->srcQ));
  EMIN_TRY(upload(b, hB, (const double***)&b->srcB));
  EMIN_TRY(upload(b, hBc, (const double***)&b->srcBc));
  EMIN_TRY(upload(b, aoff, &b->offA));
  EMIN_TRY(upload(b, qoff, &b->offQ));
  EMIN_TRY(upload(b, oB, &b->offB));
  EMIN_TRY(upload(b, oBc, &b->offBc));
  EMIN_TRY(upload(b, poff, &b->offP));
  b->host_dst.assign(count, nullptr);
  EMIN_TRY(upload(b, b->host_dst, &b->dstP));
  std::vector<int> srow(count + 1), rseg(std::max<long>(roff[count], 1), 0);
  for (int i = 0; i <= count; ++i) srow[i] = (int)roff[i];
  for (int i = 0; i < count; ++i)
    for (long r = roff[i]; r < roff[i + 1]; ++r) rseg[r] = i;
  EMIN_TRY(upload(b, srow, &b->seg_row));
  EMIN_TRY(upload(b, rseg, &b->row_seg));
  {  // first-stage chunks of the per-member reductions
    std::vector<int> crow, schunk(count + 1, 0);
    for (int i = 0; i < count; ++i) {
      schunk[i] = (int)crow.size();
      for (long r = roff[i]; r < roff[i + 1]; r += kSegChunk) crow.push_back((int)r);
    }
    schunk[count] = (int)crow.size();
    b->nchunk = (int)crow.size();
    crow.push_back((int)roff[count]);
    EMIN_TRY(upload(b, crow, &b->chunk_row));
    EMIN_TRY(upload(b, schunk, &b->seg_chunk));
    void* v;
    EMIN_TRY(b->alloc(sizeof(double) * (size_t)std::max(b->nchunk, 1), &v));
    b->chunk_sum = (double*)v;
  }
  launch_gather_map(b->srcA, b->offA, b->mapA, count, b->Av, s);
  launch_gather_map(b->srcQ, b->offQ, b->mapQ, count, b->Qv, s);
  launch_gather_map(b->srcB, b->offB, b->mapB, count, b->Bv, s);
  launch_gather_segments(b->srcBc, b->offBc, count, b->Bcv, s);
  // the block-diagonal problem, with the members' patterns concatenated
  emin_csr A = {b->N, b->N, b->NA, b->Arp, b->Aci, b->Av};
  emin_csr Q = {b->N, b->NC, b->NQ, b->Qrp, b->Qci, b->Qv};
  emin_csr P = {b->N, b->NC, b->NP, b->Prp, b->Pci, nullptr};
  emin_opts o = p0->opts;
  o.k1_slots = -1;
  o.k1_group = 0;
  o.profile = 0;
  o.pattern_power = 1;
  b->sup = new emin_problem();
  b->sup->ctx = ctx;
  EMIN_TRY(create_impl(ctx, &A, &Q, &P, m, b->Bv, b->Bcv, &o, b->sup));
  emin_problem* p = b->sup;
  if (p->k1.kind != 2) return fail(EMIN_ERR_UNSUPPORTED, "batched form needs the intersection map");
  // vector kernels: one lane per row (short, uneven rows); the final
  // assembly: 4 lanes per row, up to 4 slots each
  const int lm = std::max(p->lmax, 1);
  if (lm <= 16) {
    const int L = next_pow2((lm + 3) / 4);
    p->upd = {2, 1, 1, 1, 1};
    p->rowG = 4;
    p->rowL = L;
  }
  b->hist_len = o.maxit + 1;
  EMIN_TRY(b->alloc(sizeof(SegState) * count, &v)); b->segs = (SegState*)v;
  EMIN_TRY(b->alloc(sizeof(double) * 4 * (size_t)b->hist_len * count, &v)); b->shist = (double*)v;
  EMIN_TRY(b->alloc(sizeof(double) * std::max(b->N, 1), &v)); b->rowdot = (double*)v;
  // row lengths of the pattern, and of each row's longest neighbour row, for
  // the bucket plans; neighbour descriptors for the one-lane-per-row kernel
  std::vector<int> hrp(b->N + 1), len(b->N), nbmax(b->N, 0);
  EMIN_HIP(hipMemcpy(hrp.data(), p->prp, sizeof(int) * (b->N + 1), hipMemcpyDeviceToHost));
  for (int i = 0; i < b->N; ++i) len[i] = hrp[i + 1] - hrp[i];
  if ((int64_t)p->nnzP < (int64_t(1) << 27)) {
    EMIN_TRY(p->alloc((size_t)std::max(p->nnzA, 1) * sizeof(int), &v));
    p->anb = (int*)v;
    launch_build_anb(p->aci, p->nnzA, p->prp, p->anb, s);
    EMIN_TRY(p->alloc((size_t)std::max(b->N, 1) * sizeof(int), &v));
    launch_nb_maxlen(p->arp, p->aci, p->prp, b->N, (int*)v, s);
    EMIN_HIP(hipMemcpyAsync(nbmax.data(), v, sizeof(int) * b->N, hipMemcpyDeviceToHost, s));
    EMIN_HIP(hipStreamSynchronize(s));
  }
  EMIN_TRY(autotune(b, len, nbmax, tune_cache));
  // capture the whole solve once; emin_batch_solve replays it
  EMIN_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  EMIN_HIP(hipStreamSynchronize(s));
  EMIN_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  emin_status st = enqueue_batch(b, b->cap);
  hipGraph_t g = nullptr;
  hipError_t ce = hipStreamEndCapture(b->cap, &g);
  if (st != EMIN_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (ce != hipSuccess) return fail(EMIN_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
  b->graph = g;
  EMIN_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return EMIN_OK;
}

emin_status batch_solve_impl(emin_batch* b, double* const* P_vals, emin_stats* stats) {
  hipStream_t s = b->ctx->stream;
  for (int i = 0; i < b->count; ++i) {
    if (!P_vals[i] && b->members[i]->nnzP > 0) return fail(EMIN_ERR_ARG, "P_vals[i] is NULL");
    b->host_dst[i] = P_vals[i];
  }
  EMIN_HIP(hipMemcpyAsync(b->dstP, b->host_dst.data(), sizeof(double*) * b->count,
                          hipMemcpyHostToDevice, s));
  EMIN_HIP(hipGraphLaunch(b->exec, s));
  std::vector<SegState> hs(b->count);
  std::vector<double> hh(4 * (size_t)b->hist_len * b->count);
  DevState ds;
  EMIN_HIP(hipMemcpyAsync(hs.data(), b->segs, sizeof(SegState) * b->count, hipMemcpyDeviceToHost, s));
  EMIN_HIP(hipMemcpyAsync(hh.data(), b->shist, sizeof(double) * hh.size(), hipMemcpyDeviceToHost, s));
  EMIN_HIP(hipMemcpyAsync(&ds, b->sup->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  EMIN_HIP(hipStreamSynchronize(s));
  bool breakdown = false;
  for (int i = 0; i < b->count; ++i) {
    breakdown |= hs[i].stop == kBreakdown;
    if (!stats) continue;
    emin_stats& st = stats[i];
    std::memset(&st, 0, sizeof(st));
    const double* g = hh.data() + (size_t)i * 4 * b->hist_len;
    const double* al = g + 2 * b->hist_len;
    st.iterations = hs[i].iterations;
    st.stop = hs[i].stop;
    st.m = b->m;
    st.nnz_pattern = b->members[i]->nnzP;
    st.gamma1 = hs[i].gamma1;
    st.dE_first = st.iterations > 0 ? g[0] * al[0] : 0.0;
    st.dE_last = st.iterations > 0 ? g[st.iterations - 1] * al[st.iterations - 1] : 0.0;
    st.rank_deficient_rows = hs[i].rank_def;
  }
  if (ds.done == 4) return fail(EMIN_ERR_DIAG, "A(i,i) <= 0 in a batch member");
  if (breakdown) return fail(EMIN_ERR_BREAKDOWN, "RCG breakdown in a batch member");
  if (ds.rank_def > 0) {
    g_err = std::to_string(ds.rank_def) + " rows have rank(G_i) < m";
    return EMIN_WARN_RANK;
  }
  return EMIN_OK;
}


// ================================================================== adjoint

K1Shape map_shape(const emin_problem* p) {
  const int G = std::min(64, next_pow2(std::max(p->lmax, 1)));
  return K1Shape{2, G, G, 1, 1, 0};
}

emin_status ensure_map(emin_problem* p, hipStream_t s) {
  if (p->amap) return EMIN_OK;
  bool big = false;
  EMIN_TRY(build_map(p, s, &big));
  if (big) return fail(EMIN_ERR_UNSUPPORTED, "intersection map larger than 2^31 bytes");
  return EMIN_OK;
}

// y = K(A) x (kModeRaw) or Pi K(A) x (kModePlain), FP64, A values `av`
emin_status kmul(emin_problem* p, const double* av, int mode, const double* x, double* y,
                 hipStream_t s) {
  K1Args a{};
  a.arp = p->arp; a.aci = p->aci; a.av = av;
  a.mrp = p->mrp; a.amap = p->amap; a.aoff = p->aoff;
  a.prp = p->prp; a.pci = p->pci; a.y = x; a.out = y;
  a.bc = p->bc; a.wpk = p->wpk; a.m = p->m; a.n = p->n;
  a.part_out = p->part_d; a.st = p->st;
  if (launch_k1(map_shape(p), mode, 0, a, p->ctx->grid_cap, s))
    return fail(EMIN_ERR_UNSUPPORTED, "no masked-product kernel for the adjoint");
  return EMIN_OK;
}

// <x, y> (deterministic), returned on the host
emin_status dotd(emin_problem* p, int n, const double* x, const double* y, hipStream_t s,
                 double* out) {
  launch_dot(n, x, y, p->part_g, s);
  launch_reduce(p->part_g, dot_grid(n), &p->st->aux, s);
  EMIN_HIP(hipMemcpyAsync(out, &p->st->aux, sizeof(double), hipMemcpyDeviceToHost, s));
  EMIN_HIP(hipStreamSynchronize(s));
  return EMIN_OK;
}

emin_status ensure_csc(emin_problem* p, hipStream_t s) {
  if (p->ccp) return EMIN_OK;
  void *v, *cnt, *fill, *tmp;
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)(p->nc + 1), &v)); p->ccp = (int*)v;
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)std::max(p->nnzP, 1), &v)); p->cri = (int*)v;
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)std::max(p->nnzP, 1), &v)); p->cpos = (int*)v;
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)std::max(p->nc, 1), &cnt));
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)std::max(p->nc, 1), &fill));
  EMIN_TRY(p->alloc(sizeof(int) * (size_t)scan_tmp_ints(p->nc), &tmp));
  EMIN_HIP(hipMemsetAsync(cnt, 0, sizeof(int) * (size_t)std::max(p->nc, 1), s));
  EMIN_HIP(hipMemsetAsync(fill, 0, sizeof(int) * (size_t)std::max(p->nc, 1), s));
  launch_col_structure(p->prp, p->pci, p->n, p->nnzP, p->nc, (int*)cnt, p->ccp, (int*)tmp,
                       (int*)fill, p->cri, p->cpos, s);
  EMIN_HIP(hipGetLastError());
  return EMIN_OK;
}

emin_status taped_impl(emin_problem* p, double* P_vals, emin_tape** out) {
  if (p->opts.precision != EMIN_FP64 || p->opts.precond != EMIN_JACOBI)
    return fail(EMIN_ERR_UNSUPPORTED, "the adjoint covers the FP64 form with Jacobi");
  if (p->lmax > 64) return fail(EMIN_ERR_UNSUPPORTED, "the adjoint covers pattern rows up to 64");
  hipStream_t s = p->ctx->stream;
  EMIN_TRY(ensure_map(p, s));
  emin_tape* t = new emin_tape();
  t->p = p;
  t->slots = std::max(p->opts.maxit, 1);
  const size_t np = (size_t)std::max(p->nnzP, 1);
  emin_status st = EMIN_OK;
  if ((st = t->alloc(np * t->slots * 8, &t->Y)) != EMIN_OK ||
      (st = t->alloc(np * t->slots * 8, &t->R)) != EMIN_OK ||
      (st = t->alloc(np * 8, &t->p0p)) != EMIN_OK ||
      (st = t->alloc((size_t)std::max(p->nnzA, 1) * 8, &t->av)) != EMIN_OK ||
      (st = t->alloc((size_t)std::max(p->n, 1) * 8, &t->dinv)) != EMIN_OK) {
    delete t;
    return st;
  }
  st = solve_impl(p, P_vals, nullptr, nullptr, p->qv, t);
  if (st != EMIN_OK && st != EMIN_WARN_RANK) {
    delete t;
    return st;
  }
  *out = t;
  return st;
}

emin_status backward_impl(emin_tape* t, const double* Pbar, double* Abar, double* P0bar) {
  emin_problem* p = t->p;
  hipStream_t s = p->ctx->stream;
  const int np = p->nnzP, n = p->n;
  if (np == 0) return EMIN_OK;
  if (!t->Ybar) {
    double** arrs[] = {&t->Ybar, &t->Ynext, &t->Rbar, &t->Rnext, &t->Yhbar,
                       &t->U, &t->Zbar, &t->Z, &t->Yh, &t->p0bar};
    for (double** a : arrs) EMIN_TRY(t->alloc((size_t)np * 8, a));
    // scalars (8) and two dot-partial arrays
    EMIN_TRY(t->alloc(sizeof(double) * (size_t)(8 + 2 * (dot_grid(np) + 8)), &t->part));
  }
  launch_axpby(np, 0.0, nullptr, 0.0, t->Ynext, s);
  launch_axpby(np, 0.0, nullptr, 0.0, t->Rnext, s);
  // the sweep's scalars stay on the device: sc = [gnext, gbar, abar, dbar],
  // formed from dot partials by one small kernel per stage (no host reads)
  double* sc = t->part;
  double* pa = t->part + 8;
  double* pb = pa + dot_grid(np) + 8;
  const int gd = dot_grid(np);
  EMIN_HIP(hipMemsetAsync(sc, 0, 8 * sizeof(double), s));
  for (int k = t->iters; k >= 1; --k) {
    const double* Y = t->Y + (size_t)(k - 1) * np;
    const double* R = t->R + (size_t)(k - 1) * np;
    const double g = t->gamma[k - 1], dl = t->delta[k - 1], a = t->alpha[k - 1],
                 b = t->beta[k - 1];
    launch_rowscale(p->prp, t->dinv, n, R, 0.0, t->Z, s);          // Z_k = D^-1 R_k
    EMIN_TRY(kmul(p, t->av, kModePlain, Y, t->Yh, s));             // Yh_k = Pi K Y_k
    launch_axpby(np, 1.0, t->Ynext, 0.0, t->Ybar, s);              // Ybar = Ynext + a Pbar
    launch_axpby(np, a, Pbar, 1.0, t->Ybar, s);
    launch_dot(np, Pbar, Y, pa, s);                                // abar = <Pbar, Y>
    launch_dot(np, t->Rnext, t->Yh, pb, s);                        //      - <Rnext, Yh>
    launch_bwd_scalars(0, pa, gd, pb, gd, g, dl, 0.0, sc, s);
    launch_axpby(np, 1.0, t->Rnext, 0.0, t->Rbar, s);              // Rbar = Rnext
    launch_axpby(np, -a, t->Rnext, 0.0, t->Yhbar, s);              // Yhbar = -a Rnext
    launch_axpby_s(np, sc + 3, 1.0, t->Yh, 1.0, t->Ybar, s);       // dbar terms
    launch_axpby_s(np, sc + 3, 1.0, Y, 1.0, t->Yhbar, s);
    if (launch_project(p->prp, p->pci, p->bc, p->wpk, p->m, n, p->lmax, t->Yhbar, t->U, s))
      return fail(EMIN_ERR_UNSUPPORTED, "projector shape");
    EMIN_TRY(kmul(p, t->av, kModeRaw, t->U, t->Zbar, s));          // Ybar += K^T U
    launch_axpby(np, 1.0, t->Zbar, 1.0, t->Ybar, s);
    launch_sddmm(p->arp, p->prp, p->mrp, p->amap, p->aoff, n, t->U, Y, 1.0, Abar, s);
    launch_axpby(np, 1.0, t->Ybar, 0.0, t->Zbar, s);               // Zbar = Ybar
    if (k > 1) {
      const double* Yprev = t->Y + (size_t)(k - 2) * np;
      launch_dot(np, t->Ybar, Yprev, pa, s);                       // bbar = <Ybar, Y_{k-1}>
      launch_bwd_scalars(1, pa, gd, nullptr, 0, g, dl, t->gamma[k - 2], sc, s);
      launch_axpby(np, b, t->Ybar, 0.0, t->Ynext, s);
    } else {
      launch_bwd_scalars(2, nullptr, 0, nullptr, 0, g, dl, 0.0, sc, s);
    }
    launch_axpby_s(np, sc + 1, 1.0, t->Z, 1.0, t->Rbar, s);        // gamma = <R, Z>
    launch_axpby_s(np, sc + 1, 1.0, R, 1.0, t->Zbar, s);
    launch_rowscale(p->prp, t->dinv, n, t->Zbar, 1.0, t->Rbar, s); // Z = D^-1 R
    launch_diag_grad(p->arp, p->aci, t->av, p->prp, n, t->Zbar, R, Abar, s);
    std::swap(t->Rbar, t->Rnext);
  }
  // R_1 = -Pi K(A) p0'
  if (launch_project(p->prp, p->pci, p->bc, p->wpk, p->m, n, p->lmax, t->Rnext, t->U, s))
    return fail(EMIN_ERR_UNSUPPORTED, "projector shape");
  launch_axpby(np, -1.0, t->U, 0.0, t->U, s);                      // V = -Pi Rbar_1
  EMIN_TRY(kmul(p, t->av, kModeRaw, t->U, t->Zbar, s));
  launch_axpby(np, 1.0, Pbar, 0.0, t->p0bar, s);
  launch_axpby(np, 1.0, t->Zbar, 1.0, t->p0bar, s);
  launch_sddmm(p->arp, p->prp, p->mrp, p->amap, p->aoff, n, t->U, t->p0p, 1.0, Abar, s);
  // p0' = Pi p_hat + const: restrict Pi p0bar to P0's pattern
  if (launch_project(p->prp, p->pci, p->bc, p->wpk, p->m, n, p->lmax, t->p0bar, t->Yh, s))
    return fail(EMIN_ERR_UNSUPPORTED, "projector shape");
  launch_restrict(p->qrp, p->qci, p->prp, p->pci, n, t->Yh, P0bar, s);
  EMIN_HIP(hipGetLastError());
  EMIN_HIP(hipStreamSynchronize(s));
  return EMIN_OK;
}

struct LossWork {
  double *KP = nullptr, *wnp = nullptr;
  double *t1 = nullptr, *t2 = nullptr, *u = nullptr;                       // n
  double *b = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *pp = nullptr, *q = nullptr,
         *dc = nullptr;                                                    // nc
};

emin_status loss_impl(emin_problem* p, const double* P, const double* e, double wE, double wT,
                      double* L, double* dLdP, double* dLdA) {
  hipStream_t s = p->ctx->stream;
  EMIN_TRY(ensure_map(p, s));
  const int np = p->nnzP, n = p->n, nc = p->nc;
  LossWork w;
  void* v;
  EMIN_TRY(p->alloc((size_t)std::max(np, 1) * 8, &v)); w.KP = (double*)v;
  EMIN_TRY(kmul(p, p->av, kModeRaw, P, w.KP, s));
  double E = 0.0;
  EMIN_TRY(dotd(p, np, P, w.KP, s, &E));
  double Lv = wE * E;
  if (dLdP) launch_axpby(np, 2.0 * wE, w.KP, 0.0, dLdP, s);
  if (dLdA && wE != 0.0)
    launch_sddmm(p->arp, p->prp, p->mrp, p->amap, p->aoff, n, P, P, wE, dLdA, s);
  if (e && wT != 0.0) {
    EMIN_TRY(ensure_csc(p, s));
    double** nv[] = {&w.t1, &w.t2, &w.u};
    for (double** a : nv) { EMIN_TRY(p->alloc((size_t)std::max(n, 1) * 8, &v)); *a = (double*)v; }
    double** cv[] = {&w.b, &w.x, &w.r, &w.z, &w.pp, &w.q, &w.dc};
    for (double** a : cv) { EMIN_TRY(p->alloc((size_t)std::max(nc, 1) * 8, &v)); *a = (double*)v; }
    EMIN_TRY(p->alloc((size_t)std::max(np, 1) * 8, &v)); w.wnp = (double*)v;
    // c = (P^T A P)^{-1} P^T A e by Jacobi-preconditioned CG on the coarse operator
    launch_spmv(p->arp, p->aci, p->av, n, e, w.t1, s);
    launch_spmv_t(p->ccp, p->cri, p->cpos, nc, P, w.t1, w.b, s);
    launch_mul(np, P, w.KP, w.wnp, s);                              // diag(P^T A P)
    launch_spmv_t(p->ccp, p->cri, p->cpos, nc, w.wnp, nullptr, w.dc, s);
    // CG with its scalars on the device: no host round trip per iteration,
    // the residual is read back every 8 iterations
    const int gcg = dot_grid(nc);
    double *rzs, *pqp, *rzp, *rrp;
    EMIN_TRY(p->alloc(2 * sizeof(double), &v)); rzs = (double*)v;
    EMIN_TRY(p->alloc(sizeof(double) * (size_t)gcg, &v)); pqp = (double*)v;
    EMIN_TRY(p->alloc(sizeof(double) * (size_t)gcg, &v)); rzp = (double*)v;
    EMIN_TRY(p->alloc(sizeof(double) * (size_t)gcg, &v)); rrp = (double*)v;
    launch_axpby(nc, 0.0, nullptr, 0.0, w.x, s);
    launch_axpby(nc, 1.0, w.b, 0.0, w.r, s);
    launch_div(nc, w.r, w.dc, w.z, s);
    launch_axpby(nc, 1.0, w.z, 0.0, w.pp, s);
    launch_dot(nc, w.r, w.z, rzp, s);
    launch_reduce(rzp, gcg, rzs, s);
    double bb = 0.0;
    EMIN_TRY(dotd(p, nc, w.b, w.b, s, &bb));
    int cur = 0;
    for (int it = 0; it < 5000 && bb > 0.0; ++it) {
      launch_spmv(p->prp, p->pci, P, n, w.pp, w.t1, s);               // P p
      launch_spmv(p->arp, p->aci, p->av, n, w.t1, w.t2, s);           // A P p
      launch_spmv_t_dot(p->ccp, p->cri, p->cpos, nc, P, w.t2, w.pp, w.q, pqp, s);  // P^T A P p
      launch_cg_xr(nc, rzs + cur, pqp, w.pp, w.q, w.dc, w.x, w.r, w.z, rzp, rrp, s);
      launch_cg_p(nc, rzp, rzs + cur, rzs + 1 - cur, w.z, w.pp, s);
      cur = 1 - cur;
      if ((it + 1) % 8 == 0) {
        launch_reduce(rrp, gcg, &p->st->aux, s);
        double rr = 0.0;
        EMIN_HIP(hipMemcpyAsync(&rr, &p->st->aux, sizeof(double), hipMemcpyDeviceToHost, s));
        EMIN_HIP(hipStreamSynchronize(s));
        if (!(rr > 1e-28 * bb)) break;  // converged (or not a number: stop)
      }
    }
    launch_spmv(p->prp, p->pci, P, n, w.x, w.t1, s);                // u = e - P c
    launch_axpby(n, 1.0, e, 0.0, w.u, s);
    launch_axpby(n, -1.0, w.t1, 1.0, w.u, s);
    launch_spmv(p->arp, p->aci, p->av, n, w.u, w.t2, s);            // A u
    double T = 0.0;
    EMIN_TRY(dotd(p, n, w.u, w.t2, s, &T));
    Lv += wT * T;
    launch_tg_grads(p->prp, p->pci, p->arp, p->aci, n, w.t2, w.x, w.u, -2.0 * wT, wT, dLdP,
                    dLdA, s);
    EMIN_HIP(hipGetLastError());
    EMIN_HIP(hipStreamSynchronize(s));
    for (double* a : {w.t1, w.t2, w.u, w.b, w.x, w.r, w.z, w.pp, w.q, w.dc, w.wnp, rzs, pqp, rzp,
                      rrp}) {
      p->ctx->pool.put(a);
      p->owned.erase(std::find(p->owned.begin(), p->owned.end(), (void*)a));
    }
  }
  EMIN_HIP(hipGetLastError());
  EMIN_HIP(hipStreamSynchronize(s));
  p->ctx->pool.put(w.KP);
  p->owned.erase(std::find(p->owned.begin(), p->owned.end(), (void*)w.KP));
  *L = Lv;
  return EMIN_OK;
}

}  // namespace

// ------------------------------------------------- allocation-free energy --
// emin_energy_noalloc keeps everything its kernels need beyond the caller's
// arrays and the problem's fixed structure -- the result slot, the per-block
// partial sums and the slack-padded staging copy of P -- in this array.  In
// host code the name is only a stand-in: kernels receive the device address
// obtained with hipGetSymbolAddress, once per device.
constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (the current device must be
// `device`); NULL with *err set when the runtime does not give it.
void* scratch_on(int device, hipError_t* err) {
  *err = hipSuccess;
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" {

void emin_opts_default(emin_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = EMIN_FP64;
  o->precond = EMIN_JACOBI;
  o->block = 1;
  o->maxit = 10;
  o->tau = 0.0;
  o->pattern_power = 1;
  o->profile = 0;
  o->k1_group = 0;
  o->k1_slots = 0;
}

const char* emin_last_error(void) { return g_err.c_str(); }

emin_status emin_ctx_create(int device, void* hip_stream, emin_ctx** out) {
  if (!out) return fail(EMIN_ERR_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  EMIN_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(EMIN_ERR_HIP, "no such HIP device");
  EMIN_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  EMIN_HIP(hipGetDeviceProperties(&prop, device));
  emin_ctx* c = new emin_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c->grid_cap = c->num_cu * 8;
  *out = c;
  return EMIN_OK;
}

void emin_ctx_destroy(emin_ctx* ctx) { delete ctx; }

emin_status emin_problem_create(emin_ctx* ctx, const emin_csr* A, const emin_csr* P0,
                                const emin_csr* pattern, int m, const double* B,
                                const double* Bc, const emin_opts* opts, emin_problem** out) {
  if (!out) return fail(EMIN_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!ctx) return fail(EMIN_ERR_ARG, "ctx is NULL");
  g_err.clear();
  (void)hipSetDevice(ctx->device);
  emin_problem* p = new emin_problem();
  p->ctx = ctx;
  emin_status st = create_impl(ctx, A, P0, pattern, m, B, Bc, opts, p);
  if (st != EMIN_OK) {
    (void)hipStreamSynchronize(ctx->stream);
    delete p;
    return st;
  }
  *out = p;
  return EMIN_OK;
}

emin_status emin_problem_create_cf(emin_ctx* ctx, const emin_csr* A, const emin_csr* P0,
                                   const emin_csr* pattern, const int32_t* cf, int m,
                                   const double* B, const double* Bc, const emin_opts* opts,
                                   emin_problem** out) {
  if (!out) return fail(EMIN_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!ctx) return fail(EMIN_ERR_ARG, "ctx is NULL");
  if (!cf && A && A->n_rows > 0) return fail(EMIN_ERR_ARG, "cf is NULL");
  g_err.clear();
  (void)hipSetDevice(ctx->device);
  emin_problem* p = new emin_problem();
  p->ctx = ctx;
  emin_status st = create_impl(ctx, A, P0, pattern, m, B, Bc, opts, p, cf);
  if (st != EMIN_OK) {
    (void)hipStreamSynchronize(ctx->stream);
    delete p;
    return st;
  }
  *out = p;
  return EMIN_OK;
}

emin_status emin_ptent_setup(emin_ctx* ctx, const emin_csr* S, const int32_t* cf, int32_t nc,
                             const double* V, int m, int lmax, int64_t* nnz, int32_t* rowptr,
                             int32_t* colind, double* vals, int32_t* level) {
  if (!ctx || !S || !nnz) return fail(EMIN_ERR_ARG, "NULL argument");
  g_err.clear();
  (void)hipSetDevice(ctx->device);
  EMIN_TRY(check_csr_host(S, "S", S->n_rows, S->n_rows));
  const int64_t n = S->n_rows;
  if (m < 1 || m > EMIN_MAX_M) return fail(EMIN_ERR_UNSUPPORTED, "m must be 1..8");
  if (lmax < 1 || lmax > 16) return fail(EMIN_ERR_ARG, "lmax must be 1..16");
  if (nc < 0 || nc > n) return fail(EMIN_ERR_ARG, "nc out of range");
  if (n > 0 && (!cf || !V || !rowptr || !colind || !vals))
    return fail(EMIN_ERR_ARG, "cf, V, rowptr, colind and vals are required");
  *nnz = 0;
  if (n == 0) return EMIN_OK;
  hipStream_t s = ctx->stream;
  std::vector<void*> tmp;
  auto get = [&](size_t b, void** q) {
    emin_status r = ctx->pool.get(b, q);
    if (r == EMIN_OK) tmp.push_back(*q);
    return r;
  };
  auto release = [&]() {
    for (void* q : tmp) ctx->pool.put(q);
  };
  void *flags, *seen, *cnt, *cols, *wv, *stmp;
  emin_status st = EMIN_OK;
  if ((st = get(8 * sizeof(int), &flags)) != EMIN_OK ||
      (st = get(sizeof(int) * (size_t)std::max<int32_t>(nc, 1), &seen)) != EMIN_OK ||
      (st = get(sizeof(int) * (size_t)n, &cnt)) != EMIN_OK ||
      (st = get(sizeof(int) * (size_t)n * m, &cols)) != EMIN_OK ||
      (st = get(sizeof(double) * (size_t)n * m, &wv)) != EMIN_OK ||
      (st = get(sizeof(int) * (size_t)scan_tmp_ints((int)n), &stmp)) != EMIN_OK) {
    release();
    return st;
  }
  int fl = 0, nz = 0;
  hipError_t he = hipMemsetAsync(flags, 0, 8 * sizeof(int), s);
  if (he == hipSuccess) he = hipMemsetAsync(seen, 0, sizeof(int) * (size_t)std::max(nc, 1), s);
  if (he == hipSuccess) {
    launch_check_csr(S->rowptr, S->colind, (int)n, (int)n, (int)S->nnz, (int*)flags, kFlagCsrA, s);
    launch_cf_check(cf, (int)n, nc, (int*)seen, nullptr, nullptr, nullptr, (int*)flags, s);
    he = hipMemcpyAsync(&fl, flags, sizeof(int), hipMemcpyDeviceToHost, s);
  }
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) {
    release();
    return fail(EMIN_ERR_HIP, hipGetErrorString(he));
  }
  if (fl & (1 << kFlagCsrA)) {
    release();
    return fail(EMIN_ERR_CSR, "S: invalid CSR (rowptr, range, order)");
  }
  if (fl & (1 << kFlagCF)) {
    release();
    return fail(EMIN_ERR_ARG, "cf: an entry is outside [-1, nc) or a coarse index is not held "
                              "by exactly one node");
  }
  if (launch_ptent_rows(S->rowptr, S->colind, cf, V, (int)n, m, lmax, (int*)cnt, (int*)cols,
                        (double*)wv, level, (int*)flags, s)) {
    release();
    return fail(EMIN_ERR_UNSUPPORTED, "no Alg. 1 kernel for this m");
  }
  launch_exclusive_scan((int*)cnt, (int)n, rowptr, (int*)stmp, s);
  launch_ptent_compact((int*)cnt, (int*)cols, (double*)wv, rowptr, (int)n, m, colind, vals, s);
  he = hipGetLastError();
  if (he == hipSuccess) he = hipMemcpyAsync(&fl, flags, sizeof(int), hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipMemcpyAsync(&nz, rowptr + n, sizeof(int), hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  release();
  if (he != hipSuccess) return fail(EMIN_ERR_HIP, hipGetErrorString(he));
  if (fl & 1)
    return fail(EMIN_ERR_UNSUPPORTED, "Alg. 1: a neighbourhood within lmax holds more than "
                                      "1024 nodes or 128 COARSE nodes");
  *nnz = nz;
  return EMIN_OK;
}

void emin_problem_destroy(emin_problem* p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->ctx->stream);
  delete p;
}

emin_status emin_pattern_get(emin_problem* p, int64_t* nnz, int32_t* rowptr, int32_t* colind) {
  if (!p || !nnz) return fail(EMIN_ERR_ARG, "NULL argument");
  *nnz = p->nnzP;
  hipStream_t s = p->ctx->stream;
  if (rowptr) EMIN_HIP(hipMemcpyAsync(rowptr, p->prp, sizeof(int) * (p->n + 1), hipMemcpyDeviceToDevice, s));
  if (colind && p->nnzP) EMIN_HIP(hipMemcpyAsync(colind, p->pci, sizeof(int) * p->nnzP, hipMemcpyDeviceToDevice, s));
  EMIN_HIP(hipStreamSynchronize(s));
  return EMIN_OK;
}

emin_status emin_sgs_colours_get(emin_problem* p, int32_t* ncolours, int32_t* colour) {
  if (!p || !ncolours) return fail(EMIN_ERR_ARG, "NULL argument");
  if (p->opts.precond != EMIN_SGS) return fail(EMIN_ERR_ARG, "the problem is not EMIN_SGS");
  *ncolours = (int32_t)p->coff.size() - 1;
  if (colour && p->n > 0) {
    hipStream_t s = p->ctx->stream;
    EMIN_HIP(hipMemcpyAsync(colour, p->colour, sizeof(int) * (size_t)p->n,
                            hipMemcpyDeviceToDevice, s));
    EMIN_HIP(hipStreamSynchronize(s));
  }
  return EMIN_OK;
}

emin_status emin_solve(emin_problem* p, double* P_vals, double* dE_hist, emin_stats* stats) {
  if (!p) return fail(EMIN_ERR_ARG, "problem is NULL");
  if (!P_vals && p->nnzP > 0) return fail(EMIN_ERR_ARG, "P_vals is NULL");
  g_err.clear();
  (void)hipSetDevice(p->ctx->device);
  return solve_impl(p, P_vals, dE_hist, stats, p->qv);
}

emin_status emin_energy(emin_problem* p, const double* P_vals, double* E) {
  if (!p || !E || (!P_vals && p->nnzP > 0)) return fail(EMIN_ERR_ARG, "NULL argument");
  hipStream_t s = p->ctx->stream;
  if (p->nnzP == 0) { *E = 0.0; return EMIN_OK; }
  const double* x = staged(p, P_vals);
  if (!x) return fail(EMIN_ERR_HIP, "staging copy failed");
  EMIN_TRY(k1_call(p, kModeEnergy, 0, p->av, x, nullptr));
  launch_reduce(p->part_d, k1_grid(p->k1, p->n, p->ctx->grid_cap), &p->st->energy, s);
  EMIN_HIP(hipGetLastError());
  DevState hs;
  EMIN_HIP(hipMemcpyAsync(&hs, p->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  EMIN_HIP(hipStreamSynchronize(s));
  *E = hs.energy;
  return EMIN_OK;
}

emin_status emin_energy_noalloc(emin_problem* p, const double* P_vals, double* E) {
  if (!p || !E || (!P_vals && p->nnzP > 0)) return fail(EMIN_ERR_ARG, "NULL argument");
  if (p->nnzP == 0) { *E = 0.0; return EMIN_OK; }
  // layout: result slot | per-block partials | staged copy of P with 64 bytes of slack
  const size_t off_part = 256;
  const size_t np = (size_t)p->ctx->grid_cap + 64;
  const size_t off_stage = round256(off_part + np * sizeof(double));
  const bool stage = p->k1.kind == 3 || p->k1.kind == 4;
  const size_t need = off_stage + (stage ? (size_t)p->nnzP * sizeof(double) + 64 : 0);
  if (need > kScratchBytes)
    return fail(EMIN_ERR_UNSUPPORTED,
                "emin_energy_noalloc: nnz(pattern) = " + std::to_string(p->nnzP) +
                    " needs " + std::to_string(need) + " bytes of scratch, the limit is " +
                    std::to_string(kScratchBytes));
  (void)hipSetDevice(p->ctx->device);
  hipError_t he;
  unsigned char* base = (unsigned char*)scratch_on(p->ctx->device, &he);
  if (!base) return fail(EMIN_ERR_HIP, std::string("scratch address: ") + hipGetErrorString(he));
  hipStream_t s = p->ctx->stream;
  double* result = (double*)base;
  double* part = (double*)(base + off_part);
  const double* x = P_vals;
  if (stage) {
    EMIN_HIP(hipMemcpyAsync(base + off_stage, P_vals, sizeof(double) * (size_t)p->nnzP,
                            hipMemcpyDeviceToDevice, s));
    x = (const double*)(base + off_stage);
  }
  K1Args a{};
  a.arp = p->arp; a.aci = p->aci; a.av = p->av; a.anb = p->anb;
  a.mrp = p->mrp; a.aoff = p->aoff;
  a.amap = p->k1.kind == 4 ? p->nmap : p->k1.kind == 5 ? p->gmap : p->amap;
  a.mrp64 = p->k1.kind == 5 ? p->gmrp : p->nmrp;
  a.nnz_p = p->nnzP; a.nqrp = p->nqrp; a.nq = p->nq; a.grp = p->grp;
  a.win = p->win; a.nwin = p->k1.nwin;
  a.prp = p->prp; a.pci = p->pci;
  a.y = x; a.out = nullptr;
  a.bc = p->bc; a.wpk = p->wpk; a.m = p->m; a.n = p->n;
  a.part_out = part; a.st = p->st;  // the energy kernels do not read the state
  if (launch_k1(p->k1, kModeEnergy, 0, a, p->ctx->grid_cap, s))
    return fail(EMIN_ERR_UNSUPPORTED, "no masked-product kernel for this shape");
  launch_reduce(part, k1_grid(p->k1, p->n, p->ctx->grid_cap), result, s);
  EMIN_HIP(hipGetLastError());
  double e = 0.0;
  EMIN_HIP(hipMemcpyAsync(&e, result, sizeof(double), hipMemcpyDeviceToHost, s));
  EMIN_HIP(hipStreamSynchronize(s));
  *E = e;
  return EMIN_OK;
}

emin_status emin_constraint_error(emin_problem* p, const double* P_vals, double* rel) {
  if (!p || !rel || (!P_vals && p->nnzP > 0)) return fail(EMIN_ERR_ARG, "NULL argument");
  if (p->n == 0) { *rel = 0.0; return EMIN_OK; }
  hipStream_t s = p->ctx->stream;
  ConsArgs a{};
  a.prp = p->prp; a.pci = p->pci; a.P = P_vals; a.B = p->B; a.bc = p->bc; a.m = p->m;
  a.n = p->n; a.part_num = p->part_d; a.part_den = p->part_g;
  if (launch_constraint(p->rowG, p->rowL, a, p->ctx->grid_cap, s))
    return fail(EMIN_ERR_UNSUPPORTED, "no constraint kernel for this shape");
  const int g = constraint_grid(p->rowG, p->n, p->ctx->grid_cap);
  launch_reduce(p->part_d, g, &p->st->aux, s);
  launch_reduce(p->part_g, g, &p->st->energy, s);
  EMIN_HIP(hipGetLastError());
  DevState hs;
  EMIN_HIP(hipMemcpyAsync(&hs, p->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  EMIN_HIP(hipStreamSynchronize(s));
  *rel = hs.energy > 0.0 ? std::sqrt(hs.aux / hs.energy) : std::sqrt(hs.aux);
  return EMIN_OK;
}

emin_status emin_batch_create(emin_ctx* ctx, int count, emin_problem* const* probs,
                              const char* tune_cache, emin_batch** out) {
  if (!out) return fail(EMIN_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!ctx) return fail(EMIN_ERR_ARG, "ctx is NULL");
  g_err.clear();
  (void)hipSetDevice(ctx->device);
  emin_batch* b = new emin_batch();
  b->ctx = ctx;
  emin_status st = batch_create_impl(ctx, count, probs, tune_cache, b);
  if (st != EMIN_OK) {
    (void)hipStreamSynchronize(ctx->stream);
    delete b;
    return st;
  }
  *out = b;
  return EMIN_OK;
}

emin_status emin_batch_solve(emin_batch* b, double* const* P_vals, emin_stats* stats) {
  if (!b || !P_vals) return fail(EMIN_ERR_ARG, "NULL argument");
  g_err.clear();
  (void)hipSetDevice(b->ctx->device);
  return batch_solve_impl(b, P_vals, stats);
}

int emin_batch_plan(const emin_batch* b, char* buf, int cap) {
  if (!b) return -1;
  const int need = (int)b->plan_json.size() + 1;
  if (buf && cap > 0) {
    std::strncpy(buf, b->plan_json.c_str(), (size_t)cap - 1);
    buf[cap - 1] = 0;
  }
  return need;
}

void emin_batch_destroy(emin_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->ctx->stream);
  delete b;
}

emin_status emin_solve_taped(emin_problem* p, double* P_vals, emin_tape** tape) {
  if (!p || !tape || (!P_vals && p->nnzP > 0)) return fail(EMIN_ERR_ARG, "NULL argument");
  *tape = nullptr;
  g_err.clear();
  (void)hipSetDevice(p->ctx->device);
  return taped_impl(p, P_vals, tape);
}

emin_status emin_backward(emin_tape* tape, const double* dL_dP, double* dL_dA, double* dL_dP0) {
  if (!tape || (tape->p->nnzP > 0 && (!dL_dP || !dL_dA || !dL_dP0)))
    return fail(EMIN_ERR_ARG, "NULL argument");
  g_err.clear();
  (void)hipSetDevice(tape->p->ctx->device);
  return backward_impl(tape, dL_dP, dL_dA, dL_dP0);
}

void emin_tape_destroy(emin_tape* tape) {
  if (!tape) return;
  (void)hipStreamSynchronize(tape->p->ctx->stream);
  delete tape;
}

emin_status emin_loss(emin_problem* p, const double* P_vals, const double* e, double w_energy,
                      double w_twogrid, double* L, double* dL_dP, double* dL_dA) {
  if (!p || !L || (!P_vals && p->nnzP > 0)) return fail(EMIN_ERR_ARG, "NULL argument");
  if (p->lmax > 64) return fail(EMIN_ERR_UNSUPPORTED, "the loss covers pattern rows up to 64");
  g_err.clear();
  (void)hipSetDevice(p->ctx->device);
  return loss_impl(p, P_vals, e, w_energy, w_twogrid, L, dL_dP, dL_dA);
}

emin_status emin_loss_forward(emin_problem* p, const double* P_vals, const double* e,
                              double w_energy, double w_twogrid, double* L) {
  return emin_loss(p, P_vals, e, w_energy, w_twogrid, L, nullptr, nullptr);
}

emin_status emin_loss_backward(emin_problem* p, const double* P_vals, const double* e,
                               double w_energy, double w_twogrid, double* dL_dP, double* dL_dA) {
  double L = 0.0;
  return emin_loss(p, P_vals, e, w_energy, w_twogrid, &L, dL_dP, dL_dA);
}

emin_status emin_masked_product(emin_problem* p, const double* Y, double* Y_hat) {
  if (!p || ((!Y || !Y_hat) && p->nnzP > 0)) return fail(EMIN_ERR_ARG, "NULL argument");
  if (p->m > 1 && !p->have_factors)
    return fail(EMIN_ERR_ARG, "emin_masked_product needs a prior emin_solve (factors)");
  if (p->nnzP == 0) return EMIN_OK;
  if (p->k1.kind == 5) {
    // the node-pair product has no projecting form: mask(A Y), then Pi
    if (!p->stage) {
      void* v;
      EMIN_TRY(p->alloc(sizeof(double) * (size_t)std::max(p->nnzP, 1), &v));
      p->stage = (double*)v;
    }
    EMIN_TRY(k1_call(p, kModeRaw, 0, p->av, Y, p->stage));
    if (launch_project(p->prp, p->pci, p->bc, p->wpk, p->m, p->n, p->lmax, p->stage, Y_hat,
                       p->ctx->stream))
      return fail(EMIN_ERR_UNSUPPORTED, "no projection kernel for this row length");
    EMIN_HIP(hipGetLastError());
    return EMIN_OK;
  }
  const double* x = staged(p, Y);
  if (!x) return fail(EMIN_ERR_HIP, "staging copy failed");
  EMIN_TRY(k1_call(p, kModePlain, 0, p->av, x, Y_hat));
  EMIN_HIP(hipGetLastError());
  return EMIN_OK;
}

}  // extern "C"
