// Batched form: many independent matrices solved as one block-diagonal
// problem.  Rows of matrix b form the segment [seg_row[b], seg_row[b+1]),
// in the order the batch chose for locality; values are gathered into, and
// P scattered out of, that order through member-local index maps.
// The vector kernels run over all rows at once; every dot product is kept
// per row (rowdot) and reduced here per segment in two fixed-order stages --
// chunks of up to kSegChunk rows inside a segment, one block each, then one
// block per matrix over its chunks -- so each matrix gets its own
// deterministic CG scalars (Alg. 3: gamma, delta, alpha, beta, dE, the stop
// tests) without host round trips.
#include "common.hpp"
#include "launch.hpp"

namespace emin {

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

__global__ void k_seg_init(SegState* segs, int nseg) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  segs[s].gamma1 = 0.0;
  segs[s].dE1 = 0.0;
  segs[s].alpha = 0.0;
  segs[s].beta = 0.0;
  segs[s].stop = 0;
  segs[s].iterations = 0;
  segs[s].rank_def = 0;
}

// stage 1: one block per chunk of rows (chunks never straddle segments)
__global__ __launch_bounds__(kBlock) void k_seg_chunks(SegArgs a) {
  const int c = blockIdx.x;
  const int r0 = a.chunk_row[c], r1 = a.chunk_row[c + 1];
  double v = 0.0;
  for (int i = r0 + threadIdx.x; i < r1; i += kBlock) v += a.rowdot[i];
  const double t = block_sum(v);
  if (threadIdx.x == 0) a.chunk_sum[c] = t;
}

// stage 2: a segment's chunk sums, in order (every thread gets the total)
__device__ __forceinline__ double seg_sum(const SegArgs& a, int s) {
  const int c0 = a.seg_chunk[s], c1 = a.seg_chunk[s + 1];
  __shared__ double red[kBlock / kWave];
  double v = 0.0;
  for (int c = c0 + threadIdx.x; c < c1; c += kBlock) v += a.chunk_sum[c];
  v = wave_sum(v);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) t += red[w];
  return t;
}

// hist layout per segment: [gamma | delta | alpha | beta], hist_len each
__device__ __forceinline__ double* seg_hist(const SegArgs& a, int s, int which) {
  return a.hist + ((long)s * 4 + which) * a.hist_len;
}

// after <Y, Y_hat> of iteration k: alpha, dE, energy-monitor stop, breakdown
__global__ __launch_bounds__(kBlock) void k_seg_delta(SegArgs a) {
  const int s = blockIdx.x;
  if (a.segs[s].stop) return;
  const double delta = seg_sum(a, s);
  if (threadIdx.x != 0) return;
  SegState& sg = a.segs[s];
  const int k = a.k;
  const double gk = seg_hist(a, s, 0)[k - 1];
  seg_hist(a, s, 1)[k - 1] = delta;
  if (!(delta > 0.0)) {
    sg.stop = kBreakdown;
    return;
  }
  const double alpha = gk / delta;
  const double dE = gk * alpha;
  if (k == 1) sg.dE1 = dE;
  sg.alpha = alpha;
  seg_hist(a, s, 2)[k - 1] = alpha;
  if (a.tau > 0.0 && dE < a.tau * sg.dE1) sg.stop = kTauStop;
}

// after <R, Z> (gamma of iteration k + 1): floor, breakdown, beta
__global__ __launch_bounds__(kBlock) void k_seg_gamma(SegArgs a, int first) {
  const int s = blockIdx.x;
  if (a.segs[s].stop) return;
  const double gamma = seg_sum(a, s);
  if (threadIdx.x != 0) return;
  SegState& sg = a.segs[s];
  const int k = a.k;
  sg.iterations = k;
  if (first) sg.gamma1 = gamma;
  double beta = 0.0;
  if (gamma < 0.0 || gamma != gamma) sg.stop = kBreakdown;
  else if (gamma <= a.gamma_floor * sg.gamma1) sg.stop = kConverged;
  else if (!first) beta = gamma / seg_hist(a, s, 0)[k - 1];
  sg.beta = beta;
  if (k < a.hist_len) {
    seg_hist(a, s, 0)[k] = gamma;
    seg_hist(a, s, 3)[k] = beta;
  }
}

// one block per segment, grid-stride over its range
__global__ __launch_bounds__(kBlock) void k_gather(const double* const* __restrict__ src,
                                                  const long* __restrict__ off,
                                                  double* __restrict__ dst) {
  const int b = blockIdx.x;
  const long o = off[b], len = off[b + 1] - o;
  const double* __restrict__ s = src[b];
  for (long j = blockIdx.y * (long)kBlock + threadIdx.x; j < len; j += (long)gridDim.y * kBlock)
    dst[o + j] = s[j];
}

__global__ __launch_bounds__(kBlock) void k_scatter(const double* __restrict__ src,
                                                   const long* __restrict__ off,
                                                   double* const* __restrict__ dst) {
  const int b = blockIdx.x;
  const long o = off[b], len = off[b + 1] - o;
  double* __restrict__ d = dst[b];
  for (long j = blockIdx.y * (long)kBlock + threadIdx.x; j < len; j += (long)gridDim.y * kBlock)
    d[j] = src[o + j];
}

// the same through a member-local index map: dst[o + j] = src_b[map[o + j]]
__global__ __launch_bounds__(kBlock) void k_gather_map(const double* const* __restrict__ src,
                                                      const long* __restrict__ off,
                                                      const int* __restrict__ map,
                                                      double* __restrict__ dst) {
  const int b = blockIdx.x;
  const long o = off[b], len = off[b + 1] - o;
  const double* __restrict__ s = src[b];
  for (long j = blockIdx.y * (long)kBlock + threadIdx.x; j < len; j += (long)gridDim.y * kBlock)
    dst[o + j] = s[map[o + j]];
}

// dst_b[map[o + j]] = src[o + j]
// Member b's output in its own entry order: entry j comes from position
// inv[o + j] of the member's stretch of the batch layout (the inverse of
// the layout's permutation), so the writes are contiguous and the scattered
// reads stay inside one member's stretch.
__global__ __launch_bounds__(kBlock) void k_scatter_map(const double* __restrict__ src,
                                                       const long* __restrict__ off,
                                                       const int* __restrict__ inv,
                                                       double* const* __restrict__ dst) {
  const int b = blockIdx.x;
  const long o = off[b], len = off[b + 1] - o;
  double* __restrict__ d = dst[b];
  const long stride = (long)gridDim.y * kBlock;
  long j = blockIdx.y * (long)kBlock + threadIdx.x;
  // four entries per step, every index load issued before the value loads
  for (; j + 3 * stride < len; j += 4 * stride) {
    int q[4];
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] = inv[o + j + u * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = src[o + q[u]];
#pragma unroll
    for (int u = 0; u < 4; ++u) d[j + u * stride] = v[u];
  }
  for (; j < len; j += stride) d[j] = src[o + inv[o + j]];
}

__global__ __launch_bounds__(kBlock) void k_shift_copy(const int* __restrict__ in, int len,
                                                      int add, int* __restrict__ out) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j < len) out[j] = in[j] + add;
}

void launch_seg_init(SegState* segs, int nseg, hipStream_t s) {
  if (nseg > 0) k_seg_init<<<cdiv(nseg, kBlock), kBlock, 0, s>>>(segs, nseg);
}

void launch_seg_delta(const SegArgs& a, hipStream_t s) {
  if (a.nseg <= 0) return;
  if (a.nchunk > 0) k_seg_chunks<<<a.nchunk, kBlock, 0, s>>>(a);
  k_seg_delta<<<a.nseg, kBlock, 0, s>>>(a);
}

void launch_seg_gamma(const SegArgs& a, int first, hipStream_t s) {
  if (a.nseg <= 0) return;
  if (a.nchunk > 0) k_seg_chunks<<<a.nchunk, kBlock, 0, s>>>(a);
  k_seg_gamma<<<a.nseg, kBlock, 0, s>>>(a, first);
}

void launch_gather_segments(const double* const* src, const long* off, int count, double* dst,
                            hipStream_t s) {
  if (count > 0) k_gather<<<dim3(count, 8), kBlock, 0, s>>>(src, off, dst);
}

void launch_scatter_segments(const double* src, const long* off, int count, double* const* dst,
                             hipStream_t s) {
  if (count > 0) k_scatter<<<dim3(count, 8), kBlock, 0, s>>>(src, off, dst);
}

void launch_gather_map(const double* const* src, const long* off, const int* map, int count,
                       double* dst, hipStream_t s) {
  if (count > 0) k_gather_map<<<dim3(count, 8), kBlock, 0, s>>>(src, off, map, dst);
}

void launch_scatter_map(const double* src, const long* off, const int* inv, int count,
                        double* const* dst, hipStream_t s) {
  if (count > 0) k_scatter_map<<<dim3(count, 32), kBlock, 0, s>>>(src, off, inv, dst);
}

void launch_shift_copy(const int* in, int len, int add, int* out, hipStream_t s) {
  if (len > 0) k_shift_copy<<<cdiv(len, kBlock), kBlock, 0, s>>>(in, len, add, out);
}

}  // namespace emin
