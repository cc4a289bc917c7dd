// Device-side building blocks shared by the HIP kernels: wave/group/block
// reductions, the XCD-aware tile walk, and the per-solve device state that
// holds the CG scalars so the iteration never waits on the host.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace emin {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kBlock = 256;        // threads per block for every kernel
constexpr int kNumXcd = 8;         // MI355X: 8 XCDs x 32 CUs, blocks dealt round-robin
constexpr int kMaxM = 8;

// Values the whole wave reads at one address (A's node blocks, neighbour
// descriptors, a node's row pointers, W and block-inverse factors) go
// through the constant address space, which the compiler loads with scalar
// instructions: they leave the vector memory pipeline free for the per-lane
// traffic.  Only for data no kernel of the same launch writes.
template <class T>
using Uniform = const __attribute__((address_space(4))) T;

// Stop codes stored in DevState::done (match EMIN_STOP_*).
enum : int { kRunning = 0, kConverged = 1, kTauStop = 2, kBreakdown = 3 };

// One per problem; lives in device memory.  Written only by block 0 of the
// kernel that completes a reduction, read by later kernels in stream order.
// Values a later block of the same kernel might still need (gamma_k) are
// read from the history arrays instead, which are written once per index.
struct DevState {
  double gamma;       // <r_k, z_k>
  double gamma_old;
  double gamma1;
  double delta;       // <y_k, Pi K y_k>
  double alpha;
  double beta;
  double dE1;
  double energy;      // result slot for the energy / constraint kernels
  double aux;
  double tau;
  int k;              // iteration whose masked product ran last
  int iterations;     // updates applied
  int done;           // kRunning or a stop code
  int rank_def;       // rows with rank(G_i) < m
};

// Scalars of one matrix of a batch (a segment of consecutive rows of the
// block-diagonal batch problem).  Written by the per-segment reduction
// kernels, read by the vector kernels that follow them.
struct SegState {
  double gamma1;
  double dE1;
  double alpha;
  double beta;
  int stop;          // kRunning or a stop code
  int iterations;
  int rank_def;      // the matrix's rows with rank(G_i) < m
  int pad1;
};

// Segment holding row i: the largest s with seg_row[s] <= i.
__device__ __forceinline__ int find_seg(const int* __restrict__ seg_row, int nseg, int i) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (seg_row[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// History arrays (device), each of length maxit.
struct DevHist {
  double* gamma;
  double* delta;
  double* alpha;
  double* beta;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Sum over an aligned group of G lanes (G a power of two <= 64); every lane
// of the group receives the total.
template <int G, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int d = G / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Reduce-scatter over an aligned group of G lanes by recursive halving.  On
// entry every lane holds LEN partial sums acc[0..LEN); on exit lane l of the
// group holds, in acc[0..LEN/G), the group totals of slots l*LEN/G ..
// (l+1)*LEN/G - 1.  log2(G) exchange steps, LEN - LEN/G shuffles in total.
template <int G, int LEN, class T>
struct ReduceScatter {
  static __device__ __forceinline__ void run(T* acc, int lane) {
    if constexpr (G > 1) {
      constexpr int D = G / 2;
      constexpr int H = LEN / 2;
      const bool up = (lane & D) != 0;
#pragma unroll
      for (int j = 0; j < H; ++j) {
        T lo = acc[j], hi = acc[j + H];
        T send = up ? lo : hi;
        T keep = up ? hi : lo;
        acc[j] = keep + __shfl_xor(send, D, kWave);
      }
      ReduceScatter<D, H, T>::run(acc, lane);
    }
  }
};

// Block-wide sum of one double per thread; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kBlock / kWave];
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) t += red[i];
  }
  return t;
}

// Tiles dealt so each XCD owns one contiguous range: blocks land on XCDs
// round-robin (block b on XCD b % 8), so block b walks tiles of range
// (b % 8) with stride gridDim.x / 8.  Neighbouring rows then share an L2.
// gridDim.x must be a multiple of kNumXcd.
struct TileWalk {
  int t, end, step;
  __device__ __forceinline__ TileWalk(int ntiles) {
    const int x = blockIdx.x % kNumXcd;
    const int slot = blockIdx.x / kNumXcd;
    const int per = gridDim.x / kNumXcd;
    const int chunk = (ntiles + kNumXcd - 1) / kNumXcd;
    const int s = x * chunk;
    end = min(s + chunk, ntiles);
    t = s + slot;
    step = per;
  }
};

// Grid reductions are deferred to the next kernel in the stream: every block
// of the producer stores one partial (plain store; the kernel boundary makes
// it visible), and every block of the consumer sums all partials in index
// order with the same tree, so all blocks obtain the identical value and the
// result does not depend on scheduling.  No device-scope fences or atomics:
// on this GPU each XCD has its own L2, and an agent-scope release per block
// would write back L2 once per block.
__device__ __forceinline__ void store_partial(double v, double* partials) {
  const double t = block_sum(v);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// Sum of partials[0..np) broadcast to every thread of the block.
__device__ __forceinline__ double sum_partials(const double* __restrict__ partials, int np) {
  __shared__ double red[kBlock / kWave];
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += kBlock) v += partials[i];
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < kBlock / kWave; ++i) t += red[i];
  return t;
}

template <class T> struct Acc;
template <> struct Acc<double> { using type = double; };
template <> struct Acc<float> { using type = float; };

}  // namespace emin
