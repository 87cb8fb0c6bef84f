// Device-wide exclusive prefix sum of int32 counts (bin counts, pair counts, bucket
// counts), out[0..n-1] and the total out[n], in two launches: the totals of 1024-element
// blocks, then each block's scan from the sum of the totals before it (at most a few
// thousand, read by every block). Deterministic (integer).
#include "common.h"

namespace flare {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_PER_THREAD = 4;
constexpr int SCAN_BLOCK = SCAN_THREADS * SCAN_PER_THREAD;   // 1024 elements per block

__device__ inline int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// Phase 1: the total of every 1024-element block.
__global__ __launch_bounds__(SCAN_THREADS) void k_block_sums(const int* __restrict__ in, int n,
                                                              int* __restrict__ sums) {
  __shared__ int wsum[SCAN_THREADS / 64];
  const long long base = (long long)blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_PER_THREAD;
  int tot = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER_THREAD; ++k) tot += base + k < n ? in[base + k] : 0;
  const int incl = wave_incl_scan(tot);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int k = 0; k < SCAN_THREADS / 64; ++k) t += wsum[k];
    sums[blockIdx.x] = t;
  }
}

// Phase 2: every block adds up the totals of the blocks before it (nb of them at most),
// scans its own elements from there and writes them; the block holding element n - 1
// (block 0 when n == 0) also writes the total out[n].
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_blocks(const int* __restrict__ in, int* __restrict__ out,
                                                               int n, const int* __restrict__ sums) {
  __shared__ int wsum[SCAN_THREADS / 64];
  __shared__ int pre_s;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int pre = 0;
  for (int k = threadIdx.x; k < (int)blockIdx.x; k += SCAN_THREADS) pre += sums[k];
  pre = wave_incl_scan(pre);
  if (lane == 63) wsum[w] = pre;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int k = 0; k < SCAN_THREADS / 64; ++k) t += wsum[k];
    pre_s = t;
  }
  __syncthreads();
  const int block_pre = pre_s;
  const long long base = (long long)blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_PER_THREAD;
  int v[SCAN_PER_THREAD];
  int tot = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER_THREAD; ++k) {
    v[k] = base + k < n ? in[base + k] : 0;
    tot += v[k];
  }
  const int incl = wave_incl_scan(tot);
  __syncthreads();                       // wsum is reused
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int woff = 0;
  for (int k = 0; k < w; ++k) woff += wsum[k];
  int run = block_pre + woff + incl - tot;
#pragma unroll
  for (int k = 0; k < SCAN_PER_THREAD; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  // the total: written by the thread that holds element n - 1 (its running sum has passed
  // it; the elements past n counted as zeros), or by thread 0 when n == 0
  if (n == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
  } else if (base <= (long long)n - 1 && (long long)n - 1 < base + SCAN_PER_THREAD) {
    out[n] = run;
  }
}

int nblocks(long long n) { return (int)((n + SCAN_BLOCK - 1) / SCAN_BLOCK); }

}  // namespace

size_t scan_scratch_ints(long long n) { return (size_t)nblocks(n) + 64; }

// Two launches (one when n fits one block): block totals, then every block's scan from
// the sum of the totals before it.
void scan_exclusive(const int* in, int* out, int n, int* scratch, hipStream_t st) {
  const int nb = n > 0 ? nblocks(n) : 1;
  if (nb > 1) k_block_sums<<<nb, SCAN_THREADS, 0, st>>>(in, n, scratch);
  k_scan_blocks<<<nb, SCAN_THREADS, 0, st>>>(in, out, n, scratch);
}

}  // namespace flare
