// Device-wide exclusive prefix sum of int32 counts (bin counts, pair counts, bucket
// counts). Three phases per level: block scans with block totals, a recursive scan of
// the totals, and the add-back. Deterministic (integer, fixed order).
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

// Exclusive scan of one 1024-element block; writes block total to sums[blockIdx].
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_block(const int* __restrict__ in,
                                                              int* __restrict__ out, int n,
                                                              int* __restrict__ sums) {
  __shared__ int wsum[SCAN_THREADS / 64];
  const long long base = (long long)blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_PER_THREAD;
  int v[SCAN_PER_THREAD];
  int tot = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER_THREAD; ++k) {
    long long idx = base + k;
    v[k] = idx < n ? in[idx] : 0;
    tot += v[k];
  }
  int incl = wave_incl_scan(tot);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int woff = 0;
  for (int k = 0; k < w; ++k) woff += wsum[k];
  int run = woff + incl - tot;
#pragma unroll
  for (int k = 0; k < SCAN_PER_THREAD; ++k) {
    long long idx = base + k;
    if (idx < n) out[idx] = run;
    run += v[k];
  }
  if (threadIdx.x == SCAN_THREADS - 1) sums[blockIdx.x] = woff + incl;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_add(int* __restrict__ out, int n,
                                                            const int* __restrict__ offs) {
  const long long base = (long long)blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_PER_THREAD;
  const int add = offs[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SCAN_PER_THREAD; ++k) {
    long long idx = base + k;
    if (idx < n) out[idx] += add;
  }
}

__global__ void k_scan_total(int* __restrict__ out, int n, const int* __restrict__ in) {
  // out[n] = out[n-1] + in[n-1]  (n >= 1), or 0 when n == 0
  if (threadIdx.x == 0 && blockIdx.x == 0) out[n] = n > 0 ? out[n - 1] + in[n - 1] : 0;
}

int nblocks(long long n) { return (int)((n + SCAN_BLOCK - 1) / SCAN_BLOCK); }

// out[0..n-1] exclusive scan (no total)
void scan_level(const int* in, int* out, int n, int* scratch, hipStream_t st) {
  if (n <= 0) return;
  const int nb = nblocks(n);
  int* sums = scratch;
  int* sums_scan = scratch + nb;
  int* next = scratch + 2 * nb;
  k_scan_block<<<nb, SCAN_THREADS, 0, st>>>(in, out, n, sums);
  if (nb > 1) {
    scan_level(sums, sums_scan, nb, next, st);
    k_scan_add<<<nb, SCAN_THREADS, 0, st>>>(out, n, sums_scan);
  }
}

}  // namespace

size_t scan_scratch_ints(long long n) {
  size_t tot = 0;
  while (n > 1) {
    long long nb = nblocks(n);
    tot += 2 * nb;
    n = nb;
  }
  return tot + 64;
}

void scan_exclusive(const int* in, int* out, int n, int* scratch, hipStream_t st) {
  scan_level(in, out, n, scratch, st);
  k_scan_total<<<1, 64, 0, st>>>(out, n, in);
}

}  // namespace flare
