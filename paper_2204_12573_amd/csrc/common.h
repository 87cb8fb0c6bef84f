// Internal declarations shared by the HIP kernels of the B2 force-field evaluator.
// Model sizes are compile-time: 2 species, 8 radial functions, l <= 3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace flare {

constexpr int NS = 2;            // species (H = 0, Pt = 1)
constexpr int NR = 8;            // radial functions n = 0..7
constexpr int LMAX = 3;
constexpr int NLM = 16;          // (l, m) pairs, flat index l*l + l + m
constexpr int NCH = NS * NR;     // radial channels a = s*NR + n
constexpr int NP1 = NR * (NR + 1) / 2;   // radial pairs inside a single-species block (36)
constexpr int NX = NR * NR;              // radial pairs of the cross block (64)
constexpr int ND1 = NP1 * (LMAX + 1);    // 144: single-species block
constexpr int NDX = NX * (LMAX + 1);     // 256: cross block
constexpr int ND = 2 * ND1 + NDX;        // 544
constexpr int NBUCKET = 6;
constexpr int TILE_ROWS = 128;           // row padding of every bucket (GEMM tile height)
constexpr int MIX_ROWS = 16384;          // mixed (544-wide) rows processed together, a multiple of TILE_ROWS

// Environment class = OR of (1 << species) over listed neighbours: 1 H-only, 2 Pt-only,
// 3 mixed, 0 none. Buckets: (H, H-only) (Pt, H-only) (H, Pt-only) (Pt, Pt-only)
// (H, mixed) (Pt, mixed).
__host__ __device__ inline int bucket_of(int species, int mask) {
  if (mask == 0) return -1;
  if (mask == 3) return 4 + species;
  return (mask - 1) * 2 + species;
}
__host__ __device__ inline int bucket_width(int b) { return b < 4 ? ND1 : ND; }
// env species of a single-species bucket (0 for buckets 0,1; 1 for buckets 2,3)
__host__ __device__ inline int bucket_env(int b) { return b >> 1; }

// image shift packed as three signed bytes
__host__ __device__ inline int32_t pack_shift(int sx, int sy, int sz) {
  return (int32_t)((uint32_t)(sx & 0xff) | ((uint32_t)(sy & 0xff) << 8) | ((uint32_t)(sz & 0xff) << 16));
}
__host__ __device__ inline void unpack_shift(int32_t v, int& sx, int& sy, int& sz) {
  sx = (int)(int8_t)(v & 0xff);
  sy = (int)(int8_t)((v >> 8) & 0xff);
  sz = (int)(int8_t)((v >> 16) & 0xff);
}

// Per-cell bin grid for the cell list.
struct CellGrid {
  double L[3];       // box sides
  double inv_h[3];   // bins per Angstrom
  int nb[3];         // bins per axis
  int K[3];          // stencil half-width per axis
  int bin_base;      // first global bin id of this cell
  int atom_base;     // first atom (caller order == internal order range)
};

// Spread consecutive work-groups over the 8 XCDs in contiguous chunks: the hardware
// deals work-groups round-robin to XCDs, so work-group g runs on XCD g % 8; this maps
// it to a logical index so that each XCD walks one contiguous range (its own L2 then
// holds that range's neighbours).
__device__ inline int xcd_remap(int g, int n) {
  const int nx = 8;
  int per = n / nx, rem = n % nx;
  int x = g % nx, k = g / nx;
  int start = x * per + (x < rem ? x : rem);
  return start + k;
}

// ---- cross-lane moves on the DPP network (no LDS round trip) ----
// xor-1 / xor-2 exchanges inside quads, then mirrors inside half rows and rows: after
// sum16 every lane of a 16-lane row holds the row's total.
__device__ __forceinline__ float dpp_f(float v, int ctrl_sel) {
  int x = __float_as_int(v);
  switch (ctrl_sel) {
    case 0: x = __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, true); break;   // quad_perm 1,0,3,2
    case 1: x = __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, true); break;   // quad_perm 2,3,0,1
    case 2: x = __builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, true); break;  // row_half_mirror
    default: x = __builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, true); break; // row_mirror
  }
  return __int_as_float(x);
}
__device__ __forceinline__ float xor1(float v) { return dpp_f(v, 0); }
__device__ __forceinline__ float sum16(float v) {
  v += dpp_f(v, 0);
  v += dpp_f(v, 1);
  v += dpp_f(v, 2);
  v += dpp_f(v, 3);
  return v;
}
__device__ __forceinline__ double xor1d(double v) {
  const long long b = __double_as_longlong(v);
  int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
  lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, true);
  hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double dpp_d(double v, int sel) {
  const long long b = __double_as_longlong(v);
  const int lo = __float_as_int(dpp_f(__int_as_float((int)(b & 0xffffffffLL)), sel));
  const int hi = __float_as_int(dpp_f(__int_as_float((int)(b >> 32)), sel));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double sum16d(double v) {
  v += dpp_d(v, 0);
  v += dpp_d(v, 1);
  v += dpp_d(v, 2);
  v += dpp_d(v, 3);
  return v;
}

// ---- device-wide exclusive scan (scan.hip) ----
size_t scan_scratch_ints(long long n);
// out[0..n] = exclusive prefix of in[0..n-1], out[n] = total. in and out may alias only
// if distinct buffers are not required (they may not alias).
void scan_exclusive(const int* in, int* out, int n, int* scratch, hipStream_t st);

}  // namespace flare
