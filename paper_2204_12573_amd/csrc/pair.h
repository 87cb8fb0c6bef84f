// Pair data shared by the descriptor and adjoint kernels: the per-step geometry of every
// slot of the sliced layout and a prefetching walk over one row's slots.
#pragma once

#include "basis.h"
#include "state.h"

namespace flare {

struct PairGeom {
  float r, ux, uy, uz;
};

// The slice of row R, read as a wave-uniform (scalar) value: every caller's wave covers
// rows of one 32-row slice, so all its active lanes have the same R / 32.
__device__ __forceinline__ int wave_slice(int R) { return __builtin_amdgcn_readfirstlane(R >> 5); }

// Visit the geometry of row R's slots in order, f(g, k), with the loads PD slots ahead of
// their use, in two register groups that take turns (group b loads while group a is used,
// then a while b is): every value is used from the register it was loaded into, and each
// wait covers only the older group. Loads are unconditional: past the slice they re-read
// its last slot (unused), so that no test or register move sits between a load and its
// use. All rows of a wave share one slice (and its length): a scalar loop.
template <int PD, class F>
__device__ __forceinline__ void for_each_slot(const SlotView& v, int R, F f) {
  const int S = wave_slice(R);
  const int base = v.slice_base[S];
  const int len = v.slice_base[S + 1] - base;
  if (len <= 0) return;
  const float4* p = v.geom + (size_t)base * 32 + (R & 31);
  float4 a[PD], b[PD];
#pragma unroll
  for (int u = 0; u < PD; ++u) a[u] = p[(size_t)min(u, len - 1) * 32];
  for (int k0 = 0; k0 < len; k0 += 2 * PD) {
#pragma unroll
    for (int u = 0; u < PD; ++u) b[u] = p[(size_t)min(k0 + PD + u, len - 1) * 32];
#pragma unroll
    for (int u = 0; u < PD; ++u)
      if (k0 + u < len) f(a[u], k0 + u);
#pragma unroll
    for (int u = 0; u < PD; ++u) a[u] = p[(size_t)min(k0 + 2 * PD + u, len - 1) * 32];
#pragma unroll
    for (int u = 0; u < PD; ++u)
      if (k0 + PD + u < len) f(b[u], k0 + PD + u);
  }
}

// Geometry of one listed pair at the current positions: Delta = d0 + (delta_j - delta_i) in
// FP32 (d0 fixed at the list build, delta the displacements since), kept when |Delta|^2 <
// r_c^2, returned as (u^, r) with the sign of r carrying the neighbour species; zero outside
// the cutoff and for padding (d0 = 0).
__device__ __forceinline__ float4 slot_geom(const float4& d0, const float4& dj, const float4& di, float rc2) {
  const float fx = d0.x + (dj.x - di.x), fy = d0.y + (dj.y - di.y), fz = d0.z + (dj.z - di.z);
  const float r2 = fmaf(fz, fz, fmaf(fy, fy, fx * fx));
  if (d0.w == 0.f || !(r2 < rc2)) return make_float4(0.f, 0.f, 0.f, 0.f);
  const float r = sqrtf(r2);
  const float inv = 1.f / r;
  return make_float4(fx * inv, fy * inv, fz * inv, d0.w * r);
}

__device__ __forceinline__ bool unpack_geom(const float4& g, PairGeom& pg, int& sp) {
  pg.ux = g.x;
  pg.uy = g.y;
  pg.uz = g.z;
  pg.r = fabsf(g.w);
  sp = g.w > 0.f ? 1 : 0;
  return g.w != 0.f;
}

}  // namespace flare
