// Pair data shared by the descriptor and adjoint kernels: the per-step geometry of every
// slot of the sliced layout and a prefetching walk over one row's slots.
#pragma once

#include "basis.h"
#include "state.h"

namespace flare {

struct PairGeom {
  float r, ux, uy, uz;
};

// Visit the geometry of row R's slots in order, f(g, k), with the loads PD slots ahead of
// their use: the loop body is unrolled PD times over a ring of PD registers, so no value
// moves between registers. All rows of a wave share one slice (and its length), so the
// trip count is uniform across the wave.
template <int PD, class F>
__device__ __forceinline__ void for_each_slot(const SlotView& v, int R, F f) {
  const int base = v.slice_base[R >> 5];
  const int len = v.slice_base[(R >> 5) + 1] - base;
  const float4* p = v.geom + (size_t)base * 32 + (R & 31);
  const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
  float4 buf[PD];
#pragma unroll
  for (int u = 0; u < PD; ++u) buf[u] = u < len ? p[(size_t)u * 32] : zero;
  for (int k0 = 0; k0 < len; k0 += PD) {
#pragma unroll
    for (int u = 0; u < PD; ++u) {
      const float4 g = buf[u];
      const int kn = k0 + PD + u;
      buf[u] = kn < len ? p[(size_t)kn * 32] : zero;
      if (k0 + u < len) f(g, k0 + u);
    }
  }
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
