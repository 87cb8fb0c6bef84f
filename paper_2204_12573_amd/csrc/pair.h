// Pair data shared by the descriptor and adjoint kernels: the per-step geometry of every
// slot of the sliced layout, and the density accumulation of one row over its slots.
#pragma once

#include "basis.h"
#include "state.h"

namespace flare {

struct PairGeom {
  float r, ux, uy, uz;
};

// geometry of slot k of row R; false for padding or a pair outside the cutoff.
// sp receives the neighbour species (0 H, 1 Pt).
__device__ __forceinline__ bool slot_geom(const SlotView& v, int R, int k, PairGeom& pg, int& sp) {
  const float4 g = v.geom[slot_of(v.slice_base, R, k)];
  pg.ux = g.x;
  pg.uy = g.y;
  pg.uz = g.z;
  pg.r = fabsf(g.w);
  sp = g.w > 0.f ? 1 : 0;
  return g.w != 0.f;
}

__device__ __forceinline__ int slice_len(const SlotView& v, int R) {
  return v.slice_base[(R >> 5) + 1] - v.slice_base[R >> 5];
}

// c[n][lm] += R_n Y_lm over row R's neighbours of species `want` (-1 = all).
__device__ __forceinline__ void accumulate_densities(const SlotView& v, int R, int want,
                                                     float (*c)[NLM]) {
  const int len = slice_len(v, R);
  for (int k = 0; k < len; ++k) {
    PairGeom pg;
    int sp;
    if (!slot_geom(v, R, k, pg, sp)) continue;
    if (want >= 0 && sp != want) continue;
    float Rn[NR], Y[NLM];
    radial(pg.r, v.rc, Rn);
    sph_harm(pg.ux, pg.uy, pg.uz, Y);
#pragma unroll
    for (int nn = 0; nn < NR; ++nn)
#pragma unroll
      for (int lm = 0; lm < NLM; ++lm) c[nn][lm] += Rn[nn] * Y[lm];
  }
}

}  // namespace flare
