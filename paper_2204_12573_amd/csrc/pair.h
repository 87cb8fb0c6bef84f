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

// Rolling prefetch over one row's slots: the geometry of slot k+3 is loaded while slot k
// is processed. Usage:
//   SLOT_STREAM_BEGIN(v, R);            // declares ss_len and the prefetch registers
//   for (int k = 0; k < ss_len; ++k) { const float4 g = SLOT_STREAM_NEXT(k); ... }
#define SLOT_STREAM_BEGIN(v, R)                                                          \
  const int ss_base = (v).slice_base[(R) >> 5];                                          \
  const int ss_len = (v).slice_base[((R) >> 5) + 1] - ss_base;                           \
  const float4* ss_p = (v).geom + (size_t)ss_base * 32 + ((R) & 31);                     \
  float4 ss_g0 = ss_len > 0 ? ss_p[0] : make_float4(0.f, 0.f, 0.f, 0.f);                 \
  float4 ss_g1 = ss_len > 1 ? ss_p[32] : make_float4(0.f, 0.f, 0.f, 0.f);                \
  float4 ss_g2 = ss_len > 2 ? ss_p[64] : make_float4(0.f, 0.f, 0.f, 0.f)

__device__ __forceinline__ float4 slot_stream_next(int k, int len, const float4* p, float4& g0, float4& g1,
                                                   float4& g2) {
  const float4 g = g0;
  g0 = g1;
  g1 = g2;
  g2 = k + 3 < len ? p[(size_t)(k + 3) * 32] : make_float4(0.f, 0.f, 0.f, 0.f);
  return g;
}
#define SLOT_STREAM_NEXT(k) slot_stream_next((k), ss_len, ss_p, ss_g0, ss_g1, ss_g2)

__device__ __forceinline__ bool unpack_geom(const float4& g, PairGeom& pg, int& sp) {
  pg.ux = g.x;
  pg.uy = g.y;
  pg.uz = g.z;
  pg.r = fabsf(g.w);
  sp = g.w > 0.f ? 1 : 0;
  return g.w != 0.f;
}

// c[n][lm] += R_n Y_lm over row R's neighbours of species `want` (-1 = all).
__device__ __forceinline__ void accumulate_densities(const SlotView& v, int R, int want,
                                                     float (*c)[NLM]) {
  SLOT_STREAM_BEGIN(v, R);
  for (int k = 0; k < ss_len; ++k) {
    PairGeom pg;
    int sp;
    if (!unpack_geom(SLOT_STREAM_NEXT(k), pg, sp)) continue;
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
