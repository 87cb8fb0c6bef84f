// Two lanes per descriptor row: lane h = 0 owns (l, m) indices 0..7 (l = 0, 1 and the
// first four m of l = 2), lane h = 1 owns 8..15 (the last m of l = 2 and l = 3). Both
// lanes of a row sit next to each other in one wave, so per-row sums combine with one
// xor-1 exchange and no barrier. Used by the fused descriptor/quadratic-form kernel
// and by the adjoint kernel.
#pragma once

#include "pair.h"

namespace flare {

constexpr int NQ = 8;   // (l, m) indices per lane

// c[n][q] += R_n Y_{8h+q} over the neighbours of row R inside the cutoff. All rows of a
// wave share one slice, so the trip count is uniform across the wave.
__device__ __forceinline__ void accumulate_half(const SlotView& v, int Rw, int h, float (*c)[NQ]) {
  for_each_slot<4>(v, Rw, [&](const float4& g, int) {
    PairGeom pg;
    int sp;
    if (!unpack_geom(g, pg, sp)) return;
    float R[NR], Y[NLM];
    radial(pg.r, v.rc, R);
    sph_harm(pg.ux, pg.uy, pg.uz, Y);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const float y = h ? Y[NQ + q] : Y[q];
#pragma unroll
      for (int nn = 0; nn < NR; ++nn) c[nn][q] += R[nn] * y;
    }
  });
}

// One B2 radial pair (a, b) of a single-species block, split between the two lanes of
// the row: lane 0 returns the components l = 0, 1, lane 1 the components l = 2, 3 (the
// lane's half of the packed float4 at 4k). Products c_a,q c_b,q: lane 0 holds l = 0 (q0),
// l = 1 (q1..3) and part of l = 2 (q4..7); lane 1 the rest of l = 2 (q0) and l = 3
// (q1..7). One cross-lane move per pair brings lane 0's part of l = 2 to lane 1.
__device__ __forceinline__ float2 b2_half(const float* ca, const float* cb, int h) {
  const float v0 = ca[0] * cb[0];
  const float v1 = ca[1] * cb[1] + ca[2] * cb[2] + ca[3] * cb[3];
  const float v2 = ca[4] * cb[4] + ca[5] * cb[5] + ca[6] * cb[6] + ca[7] * cb[7];
  const float x = xor1(v2);            // lane 1 receives lane 0's part of l = 2
  return h ? make_float2(v0 + x, v1 + v2) : make_float2(v0, v1);
}

}  // namespace flare
