// Mixed-environment rows (both species among the neighbours, 544 components) with 16
// lanes per row: a work-group of 256 threads owns 16 rows. Lane L = s*8 + n of a row
// accumulates the density channel c_{(s,n), lm} for all 16 (l, m) over the row's slots
// (paper, Section V.B); the channels then meet in LDS, where the B2 contraction, the
// adjoint transform u = G^ c and the pair terms read them. Densities of all 16 channels
// of a row sit at cidx(a, lm) of the row's LDS block; the Pt channels are shifted by 8
// floats so that H and Pt reads of one row fall in different banks.
#pragma once

#include "basis.h"
#include "pair.h"

namespace flare {

constexpr int MROWS = 16;                  // rows per work-group
constexpr int MTHREADS = MROWS * 16;       // threads per work-group
constexpr int MSTRIDE = 16 * NLM + 16;     // LDS floats per row (4 rows of a wave: distinct banks)

__device__ __forceinline__ int cidx(int a, int lm) { return a * NLM + (a >> 3) * 8 + lm; }

// c[lm] = sum over the row's neighbours of species (L >> 3) of R_{L & 7}(r) Y_lm(r^).
__device__ __forceinline__ void mixed_channel_density(const SlotView& v, int R, int L, float (&c)[NLM]) {
  const int s = L >> 3, n = L & 7;
  for_each_slot<4>(v, R, [&](const float4& g, int) {
    PairGeom pg;
    int sp;
    if (!unpack_geom(g, pg, sp)) return;
    if (sp != s) return;
    float Rn[NR], Y[NLM];
    radial(pg.r, v.rc, Rn);
    sph_harm(pg.ux, pg.uy, pg.uz, Y);
    float rn = Rn[0];
#pragma unroll
    for (int q = 1; q < NR; ++q) rn = n == q ? Rn[q] : rn;   // select, no dynamic register index
#pragma unroll
    for (int lm = 0; lm < NLM; ++lm) c[lm] += rn * Y[lm];
  });
}

// Channels (a, b) of packed B2 pair P of a 544-wide row: (H,H) pairs 0..35 (na <= nb,
// row-major), (H,Pt) pairs 36..99 (row-major, a = H channel), (Pt,Pt) pairs 100..135.
__device__ __forceinline__ void mixed_pair_channels(int P, int& a, int& b) {
  if (P >= NP1 && P < NP1 + NX) {
    a = (P - NP1) / NR;
    b = NR + (P - NP1) % NR;
    return;
  }
  const int off = P < NP1 ? 0 : NR;
  int q = P < NP1 ? P : P - NP1 - NX;
  int na = 0;
#pragma unroll
  for (int t = 0; t < NR; ++t) {
    const int w = NR - na;          // pairs (na, na..7)
    if (q >= w) {
      q -= w;
      ++na;
    }
  }
  a = off + na;
  b = off + na + q;
}

}  // namespace flare
