// Pair geometry and density accumulation shared by the descriptor and adjoint kernels.
#pragma once

#include "basis.h"
#include "state.h"

namespace flare {

struct PairGeom {
  float r, ux, uy, uz;
};

// Delta = (x_j - x_i) + s*L in FP64, kept when |Delta|^2 < r_c^2, then rounded to FP32.
__device__ __forceinline__ bool pair_geom(const PairView& v, int j, double xi, double yi,
                                          double zi, const double* L, int32_t packed,
                                          PairGeom& pg) {
  int sx, sy, sz;
  unpack_shift(packed, sx, sy, sz);
  const size_t n = (size_t)v.n;
  const double dx = (v.pos[j] - xi) + (double)sx * L[0];
  const double dy = (v.pos[n + j] - yi) + (double)sy * L[1];
  const double dz = (v.pos[2 * n + j] - zi) + (double)sz * L[2];
  const double r2 = dx * dx + dy * dy + dz * dz;
  if (!(r2 < v.rc2)) return false;
  const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
  const float r = sqrtf(fx * fx + fy * fy + fz * fz);
  const float inv = 1.f / r;
  pg.r = r;
  pg.ux = fx * inv;
  pg.uy = fy * inv;
  pg.uz = fz * inv;
  return true;
}

// c[n][lm] += R_n Y_lm over the neighbours of atom i (species `want` only; -1 = all).
__device__ __forceinline__ void accumulate_densities(const PairView& v, int i, int want,
                                                     float (*c)[NLM]) {
  const size_t n = (size_t)v.n;
  const double xi = v.pos[i], yi = v.pos[n + i], zi = v.pos[2 * n + i];
  const CellGrid* g = v.grids + v.sid[i];
  const double L[3] = {g->L[0], g->L[1], g->L[2]};
  const int p0 = v.nl_off[i], p1 = v.nl_off[i + 1];
  for (int p = p0; p < p1; ++p) {
    const int j = v.nl_j[p];
    if (want >= 0 && v.sp[j] != want) continue;
    PairGeom pg;
    if (!pair_geom(v, j, xi, yi, zi, L, v.nl_s[p], pg)) continue;
    float R[NR], Y[NLM];
    radial(pg.r, v.rc, R);
    sph_harm(pg.ux, pg.uy, pg.uz, Y);
#pragma unroll
    for (int nn = 0; nn < NR; ++nn)
#pragma unroll
      for (int lm = 0; lm < NLM; ++lm) c[nn][lm] += R[nn] * Y[lm];
  }
}

}  // namespace flare
