// Adjoint (force) terms of the paper's Section V.B reordering, shared by the standalone
// adjoint kernel and the fused descriptor / quadratic-form / adjoint kernel.
//
// With g_i = de_i/dd~_i and d~_{(a,b),l} = sum_m c_a c_b:
//   u_{a,l,m} = de_i/dc_{a,l,m} = sum_b G^_{ab,l} c_{b,l,m},
//               G^_{ab,l} = g_{(min,max),l}, doubled on the diagonal a = b.
// For each listed pair p = (i, j, s) inside the cutoff, with Delta = r_j + s L - r_i:
//   w_p = de_i/dDelta = sum_{n,l,m} u_{(s_j,n),l,m} grad_Delta [R_n(r) Y_lm(Delta/r)]
//       = u^ sum_n (R_n' Z_n - R_n Zl_n / r) + (1/r) sum_lm A_lm grad P_lm(u^)
//   with Z_n = sum_lm u_{n,lm} Y_lm, Zl_n = sum_lm l u_{n,lm} Y_lm, A_lm = sum_n u_{n,lm} R_n,
// and w_p = 0 outside the cutoff.
#pragma once

#include "basis.h"
#include "half.h"
#include "pair.h"

namespace flare {

// sum_lm A_lm grad P_lm(x, y, z)
__device__ __forceinline__ void poly_grad_dot(const float* A, float x, float y, float z,
                                              float& gx, float& gy, float& gz) {
  const float xx = x * x, yy = y * y, zz = z * z;
  gx = kY1 * A[3] + kY2a * (y * A[4] + z * A[7]) + kY20 * (-2.f * x) * A[6] + 2.f * kY22 * x * A[8] +
       6.f * kY33 * x * y * A[9] + kY32a * y * z * A[10] - 2.f * kY31 * x * y * A[11] -
       6.f * kY30 * x * z * A[12] + kY31 * (4.f * zz - 3.f * xx - yy) * A[13] +
       2.f * kY32b * x * z * A[14] + 3.f * kY33 * (xx - yy) * A[15];
  gy = kY1 * A[1] + kY2a * (x * A[4] + z * A[5]) + kY20 * (-2.f * y) * A[6] - 2.f * kY22 * y * A[8] +
       3.f * kY33 * (xx - yy) * A[9] + kY32a * x * z * A[10] + kY31 * (4.f * zz - xx - 3.f * yy) * A[11] -
       6.f * kY30 * y * z * A[12] - 2.f * kY31 * x * y * A[13] - 2.f * kY32b * y * z * A[14] -
       6.f * kY33 * x * y * A[15];
  gz = kY1 * A[2] + kY2a * (y * A[5] + x * A[7]) + 4.f * kY20 * z * A[6] + kY32a * x * y * A[10] +
       8.f * kY31 * y * z * A[11] + kY30 * (6.f * zz - 3.f * xx - 3.f * yy) * A[12] +
       8.f * kY31 * x * z * A[13] + kY32b * (xx - yy) * A[14];
}

// w = de_i/dDelta for one pair from the adjoint densities u[n][lm] of the neighbour's
// species (all 16 (l, m) in one thread).
// The radial sums are taken per (l, m): A_lm = sum_n u_{n,lm} R_n and B_lm = sum_n
// u_{n,lm} R_n', so that sum_n (R_n' Z_n - R_n Zl_n / r) = sum_lm Y_lm (B_lm - (l/r) A_lm).
template <class U>
__device__ __forceinline__ void pair_force(const PairGeom& pg, float rc, U u, float& wx, float& wy,
                                           float& wz) {
  float R[NR], dR[NR], Y[NLM];
  radial_d(pg.r, rc, R, dR);
  sph_harm(pg.ux, pg.uy, pg.uz, Y);
  float A[NLM], B[NLM];
#pragma unroll
  for (int lm = 0; lm < NLM; ++lm) {
    A[lm] = 0.f;
    B[lm] = 0.f;
  }
#pragma unroll
  for (int n = 0; n < NR; ++n)
#pragma unroll
    for (int lm = 0; lm < NLM; ++lm) {
      const float un = u(n, lm);
      A[lm] += un * R[n];
      B[lm] += un * dR[n];
    }
  const float inv_r = __builtin_amdgcn_rcpf(pg.r);   // 1 ulp; r >= the shortest pair distance
  const float il[LMAX + 1] = {0.f, inv_r, 2.f * inv_r, 3.f * inv_r};
  float s1 = 0.f;
#pragma unroll
  for (int lm = 0; lm < NLM; ++lm) s1 = fmaf(Y[lm], fmaf(-il[lm_l(lm)], A[lm], B[lm]), s1);
  float gx, gy, gz;
  poly_grad_dot(A, pg.ux, pg.uy, pg.uz, gx, gy, gz);
  wx = pg.ux * s1 + gx * inv_r;
  wy = pg.uy * s1 + gy * inv_r;
  wz = pg.uz * s1 + gz * inv_r;
}

__device__ __forceinline__ int pair_index_same(int na, int nb) {
  // packed index of (na <= nb) inside a single-species block, row-major
  return na * NR - na * (na - 1) / 2 + (nb - na);
}

// Two lanes per row (see half.h): c[n][q] holds the densities of (l, m) = 8h + q of the
// row's single neighbour species. In place, c becomes u = G^ c, group by group: lane h's
// q fall in three groups of constant l, {0}, {1,2,3}, {4..7}, with l = (0,1,2) for h = 0
// and (2,3,3) for h = 1. g(k) = g of packed component k = 4*(radial pair) + l, read as
// g[k * gstride].
__device__ __forceinline__ void u_transform_half(const float* g, int gstride, int h, float (&c)[NR][NQ]) {
  const int lg0 = h ? 2 : 0, lg1 = h ? 3 : 1, lg2 = h ? 3 : 2;
#pragma unroll
  for (int grp = 0; grp < 3; ++grp) {
    const int l = grp == 0 ? lg0 : (grp == 1 ? lg1 : lg2);
    const int q0 = grp == 0 ? 0 : (grp == 1 ? 1 : 4);
    const int q1 = grp == 0 ? 1 : (grp == 1 ? 4 : 8);
    float gh[NR][NR];
#pragma unroll
    for (int na = 0; na < NR; ++na)
#pragma unroll
      for (int nb = na; nb < NR; ++nb) {
        const float val = g[(size_t)(pair_index_same(na, nb) * 4 + l) * gstride];
        gh[na][nb] = na == nb ? 2.f * val : val;
        gh[nb][na] = gh[na][nb];
      }
#pragma unroll
    for (int q = q0; q < q1; ++q) {
      float col[NR];
#pragma unroll
      for (int n = 0; n < NR; ++n) col[n] = c[n][q];
#pragma unroll
      for (int n = 0; n < NR; ++n) {
        float acc = 0.f;
#pragma unroll
        for (int m = 0; m < NR; ++m) acc += gh[n][m] * col[m];
        c[n][q] = acc;
      }
    }
  }
}

// Exchange the two halves of u so that both lanes of the row hold all of it, then split
// the row's slots between the lanes (k = h, h + 2, ...): each pair term is evaluated once
// and scattered to the reverse pair's slot of w_in, where the force gather of the
// neighbour reads it; the row's own terms are summed (each lane over its slots in order,
// then the two lanes) into f_own[R].
__device__ __forceinline__ void adjoint_pairs_half(const SlotView& v, int R, int h, const float (&c)[NR][NQ],
                                                   float4* __restrict__ f_own) {
  float u[NR][NLM];
#pragma unroll
  for (int n = 0; n < NR; ++n)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const float other = xor1(c[n][q]);
      u[n][q] = h ? other : c[n][q];
      u[n][NQ + q] = h ? c[n][q] : other;
    }
  const int S = wave_slice(R);
  const int base = v.slice_base[S];
  const int len = v.slice_base[S + 1] - base;
  const size_t s0 = (size_t)base * 32 + (R & 31);
  float sx = 0.f, sy = 0.f, sz = 0.f;
  // lane h takes slots k = h, h + 2, ...: the geometry and reverse index of its next two
  // slots are in flight while two are evaluated, in two register groups that take turns
  // (as in for_each_slot: unconditional loads, past the slice re-reading its last slot)
  auto load = [&](int k, float4& g, int& r) {
    const size_t sl = s0 + (size_t)min(k, len - 1) * 32;
    g = v.geom[sl];
    r = v.rev[sl];
  };
  auto term = [&](int k, const float4& gk, int rk) {
    if (k >= len) return;
    PairGeom pg;
    int sp;
    float wx = 0.f, wy = 0.f, wz = 0.f;
    if (unpack_geom(gk, pg, sp)) pair_force(pg, v.rc, [&](int n, int lm) { return u[n][lm]; }, wx, wy, wz);
    v.w_in[rk] = make_float4(wx, wy, wz, 0.f);
    sx += wx;
    sy += wy;
    sz += wz;
  };
  if (len > 0) {
    float4 ga[2], gb[2];
    int ra[2], rb[2];
    load(h, ga[0], ra[0]);
    load(h + 2, ga[1], ra[1]);
    for (int k0 = h; k0 < len; k0 += 8) {
      load(k0 + 4, gb[0], rb[0]);
      load(k0 + 6, gb[1], rb[1]);
      term(k0, ga[0], ra[0]);
      term(k0 + 2, ga[1], ra[1]);
      load(k0 + 8, ga[0], ra[0]);
      load(k0 + 10, ga[1], ra[1]);
      term(k0 + 4, gb[0], rb[0]);
      term(k0 + 6, gb[1], rb[1]);
    }
  }
  sx += xor1(sx);
  sy += xor1(sy);
  sz += xor1(sz);
  if (h == 0) f_own[R] = make_float4(sx, sy, sz, 0.f);
}

}  // namespace flare
