// Forces by the reordered (adjoint) sum of the paper's Section V.B: the descriptor
// gradient is never formed.
//
// With g_i = de_i/dd~_i from the quadratic-form pass and d~_{(a,b),l} = sum_m c_a c_b:
//   u_{a,l,m} = de_i/dc_{a,l,m} = sum_b G^_{ab,l} c_{b,l,m},
//               G^_{ab,l} = g_{(min,max),l}, doubled on the diagonal a = b.
// For each listed pair (i, j) inside the cutoff, with Delta = r_j - r_i (+ image):
//   w_ij = de_i/dDelta = sum_{n,l,m} u_{(s_j,n),l,m} grad_Delta [R_n(r) Y_lm(Delta/r)]
//        = u^ sum_n (R_n' Z_n - R_n Zl_n / r) + (1/r) sum_lm A_lm grad P_lm(u^)
//   with Z_n = sum_lm u_{n,lm} Y_lm, Zl_n = sum_lm l u_{n,lm} Y_lm, A_lm = sum_n u_{n,lm} R_n.
//   F_i += w_ij and F_j -= w_ij (device atomics).
// The densities c are recomputed from the pair list instead of being stored.
#include "basis.h"
#include "pair.h"
#include "state.h"

namespace flare {
namespace {

constexpr int NT = 128;
constexpr int NTX = 64;

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
// species.
template <class U>
__device__ __forceinline__ void pair_force(const PairGeom& pg, float rc, U u, float& wx, float& wy,
                                           float& wz) {
  float R[NR], dR[NR], Y[NLM];
  radial_d(pg.r, rc, R, dR);
  sph_harm(pg.ux, pg.uy, pg.uz, Y);
  float A[NLM];
#pragma unroll
  for (int lm = 0; lm < NLM; ++lm) A[lm] = 0.f;
  float s1 = 0.f;
  const float inv_r = 1.f / pg.r;
#pragma unroll
  for (int n = 0; n < NR; ++n) {
    float S[LMAX + 1] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int lm = 0; lm < NLM; ++lm) {
      const float un = u(n, lm);
      S[lm_l(lm)] += un * Y[lm];
      A[lm] += un * R[n];
    }
    const float z = S[0] + S[1] + S[2] + S[3];
    const float zl = S[1] + 2.f * S[2] + 3.f * S[3];
    s1 += dR[n] * z - R[n] * zl * inv_r;
  }
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

__global__ __launch_bounds__(NT) void k_force_single(PairView v, int rows,
                                                     const int* __restrict__ atom_of_row,
                                                     const float* __restrict__ G,
                                                     float* __restrict__ F) {
  const int row = xcd_remap(blockIdx.x, gridDim.x) * NT + threadIdx.x;
  if (row >= rows) return;
  const int i = atom_of_row[row];
  if (i < 0) return;
  float c[NR][NLM];
#pragma unroll
  for (int n = 0; n < NR; ++n)
#pragma unroll
    for (int lm = 0; lm < NLM; ++lm) c[n][lm] = 0.f;
  accumulate_densities(v, i, -1, c);
  // u = G^ c, in place, one (l, m) column at a time
  const float* g = G + (size_t)row * ND1;
#pragma unroll
  for (int l = 0; l <= LMAX; ++l) {
    float gh[NR][NR];
#pragma unroll
    for (int na = 0; na < NR; ++na)
#pragma unroll
      for (int nb = na; nb < NR; ++nb) {
        const float val = g[pair_index_same(na, nb) * 4 + l];
        gh[na][nb] = na == nb ? 2.f * val : val;
        gh[nb][na] = gh[na][nb];
      }
#pragma unroll
    for (int lm = l * l; lm < (l + 1) * (l + 1); ++lm) {
      float col[NR];
#pragma unroll
      for (int n = 0; n < NR; ++n) col[n] = c[n][lm];
#pragma unroll
      for (int n = 0; n < NR; ++n) {
        float acc = 0.f;
#pragma unroll
        for (int m = 0; m < NR; ++m) acc += gh[n][m] * col[m];
        c[n][lm] = acc;
      }
    }
  }
  // pair loop
  const size_t nn = (size_t)v.n;
  const double xi = v.pos[i], yi = v.pos[nn + i], zi = v.pos[2 * nn + i];
  const CellGrid* cg = v.grids + v.sid[i];
  const double L[3] = {cg->L[0], cg->L[1], cg->L[2]};
  float fx = 0.f, fy = 0.f, fz = 0.f;
  const int p0 = v.nl_off[i], p1 = v.nl_off[i + 1];
  for (int p = p0; p < p1; ++p) {
    const int j = v.nl_j[p];
    PairGeom pg;
    if (!pair_geom(v, j, xi, yi, zi, L, v.nl_s[p], pg)) continue;
    float wx, wy, wz;
    pair_force(pg, v.rc, [&](int n, int lm) { return c[n][lm]; }, wx, wy, wz);
    fx += wx;
    fy += wy;
    fz += wz;
    unsafeAtomicAdd(&F[j], -wx);
    unsafeAtomicAdd(&F[nn + j], -wy);
    unsafeAtomicAdd(&F[2 * nn + j], -wz);
  }
  unsafeAtomicAdd(&F[i], fx);
  unsafeAtomicAdd(&F[nn + i], fy);
  unsafeAtomicAdd(&F[2 * nn + i], fz);
}

__global__ __launch_bounds__(NTX) void k_force_mixed(PairView v, int rows,
                                                     const int* __restrict__ atom_of_row,
                                                     const float* __restrict__ G,
                                                     float* __restrict__ F) {
  // densities, then adjoints, of both species halves; one column per thread
  __shared__ float uh[NR * NLM][NTX];
  __shared__ float up[NR * NLM][NTX];
  const int t = threadIdx.x;
  const int row = blockIdx.x * NTX + t;
  if (row >= rows) return;
  const int i = atom_of_row[row];
  if (i < 0) return;
  for (int half = 0; half < 2; ++half) {
    float c[NR][NLM];
#pragma unroll
    for (int n = 0; n < NR; ++n)
#pragma unroll
      for (int lm = 0; lm < NLM; ++lm) c[n][lm] = 0.f;
    accumulate_densities(v, i, half, c);
    float (*dst)[NTX] = half ? up : uh;
#pragma unroll
    for (int n = 0; n < NR; ++n)
#pragma unroll
      for (int lm = 0; lm < NLM; ++lm) dst[n * NLM + lm][t] = c[n][lm];
  }
  const float* g = G + (size_t)row * ND;
  const float* gHH = g;
  const float* gHP = g + ND1;
  const float* gPP = g + ND1 + NDX;
  for (int lm = 0; lm < NLM; ++lm) {
    const int l = lm_l(lm);
    float ch[NR], cp[NR], oh[NR], op[NR];
#pragma unroll
    for (int n = 0; n < NR; ++n) {
      ch[n] = uh[n * NLM + lm][t];
      cp[n] = up[n * NLM + lm][t];
    }
#pragma unroll
    for (int a = 0; a < NR; ++a) {
      float acc_h = 0.f, acc_p = 0.f;
#pragma unroll
      for (int b = 0; b < NR; ++b) {
        const int ia = a < b ? a : b, ib = a < b ? b : a;
        const float w2 = a == b ? 2.f : 1.f;
        acc_h += w2 * gHH[pair_index_same(ia, ib) * 4 + l] * ch[b] + gHP[(a * NR + b) * 4 + l] * cp[b];
        acc_p += w2 * gPP[pair_index_same(ia, ib) * 4 + l] * cp[b] + gHP[(b * NR + a) * 4 + l] * ch[b];
      }
      oh[a] = acc_h;
      op[a] = acc_p;
    }
#pragma unroll
    for (int n = 0; n < NR; ++n) {
      uh[n * NLM + lm][t] = oh[n];
      up[n * NLM + lm][t] = op[n];
    }
  }
  const size_t nn = (size_t)v.n;
  const double xi = v.pos[i], yi = v.pos[nn + i], zi = v.pos[2 * nn + i];
  const CellGrid* cg = v.grids + v.sid[i];
  const double L[3] = {cg->L[0], cg->L[1], cg->L[2]};
  float fx = 0.f, fy = 0.f, fz = 0.f;
  const int p0 = v.nl_off[i], p1 = v.nl_off[i + 1];
  for (int p = p0; p < p1; ++p) {
    const int j = v.nl_j[p];
    PairGeom pg;
    if (!pair_geom(v, j, xi, yi, zi, L, v.nl_s[p], pg)) continue;
    float (*u)[NTX] = v.sp[j] == 0 ? uh : up;
    float wx, wy, wz;
    pair_force(pg, v.rc, [&](int n, int lm) { return u[n * NLM + lm][t]; }, wx, wy, wz);
    fx += wx;
    fy += wy;
    fz += wz;
    unsafeAtomicAdd(&F[j], -wx);
    unsafeAtomicAdd(&F[nn + j], -wy);
    unsafeAtomicAdd(&F[2 * nn + j], -wz);
  }
  unsafeAtomicAdd(&F[i], fx);
  unsafeAtomicAdd(&F[nn + i], fy);
  unsafeAtomicAdd(&F[2 * nn + i], fz);
}

}  // namespace

void compute_forces(flare_state* s) {
  const PairView v = pair_view(s);
  StageTimer tm(s, FLARE_T_FORCE1);
  (void)hipMemsetAsync(s->f_int, 0, 3 * (size_t)s->n_atoms * sizeof(float), s->stream);
  if (s->rows1 > 0)
    k_force_single<<<(s->rows1 + NT - 1) / NT, NT, 0, s->stream>>>(v, s->rows1, s->atom_of_row1.p, s->G1.p,
                                                                   s->f_int);
  StageTimer tm2(s, FLARE_T_FORCEX);
  if (s->rowsx > 0)
    k_force_mixed<<<(s->rowsx + NTX - 1) / NTX, NTX, 0, s->stream>>>(v, s->rowsx, s->atom_of_rowx.p,
                                                                     s->Gx.p, s->f_int);
}

}  // namespace flare
