// Forces by the reordered (adjoint) sum of the paper's Section V.B: the descriptor
// gradient is never formed (the per-pair terms are in adjoint.h). The densities c are
// recomputed from the pair list. Forces follow without atomics:
// F_i = sum_{p in list(i)} (w_p - w_rev(p)), rev(p) being the pair (j, i, -s)
// (reduce.hip), so they are deterministic and independent of how cells are batched.
#include "adjoint.h"
#include "state.h"

namespace flare {
namespace {

constexpr int NTX = 64;
constexpr int TA = 256;   // threads of the 144-row adjoint kernel (128 rows, 2 lanes each)

// One row per lane pair (see half.h and adjoint.h), reading g from the tile-transposed
// G[tile][k][128] written by the quadratic-form kernel.
__global__ __launch_bounds__(TA) void k_adjoint144(SlotView v, const int* __restrict__ atom_of_row,
                                                   const float* __restrict__ G, float4* __restrict__ w) {
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int t = threadIdx.x, rl = t >> 1, h = t & 1;
  const int i = atom_of_row[tile * 128 + rl];
  if (i < 0) return;
  float c[NR][NQ];
#pragma unroll
  for (int n = 0; n < NR; ++n)
#pragma unroll
    for (int q = 0; q < NQ; ++q) c[n][q] = 0.f;
  const int R = tile * 128 + rl;
  accumulate_half(v, R, h, c);
  u_transform_half(G + (size_t)tile * ND1 * 128 + rl, 128, h, c);
  adjoint_pairs_half(v, R, h, c, w);
}

__global__ __launch_bounds__(NTX) void k_adjoint_mixed(SlotView v, int rows1, int rows,
                                                       const int* __restrict__ atom_of_row,
                                                       const float* __restrict__ G,
                                                       float4* __restrict__ w) {
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
    accumulate_densities(v, rows1 + row, half, c);
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
  const int R = rows1 + row;
  SLOT_STREAM_BEGIN(v, R);
  for (int k = 0; k < ss_len; ++k) {
    PairGeom pg;
    int sp;
    float wx = 0.f, wy = 0.f, wz = 0.f;
    if (unpack_geom(SLOT_STREAM_NEXT(k), pg, sp)) {
      float (*u)[NTX] = sp == 0 ? uh : up;
      pair_force(pg, v.rc, [&](int n, int lm) { return u[n * NLM + lm][t]; }, wx, wy, wz);
    }
    w[slot_of(v.slice_base, R, k)] = make_float4(wx, wy, wz, 0.f);
  }
}

}  // namespace

void compute_forces(flare_state* s, bool rows144) {
  const SlotView v = slot_view(s);
  if (rows144) {
    StageTimer tm(s, FLARE_T_FORCE1);
    if (s->rows1 > 0)
      k_adjoint144<<<s->rows1 / 128, TA, 0, s->stream>>>(v, s->atom_of_row1.p, s->G1.p, s->w_slot.p);
  }
  {
    StageTimer tm(s, FLARE_T_FORCEX);
    if (s->rowsx > 0)
      k_adjoint_mixed<<<(s->rowsx + NTX - 1) / NTX, NTX, 0, s->stream>>>(v, s->rows1, s->rowsx,
                                                                          s->atom_of_rowx.p, s->Gx.p, s->w_slot.p);
  }
}

}  // namespace flare
