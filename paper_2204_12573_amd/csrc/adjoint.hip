// Forces by the reordered (adjoint) sum of the paper's Section V.B: the descriptor
// gradient is never formed (the per-pair terms are in adjoint.h). The densities c are
// recomputed from the pair list. Forces follow without atomics:
// F_i = sum_{p in list(i)} (w_p - w_rev(p)), rev(p) being the pair (j, i, -s): every w_p
// is also stored at the slot of rev(p) in w_in, and the gather (reduce.hip) reads both
// arrays at the row's own slots, in slot order, so forces are deterministic and
// independent of how cells are batched.
#include "adjoint.h"
#include "mixed.h"
#include "state.h"

namespace flare {
namespace {

constexpr int TA = 256;   // threads of the 144-row adjoint kernel (128 rows, 2 lanes each)

// One row per lane pair (see half.h and adjoint.h), reading g from the tile-transposed
// G[tile][k][128] written by the quadratic-form kernel.
__global__ __launch_bounds__(TA) void k_adjoint144(SlotView v, const int* __restrict__ atom_of_row,
                                                   const float* __restrict__ G, float4* __restrict__ f_own) {
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
  adjoint_pairs_half(v, R, h, c, f_own);
}

// Mixed rows, 16 lanes per row (mixed.h): lane a = s*8 + n forms its density channel,
// then its adjoint channel u_{a,lm} = sum_b G^_{ab,l} c_{b,lm} over the 16 channels of
// the row (G^ from the row's 544 gradient components: (H,H) and (Pt,Pt) blocks doubled on
// the diagonal, the (H,Pt) block shared by both orders), and the row's slots are split
// over the lanes (k = L, L + 16, ...), each pair reading u of its neighbour species from LDS.
// Rows [r0, r0 + gridDim.x * MROWS) of the mixed class; G holds the chunk's gradients
// (row r - r0).
__global__ __launch_bounds__(MTHREADS) void k_adjoint_mixed(SlotView v, int rows1, int r0,
                                                            const int* __restrict__ atom_of_row,
                                                            const float* __restrict__ G, float4* __restrict__ f_own) {
  __shared__ __attribute__((aligned(16))) float cs[MROWS * MSTRIDE];
  const int rl = threadIdx.x >> 4, L = threadIdx.x & 15;
  const int local = blockIdx.x * MROWS + rl;
  const int row = r0 + local;
  const int R = rows1 + row;
  const int i = atom_of_row[row];
  float c[NLM];
#pragma unroll
  for (int lm = 0; lm < NLM; ++lm) c[lm] = 0.f;
  if (i >= 0) mixed_channel_density(v, R, L, c);
  float* crow = cs + rl * MSTRIDE;
#pragma unroll
  for (int lm = 0; lm < NLM; ++lm) crow[cidx(L, lm)] = c[lm];
  __syncthreads();
  float u[NLM];
#pragma unroll
  for (int lm = 0; lm < NLM; ++lm) u[lm] = 0.f;
  if (i >= 0) {
    const float* g = G + (size_t)local * ND;
    const int sa = L >> 3, na = L & 7;
#pragma unroll 2
    for (int b = 0; b < 2 * NR; ++b) {
      const int sb = b >> 3, nb = b & 7;
      int base;
      float f = 1.f;
      if (sa == sb) {
        const int lo = na < nb ? na : nb, hi = na < nb ? nb : na;
        base = (sa ? ND1 + NDX : 0) + pair_index_same(lo, hi) * 4;
        f = na == nb ? 2.f : 1.f;
      } else {
        base = ND1 + (sa == 0 ? na * NR + nb : nb * NR + na) * 4;
      }
      const float4 gl = *reinterpret_cast<const float4*>(g + base);
      const float g0 = f * gl.x, g1 = f * gl.y, g2 = f * gl.z, g3 = f * gl.w;
      const float* cb = crow + cidx(b, 0);
      u[0] += g0 * cb[0];
#pragma unroll
      for (int lm = 1; lm < 4; ++lm) u[lm] += g1 * cb[lm];
#pragma unroll
      for (int lm = 4; lm < 9; ++lm) u[lm] += g2 * cb[lm];
#pragma unroll
      for (int lm = 9; lm < 16; ++lm) u[lm] += g3 * cb[lm];
    }
  }
  __syncthreads();   // all channels read: the block now takes u
#pragma unroll
  for (int lm = 0; lm < NLM; ++lm) crow[cidx(L, lm)] = u[lm];
  __syncthreads();
  if (i < 0) return;
  const int S = wave_slice(R);
  const int base = v.slice_base[S];
  const int len = v.slice_base[S + 1] - base;
  float sx = 0.f, sy = 0.f, sz = 0.f;
  for (int k = L; k < len; k += 16) {
    const size_t slot = (size_t)(base + k) * 32 + (R & 31);
    PairGeom pg;
    int sp;
    float wx = 0.f, wy = 0.f, wz = 0.f;
    if (unpack_geom(v.geom[slot], pg, sp))
      pair_force(pg, v.rc, [&](int n, int lm) { return crow[cidx(sp * NR + n, lm)]; }, wx, wy, wz);
    v.w_in[v.rev[slot]] = make_float4(wx, wy, wz, 0.f);
    sx += wx;
    sy += wy;
    sz += wz;
  }
  // the row's own terms: each lane's slots in order, then the 16 lanes
  sx = sum16(sx);
  sy = sum16(sy);
  sz = sum16(sz);
  if (L == 0) f_own[R] = make_float4(sx, sy, sz, 0.f);
}

}  // namespace

void adjoint_rows144(flare_state* s) {
  const SlotView v = slot_view(s);
  StageTimer tm(s, FLARE_T_FORCE1);
  if (s->rows1 > 0) k_adjoint144<<<s->rows1 / 128, TA, 0, s->stream>>>(v, s->atom_of_row1, s->G1, s->f_own);
}

void adjoint_mixed_chunk(flare_state* s, int r0, int nr) {
  const SlotView v = slot_view(s);
  StageTimer tm(s, FLARE_T_FORCEX);
  if (nr > 0)
    k_adjoint_mixed<<<nr / MROWS, MTHREADS, 0, s->stream>>>(v, s->rows1, r0, s->atom_of_rowx, s->Gx, s->f_own);
}

}  // namespace flare
