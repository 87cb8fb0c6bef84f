// Per-atom densities, B2 contraction over m and normalisation (paper, Section V.B).
//
//   c_{(s,n),l,m} = sum_{j in rho_i, s_j = s, r_ij < r_c} R_n(r_ij) Y_lm(r^_ij)
//   d~_{(a,b),l}  = sum_m c_{a,l,m} c_{b,l,m}    (a <= b, packed)
//   d             = d~ / |d~|
//
// This file holds the mixed-environment rows (544 components, 16 lanes per row, see
// mixed.h). Single-species rows are formed inside the fused quadratic-form kernel
// (fused.hip).
// Pair geometry: positions are FP64; Delta = (x_j - x_i) + s*L is formed in FP64 and
// rounded to FP32 before the basis is evaluated.
#include "mixed.h"
#include "state.h"

namespace flare {
namespace {


// One mixed row per 16 lanes (mixed.h): channel densities into LDS, then the 136 B2
// channel pairs spread over the row's lanes (pair P = L + 16q), the norm summed in FP64
// across the lanes, and the normalised row written as float4 per pair: into the chunk's
// workspace D (row - r0) and, when exporting, into d_out at the atom's caller index.
__global__ __launch_bounds__(MTHREADS) void k_desc_mixed(SlotView v, int rows1, int r0,
                                                         const int* __restrict__ atom_of_row,
                                                         const int* __restrict__ perm, float* __restrict__ D,
                                                         float* __restrict__ nrm_out, float* __restrict__ d_out) {
  __shared__ __attribute__((aligned(16))) float cs[MROWS * MSTRIDE];
  const int rl = threadIdx.x >> 4, L = threadIdx.x & 15;
  const int local = blockIdx.x * MROWS + rl;
  const int row = r0 + local;
  const int i = atom_of_row[row];
  float c[NLM];
#pragma unroll
  for (int lm = 0; lm < NLM; ++lm) c[lm] = 0.f;
  if (i >= 0) mixed_channel_density(v, rows1 + row, L, c);
  float* crow = cs + rl * MSTRIDE;
#pragma unroll
  for (int lm = 0; lm < NLM; ++lm) crow[cidx(L, lm)] = c[lm];
  __syncthreads();
  constexpr int NPAIR = ND / 4;           // 136 channel pairs
  constexpr int NQP = (NPAIR + 15) / 16;  // 9 per lane
  float4 d[NQP];
  double nrm2 = 0.0;
#pragma unroll
  for (int q = 0; q < NQP; ++q) {
    const int P = L + 16 * q;
    d[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (P < NPAIR) {
      int ca, cb;
      mixed_pair_channels(P, ca, cb);
      const float* x = crow + cidx(ca, 0);
      const float* y = crow + cidx(cb, 0);
      float d0 = x[0] * y[0];
      float d1 = x[1] * y[1] + x[2] * y[2] + x[3] * y[3];
      float d2 = 0.f, d3 = 0.f;
#pragma unroll
      for (int lm = 4; lm < 9; ++lm) d2 += x[lm] * y[lm];
#pragma unroll
      for (int lm = 9; lm < 16; ++lm) d3 += x[lm] * y[lm];
      d[q] = make_float4(d0, d1, d2, d3);
      nrm2 += (double)(d0 * d0 + d1 * d1) + (double)(d2 * d2 + d3 * d3);
    }
  }
  nrm2 = sum16d(nrm2);                    // the row's 16 lanes form one DPP row
  const float nrm = (float)sqrt(nrm2);
  const float scale = nrm > 0.f ? 1.f / nrm : 0.f;
  float4* out = reinterpret_cast<float4*>(D + (size_t)local * ND);
  float4* ext = d_out && i >= 0 ? reinterpret_cast<float4*>(d_out + (size_t)perm[i] * ND) : nullptr;
#pragma unroll
  for (int q = 0; q < NQP; ++q) {
    const int P = L + 16 * q;
    if (P < NPAIR) {
      const float4 o = make_float4(d[q].x * scale, d[q].y * scale, d[q].z * scale, d[q].w * scale);
      out[P] = o;
      if (ext) ext[P] = o;
    }
  }
  if (L == 0 && i >= 0) nrm_out[i] = nrm;
}

constexpr int NTG = 256;

// Displacement of every atom since the list build, x - xb in FP64, in caller order (the
// loads coalesced), stored in FP32 at the atom's internal index. It must stay within half
// the skin; it is kept in FP32 because it is smaller than half the skin, so its rounding is
// far below that of the pair vectors.
__global__ __launch_bounds__(NTG) void k_disp(int n, const int* __restrict__ inv_perm,
                                              const double* __restrict__ x, const double* __restrict__ y,
                                              const double* __restrict__ z, const double* __restrict__ xb,
                                              float4* __restrict__ dlt, double lim2, int* __restrict__ status) {
  const int a = blockIdx.x * NTG + threadIdx.x;
  if (a >= n) return;
  store_displacement(a, n, x[a], y[a], z[a], xb, inv_perm, dlt, lim2, status);
}

// Per-step geometry of every listed pair (slot_geom). The pair vector is split as
//   Delta = [(w_j - w_i) + s*L] + (delta_j - delta_i),
// the bracket fixed at the list build (FP64, stored rounded to FP32 with the neighbour's
// species in .w) and the displacements since the build added in FP32. One thread per slot
// (its loads independent of each other's); padding slots keep the zero geometry the list
// build gave them.
__global__ __launch_bounds__(NTG) void k_geom(long long nslots, const int* __restrict__ slot_atom,
                                              const int* __restrict__ slot_j,
                                              const float4* __restrict__ slot_d0,
                                              const float4* __restrict__ dlt, float rc2,
                                              float4* __restrict__ geom) {
  const long long slot = (long long)blockIdx.x * NTG + threadIdx.x;
  if (slot >= nslots) return;
  const int i = slot_atom[slot];
  if (i < 0) return;
  geom[slot] = slot_geom(slot_d0[slot], dlt[slot_j[slot]], dlt[i], rc2);
}

// |d~| of every atom in caller order (0 for an atom without neighbours).
__global__ __launch_bounds__(NTG) void k_export_norms(int n, const int* __restrict__ perm,
                                                      const int* __restrict__ bucket,
                                                      const float* __restrict__ nrm,
                                                      float* __restrict__ norm_out) {
  const int i = blockIdx.x * NTG + threadIdx.x;
  if (i >= n) return;
  norm_out[perm[i]] = bucket[i] < 0 ? 0.f : nrm[i];
}

}  // namespace

void gather_positions(flare_state* s, const double* x, const double* y, const double* z) {
  const int n = s->n_atoms;
  if (n == 0) return;
  const double lim = 0.5 * s->skin;
  k_disp<<<(n + NTG - 1) / NTG, NTG, 0, s->stream>>>(n, s->inv_perm, x, y, z, s->xb, s->dlt, lim * lim,
                                                     s->d_status);
}

void pair_geometry(flare_state* s) {
  const long long ns = s->n_slots;
  if (ns == 0) return;
  const double rc = s->model->r_cut;
  k_geom<<<(int)((ns + NTG - 1) / NTG), NTG, 0, s->stream>>>(ns, s->slot_atom, s->slot_j, s->slot_d0, s->dlt,
                                                             (float)(rc * rc), s->geom);
}

void desc_mixed_chunk(flare_state* s, int r0, int nr, float* d_out) {
  const SlotView v = slot_view(s);
  StageTimer tm(s, FLARE_T_DESCX);
  if (nr > 0)
    k_desc_mixed<<<nr / MROWS, MTHREADS, 0, s->stream>>>(v, s->rows1, r0, s->atom_of_rowx, s->perm, s->Dx, s->nrm,
                                                         d_out);
}

void export_norms(flare_state* s, float* norm_out) {
  const int n = s->n_atoms;
  if (n == 0 || !norm_out) return;
  k_export_norms<<<(n + NTG - 1) / NTG, NTG, 0, s->stream>>>(n, s->perm, s->bucket, s->nrm, norm_out);
}

}  // namespace flare
