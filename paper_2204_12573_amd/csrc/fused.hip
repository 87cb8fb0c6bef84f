// Descriptors and mapped quadratic forms of the single-species rows in one kernel
// (paper: B2 descriptors of Section V.B, Eq. 1 and Eq. 2 after the exact mapping).
//
// A work-group owns a tile of 128 rows of one environment bucket (one central species,
// one neighbour species, 144-component block):
//   1. descriptors: two lanes per row accumulate the densities, form d~ (B2), |d~| and
//      d = d~/|d~| straight into an LDS tile [128][148] (the padding makes the 16-byte
//      fragment reads below conflict-free); nothing goes to HBM;
//   2. quadratic forms on the FP32 matrix cores (v_mfma_f32_16x16x4_f32): Y = D W for
//      W = Sigma_b then W = beta_b, A fragments from LDS, B fragments streamed from L2 in a
//      fragment-major copy of W (one contiguous 1 KB load per 16x16 block and K chunk);
//   3. epilogue: V_i = Y_i . d_i, e_i = Y_i . d_i, g_i = (2/|d~_i|)(Y_i - e_i d_i) written
//      into the tile and copied out coalesced as G[tile][k][row] (the layout the adjoint
//      kernel reads with one lane pair per row).
// Inside a 16-wide K chunk, k-step t of lane group q uses k = 4q + t for A and B alike.
#include "half.h"
#include "state.h"

namespace flare {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int FT = 256;       // threads
constexpr int FR = 128;       // rows per tile
constexpr int AS = ND1 + 4;   // LDS row stride of the tile (floats)
constexpr int NKC = ND1 / 16; // 9 K chunks
constexpr int NCB = ND1 / 16; // 9 column blocks

struct FusedArgs {
  SlotView v;
  const int* aor;        // atom of row, -1 for padding
  int nbk;
  int row0[4], row1[4];
  const float4* Wf[4];   // per bucket [part 2][kc 9][cb 9][lane 64]
  const uint4* Wb[4];    // split form: beta as [ks 5][cb 9][hi/lo 2][lane 64] x 8 bf16
  int mode;              // bit 0: energy + gradient (beta), bit 1: variance (Sigma)
  float* G;              // [tiles][144][128]
  float* nrm;            // per atom
  float* e_int;
  float* v_int;
  float* D_out;          // optional [rows][144] normalised descriptors
};

template <int PART, bool TRI = false>
__device__ __forceinline__ void mfma_pass(const float* As, const float4* __restrict__ W, int wave, int lane,
                                          f4 (&acc)[2][NCB]) {
  const int l16 = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NCB; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const float4* Wp = W + (size_t)PART * NKC * NCB * 64 + lane;
  float4 bA[NCB], bB[NCB];
#pragma unroll
  for (int j = 0; j < NCB; ++j)
    if (!TRI || j == 0) bA[j] = Wp[j * 64];
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc) {
    float4* cur = (kc & 1) ? bB : bA;
    float4* nxt = (kc & 1) ? bA : bB;
    if (kc + 1 < NKC) {
#pragma unroll
      for (int j = 0; j < NCB; ++j)
        if (!TRI || j <= kc + 1) nxt[j] = Wp[((kc + 1) * NCB + j) * 64];
    }
    float4 a[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      a[i] = *reinterpret_cast<const float4*>(&As[(wave * 32 + i * 16 + l16) * AS + kc * 16 + 4 * grp]);
#pragma unroll
    for (int j = 0; j < NCB; ++j) {
      if (TRI && j > kc) continue;      // lower-triangular W: rows k < column j vanish
      const float4 b = cur[j];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].x, b.x, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].y, b.y, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].z, b.z, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].w, b.w, acc[i][j], 0, 0, 0);
      }
    }
  }
}

// Split form of the energy pass on v_mfma_f32_16x16x32_bf16: D = D_hi + D_lo and
// beta = beta_hi + beta_lo in BF16, Y = D_hi beta_hi + D_hi beta_lo + D_lo beta_hi with FP32
// accumulation (the dropped D_lo beta_lo is ~2^-16 relative). K = 144 runs as five 32-wide
// steps; in the last one lane groups 2-3 (k = 144..159) feed zeros and the stored beta is
// zero there. Lane (m, q) supplies A[m][32t + 8q .. +7] and B[32t + 8q .. +7][n].
// The variance pass of the split form stays on FP32 cores with the Cholesky factor L of
// Sigma: V = |L^T d|^2 turns the possibly near-cancelling d^T Sigma d into a sum of
// squares whose error follows the rounding of d, not the size of the cancelled terms.
constexpr int NKS = 5;

__device__ __forceinline__ void split8(const float* p, bool zero, bf8& hi, bf8& lo) {
  float v[8];
  if (zero) {
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = 0.f;
  } else {
    const float4 x0 = *reinterpret_cast<const float4*>(p);
    const float4 x1 = *reinterpret_cast<const float4*>(p + 4);
    v[0] = x0.x; v[1] = x0.y; v[2] = x0.z; v[3] = x0.w;
    v[4] = x1.x; v[5] = x1.y; v[6] = x1.z; v[7] = x1.w;
  }
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    hi[t] = (__bf16)v[t];
    lo[t] = (__bf16)(v[t] - (float)hi[t]);
  }
}

template <int PART>
__device__ __forceinline__ void mfma_pass_bf16(const float* As, const uint4* __restrict__ W, int wave,
                                               int lane, f4 (&acc)[2][NCB]) {
  const int l16 = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NCB; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const uint4* Wp = W + lane;
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks) {
    bf8 ahi[2], alo[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      split8(&As[(wave * 32 + i * 16 + l16) * AS + ks * 32 + 8 * grp], ks == NKS - 1 && grp >= 2, ahi[i], alo[i]);
#pragma unroll
    for (int j = 0; j < NCB; ++j) {
      const uint4 bh = Wp[((ks * NCB + j) * 2 + 0) * 64];
      const uint4 bl = Wp[((ks * NCB + j) * 2 + 1) * 64];
      const bf8 bhv = __builtin_bit_cast(bf8, bh);
      const bf8 blv = __builtin_bit_cast(bf8, bl);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[i], bhv, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[i], blv, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[i], bhv, acc[i][j], 0, 0, 0);
      }
    }
  }
}

// Sum of squares of the 8 rows a lane touches (Z = D L, V = |z|^2), accumulated in FP64.
__device__ __forceinline__ void row_sumsq(const f4 (&acc)[2][NCB], float (&out)[2][4]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < NCB; ++j) {
        const double z = (double)acc[i][j][r];
        s += z * z;
      }
#pragma unroll
      for (int m = 1; m < 16; m <<= 1) s += __shfl_xor(s, m, 64);
      out[i][r] = (float)s;
    }
}

// Row-dots Y_row . d_row of the 8 rows a lane touches; all 16 lanes of a group get the sum.
__device__ __forceinline__ void row_dots(const float* As, const f4 (&acc)[2][NCB], int wave, int lane,
                                         float (&out)[2][4]) {
  const int l16 = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float* d = As + (wave * 32 + i * 16 + 4 * grp + r) * AS + l16;
      float s = 0.f;
#pragma unroll
      for (int j = 0; j < NCB; ++j) s += acc[i][j][r] * d[j * 16];
#pragma unroll
      for (int m = 1; m < 16; m <<= 1) s += __shfl_xor(s, m, 64);
      out[i][r] = s;
    }
}

template <int PREC>
__global__ __launch_bounds__(FT, 2) void k_fused144(FusedArgs a) {
  __shared__ __attribute__((aligned(16))) float As[FR * AS];
  __shared__ float nrm_s[FR];
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int row0 = tile * FR;
  const float4* Wb = a.Wf[0];
  const uint4* Wh = a.Wb[0];
#pragma unroll
  for (int k = 1; k < 4; ++k)
    if (k < a.nbk && row0 >= a.row0[k] && row0 < a.row1[k]) {
      Wb = a.Wf[k];
      Wh = a.Wb[k];
    }
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;

  // ---- 1. descriptors into the LDS tile ----
  {
    const int rl = t >> 1, h = t & 1;
    const int i = a.aor[row0 + rl];
    float c[NR][NQ];
#pragma unroll
    for (int n = 0; n < NR; ++n)
#pragma unroll
      for (int q = 0; q < NQ; ++q) c[n][q] = 0.f;
    if (i >= 0) accumulate_half(a.v, row0 + rl, h, c);
    double nrm2 = 0.0;    // |d~|^2 accumulated in FP64
#pragma unroll
    for (int na = 0; na < NR; ++na)
#pragma unroll
      for (int nb = na; nb < NR; ++nb) {
        const float4 d = b2_half(c[na], c[nb], h);
        nrm2 += (double)(d.x * d.x + d.y * d.y) + (double)(d.z * d.z + d.w * d.w);
      }
    const float nrm = (float)sqrt(nrm2);
    const float inv = nrm > 0.f ? 1.f / nrm : 0.f;
    float* rowp = As + rl * AS + 2 * h;
    int k = 0;
#pragma unroll
    for (int na = 0; na < NR; ++na)
#pragma unroll
      for (int nb = na; nb < NR; ++nb) {
        const float4 d = b2_half(c[na], c[nb], h);
        *reinterpret_cast<float2*>(rowp + 4 * k) =
            h ? make_float2(d.z * inv, d.w * inv) : make_float2(d.x * inv, d.y * inv);
        ++k;
      }
    if (h == 0) {
      nrm_s[rl] = nrm;
      if (i >= 0) a.nrm[i] = nrm;
    }
  }
  __syncthreads();
  if (a.D_out) {
    for (int idx = t; idx < FR * ND1; idx += FT) {
      const int r = idx / ND1, k = idx % ND1;
      a.D_out[(size_t)(row0 + r) * ND1 + k] = As[r * AS + k];
    }
  }

  // ---- 2/3. quadratic forms and epilogue ----
  const int l16 = lane & 15, grp = lane >> 4;
  f4 acc[2][NCB];
  float dots[2][4];
  if (a.mode & 2) {
    if (PREC == FLARE_BF16_SPLIT) {
      mfma_pass<1, true>(As, Wb, wave, lane, acc);   // Z = D L on FP32 cores, L lower-triangular
      row_sumsq(acc, dots);
    } else {
      mfma_pass<1>(As, Wb, wave, lane, acc);
      row_dots(As, acc, wave, lane, dots);
    }
    if (l16 == 0) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int atom = a.aor[row0 + wave * 32 + i * 16 + 4 * grp + r];
          if (atom >= 0) a.v_int[atom] = dots[i][r];
        }
    }
  }
  if (a.mode & 1) {
    if (PREC == FLARE_BF16_SPLIT) mfma_pass_bf16<0>(As, Wh, wave, lane, acc);
    else mfma_pass<0>(As, Wb, wave, lane, acc);
    row_dots(As, acc, wave, lane, dots);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rl = wave * 32 + i * 16 + 4 * grp + r;
        const int atom = a.aor[row0 + rl];
        if (l16 == 0 && atom >= 0) a.e_int[atom] = dots[i][r];
        const float nv = nrm_s[rl];
        const float s2 = nv > 0.f ? 2.f / nv : 0.f;
        float* d = As + rl * AS + l16;
        // each lane reads its own d-elements before overwriting them with g
#pragma unroll
        for (int j = 0; j < NCB; ++j) d[j * 16] = s2 * (acc[i][j][r] - dots[i][r] * d[j * 16]);
      }
    __syncthreads();
    float* G = a.G + (size_t)tile * ND1 * FR;
    for (int idx = t; idx < FR * ND1; idx += FT) {
      const int k = idx >> 7, r = idx & (FR - 1);
      G[idx] = As[r * AS + k];
      (void)k;
    }
  }
}

}  // namespace

void fused_quadratic_forms(flare_state* s, int mode, float* d_out) {
  if (s->rows1 == 0 || (!mode && !d_out)) return;
  FusedArgs a{};
  a.v = slot_view(s);
  a.aor = s->atom_of_row1.p;
  a.nbk = 4;
  for (int k = 0; k < 4; ++k) {
    const int padded = (s->bucket_count[k] + TILE_ROWS - 1) / TILE_ROWS * TILE_ROWS;
    a.row0[k] = s->bucket_row0[k];
    a.row1[k] = s->bucket_row0[k] + padded;
    a.Wf[k] = reinterpret_cast<const float4*>(s->model->Wf[k]);
    a.Wb[k] = reinterpret_cast<const uint4*>(s->model->Wb[k]);
  }
  a.mode = mode;
  a.G = s->G1.p;
  a.nrm = s->nrm;
  a.e_int = s->e_int;
  a.v_int = s->v_int;
  a.D_out = d_out;
  if (s->model->precision == FLARE_BF16_SPLIT)
    k_fused144<FLARE_BF16_SPLIT><<<s->rows1 / FR, FT, 0, s->stream>>>(a);
  else
    k_fused144<FLARE_FP32><<<s->rows1 / FR, FT, 0, s->stream>>>(a);
}

}  // namespace flare
