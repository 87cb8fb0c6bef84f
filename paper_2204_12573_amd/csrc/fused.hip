// Descriptors and mapped quadratic forms of the single-species rows in one kernel
// (paper: B2 descriptors of Section V.B, Eq. 1 and Eq. 2 after the exact mapping).
//
// A work-group owns a tile of 128 rows of one environment bucket (one central species,
// one neighbour species, 144-component block):
//   1. descriptors: two lanes per row accumulate the densities and form d~ (B2) and |d~|
//      straight into an LDS tile [128][148] (the padding makes the 16-byte fragment reads
//      below conflict-free); nothing goes to HBM. The tile holds the unnormalised d~: the
//      products are linear in the row, so the epilogue applies 1/|d~|^2 once;
//   2. quadratic forms on the FP32 matrix cores (v_mfma_f32_16x16x4_f32): Y = D W for
//      W = Sigma_b then W = beta_b, A fragments from LDS, B fragments streamed from L2 in a
//      fragment-major copy of W (one contiguous 1 KB load per 16x16 block and K chunk);
//   3. epilogue, with Y~ = d~ W: V_i = Y~ . d~ / |d~|^2 (or |Z~|^2/|d~|^2 in the split form),
//      e_i = Y~ . d~ / |d~|^2, g_i = de_i/dd~_i = (2/|d~|^2)(Y~ - e_i d~) written into the
//      tile;
//   4. either g is copied out coalesced as G[tile][k][row] (the layout the standalone
//      adjoint kernel reads with one lane pair per row), or, when the forces are wanted
//      now, the lane pairs keep their row's densities from step 1 in registers, form
//      u = G^ c from the gradient tile in LDS and write the per-pair terms w (adjoint.h):
//      neither g nor c goes to HBM. The forces variant runs with every wave on its own 32-row
//      sub-tiles (k_fused144_w): each of the steps touches only the wave's own rows.
// Inside a 16-wide K chunk, k-step t of lane group q uses k = 4q + t for A and B alike.
#include <type_traits>

#include "adjoint.h"
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
  const uint64_t* W8[4]; // FP8 split form: s_b beta as [ks 5][cb 9][hi/lo' 2][lane 64] x 8 e4m3
  float bscale[4];       // FP8 split form: s_b per bucket (a power of two)
  const uint4* W6[4];    // three-way BF16 form: beta as [ks 5][cb 9][part 3][lane 64] x 8 bf16
  const double* L64[4];  // split forms: the Cholesky factor L in FP64, [cb 9][kc 9][t 4][lane 64]
  const float* D_in;     // optional [rows][144] given vectors (replace the descriptor phase; no
                         // normalisation: the forms are those of the vectors as given)
  int n_given;           // with D_in: rows 0 .. n_given - 1 are the given vectors
  int mode;              // bit 0: energy + gradient (beta), bit 1: variance (Sigma)
  int vchol;             // part 1 of Wf holds the Cholesky factor L: V = |L^T d|^2
  float* G;              // [tiles][144][128]: g, when the forces are not formed here
  float4* f_own;         // per row: sum of its own pair terms (written when the forces are formed here)
  float* nrm;            // per atom
  float* e_int;
  float* v_int;
  float* e_row;          // the same per row
  float* v_row;
  float* D_out;          // optional normalised descriptors in caller order, [n][544]: the
                         // row's block from component dstart of its bucket (others untouched)
  const int* perm;       // internal -> caller index (with D_out)
  int dstart[4];         // first component of each bucket's block in the 544 vector
};

// TRI: W = L lower-triangular, blocks of chunk kc with column block j > kc vanish. The
// chunks then run from the last (all 9 column blocks) to the first (1 block), so the
// loads of the next chunk are always covered by the larger MFMA work of the current one.
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
  constexpr int K0 = TRI ? NKC - 1 : 0;
#pragma unroll
  for (int j = 0; j < NCB; ++j)
    if (!TRI || j <= K0) bA[j] = Wp[(K0 * NCB + j) * 64];
#pragma unroll
  for (int it = 0; it < NKC; ++it) {
    const int kc = TRI ? NKC - 1 - it : it;      // chunk of this iteration
    const int kn = TRI ? kc - 1 : kc + 1;        // chunk of the next
    float4* cur = (it & 1) ? bB : bA;
    float4* nxt = (it & 1) ? bA : bB;
    if (it + 1 < NKC) {
#pragma unroll
      for (int j = 0; j < NCB; ++j)
        if (!TRI || j <= kn) nxt[j] = Wp[(kn * NCB + j) * 64];
    }
    float4 a[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      a[i] = *reinterpret_cast<const float4*>(&As[(wave * 32 + i * 16 + l16) * AS + kc * 16 + 4 * grp]);
    // keep the next chunk's loads ahead of this chunk's MFMAs (the scheduler would
    // otherwise sink them next to their use to shorten live ranges)
    __builtin_amdgcn_sched_barrier(0);
    // k-step outermost: consecutive MFMAs write different accumulators, so none waits
    // for the previous result
#define FQ_STEP(C)                                                                           \
  _Pragma("unroll") for (int j = 0; j < NCB; ++j) {                                         \
    if (TRI && j > kc) continue; /* lower-triangular W: rows k < column j vanish */         \
    _Pragma("unroll") for (int i = 0; i < 2; ++i)                                           \
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].C, cur[j].C, acc[i][j], 0, 0, 0); \
  }
    FQ_STEP(x)
    FQ_STEP(y)
    FQ_STEP(z)
    FQ_STEP(w)
#undef FQ_STEP
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

typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// two FP32 values to a packed BF16 pair (round to nearest even), and back
__device__ __forceinline__ unsigned int pk_bf16(float a, float b) {
  return __builtin_bit_cast(unsigned int, __builtin_convertvector((f2v){a, b}, bf2));
}
__device__ __forceinline__ float bf16_lo(unsigned int p) { return __builtin_bit_cast(float, p << 16); }
__device__ __forceinline__ float bf16_hi(unsigned int p) { return __builtin_bit_cast(float, p & 0xffff0000u); }

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
  u4v ph, pl;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    ph[t] = pk_bf16(v[2 * t], v[2 * t + 1]);
    pl[t] = pk_bf16(v[2 * t] - bf16_lo(ph[t]), v[2 * t + 1] - bf16_hi(ph[t]));
  }
  hi = __builtin_bit_cast(bf8, ph);
  lo = __builtin_bit_cast(bf8, pl);
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
  // column blocks in groups of three with one register buffer of B (hi, lo) fragments:
  // the lo parts for the next group load after the d_hi x beta_lo products, the hi parts
  // after the last use
  bf8 bh[3], bl[3];
#pragma unroll
  for (int jj = 0; jj < 3; ++jj) {
    bh[jj] = __builtin_bit_cast(bf8, Wp[(jj * 2 + 0) * 64]);
    bl[jj] = __builtin_bit_cast(bf8, Wp[(jj * 2 + 1) * 64]);
  }
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks) {
    bf8 ahi[2], alo[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      split8(&As[(wave * 32 + i * 16 + l16) * AS + ks * 32 + 8 * grp], ks == NKS - 1 && grp >= 2, ahi[i], alo[i]);
#pragma unroll
    for (int jg = 0; jg < NCB / 3; ++jg) {
      const int nks = jg + 1 < NCB / 3 ? ks : ks + 1, njg = jg + 1 < NCB / 3 ? jg + 1 : 0;
      const bool more = nks < NKS;
#pragma unroll
      for (int jj = 0; jj < 3; ++jj)
#pragma unroll
        for (int i = 0; i < 2; ++i)
          acc[i][3 * jg + jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[i], bl[jj], acc[i][3 * jg + jj], 0, 0, 0);
      if (more) {
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) bl[jj] = __builtin_bit_cast(bf8, Wp[((nks * NCB + 3 * njg + jj) * 2 + 1) * 64]);
      }
#pragma unroll
      for (int jj = 0; jj < 3; ++jj)
#pragma unroll
        for (int i = 0; i < 2; ++i)
          acc[i][3 * jg + jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[i], bh[jj], acc[i][3 * jg + jj], 0, 0, 0);
#pragma unroll
      for (int jj = 0; jj < 3; ++jj)
#pragma unroll
        for (int i = 0; i < 2; ++i)
          acc[i][3 * jg + jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[i], bh[jj], acc[i][3 * jg + jj], 0, 0, 0);
      if (more) {
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) bh[jj] = __builtin_bit_cast(bf8, Wp[((nks * NCB + 3 * njg + jj) * 2 + 0) * 64]);
      }
    }
  }
}

// Three-way BF16 form of both passes: x = x0 + x1 + x2 holds all 24 significant bits of
// an FP32 value exactly (x0 and x1 round the remainder of the previous parts to 8 bits,
// the remainders are exact in FP32, and the last one fits 8 bits), and the same for the
// model matrix. Of the nine part
// products the six with a part-index sum <= 2 are formed on v_mfma_f32_16x16x32_bf16
// (exact products, FP32 accumulation); the dropped x1 w2 + x2 w1 + x2 w2 are below
// 2^-23 |x||w|, the size of an FP32 rounding. K = 144 runs as five 32-wide steps
// as in the two-way form; column blocks go in groups of three so that the six products
// of a block are five other MFMAs apart.
// x0 = bf16(v), x1 = bf16(v - x0), x2 = v - x0 - x1: the last remainder has at most 8
// significant bits, so its BF16 pattern is the upper half of its FP32 pattern (exact)
__device__ __forceinline__ void split8x3(const float4 (&u)[2], bf8& x0, bf8& x1, bf8& x2) {
  const float v[8] = {u[0].x, u[0].y, u[0].z, u[0].w, u[1].x, u[1].y, u[1].z, u[1].w};
  u4v p0, p1, p2;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    p0[t] = pk_bf16(v[2 * t], v[2 * t + 1]);
    const float ra = v[2 * t] - bf16_lo(p0[t]), rb = v[2 * t + 1] - bf16_hi(p0[t]);
    p1[t] = pk_bf16(ra, rb);
    const float sa = ra - bf16_lo(p1[t]), sb = rb - bf16_hi(p1[t]);
    p2[t] = __builtin_amdgcn_perm(__builtin_bit_cast(unsigned int, sb), __builtin_bit_cast(unsigned int, sa),
                                  0x07060302u);
  }
  x0 = __builtin_bit_cast(bf8, p0);
  x1 = __builtin_bit_cast(bf8, p1);
  x2 = __builtin_bit_cast(bf8, p2);
}

// A operand of K step ks for row block i: 8 FP32 values (zeros past K = 144)
__device__ __forceinline__ void load_a8(const float* As, int wave, int l16, int grp, int i, int ks,
                                        float4 (&u)[2]) {
  if (ks == NKS - 1 && grp >= 2) {
    u[0] = u[1] = make_float4(0.f, 0.f, 0.f, 0.f);
  } else {
    const float* p = &As[(wave * 32 + i * 16 + l16) * AS + ks * 32 + 8 * grp];
    u[0] = *reinterpret_cast<const float4*>(p);
    u[1] = *reinterpret_cast<const float4*>(p + 4);
  }
}

// Steps (ks, jg) in order. One register buffer of B fragments: the products run B part 2
// first and part 0 last, and each part's fragments for the next step are loaded as soon as
// its last product here is issued; the next K step's A values are loaded at the start of a
// K step's last group.
__device__ __forceinline__ void mfma_pass_bf16x6(const float* As, const uint4* __restrict__ W, int wave,
                                                 int lane, f4 (&acc)[2][NCB]) {
  const int l16 = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NCB; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const uint4* Wp = W + lane;
  bf8 b[3][3];              // [block of the group][part]
  float4 araw[2][2];
  bf8 a[3][2];              // [part][row block]
#pragma unroll
  for (int jj = 0; jj < 3; ++jj)
#pragma unroll
    for (int pt = 0; pt < 3; ++pt)
      b[jj][pt] = __builtin_bit_cast(bf8, Wp[(jj * 3 + pt) * 64]);
#pragma unroll
  for (int i = 0; i < 2; ++i) load_a8(As, wave, l16, grp, i, 0, araw[i]);
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks) {
#pragma unroll
    for (int i = 0; i < 2; ++i) split8x3(araw[i], a[0][i], a[1][i], a[2][i]);
#pragma unroll
    for (int jg = 0; jg < NCB / 3; ++jg) {
      // the next step
      const bool same = jg + 1 < NCB / 3;
      const int nks = same ? ks : ks + 1, njg = same ? jg + 1 : 0;
      const bool more = nks < NKS;
      if (more && !same) {
#pragma unroll
        for (int i = 0; i < 2; ++i) load_a8(As, wave, l16, grp, i, nks, araw[i]);
      }
#define X6_PROD(PA, PB)                                                                       \
  _Pragma("unroll") for (int jj = 0; jj < 3; ++jj) {                                          \
    _Pragma("unroll") for (int i = 0; i < 2; ++i) acc[i][3 * jg + jj] =                       \
        __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[PA][i], b[jj][PB], acc[i][3 * jg + jj], 0, 0, 0); \
  }
#define X6_NEXT(PT)                                                                           \
  if (more) {                                                                                 \
    _Pragma("unroll") for (int jj = 0; jj < 3; ++jj)                                          \
      b[jj][PT] = __builtin_bit_cast(bf8, Wp[((nks * NCB + 3 * njg + jj) * 3 + PT) * 64]);     \
  }
      X6_PROD(0, 2)
      X6_NEXT(2)
      X6_PROD(1, 1)
      X6_PROD(0, 1)
      X6_NEXT(1)
      X6_PROD(2, 0)
      X6_PROD(1, 0)
      X6_PROD(0, 0)
      X6_NEXT(0)
#undef X6_PROD
#undef X6_NEXT
    }
  }
}

// FP8 split form on v_mfma_f32_16x16x32_fp8_fp8 (OCP e4m3, 3 mantissa bits). Each row is
// pre-scaled by a power of two s_r so that |s_r d~| < 16, and beta by s_b so that
// |s_b beta| < 16. With x = s_r d~ = x_hi + x_lo and b = s_b beta = b_hi + b_lo, the
// operands x_hi, x_lo' = fp8(16 x_lo), b_hi, b_lo' = fp8(16 b_lo) and 16 x_hi (exact: a
// power-of-two multiple of an e4m3 value that stays below 448) let one accumulator hold
//   (16 x_hi) b_hi + x_hi b_lo' + x_lo' b_hi  =  16 x b  minus the dropped 16 x_lo b_lo,
// so Y~ = acc / (16 s_r s_b). Lane (m, q) supplies k = 32t + 8q .. +7 as 8 bytes.
__device__ __forceinline__ long fp8x8(const float (&v)[8]) {
  int lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], 0, false);
  lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], lo, true);
  int hi = __builtin_amdgcn_cvt_pk_fp8_f32(v[4], v[5], 0, false);
  hi = __builtin_amdgcn_cvt_pk_fp8_f32(v[6], v[7], hi, true);
  return (long)(((unsigned long)(unsigned int)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ void fp8_unpack(long w, float (&v)[8]) {
  const int lo = (int)(w & 0xffffffffL), hi = (int)((unsigned long)w >> 32);
  v[0] = __builtin_amdgcn_cvt_f32_fp8(lo, 0);
  v[1] = __builtin_amdgcn_cvt_f32_fp8(lo, 1);
  v[2] = __builtin_amdgcn_cvt_f32_fp8(lo, 2);
  v[3] = __builtin_amdgcn_cvt_f32_fp8(lo, 3);
  v[4] = __builtin_amdgcn_cvt_f32_fp8(hi, 0);
  v[5] = __builtin_amdgcn_cvt_f32_fp8(hi, 1);
  v[6] = __builtin_amdgcn_cvt_f32_fp8(hi, 2);
  v[7] = __builtin_amdgcn_cvt_f32_fp8(hi, 3);
}
// split of 8 already-scaled values into (16 x_hi, x_hi, x_lo')
__device__ __forceinline__ void split8_fp8(const float (&x)[8], long& hi16, long& hi, long& lo) {
  hi = fp8x8(x);
  float h[8], r[8], h16[8];
  fp8_unpack(hi, h);
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    r[t] = 16.f * (x[t] - h[t]);
    h16[t] = 16.f * h[t];
  }
  lo = fp8x8(r);
  hi16 = fp8x8(h16);
}

__device__ __forceinline__ void mfma_pass_fp8(const float* As, const float* rs, const uint64_t* __restrict__ W,
                                              int wave, int lane, f4 (&acc)[2][NCB]) {
  const int l16 = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NCB; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const uint64_t* Wp = W + lane;
  float sr[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) sr[i] = rs[wave * 32 + i * 16 + l16];
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks) {
    long a16[2], ah[2], al[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      float x[8];
      if (ks == NKS - 1 && grp >= 2) {
#pragma unroll
        for (int t = 0; t < 8; ++t) x[t] = 0.f;
      } else {
        const float* p = &As[(wave * 32 + i * 16 + l16) * AS + ks * 32 + 8 * grp];
        const float4 x0 = *reinterpret_cast<const float4*>(p);
        const float4 x1 = *reinterpret_cast<const float4*>(p + 4);
        x[0] = x0.x * sr[i]; x[1] = x0.y * sr[i]; x[2] = x0.z * sr[i]; x[3] = x0.w * sr[i];
        x[4] = x1.x * sr[i]; x[5] = x1.y * sr[i]; x[6] = x1.z * sr[i]; x[7] = x1.w * sr[i];
      }
      split8_fp8(x, a16[i], ah[i], al[i]);
    }
    long bh[NCB], bl[NCB];
#pragma unroll
    for (int j = 0; j < NCB; ++j) {
      bh[j] = (long)Wp[((ks * NCB + j) * 2 + 0) * 64];
      bl[j] = (long)Wp[((ks * NCB + j) * 2 + 1) * 64];
    }
    // product outermost: consecutive MFMAs write different accumulators
#pragma unroll
    for (int j = 0; j < NCB; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a16[i], bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int j = 0; j < NCB; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int j = 0; j < NCB; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(al[i], bh[j], acc[i][j], 0, 0, 0);
  }
}

// FP8 fragments of beta for the split form: vals [groups][lane 64][8] (already scaled by
// s_b) -> out [groups][hi, lo' 2][lane 64], hi = fp8(v), lo' = fp8(16 (v - hi)); the same
// conversion instruction as the row operands, so both sides share one number format.
__global__ __launch_bounds__(256) void k_fp8_fragments(const float* __restrict__ vals, int groups,
                                                       uint64_t* __restrict__ out) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= groups * 64) return;
  const int g = idx >> 6, lane = idx & 63;
  float x[8], h[8], r[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) x[t] = vals[(size_t)idx * 8 + t];
  const long hi = fp8x8(x);
  fp8_unpack(hi, h);
#pragma unroll
  for (int t = 0; t < 8; ++t) r[t] = 16.f * (x[t] - h[t]);
  out[((size_t)g * 2 + 0) * 64 + lane] = (uint64_t)hi;
  out[((size_t)g * 2 + 1) * 64 + lane] = (uint64_t)fp8x8(r);
}

// Sum of squares of the 8 rows a lane touches (Z = D L, V = |z|^2): the terms are all
// non-negative, so there is no cancellation; the split forms accumulate in FP64 (the
// precision form keeps its variance sums FP64), the FP32 form in FP32 (relative rounding
// below 1e-6 for 144 terms).
template <bool F64>
__device__ __forceinline__ void row_sumsq(const f4 (&acc)[2][NCB], float (&out)[2][4]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (F64) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NCB; ++j) {
          const double z = (double)acc[i][j][r];
          s += z * z;
        }
        out[i][r] = (float)sum16d(s);
      } else {
        float s = 0.f;
#pragma unroll
        for (int j = 0; j < NCB; ++j) s = fmaf(acc[i][j][r], acc[i][j][r], s);
        out[i][r] = sum16(s);
      }
    }
}

// Variance of the split forms in FP64: Z~ = D~ L on v_mfma_f64_16x16x4_f64 (lane (m, q)
// supplies A[m][k] and B[k][n = m] for k = 4q + t of the chunk, as in the FP32 pass; D~ is
// exact in FP64, L is the FP64 Cholesky factor), V~ = |Z~|^2 summed in FP64. The FP64
// instruction returns row q + 4 r of the block in accumulator r of lane (n, q) (the FP32
// one row 4 q + r), so out[i][r] belongs to row 16 i + q + 4 r. A near-
// cancelling d^T Sigma d (an environment close to the sparse set: V << sigma^2 |d|^2) then
// keeps FP64 accuracy in the form itself; only the rounding of d~ remains. Column blocks go
// in three groups of three (six independent accumulators per k-step); the group's chunks
// start at its first block (L[k][n] = 0 for k < n) and the B fragments of the next chunk
// load while the current one runs.
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void var_pass_f64(const float* As, const double* __restrict__ L, int wave, int lane,
                                             double (&out)[2][4]) {
  const int l16 = lane & 15, grp = lane >> 4;
  double ss[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) ss[i][r] = 0.0;
  const double* Lp = L + lane;
#pragma unroll
  for (int jg = 0; jg < 3; ++jg) {
    d4 acc[2][3];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) acc[i][jj] = d4{0.0, 0.0, 0.0, 0.0};
    double bA[3][4], bB[3][4];
#pragma unroll
    for (int jj = 0; jj < 3; ++jj)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (jj == 0) bA[jj][t] = Lp[(((3 * jg + jj) * NKC + 3 * jg) * 4 + t) * 64];
#pragma unroll
    for (int kc = 3 * jg; kc < NKC; ++kc) {
      const bool odd = (kc - 3 * jg) & 1;
      double (&cur)[3][4] = odd ? bB : bA;
      double (&nxt)[3][4] = odd ? bA : bB;
      if (kc + 1 < NKC) {
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
          if (3 * jg + jj <= kc + 1)
#pragma unroll
            for (int t = 0; t < 4; ++t) nxt[jj][t] = Lp[(((3 * jg + jj) * NKC + kc + 1) * 4 + t) * 64];
      }
      float4 a[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[i] = *reinterpret_cast<const float4*>(&As[(wave * 32 + i * 16 + l16) * AS + kc * 16 + 4 * grp]);
      const float av[2][4] = {{a[0].x, a[0].y, a[0].z, a[0].w}, {a[1].x, a[1].y, a[1].z, a[1].w}};
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
          if (3 * jg + jj > kc) continue;     // block above the diagonal of L
#pragma unroll
          for (int i = 0; i < 2; ++i)
            acc[i][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)av[i][t], cur[jj][t], acc[i][jj], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int jj = 0; jj < 3; ++jj)
#pragma unroll
        for (int r = 0; r < 4; ++r) ss[i][r] = fma(acc[i][jj][r], acc[i][jj][r], ss[i][r]);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) out[i][r] = sum16d(ss[i][r]);
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
      out[i][r] = sum16(s);
    }
}

// Atom of a row (-1: padding); for given vectors (GIVEN) row r < n_given is "atom" r.
template <bool GIVEN>
__device__ __forceinline__ int atom_of(const FusedArgs& a, int row) {
  return GIVEN ? (row < a.n_given ? row : -1) : a.aor[row];
}

// Model operands of the bucket that holds rows [row0, row0 + 128).
struct TileModel {
  const float4* Wf;
  const uint4* Wb;
  const uint64_t* W8;
  const uint4* W6;
  const double* L64;
  float bsc;
  int dstart;
};
__device__ __forceinline__ TileModel tile_model(const FusedArgs& a, int row0) {
  TileModel m{a.Wf[0], a.Wb[0], a.W8[0], a.W6[0], a.L64[0], a.bscale[0], a.dstart[0]};
#pragma unroll
  for (int k = 1; k < 4; ++k)   // static indexing keeps the argument arrays out of scratch
    if (k < a.nbk && row0 >= a.row0[k] && row0 < a.row1[k])
      m = TileModel{a.Wf[k], a.Wb[k], a.W8[k], a.W6[k], a.L64[k], a.bscale[k], a.dstart[k]};
  return m;
}

// Per-row scalars of the tile (LDS): |d~| (FP32), |d~|^2 in FP64 (split forms), the FP8 row
// scale, the row's atom (-1: padding) and 1/|d~|^2, set by the descriptor phase so that the
// later phases read them from LDS instead of global memory.
struct RowScalars {
  float* nrm;
  double* nrm2;
  float* rsc;
  int* atom;
  float* inv2;
};

// 1. descriptors of the tile's rows into the LDS tile (thread t of 256: row t/2, half t&1);
// the densities are left in c for the adjoint phase of the same rows. With given
// descriptors (D_in) the lane pair copies its row instead and c stays zero.
template <int PREC, bool GIVEN>
__device__ __forceinline__ void desc_phase(const FusedArgs& a, float* As, const RowScalars& rs, int row0,
                                           int t, float (&c)[NR][NQ]) {
  const int rl = t >> 1, h = t & 1;
  const int i = atom_of<GIVEN>(a, row0 + rl);
#pragma unroll
  for (int n = 0; n < NR; ++n)
#pragma unroll
    for (int q = 0; q < NQ; ++q) c[n][q] = 0.f;
  if (i >= 0 && !GIVEN) accumulate_half(a.v, row0 + rl, h, c);
  // one B2 pass: the unnormalised d~ goes into the tile; 1/|d~| is applied in the
  // epilogue (Y is linear in the row, so Y(d) = Y(d~)/|d~|)
  // |d~|^2: FP64 in the split forms (their norms stay FP64), FP32 in the FP32 form (144
  // non-negative terms)
  typedef typename std::conditional<PREC == FLARE_FP32, float, double>::type NormT;
  NormT nrm2 = 0;
  float amax = 0.f;     // max |d~_k| (FP8 row scale)
  if (GIVEN) {
    // lane h copies components 72 h .. 72 h + 71 of its row (zeros for padding rows)
    const float4* src = reinterpret_cast<const float4*>(a.D_in + (size_t)(row0 + rl) * ND1 + 72 * h);
    float* dst = As + rl * AS + 72 * h;
#pragma unroll
    for (int q = 0; q < 18; ++q) {
      const float4 v = i >= 0 ? src[q] : make_float4(0.f, 0.f, 0.f, 0.f);
      nrm2 += (NormT)(v.x * v.x + v.y * v.y) + (NormT)(v.z * v.z + v.w * v.w);
      if (PREC == FLARE_FP8_SPLIT) amax = fmaxf(amax, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
      *reinterpret_cast<float4*>(dst + 4 * q) = v;
    }
  } else {
    float* rowp = As + rl * AS + 2 * h;
    int k = 0;
#pragma unroll
    for (int na = 0; na < NR; ++na) {
#pragma unroll
      for (int nb = na; nb < NR; ++nb) {
        const float2 mine = b2_half(c[na], c[nb], h);    // this lane's two components
        nrm2 += (NormT)(mine.x * mine.x + mine.y * mine.y);
        if (PREC == FLARE_FP8_SPLIT) amax = fmaxf(amax, fmaxf(fabsf(mine.x), fabsf(mine.y)));
        *reinterpret_cast<float2*>(rowp + 4 * k) = mine;
        ++k;
      }
    }
  }
  if (PREC == FLARE_FP32) nrm2 += xor1((float)nrm2);    // the row's other half
  else nrm2 += xor1d((double)nrm2);
  if (GIVEN) nrm2 = i >= 0 ? 1 : 0;     // given vectors: no normalisation
  const float nrm = (float)sqrt(nrm2);   // sqrtf in the FP32 form
  if (PREC == FLARE_FP8_SPLIT) {
    amax = fmaxf(amax, xor1(amax));
    int ex = 0;
    frexpf(amax > 0.f ? amax : 1.f, &ex);      // amax = f 2^ex, f in [0.5, 1)
    if (h == 0) rs.rsc[rl] = ldexpf(1.f, 4 - ex);   // |s_r d~| < 16
  }
  if (h == 0) {
    rs.nrm[rl] = nrm;
    rs.atom[rl] = i;
    rs.inv2[rl] = nrm > 0.f ? 1.f / (nrm * nrm) : 0.f;
    if (PREC != FLARE_FP32) rs.nrm2[rl] = (double)nrm2;
    if (i >= 0) a.nrm[i] = nrm;
  }
}

// 2/3. quadratic forms and epilogue on a complete descriptor tile; leaves g in the tile
// when the energy pass runs. Wave w of the 4 owns rows 32w .. 32w + 31.
// V64: the variance in FP64 (split forms); otherwise through the FP32 factor (or the full
// Sigma in the FP32 form without a factor).
template <int PREC, bool V64, bool GIVEN>
__device__ __forceinline__ void forms_phase(const FusedArgs& a, float* As, const RowScalars& rs, int row0, int t,
                                            const TileModel& tm) {
  const int lane = t & 63, wave = t >> 6;
  const int l16 = lane & 15, grp = lane >> 4;
  const float* nrm_s = rs.nrm;
  const float* rsc_s = rs.rsc;
  f4 acc[2][NCB];
  float dots[2][4];
  if ((a.mode & 2) && V64) {
    // split forms: V = |L^T d~|^2 / |d~|^2 with FP64 products, sums and division
    double vv[2][4];
    var_pass_f64(As, tm.L64, wave, lane, vv);
    if (l16 == 0) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rl = wave * 32 + i * 16 + grp + 4 * r;     // FP64 accumulator layout
          const int atom = rs.atom[rl];
          const double n2 = rs.nrm2[rl];
          if (atom >= 0) {
            const float v = n2 > 0.0 ? (float)(vv[i][r] / n2) : 0.f;
            a.v_int[atom] = v;
            a.v_row[row0 + rl] = v;
          }
        }
    }
  } else if (a.mode & 2) {
    if (a.vchol) {
      // Z = D L on FP32 cores, L lower-triangular
      mfma_pass<1, true>(As, tm.Wf, wave, lane, acc);
      row_sumsq<PREC != FLARE_FP32>(acc, dots);
    } else {
      mfma_pass<1>(As, tm.Wf, wave, lane, acc);
      row_dots(As, acc, wave, lane, dots);
    }
    if (l16 == 0) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rl = wave * 32 + i * 16 + 4 * grp + r;
          const int atom = rs.atom[rl];
          const float nv = nrm_s[rl];
          if (atom >= 0) {
            const float v = nv > 0.f ? dots[i][r] / (nv * nv) : 0.f;
            a.v_int[atom] = v;
            a.v_row[row0 + rl] = v;
          }
        }
    }
  }
  if (a.mode & 1) {
    if (PREC == FLARE_BF16_SPLIT) {
      mfma_pass_bf16<0>(As, tm.Wb, wave, lane, acc);
    } else if (PREC == FLARE_BF16X6_SPLIT) {
      mfma_pass_bf16x6(As, tm.W6, wave, lane, acc);
    } else if (PREC == FLARE_FP8_SPLIT) {
      mfma_pass_fp8(As, rsc_s, tm.W8, wave, lane, acc);
      // undo the power-of-two scales: Y~ = acc / (16 s_r s_b), exact
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float inv = 1.f / (16.f * rsc_s[wave * 32 + i * 16 + 4 * grp + r] * tm.bsc);
#pragma unroll
          for (int j = 0; j < NCB; ++j) acc[i][j][r] *= inv;
        }
    } else {
      mfma_pass<0>(As, tm.Wf, wave, lane, acc);
    }
    row_dots(As, acc, wave, lane, dots);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rl = wave * 32 + i * 16 + 4 * grp + r;
        const int atom = rs.atom[rl];
        const float inv2 = rs.inv2[rl];
        const float e = dots[i][r] * inv2;        // e = Y~ . d~ / |d~|^2
        if (l16 == 0 && atom >= 0) {
          a.e_int[atom] = e;
          a.e_row[row0 + rl] = e;
        }
        const float s2 = 2.f * inv2;              // g = (2/|d~|^2) (Y~ - e d~)
        float* d = As + rl * AS + l16;
        // each lane reads its own d-elements before overwriting them with g
#pragma unroll
        for (int j = 0; j < NCB; ++j) d[j * 16] = s2 * (acc[i][j][r] - e * d[j * 16]);
      }
  }
}

// 4. adjoint in place: u = G^ c from the gradient tile, then the per-pair terms. The
// densities c come from the descriptor phase of the same rows, kept in registers through
// the forms phase (no second pass over the pairs, no round trip through memory).
__device__ __forceinline__ void adjoint_phase(const FusedArgs& a, const float* As, const RowScalars& rs, int row0,
                                              int t, float (&c)[NR][NQ]) {
  const int rl = t >> 1, h = t & 1;
  if (rs.atom[rl] < 0) return;     // descriptor rows only
  u_transform_half(As + rl * AS, 1, h, c);
  adjoint_pairs_half(a.v, row0 + rl, h, c, a.f_own);
}

// One tile per work-group, phases in sequence (descriptor export, energies or variances
// without forces: g leaves as G[tile][k][row] for the separate adjoint kernel).
template <int PREC, bool V64, bool GIVEN>
__global__ __launch_bounds__(FT, 2) void k_fused144(FusedArgs a) {
  __shared__ __attribute__((aligned(16))) float As[FR * AS];
  __shared__ float nrm_s[FR];
  __shared__ double nrm2_s[FR];   // split forms: |d~|^2 in FP64
  __shared__ float rsc_s[FR];     // FP8 split form: power-of-two row scale s_r
  __shared__ int atom_s[FR];
  __shared__ float inv2_s[FR];
  const RowScalars rs{nrm_s, nrm2_s, rsc_s, atom_s, inv2_s};
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int row0 = tile * FR;
  const int t = threadIdx.x;
  {
    float c[NR][NQ];
    desc_phase<PREC, GIVEN>(a, As, rs, row0, t, c);
  }
  __syncthreads();
  const TileModel tm = tile_model(a, row0);
  if (!GIVEN && a.D_out) {
    for (int idx = t; idx < FR * ND1; idx += FT) {
      const int r = idx / ND1, k = idx % ND1;
      const int i = atom_s[r];
      const float nv = nrm_s[r];
      if (i >= 0) a.D_out[(size_t)a.perm[i] * ND + tm.dstart + k] = nv > 0.f ? As[r * AS + k] / nv : 0.f;
    }
  }
  forms_phase<PREC, V64, GIVEN>(a, As, rs, row0, t, tm);
  if (a.mode & 1) {
    __syncthreads();
    float* G = a.G + (size_t)tile * ND1 * FR;
    for (int idx = t; idx < FR * ND1; idx += FT) {
      const int k = idx >> 7, r = idx & (FR - 1);
      G[idx] = As[r * AS + k];
    }
  }
}

// Energies, forces (and variances) with every wave on its own: a wave's rows are touched
// only by that wave in all three phases (desc_phase: lane pair per row; forms_phase: wave
// w of a tile owns rows 32w..32w+31; adjoint_phase: lane pair per row), so each wave takes
// 32-row sub-tiles (its index, then + the number of waves in the grid) and runs
// descriptors, forms and adjoint on them back to back, with no work-group barrier. The two
// waves that share a SIMD drift apart, so their vector and matrix work interleave on the
// shared datapath.
constexpr int WR = 32;          // rows per wave sub-tile
constexpr int WW = 8;           // waves per work-group

// Between two phases of a wave: orders its LDS accesses (other lanes of the wave read what
// this lane wrote; the hardware keeps one wave's LDS operations in order) and keeps the
// compiler from moving memory operations or other work from one phase into the next.
__device__ __forceinline__ void wave_phase_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  asm volatile("" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

template <int PREC, bool V64>
__global__ __launch_bounds__(WW * 64, 1) void k_fused144_w(FusedArgs a, int nsub) {
  __shared__ __attribute__((aligned(16))) float As[WW][WR * AS];
  __shared__ float nrm_s[WW][WR];
  __shared__ double nrm2_s[WW][WR];
  __shared__ float rsc_s[WW][WR];
  __shared__ int atom_s[WW][WR];
  __shared__ float inv2_s[WW][WR];
  // the wave index is uniform over the wave: scalar, and with it the sub-tile loop and rows
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int nw = gridDim.x * WW;
  float* A = As[wv];
  const RowScalars rs{nrm_s[wv], nrm2_s[wv], rsc_s[wv], atom_s[wv], inv2_s[wv]};
  for (int st = blockIdx.x * WW + wv; st < nsub; st += nw) {
    const int row0 = st * WR;
    float c[NR][NQ];
    // wave priorities by phase, for when both waves of a SIMD can issue: the matrix-core
    // phase first (its MFMAs keep the shared datapath busy 32 cycles each and the other
    // wave fills the gaps), then the descriptor phase (its pair loads start early), the
    // adjoint phase last; measured 811 -> 786 us against the matrix phase alone raised,
    // no gain with the adjoint level with the descriptors, a loss with the descriptors
    // above the matrix phase
    __builtin_amdgcn_s_setprio(1);
    desc_phase<PREC, false>(a, A, rs, row0, lane, c);
    wave_phase_fence();
    __builtin_amdgcn_s_setprio(2);
    forms_phase<PREC, V64, false>(a, A, rs, row0, lane, tile_model(a, row0));
    __builtin_amdgcn_s_setprio(0);
    wave_phase_fence();
    adjoint_phase(a, A, rs, row0, lane, c);
    wave_phase_fence();
  }
}

}  // namespace

void make_fp8_fragments(const float* vals, int groups, uint64_t* out) {
  k_fp8_fragments<<<(groups * 64 + 255) / 256, 256>>>(vals, groups, out);
}

// Launch k_fused144 (one tile per work-group) for the model's arithmetic.
template <bool GIVEN>
void launch_tiles(const flare_model* m, const FusedArgs& a, int ntiles, hipStream_t st) {
  const bool v64 = m->var64;
  if (m->precision == FLARE_BF16_SPLIT) {
    if (v64) k_fused144<FLARE_BF16_SPLIT, true, GIVEN><<<ntiles, FT, 0, st>>>(a);
    else k_fused144<FLARE_BF16_SPLIT, false, GIVEN><<<ntiles, FT, 0, st>>>(a);
  } else if (m->precision == FLARE_BF16X6_SPLIT) {
    if (v64) k_fused144<FLARE_BF16X6_SPLIT, true, GIVEN><<<ntiles, FT, 0, st>>>(a);
    else k_fused144<FLARE_BF16X6_SPLIT, false, GIVEN><<<ntiles, FT, 0, st>>>(a);
  } else if (m->precision == FLARE_FP8_SPLIT) {
    if (v64) k_fused144<FLARE_FP8_SPLIT, true, GIVEN><<<ntiles, FT, 0, st>>>(a);
    else k_fused144<FLARE_FP8_SPLIT, false, GIVEN><<<ntiles, FT, 0, st>>>(a);
  } else {
    k_fused144<FLARE_FP32, false, GIVEN><<<ntiles, FT, 0, st>>>(a);
  }
}

// Quadratic forms of given 144-wide vectors (rows 0 .. n-1) with the model block of single-
// species bucket `bucket`: e_r = d_r^T beta d_r, v_r = d_r^T Sigma d_r, by the same forms
// phase as the descriptor path. Per-row scratch: the state's e_row, v_row, G1 and nrm.
void forms_given_144(flare_state* s, int bucket, int n, const float* d, float* e, float* v) {
  const int rows = (n + FR - 1) / FR * FR;
  if (rows == 0) return;
  const flare_model* m = s->model;
  FusedArgs a{};
  a.aor = nullptr;
  a.n_given = n;
  a.D_in = d;
  a.nbk = 1;
  a.row0[0] = 0;
  a.row1[0] = rows;
  a.Wf[0] = reinterpret_cast<const float4*>(m->Wf[bucket]);
  a.Wb[0] = reinterpret_cast<const uint4*>(m->Wb[bucket]);
  a.W8[0] = m->W8[bucket];
  a.W6[0] = reinterpret_cast<const uint4*>(m->W6[bucket]);
  a.L64[0] = m->L64[bucket];
  a.bscale[0] = m->beta_scale[bucket];
  a.vchol = m->vchol ? 1 : 0;
  a.G = s->G1;
  a.nrm = s->nrm;
  a.e_int = e;
  a.v_int = v;
  a.e_row = s->e_row;
  a.v_row = s->v_row;
  a.mode = 3;
  launch_tiles<true>(m, a, rows / FR, s->stream);
}

void fused_quadratic_forms(flare_state* s, int mode, float* d_out) {
  if (s->rows1 == 0 || (!(mode & (3 | FORMS_DESCRIPTORS)) && !d_out)) return;
  FusedArgs a{};
  a.v = slot_view(s);
  a.aor = s->atom_of_row1;
  a.nbk = 4;
  for (int k = 0; k < 4; ++k) {
    const int padded = (s->bucket_count[k] + TILE_ROWS - 1) / TILE_ROWS * TILE_ROWS;
    a.row0[k] = s->bucket_row0[k];
    a.row1[k] = s->bucket_row0[k] + padded;
    a.Wf[k] = reinterpret_cast<const float4*>(s->model->Wf[k]);
    a.Wb[k] = reinterpret_cast<const uint4*>(s->model->Wb[k]);
    a.W8[k] = s->model->W8[k];
    a.W6[k] = reinterpret_cast<const uint4*>(s->model->W6[k]);
    a.L64[k] = s->model->L64[k];
    a.bscale[k] = s->model->beta_scale[k];
  }
  a.vchol = s->model->vchol ? 1 : 0;
  a.G = s->G1;
  a.f_own = s->f_own;
  a.nrm = s->nrm;
  a.e_int = s->e_int;
  a.v_int = s->v_int;
  a.e_row = s->e_row;
  a.v_row = s->v_row;
  a.D_out = d_out;
  a.perm = s->perm;
  for (int k = 0; k < 4; ++k) a.dstart[k] = bucket_env(k) == 0 ? 0 : ND - ND1;
  const int ntiles = s->rows1 / FR;
  a.mode = mode & 3;
  if ((mode & 5) == 5) {
    // energies + forces: persistent work-groups, one per CU, waves independent
    const int nsub = s->rows1 / WR;
    const int grid = std::min(256, (nsub + WW - 1) / WW);
    const flare_model* m = s->model;
    const bool v64 = m->var64;
    hipStream_t st = s->stream;
    if (m->precision == FLARE_BF16_SPLIT) {
      if (v64) k_fused144_w<FLARE_BF16_SPLIT, true><<<grid, WW * 64, 0, st>>>(a, nsub);
      else k_fused144_w<FLARE_BF16_SPLIT, false><<<grid, WW * 64, 0, st>>>(a, nsub);
    } else if (m->precision == FLARE_BF16X6_SPLIT) {
      if (v64) k_fused144_w<FLARE_BF16X6_SPLIT, true><<<grid, WW * 64, 0, st>>>(a, nsub);
      else k_fused144_w<FLARE_BF16X6_SPLIT, false><<<grid, WW * 64, 0, st>>>(a, nsub);
    } else if (m->precision == FLARE_FP8_SPLIT) {
      if (v64) k_fused144_w<FLARE_FP8_SPLIT, true><<<grid, WW * 64, 0, st>>>(a, nsub);
      else k_fused144_w<FLARE_FP8_SPLIT, false><<<grid, WW * 64, 0, st>>>(a, nsub);
    } else {
      k_fused144_w<FLARE_FP32, false><<<grid, WW * 64, 0, st>>>(a, nsub);
    }
    return;
  }
  launch_tiles<false>(s->model, a, ntiles, s->stream);
}

}  // namespace flare
