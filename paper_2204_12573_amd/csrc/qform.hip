// Mapped quadratic forms of the mixed-environment rows (paper, Eq. 1 and Eq. 2 after the
// exact mapping of Section V.B): for the 544-wide descriptor rows D of a bucket,
//   Y = D beta_s (dense GEMM on the FP32 matrix cores, FP32 accumulate), e_i = Y_i . D_i,
//   V_i = D_i . Sigma_s D_i, or |L_s^T D_i|^2 with the Cholesky factor of Sigma_s,
//   g_i = (2/|d~_i|) (Y_i - e_i d_i)  (de_i/dd~_i, used by the adjoint; k_qform_finish).
// A launch covers column tiles of 272: the beta part first, then the Sigma part; each
// tile writes its partial row sums, the beta tiles also Y.
//
// Tiling: a work-group of 4 waves owns 64 RB rows; each wave owns RB 16-row blocks x CB
// 16-column blocks, accumulated by v_mfma_f32_16x16x4_f32. Three work-groups share a CU
// (LDS allows three; the B fragments are read in groups of four column blocks so that the
// registers allow three waves per SIMD as well). K advances in
// chunks of 16 staged in LDS (double-buffered). Inside a chunk the four k-steps are
// interleaved so that each lane reads its four k-values of A and of B with one
// 128-bit LDS load: k-step t, lane group g uses k = 4g + t (the same map for A and B,
// which is all a sum over k requires). LDS rows are padded to 20 floats, which spreads
// the eight 16-byte reads of each lane octet over distinct banks.
#include <algorithm>
#include <type_traits>

#include "state.h"

namespace flare {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int NTQ = 256;
constexpr int KC = 16;          // K chunk
constexpr int LDSW = KC + 4;    // padded LDS row (floats)


struct QArgs {
  const float* D;        // [rows][KD]
  const int* aor;        // atom of row (-1 padding)
  float* Y;              // [rows][KD]      beta-part products
  float* P;              // [rows][4]       partial row sums of each column tile
  int mode;              // bit 0: beta part, bit 1: Sigma part
  int sumsq;             // Sigma part given as its Cholesky factor L: V = |d L|^2
  int nbk;               // buckets in this launch
  int row0[4];           // first row of each bucket (padded to TM)
  int row1[4];           // one past its last padded row
  const float* W[4];     // [(parts)*KD][KD] row n = column n of [beta | Sigma]
  const float* L[4];     // sumsq: [KD][KD] row n = column n of the Cholesky factor of Sigma
};

template <int KD, int CB, int RB>
__global__ __launch_bounds__(NTQ, 3) void k_qform(QArgs q) {
  constexpr int TM = 4 * RB * 16;              // rows per work-group
  constexpr int NC = CB * 16;                  // columns per work-group
  constexpr int NCHUNK = KD / KC;
  static_assert(KD % KC == 0, "K must be a multiple of the chunk");
  __shared__ __attribute__((aligned(16))) float As[2][TM * LDSW];
  __shared__ __attribute__((aligned(16))) float Bs[2][NC * LDSW];

  const int tile = blockIdx.x;
  const int ntile = blockIdx.y;
  const int row0 = tile * TM;
  // column tiles: the beta part first (if any), then the Sigma part, from L when sumsq
  const int nbeta = (q.mode & 1) ? KD / NC : 0;
  const bool lpart = q.sumsq && ntile >= nbeta;
  // bucket of this tile (static indexing keeps the argument arrays out of scratch)
  const float* Wb = lpart ? q.L[0] : q.W[0];
#pragma unroll
  for (int k = 1; k < 4; ++k)
    if (k < q.nbk && row0 >= q.row0[k] && row0 < q.row1[k]) Wb = lpart ? q.L[k] : q.W[k];
  const int ct = lpart ? ntile - nbeta : ntile;
  const float* __restrict__ W = Wb + (size_t)ct * NC * KD;
  const float* __restrict__ D = q.D;

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int l16 = lane & 15, grp = lane >> 4;

  // global -> register staging of one K chunk: A TM*KC/4 float4, B NC*KC/4 float4 (the
  // last B round is partial); kept in named registers (an indexed array ends in scratch)
  constexpr int A_F4 = TM * KC / 4;
  constexpr int B_F4 = NC * KC / 4;
  static_assert(A_F4 == NTQ, "one A float4 per thread");
  static_assert(B_F4 > 4 * NTQ && B_F4 <= 5 * NTQ, "four full B rounds and a partial one");
  float4 ra, rb0, rb1, rb2, rb3, rb4;
  const bool b4 = t + 4 * NTQ < B_F4;
  auto bsrc = [&](int u, int k0) {
    const int idx = t + u * NTQ;
    return reinterpret_cast<const float4*>(W + (size_t)(idx >> 2) * KD + k0 + (idx & 3) * 4);
  };
  auto bdst = [&](int u, int buf) {
    const int idx = t + u * NTQ;
    return reinterpret_cast<float4*>(&Bs[buf][(idx >> 2) * LDSW + (idx & 3) * 4]);
  };
#define QF_GLOAD(chunk)                                                                       \
  do {                                                                                        \
    const int k0_ = (chunk) * KC;                                                             \
    ra = *reinterpret_cast<const float4*>(D + (size_t)(row0 + (t >> 2)) * KD + k0_ + (t & 3) * 4); \
    rb0 = *bsrc(0, k0_);                                                                      \
    rb1 = *bsrc(1, k0_);                                                                      \
    rb2 = *bsrc(2, k0_);                                                                      \
    rb3 = *bsrc(3, k0_);                                                                      \
    if (b4) rb4 = *bsrc(4, k0_);                                                              \
  } while (0)

#define QF_LSTORE(buf)                                                                        \
  do {                                                                                        \
    *reinterpret_cast<float4*>(&As[buf][(t >> 2) * LDSW + (t & 3) * 4]) = ra;                 \
    *bdst(0, buf) = rb0;                                                                      \
    *bdst(1, buf) = rb1;                                                                      \
    *bdst(2, buf) = rb2;                                                                      \
    *bdst(3, buf) = rb3;                                                                      \
    if (b4) *bdst(4, buf) = rb4;                                                              \
  } while (0)

  f4 acc[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  // with W = L (row n of W = column n of L, zero for k < n) the chunks k < first column vanish
  const int c0 = lpart ? (ct * NC) / KC : 0;
  QF_GLOAD(c0);
  QF_LSTORE(c0 & 1);
  __syncthreads();
  // the main loop once without the triangular skip (beta tiles) and once with it (L tiles),
  // so that the beta tiles' MFMAs carry no per-block test
  auto main_loop = [&](auto lp) {
  constexpr bool LP = decltype(lp)::value;
  for (int c = c0; c < NCHUNK; ++c) {
    const int buf = c & 1;
    if (c + 1 < NCHUNK) QF_GLOAD(c + 1);
    float4 a[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
      a[i] = *reinterpret_cast<const float4*>(&As[buf][(wave * RB * 16 + i * 16 + l16) * LDSW + 4 * grp]);
    // B fragments in groups of four column blocks, each group used for all four k-steps
    // (consecutive MFMAs still write different accumulators), so only a group is live
#pragma unroll
    for (int j0 = 0; j0 < CB; j0 += 4) {
      float4 bg[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (j0 + u < CB) bg[u] = *reinterpret_cast<const float4*>(&Bs[buf][((j0 + u) * 16 + l16) * LDSW + 4 * grp]);
#define QF_STEP(C)                                                                              \
  _Pragma("unroll") for (int u = 0; u < 4; ++u) {                                              \
    const int j = j0 + u;                                                                      \
    if (j >= CB || (LP && c < ct * CB + j)) continue;                                          \
    _Pragma("unroll") for (int i = 0; i < RB; ++i)                                             \
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].C, bg[u].C, acc[i][j], 0, 0, 0);   \
  }
      QF_STEP(x)
      QF_STEP(y)
      QF_STEP(z)
      QF_STEP(w)
#undef QF_STEP
    }
    if (c + 1 < NCHUNK) QF_LSTORE(buf ^ 1);
    __syncthreads();
  }
  };
  if (lpart) main_loop(std::true_type{});
  else main_loop(std::false_type{});

  // ---- epilogue: lane holds Y[row = 4*grp + r][col = 16*j + l16] of each block ----
  // A tile lies wholly in the beta part or wholly in the Sigma / L part (272 divides 544).
  // The D values of a row dot are loaded together before they are used (no test between a
  // load and its use); the factor's part needs none (a sum of squares).
  const bool has_e = q.mode & 1;
  const int col_base = ntile * NC;
  const bool beta_tile = has_e && col_base < KD;
  const bool squares = !beta_tile && q.sumsq;
  const int kbase = beta_tile ? col_base : col_base - (has_e ? KD : 0);   // the tile's first column of D
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    float ps[4] = {0.f, 0.f, 0.f, 0.f};
    if (squares) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < CB; ++j) ps[r] += acc[i][j][r] * acc[i][j][r];
    } else {
      float dv[4][CB];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float* drow = D + (size_t)(row0 + wave * RB * 16 + i * 16 + 4 * grp + r) * KD + kbase + l16;
#pragma unroll
        for (int j = 0; j < CB; ++j) dv[r][j] = drow[j * 16];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < CB; ++j) ps[r] += acc[i][j][r] * dv[r][j];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) ps[r] = sum16(ps[r]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = row0 + wave * RB * 16 + i * 16 + 4 * grp + r;
      if (l16 == 0) q.P[(size_t)row * 4 + ntile] = ps[r];
      if (beta_tile) {
        float* yrow = q.Y + (size_t)row * KD;
#pragma unroll
        for (int j = 0; j < CB; ++j) yrow[col_base + j * 16 + l16] = acc[i][j][r];
      }
    }
  }
}

#undef QF_GLOAD
#undef QF_LSTORE

// Finish the split path (544-wide rows): sum the partial row-dots, form g.
__global__ __launch_bounds__(256) void k_qform_finish(int rows, int mode, int ntiles,
                                                      const float* __restrict__ D,
                                                      const float* __restrict__ Y,
                                                      const float* __restrict__ P,
                                                      const int* __restrict__ aor, int n_given,
                                                      const float* __restrict__ nrm,
                                                      float* __restrict__ G,
                                                      float* __restrict__ e_int,
                                                      float* __restrict__ v_int,
                                                      float* __restrict__ e_row,
                                                      float* __restrict__ v_row) {
  // one wave per row
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= rows) return;
  const int atom = aor ? aor[row] : (row < n_given ? row : -1);   // no table: given vectors
  if (atom < 0) return;
  const float* p = P + (size_t)row * 4;
  const bool has_e = mode & 1, has_v = mode & 2;
  const int half = ntiles / ((has_e && has_v) ? 2 : 1);
  float e = 0.f, v = 0.f;
  if (has_e) {
    for (int k = 0; k < half; ++k) e += p[k];
  }
  if (has_v) {
    const int first = has_e ? half : 0;
    for (int k = first; k < first + half; ++k) v += p[k];
  }
  if (lane == 0) {
    if (has_e) e_int[atom] = e, e_row[row] = e;
    if (has_v) v_int[atom] = v, v_row[row] = v;
  }
  if (!has_e) return;
  const float nv = nrm[atom];
  const float s2 = nv > 0.f ? 2.f / nv : 0.f;
  const float* d = D + (size_t)row * ND;
  const float* y = Y + (size_t)row * ND;
  float* g = G + (size_t)row * ND;
  for (int k = lane; k < ND; k += 64) g[k] = s2 * (y[k] - e * d[k]);
}

// Variance of the mixed rows in the split forms, in FP64: V_i = |L_s^T d_i|^2 with the FP64
// Cholesky factor of Sigma_s on v_mfma_f64_16x16x4_f64 (exact products of the FP32 row and
// the FP64 factor, FP64 sums), so the near-cancelling d^T Sigma d keeps FP64 accuracy in the
// form. A wave owns 32 rows (two 16-row blocks, which share every B fragment) and a group of
// four column blocks of Z = D L: for every K chunk from the group's first block (L[k][n] = 0
// for k < n) lane (m, q) supplies D[row m][16 kc + 4 q + t] and the fragments
// L[16 kc + 4 q + t][16 cb + m] (fragment order [cb][kc][t][lane]); eight independent
// accumulators per k-step, and the next chunk's fragments load while this one runs.
// Accumulator r of lane (n, q) holds row q + 4 r of the block (the FP64 instruction's
// layout). The group's sum of squares per row goes to P64[row][group]; k_var544_finish adds
// the groups in a fixed order.
constexpr int XCB = ND / 16;                 // 34 column blocks
constexpr int XG = 4;                        // column blocks per wave
constexpr int NXG = (XCB + XG - 1) / XG;     // 9 groups
typedef double d4 __attribute__((ext_vector_type(4)));

struct VarArgs {
  const float* D;          // [rows][544]
  int rows;                // padded rows (a multiple of 64)
  int split_row;           // rows >= split_row belong to the second bucket (Pt centre)
  const double* L[2];      // per bucket: fragments of the factor
  double* P64;             // [rows][NXG]
};

// One column group g of one 32-row block.
__device__ __forceinline__ void var544_group(const VarArgs& q, int row0, int g, int lane) {
  const int l16 = lane & 15, grp = lane >> 4;
  // the split between the two buckets falls on a 128-row boundary: one factor per block
  const double* __restrict__ L = (row0 >= q.split_row ? q.L[1] : q.L[0]) + lane;
  const float* __restrict__ d0 = q.D + (size_t)(row0 + l16) * ND + 4 * grp;
  const float* __restrict__ d1 = d0 + (size_t)16 * ND;
  d4 acc[2][XG];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int u = 0; u < XG; ++u) acc[i][u] = d4{0.0, 0.0, 0.0, 0.0};
  const int cb0 = g * XG;
  auto load_b = [&](int kc, double (&b)[XG][4]) {
#pragma unroll
    for (int u = 0; u < XG; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        b[u][t] = (cb0 + u < XCB && cb0 + u <= kc) ? L[(((size_t)(cb0 + u) * XCB + kc) * 4 + t) * 64] : 0.0;
  };
  double bA[XG][4], bB[XG][4];
  load_b(cb0, bA);
  for (int kc = cb0; kc < XCB; kc += 2) {
    // two chunks per trip, one B buffer each; the next one's loads ahead of the MFMAs
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int k = kc + half;
      if (k >= XCB) break;
      double (&cur)[XG][4] = half ? bB : bA;
      double (&nxt)[XG][4] = half ? bA : bB;
      if (k + 1 < XCB) load_b(k + 1, nxt);
      const float4 a0 = *reinterpret_cast<const float4*>(d0 + k * 16);
      const float4 a1 = *reinterpret_cast<const float4*>(d1 + k * 16);
      const double av[2][4] = {{a0.x, a0.y, a0.z, a0.w}, {a1.x, a1.y, a1.z, a1.w}};
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < XG; ++u)
#pragma unroll
          for (int i = 0; i < 2; ++i)
            acc[i][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][t], cur[u][t], acc[i][u], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double ss = 0.0;
#pragma unroll
      for (int u = 0; u < XG; ++u) ss = fma(acc[i][u][r], acc[i][u][r], ss);
      ss = sum16d(ss);
      if (l16 == 0) q.P64[(size_t)(row0 + 16 * i + grp + 4 * r) * NXG + g] = ss;
    }
}

// Group g of a row block runs 34 - 4 g chunks, so groups g and 8 - g together run 36: the
// first four tasks of every 32-row block are such pairs, the fifth the middle group alone
// (18 chunks). Tasks go out longest first (all pairs, then the middle groups), so the
// short ones fill in at the end.
__global__ __launch_bounds__(256) void k_var544_f64(VarArgs q) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int task = blockIdx.x * 4 + wave;
  const int nrb = q.rows / 32;
  if (task < 4 * nrb) {
    const int pr = task / nrb, rb = task % nrb;
    var544_group(q, rb * 32, pr, lane);
    var544_group(q, rb * 32, NXG - 1 - pr, lane);
  } else if (task < 5 * nrb) {
    var544_group(q, (task - 4 * nrb) * 32, NXG / 2, lane);
  }
}

// V of each mixed row from its group sums (fixed order), rounded to FP32 once.
__global__ __launch_bounds__(256) void k_var544_finish(int rows, const double* __restrict__ P64,
                                                       const int* __restrict__ aor, int n_given,
                                                       float* __restrict__ v_int, float* __restrict__ v_row) {
  const int row = blockIdx.x * 256 + threadIdx.x;
  if (row >= rows) return;
  const int atom = aor ? aor[row] : (row < n_given ? row : -1);
  if (atom < 0) return;
  double v = 0.0;
#pragma unroll
  for (int g = 0; g < NXG; ++g) v += P64[(size_t)row * NXG + g];
  v_int[atom] = (float)v;
  v_row[row] = (float)v;
}

void var544_f64(flare_state* s, const float* D, int rows, int split_row, const int* aor, int n_given,
                float* v_int, float* v_row) {
  VarArgs q{};
  q.D = D;
  q.rows = rows;
  q.split_row = split_row;
  q.L[0] = s->model->Lx64[0];
  q.L[1] = s->model->Lx64[1];
  q.P64 = s->Px64;
  const int tasks = rows / 32 * 5;      // per 32-row block: four pairs of groups and the middle group
  k_var544_f64<<<(tasks + 3) / 4, 256, 0, s->stream>>>(q);
  k_var544_finish<<<(rows + 255) / 256, 256, 0, s->stream>>>(rows, s->Px64, aor, n_given, v_int, v_row);
}

}  // namespace

// Quadratic forms of the mixed-environment rows [r0, r0 + nr) (544-wide, one chunk of the
// workspace: Dx row r - r0), split over four column tiles. In the split forms the variance
// runs in FP64 (var544_f64) and the tiles cover beta only.
void forms_mixed_chunk(flare_state* s, int r0, int nr, bool want_e, bool want_v) {
  if ((!want_e && !want_v) || nr == 0) return;
  StageTimer tm(s, FLARE_T_QFORMX);
  const flare_model* m = s->model;
  const int* aor = s->atom_of_rowx + r0;
  float* e_row = s->e_row + s->rows1 + r0;
  float* v_row = s->v_row + s->rows1 + r0;
  if (want_v && m->var64) {
    var544_f64(s, s->Dx, nr, s->bucket_row0[5] - r0, aor, 0, s->v_int, v_row);
    want_v = false;
    if (!want_e) return;
  }
  const int mode = (want_e ? 1 : 0) | (want_v ? 2 : 0);
  QArgs q{};
  q.mode = mode;
  q.nbk = 2;
  for (int k = 0; k < 2; ++k) {
    const int bk = 4 + k;
    const int padded = (s->bucket_count[bk] + TILE_ROWS - 1) / TILE_ROWS * TILE_ROWS;
    q.row0[k] = s->bucket_row0[bk] - r0;     // chunk-local rows
    q.row1[k] = s->bucket_row0[bk] + padded - r0;
    q.W[k] = m->Wx[k] + ((mode & 1) ? 0 : (size_t)ND * ND);
  }
  // with Cholesky factors the Sigma columns come from L (V = |d L|^2)
  q.sumsq = m->vchol ? 1 : 0;
  for (int k = 0; k < 2; ++k) q.L[k] = m->Lx[k];
  q.D = s->Dx;
  q.aor = aor;
  q.Y = s->Yx;
  q.P = s->Px;
  const int parts = ((mode & 1) ? 1 : 0) + ((mode & 2) ? 1 : 0);
  const int ntiles = 2 * parts;   // 272 columns per tile
  k_qform<ND, 17, 1><<<dim3(nr / 64, ntiles), NTQ, 0, s->stream>>>(q);
  k_qform_finish<<<(nr + 3) / 4, 256, 0, s->stream>>>(nr, mode, ntiles, s->Dx, s->Yx, s->Px, aor, 0, s->nrm, s->Gx,
                                                      s->e_int, s->v_int, e_row, v_row);
}

// Quadratic forms of given 544-wide vectors (rows 0 .. n-1) with the model of mixed bucket
// `bucket` (4: H centre, 5: Pt centre): e_r = d_r^T beta_s d_r, v_r = d_r^T Sigma_s d_r, by
// the same kernels as the descriptor path. The vectors are copied into the state's padded
// row buffer Dx (zeros past n); scratch: Yx, Px, Px64, Gx, e_row, v_row, nrm.
int forms_given_544(flare_state* s, int bucket, int n, const float* d, float* e, float* v) {
  const flare_model* m = s->model;
  for (int c0 = 0; c0 < n; c0 += s->mix_cap) {
    const int nc = std::min(s->mix_cap, n - c0);
    const int rows = (nc + TILE_ROWS - 1) / TILE_ROWS * TILE_ROWS;
    hipError_t err = hipMemcpyAsync(s->Dx, d + (size_t)c0 * ND, (size_t)nc * ND * sizeof(float),
                                    hipMemcpyDeviceToDevice, s->stream);
    if (err == hipSuccess && rows > nc)
      err = hipMemsetAsync(s->Dx + (size_t)nc * ND, 0, (size_t)(rows - nc) * ND * sizeof(float), s->stream);
    if (err != hipSuccess) return (int)err;
    // every row of the chunk has the model of `bucket`: the Pt-centre factor from row 0 for
    // bucket 5, the H-centre one throughout for bucket 4
    const int split = bucket == 5 ? 0 : rows;
    QArgs q{};
    q.nbk = 1;
    q.row0[0] = 0;
    q.row1[0] = rows;
    q.W[0] = m->Wx[bucket - 4];
    q.L[0] = m->Lx[bucket - 4];
    q.sumsq = m->vchol ? 1 : 0;
    q.D = s->Dx;
    q.aor = nullptr;
    q.Y = s->Yx;
    q.P = s->Px;
    int mode = 3;
    if (m->var64) {
      var544_f64(s, s->Dx, rows, split, nullptr, nc, v + c0, s->v_row);
      mode = 1;
    }
    q.mode = mode;
    const int ntiles = 2 * (mode == 3 ? 2 : 1);
    k_qform<ND, 17, 1><<<dim3(rows / 64, ntiles), NTQ, 0, s->stream>>>(q);
    k_qform_finish<<<(rows + 3) / 4, 256, 0, s->stream>>>(rows, mode, ntiles, s->Dx, s->Yx, s->Px, nullptr, nc,
                                                          s->nrm, s->Gx, e + c0, v + c0, s->e_row, s->v_row);
  }
  return 0;
}

}  // namespace flare
