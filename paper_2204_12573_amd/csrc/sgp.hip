// Mapped model from a sparse set (paper, Section V.B, Eqs. 1-2: the exact mapping of the
// sparse GP onto the quadratic forms).
//
// With the normalised inner-product kernel k_xi(d1, d2) = sigma^2 (d1 . d2)^xi, one sparse
// set S_s of normalised descriptors D_s [n_s][n_d] and weights alpha_s per central species:
//   mean (xi = 2)      e(d) = sum_t sigma^2 (d . d_t)^2 alpha_t = d^T beta_s d,
//                      beta_s = sigma^2 D_s^T diag(alpha_s) D_s;
//   variance (xi = 1)  V(d) = sigma^2 d . d - sigma^4 k^T K^-1 k,  k_t = d . d_t,
//                      K = sigma^2 D_s D_s^T + noise I  (the sparse-set kernel matrix),
//                      = d^T gamma_s d,  gamma_s = sigma^2 I - sigma^4 D_s^T K^-1 D_s.
// gamma_s is formed as sigma^2 I - sigma^4 Y^T Y with Y = C^-1 D_s and K = C C^T (Cholesky):
// no inverse is formed. Everything runs in FP64 on the device:
//   K      C = a A B^T + b I         (k_gemm_f64<NT>)
//   C      one column per launch    (k_chol_col), kept transposed (U = C^T, row-major), so
//                                    that the threads of a column read consecutive addresses
//   Y      forward substitution     (k_trsm_cols, one thread per descriptor component)
//   beta   a A^T diag(w) B          (k_gemm_f64<TN>)
//   gamma  a Y^T Y + b I            (k_gemm_f64<TN>)
// The model is then created from beta_s and gamma_s as by flare_model_create.
#include <algorithm>
#include <cmath>
#include <vector>

#include "state.h"

namespace flare {
namespace {

constexpr int GT = 16;   // output tile side of the FP64 product kernel

// C[m][n] = a * sum_k A(m, k) w_k B(n, k) + (m == n ? b : 0) for m < M, n < N, with
//   TN = true:  A(m, k) = A[k * lda + m], B(n, k) = B[k * ldb + n]   (C = a A^T diag(w) B)
//   TN = false: A(m, k) = A[m * lda + k], B(n, k) = B[n * ldb + k]   (C = a A B^T)
// w may be null (all ones). 16 x 16 tiles staged through LDS, K in steps of 16; each
// product is summed in increasing k, so C[m][n] and C[n][m] of A == B are bitwise equal.
template <bool TN>
__global__ __launch_bounds__(GT * GT) void k_gemm_f64(int M, int N, int K, double a, const double* __restrict__ A,
                                                     int lda, const double* __restrict__ B, int ldb,
                                                     const double* __restrict__ w, double b, double* __restrict__ C,
                                                     int ldc) {
  __shared__ double As[GT][GT + 1], Bs[GT][GT + 1];   // [k][m], [k][n]
  const int tx = threadIdx.x % GT, ty = threadIdx.x / GT;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int m = m0 + ty, n = n0 + tx;
  double acc = 0.0;
  for (int k0 = 0; k0 < K; k0 += GT) {
    // thread (ty, tx) loads A(m0 + ., k0 + .) and B(n0 + ., k0 + .): in the TN layout the
    // row index runs along the contiguous axis, so tx walks m (or n) there
    {
      const int kk = TN ? ty : tx, mm = TN ? tx : ty;
      const int gk = k0 + kk, gm = m0 + mm, gn = n0 + mm;
      double av = 0.0, bv = 0.0;
      if (gk < K && gm < M) av = TN ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
      if (gk < K && gn < N) {
        bv = TN ? B[(size_t)gk * ldb + gn] : B[(size_t)gn * ldb + gk];
        if (w) bv *= w[gk];
      }
      As[kk][mm] = av;
      Bs[kk][mm] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GT; ++kk) acc = fma(As[kk][ty], Bs[kk][tx], acc);
    __syncthreads();
  }
  if (m < M && n < N) C[(size_t)m * ldc + n] = a * acc + (m == n ? b : 0.0);
}

// Column j of the Cholesky factor of the n x n symmetric K (row-major), stored as row j of
// U = C^T (U[k][i] = C[i][k], k <= i). Columns 0 .. j-1 are done:
//   v_i = K[j][i] - sum_{k<j} U[k][i] U[k][j]   (i >= j),   U[j][j] = sqrt(v_j),
//   U[j][i] = v_i / U[j][j].
// Every work-group forms v_j itself (a block reduction), then its own range of i. A pivot
// that is not positive sets *bad.
constexpr int CT = 256;
__global__ __launch_bounds__(CT) void k_chol_col(int n, int j, const double* __restrict__ K, double* __restrict__ U,
                                                int* __restrict__ bad) {
  __shared__ double red[CT];
  double s = 0.0;
  for (int k = threadIdx.x; k < j; k += CT) {
    const double u = U[(size_t)k * n + j];
    s = fma(u, u, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = CT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double vj = K[(size_t)j * n + j] - red[0];
  if (!(vj > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *bad = 1;
    return;
  }
  const double piv = sqrt(vj);
  const int i = j + blockIdx.x * CT + threadIdx.x;
  if (i >= n) return;
  if (i == j) {
    U[(size_t)j * n + j] = piv;
    return;
  }
  double v = K[(size_t)j * n + i];
  for (int k = 0; k < j; ++k) v = fma(-U[(size_t)k * n + i], U[(size_t)k * n + j], v);
  U[(size_t)j * n + i] = v / piv;
}

// Y = C^-1 D by forward substitution, C = U^T lower-triangular n x n, D and Y [n][m]:
//   Y[i][c] = (D[i][c] - sum_{k<i} C[i][k] Y[k][c]) / C[i][i],  C[i][k] = U[k][i].
// One thread per column c (the columns are independent).
__global__ __launch_bounds__(256) void k_trsm_cols(int n, int m, const double* __restrict__ U,
                                                  const double* __restrict__ D, double* __restrict__ Y) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= m) return;
  for (int i = 0; i < n; ++i) {
    double v = D[(size_t)i * m + c];
    for (int k = 0; k < i; ++k) v = fma(-U[(size_t)k * n + i], Y[(size_t)k * m + c], v);
    Y[(size_t)i * m + c] = v / U[(size_t)i * n + i];
  }
}

template <bool TN>
void gemm_f64(int M, int N, int K, double a, const double* A, int lda, const double* B, int ldb, const double* w,
              double b, double* C, int ldc) {
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  k_gemm_f64<TN><<<grid, GT * GT>>>(M, N, K, a, A, lda, B, ldb, w, b, C, ldc);
}

struct DevScratch {
  std::vector<void*> p;
  ~DevScratch() {
    for (void* q : p) (void)hipFree(q);
  }
  hipError_t alloc(double** out, size_t count) {
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(double));
    if (e == hipSuccess) p.push_back(q);
    *out = static_cast<double*>(q);
    return e;
  }
};

}  // namespace
}  // namespace flare

using namespace flare;

#define SCHK(call)                                                       \
  do {                                                                   \
    hipError_t e_ = (call);                                              \
    if (e_ != hipSuccess) {                                              \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));      \
      return e_ == hipErrorOutOfMemory ? FLARE_E_OOM : FLARE_E_HIP;      \
    }                                                                    \
  } while (0)

extern "C" int flare_model_from_sparse_set(flare_model** out, int n_species, int n_rad, int l_max, double r_cut,
                                           const int32_t* n_sparse_host, const double* d_sparse,
                                           const double* alpha, double signal_var, double noise, int precision,
                                           double* beta_out, double* gamma_out) {
  if (!out || !n_sparse_host) {
    set_error("null pointer");
    return FLARE_E_ARG;
  }
  *out = nullptr;
  if (n_species != NS || n_rad != NR || l_max != LMAX) {
    set_error("this build has kernels for n_species=2, n_rad=8, l_max=3 only");
    return FLARE_E_UNSUPPORTED;
  }
  if (!(std::isfinite(signal_var) && signal_var > 0.0) || !(std::isfinite(noise) && noise >= 0.0)) {
    set_error("signal variance must be positive and the noise non-negative");
    return FLARE_E_ARG;
  }
  long long total = 0;
  for (int s = 0; s < NS; ++s) {
    if (n_sparse_host[s] < 0) {
      set_error("negative sparse-set size");
      return FLARE_E_ARG;
    }
    total += n_sparse_host[s];
  }
  if (total > 0 && (!d_sparse || !alpha)) {
    set_error("null sparse-set array");
    return FLARE_E_ARG;
  }
  int nmax = 0;
  for (int s = 0; s < NS; ++s) nmax = std::max(nmax, (int)n_sparse_host[s]);
  DevScratch tmp;
  double *beta = nullptr, *gamma = nullptr, *Kd = nullptr, *U = nullptr, *Y = nullptr;
  int* bad = nullptr;
  const size_t mm = (size_t)ND * ND;
  SCHK(tmp.alloc(&beta, NS * mm));
  SCHK(tmp.alloc(&gamma, NS * mm));
  SCHK(tmp.alloc(&Kd, (size_t)nmax * nmax));
  SCHK(tmp.alloc(&U, (size_t)nmax * nmax));
  SCHK(tmp.alloc(&Y, (size_t)nmax * ND));
  double* badd = nullptr;
  SCHK(tmp.alloc(&badd, 1));
  bad = reinterpret_cast<int*>(badd);
  const double s2 = signal_var, s4 = signal_var * signal_var;
  long long first = 0;
  for (int s = 0; s < NS; ++s) {
    const int ns = n_sparse_host[s];
    const double* Ds = d_sparse + (size_t)first * ND;
    double* bs = beta + s * mm;
    double* gs = gamma + s * mm;
    if (ns == 0) {
      // no sparse environments of this species: zero mean, the prior variance sigma^2 |d|^2
      gemm_f64<true>(ND, ND, 0, 0.0, nullptr, ND, nullptr, ND, nullptr, 0.0, bs, ND);
      gemm_f64<true>(ND, ND, 0, 0.0, nullptr, ND, nullptr, ND, nullptr, s2, gs, ND);
      continue;
    }
    // beta_s = sigma^2 D^T diag(alpha) D
    gemm_f64<true>(ND, ND, ns, s2, Ds, ND, Ds, ND, alpha + first, 0.0, bs, ND);
    // K = sigma^2 D D^T + noise I, its Cholesky factor, Y = C^-1 D
    gemm_f64<false>(ns, ns, ND, s2, Ds, ND, Ds, ND, nullptr, noise, Kd, ns);
    SCHK(hipMemset(U, 0, (size_t)ns * ns * sizeof(double)));
    SCHK(hipMemset(bad, 0, sizeof(int)));
    for (int j = 0; j < ns; ++j) k_chol_col<<<(ns - j + CT - 1) / CT, CT>>>(ns, j, Kd, U, bad);
    int h_bad = 0;
    SCHK(hipMemcpy(&h_bad, bad, sizeof(int), hipMemcpyDeviceToHost));
    if (h_bad) {
      set_error("sparse-set kernel matrix sigma^2 D D^T + noise I is not positive definite (species " +
                std::to_string(s) + ")");
      return FLARE_E_ARG;
    }
    k_trsm_cols<<<(ND + 255) / 256, 256>>>(ns, ND, U, Ds, Y);
    // gamma_s = sigma^2 I - sigma^4 Y^T Y
    gemm_f64<true>(ND, ND, ns, -s4, Y, ND, Y, ND, nullptr, s2, gs, ND);
    first += ns;
  }
  SCHK(hipGetLastError());
  std::vector<double> hb(NS * mm), hg(NS * mm);
  SCHK(hipMemcpy(hb.data(), beta, NS * mm * sizeof(double), hipMemcpyDeviceToHost));
  SCHK(hipMemcpy(hg.data(), gamma, NS * mm * sizeof(double), hipMemcpyDeviceToHost));
  // gamma is symmetric bit for bit (its products commute); beta's weighted products are
  // rounded in a different order on the two sides of the diagonal: take the mean of the two
  for (int s = 0; s < NS; ++s)
    for (int r = 0; r < ND; ++r)
      for (int c = r + 1; c < ND; ++c) {
        double& x = hb[s * mm + (size_t)r * ND + c];
        double& y = hb[s * mm + (size_t)c * ND + r];
        x = y = 0.5 * (x + y);
      }
  if (beta_out) SCHK(hipMemcpy(beta_out, hb.data(), NS * mm * sizeof(double), hipMemcpyHostToDevice));
  if (gamma_out) SCHK(hipMemcpy(gamma_out, gamma, NS * mm * sizeof(double), hipMemcpyDeviceToDevice));
  return flare_model_create(out, n_species, n_rad, l_max, r_cut, hb.data(), hg.data(), precision);
}
