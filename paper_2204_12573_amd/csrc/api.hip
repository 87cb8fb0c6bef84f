// C ABI: model and state objects, argument checks, call sequencing.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "state.h"

namespace flare {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

SlotView slot_view(const flare_state* s) {
  SlotView v;
  v.geom = s->geom;
  v.slice_base = s->slice_base;
  v.rev = s->slot_rev;
  v.w_in = s->w_in;
  v.rc = (float)s->model->r_cut;
  return v;
}

namespace {
hipEvent_t take_event(flare_state* s) {
  if (!s->timers.pool.empty()) {
    hipEvent_t e = s->timers.pool.back();
    s->timers.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

StageTimer::StageTimer(flare_state* st, int stg) : s(st), stage(stg) {
  if (!s->timers.on) return;
  hipEvent_t start = take_event(s);
  stop = take_event(s);
  if (!start || !stop) {
    stop = nullptr;
    return;
  }
  (void)hipEventRecord(start, s->stream);
  s->timers.pending.push_back({stage, {start, stop}});
}

StageTimer::~StageTimer() {
  if (stop) (void)hipEventRecord(stop, s->stream);
}

}  // namespace flare

using namespace flare;

#define CHK(call)                                                        \
  do {                                                                   \
    hipError_t e_ = (call);                                              \
    if (e_ != hipSuccess) {                                              \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));      \
      return e_ == hipErrorOutOfMemory ? FLARE_E_OOM : FLARE_E_HIP;      \
    }                                                                    \
  } while (0)

#define ARG(cond, msg)          \
  do {                          \
    if (!(cond)) {              \
      set_error(msg);           \
      return FLARE_E_ARG;       \
    }                           \
  } while (0)

namespace {

// FP32 -> BF16, round to nearest even (finite inputs)
uint16_t bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float bf16_to_f32(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}

// Cholesky factor (lower) of a symmetric positive definite n x n matrix, FP64, in place
// on a copy; returns false when a pivot is not positive.
bool cholesky(std::vector<double>& a, int n) {
  for (int j = 0; j < n; ++j) {
    double d = a[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= a[(size_t)j * n + k] * a[(size_t)j * n + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    a[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = a[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) v -= a[(size_t)i * n + k] * a[(size_t)j * n + k];
      a[(size_t)i * n + j] = v / d;
    }
    for (int k = j + 1; k < n; ++k) a[(size_t)j * n + k] = 0.0;
  }
  return true;
}

// sub-block [start, start+nb)^2 of an n_d x n_d FP64 matrix
std::vector<double> sub_block(const double* m, int start, int nb) {
  std::vector<double> out((size_t)nb * nb);
  for (int r = 0; r < nb; ++r)
    for (int c = 0; c < nb; ++c) out[(size_t)r * nb + c] = m[(size_t)(start + r) * ND + (start + c)];
  return out;
}

int upload(void** dst, const void* src, size_t bytes) {
  hipError_t e = hipMalloc(dst, bytes);
  if (e == hipSuccess) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    set_error(std::string("model upload: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? FLARE_E_OOM : FLARE_E_HIP;
  }
  return FLARE_OK;
}

// BF16 split fragments of one 144-block: B[k][n] = M[k][n], K padded to 160.
// Layout [ks 5][cb 9][hi/lo 2][lane 64][8].
void bf16_fragments(const std::vector<double>& M, uint16_t* out /* [5][9][2][64][8] */) {
  const int nks = 5, ncb = ND1 / 16;
  for (int ks = 0; ks < nks; ++ks)
    for (int cb = 0; cb < ncb; ++cb)
      for (int lane = 0; lane < 64; ++lane)
        for (int t = 0; t < 8; ++t) {
          const int k = ks * 32 + 8 * (lane / 16) + t, n = cb * 16 + lane % 16;
          const float v = k < ND1 ? (float)M[(size_t)k * ND1 + n] : 0.f;
          const uint16_t hi = bf16_rne(v);
          const uint16_t lo = bf16_rne(v - bf16_to_f32(hi));
          const size_t base = ((((size_t)ks * ncb + cb) * 2) * 64 + lane) * 8 + t;
          out[base] = hi;
          out[base + 64 * 8] = lo;
        }
}

// Three-way BF16 fragments of one 144-block: B[k][n] = M[k][n] rounded to FP32, then
// x0 = bf16(x), x1 = bf16(x - x0), x2 = bf16(x - x0 - x1) (both remainders exact in FP32).
// Layout [ks 5][cb 9][part 3][lane 64][8], K padded to 160 with zeros.
void bf16x3_fragments(const std::vector<double>& M, uint16_t* out /* [5][9][3][64][8] */) {
  const int nks = 5, ncb = ND1 / 16;
  for (int ks = 0; ks < nks; ++ks)
    for (int cb = 0; cb < ncb; ++cb)
      for (int lane = 0; lane < 64; ++lane)
        for (int t = 0; t < 8; ++t) {
          const int k = ks * 32 + 8 * (lane / 16) + t, n = cb * 16 + lane % 16;
          const float v = k < ND1 ? (float)M[(size_t)k * ND1 + n] : 0.f;
          const uint16_t x0 = bf16_rne(v);
          const float r1 = v - bf16_to_f32(x0);
          const uint16_t x1 = bf16_rne(r1);
          const uint16_t x2 = bf16_rne(r1 - bf16_to_f32(x1));
          const size_t base = ((((size_t)ks * ncb + cb) * 3) * 64 + lane) * 8 + t;
          out[base] = x0;
          out[base + 64 * 8] = x1;
          out[base + 2 * 64 * 8] = x2;
        }
}

// FP32 fragments of an n x n matrix M (row-major, leading dimension ld) for
// v_mfma_f32_16x16x4_f32 B operands: [K chunk n/16][column block n/16][lane 64][t 4],
// element M[16 kc + 4 (lane / 16) + t][16 cb + lane % 16].
std::vector<float> f32_fragments(const double* M, int ld, int n) {
  const int nc = n / 16;
  std::vector<float> f((size_t)nc * nc * 64 * 4);
  for (int kc = 0; kc < nc; ++kc)
    for (int cb = 0; cb < nc; ++cb)
      for (int lane = 0; lane < 64; ++lane)
        for (int t = 0; t < 4; ++t)
          f[(((size_t)kc * nc + cb) * 64 + lane) * 4 + t] =
              (float)M[(size_t)(kc * 16 + 4 * (lane / 16) + t) * ld + cb * 16 + lane % 16];
  return f;
}

// FP64 fragments of an n x n lower-triangular factor L (row-major) for
// v_mfma_f64_16x16x4_f64 B operands: [cb][kc][t 4][lane 64], element
// L[16 kc + 4 (lane / 16) + t][16 cb + lane % 16] (blocks with kc < cb are zero).
std::vector<double> f64_fragments(const std::vector<double>& L, int n) {
  const int nb = n / 16;
  std::vector<double> f((size_t)nb * nb * 4 * 64);
  for (int cb = 0; cb < nb; ++cb)
    for (int kc = 0; kc < nb; ++kc)
      for (int t = 0; t < 4; ++t)
        for (int lane = 0; lane < 64; ++lane)
          f[(((size_t)cb * nb + kc) * 4 + t) * 64 + lane] =
              L[(size_t)(kc * 16 + 4 * (lane / 16) + t) * n + cb * 16 + lane % 16];
  return f;
}

}  // namespace

// Every device array of a state, with its size in bytes for the capacities of the state.
template <class F>
static void state_arrays(flare_state* s, F&& f) {
  const size_t n = (size_t)s->max_atoms, P = (size_t)s->max_pairs, R = (size_t)s->row_cap;
  const size_t SL = (size_t)s->slice_cap, SC = (size_t)s->slot_cap, BC = (size_t)s->bin_cap;
  const size_t NC = (size_t)s->cell_cap, TC = (size_t)s->task_cap, X = (size_t)s->mix_cap;
  const size_t keys = (size_t)list_key_count() * s->nblk_cap + 1;
  const size_t scan_n = std::max({BC + 1, n + 1, keys, SL + 1});
  f((void**)&s->perm, n * 4);
  f((void**)&s->sp, n * 4);
  f((void**)&s->sid, n * 4);
  f((void**)&s->bin, n * 4);
  f((void**)&s->envmask, n * 4);
  f((void**)&s->bucket, n * 4);
  f((void**)&s->row_of, n * 4);
  f((void**)&s->nl_cnt, n * 4);
  f((void**)&s->nl_off, (n + 1) * 4);
  f((void**)&s->w, n * sizeof(double4));
  f((void**)&s->wf, n * sizeof(float4));
  f((void**)&s->off, 3 * n * 8);
  f((void**)&s->dlt, n * 16);
  f((void**)&s->xb, 3 * n * 8);
  f((void**)&s->inv_perm, n * 4);
  f((void**)&s->nrm, n * 4);
  f((void**)&s->e_int, n * 4);
  f((void**)&s->v_int, n * 4);
  f((void**)&s->crec, n * sizeof(CallerRec));
  f((void**)&s->sorted, n * 4);
  f((void**)&s->row_caller, (n + 1) * 4);
  f((void**)&s->slot0, n * 4);
  f((void**)&s->pair_cache, (size_t)list_pair_cache() * n * sizeof(int2));
  f((void**)&s->nl_j, P * 4);
  f((void**)&s->nl_s, P * 4);
  f((void**)&s->nl_rev, P * 4);
  f((void**)&s->d_grids, NC * sizeof(CellGrid));
  f((void**)&s->d_struct_off, (NC + 1) * 4);
  f((void**)&s->bin_count, (BC + 1) * 4);
  f((void**)&s->bin_start, (BC + 1) * 4);
  f((void**)&s->bin_fill, (BC + 1) * 4);
  f((void**)&s->blk_bucket, keys * 4);
  f((void**)&s->blk_bucket_scan, (keys + 1) * 4);
  f((void**)&s->scan_scratch, scan_scratch_ints((long long)scan_n) * 4);
  f((void**)&s->d_tasks, TC * sizeof(RedTask));
  f((void**)&s->d_first_task, (NC + 1) * 4);
  f((void**)&s->red_e, TC * 2 * 8);
  f((void**)&s->red_s, TC * 4);
  f((void**)&s->atom_of_row1, (R + 1) * 4);
  f((void**)&s->atom_of_rowx, (R + 1) * 4);
  f((void**)&s->cnt_row, R * 4);
  f((void**)&s->sid_row, R * 4);
  f((void**)&s->e_row, R * 4);
  f((void**)&s->v_row, R * 4);
  f((void**)&s->row_out, R * 16);
  f((void**)&s->f_own, R * 16);
  f((void**)&s->G1, R * ND1 * 4);
  f((void**)&s->Dx, X * ND * 4);
  f((void**)&s->Gx, X * ND * 4);
  f((void**)&s->Yx, X * ND * 4);
  f((void**)&s->Px, X * 4 * 4);
  f((void**)&s->Px64, X * 9 * 8);
  f((void**)&s->slice_len, (SL + 1) * 4);
  f((void**)&s->slice_base, (SL + 1) * 4);
  f((void**)&s->slot_atom, SC * 4);
  f((void**)&s->slot_j, SC * 4);
  f((void**)&s->slot_rev, SC * 4);
  f((void**)&s->slot_d0, SC * 16);
  f((void**)&s->geom, SC * 16);
  f((void**)&s->w_in, SC * 16);
  f((void**)&s->d_status, 64);
  f((void**)&s->d_layout, (size_t)list_layout_words() * 4 + 64);
}

extern "C" {

const char* flare_last_error(void) { return g_last_error.c_str(); }

const char* flare_strerror(int code) {
  switch (code) {
    case FLARE_OK: return "ok";
    case FLARE_E_ARG: return "invalid argument";
    case FLARE_E_SPECIES: return "species index out of range";
    case FLARE_E_BOX: return "invalid box";
    case FLARE_E_CAPACITY: return "capacity exceeded";
    case FLARE_E_NONFINITE: return "non-finite position";
    case FLARE_E_STALE: return "call order: missing neighbour list or descriptors";
    case FLARE_E_OOM: return "device out of memory";
    case FLARE_E_HIP: return "HIP runtime error";
    case FLARE_E_UNSUPPORTED: return "unsupported model size or precision";
    default: return "unknown status";
  }
}

int flare_model_create(flare_model** out, int n_species, int n_rad, int l_max, double r_cut,
                       const double* beta_host, const double* sigma_host, int precision) {
  ARG(out && beta_host && sigma_host, "null pointer");
  *out = nullptr;
  ARG(std::isfinite(r_cut) && r_cut > 0.0, "r_cut must be positive");
  if (n_species != NS || n_rad != NR || l_max != LMAX) {
    set_error("this build has kernels for n_species=2, n_rad=8, l_max=3 only");
    return FLARE_E_UNSUPPORTED;
  }
  const int flags = precision;
  precision &= ~FLARE_VAR_FP32;
  if ((precision != FLARE_FP32 && precision != FLARE_BF16_SPLIT && precision != FLARE_FP8_SPLIT &&
       precision != FLARE_BF16X6_SPLIT) || flags == (FLARE_FP32 | FLARE_VAR_FP32)) {
    set_error("precision must be FLARE_FP32, or FLARE_BF16_SPLIT, FLARE_FP8_SPLIT or FLARE_BF16X6_SPLIT "
              "(optionally | FLARE_VAR_FP32)");
    return FLARE_E_UNSUPPORTED;
  }
  flare_model* m = new (std::nothrow) flare_model();
  if (!m) return FLARE_E_OOM;
  m->precision = precision;
  m->flags = flags;
  m->var64 = precision != FLARE_FP32 && !(flags & FLARE_VAR_FP32);
  m->r_cut = r_cut;
  CHK(hipGetDevice(&m->device));
  // beta and Sigma of each single-species bucket's 144-wide block in fragment order
  for (int b = 0; b < 4; ++b) {
    const int sp = b & 1;                          // central species
    const int st = b < 2 ? 0 : ND - ND1;           // the block inside the packed 544 vector
    std::vector<float> f0 = f32_fragments(beta_host + (size_t)sp * ND * ND + (size_t)st * ND + st, ND, ND1);
    std::vector<float> f1 = f32_fragments(sigma_host + (size_t)sp * ND * ND + (size_t)st * ND + st, ND, ND1);
    f0.insert(f0.end(), f1.begin(), f1.end());
    const int rc = upload((void**)&m->Wf[b], f0.data(), f0.size() * sizeof(float));
    if (rc != FLARE_OK) {
      flare_model_destroy(m);
      return rc;
    }
  }
  // Cholesky factors of the Sigma blocks: V = |L^T d|^2, a sum of squares that does not
  // cancel, and the zero upper triangle of L skips 36 of the 81 16x16 blocks of the
  // 144-wide variance pass. The split forms need them; the FP32 form uses them when every
  // block is positive definite and keeps the full Sigma otherwise.
  const int nkc = ND1 / 16, ncb = ND1 / 16;
  std::vector<std::vector<double>> L1(4), Lx(NS);
  bool chol = true;
  for (int b = 0; b < 4 && chol; ++b) {
    const int s = b & 1;
    L1[b] = sub_block(sigma_host + (size_t)s * ND * ND, b < 2 ? 0 : ND - ND1, ND1);
    chol = cholesky(L1[b], ND1);
  }
  for (int s = 0; s < NS && chol; ++s) {
    Lx[s].assign(sigma_host + (size_t)s * ND * ND, sigma_host + (size_t)(s + 1) * ND * ND);
    chol = cholesky(Lx[s], ND);
  }
  if (!chol && precision != FLARE_FP32) {
    set_error("Sigma is not positive definite (needed by the split forms)");
    flare_model_destroy(m);
    return FLARE_E_ARG;
  }
  m->vchol = chol;
  if (chol) {
    for (int b = 0; b < 4; ++b) {
      // FP32 fragments of L replace the Sigma part (part 1) of Wf
      std::vector<float> f = f32_fragments(L1[b].data(), ND1, ND1);
      hipError_t e = hipMemcpy(m->Wf[b] + (size_t)nkc * ncb * 64 * 4, f.data(), f.size() * sizeof(float),
                               hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        set_error(std::string("model upload: ") + hipGetErrorString(e));
        flare_model_destroy(m);
        return FLARE_E_HIP;
      }
    }
  }
  // the mixed buckets: beta, Sigma (and L) of the central species over all 544 components,
  // row n of each stored part = column n of the matrix
  for (int sp = 0; sp < NS; ++sp) {
    const int parts = chol ? 3 : 2;
    std::vector<float> w((size_t)parts * ND * ND);
    for (int part = 0; part < parts; ++part) {
      const double* M = part == 0 ? beta_host + (size_t)sp * ND * ND
                                  : part == 1 ? sigma_host + (size_t)sp * ND * ND : Lx[sp].data();
      for (int n = 0; n < ND; ++n)
        for (int k = 0; k < ND; ++k) w[((size_t)part * ND + n) * ND + k] = (float)M[(size_t)k * ND + n];
    }
    int rc = upload((void**)&m->Wx[sp], w.data(), (size_t)2 * ND * ND * sizeof(float));
    if (rc == FLARE_OK && chol) rc = upload((void**)&m->Lx[sp], w.data() + (size_t)2 * ND * ND, (size_t)ND * ND * sizeof(float));
    if (rc != FLARE_OK) {
      flare_model_destroy(m);
      return rc;
    }
  }
  if (m->var64) {
    // FP64 fragments of the factors for the variance of the split forms
    for (int b = 0; b < 4; ++b) {
      std::vector<double> f = f64_fragments(L1[b], ND1);
      const int rc = upload((void**)&m->L64[b], f.data(), f.size() * sizeof(double));
      if (rc != FLARE_OK) {
        flare_model_destroy(m);
        return rc;
      }
    }
    for (int s = 0; s < NS; ++s) {
      std::vector<double> f = f64_fragments(Lx[s], ND);
      const int rc = upload((void**)&m->Lx64[s], f.data(), f.size() * sizeof(double));
      if (rc != FLARE_OK) {
        flare_model_destroy(m);
        return rc;
      }
    }
  }
  if (precision == FLARE_BF16X6_SPLIT) {
    for (int b = 0; b < 4; ++b) {
      const int s = b & 1;
      const int st = b < 2 ? 0 : ND - ND1;
      std::vector<double> beta = sub_block(beta_host + (size_t)s * ND * ND, st, ND1);
      std::vector<uint16_t> frag((size_t)5 * ncb * 3 * 64 * 8);
      bf16x3_fragments(beta, frag.data());
      const int rc = upload((void**)&m->W6[b], frag.data(), frag.size() * sizeof(uint16_t));
      if (rc != FLARE_OK) {
        flare_model_destroy(m);
        return rc;
      }
    }
  }
  if (precision == FLARE_BF16_SPLIT || precision == FLARE_FP8_SPLIT) {
    for (int b = 0; b < 4; ++b) {
      const int s = b & 1;
      const int st = b < 2 ? 0 : ND - ND1;
      std::vector<double> beta = sub_block(beta_host + (size_t)s * ND * ND, st, ND1);
      int rc = FLARE_OK;
      if (precision == FLARE_BF16_SPLIT) {
        const size_t per = (size_t)5 * ncb * 2 * 64 * 8;
        std::vector<uint16_t> frag(per);
        bf16_fragments(beta, frag.data());
        rc = upload((void**)&m->Wb[b], frag.data(), frag.size() * sizeof(uint16_t));
      } else {
        double mx = 0.0;
        for (double x : beta) mx = std::max(mx, std::fabs(x));
        int ex = 0;
        std::frexp(mx > 0.0 ? mx : 1.0, &ex);               // mx = f 2^ex, f in [0.5, 1)
        const float sb = std::ldexp(1.0f, 4 - ex);         // |sb beta| < 16
        m->beta_scale[b] = sb;
        std::vector<float> vals((size_t)5 * ncb * 64 * 8);
        for (int ks = 0; ks < 5; ++ks)
          for (int cb = 0; cb < ncb; ++cb)
            for (int lane = 0; lane < 64; ++lane)
              for (int t = 0; t < 8; ++t) {
                const int k = ks * 32 + 8 * (lane / 16) + t, n = cb * 16 + lane % 16;
                vals[(((size_t)ks * ncb + cb) * 64 + lane) * 8 + t] =
                    k < ND1 ? sb * (float)beta[(size_t)k * ND1 + n] : 0.f;
              }
        float* dvals = nullptr;
        rc = upload((void**)&dvals, vals.data(), vals.size() * sizeof(float));
        if (rc == FLARE_OK) {
          hipError_t e = hipMalloc((void**)&m->W8[b], (size_t)5 * ncb * 2 * 64 * sizeof(uint64_t));
          if (e == hipSuccess) {
            make_fp8_fragments(dvals, 5 * ncb, m->W8[b]);
            e = hipDeviceSynchronize();
          }
          (void)hipFree(dvals);
          if (e != hipSuccess) {
            set_error(std::string("fp8 model: ") + hipGetErrorString(e));
            rc = FLARE_E_HIP;
          }
        }
      }
      if (rc != FLARE_OK) {
        flare_model_destroy(m);
        return rc;
      }
    }
  }
  *out = m;
  return FLARE_OK;
}

int flare_model_info(const flare_model* m, int* precision, int* variance_cholesky) {
  ARG(m, "null model");
  if (precision) *precision = m->flags;
  if (variance_cholesky) *variance_cholesky = m->vchol ? 1 : 0;
  return FLARE_OK;
}

int flare_model_destroy(flare_model* m) {
  if (!m) return FLARE_OK;
  for (int b = 0; b < 4; ++b) {
    if (m->Wf[b]) (void)hipFree(m->Wf[b]);
    if (m->Wb[b]) (void)hipFree(m->Wb[b]);
    if (m->W8[b]) (void)hipFree(m->W8[b]);
    if (m->W6[b]) (void)hipFree(m->W6[b]);
    if (m->L64[b]) (void)hipFree(m->L64[b]);
  }
  for (int k = 0; k < 2; ++k) {
    if (m->Wx[k]) (void)hipFree(m->Wx[k]);
    if (m->Lx[k]) (void)hipFree(m->Lx[k]);
    if (m->Lx64[k]) (void)hipFree(m->Lx64[k]);
  }
  delete m;
  return FLARE_OK;
}

int flare_descriptor_dim(const flare_model* m, int* n_d) {
  ARG(m && n_d, "null pointer");
  *n_d = ND;
  return FLARE_OK;
}

static void free_state(flare_state* s) {
  state_arrays(s, [](void** p, size_t) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  });
  if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
  if (s->ev_join) (void)hipEventDestroy(s->ev_join);
  if (s->side) (void)hipStreamDestroy(s->side);
  if (s->h_info) (void)hipHostFree(s->h_info);
  if (s->h_stage) (void)hipHostFree(s->h_stage);
  s->red_w.release();
}

int flare_state_create(flare_state** out, const flare_model* model, int max_atoms,
                       long long max_pairs, void* stream) {
  ARG(out && model, "null pointer");
  *out = nullptr;
  ARG(max_atoms > 0 && max_pairs > 0, "capacities must be positive");
  ARG(max_pairs <= 0x7fffffffLL, "max_pairs must fit in int32");
  flare_state* s = new (std::nothrow) flare_state();
  if (!s) return FLARE_E_OOM;
  s->model = model;
  s->stream = (hipStream_t)stream;
  s->max_atoms = max_atoms;
  s->max_pairs = max_pairs;
  // capacities of everything a list build and a step can need (see flare.h)
  s->row_cap = (max_atoms + NBUCKET * TILE_ROWS + TILE_ROWS - 1) / TILE_ROWS * TILE_ROWS;
  s->slice_cap = s->row_cap / 32;
  s->slot_cap = (max_pairs + max_pairs / 4 + 32LL * 64 * NBUCKET + 31) / 32 * 32;
  s->bin_cap = (int)std::min<long long>(std::max<long long>(4LL * max_atoms, 1 << 16), 1LL << 30);
  s->cell_cap = max_atoms + 1;
  s->task_cap = s->cell_cap + max_atoms / 2048 + 1;
  s->nblk_cap = (max_atoms + 255) / 256;
  s->mix_cap = std::min(s->row_cap, MIX_ROWS);
  hipError_t e = hipGetDevice(&s->device);
  state_arrays(s, [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes ? bytes : 4);
    if (e == hipSuccess) s->fixed_bytes += (long long)(bytes ? bytes : 4);
  });
  s->h_stage_bytes = (size_t)s->cell_cap * sizeof(CellGrid) + 2 * ((size_t)s->cell_cap + 1) * sizeof(int) +
                     (size_t)s->task_cap * sizeof(RedTask) + 64;
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_info, 256, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_stage, s->h_stage_bytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemsetAsync(s->d_status, 0, 64, s->stream);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming);
  if (e != hipSuccess) {
    set_error(std::string("state allocation: ") + hipGetErrorString(e));
    free_state(s);
    delete s;
    return e == hipErrorOutOfMemory ? FLARE_E_OOM : FLARE_E_HIP;
  }
  *out = s;
  return FLARE_OK;
}

int flare_state_destroy(flare_state* s) {
  if (!s) return FLARE_OK;
  (void)hipStreamSynchronize(s->stream);
  for (auto& pe : s->timers.pending) {
    (void)hipEventDestroy(pe.second.first);
    (void)hipEventDestroy(pe.second.second);
  }
  for (hipEvent_t e : s->timers.pool) (void)hipEventDestroy(e);
  free_state(s);
  delete s;
  return FLARE_OK;
}

int flare_neighbors(flare_state* s, int n_atoms, const double* x, const double* y, const double* z,
                    const int32_t* species, int n_struct, const int32_t* struct_offsets_host,
                    const double* boxes_host, double skin) {
  ARG(s, "null state");
  s->have_list = false;
  s->have_desc = false;
  ARG(n_atoms >= 0, "n_atoms < 0");
  ARG(n_struct >= 1, "n_struct must be >= 1");
  ARG(struct_offsets_host && boxes_host, "null host array");
  ARG(n_atoms == 0 || (x && y && z && species), "null device array");
  ARG(std::isfinite(skin) && skin >= 0.0, "skin must be >= 0");
  if (n_atoms > s->max_atoms) {
    set_error("n_atoms exceeds max_atoms");
    return FLARE_E_CAPACITY;
  }
  ARG(struct_offsets_host[0] == 0 && struct_offsets_host[n_struct] == n_atoms,
      "struct offsets must start at 0 and end at n_atoms");
  for (int c = 0; c < n_struct; ++c)
    ARG(struct_offsets_host[c + 1] >= struct_offsets_host[c], "struct offsets must be non-decreasing");
  if (n_struct > s->cell_cap) {
    set_error("more cells than the state holds (max_atoms + 1)");
    return FLARE_E_CAPACITY;
  }
  const double rl = s->model->r_cut + skin;
  s->grids.resize(n_struct);
  s->struct_off.assign(struct_offsets_host, struct_offsets_host + n_struct + 1);
  for (int c = 0; c < n_struct; ++c)
    for (int ax = 0; ax < 3; ++ax) {
      const double L = boxes_host[3 * c + ax];
      if (!(std::isfinite(L) && L > 0.0)) {
        set_error("box side must be positive and finite");
        return FLARE_E_BOX;
      }
    }
  // bins at least r_list wide (with a relative margin far above rounding); when the cells
  // need more bins than the state holds, wider ones (a factor 2^(1/3) per try, so the
  // search visits more candidates but the list is the same)
  long long nbins = 0;
  for (double widen = 1.0;; widen *= 1.2599210498948732) {
    nbins = 0;
    for (int c = 0; c < n_struct; ++c) {
      CellGrid& g = s->grids[c];
      for (int ax = 0; ax < 3; ++ax) {
        const double L = boxes_host[3 * c + ax];
        long long nb = (long long)std::floor(L / (rl * widen * (1.0 + 1e-9)));
        nb = std::max(1LL, std::min(nb, 4096LL));
        const double h = L / (double)nb;
        g.L[ax] = L;
        g.nb[ax] = (int)nb;
        g.inv_h[ax] = (double)nb / L;
        g.K[ax] = (int)std::ceil(rl / h);
        if (g.K[ax] > 100) {
          set_error("box side too small for the list radius");
          return FLARE_E_BOX;
        }
      }
      g.bin_base = (int)nbins;
      g.atom_base = struct_offsets_host[c];
      nbins += (long long)g.nb[0] * g.nb[1] * g.nb[2];
    }
    if (nbins <= s->bin_cap) break;
    if (nbins <= n_struct) {        // one bin per cell already
      set_error("more cells than the state's bins");
      return FLARE_E_CAPACITY;
    }
  }
  s->n_atoms = n_atoms;
  s->n_struct = n_struct;
  s->n_bins = (int)nbins;
  s->skin = skin;
  s->r_list = rl;
  int rc;
  {
    StageTimer tm(s, FLARE_T_LIST);
    rc = build_list(s, x, y, z, species);
  }
  if (rc != FLARE_OK) return rc;
  s->have_list = true;
  return FLARE_OK;
}

int flare_list_info(const flare_state* s, long long* n_pairs, int* counts) {
  ARG(s, "null state");
  if (!s->have_list) {
    set_error("no neighbour list");
    return FLARE_E_STALE;
  }
  if (n_pairs) *n_pairs = s->n_pairs;
  if (counts)
    for (int b = 0; b < NBUCKET; ++b) counts[b] = s->bucket_count[b];
  return FLARE_OK;
}

int flare_neighbors_export(flare_state* s, long long* offsets, int32_t* j_out, int32_t* shifts) {
  ARG(s && offsets && j_out && shifts, "null pointer");
  if (!s->have_list) {
    set_error("no neighbour list");
    return FLARE_E_STALE;
  }
  const int n = s->n_atoms;
  const long long P = s->n_pairs;
  std::vector<int> perm(n), off(n + 1), jj(P), ss(P);
  CHK(hipStreamSynchronize(s->stream));
  CHK(hipMemcpy(perm.data(), s->perm, n * sizeof(int), hipMemcpyDeviceToHost));
  CHK(hipMemcpy(off.data(), s->nl_off, (n + 1) * sizeof(int), hipMemcpyDeviceToHost));
  CHK(hipMemcpy(jj.data(), s->nl_j, P * sizeof(int), hipMemcpyDeviceToHost));
  CHK(hipMemcpy(ss.data(), s->nl_s, P * sizeof(int), hipMemcpyDeviceToHost));
  std::vector<int> inv(n);
  for (int i = 0; i < n; ++i) inv[perm[i]] = i;
  struct E {
    int j, sx, sy, sz;
  };
  std::vector<E> row;
  long long k = 0;
  for (int a = 0; a < n; ++a) {
    offsets[a] = k;
    const int i = inv[a];
    row.clear();
    for (int p = off[i]; p < off[i + 1]; ++p) {
      E e;
      e.j = perm[jj[p]];
      unpack_shift(ss[p], e.sx, e.sy, e.sz);
      row.push_back(e);
    }
    std::sort(row.begin(), row.end(), [](const E& u, const E& v) {
      if (u.j != v.j) return u.j < v.j;
      if (u.sx != v.sx) return u.sx < v.sx;
      if (u.sy != v.sy) return u.sy < v.sy;
      return u.sz < v.sz;
    });
    for (const E& e : row) {
      j_out[k] = e.j;
      shifts[3 * k] = e.sx;
      shifts[3 * k + 1] = e.sy;
      shifts[3 * k + 2] = e.sz;
      ++k;
    }
  }
  offsets[n] = k;
  return FLARE_OK;
}

// The mixed (544-wide) rows in chunks of mix_cap rows: descriptors (exported to d_out in
// caller order when given), quadratic forms (energies and gradients when want_e or want_f,
// variances when want_v), adjoint terms when want_f.
static void mixed_rows(flare_state* s, float* d_out, bool want_e, bool want_v, bool want_f) {
  for (int r0 = 0; r0 < s->rowsx; r0 += s->mix_cap) {
    const int nr = std::min(s->mix_cap, s->rowsx - r0);
    desc_mixed_chunk(s, r0, nr, d_out);
    forms_mixed_chunk(s, r0, nr, want_e || want_f, want_v);
    if (want_f) adjoint_mixed_chunk(s, r0, nr);
  }
  // with one chunk the workspace keeps the gradients of these positions for a later backward
  if ((want_e || want_f) && s->rowsx <= s->mix_cap) s->gx_gen = s->pos_gen;
}

int flare_descriptors(flare_state* s, const double* x, const double* y, const double* z, float* d_out,
                      float* norm_out) {
  ARG(s, "null state");
  if (!s->have_list) {
    set_error("flare_descriptors before flare_neighbors");
    return FLARE_E_STALE;
  }
  ARG(s->n_atoms == 0 || (x && y && z), "null positions");
  {
    StageTimer tm(s, FLARE_T_DESC1);
    gather_positions(s, x, y, z);
    pair_geometry(s);
  }
  if (d_out || norm_out) {
    // the single-species rows come from the fused kernel run without quadratic forms
    if (d_out) CHK(hipMemsetAsync(d_out, 0, (size_t)s->n_atoms * ND * sizeof(float), s->stream));
    fused_quadratic_forms(s, FORMS_DESCRIPTORS, d_out);
    mixed_rows(s, d_out, false, false, false);
    export_norms(s, norm_out);
  }
  CHK(hipGetLastError());
  s->have_desc = true;
  s->pos_gen += 1;
  return FLARE_OK;
}

// Energies (and gradients), forces and variances of the positions staged last, up to the
// per-row results (row_out is formed by the output kernels).
static int evaluate_forms(flare_state* s, bool want_f, bool want_v) {
  // With forces the mixed rows run on a second stream beside the fused kernel: both read
  // the step's pair geometry and write disjoint rows and disjoint slots of w_in, so the
  // mixed rows' kernels fill the fused kernel's tail. The main stream waits for them
  // before anything that reads their results. With the stage timers on, everything runs
  // in order on the one stream.
  const bool beside = want_f && s->rowsx > 0 && !s->timers.on;
  if (beside) {
    CHK(hipEventRecord(s->ev_fork, s->stream));
    CHK(hipStreamWaitEvent(s->side, s->ev_fork, 0));
  }
  {
    // with forces, the fused kernel also runs the adjoint of the 144-wide rows in place
    StageTimer tm(s, FLARE_T_QFORM1);
    fused_quadratic_forms(s, 1 | (want_v ? 2 : 0) | (want_f ? 4 : 0), nullptr);
  }
  if (beside) {
    hipStream_t main = s->stream;
    s->stream = s->side;
    mixed_rows(s, nullptr, true, want_v, want_f);
    s->stream = main;
    CHK(hipEventRecord(s->ev_join, s->side));
    CHK(hipStreamWaitEvent(s->stream, s->ev_join, 0));
  } else {
    mixed_rows(s, nullptr, true, want_v, want_f);
  }
  if (want_f) {
    s->w_gen = s->pos_gen;
    s->g_gen = -1;          // the 144-wide gradients stayed on chip
  } else {
    s->g_gen = s->pos_gen;
  }
  return FLARE_OK;
}

int flare_energy_forces(flare_state* s, float* e_atom, float* fx, float* fy, float* fz, double* e_struct,
                        float* var_atom, float* sigma_atom) {
  ARG(s, "null state");
  if (!s->have_desc) {
    set_error("flare_energy_forces before flare_descriptors");
    return FLARE_E_STALE;
  }
  const bool want_f = fx || fy || fz;
  ARG(!want_f || (fx && fy && fz), "pass all three force arrays or none");
  const bool want_v = var_atom || sigma_atom;
  {
    const int rc = evaluate_forms(s, want_f, want_v);
    if (rc != FLARE_OK) return rc;
  }
  {
    StageTimer tm(s, FLARE_T_OUT);
    finalize_outputs(s, e_atom, fx, fy, fz, var_atom, sigma_atom);
    reduce_cells(s, e_struct, nullptr);
  }
  if (want_v) s->v_gen = s->pos_gen;
  CHK(hipGetLastError());
  return FLARE_OK;
}

int flare_forces(flare_state* s, const double* cell_scale, float* fx, float* fy, float* fz) {
  ARG(s, "null state");
  ARG(fx && fy && fz, "null force array");
  if (!s->have_desc || (s->w_gen != s->pos_gen && s->g_gen != s->pos_gen)) {
    set_error("flare_forces needs flare_energy_forces for the current positions");
    return FLARE_E_STALE;
  }
  if (s->w_gen != s->pos_gen) {
    // the 144-wide rows from the gradients the energies left resident, the mixed rows
    // recomputed chunk by chunk
    adjoint_rows144(s);
    if (s->gx_gen == s->pos_gen) adjoint_mixed_chunk(s, 0, s->rowsx);
    else mixed_rows(s, nullptr, true, false, true);
    s->w_gen = s->pos_gen;
  }
  {
    StageTimer tm(s, FLARE_T_OUT);
    finalize_outputs(s, nullptr, fx, fy, fz, nullptr, nullptr, cell_scale);
  }
  CHK(hipGetLastError());
  return FLARE_OK;
}

int flare_virial(flare_state* s, double* virial_struct) {
  ARG(s && virial_struct, "null pointer");
  if (!s->have_desc || s->w_gen != s->pos_gen) {
    set_error("flare_virial needs forces (flare_energy_forces or flare_forces) for the current positions");
    return FLARE_E_STALE;
  }
  CHK(s->red_w.reserve((size_t)9 * s->tasks.size() + 9));
  {
    StageTimer tm(s, FLARE_T_OUT);
    virial_cells(s, virial_struct, s->red_w.p);
  }
  CHK(hipGetLastError());
  return FLARE_OK;
}

int flare_variance(flare_state* s, float* var_atom, float* sigma_atom, float* sigma_max) {
  ARG(s, "null state");
  if (!s->have_desc) {
    set_error("flare_variance before flare_descriptors");
    return FLARE_E_STALE;
  }
  if (s->v_gen != s->pos_gen) {
    {
      StageTimer tm(s, FLARE_T_QFORM1);
      fused_quadratic_forms(s, 2, nullptr);
    }
    mixed_rows(s, nullptr, false, true, false);
    s->v_gen = s->pos_gen;
  }
  {
    StageTimer tm(s, FLARE_T_OUT);
    finalize_outputs(s, nullptr, nullptr, nullptr, nullptr, var_atom, sigma_atom);
    reduce_cells(s, nullptr, sigma_max);
  }
  CHK(hipGetLastError());
  return FLARE_OK;
}

int flare_quadratic_forms(flare_state* s, int bucket, int n_rows, const float* d_rows, float* e_out,
                          float* var_out) {
  ARG(s, "null state");
  ARG(bucket >= 0 && bucket < NBUCKET, "bucket must be 0..5");
  ARG(n_rows >= 0 && n_rows <= s->max_atoms, "n_rows must be in [0, max_atoms]");
  ARG(n_rows == 0 || (d_rows && e_out && var_out), "null device array");
  // the resident descriptors of the last flare_descriptors call are overwritten
  s->have_desc = false;
  s->v_gen = s->g_gen = s->w_gen = s->gx_gen = -1;
  if (n_rows == 0) return FLARE_OK;
  if (bucket_width(bucket) == ND1) {
    forms_given_144(s, bucket, n_rows, d_rows, e_out, var_out);
  } else {
    const int e = forms_given_544(s, bucket, n_rows, d_rows, e_out, var_out);
    if (e) CHK((hipError_t)e);
  }
  CHK(hipGetLastError());
  return FLARE_OK;
}

int flare_uncertainty_monitor(flare_state* s, double threshold, float* sigma_max_run, int32_t* over_count) {
  ARG(s && sigma_max_run && over_count, "null pointer");
  ARG(std::isfinite(threshold), "threshold must be finite");
  if (!s->have_desc) {
    set_error("flare_uncertainty_monitor before flare_descriptors");
    return FLARE_E_STALE;
  }
  if (s->v_gen != s->pos_gen) {
    {
      StageTimer tm(s, FLARE_T_QFORM1);
      fused_quadratic_forms(s, 2, nullptr);
    }
    mixed_rows(s, nullptr, false, true, false);
    s->v_gen = s->pos_gen;
  }
  {
    StageTimer tm(s, FLARE_T_OUT);
    reduce_cells(s, nullptr, nullptr, (float)threshold, sigma_max_run, over_count);
  }
  CHK(hipGetLastError());
  return FLARE_OK;
}

int flare_md_first_half(flare_state* s, double* x, double* y, double* z, double* vx, double* vy, double* vz,
                        const float* fx, const float* fy, const float* fz, const int32_t* species,
                        const double* masses_host, double dt) {
  ARG(s && masses_host, "null pointer");
  if (!s->have_list) {
    set_error("integrator needs the atom count of a neighbour list");
    return FLARE_E_STALE;
  }
  ARG(s->n_atoms == 0 || (x && y && z && vx && vy && vz && fx && fy && fz && species), "null device array");
  ARG(masses_host[0] > 0 && masses_host[1] > 0, "masses must be positive");
  {
    StageTimer tm(s, FLARE_T_MD);
    md_first(s, x, y, z, vx, vy, vz, fx, fy, fz, species, 1.0 / masses_host[0], 1.0 / masses_host[1], dt);
  }
  CHK(hipGetLastError());
  return FLARE_OK;
}

int flare_md_second_half(flare_state* s, double* vx, double* vy, double* vz, const float* fx, const float* fy,
                         const float* fz, const int32_t* species, const double* masses_host, double dt) {
  ARG(s && masses_host, "null pointer");
  if (!s->have_list) {
    set_error("integrator needs the atom count of a neighbour list");
    return FLARE_E_STALE;
  }
  ARG(s->n_atoms == 0 || (vx && vy && vz && fx && fy && fz && species), "null device array");
  ARG(masses_host[0] > 0 && masses_host[1] > 0, "masses must be positive");
  {
    StageTimer tm(s, FLARE_T_MD);
    md_second(s, vx, vy, vz, fx, fy, fz, species, 1.0 / masses_host[0], 1.0 / masses_host[1], dt);
  }
  CHK(hipGetLastError());
  return FLARE_OK;
}

int flare_md_step(flare_state* s, double* x, double* y, double* z, double* vx, double* vy, double* vz, float* fx,
                  float* fy, float* fz, const int32_t* species, const double* masses_host, double dt, int rebuild,
                  float* e_atom, double* e_struct, float* var_atom, float* sigma_atom) {
  ARG(s && masses_host, "null pointer");
  if (!s->have_list) {
    set_error("flare_md_step needs a neighbour list (flare_neighbors)");
    return FLARE_E_STALE;
  }
  ARG(s->n_atoms == 0 || (x && y && z && vx && vy && vz && fx && fy && fz && species), "null device array");
  ARG(masses_host[0] > 0 && masses_host[1] > 0, "masses must be positive");
  const double im0 = 1.0 / masses_host[0], im1 = 1.0 / masses_host[1];
  {
    StageTimer tm(s, FLARE_T_MD);
    md_first_drift(s, x, y, z, vx, vy, vz, fx, fy, fz, species, im0, im1, dt, rebuild == 0);
  }
  if (rebuild) {
    // the same cells, boxes and skin as the last flare_neighbors
    s->have_list = false;
    s->have_desc = false;
    int rc;
    {
      StageTimer tm(s, FLARE_T_LIST);
      rc = build_list(s, x, y, z, species);
    }
    if (rc != FLARE_OK) return rc;
    s->have_list = true;
  }
  {
    StageTimer tm(s, FLARE_T_DESC1);
    if (rebuild) gather_positions(s, x, y, z);   // the displacements from the new build (zero)
    pair_geometry(s);
  }
  s->have_desc = true;
  s->pos_gen += 1;
  const bool want_v = var_atom || sigma_atom;
  {
    const int rc = evaluate_forms(s, true, want_v);
    if (rc != FLARE_OK) return rc;
  }
  {
    StageTimer tm(s, FLARE_T_OUT);
    outputs_second_half(s, e_atom, fx, fy, fz, var_atom, sigma_atom, vx, vy, vz, species, im0, im1, dt);
    reduce_cells(s, e_struct, nullptr);
  }
  if (want_v) s->v_gen = s->pos_gen;
  CHK(hipGetLastError());
  return FLARE_OK;
}

int flare_nvt_first_half(flare_state* s, double* x, double* y, double* z, double* vx, double* vy, double* vz,
                         const float* fx, const float* fy, const float* fz, const int32_t* species,
                         const double* masses_host, double dt, double t_target, double tau, double* thermo) {
  ARG(s && masses_host && thermo, "null pointer");
  if (!s->have_list) {
    set_error("integrator needs the atom count of a neighbour list");
    return FLARE_E_STALE;
  }
  ARG(s->n_atoms == 0 || (x && y && z && vx && vy && vz && fx && fy && fz && species), "null device array");
  ARG(masses_host[0] > 0 && masses_host[1] > 0, "masses must be positive");
  ARG(std::isfinite(dt) && t_target > 0 && tau > 0, "dt finite, t_target and tau positive");
  {
    StageTimer tm(s, FLARE_T_MD);
    nvt_first(s, x, y, z, vx, vy, vz, fx, fy, fz, species, masses_host, dt, t_target, tau, thermo);
  }
  CHK(hipGetLastError());
  return FLARE_OK;
}

int flare_nvt_second_half(flare_state* s, double* vx, double* vy, double* vz, const float* fx, const float* fy,
                          const float* fz, const int32_t* species, const double* masses_host, double dt,
                          double t_target, double tau, double* thermo) {
  ARG(s && masses_host && thermo, "null pointer");
  if (!s->have_list) {
    set_error("integrator needs the atom count of a neighbour list");
    return FLARE_E_STALE;
  }
  ARG(s->n_atoms == 0 || (vx && vy && vz && fx && fy && fz && species), "null device array");
  ARG(masses_host[0] > 0 && masses_host[1] > 0, "masses must be positive");
  ARG(std::isfinite(dt) && t_target > 0 && tau > 0, "dt finite, t_target and tau positive");
  {
    StageTimer tm(s, FLARE_T_MD);
    nvt_second(s, vx, vy, vz, fx, fy, fz, species, masses_host, dt, t_target, tau, thermo, true);
  }
  CHK(hipGetLastError());
  return FLARE_OK;
}

int flare_kinetic(flare_state* s, double* vx, double* vy, double* vz, const int32_t* species,
                  const double* masses_host, double* thermo) {
  ARG(s && masses_host && thermo, "null pointer");
  if (!s->have_list) {
    set_error("flare_kinetic needs the cell layout of a neighbour list");
    return FLARE_E_STALE;
  }
  ARG(s->n_atoms == 0 || (vx && vy && vz && species), "null device array");
  ARG(masses_host[0] > 0 && masses_host[1] > 0, "masses must be positive");
  nvt_second(s, vx, vy, vz, nullptr, nullptr, nullptr, species, masses_host, 0.0, 1.0, 1.0, thermo, false);
  CHK(hipGetLastError());
  return FLARE_OK;
}

int flare_coordination(flare_state* s, const double* x, const double* y, const double* z, int32_t* coord,
                       const int32_t* coord_prev, int64_t* events) {
  ARG(s && coord, "null pointer");
  ARG(s->n_atoms == 0 || (x && y && z), "null positions");
  ARG((coord_prev == nullptr) == (events == nullptr), "pass coord_prev and events together");
  if (!s->have_desc) {
    set_error("flare_coordination needs positions staged by flare_descriptors");
    return FLARE_E_STALE;
  }
  coordination(s, x, y, z, coord, coord_prev, events);
  CHK(hipGetLastError());
  return FLARE_OK;
}

int flare_memory_bytes(const flare_model* m, const flare_state* s, long long* bytes) {
  ARG(bytes, "null pointer");
  long long b = 0;
  if (m) {
    b += (4LL * 2 * ND1 * ND1 + 2LL * 2 * ND * ND) * sizeof(float);   // Wf, Wx
    if (m->vchol) b += 2LL * ND * ND * sizeof(float);                    // Lx
    if (m->precision == FLARE_BF16_SPLIT) b += 4LL * 5 * 9 * 2 * 64 * 8 * sizeof(uint16_t);
    if (m->precision == FLARE_FP8_SPLIT) b += 4LL * 5 * 9 * 2 * 64 * sizeof(uint64_t);
    if (m->precision == FLARE_BF16X6_SPLIT) b += 4LL * 5 * 9 * 3 * 64 * 8 * sizeof(uint16_t);
    if (m->var64) b += (4LL * ND1 * ND1 + 2LL * ND * ND) * sizeof(double);
  }
  if (s) b += s->fixed_bytes + (long long)s->red_w.bytes();
  *bytes = b;
  return FLARE_OK;
}

int flare_timers_enable(flare_state* s, int on) {
  ARG(s, "null state");
  s->timers.on = on != 0;
  return FLARE_OK;
}

int flare_timers_read(flare_state* s, double* ms, long long* counts, int reset) {
  ARG(s, "null state");
  CHK(hipStreamSynchronize(s->stream));
  for (auto& pe : s->timers.pending) {
    float t = 0.f;
    CHK(hipEventElapsedTime(&t, pe.second.first, pe.second.second));
    s->timers.ms[pe.first] += t;
    s->timers.cnt[pe.first] += 1;
    s->timers.pool.push_back(pe.second.first);
    s->timers.pool.push_back(pe.second.second);
  }
  s->timers.pending.clear();
  for (int k = 0; k < FLARE_NTIMERS; ++k) {
    if (ms) ms[k] = s->timers.ms[k];
    if (counts) counts[k] = s->timers.cnt[k];
    if (reset) {
      s->timers.ms[k] = 0.0;
      s->timers.cnt[k] = 0;
    }
  }
  return FLARE_OK;
}

int flare_status(flare_state* s, int32_t* flags_host) {
  ARG(s && flags_host, "null pointer");
  CHK(hipMemcpyAsync(s->h_info + 11, s->d_status, sizeof(int), hipMemcpyDeviceToHost, s->stream));
  CHK(hipMemsetAsync(s->d_status, 0, sizeof(int), s->stream));
  CHK(hipStreamSynchronize(s->stream));
  *flags_host = s->h_info[11] | s->flags_pending;
  s->flags_pending = 0;
  return FLARE_OK;
}

int flare_interval_status(const flare_state* s, int32_t* flags_host) {
  ARG(s && flags_host, "null pointer");
  *flags_host = s->flags_at_build;
  return FLARE_OK;
}

}  // extern "C"
