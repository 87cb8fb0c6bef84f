// Library-owned model and evaluation state (device buffers and host-side bookkeeping).
#pragma once

#include "common.h"
#include "flare.h"

namespace flare {

// Small device array that grows at list builds (never on the per-step path).
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t cap = 0;
  size_t bytes() const { return cap * sizeof(T); }
  hipError_t reserve(size_t n) {
    if (n <= cap) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    size_t want = n + n / 4 + 64;
    hipError_t e = hipMalloc((void**)&p, want * sizeof(T));
    if (e == hipSuccess) cap = want;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

// HIP-event stage timers (enabled on demand; see flare_timers_enable).
struct Timers {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  double ms[FLARE_NTIMERS] = {};
  long long cnt[FLARE_NTIMERS] = {};
};

// Per-step pair data in the sliced layout (see nlist.hip): rows are grouped in slices of
// 32 consecutive rows; the k-th pair of every row of a slice sits in one contiguous group
// of 32 slots, so a wave reading "pair k of its 32 rows" reads 512 contiguous bytes.
//   row R: 144-wide rows are R = 0..rows1-1, mixed rows R = rows1 + r
//   slot(R, k) = (slice_base[R / 32] + k) * 32 + R % 32
struct SlotView {
  const float4* geom;       // per slot: (u_x, u_y, u_z, r) of the pair, r = 0 outside the
                            // cutoff or padding; r < 0 marks an H neighbour, r > 0 Pt
  const int* slice_base;    // [slices + 1] in groups of 32 slots
  const int* rev;           // per slot: slot of the reverse pair (padding: itself)
  float4* w_in;             // per slot: the adjoint term de_j/dDelta of the reverse pair
  float rc;
};

__host__ __device__ inline int slot_of(const int* slice_base, int R, int k) {
  return (slice_base[R >> 5] + k) * 32 + (R & 31);
}

// Caller-order record of one atom written by the first pass of the list build and read
// once, by the bin-sorted gather: one 64-byte line per atom.
struct __attribute__((aligned(64))) CallerRec {
  double wx, wy, wz;         // wrapped position
  double ox, oy, oz;         // image offset: wrapped = x + offset
  int bin, cell, pad0, pad1;
};

// Reduction task: a contiguous internal atom range of one cell.
struct RedTask {
  int cell;
  int begin;
  int end;
};

}  // namespace flare

struct flare_model {
  int device = 0;
  int precision = FLARE_FP32;     // arithmetic form of the energy pass (FLARE_FP32 .. FLARE_BF16X6_SPLIT)
  int flags = 0;                  // the precision argument as given (form | FLARE_VAR_FP32)
  bool var64 = false;             // variance on the FP64 matrix cores (split forms without FLARE_VAR_FP32)
  // variances from Cholesky factors (part 1 of Wf and Wxf holds L)
  bool vchol = false;
  double r_cut = 0.0;
  // Single-species buckets: beta (part 0) and Sigma or its Cholesky factor L (part 1) of
  // the central species, restricted to the bucket's 144-wide block, in MFMA fragment
  // order [part 2][K chunk 9][column block 9][lane 64] float4: element t of lane l of
  // (kc, cb) is M[16 kc + 4 (l / 16) + t][16 cb + l % 16] (see fused.hip).
  float* Wf[4] = {};
  // Mixed buckets (4: H centre, 5: Pt centre): beta then Sigma of the central species over
  // all 544 components, [2][544][544] with row n = column n of the matrix (see qform.hip);
  // with Cholesky factors, Lx holds L in the same form.
  float* Wx[2] = {};
  float* Lx[2] = {};
  // BF16 split form (precision FLARE_BF16_SPLIT), single-species buckets: beta as
  // [K step 5][column block 9][hi/lo 2][lane 64] x 8 bf16 (K padded 144 -> 160). In this
  // form the Sigma part of Wf holds the Cholesky factor L of Sigma (Sigma = L L^T).
  uint16_t* Wb[4] = {};
  // FP8 split form (precision FLARE_FP8_SPLIT): s_b * beta as [K step 5][column block 9]
  // [hi, lo' 2][lane 64] x 8 OCP e4m3 bytes, converted on the device by the same
  // instruction the kernel uses for d; lo' = fp8(16 (x - hi)). s_b = 2^k keeps |s_b beta| <= 16.
  uint64_t* W8[4] = {};
  float beta_scale[4] = {1.f, 1.f, 1.f, 1.f};
  // Three-way BF16 form (precision FLARE_BF16X6_SPLIT): beta as [K step 5][column block 9]
  // [part 3][lane 64] x 8 bf16, parts x0 + x1 + x2 = FP32 value.
  uint16_t* W6[4] = {};
  // Split forms: Cholesky factors in FP64 for the variance on the FP64 matrix cores, in
  // fragment order [column block][K chunk][k-step 4][lane 64]: element L[16 kc + 4 (lane / 16)
  // + t][16 cb + lane % 16]. Single-species buckets: the factor of the bucket's 144 x 144
  // block of Sigma (9 x 9 blocks); mixed buckets: the factor of Sigma_s (34 x 34 blocks).
  double* L64[4] = {};
  double* Lx64[2] = {};
};

struct flare_state {
  const flare_model* model = nullptr;
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;         // the mixed rows beside the fused kernel (default priority)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int device = 0;
  int max_atoms = 0;
  long long max_pairs = 0;

  // ---- current list ----
  bool have_list = false;
  bool have_desc = false;
  long long pos_gen = 0;     // positions staged by flare_descriptors
  long long v_gen = -1;      // positions the variances were computed for
  long long g_gen = -1;      // positions the energy gradients were computed for
  long long w_gen = -1;      // positions the per-pair adjoint terms were computed for
  long long gx_gen = -1;     // positions the mixed rows' gradients in the workspace are for
                             // (only when all mixed rows fit one chunk)
  long long fixed_bytes = 0; // device bytes of the fixed-size arrays
  int n_atoms = 0;
  int n_struct = 0;
  int n_bins = 0;
  double skin = 0.0;
  double r_list = 0.0;
  long long n_pairs = 0;
  int bucket_count[flare::NBUCKET] = {};
  int bucket_row0[flare::NBUCKET] = {};   // first row of each bucket inside its class
  int rows1 = 0;                           // padded rows of the 144-wide class
  int rowsx = 0;                           // padded rows of the 544-wide class
  std::vector<flare::CellGrid> grids;
  std::vector<int> struct_off;
  std::vector<flare::RedTask> tasks;
  std::vector<int> first_task;

  // ---- capacities, fixed at flare_state_create (no device allocation after it) ----
  int row_cap = 0;           // rows of both width classes: max_atoms + bucket padding
  int slice_cap = 0;         // row_cap / 32
  long long slot_cap = 0;    // slots of the sliced pair layout
  int bin_cap = 0;           // cell-list bins over all cells of a build
  int cell_cap = 0;          // cells (structures) per build
  int task_cap = 0;          // reduction tasks
  int nblk_cap = 0;          // 256-atom blocks
  int mix_cap = 0;           // mixed rows processed together (the 544-wide workspace)

  // ---- per-atom device arrays (capacity max_atoms) ----
  int* perm = nullptr;       // internal -> caller index
  int* sp = nullptr;         // species, internal order
  int* sid = nullptr;        // cell id, internal order
  int* bin = nullptr;        // global bin id, internal order
  int* envmask = nullptr;    // species bits of listed neighbours
  int* bucket = nullptr;
  int* row_of = nullptr;     // row of each internal atom inside its width class (-1: none)
  int* nl_cnt = nullptr;
  int* nl_off = nullptr;     // [max_atoms + 1]
  double4* w = nullptr;      // [N] wrapped positions at the list build (x, y, z, species)
  float4* wf = nullptr;      // [N] the same rounded to FP32 (species in .w), for the search's first test
  double* off = nullptr;     // [3][N] image offset: internal position = x + off
  float4* dlt = nullptr;     // [N] displacement of the current step from the build, FP32 (x, y, z, 0)
  double* xb = nullptr;      // [3][N] positions at the list build, caller order
  int* inv_perm = nullptr;   // [N] caller -> internal index
  float* nrm = nullptr;      // |d~| per internal atom
  float* e_int = nullptr;
  float* v_int = nullptr;
  flare::CallerRec* crec = nullptr;   // list build: caller-order wrapped position, image offset, bin, cell
  int* sorted = nullptr;     // bin-sorted caller indices
  int* row_caller = nullptr; // [N] row of each atom, caller order (-1: none)
  int* slot0 = nullptr;      // [N] slot of each internal atom's first pair (-1: no row)
  int2* pair_cache = nullptr;  // list build: first PAIR_CACHE pairs of each atom, [k][N]

  // ---- per-pair (capacity max_pairs) ----
  int* nl_j = nullptr;       // internal index of the neighbour
  int32_t* nl_s = nullptr;   // packed image shift
  int* nl_rev = nullptr;     // position of the reverse pair (j, i, -s) inside j's list

  // ---- per cell, bin, block ----
  flare::CellGrid* d_grids = nullptr;   // [cell_cap]
  int* d_struct_off = nullptr;          // [cell_cap + 1]
  int* bin_count = nullptr;             // [bin_cap + 1]
  int* bin_start = nullptr;
  int* bin_fill = nullptr;
  int* blk_bucket = nullptr;            // [NKEY][nblk_cap]
  int* blk_bucket_scan = nullptr;
  int* scan_scratch = nullptr;
  flare::RedTask* d_tasks = nullptr;    // [task_cap]
  int* d_first_task = nullptr;          // [cell_cap + 1] task range of each cell
  double* red_e = nullptr;              // [task_cap][2] (sum, compensation)
  float* red_s = nullptr;               // [task_cap]

  // ---- per row (capacity row_cap; 144-wide rows, then mixed rows) ----
  int* atom_of_row1 = nullptr;
  int* atom_of_rowx = nullptr;
  int* cnt_row = nullptr;               // pairs
  int* sid_row = nullptr;               // cell
  float* e_row = nullptr;               // per step: e_i, V_i
  float* v_row = nullptr;
  float4* row_out = nullptr;            // per step: (F_i, e_i) in row order
  float4* f_own = nullptr;              // per row: sum of de_i/dDelta over its own pairs
  float* G1 = nullptr;                  // [row_cap / 128][144][128] gradients (energies without forces)
  // mixed rows, one chunk of mix_cap rows at a time
  float* Dx = nullptr;                  // [mix_cap][544] descriptors
  float* Gx = nullptr;                  // gradients
  float* Yx = nullptr;                  // D beta
  float* Px = nullptr;                  // [mix_cap][4] partial row sums of the column tiles
  double* Px64 = nullptr;               // [mix_cap][9] FP64 variance partials (split forms)

  // ---- sliced pair layout (capacity slot_cap) ----
  int n_slices = 0;
  long long n_slots = 0;
  int* slice_len = nullptr;             // [slice_cap + 1]
  int* slice_base = nullptr;
  int* slot_atom = nullptr;              // row's atom (padding: -1)
  int* slot_j = nullptr;
  int* slot_rev = nullptr;
  float4* slot_d0 = nullptr;            // per slot: (w_j - w_i) + s*L in FP32, neighbour species sign
  float4* geom = nullptr;               // per slot, per step
  float4* w_in = nullptr;               // per slot: w of the reverse pair

  // virial task sums (allocated at the first flare_virial call)
  flare::DevBuf<double> red_w;          // [tasks][9]

  flare::Timers timers;

  // ---- status ----
  int* d_status = nullptr;   // [0] caller-visible status word (sticky), [1] list-build checks
  int flags_at_build = 0;    // word [0] as the last list build found it
  int flags_pending = 0;     // flags moved to the host by list builds, not yet returned by flare_status
  int* d_layout = nullptr;   // list build: sizes formed on the device (see nlist.hip)
  int* h_info = nullptr;     // pinned host copy of d_layout, read once per build
  char* h_stage = nullptr;   // pinned staging of the per-cell host data of a build
  size_t h_stage_bytes = 0;
};

namespace flare {
SlotView slot_view(const flare_state* s);

// Records the stage's start event on construction and its stop event on destruction.
struct StageTimer {
  flare_state* s;
  int stage;
  hipEvent_t stop = nullptr;
  StageTimer(flare_state* st, int stg);
  ~StageTimer();
};
// Displacement of caller atom a since the list build, d = (x, y, z) - xb in FP64, stored in
// FP32 at its internal index; it must stay within half the skin (lim2 = (skin/2)^2), else a
// status bit is raised. Shared by the standalone kernel and the integrator's drift.
__device__ __forceinline__ void store_displacement(int a, int n, double x, double y, double z,
                                                   const double* __restrict__ xb, const int* __restrict__ inv_perm,
                                                   float4* __restrict__ dlt, double lim2, int* __restrict__ status) {
  const double d0 = x - xb[a];
  const double d1 = y - xb[(size_t)n + a];
  const double d2 = z - xb[2 * (size_t)n + a];
  dlt[inv_perm[a]] = make_float4((float)d0, (float)d1, (float)d2, 0.f);
  const double d2s = d0 * d0 + d1 * d1 + d2 * d2;
  if (!(d2s <= lim2)) {
    if (!isfinite(d2s)) atomicOr(status, FLARE_FLAG_NONFINITE);
    else atomicOr(status, FLARE_FLAG_DISPLACED);
  }
}
// list-build constants for the capacities of a state (nlist.hip)
int list_key_count();      // sort keys of the row order (per 256-atom block)
int list_pair_cache();     // pairs per atom kept by the counting pass
int list_layout_words();   // ints of the device layout record
// launchers (nlist.hip, desc.hip, qform.hip, adjoint.hip, reduce.hip)
int build_list(flare_state* s, const double* x, const double* y, const double* z,
               const int32_t* species);
void gather_positions(flare_state* s, const double* x, const double* y, const double* z);
void pair_geometry(flare_state* s);
// 144-wide rows: mode bit 0 energies and gradients, bit 1 variances, bit 2 forces in the same
// kernel, FORMS_DESCRIPTORS the descriptors (and norms) alone; d_out (caller order, [n][544],
// zeroed by the caller) receives their descriptors
constexpr int FORMS_DESCRIPTORS = 8;
void fused_quadratic_forms(flare_state* s, int mode, float* d_out);
// mixed rows [r0, r0 + nr) of the 544-wide class (nr <= mix_cap, r0 a multiple of mix_cap),
// in the chunk workspace Dx/Yx/Gx/Px: descriptors (and their export to caller order),
// quadratic forms, adjoint terms
void desc_mixed_chunk(flare_state* s, int r0, int nr, float* d_out);
void forms_mixed_chunk(flare_state* s, int r0, int nr, bool want_e, bool want_v);
void adjoint_mixed_chunk(flare_state* s, int r0, int nr);
// |d~| of every atom in caller order
void export_norms(flare_state* s, float* norm_out);
// quadratic forms of given vectors with the model of one bucket (fused.hip, qform.hip)
void forms_given_144(flare_state* s, int bucket, int n, const float* d, float* e, float* v);
int forms_given_544(flare_state* s, int bucket, int n, const float* d, float* e, float* v);
// adjoint terms of the 144-wide rows from G1 (separate from the energies)
void adjoint_rows144(flare_state* s);
void finalize_outputs(flare_state* s, float* e_atom, float* fx, float* fy, float* fz,
                      float* var_atom, float* sigma_atom, const double* cell_scale = nullptr);
// per-cell E and max sigma; with run_max, the uncertainty monitor (threshold thr, counts in over)
void reduce_cells(flare_state* s, double* e_struct, float* sigma_max, float thr = 0.f, float* run_max = nullptr,
                  int* over = nullptr);
// per-cell virial; red_w: [tasks][9] FP64 task sums (scratch)
void virial_cells(flare_state* s, double* virial_struct, double* red_w);
void md_first(flare_state* s, double* x, double* y, double* z, double* vx, double* vy,
              double* vz, const float* fx, const float* fy, const float* fz,
              const int32_t* species, double inv_m0, double inv_m1, double dt);
// one NVE step's kernels: first half and drift with the displacements of the new positions
// (when the list stays), and the caller-order outputs with the second half
void md_first_drift(flare_state* s, double* x, double* y, double* z, double* vx, double* vy, double* vz,
                    const float* fx, const float* fy, const float* fz, const int32_t* species, double inv_m0,
                    double inv_m1, double dt, bool displacements);
void outputs_second_half(flare_state* s, float* e_atom, float* fx, float* fy, float* fz, float* var_atom,
                         float* sigma_atom, double* vx, double* vy, double* vz, const int32_t* species,
                         double inv_m0, double inv_m1, double dt);
void md_second(flare_state* s, double* vx, double* vy, double* vz, const float* fx,
               const float* fy, const float* fz, const int32_t* species, double inv_m0,
               double inv_m1, double dt);
// Nose-Hoover halves, kinetic energy, coordination (thermo.hip)
void nvt_first(flare_state* s, double* x, double* y, double* z, double* vx, double* vy, double* vz,
               const float* fx, const float* fy, const float* fz, const int32_t* species, const double* masses,
               double dt, double t0, double tau, double* thermo);
void nvt_second(flare_state* s, double* vx, double* vy, double* vz, const float* fx, const float* fy,
                const float* fz, const int32_t* species, const double* masses, double dt, double t0, double tau,
                double* thermo, bool update);
void coordination(flare_state* s, const double* x, const double* y, const double* z, int32_t* coord,
                  const int32_t* prev, int64_t* events);
void set_error(const std::string& msg);
// FP8 fragments from FP32 values in fragment order [groups][lane 64][8] (fused.hip)
void make_fp8_fragments(const float* vals, int groups, uint64_t* out);
}  // namespace flare
