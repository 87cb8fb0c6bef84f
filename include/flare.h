/*
 * flare.h - C ABI of the MI355X (gfx950) evaluator for the FLARE B2 Bayesian force field.
 *
 * What it computes (paper: Section V.B and Eqs. 1-2). For every atom i of one or more
 * periodic orthorhombic cells:
 *   rho_i      all neighbours j (and periodic images) closer than r_cut         (Sec. V.B)
 *   c_i        c_{(s,n),l,m} = sum_{j in rho_i, s_j = s} T_n(2r/r_c - 1) (r_c - r)^2 Y_lm(r^)
 *   d~_i       B2: d~_{(a,b),l} = sum_m c_{a,l,m} c_{b,l,m}, a <= b            (Sec. V.B, Fig. 3)
 *   d_i        d~_i / |d~_i|
 *   e_i        d_i^T beta_{s_i} d_i      (mapped posterior mean, Eq. 1)
 *   V_i        d_i^T Sigma_{s_i} d_i     (mapped posterior variance, Eq. 2; sigma_i = sqrt V_i)
 *   F_k        -dE/dr_k, E = sum_i e_i  (by the reordered adjoint sum of Sec. V.B: no
 *              descriptor gradient is ever formed)
 * Atoms whose neighbours within the list radius are all of one species use only that
 * species-pair block of d and of beta/Sigma (the reduction of Sec. V.B); the result
 * is identical because the other components are exactly zero.
 *
 * Conventions shared by every call:
 *   - Units: Angstrom, eV, eV/A, amu, fs. Species are 0 .. n_species-1 (H = 0, Pt = 1).
 *   - Pointers documented as DEVICE must point to memory the caller allocated on the
 *     current HIP device (for example torch tensors); the caller owns them and keeps
 *     them alive until the enqueued work completes. HOST pointers are read during the call.
 *   - Every call enqueues on the stream given at flare_state_create and returns without
 *     waiting, unless documented as SYNCHRONISING.
 *   - Atom arrays are in the caller's order. Structures (cells) occupy consecutive atom
 *     ranges struct_offsets[k] .. struct_offsets[k+1]-1; each has its own box.
 *   - Return value: FLARE_OK (0) or a negative FLARE_E_* code. Nothing throws across the
 *     ABI. flare_last_error() gives a human-readable detail of the last failure on the
 *     calling thread.
 *   - Conditions found on the device (non-finite input, list overflow, atoms moved more
 *     than half the skin since the last list build) set bits of a status word that only
 *     flare_status reads, so the per-step calls stay asynchronous.
 */
#ifndef FLARE_H
#define FLARE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define FLARE_OK             0
#define FLARE_E_ARG         -1  /* null pointer, bad size or out-of-range parameter            */
#define FLARE_E_SPECIES     -2  /* a species index outside [0, n_species)                       */
#define FLARE_E_BOX         -3  /* a box side <= 0 or not finite                                */
#define FLARE_E_CAPACITY    -4  /* more atoms or pairs than the state was created for           */
#define FLARE_E_NONFINITE   -5  /* a position is NaN or infinite                                */
#define FLARE_E_STALE       -6  /* call order: no neighbour list / no descriptors for this step */
#define FLARE_E_OOM         -7  /* device allocation failed                                     */
#define FLARE_E_HIP         -8  /* HIP runtime error (detail in flare_last_error)                */
#define FLARE_E_UNSUPPORTED -9  /* model sizes this build has no kernels for                    */

/* ---- arithmetic of the quadratic forms ---- */
/* The split forms change the energy contraction d.beta.d of the single-species rows
 * (144-wide): the two-part forms (BF16, FP8) split the operands into a high and a low part
 * in a narrow format and recombine them in FP32 accumulators; the three-way BF16 form
 * splits d and beta into three BF16 parts each (together the 24 significant bits of the
 * FP32 value) and keeps six of the nine part products, so its error is that of FP32
 * arithmetic. Mixed-environment rows (544-wide) keep FP32 energy products in all forms.
 * The variance d.Sigma.d is computed as |L^T d|^2 with the FP64 Cholesky factor L of each
 * Sigma block, a sum of squares, whenever all Sigma blocks are positive definite (the split
 * forms require it; the FP32 form falls back to the full matrix otherwise): in the FP32
 * form with L rounded to FP32 on FP32 matrix cores, in the split forms (all rows) with L in
 * FP64 on the FP64 matrix cores, FP64 sums and an FP64 division by |d~|^2, so that a
 * near-cancelling variance (an environment close to the sparse set of Eq. 2) keeps FP64
 * accuracy in the form and only the FP32 rounding of the descriptors remains. Norms and
 * per-structure sums are FP64 in the split forms. */
#define FLARE_FP32        0  /* FP32 matrix cores, FP32 accumulation                          */
#define FLARE_BF16_SPLIT  1  /* d and beta as BF16 hi + lo, three products; FP64 variance     */
#define FLARE_FP8_SPLIT   2  /* OCP e4m3 hi + lo, power-of-two scales; FP64 variance          */
#define FLARE_BF16X6_SPLIT 3 /* d and beta as three BF16 parts, six products (FP32 error);
                                FP64 variance                                                  */
#define FLARE_VAR_FP32   16  /* OR-ed with a split form: the variance through the FP32 factor
                                on FP32 matrix cores (FP64 sums) as in the FP32 form, instead
                                of FP64: faster, with the FP32 form's variance error           */

/* ---- device status bits (flare_status) ---- */
#define FLARE_FLAG_NONFINITE  1  /* a position was NaN/inf                                     */
#define FLARE_FLAG_SPECIES    2  /* a species index was out of range                            */
#define FLARE_FLAG_DISPLACED  4  /* some atom moved more than skin/2 since the list was built:
                                    the list may miss pairs inside r_cut, results of that step
                                    are not to be trusted                                      */
#define FLARE_FLAG_UNCERTAIN  8  /* flare_uncertainty_monitor: a cell's largest sigma exceeded
                                    the threshold (the active-learning trigger)               */

typedef struct flare_model flare_model;
typedef struct flare_state flare_state;

/* Last error detail of the calling thread (static storage, never NULL). */
const char* flare_last_error(void);
/* Short name of a status code. */
const char* flare_strerror(int code);

/*
 * Create a model: one mapped pair (beta_s, Sigma_s) per central species s (Eqs. 1-2).
 *   beta_host, sigma_host: HOST, FP64, [n_species][n_d][n_d] row-major, symmetric,
 *   indexed in the packed B2 order: species-pair blocks (s1 <= s2) in order, inside a
 *   block the radial pairs (n_a, n_b) row-major (n_a <= n_b when s1 == s2), l fastest.
 *   n_d = n_species*n_rad*(n_species*n_rad+1)/2 * (l_max+1).
 * This build has kernels for n_species = 2, n_rad = 8, l_max = 3 (n_d = 544); other
 * sizes return FLARE_E_UNSUPPORTED. precision: FLARE_FP32, FLARE_BF16_SPLIT,
 * FLARE_FP8_SPLIT or FLARE_BF16X6_SPLIT, a split form optionally | FLARE_VAR_FP32; the
 * split forms need every 144 x 144 single-species block of Sigma positive definite
 * (FLARE_E_ARG otherwise).
 * The library copies the matrices to device memory it owns. Runs on the current device.
 */
int flare_model_create(flare_model** out, int n_species, int n_rad, int l_max, double r_cut,
                       const double* beta_host, const double* sigma_host, int precision);
/*
 * Create a model from a sparse set: the exact mapping of the sparse GP onto the quadratic
 * forms (Section V.B, Eqs. 1-2). Kernel k_xi(d1, d2) = sigma^2 (d1 . d2)^xi; per central
 * species s with sparse descriptors D_s [n_s][n_d] and weights alpha_s:
 *   beta_s  = sigma^2 D_s^T diag(alpha_s) D_s                       (mean, xi = 2)
 *   gamma_s = sigma^2 I - sigma^4 D_s^T K_s^-1 D_s,                  (variance, xi = 1)
 *   K_s     = sigma^2 D_s D_s^T + noise I  (the sparse-set kernel matrix),
 * so that d^T beta_s d and d^T gamma_s d equal the unmapped SGP mean and variance. The
 * variance model is gamma (Sigma of flare_model_create). All of it is computed in FP64 on
 * the current device (K_s by Cholesky, gamma_s = sigma^2 I - sigma^4 Y^T Y with
 * Y = C^-1 D_s; no inverse is formed), then the model is created as by flare_model_create.
 *   n_sparse_host  HOST int32 [n_species]: sparse environments of each central species
 *   d_sparse       DEVICE FP64 [sum n_s][n_d]: normalised descriptors in the packed order of
 *                  flare_model_create, species 0 first, then species 1
 *   alpha          DEVICE FP64 [sum n_s], same order
 *   signal_var     sigma^2 > 0;  noise >= 0 (added to the diagonal of K_s)
 *   beta_out, gamma_out  optional DEVICE FP64 [n_species][n_d][n_d] copies (NULL = skip)
 * SYNCHRONISING (runs on the default stream). Allocates device temporaries of
 * (2 n_max^2 + n_max n_d + 4 n_d^2) doubles, n_max = max_s n_s. A species without sparse
 * environments gets beta = 0 and gamma = sigma^2 I. Errors: FLARE_E_ARG (sizes, a kernel
 * matrix that is not positive definite, or a gamma block without a Cholesky factor in a
 * split precision form), FLARE_E_UNSUPPORTED, FLARE_E_OOM, FLARE_E_HIP.
 */
int flare_model_from_sparse_set(flare_model** out, int n_species, int n_rad, int l_max, double r_cut,
                                const int32_t* n_sparse_host, const double* d_sparse, const double* alpha,
                                double signal_var, double noise, int precision, double* beta_out,
                                double* gamma_out);
int flare_model_destroy(flare_model* model);
/*
 * How the model evaluates: *precision as passed at creation (form | FLARE_VAR_FP32);
 * *variance_cholesky = 1 when
 * the variance is computed as |L^T d|^2 from the FP64 Cholesky factor L of every Sigma
 * block (all blocks positive definite; always so in the split forms), 0 when the FP32
 * form uses d^T Sigma d with the full matrix. Either pointer may be NULL. HOST pointers.
 */
int flare_model_info(const flare_model* model, int* precision, int* variance_cholesky);
/* n_d of the model (544 for the supported sizes). */
int flare_descriptor_dim(const flare_model* model, int* n_d);

/*
 * Create evaluation state for up to max_atoms atoms and max_pairs directed list pairs.
 * stream: a hipStream_t (passed as void*; NULL = the default stream). The state keeps
 * the neighbour list, the descriptors and the gradients on the device between calls.
 * Every device buffer is allocated here, sized from max_atoms and max_pairs: per atom,
 * per listed pair, per row (max_atoms plus the 128-row padding of the six environment
 * classes), the sliced pair layout (max_pairs * 5/4 + 12,288 slots), cell-list bins
 * (4 max_atoms, at least 65,536; wider bins are used when the cells need more), cells
 * (max_atoms + 1) and a workspace of 16,384 mixed-environment rows (the 544-wide rows are
 * processed in chunks of that many). No later call allocates device memory, except the
 * first flare_virial (its task sums; flare_virial_noalloc allocates nothing).
 * flare_memory_bytes reports the total. One state serves one stream; calls on one state
 * must not overlap. The state also creates one internal stream (default priority, on the
 * current device) and two events: with forces, the 544-wide rows run on it beside the
 * single-species kernel, forked from and joined back into the caller's stream inside the
 * call, so the caller's stream alone orders every result, as with one stream.
 */
int flare_state_create(flare_state** out, const flare_model* model, int max_atoms,
                       long long max_pairs, void* stream);
int flare_state_destroy(flare_state* state);

/*
 * Build the neighbour list (SYNCHRONISING: waits for the stream once, at the end, to read
 * the sizes the build found on the device and its status words; allocates nothing).
 *   x, y, z       DEVICE FP64 [n_atoms] positions (any periodic image)
 *   species       DEVICE int32 [n_atoms]
 *   n_struct      number of cells; struct_offsets_host HOST int32 [n_struct+1]
 *                 (offsets[0] = 0, offsets[n_struct] = n_atoms, non-decreasing)
 *   boxes_host    HOST FP64 [n_struct][3] orthorhombic sides, periodic on every axis
 *   skin          list radius = r_cut + skin (skin >= 0)
 * A pair (i, j, s) is listed when |w_j - w_i + s*L|^2 < (r_cut+skin)^2, with
 * w = x - L*floor(x/L) and the squared distance evaluated in FP64 as
 * (dx*dx + dy*dy) + dz*dz without fused multiply-add; (i, i, 0) is excluded.
 * Errors: FLARE_E_ARG, FLARE_E_BOX, FLARE_E_SPECIES, FLARE_E_NONFINITE,
 * FLARE_E_CAPACITY (n_atoms > max_atoms, more than max_atoms + 1 cells, pairs > max_pairs,
 * or a sliced layout beyond its slots: the list is not usable; create a larger state),
 * FLARE_E_HIP.
 */
int flare_neighbors(flare_state* state, int n_atoms, const double* x, const double* y,
                    const double* z, const int32_t* species, int n_struct,
                    const int32_t* struct_offsets_host, const double* boxes_host, double skin);

/* Number of directed pairs in the current list and the atom count per environment
 * class (HOST outputs; counts[6] in the order (H centre, H-only), (Pt, H-only),
 * (H, Pt-only), (Pt, Pt-only), (H, mixed), (Pt, mixed); atoms with no neighbour are
 * not counted). Either pointer may be NULL. Needs a list. Not synchronising. */
int flare_list_info(const flare_state* state, long long* n_pairs, int* counts);

/*
 * Copy the list out in the caller's atom order and canonical per-atom order
 * (j, sx, sy, sz) ascending (SYNCHRONISING). HOST outputs:
 *   offsets [n_atoms+1] int64, j [n_pairs] int32, shifts [n_pairs][3] int32 (image s).
 */
int flare_neighbors_export(flare_state* state, long long* offsets, int32_t* j, int32_t* shifts);

/*
 * Descriptors for the current positions (same atoms, order and cells as the last list).
 *   x, y, z   DEVICE FP64 [n_atoms]; the positions may have moved since the list build
 *             (the status bit FLARE_FLAG_DISPLACED is set if any atom moved > skin/2).
 *   d_out     optional DEVICE FP32 [n_atoms][n_d] normalised descriptors in the packed
 *             order, zeros outside an atom's block (NULL = not written)
 *   norm_out  optional DEVICE FP32 [n_atoms] |d~_i| (NULL = not written)
 * Pair vectors are formed as the FP64 difference of the positions at the list build (plus
 * the image shift), rounded to FP32, plus the FP32 displacements of both atoms since the
 * build; pairs with |Delta|^2 < r_cut^2 (FP32) enter the descriptors.
 * The descriptors stay resident in the state for flare_energy_forces / flare_variance.
 */
int flare_descriptors(flare_state* state, const double* x, const double* y, const double* z,
                      float* d_out, float* norm_out);

/*
 * Energies and forces for the positions staged by the last flare_descriptors call.
 *   e_atom         DEVICE FP32 [n_atoms] e_i                         (NULL = not written)
 *   fx, fy, fz     DEVICE FP32 [n_atoms] forces, eV/A. Pass all three, or all three NULL
 *                  to evaluate energies only; the gradients stay resident so that a later
 *                  flare_forces call for the same positions returns the forces.
 *   e_struct       DEVICE FP64 [n_struct] sum of e_i per cell, compensated (NULL = skip)
 *   var_atom, sigma_atom  DEVICE FP32 [n_atoms]: when either is non-NULL the variance
 *                  quadratic form is evaluated in the same pass over the descriptors.
 * Forces are gathered per atom in a fixed order (no atomics): results are bitwise
 * reproducible and do not depend on which other cells share the call.
 */
int flare_energy_forces(flare_state* state, float* e_atom, float* fx, float* fy, float* fz,
                        double* e_struct, float* var_atom, float* sigma_atom);

/*
 * Forces (the adjoint of the energy) for the positions of the last flare_energy_forces
 * call, which must have run for the current flare_descriptors positions.
 *   cell_scale     optional DEVICE FP64 [n_struct]: the forces of cell k are multiplied
 *                  by cell_scale[k] (a backward pass passes -dL/dE_k to obtain dL/dr)
 *   fx, fy, fz     DEVICE FP32 [n_atoms]
 */
int flare_forces(flare_state* state, const double* cell_scale, float* fx, float* fy, float* fz);

/*
 * Virial of each cell, the strain derivative behind the stress the model predicts
 * (Section VI): under x -> (I + eps) x of positions and box every pair vector Delta
 * becomes (I + eps) Delta, so
 *   W_ab = -dE/deps_ab = -sum over list pairs (i, j) inside r_cut of Delta_a * (de_i/dDelta)_b
 * (the stress is -W / volume). Uses the per-pair adjoint terms of the last force
 * evaluation, which must be for the current positions (FLARE_E_STALE otherwise).
 *   virial_struct  DEVICE FP64 [n_struct][9], row-major W_xx W_xy W_xz W_yx ... W_zz.
 * Per-atom terms are summed in FP32 over each atom's pairs in list order, then in FP64
 * over the cell's atoms in a fixed order (deterministic). Allocates one internal buffer
 * (the FP64 task sums, 72 bytes per reduction task of up to 2,048 atoms) on the first call.
 */
int flare_virial(flare_state* state, double* virial_struct);

/*
 * flare_virial without any device allocation, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels
 * and the same result, bit for bit, but the FP64 per-task sums go to a fixed 1 MiB device
 * array of the library (one copy per GPU, held until the process ends) instead of state
 * memory that flare_virial grows on its first call. No hipMalloc, hipFree or stage-timer
 * event is made. Limit: at most 14,563 reduction tasks (a task is up to 2,048 atoms of one
 * cell: about 29 M atoms in one cell, fewer with many small cells); beyond it
 * FLARE_E_CAPACITY. The state's device must be current (FLARE_E_ARG otherwise). All calls
 * on one GPU share the array: calls that overlap on one GPU (different streams at once) race.
 *   virial_struct  DEVICE FP64 [n_struct][9], as flare_virial.
 */
int flare_virial_noalloc(flare_state* state, double* virial_struct);

/*
 * Variance and uncertainty only (Eq. 2), from the resident descriptors.
 *   var_atom, sigma_atom  DEVICE FP32 [n_atoms] (either may be NULL)
 *   sigma_max             DEVICE FP32 [n_struct] largest sigma per cell (NULL = skip)
 */
int flare_variance(flare_state* state, float* var_atom, float* sigma_atom, float* sigma_max);

/*
 * The mapped quadratic forms (Eqs. 1-2) of given vectors, by the same kernels as the
 * descriptor path for the rows of one environment bucket:
 *   e_r = d_r^T beta_s d_r,   V_r = d_r^T Sigma_s d_r      (no normalisation of d_r)
 * bucket: 0 (H centre, H-only), 1 (Pt, H-only), 2 (H, Pt-only), 3 (Pt, Pt-only): d_r is
 * the 144-wide block of that neighbour species (H-H block, or Pt-Pt block) and beta_s,
 * Sigma_s the matching 144 x 144 blocks; 4 (H, mixed), 5 (Pt, mixed): the full 544 vector.
 * Arithmetic as in flare_energy_forces for the model's precision: in the split forms V is
 * |L^T d|^2 with the FP64 Cholesky factor on the FP64 matrix cores, so a near-cancelling
 * V << sigma_max(Sigma) |d|^2 keeps FP64 accuracy of the form.
 *   d_rows          DEVICE FP32 [n_rows][144 or 544]
 *   e_out, var_out  DEVICE FP32 [n_rows]
 * n_rows <= max_atoms of the state. Grows the state's row buffers when needed and
 * overwrites its resident descriptors (call flare_descriptors again before
 * flare_energy_forces). Not synchronising.
 */
int flare_quadratic_forms(flare_state* state, int bucket, int n_rows, const float* d_rows, float* e_out,
                          float* var_out);

/*
 * Uncertainty monitor of a production run (the paper's Section V.A active-learning
 * trigger and Section VII.B runs, which watch the largest atomic uncertainty against a
 * threshold): from the variances of the positions staged by the last flare_descriptors
 * call (computed here if no earlier call formed them), per cell c
 *   m_c = max_i sigma_i;  sigma_max_run[c] = max(sigma_max_run[c], m_c);
 *   if m_c > threshold: over_count[c] += 1 and the status bit FLARE_FLAG_UNCERTAIN is raised.
 *   sigma_max_run  DEVICE FP32 [n_struct], read and written (start it at 0)
 *   over_count     DEVICE int32 [n_struct], read and written (start it at 0)
 * Not synchronising: the caller reads the arrays, or the status bit through
 * flare_status / flare_interval_status, when it next waits for the stream.
 */
int flare_uncertainty_monitor(flare_state* state, double threshold, float* sigma_max_run,
                              int32_t* over_count);

/*
 * Velocity-Verlet halves on caller arrays (DEVICE FP64 [n_atoms] each; forces FP32).
 *   first:  v += dt/2 * KAPPA * F / m ;  x += dt * v
 *   second: v += dt/2 * KAPPA * F / m
 * KAPPA = 9.648533212e-3 A^2 fs^-2 per eV/amu; masses_host HOST FP64 [n_species].
 */
int flare_md_first_half(flare_state* state, double* x, double* y, double* z, double* vx,
                        double* vy, double* vz, const float* fx, const float* fy,
                        const float* fz, const int32_t* species, const double* masses_host,
                        double dt);
int flare_md_second_half(flare_state* state, double* vx, double* vy, double* vz,
                         const float* fx, const float* fy, const float* fz,
                         const int32_t* species, const double* masses_host, double dt);

/*
 * One whole velocity-Verlet NVE step, the same arithmetic as the sequence
 *   flare_md_first_half; flare_neighbors (when rebuild != 0, with the cells, boxes and skin
 *   of the last flare_neighbors call); flare_descriptors; flare_energy_forces (with
 *   forces); flare_md_second_half
 * and the same results bit for bit, in fewer kernels: the drift also forms the
 * displacements of the new positions, and the caller-order outputs carry the second half.
 *   x, y, z, vx, vy, vz  DEVICE FP64 [n_atoms], read and written
 *   fx, fy, fz           DEVICE FP32 [n_atoms]: in, the forces at the current positions;
 *                        out, the forces at the new positions (required)
 *   e_atom, var_atom, sigma_atom  DEVICE FP32 [n_atoms] or NULL; e_struct DEVICE FP64
 *                        [n_struct] or NULL: the other outputs of flare_energy_forces
 * A rebuild waits for the stream once (as flare_neighbors) and moves the status bits of
 * the interval it ends to flare_interval_status / flare_status; its errors are those of
 * flare_neighbors (positions and velocities are then already advanced by the first half).
 * Without a rebuild the call does not wait.
 */
int flare_md_step(flare_state* state, double* x, double* y, double* z, double* vx, double* vy,
                  double* vz, float* fx, float* fy, float* fz, const int32_t* species,
                  const double* masses_host, double dt, int rebuild, float* e_atom,
                  double* e_struct, float* var_atom, float* sigma_atom);

/*
 * Nose-Hoover NVT halves (the paper's production runs, Section VI.A: 450 K). One
 * thermostat variable zeta per cell, no chain:
 *   dv/dt = KAPPA F/m - zeta v,  dzeta/dt = (2K / (N_f k_B T) - 1) / tau^2,  deta/dt = zeta,
 * N_f = max(3 N_cell - 3, 1), k_B = 8.617333262e-5 eV/K, K the cell's kinetic energy (eV).
 *   first:  zeta += dt/2 G(K); v *= exp(-zeta dt/2); eta += zeta dt/2;
 *           v += dt/2 KAPPA F/m; x += dt v
 *   second: v += dt/2 KAPPA F/m; v *= exp(-zeta dt/2); eta += zeta dt/2; K = sum m v^2/2;
 *           zeta += dt/2 G(K)
 * (time-reversible; H' = E_pot + K + Q zeta^2/2 + N_f k_B T eta with Q = N_f k_B T tau^2
 * is conserved to O(dt^2)).
 *   thermo       DEVICE FP64 [n_struct][3] = (zeta [1/fs], eta, K [eV]) per cell, owned by
 *                the caller: zero zeta and eta to start, and fill K with flare_kinetic.
 *   t_target     K; tau: damping time in fs (> 0; a large tau decouples the thermostat).
 * Arrays as in flare_md_*_half. K is summed in FP64 (compensated) over fixed atom ranges
 * of each cell (deterministic, independent of the other cells).
 */
int flare_nvt_first_half(flare_state* state, double* x, double* y, double* z, double* vx,
                         double* vy, double* vz, const float* fx, const float* fy,
                         const float* fz, const int32_t* species, const double* masses_host,
                         double dt, double t_target, double tau, double* thermo);
int flare_nvt_second_half(flare_state* state, double* vx, double* vy, double* vz,
                          const float* fx, const float* fy, const float* fz,
                          const int32_t* species, const double* masses_host, double dt,
                          double t_target, double tau, double* thermo);
/* Kinetic energy per cell into thermo[c][2] (eV); velocities unchanged. */
int flare_kinetic(flare_state* state, double* vx, double* vy, double* vz, const int32_t* species,
                  const double* masses_host, double* thermo);

/*
 * Hydrogen coordination numbers (Section VI.A): coord[a] = 1 when atom a is H and another
 * H atom is within 1 A (squared FP64 distance of the given positions, moved to the images
 * of the list build, below 1), else 0 (always 0 for other species). A change 1 -> 0
 * between two snapshots is a dissociation, 0 -> 1 a recombination.
 *   x, y, z     DEVICE FP64 [n_atoms] each, caller order: the positions last passed to
 *               flare_descriptors (the list covers them only within half the skin of the
 *               build, which that call checked); read only
 *   coord       DEVICE int32 [n_atoms], caller order (written)
 *   coord_prev  DEVICE int32 [n_atoms] of an earlier snapshot, or NULL
 *   events      DEVICE int64 [n_struct][2] (dissociations, recombinations) per cell
 *               between coord_prev and coord, or NULL (both or neither)
 * Needs the list to cover 1 A (it does: r_list > r_cut > 1 A) and descriptors staged
 * for the current positions (FLARE_E_STALE otherwise).
 */
int flare_coordination(flare_state* state, const double* x, const double* y, const double* z,
                       int32_t* coord, const int32_t* coord_prev, int64_t* events);

/*
 * Stage timers. When enabled, the library records a pair of HIP events on the state's
 * stream around each stage it launches; flare_timers_read (SYNCHRONISING) returns the
 * accumulated milliseconds and launch counts per stage (HOST outputs, FLARE_NTIMERS
 * entries each; either may be NULL) and clears them when reset != 0.
 */
#define FLARE_NTIMERS 9
#define FLARE_T_LIST      0  /* flare_neighbors device work                    */
#define FLARE_T_DESC1     1  /* position gather + descriptors, 144-wide rows    */
#define FLARE_T_DESCX     2  /* descriptors, 544-wide (mixed) rows              */
#define FLARE_T_QFORM1    3  /* quadratic forms on the matrix cores, 144 rows   */
#define FLARE_T_QFORMX    4  /* quadratic forms, 544 rows (GEMM + finish)       */
#define FLARE_T_FORCE1    5  /* adjoint forces, 144 rows (incl. force clear)    */
#define FLARE_T_FORCEX    6  /* adjoint forces, 544 rows                        */
#define FLARE_T_OUT       7  /* caller-order outputs and per-cell reductions    */
#define FLARE_T_MD        8  /* integrator halves                              */
int flare_timers_enable(flare_state* state, int on);
int flare_timers_read(flare_state* state, double* ms, long long* counts, int reset);

/* Device memory held by the model (model may be NULL) and the state, in bytes (HOST). */
int flare_memory_bytes(const flare_model* model, const flare_state* state, long long* bytes);

/* Read and clear the status bits raised since the previous flare_status call
 * (SYNCHRONISING). flags_host: HOST int32. The bits are sticky: a list build moves the
 * device word to the host at its synchronisation point and does not drop it, so a bit
 * raised in any interval between two list builds is returned here. */
int flare_status(flare_state* state, int32_t* flags_host);

/* The status bits raised between the previous list build (or flare_status call) and the
 * last flare_neighbors call, i.e. during the interval that call ended (not synchronising:
 * flare_neighbors read them at its own synchronisation point). They stay pending for
 * flare_status as well. An MD driver checks FLARE_FLAG_DISPLACED | FLARE_FLAG_NONFINITE
 * here after every rebuild. flags_host: HOST int32. */
int flare_interval_status(const flare_state* state, int32_t* flags_host);

#ifdef __cplusplus
}
#endif

#endif /* FLARE_H */
