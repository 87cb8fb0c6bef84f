// Outputs in the caller's atom order, per-cell reductions and the velocity-Verlet halves.
//
// Per-cell energy E = sum_i e_i is accumulated in FP64 with Neumaier compensation, over
// fixed atom ranges in a fixed order (deterministic for given e_i). The per-cell
// maximum uncertainty is the largest sigma_i = sqrt(max(V_i, 0)).
#include "state.h"

namespace flare {
namespace {

constexpr int NT = 256;

// Outputs in two coalesced passes. Rows (row order): F_i = sum_k w(i,k) - sum_k
// w_in(slot(i,k)), the first sum (the row's own pair terms) formed by the adjoint as f_own,
// the second over the row's own pairs k < count in slot order (deterministic), written with
// e_i as one 16-byte record per row. Atoms (caller order): each atom reads its row's record
// and variance and writes every requested output; atoms without a row get zeros.
__global__ __launch_bounds__(NT) void k_outputs_rows(int rows, int want_f, const int* __restrict__ slice_base,
                                                     const float4* __restrict__ f_own,
                                                     const float4* __restrict__ w_in,
                                                     const int* __restrict__ cnt_row,
                                                     const int* __restrict__ sid_row,
                                                     const double* __restrict__ cell_scale,
                                                     const float* __restrict__ e_row,
                                                     float4* __restrict__ row_out) {
  const int R = xcd_remap(blockIdx.x, gridDim.x) * NT + threadIdx.x;
  if (R >= rows) return;
  float sx = 0.f, sy = 0.f, sz = 0.f;
  if (want_f) {
    const int base = slice_base[R >> 5], len = cnt_row[R];   // the row's own pairs (no padding)
    const float4* wp = w_in + (size_t)base * 32 + (R & 31);
    float rx = 0.f, ry = 0.f, rz = 0.f;
    int k = 0;
    // four loads in flight at a time; the sums stay in slot order
    for (; k + 4 <= len; k += 4) {
      float4 wr[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) wr[u] = wp[(size_t)(k + u) * 32];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        rx += wr[u].x;
        ry += wr[u].y;
        rz += wr[u].z;
      }
    }
    for (; k < len; ++k) {
      const float4 wr = wp[(size_t)k * 32];
      rx += wr.x;
      ry += wr.y;
      rz += wr.z;
    }
    const float4 fo = f_own[R];
    sx = fo.x - rx;
    sy = fo.y - ry;
    sz = fo.z - rz;
    if (cell_scale) {
      const float k = (float)cell_scale[sid_row[R]];
      sx *= k;
      sy *= k;
      sz *= k;
    }
  }
  row_out[R] = make_float4(sx, sy, sz, e_row[R]);
}

__global__ __launch_bounds__(NT) void k_outputs_atoms(int n, const int* __restrict__ row_caller,
                                                      const float4* __restrict__ row_out,
                                                      const float* __restrict__ v_row,
                                                      float* __restrict__ e_atom, float* __restrict__ fx,
                                                      float* __restrict__ fy, float* __restrict__ fz,
                                                      float* __restrict__ var_atom,
                                                      float* __restrict__ sigma_atom) {
  const int a = blockIdx.x * NT + threadIdx.x;
  if (a >= n) return;
  const int R = row_caller[a];
  float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
  float v = 0.f;
  if (R >= 0) {
    o = row_out[R];
    if (var_atom || sigma_atom) v = v_row[R];
  }
  if (e_atom) e_atom[a] = o.w;
  if (fx) {
    fx[a] = o.x;
    fy[a] = o.y;
    fz[a] = o.z;
  }
  if (var_atom) var_atom[a] = v;
  if (sigma_atom) sigma_atom[a] = sqrtf(fmaxf(v, 0.f));
}

__device__ inline void two_sum_add(double& s, double& c, double x) {
  const double t = s + x;
  if (fabs(s) >= fabs(x)) c += (s - t) + x;
  else c += (x - t) + s;
  s = t;
}

// One block per task: compensated FP64 sum of e and max of sigma over [begin, end).
__global__ __launch_bounds__(NT) void k_reduce_tasks(const RedTask* __restrict__ tasks,
                                                     const int* __restrict__ bucket,
                                                     const float* __restrict__ e_int,
                                                     const float* __restrict__ v_int,
                                                     int want_e, int want_s,
                                                     double* __restrict__ red_e,
                                                     float* __restrict__ red_s) {
  __shared__ double ss[NT], sc[NT];
  __shared__ float sm[NT];
  const RedTask tk = tasks[blockIdx.x];
  double s = 0.0, c = 0.0;
  float mx = 0.f;
  for (int i = tk.begin + threadIdx.x; i < tk.end; i += NT) {
    if (bucket[i] < 0) continue;
    if (want_e) two_sum_add(s, c, (double)e_int[i]);
    if (want_s) mx = fmaxf(mx, sqrtf(fmaxf(v_int[i], 0.f)));
  }
  ss[threadIdx.x] = s;
  sc[threadIdx.x] = c;
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      double s2 = ss[threadIdx.x], c2 = sc[threadIdx.x] + sc[threadIdx.x + h];
      two_sum_add(s2, c2, ss[threadIdx.x + h]);
      ss[threadIdx.x] = s2;
      sc[threadIdx.x] = c2;
      sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    red_e[2 * blockIdx.x] = ss[0];
    red_e[2 * blockIdx.x + 1] = sc[0];
    red_s[blockIdx.x] = sm[0];
  }
}

// One wave per cell: its tasks [first_task[c], first_task[c + 1]) are folded by the 64
// lanes in a fixed stride, then combined in a fixed tree (deterministic).
constexpr int NC = 64;

// With a monitor (run_max != nullptr) the cell's largest sigma also updates its running
// maximum, and a value above the threshold counts in over[cell] and raises the status bit.
__global__ __launch_bounds__(NC) void k_reduce_cells(const double* __restrict__ red_e,
                                                     const float* __restrict__ red_s,
                                                     const int* __restrict__ first_task,
                                                     double* __restrict__ e_struct,
                                                     float* __restrict__ sigma_max, float thr,
                                                     float* __restrict__ run_max,
                                                     int* __restrict__ over,
                                                     int* __restrict__ status) {
  __shared__ double ss[NC], sc[NC];
  __shared__ float sm[NC];
  const int cell = blockIdx.x, t = threadIdx.x;
  double s = 0.0, c = 0.0;
  float mx = 0.f;
  for (int k = first_task[cell] + t; k < first_task[cell + 1]; k += NC) {
    two_sum_add(s, c, red_e[2 * k]);
    c += red_e[2 * k + 1];
    mx = fmaxf(mx, red_s[k]);
  }
  ss[t] = s;
  sc[t] = c;
  sm[t] = mx;
  __syncthreads();
  for (int h = NC / 2; h > 0; h >>= 1) {
    if (t < h) {
      double s2 = ss[t], c2 = sc[t] + sc[t + h];
      two_sum_add(s2, c2, ss[t + h]);
      ss[t] = s2;
      sc[t] = c2;
      sm[t] = fmaxf(sm[t], sm[t + h]);
    }
    __syncthreads();
  }
  if (t == 0) {
    if (e_struct) e_struct[cell] = ss[0] + sc[0];
    if (sigma_max) sigma_max[cell] = sm[0];
    if (run_max) {
      run_max[cell] = fmaxf(run_max[cell], sm[0]);
      if (sm[0] > thr) {
        over[cell] += 1;
        atomicOr(status, FLARE_FLAG_UNCERTAIN);
      }
    }
  }
}

// Virial of one reduction task (a contiguous internal atom range of one cell): per atom
// the nine products over its own pairs in slot order, summed in FP32; then the atoms of
// the task in FP64 in a fixed order. The cell's W = -sum_p Delta_p (x) w_p runs over all its
// pairs; the reverse q of p has Delta_q = -Delta_p and w_in(slot p) = w_q, so relabelling the
// sum gives W = sum_p Delta_p (x) w_in(slot p), which each atom forms from its own slots
// (Delta = r u from the geometry). red_w [tasks][9] holds the task sums.
__global__ __launch_bounds__(NT) void k_virial_tasks(const RedTask* __restrict__ tasks,
                                                     const int* __restrict__ bucket,
                                                     const int* __restrict__ row_of, int rows1,
                                                     const int* __restrict__ slice_base,
                                                     const float4* __restrict__ geom,
                                                     const float4* __restrict__ w_in,
                                                     const int* __restrict__ cnt,
                                                     double* __restrict__ red_w) {
  __shared__ double sw[9][NT];
  const RedTask tk = tasks[blockIdx.x];
  double acc[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) acc[c] = 0.0;
  for (int i = tk.begin + threadIdx.x; i < tk.end; i += NT) {
    const int b = bucket[i];
    if (b < 0) continue;
    const int R = b < 4 ? row_of[i] : rows1 + row_of[i];
    const int base = slice_base[R >> 5], len = cnt[i];
    float va[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) va[c] = 0.f;
    for (int k = 0; k < len; ++k) {
      const int slot = (base + k) * 32 + (R & 31);
      const float4 g = geom[slot];
      const float4 wk = w_in[slot];
      const float r = fabsf(g.w);      // 0 outside the cutoff: no contribution
      const float d[3] = {r * g.x, r * g.y, r * g.z};
      const float ww[3] = {wk.x, wk.y, wk.z};
#pragma unroll
      for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) va[3 * x + y] += d[x] * ww[y];
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c] += (double)va[c];
  }
#pragma unroll
  for (int c = 0; c < 9; ++c) sw[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
#pragma unroll
      for (int c = 0; c < 9; ++c) sw[c][threadIdx.x] += sw[c][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x < 9) red_w[(size_t)blockIdx.x * 9 + threadIdx.x] = sw[threadIdx.x][0];
}

__global__ __launch_bounds__(NC) void k_virial_cells(const double* __restrict__ red_w,
                                                     const int* __restrict__ first_task,
                                                     double* __restrict__ out) {
  __shared__ double sw[9][NC];
  const int cell = blockIdx.x, t = threadIdx.x;
  double acc[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) acc[c] = 0.0;
  for (int k = first_task[cell] + t; k < first_task[cell + 1]; k += NC)
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c] += red_w[(size_t)k * 9 + c];
#pragma unroll
  for (int c = 0; c < 9; ++c) sw[c][t] = acc[c];
  __syncthreads();
  for (int h = NC / 2; h > 0; h >>= 1) {
    if (t < h) {
#pragma unroll
      for (int c = 0; c < 9; ++c) sw[c][t] += sw[c][t + h];
    }
    __syncthreads();
  }
  if (t < 9) out[(size_t)cell * 9 + t] = sw[t][0];
}

constexpr double KAPPA = 9.648533212e-3;   // (eV/A)/amu in A/fs^2

__global__ __launch_bounds__(NT) void k_md_first(int n, double* __restrict__ x, double* __restrict__ y,
                                                 double* __restrict__ z, double* __restrict__ vx,
                                                 double* __restrict__ vy, double* __restrict__ vz,
                                                 const float* __restrict__ fx,
                                                 const float* __restrict__ fy,
                                                 const float* __restrict__ fz,
                                                 const int32_t* __restrict__ species, double h0,
                                                 double h1, double dt) {
  const int a = blockIdx.x * NT + threadIdx.x;
  if (a >= n) return;
  const double h = species[a] == 0 ? h0 : h1;    // dt/2 * KAPPA / m
  const double ux = vx[a] + h * (double)fx[a];
  const double uy = vy[a] + h * (double)fy[a];
  const double uz = vz[a] + h * (double)fz[a];
  vx[a] = ux;
  vy[a] = uy;
  vz[a] = uz;
  x[a] += dt * ux;
  y[a] += dt * uy;
  z[a] += dt * uz;
}

// The first half and drift of a step (as k_md_first) with, when the list stays, the
// displacement of each new position since the list build (as k_disp).
__global__ __launch_bounds__(NT) void k_md_first_drift(int n, double* __restrict__ x, double* __restrict__ y,
                                                       double* __restrict__ z, double* __restrict__ vx,
                                                       double* __restrict__ vy, double* __restrict__ vz,
                                                       const float* __restrict__ fx, const float* __restrict__ fy,
                                                       const float* __restrict__ fz,
                                                       const int32_t* __restrict__ species, double h0, double h1,
                                                       double dt, int disp, const double* __restrict__ xb,
                                                       const int* __restrict__ inv_perm, float4* __restrict__ dlt,
                                                       double lim2, int* __restrict__ status) {
  const int a = blockIdx.x * NT + threadIdx.x;
  if (a >= n) return;
  const double h = species[a] == 0 ? h0 : h1;    // dt/2 * KAPPA / m
  const double ux = vx[a] + h * (double)fx[a];
  const double uy = vy[a] + h * (double)fy[a];
  const double uz = vz[a] + h * (double)fz[a];
  vx[a] = ux;
  vy[a] = uy;
  vz[a] = uz;
  const double px = x[a] + dt * ux, py = y[a] + dt * uy, pz = z[a] + dt * uz;
  x[a] = px;
  y[a] = py;
  z[a] = pz;
  if (disp) store_displacement(a, n, px, py, pz, xb, inv_perm, dlt, lim2, status);
}

// The caller-order outputs (as k_outputs_atoms) and the second half of the step with the
// new forces (as k_md_second).
__global__ __launch_bounds__(NT) void k_outputs_second_half(int n, const int* __restrict__ row_caller,
                                                            const float4* __restrict__ row_out,
                                                            const float* __restrict__ v_row,
                                                            float* __restrict__ e_atom, float* __restrict__ fx,
                                                            float* __restrict__ fy, float* __restrict__ fz,
                                                            float* __restrict__ var_atom,
                                                            float* __restrict__ sigma_atom,
                                                            double* __restrict__ vx, double* __restrict__ vy,
                                                            double* __restrict__ vz,
                                                            const int32_t* __restrict__ species, double h0,
                                                            double h1) {
  const int a = blockIdx.x * NT + threadIdx.x;
  if (a >= n) return;
  const int R = row_caller[a];
  float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
  float v = 0.f;
  if (R >= 0) {
    o = row_out[R];
    if (var_atom || sigma_atom) v = v_row[R];
  }
  if (e_atom) e_atom[a] = o.w;
  fx[a] = o.x;
  fy[a] = o.y;
  fz[a] = o.z;
  if (var_atom) var_atom[a] = v;
  if (sigma_atom) sigma_atom[a] = sqrtf(fmaxf(v, 0.f));
  const double h = species[a] == 0 ? h0 : h1;
  vx[a] += h * (double)o.x;
  vy[a] += h * (double)o.y;
  vz[a] += h * (double)o.z;
}

__global__ __launch_bounds__(NT) void k_md_second(int n, double* __restrict__ vx,
                                                  double* __restrict__ vy, double* __restrict__ vz,
                                                  const float* __restrict__ fx,
                                                  const float* __restrict__ fy,
                                                  const float* __restrict__ fz,
                                                  const int32_t* __restrict__ species, double h0,
                                                  double h1) {
  const int a = blockIdx.x * NT + threadIdx.x;
  if (a >= n) return;
  const double h = species[a] == 0 ? h0 : h1;
  vx[a] += h * (double)fx[a];
  vy[a] += h * (double)fy[a];
  vz[a] += h * (double)fz[a];
}

}  // namespace

void finalize_outputs(flare_state* s, float* e_atom, float* fx, float* fy, float* fz,
                      float* var_atom, float* sigma_atom, const double* cell_scale) {
  const int n = s->n_atoms;
  if (n == 0) return;
  const int rows = s->rows1 + s->rowsx;
  if (rows > 0)
    k_outputs_rows<<<(rows + NT - 1) / NT, NT, 0, s->stream>>>(rows, fx != nullptr, s->slice_base, s->f_own,
                                                              s->w_in, s->cnt_row, s->sid_row, cell_scale,
                                                              s->e_row, s->row_out);
  k_outputs_atoms<<<(n + NT - 1) / NT, NT, 0, s->stream>>>(n, s->row_caller, s->row_out, s->v_row, e_atom, fx,
                                                           fy, fz, var_atom, sigma_atom);
}

void reduce_cells(flare_state* s, double* e_struct, float* sigma_max, float thr, float* run_max, int* over) {
  if (!e_struct && !sigma_max && !run_max) return;
  const int nt = (int)s->tasks.size();
  if (nt == 0) return;
  k_reduce_tasks<<<nt, NT, 0, s->stream>>>(s->d_tasks, s->bucket, s->e_int, s->v_int, e_struct != nullptr,
                                           sigma_max != nullptr || run_max != nullptr, s->red_e, s->red_s);
  if (s->n_struct > 0)
    k_reduce_cells<<<s->n_struct, NC, 0, s->stream>>>(s->red_e, s->red_s, s->d_first_task, e_struct,
                                                      sigma_max, thr, run_max, over, s->d_status);
}

void virial_cells(flare_state* s, double* virial_struct, double* red_w) {
  const int nt = (int)s->tasks.size();
  if (nt > 0)
    k_virial_tasks<<<nt, NT, 0, s->stream>>>(s->d_tasks, s->bucket, s->row_of, s->rows1, s->slice_base,
                                             s->geom, s->w_in, s->nl_cnt, red_w);
  if (s->n_struct > 0)
    k_virial_cells<<<s->n_struct, NC, 0, s->stream>>>(red_w, s->d_first_task, virial_struct);
}

void md_first(flare_state* s, double* x, double* y, double* z, double* vx, double* vy, double* vz,
              const float* fx, const float* fy, const float* fz, const int32_t* species,
              double inv_m0, double inv_m1, double dt) {
  const int n = s->n_atoms;
  if (n == 0) return;
  const double h0 = 0.5 * dt * KAPPA * inv_m0, h1 = 0.5 * dt * KAPPA * inv_m1;
  k_md_first<<<(n + NT - 1) / NT, NT, 0, s->stream>>>(n, x, y, z, vx, vy, vz, fx, fy, fz, species, h0, h1, dt);
}

void md_first_drift(flare_state* s, double* x, double* y, double* z, double* vx, double* vy, double* vz,
                    const float* fx, const float* fy, const float* fz, const int32_t* species, double inv_m0,
                    double inv_m1, double dt, bool displacements) {
  const int n = s->n_atoms;
  if (n == 0) return;
  const double h0 = 0.5 * dt * KAPPA * inv_m0, h1 = 0.5 * dt * KAPPA * inv_m1;
  const double lim = 0.5 * s->skin;
  k_md_first_drift<<<(n + NT - 1) / NT, NT, 0, s->stream>>>(n, x, y, z, vx, vy, vz, fx, fy, fz, species, h0, h1,
                                                            dt, displacements ? 1 : 0, s->xb, s->inv_perm, s->dlt,
                                                            lim * lim, s->d_status);
}

void outputs_second_half(flare_state* s, float* e_atom, float* fx, float* fy, float* fz, float* var_atom,
                         float* sigma_atom, double* vx, double* vy, double* vz, const int32_t* species,
                         double inv_m0, double inv_m1, double dt) {
  const int n = s->n_atoms;
  if (n == 0) return;
  const int rows = s->rows1 + s->rowsx;
  if (rows > 0)
    k_outputs_rows<<<(rows + NT - 1) / NT, NT, 0, s->stream>>>(rows, 1, s->slice_base, s->f_own, s->w_in,
                                                              s->cnt_row, s->sid_row, nullptr, s->e_row,
                                                              s->row_out);
  const double h0 = 0.5 * dt * KAPPA * inv_m0, h1 = 0.5 * dt * KAPPA * inv_m1;
  k_outputs_second_half<<<(n + NT - 1) / NT, NT, 0, s->stream>>>(n, s->row_caller, s->row_out, s->v_row, e_atom,
                                                                 fx, fy, fz, var_atom, sigma_atom, vx, vy, vz,
                                                                 species, h0, h1);
}

void md_second(flare_state* s, double* vx, double* vy, double* vz, const float* fx, const float* fy,
               const float* fz, const int32_t* species, double inv_m0, double inv_m1, double dt) {
  const int n = s->n_atoms;
  if (n == 0) return;
  const double h0 = 0.5 * dt * KAPPA * inv_m0, h1 = 0.5 * dt * KAPPA * inv_m1;
  k_md_second<<<(n + NT - 1) / NT, NT, 0, s->stream>>>(n, vx, vy, vz, fx, fy, fz, species, h0, h1);
}

}  // namespace flare
