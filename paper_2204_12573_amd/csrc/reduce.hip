// Outputs in the caller's atom order, per-cell reductions and the velocity-Verlet halves.
//
// Per-cell energy E = sum_i e_i is accumulated in FP64 with Neumaier compensation, over
// fixed atom ranges in a fixed order (deterministic for given e_i). The per-cell
// maximum uncertainty is the largest sigma_i = sqrt(max(V_i, 0)).
#include "state.h"

namespace flare {
namespace {

constexpr int NT = 256;

// Caller-order outputs. Forces by gathering the per-pair adjoint terms:
// F_i = sum_{p in list(i)} (w_p - w_rev(p)), in list order (deterministic).
__global__ __launch_bounds__(NT) void k_outputs(int n, const int* __restrict__ perm,
                                                const int* __restrict__ bucket,
                                                const int* __restrict__ nl_off,
                                                const int* __restrict__ rev,
                                                const float* __restrict__ w, long long P,
                                                const float* __restrict__ e_int,
                                                const float* __restrict__ v_int,
                                                float* __restrict__ e_atom, float* __restrict__ fx,
                                                float* __restrict__ fy, float* __restrict__ fz,
                                                float* __restrict__ var_atom,
                                                float* __restrict__ sigma_atom) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const int a = perm[i];
  const bool has = bucket[i] >= 0;
  if (e_atom) e_atom[a] = has ? e_int[i] : 0.f;
  if (fx) {
    float sx = 0.f, sy = 0.f, sz = 0.f;
    for (int p = nl_off[i]; p < nl_off[i + 1]; ++p) {
      const int q = rev[p];
      sx += w[p] - w[q];
      sy += w[P + p] - w[P + q];
      sz += w[2 * P + p] - w[2 * P + q];
    }
    fx[a] = sx;
    fy[a] = sy;
    fz[a] = sz;
  }
  const float v = has ? v_int[i] : 0.f;
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

// One thread per cell: fold its tasks in order.
__global__ __launch_bounds__(NT) void k_reduce_cells(int ntask, const RedTask* __restrict__ tasks,
                                                     const double* __restrict__ red_e,
                                                     const float* __restrict__ red_s,
                                                     const int* __restrict__ first_task, int ncell,
                                                     double* __restrict__ e_struct,
                                                     float* __restrict__ sigma_max) {
  const int cell = blockIdx.x * NT + threadIdx.x;
  if (cell >= ncell) return;
  double s = 0.0, c = 0.0;
  float mx = 0.f;
  for (int k = first_task[cell]; k < ntask && tasks[k].cell == cell; ++k) {
    two_sum_add(s, c, red_e[2 * k]);
    c += red_e[2 * k + 1];
    mx = fmaxf(mx, red_s[k]);
  }
  if (e_struct) e_struct[cell] = s + c;
  if (sigma_max) sigma_max[cell] = mx;
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
                      float* var_atom, float* sigma_atom) {
  const int n = s->n_atoms;
  if (n == 0) return;
  k_outputs<<<(n + NT - 1) / NT, NT, 0, s->stream>>>(n, s->perm, s->bucket, s->nl_off, s->nl_rev, s->w_pair,
                                                     s->max_pairs, s->e_int, s->v_int, e_atom, fx, fy, fz,
                                                     var_atom, sigma_atom);
}

void reduce_cells(flare_state* s, double* e_struct, float* sigma_max) {
  if (!e_struct && !sigma_max) return;
  const int nt = (int)s->tasks.size();
  if (nt == 0) return;
  k_reduce_tasks<<<nt, NT, 0, s->stream>>>(s->d_tasks.p, s->bucket, s->e_int, s->v_int, e_struct != nullptr,
                                           sigma_max != nullptr, s->red_e.p, s->red_s.p);
  k_reduce_cells<<<(s->n_struct + NT - 1) / NT, NT, 0, s->stream>>>(
      nt, s->d_tasks.p, s->red_e.p, s->red_s.p, s->d_first_task.p, s->n_struct, e_struct, sigma_max);
}

void md_first(flare_state* s, double* x, double* y, double* z, double* vx, double* vy, double* vz,
              const float* fx, const float* fy, const float* fz, const int32_t* species,
              double inv_m0, double inv_m1, double dt) {
  const int n = s->n_atoms;
  if (n == 0) return;
  const double h0 = 0.5 * dt * KAPPA * inv_m0, h1 = 0.5 * dt * KAPPA * inv_m1;
  k_md_first<<<(n + NT - 1) / NT, NT, 0, s->stream>>>(n, x, y, z, vx, vy, vz, fx, fy, fz, species, h0, h1, dt);
}

void md_second(flare_state* s, double* vx, double* vy, double* vz, const float* fx, const float* fy,
               const float* fz, const int32_t* species, double inv_m0, double inv_m1, double dt) {
  const int n = s->n_atoms;
  if (n == 0) return;
  const double h0 = 0.5 * dt * KAPPA * inv_m0, h1 = 0.5 * dt * KAPPA * inv_m1;
  k_md_second<<<(n + NT - 1) / NT, NT, 0, s->stream>>>(n, vx, vy, vz, fx, fy, fz, species, h0, h1);
}

}  // namespace flare
