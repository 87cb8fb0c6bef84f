// Production-run pieces of the paper's Section VI.A: a Nose-Hoover thermostat per cell
// around the velocity-Verlet halves, and hydrogen coordination numbers with the reaction
// events they imply.
//
// Nose-Hoover (one thermostat variable per cell, no chain): dv/dt = KAPPA F/m - zeta v,
// dzeta/dt = G(K) = (2K / (N_f k_B T0) - 1) / tau^2, deta/dt = zeta, N_f = max(3N - 3, 1).
// One time step is the time-reversible splitting
//   zeta += dt/2 G(K); v *= exp(-zeta dt/2); eta += zeta dt/2; v += dt/2 a; x += dt v
//   [forces]  v += dt/2 a; v *= exp(-zeta dt/2); eta += zeta dt/2; K = sum m v^2 / 2;
//   zeta += dt/2 G(K)
// with the per-cell state (zeta, eta, K) on the device. K is summed in FP64 with Neumaier
// compensation over the same fixed atom ranges (tasks) as the energies, so a cell's
// trajectory does not depend on the other cells of the batch.
//
// Coordination of an H atom: 1 when another H atom is within 1 A (squared FP64 distance of
// the current positions below 1), else 0; 0 for other species. The list radius exceeds
// 1 A, so the listed pairs hold every candidate.
#include "state.h"

namespace flare {
namespace {

constexpr int NT = 256;
constexpr int NC = 64;
constexpr double KAPPA = 9.648533212e-3;   // (eV/A)/amu in A/fs^2
constexpr double KB = 8.617333262e-5;      // eV/K

__device__ inline void two_sum_add(double& s, double& c, double x) {
  const double t = s + x;
  if (fabs(s) >= fabs(x)) c += (s - t) + x;
  else c += (x - t) + s;
  s = t;
}

__device__ inline double nh_force(double kin, int n_atoms, double t0, double tau) {
  const double nf = (double)max(3 * n_atoms - 3, 1);
  return (2.0 * kin / (nf * KB * t0) - 1.0) / (tau * tau);
}

// thermo[3c] = zeta, [3c+1] = eta, [3c+2] = K of cell c
__global__ void k_nh_open(int ncell, const int* __restrict__ struct_off, double* __restrict__ thermo, double dt,
                          double t0, double tau) {
  const int c = blockIdx.x * NC + threadIdx.x;
  if (c >= ncell) return;
  const int n = struct_off[c + 1] - struct_off[c];
  double zeta = thermo[3 * c];
  if (n > 0) zeta += 0.5 * dt * nh_force(thermo[3 * c + 2], n, t0, tau);
  thermo[3 * c] = zeta;
  thermo[3 * c + 1] += 0.5 * dt * zeta;
}

// one block per task (an atom range inside one cell): scale by exp(-zeta dt/2), kick, drift
__global__ __launch_bounds__(NT) void k_nvt_first(const RedTask* __restrict__ tasks, double* __restrict__ x,
                                                  double* __restrict__ y, double* __restrict__ z,
                                                  double* __restrict__ vx, double* __restrict__ vy,
                                                  double* __restrict__ vz, const float* __restrict__ fx,
                                                  const float* __restrict__ fy, const float* __restrict__ fz,
                                                  const int32_t* __restrict__ species,
                                                  const double* __restrict__ thermo, double h0, double h1,
                                                  double dt) {
  const RedTask tk = tasks[blockIdx.x];
  const double sc = exp(-0.5 * dt * thermo[3 * tk.cell]);
  for (int a = tk.begin + threadIdx.x; a < tk.end; a += NT) {
    const double h = species[a] == 0 ? h0 : h1;    // dt/2 * KAPPA / m
    const double ux = sc * vx[a] + h * (double)fx[a];
    const double uy = sc * vy[a] + h * (double)fy[a];
    const double uz = sc * vz[a] + h * (double)fz[a];
    vx[a] = ux;
    vy[a] = uy;
    vz[a] = uz;
    x[a] += dt * ux;
    y[a] += dt * uy;
    z[a] += dt * uz;
  }
}

// one block per task: kick and scale (when `update`), then the task's kinetic energy
// (sum, compensation) into red[2 * task]
__global__ __launch_bounds__(NT) void k_nvt_second(const RedTask* __restrict__ tasks, double* __restrict__ vx,
                                                   double* __restrict__ vy, double* __restrict__ vz,
                                                   const float* __restrict__ fx, const float* __restrict__ fy,
                                                   const float* __restrict__ fz,
                                                   const int32_t* __restrict__ species,
                                                   const double* __restrict__ thermo, double h0, double h1,
                                                   double m0, double m1, double dt, int update,
                                                   double* __restrict__ red) {
  __shared__ double ss[NT], sc2[NT];
  const RedTask tk = tasks[blockIdx.x];
  const double sc = update ? exp(-0.5 * dt * thermo[3 * tk.cell]) : 1.0;
  double s = 0.0, c = 0.0;
  for (int a = tk.begin + threadIdx.x; a < tk.end; a += NT) {
    const bool hyd = species[a] == 0;
    double ux = vx[a], uy = vy[a], uz = vz[a];
    if (update) {
      const double h = hyd ? h0 : h1;
      ux = (ux + h * (double)fx[a]) * sc;
      uy = (uy + h * (double)fy[a]) * sc;
      uz = (uz + h * (double)fz[a]) * sc;
      vx[a] = ux;
      vy[a] = uy;
      vz[a] = uz;
    }
    two_sum_add(s, c, 0.5 * (hyd ? m0 : m1) * (ux * ux + uy * uy + uz * uz) / KAPPA);
  }
  ss[threadIdx.x] = s;
  sc2[threadIdx.x] = c;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      double s2 = ss[threadIdx.x], c2 = sc2[threadIdx.x] + sc2[threadIdx.x + h];
      two_sum_add(s2, c2, ss[threadIdx.x + h]);
      ss[threadIdx.x] = s2;
      sc2[threadIdx.x] = c2;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    red[2 * blockIdx.x] = ss[0];
    red[2 * blockIdx.x + 1] = sc2[0];
  }
}

// one wave per cell: K from its tasks in a fixed order; with `update`, close the step
// (eta += zeta dt/2, zeta += dt/2 G(K))
__global__ __launch_bounds__(NC) void k_nh_close(const double* __restrict__ red, const int* __restrict__ first_task,
                                                 const int* __restrict__ struct_off, double* __restrict__ thermo,
                                                 double dt, double t0, double tau, int update) {
  __shared__ double ss[NC], sc[NC];
  const int cell = blockIdx.x, t = threadIdx.x;
  double s = 0.0, c = 0.0;
  for (int k = first_task[cell] + t; k < first_task[cell + 1]; k += NC) {
    two_sum_add(s, c, red[2 * k]);
    c += red[2 * k + 1];
  }
  ss[t] = s;
  sc[t] = c;
  __syncthreads();
  for (int h = NC / 2; h > 0; h >>= 1) {
    if (t < h) {
      double s2 = ss[t], c2 = sc[t] + sc[t + h];
      two_sum_add(s2, c2, ss[t + h]);
      ss[t] = s2;
      sc[t] = c2;
    }
    __syncthreads();
  }
  if (t == 0) {
    const double kin = ss[0] + sc[0];
    thermo[3 * cell + 2] = kin;
    if (update) {
      const int n = struct_off[cell + 1] - struct_off[cell];
      double zeta = thermo[3 * cell];
      thermo[3 * cell + 1] += 0.5 * dt * zeta;
      if (n > 0) zeta += 0.5 * dt * nh_force(kin, n, t0, tau);
      thermo[3 * cell] = zeta;
    }
  }
}

// coordination of every atom (internal index i, written in caller order); positions are
// the caller's FP64 ones moved to the atom's image, x + off, exactly as staged for the step
__global__ __launch_bounds__(NT) void k_coord(int n, const int* __restrict__ perm, const int* __restrict__ sp,
                                              const int* __restrict__ sid, const CellGrid* __restrict__ grids,
                                              const double* __restrict__ x, const double* __restrict__ y,
                                              const double* __restrict__ z, const double* __restrict__ off,
                                              const int* __restrict__ nl_off, const int* __restrict__ nl_j,
                                              const int32_t* __restrict__ nl_s, int32_t* __restrict__ coord) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  int c = 0;
  if (sp[i] == 0) {
    const CellGrid* g = grids + sid[i];
    const int a = perm[i];
    const double pix = x[a] + off[i], piy = y[a] + off[(size_t)n + i], piz = z[a] + off[2 * (size_t)n + i];
    for (int p = nl_off[i]; p < nl_off[i + 1] && c == 0; ++p) {
      const int j = nl_j[p];
      if (sp[j] != 0) continue;
      int sx, sy, sz;
      unpack_shift(nl_s[p], sx, sy, sz);
      const int b = perm[j];
      const double pjx = x[b] + off[j], pjy = y[b] + off[(size_t)n + j], pjz = z[b] + off[2 * (size_t)n + j];
      const double dx = (pjx - pix) + (double)sx * g->L[0];
      const double dy = (pjy - piy) + (double)sy * g->L[1];
      const double dz = (pjz - piz) + (double)sz * g->L[2];
      if (dx * dx + dy * dy + dz * dz < 1.0) c = 1;
    }
  }
  coord[perm[i]] = c;
}

// one block per task: (1 -> 0, 0 -> 1) transitions into red[2 * task] (exact in FP64)
__global__ __launch_bounds__(NT) void k_events_tasks(const RedTask* __restrict__ tasks,
                                                     const int32_t* __restrict__ prev,
                                                     const int32_t* __restrict__ now, double* __restrict__ red) {
  __shared__ int sd[NT], sr[NT];
  const RedTask tk = tasks[blockIdx.x];
  int d = 0, r = 0;
  for (int a = tk.begin + threadIdx.x; a < tk.end; a += NT) {
    d += (prev[a] == 1 && now[a] == 0) ? 1 : 0;
    r += (prev[a] == 0 && now[a] == 1) ? 1 : 0;
  }
  sd[threadIdx.x] = d;
  sr[threadIdx.x] = r;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      sd[threadIdx.x] += sd[threadIdx.x + h];
      sr[threadIdx.x] += sr[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    red[2 * blockIdx.x] = (double)sd[0];
    red[2 * blockIdx.x + 1] = (double)sr[0];
  }
}

__global__ void k_events_cells(int ncell, const double* __restrict__ red, const int* __restrict__ first_task,
                               int64_t* __restrict__ events) {
  const int c = blockIdx.x * NC + threadIdx.x;
  if (c >= ncell) return;
  long long d = 0, r = 0;
  for (int k = first_task[c]; k < first_task[c + 1]; ++k) {
    d += (long long)red[2 * k];
    r += (long long)red[2 * k + 1];
  }
  events[2 * c] = d;
  events[2 * c + 1] = r;
}

}  // namespace

void nvt_first(flare_state* s, double* x, double* y, double* z, double* vx, double* vy, double* vz,
               const float* fx, const float* fy, const float* fz, const int32_t* species, const double* masses,
               double dt, double t0, double tau, double* thermo) {
  const int nc = s->n_struct, nt = (int)s->tasks.size();
  if (nc > 0) k_nh_open<<<(nc + NC - 1) / NC, NC, 0, s->stream>>>(nc, s->d_struct_off, thermo, dt, t0, tau);
  const double h0 = 0.5 * dt * KAPPA / masses[0], h1 = 0.5 * dt * KAPPA / masses[1];
  if (nt > 0)
    k_nvt_first<<<nt, NT, 0, s->stream>>>(s->d_tasks, x, y, z, vx, vy, vz, fx, fy, fz, species, thermo, h0, h1,
                                          dt);
}

void nvt_second(flare_state* s, double* vx, double* vy, double* vz, const float* fx, const float* fy,
                const float* fz, const int32_t* species, const double* masses, double dt, double t0, double tau,
                double* thermo, bool update) {
  const int nc = s->n_struct, nt = (int)s->tasks.size();
  const double h0 = 0.5 * dt * KAPPA / masses[0], h1 = 0.5 * dt * KAPPA / masses[1];
  if (nt > 0)
    k_nvt_second<<<nt, NT, 0, s->stream>>>(s->d_tasks, vx, vy, vz, fx, fy, fz, species, thermo, h0, h1, masses[0],
                                           masses[1], dt, update ? 1 : 0, s->red_e);
  if (nc > 0)
    k_nh_close<<<nc, NC, 0, s->stream>>>(s->red_e, s->d_first_task, s->d_struct_off, thermo, dt, t0, tau,
                                         update ? 1 : 0);
}

void coordination(flare_state* s, const double* x, const double* y, const double* z, int32_t* coord,
                  const int32_t* prev, int64_t* events) {
  const int n = s->n_atoms, nc = s->n_struct, nt = (int)s->tasks.size();
  if (n > 0)
    k_coord<<<(n + NT - 1) / NT, NT, 0, s->stream>>>(n, s->perm, s->sp, s->sid, s->d_grids, x, y, z, s->off,
                                                     s->nl_off, s->nl_j, s->nl_s, coord);
  if (prev && events) {
    if (nt > 0) k_events_tasks<<<nt, NT, 0, s->stream>>>(s->d_tasks, prev, coord, s->red_e);
    if (nc > 0) k_events_cells<<<(nc + NC - 1) / NC, NC, 0, s->stream>>>(nc, s->red_e, s->d_first_task, events);
  }
}

}  // namespace flare
