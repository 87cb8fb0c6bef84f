// Cell-binned neighbour list and environment classification.
//
// The local environment rho_i is every atom (and periodic image) within the cutoff
// (paper, Section V.B). The list is built with radius r_list = r_cut + skin:
//   1. wrap every position into its cell, w = x - L*floor(x/L), and bin it on a grid
//      of cells >= r_list per axis;
//   2. counting sort by (cell, bin) with a deterministic order inside each bin, which
//      also defines the internal atom order (spatially local);
//   3. per atom, scan the (2K+1)^3 bins around it on the unwrapped bin lattice, so a
//      box with fewer than three bins per axis (or narrower than r_list) visits each
//      (bin, image shift) once; keep (j, s) with |w_j - w_i + s*L|^2 < r_list^2,
//      evaluated in FP64 without fused multiply-add;
//   4. OR the species bits of the neighbours: atoms that see one species only use that
//      species-pair block of the descriptor (the reduction of Section V.B).
#include "state.h"

namespace flare {
namespace {

constexpr int NT = 256;

__device__ inline int floor_div(int u, int n) { return u >= 0 ? u / n : -((-u + n - 1) / n); }

__global__ __launch_bounds__(NT) void k_wrap_bin(int n, const double* __restrict__ x,
                                                 const double* __restrict__ y,
                                                 const double* __restrict__ z,
                                                 const int32_t* __restrict__ species,
                                                 const int* __restrict__ cell_off, int n_cell,
                                                 const CellGrid* __restrict__ grids,
                                                 int* __restrict__ o_bin, int* __restrict__ o_sid,
                                                 double* __restrict__ o_w,
                                                 double* __restrict__ o_off,
                                                 int* __restrict__ status) {
#pragma clang fp contract(off)
  const int a = blockIdx.x * NT + threadIdx.x;
  if (a >= n) return;
  int lo = 0, hi = n_cell - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (cell_off[mid] <= a) lo = mid;
    else hi = mid - 1;
  }
  const CellGrid g = grids[lo];
  int s = species[a];
  if (s < 0 || s >= NS) atomicOr(status, FLARE_FLAG_SPECIES);
  double p[3] = {x[a], y[a], z[a]};
  int b[3];
  bool finite = true;
  for (int ax = 0; ax < 3; ++ax) finite = finite && isfinite(p[ax]);
  if (!finite) {
    atomicOr(status, FLARE_FLAG_NONFINITE);
    p[0] = p[1] = p[2] = 0.0;
  }
  for (int ax = 0; ax < 3; ++ax) {
    const double L = g.L[ax];
    const double k = floor(p[ax] / L);
    const double kl = L * k;
    const double wv = p[ax] - kl;
    int bi = (int)floor(wv * g.inv_h[ax]);
    bi = bi < 0 ? 0 : (bi >= g.nb[ax] ? g.nb[ax] - 1 : bi);
    b[ax] = bi;
    o_w[(size_t)ax * n + a] = wv;
    o_off[(size_t)ax * n + a] = -kl;
  }
  o_bin[a] = g.bin_base + (b[2] * g.nb[1] + b[1]) * g.nb[0] + b[0];
  o_sid[a] = lo;
}

__global__ __launch_bounds__(NT) void k_bin_count(int n, const int* __restrict__ o_bin,
                                                  int* __restrict__ cnt) {
  const int a = blockIdx.x * NT + threadIdx.x;
  if (a < n) atomicAdd(&cnt[o_bin[a]], 1);
}

__global__ __launch_bounds__(NT) void k_bin_scatter(int n, const int* __restrict__ o_bin,
                                                    const int* __restrict__ start,
                                                    int* __restrict__ fill,
                                                    int* __restrict__ sorted) {
  const int a = blockIdx.x * NT + threadIdx.x;
  if (a >= n) return;
  const int b = o_bin[a];
  sorted[start[b] + atomicAdd(&fill[b], 1)] = a;
}

// Inside each bin, order atoms by caller index (the scatter order is racy).
__global__ __launch_bounds__(NT) void k_bin_sort(int nbins, const int* __restrict__ start,
                                                 int* __restrict__ sorted) {
  const int b = blockIdx.x * NT + threadIdx.x;
  if (b >= nbins) return;
  const int lo = start[b], hi = start[b + 1];
  for (int k = lo + 1; k < hi; ++k) {
    int v = sorted[k];
    int m = k - 1;
    while (m >= lo && sorted[m] > v) {
      sorted[m + 1] = sorted[m];
      --m;
    }
    sorted[m + 1] = v;
  }
}

__global__ __launch_bounds__(NT) void k_to_internal(int n, const int* __restrict__ sorted,
                                                    const int* __restrict__ o_bin,
                                                    const int* __restrict__ o_sid,
                                                    const double* __restrict__ o_w,
                                                    const double* __restrict__ o_off,
                                                    const int32_t* __restrict__ species,
                                                    int* __restrict__ perm, int* __restrict__ sp,
                                                    int* __restrict__ sid, int* __restrict__ bin,
                                                    double4* __restrict__ w,
                                                    double* __restrict__ off) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const int a = sorted[i];
  perm[i] = a;
  int s = species[a];
  sp[i] = (s < 0 || s >= NS) ? 0 : s;
  sid[i] = o_sid[a];
  bin[i] = o_bin[a];
  w[i] = make_double4(o_w[a], o_w[(size_t)n + a], o_w[2 * (size_t)n + a], 0.0);
  for (int ax = 0; ax < 3; ++ax) off[(size_t)ax * n + i] = o_off[(size_t)ax * n + a];
}

// Row order inside a bucket: by neighbour count, largest first (counts of NCK - 1 and more
// share the last class), ties by internal index. The 32-row slices of the sliced layout
// then hold rows of nearly equal length, so a wave's trip count over its slice (the
// longest row) wastes few lanes. (Measured: ordering only inside 128-row tiles, or inside
// windows of 4096 atoms, keeps more spatial locality for the per-slot gathers but leaves
// enough padding in the slices to cost more in the fused kernel than it saves there.)
// Sort key of an atom in bucket b with count c: b * NCK + (NCK - 1 - min(c, NCK - 1)).
constexpr int NCK = 64;
constexpr int NKEY = NBUCKET * NCK;
__device__ inline int row_key(int b, int c) { return b * NCK + (NCK - 1 - min(c, NCK - 1)); }

// Per-block counts of each sort key, blk[key * nblk + block] (key < 0: no row).
__device__ inline void block_key_counts(int key, int* __restrict__ blk, int nblk) {
  __shared__ int cnt[NKEY];
  for (int k = threadIdx.x; k < NKEY; k += NT) cnt[k] = 0;
  __syncthreads();
  if (key >= 0) atomicAdd(&cnt[key], 1);
  __syncthreads();
  for (int k = threadIdx.x; k < NKEY; k += NT) blk[(size_t)k * nblk + blockIdx.x] = cnt[k];
}

// The counting pass (FILL = false) also keeps the first PAIR_CACHE pairs of every atom in
// cache[c * n + i] (j, packed shift); the filling pass copies them for atoms whose count
// fits and repeats the search only for the others (32 covers every atom of the 1 M-atom
// H2/Pt(111) cell at r_list 4.7 A, whose largest count is 28).
constexpr int PAIR_CACHE = 32;

template <bool FILL>
__global__ __launch_bounds__(NT) void k_pairs(int n, const CellGrid* __restrict__ grids,
                                              const int* __restrict__ sid,
                                              const int* __restrict__ bin,
                                              const double4* __restrict__ w,
                                              const int* __restrict__ sp,
                                              const int* __restrict__ bstart, double rl2,
                                              int* __restrict__ cnt_out,
                                              int* __restrict__ envmask,
                                              int* __restrict__ bucket, int* __restrict__ blk,
                                              int nblk, const int* __restrict__ nl_off,
                                              int* __restrict__ nl_j, int32_t* __restrict__ nl_s,
                                              int2* __restrict__ cache) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * NT + threadIdx.x;
  int key_out = -1;
  if (FILL) {
    // The work-group's atoms own one contiguous range of the list. Copy the cached pairs
    // in list order (thread t takes positions t, t + NT, ...; the atom by bisection in the
    // offsets, in LDS), so that the writes are coalesced; an atom with more pairs than the
    // cache holds is searched again by its own thread below.
    __shared__ int offs[NT + 1];
    const int a0 = blockIdx.x * NT;
    const int na = min(NT, n - a0);
    for (int k = threadIdx.x; k <= na; k += NT) offs[k] = nl_off[a0 + k];
    __syncthreads();
    for (int p = offs[0] + threadIdx.x; p < offs[na]; p += NT) {
      int lo = 0, hi = na;            // largest k with offs[k] <= p
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (offs[mid] <= p) lo = mid;
        else hi = mid;
      }
      if (offs[lo + 1] - offs[lo] > PAIR_CACHE) continue;
      const int2 e = cache[(size_t)(p - offs[lo]) * n + a0 + lo];
      nl_j[p] = e.x;
      nl_s[p] = e.y;
    }
    if (i >= n || offs[threadIdx.x + 1] - offs[threadIdx.x] <= PAIR_CACHE) return;
  }
  if (i < n) {
    const CellGrid g = grids[sid[i]];
    const int local = bin[i] - g.bin_base;
    const int bx = local % g.nb[0];
    const int by = (local / g.nb[0]) % g.nb[1];
    const int bz = local / (g.nb[0] * g.nb[1]);
    const double4 wi = w[i];
    const double wx = wi.x, wy = wi.y, wz = wi.z;
    int cnt = 0, mask = 0;
    long long o = FILL ? nl_off[i] : 0;
    for (int oz = -g.K[2]; oz <= g.K[2]; ++oz) {
      const int uz = bz + oz;
      const int sz = floor_div(uz, g.nb[2]);
      const int cz = uz - sz * g.nb[2];
      const double tz = (double)sz * g.L[2];
      for (int oy = -g.K[1]; oy <= g.K[1]; ++oy) {
        const int uy = by + oy;
        const int sy = floor_div(uy, g.nb[1]);
        const int cy = uy - sy * g.nb[1];
        const double ty = (double)sy * g.L[1];
        // the atoms of bin bb (image shift sx along x) in order, four positions per step
        auto scan_bin = [&](int j0, int j1, int sx) {
          const double tx = (double)sx * g.L[0];
          const bool zero_shift = (sx == 0) && (sy == 0) && (sz == 0);
          for (int j4 = j0; j4 < j1; j4 += 4) {
            double4 wq[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) wq[u] = j4 + u < j1 ? w[j4 + u] : make_double4(0.0, 0.0, 0.0, 0.0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int j = j4 + u;
              if (j >= j1) break;
              const double dx = (wq[u].x - wx) + tx;
              const double dy = (wq[u].y - wy) + ty;
              const double dz = (wq[u].z - wz) + tz;
              const double r2 = dx * dx + dy * dy + dz * dz;
              if (r2 < rl2 && !(zero_shift && j == i)) {
                if (FILL) {
                  nl_j[o + cnt] = j;
                  nl_s[o + cnt] = pack_shift(sx, sy, sz);
                } else if (cnt < PAIR_CACHE) {
                  cache[(size_t)cnt * n + i] = make_int2(j, pack_shift(sx, sy, sz));
                }
                mask |= 1 << sp[j];
                ++cnt;
              }
            }
          }
        };
        const int rb = g.bin_base + (cz * g.nb[1] + cy) * g.nb[0];
        if (g.K[0] == 1) {
          // one-bin stencil in x: the row's three bin ranges are loaded together
          int sxs[3], j0s[3], j1s[3];
#pragma unroll
          for (int u = 0; u < 3; ++u) {
            const int ux = bx + u - 1;
            sxs[u] = floor_div(ux, g.nb[0]);
            const int bb = rb + (ux - sxs[u] * g.nb[0]);
            j0s[u] = bstart[bb];
            j1s[u] = bstart[bb + 1];
          }
#pragma unroll
          for (int u = 0; u < 3; ++u) scan_bin(j0s[u], j1s[u], sxs[u]);
        } else {
          for (int ox = -g.K[0]; ox <= g.K[0]; ++ox) {
            const int ux = bx + ox;
            const int sx = floor_div(ux, g.nb[0]);
            const int bb = rb + (ux - sx * g.nb[0]);
            scan_bin(bstart[bb], bstart[bb + 1], sx);
          }
        }
      }
    }
    if (!FILL) {
      cnt_out[i] = cnt;
      envmask[i] = mask;
      const int b = bucket_of(sp[i], mask);
      bucket[i] = b;
      if (b >= 0) key_out = row_key(b, cnt);
    }
  }
  if (!FILL) block_key_counts(key_out, blk, nblk);
}

// For every pair p = (i, j, s) find q = (j, i, -s) in j's list. The list is symmetric
// because the FP64 distance test gives the same value for both orders (negating a
// rounded difference is exact). Only pairs with i < j search (and write both rev[p] and
// rev[q]); a pair of an atom with its own image (i == j) searches too, so both threads of
// such a pair write the same two values; rev was filled with -1 before, so a pair left
// without a partner shows in k_rev_check.
// One thread per pair: a work-group takes the pairs of NT consecutive atoms, finds each
// pair's atom by bisection in the group's offsets (in LDS), then scans j's list.
__global__ __launch_bounds__(NT) void k_reverse(int n, const int* __restrict__ nl_off,
                                                const int* __restrict__ nl_j,
                                                const int32_t* __restrict__ nl_s,
                                                int* __restrict__ rev) {
  __shared__ int offs[NT + 1];
  const int a0 = blockIdx.x * NT;
  const int na = min(NT, n - a0);
  for (int k = threadIdx.x; k <= na; k += NT) offs[k] = nl_off[a0 + k];
  __syncthreads();
  const int p0 = offs[0], p1 = offs[na];
  for (int p = p0 + threadIdx.x; p < p1; p += NT) {
    const int j = nl_j[p];
    int lo = 0, hi = na;            // largest k with offs[k] <= p
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (offs[mid] <= p) lo = mid;
      else hi = mid;
    }
    const int i = a0 + lo;
    if (j < i) continue;            // found by the partner's thread
    int sx, sy, sz;
    unpack_shift(nl_s[p], sx, sy, sz);
    const int32_t want = pack_shift(-sx, -sy, -sz);
    int found = -1;
    const int q1 = nl_off[j + 1];
    // four entries per step, their loads issued together
    for (int q = nl_off[j]; q < q1 && found < 0; q += 4) {
      int jj[4];
      int32_t ss[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        jj[u] = q + u < q1 ? nl_j[q + u] : -1;
        ss[u] = q + u < q1 ? nl_s[q + u] : 0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (found < 0 && jj[u] == i && ss[u] == want) found = q + u;
    }
    if (found >= 0) {
      rev[p] = found;
      rev[found] = p;
    }
  }
}

// Every pair must have its reverse (species flag bit 8 otherwise).
__global__ __launch_bounds__(NT) void k_rev_check(int npairs, const int* __restrict__ rev,
                                                  int* __restrict__ status) {
  const int p = blockIdx.x * NT + threadIdx.x;
  if (p < npairs && rev[p] < 0) atomicOr(status, 256);
}

// ---- sliced pair layout ----
// Row R of atom i: 144-wide rows R = row_of[i], mixed rows R = rows1 + row_of[i].
__device__ inline int global_row(int b, int r, int rows1) { return b < 4 ? r : rows1 + r; }

// Length of each 32-row slice: the largest pair count of its rows (padding rows count 0).
__global__ __launch_bounds__(NT) void k_slice_len(int nslices, const int* __restrict__ cnt_row,
                                                  int* __restrict__ slice_len) {
  const int S = blockIdx.x * NT + threadIdx.x;
  if (S >= nslices) return;
  int m = 0;
  for (int r = 0; r < 32; ++r) m = max(m, cnt_row[S * 32 + r]);
  slice_len[S] = m;
}

// Per-row copies of the atom's pair count and cell (padding rows: 0, 0).
__global__ __launch_bounds__(NT) void k_row_meta(int rows, int rows1, const int* __restrict__ aor1,
                                                 const int* __restrict__ aorx, const int* __restrict__ cnt,
                                                 const int* __restrict__ sid, int* __restrict__ cnt_row,
                                                 int* __restrict__ sid_row) {
  const int R = blockIdx.x * NT + threadIdx.x;
  if (R >= rows) return;
  const int i = R < rows1 ? aor1[R] : aorx[R - rows1];
  cnt_row[R] = i >= 0 ? cnt[i] : 0;
  sid_row[R] = i >= 0 ? sid[i] : 0;
}

// Row of every atom in caller order (-1: no listed pair, no row).
__global__ __launch_bounds__(NT) void k_caller_rows(int n, const int* __restrict__ bucket,
                                                    const int* __restrict__ row_of, int rows1,
                                                    const int* __restrict__ perm, int* __restrict__ row_caller) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const int b = bucket[i];
  row_caller[perm[i]] = b < 0 ? -1 : global_row(b, row_of[i], rows1);
}

// One thread per row: the row's own pairs into its slots, the rest of its slice length
// (and every slot of a padding row) marked empty. Writes of a slice's 32 rows are
// contiguous for each k.
__global__ __launch_bounds__(NT) void k_fill_slots(int rows, int rows1, const int* __restrict__ aor1,
                                                   const int* __restrict__ aorx,
                                                   const int* __restrict__ nl_off,
                                                   const int* __restrict__ nl_j,
                                                   const int* __restrict__ slice_base,
                                                   int* __restrict__ slot_atom, int* __restrict__ slot_j,
                                                   int* __restrict__ slot_rev, float4* __restrict__ slot_d0) {
  const int R = blockIdx.x * NT + threadIdx.x;
  if (R >= rows) return;
  const int i = R < rows1 ? aor1[R] : aorx[R - rows1];
  const int base = slice_base[R >> 5], len = slice_base[(R >> 5) + 1] - base;
  const int p0 = i >= 0 ? nl_off[i] : 0, own = i >= 0 ? nl_off[i + 1] - p0 : 0;
  for (int k = 0; k < len; ++k) {
    const int slot = (base + k) * 32 + (R & 31);
    if (k < own) {
      slot_atom[slot] = i;
      slot_j[slot] = nl_j[p0 + k];
    } else {
      slot_atom[slot] = -1;
      slot_j[slot] = 0;
      slot_rev[slot] = slot;            // padding slots point at themselves
      slot_d0[slot] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
}

// Slot of every listed pair, in list order: a work-group takes the pairs of NT consecutive
// atoms (one contiguous range of the list), keeps each atom's row and slice base in LDS and
// finds each position's atom by bisection, so that the writes are coalesced.
__global__ __launch_bounds__(NT) void k_slot_of_pair(int n, const int* __restrict__ bucket,
                                                     const int* __restrict__ row_of, int rows1,
                                                     const int* __restrict__ nl_off,
                                                     const int* __restrict__ slice_base,
                                                     int* __restrict__ slot_of_pair) {
  __shared__ int offs[NT + 1], lane_row[NT], sbase[NT];
  const int a0 = blockIdx.x * NT;
  const int na = min(NT, n - a0);
  for (int k = threadIdx.x; k <= na; k += NT) offs[k] = nl_off[a0 + k];
  if (threadIdx.x < na) {
    const int b = bucket[a0 + threadIdx.x];
    // an atom without pairs owns no position of the list; its entries are never read
    const int R = b < 0 ? 0 : global_row(b, row_of[a0 + threadIdx.x], rows1);
    lane_row[threadIdx.x] = R & 31;
    sbase[threadIdx.x] = b < 0 ? 0 : slice_base[R >> 5];
  }
  __syncthreads();
  for (int p = offs[0] + threadIdx.x; p < offs[na]; p += NT) {
    int lo = 0, hi = na;            // largest k with offs[k] <= p
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (offs[mid] <= p) lo = mid;
      else hi = mid;
    }
    slot_of_pair[p] = (sbase[lo] + (p - offs[lo])) * 32 + lane_row[lo];
  }
}

// Per listed pair p = (i, j, s), in list order: the slot of its reverse pair and the fixed
// part of its pair vector, (w_j - w_i) + s*L from the reference positions in FP64, kept in
// FP32 with the neighbour species as +-1. A work-group takes the pairs of NT consecutive
// atoms (i by bisection in the group's offsets, in LDS); the atoms are in spatial order, so
// the neighbour positions it reads are close together.
__global__ __launch_bounds__(NT) void k_pair_slots(int n, const int* __restrict__ nl_off,
                                                   const int* __restrict__ nl_j,
                                                   const int32_t* __restrict__ nl_s,
                                                   const int* __restrict__ nl_rev,
                                                   const int* __restrict__ slot_of_pair,
                                                   const double4* __restrict__ w, const int* __restrict__ sp,
                                                   const int* __restrict__ sid,
                                                   const CellGrid* __restrict__ grids,
                                                   int* __restrict__ slot_rev, float4* __restrict__ slot_d0) {
  __shared__ int offs[NT + 1];
  const int a0 = blockIdx.x * NT;
  const int na = min(NT, n - a0);
  for (int k = threadIdx.x; k <= na; k += NT) offs[k] = nl_off[a0 + k];
  __syncthreads();
  const int p0 = offs[0], p1 = offs[na];
  for (int p = p0 + threadIdx.x; p < p1; p += NT) {
    int lo = 0, hi = na;            // largest k with offs[k] <= p
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (offs[mid] <= p) lo = mid;
      else hi = mid;
    }
    const int i = a0 + lo;
    const int j = nl_j[p];
    int sx, sy, sz;
    unpack_shift(nl_s[p], sx, sy, sz);
    const CellGrid* g = grids + sid[i];
    const double4 wj = w[j], wi = w[i];
    const double dx = (wj.x - wi.x) + (double)sx * g->L[0];
    const double dy = (wj.y - wi.y) + (double)sy * g->L[1];
    const double dz = (wj.z - wi.z) + (double)sz * g->L[2];
    const int slot = slot_of_pair[p];
    slot_rev[slot] = slot_of_pair[nl_rev[p]];
    slot_d0[slot] = make_float4((float)dx, (float)dy, (float)dz, sp[j] ? 1.f : -1.f);
  }
}

struct Row0 {
  int r[NBUCKET];
};

// Rows of each bucket in key order (see row_key); the rank among equal keys follows the
// internal index (block scan of the key counts, then the rank inside the block).
__global__ __launch_bounds__(NT) void k_assign_rows(int n, const int* __restrict__ bucket,
                                                    const int* __restrict__ cnt,
                                                    const int* __restrict__ blk_scan, int nblk,
                                                    Row0 row0, int* __restrict__ row_of,
                                                    int* __restrict__ aor1,
                                                    int* __restrict__ aorx) {
  __shared__ int keys[NT];
  const int i = blockIdx.x * NT + threadIdx.x;
  const int b = i < n ? bucket[i] : -1;
  const int key = b >= 0 ? row_key(b, cnt[i]) : -1;
  keys[threadIdx.x] = key;
  __syncthreads();
  if (i >= n) return;
  if (b < 0) {
    row_of[i] = -1;
    return;
  }
  int rank = 0;
  for (int q = 0; q < (int)threadIdx.x; ++q) rank += keys[q] == key ? 1 : 0;
  const int row = row0.r[b] + (blk_scan[(size_t)key * nblk + blockIdx.x] - blk_scan[(size_t)b * NCK * nblk]) + rank;
  row_of[i] = row;
  if (b < 4) aor1[row] = i;
  else aorx[row] = i;
}

// The per-atom counts are non-negative and each is below 2^31, so their int32 prefix sum
// has run past 2^31 - 1 exactly when one of its entries is negative: then the list does
// not fit any state (status bit 512).
__global__ __launch_bounds__(NT) void k_off_check(int n, const int* __restrict__ nl_off, int* __restrict__ status) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i <= n && nl_off[i] < 0) atomicOr(status, 512);
}

// info[0] = total pairs, info[1..6] = bucket totals, info[7] = the build's own status
// word, info[8] = the caller-visible status word raised since it was last read, which is
// moved to the host here (and cleared) so that no flag of the ended interval is lost
__global__ void k_info(int n, const int* __restrict__ nl_off, const int* __restrict__ blk_scan,
                       int nblk, int* __restrict__ status, int* __restrict__ info) {
  if (threadIdx.x == 0) {
    info[0] = nl_off[n];
    for (int b = 0; b < NBUCKET; ++b)
      info[1 + b] = blk_scan[(size_t)(b + 1) * NCK * nblk] - blk_scan[(size_t)b * NCK * nblk];
    info[7] = status[1];
    info[8] = status[0];
    status[0] = 0;
  }
}

inline int grid_of(long long n) { return (int)((n + NT - 1) / NT); }

#define HIPCHK(call)                                                     \
  do {                                                                   \
    hipError_t e_ = (call);                                              \
    if (e_ != hipSuccess) {                                              \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));      \
      return e_ == hipErrorOutOfMemory ? FLARE_E_OOM : FLARE_E_HIP;      \
    }                                                                    \
  } while (0)

}  // namespace

int build_list(flare_state* s, const double* x, const double* y, const double* z,
               const int32_t* species) {
  const int n = s->n_atoms;
  hipStream_t st = s->stream;
  const int nc = s->n_struct;
  HIPCHK(s->d_grids.reserve(nc));
  HIPCHK(s->d_struct_off.reserve(nc + 1));
  HIPCHK(hipMemcpyAsync(s->d_grids.p, s->grids.data(), nc * sizeof(CellGrid), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(s->d_struct_off.p, s->struct_off.data(), (nc + 1) * sizeof(int), hipMemcpyHostToDevice, st));
  const int nbins = s->n_bins;
  HIPCHK(s->bin_count.reserve(nbins + 1));
  HIPCHK(s->bin_start.reserve(nbins + 1));
  HIPCHK(s->bin_fill.reserve(nbins + 1));
  const int nblk = grid_of(n);
  HIPCHK(s->blk_bucket.reserve((size_t)NKEY * nblk + 1));
  HIPCHK(s->blk_bucket_scan.reserve((size_t)NKEY * nblk + 1));
  long long scan_n = std::max<long long>({(long long)nbins, (long long)n, (long long)NKEY * nblk});
  HIPCHK(s->scan_scratch.reserve(scan_scratch_ints(scan_n)));
  // the build checks its inputs in a word of its own (d_status[1]); the caller-visible
  // word d_status[0] keeps what the per-step calls raised until k_info moves it to the host
  int* bst = s->d_status + 1;
  HIPCHK(hipMemsetAsync(bst, 0, sizeof(int), st));
  if (n > 0) {
    k_wrap_bin<<<grid_of(n), NT, 0, st>>>(n, x, y, z, species, s->d_struct_off.p, nc, s->d_grids.p,
                                          s->o_bin, s->o_sid, s->o_w, s->o_off, bst);
  }
  HIPCHK(hipMemsetAsync(s->bin_count.p, 0, (nbins + 1) * sizeof(int), st));
  HIPCHK(hipMemsetAsync(s->bin_fill.p, 0, (nbins + 1) * sizeof(int), st));
  if (n > 0) k_bin_count<<<grid_of(n), NT, 0, st>>>(n, s->o_bin, s->bin_count.p);
  scan_exclusive(s->bin_count.p, s->bin_start.p, nbins, s->scan_scratch.p, st);
  if (n > 0) {
    k_bin_scatter<<<grid_of(n), NT, 0, st>>>(n, s->o_bin, s->bin_start.p, s->bin_fill.p, s->sorted);
    k_bin_sort<<<grid_of(nbins), NT, 0, st>>>(nbins, s->bin_start.p, s->sorted);
    k_to_internal<<<grid_of(n), NT, 0, st>>>(n, s->sorted, s->o_bin, s->o_sid, s->o_w, s->o_off,
                                             species, s->perm, s->sp, s->sid, s->bin, s->w, s->off);
  }
  const double rl2 = s->r_list * s->r_list;
  HIPCHK(s->pair_cache.reserve((size_t)PAIR_CACHE * n + 1));
  if (n > 0) {
    k_pairs<false><<<nblk, NT, 0, st>>>(n, s->d_grids.p, s->sid, s->bin, s->w, s->sp, s->bin_start.p,
                                         rl2, s->nl_cnt, s->envmask, s->bucket, s->blk_bucket.p, nblk,
                                         nullptr, nullptr, nullptr, s->pair_cache.p);
  }
  scan_exclusive(s->nl_cnt, s->nl_off, n, s->scan_scratch.p, st);
  scan_exclusive(s->blk_bucket.p, s->blk_bucket_scan.p, NKEY * nblk, s->scan_scratch.p, st);
  k_off_check<<<grid_of(n + 1), NT, 0, st>>>(n, s->nl_off, bst);
  k_info<<<1, 64, 0, st>>>(n, s->nl_off, s->blk_bucket_scan.p, nblk, s->d_status, s->d_info);
  HIPCHK(hipMemcpyAsync(s->h_info, s->d_info, 9 * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  s->flags_at_build = s->h_info[8];
  s->flags_pending |= s->h_info[8];
  const int flags = s->h_info[7];
  if (flags & FLARE_FLAG_SPECIES) {
    set_error("species index outside [0, n_species)");
    return FLARE_E_SPECIES;
  }
  if (flags & FLARE_FLAG_NONFINITE) {
    set_error("non-finite position");
    return FLARE_E_NONFINITE;
  }
  const long long pairs = (long long)(unsigned)s->h_info[0];
  if ((flags & 512) || pairs > s->max_pairs) {
    set_error((flags & 512) ? std::string("list needs more than 2^31 pairs")
                            : "list needs " + std::to_string(pairs) + " pairs, state holds " +
                                  std::to_string(s->max_pairs));
    return FLARE_E_CAPACITY;
  }
  s->n_pairs = pairs;
  Row0 row0;
  int r1 = 0, rx = 0;
  for (int b = 0; b < NBUCKET; ++b) {
    s->bucket_count[b] = s->h_info[1 + b];
    const int padded = (s->bucket_count[b] + TILE_ROWS - 1) / TILE_ROWS * TILE_ROWS;
    if (b < 4) {
      row0.r[b] = r1;
      r1 += padded;
    } else {
      row0.r[b] = rx;
      rx += padded;
    }
    s->bucket_row0[b] = row0.r[b];
  }
  s->rows1 = r1;
  s->rowsx = rx;
  HIPCHK(s->atom_of_row1.reserve(r1 + 1));
  HIPCHK(s->atom_of_rowx.reserve(rx + 1));
  HIPCHK(s->D1.reserve((size_t)r1 * ND1 + 64));
  HIPCHK(s->G1.reserve((size_t)r1 * ND1 + 64));
  HIPCHK(s->Dx.reserve((size_t)rx * ND + 64));
  HIPCHK(s->Gx.reserve((size_t)rx * ND + 64));
  HIPCHK(s->Yx.reserve((size_t)rx * ND + 64));
  HIPCHK(s->Px.reserve((size_t)rx * 4 + 64));
  if (s->model->var64) HIPCHK(s->Px64.reserve((size_t)rx * 9 + 64));
  HIPCHK(hipMemsetAsync(s->atom_of_row1.p, 0xff, (r1 + 1) * sizeof(int), st));
  HIPCHK(hipMemsetAsync(s->atom_of_rowx.p, 0xff, (rx + 1) * sizeof(int), st));
  if (n > 0) {
    k_pairs<true><<<nblk, NT, 0, st>>>(n, s->d_grids.p, s->sid, s->bin, s->w, s->sp, s->bin_start.p,
                                        rl2, nullptr, nullptr, nullptr, nullptr, nblk, s->nl_off,
                                        s->nl_j, s->nl_s, s->pair_cache.p);
    if (pairs > 0) {
      HIPCHK(hipMemsetAsync(s->nl_rev, 0xff, (size_t)pairs * sizeof(int), st));
      k_reverse<<<nblk, NT, 0, st>>>(n, s->nl_off, s->nl_j, s->nl_s, s->nl_rev);
      k_rev_check<<<(int)((pairs + NT - 1) / NT), NT, 0, st>>>((int)pairs, s->nl_rev, bst);
    }
    k_assign_rows<<<nblk, NT, 0, st>>>(n, s->bucket, s->nl_cnt, s->blk_bucket_scan.p, nblk, row0, s->row_of,
                                        s->atom_of_row1.p, s->atom_of_rowx.p);
  }
  HIPCHK(s->cnt_row.reserve((size_t)r1 + rx + 1));
  HIPCHK(s->sid_row.reserve((size_t)r1 + rx + 1));
  HIPCHK(s->e_row.reserve((size_t)r1 + rx + 1));
  HIPCHK(s->v_row.reserve((size_t)r1 + rx + 1));
  HIPCHK(s->row_out.reserve((size_t)r1 + rx + 1));
  HIPCHK(s->row_caller.reserve((size_t)n + 1));
  if (n > 0) k_caller_rows<<<nblk, NT, 0, st>>>(n, s->bucket, s->row_of, r1, s->perm, s->row_caller.p);
  if (r1 + rx > 0)
    k_row_meta<<<(r1 + rx + NT - 1) / NT, NT, 0, st>>>(r1 + rx, r1, s->atom_of_row1.p, s->atom_of_rowx.p,
                                                      s->nl_cnt, s->sid, s->cnt_row.p, s->sid_row.p);
  // sliced layout: slice lengths, their prefix, then the slots
  s->n_slices = (r1 + rx) / 32;
  HIPCHK(s->slice_len.reserve(s->n_slices + 1));
  HIPCHK(s->slice_base.reserve(s->n_slices + 1));
  if (s->n_slices > 0)
    k_slice_len<<<(s->n_slices + NT - 1) / NT, NT, 0, st>>>(s->n_slices, s->cnt_row.p, s->slice_len.p);
  HIPCHK(s->scan_scratch.reserve(scan_scratch_ints(std::max<long long>(scan_n, s->n_slices))));
  scan_exclusive(s->slice_len.p, s->slice_base.p, s->n_slices, s->scan_scratch.p, st);
  HIPCHK(hipMemcpyAsync(s->h_info + 9, s->slice_base.p + s->n_slices, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(s->h_info + 10, bst, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (s->h_info[10] & 256) {
    set_error("internal: neighbour list is not symmetric");
    return FLARE_E_HIP;
  }
  const long long nslots = 32LL * s->h_info[9];
  if (nslots > 0x7fffffffLL) {
    set_error("sliced pair layout needs " + std::to_string(nslots) + " slots, more than int32 indexes");
    return FLARE_E_CAPACITY;
  }
  s->n_slots = nslots;
  HIPCHK(s->slot_atom.reserve(nslots + 1));
  HIPCHK(s->slot_j.reserve(nslots + 1));
  HIPCHK(s->slot_d0.reserve(nslots + 1));
  HIPCHK(s->slot_rev.reserve(nslots + 1));
  HIPCHK(s->geom.reserve(nslots + 1));
  HIPCHK(s->f_own.reserve((size_t)r1 + rx + 1));
  HIPCHK(s->w_in.reserve(nslots + 1));
  if (r1 + rx > 0)
    k_fill_slots<<<(r1 + rx + NT - 1) / NT, NT, 0, st>>>(r1 + rx, r1, s->atom_of_row1.p, s->atom_of_rowx.p,
                                                        s->nl_off, s->nl_j, s->slice_base.p, s->slot_atom.p,
                                                        s->slot_j.p, s->slot_rev.p, s->slot_d0.p);
  if (n > 0) {
    k_slot_of_pair<<<nblk, NT, 0, st>>>(n, s->bucket, s->row_of, r1, s->nl_off, s->slice_base.p, s->slot_of_pair);
    k_pair_slots<<<nblk, NT, 0, st>>>(n, s->nl_off, s->nl_j, s->nl_s, s->nl_rev, s->slot_of_pair, s->w, s->sp,
                                       s->sid, s->d_grids.p, s->slot_rev.p, s->slot_d0.p);
  }
  // reduction tasks: contiguous internal ranges of one cell, at most 2048 atoms each (one
  // work-group per task); cell c owns tasks [first_task[c], first_task[c + 1])
  s->tasks.clear();
  s->first_task.assign(nc + 1, 0);
  for (int c = 0; c < nc; ++c) {
    s->first_task[c] = (int)s->tasks.size();
    int a = s->struct_off[c], b = s->struct_off[c + 1];
    if (a == b) s->tasks.push_back({c, a, a});
    for (int k = a; k < b; k += 2048) s->tasks.push_back({c, k, std::min(b, k + 2048)});
  }
  s->first_task[nc] = (int)s->tasks.size();
  HIPCHK(s->d_tasks.reserve(s->tasks.size()));
  HIPCHK(s->d_first_task.reserve(nc + 1));
  HIPCHK(hipMemcpyAsync(s->d_first_task.p, s->first_task.data(), (nc + 1) * sizeof(int), hipMemcpyHostToDevice,
                        st));
  HIPCHK(s->red_e.reserve(2 * s->tasks.size()));
  HIPCHK(s->red_s.reserve(s->tasks.size()));
  HIPCHK(hipMemcpyAsync(s->d_tasks.p, s->tasks.data(), s->tasks.size() * sizeof(RedTask),
                        hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(s->e_int, 0, (size_t)n * sizeof(float), st));
  HIPCHK(hipMemsetAsync(s->v_int, 0, (size_t)n * sizeof(float), st));
  HIPCHK(hipMemsetAsync(s->nrm, 0, (size_t)n * sizeof(float), st));
  HIPCHK(hipGetLastError());
  return FLARE_OK;
}

}  // namespace flare
