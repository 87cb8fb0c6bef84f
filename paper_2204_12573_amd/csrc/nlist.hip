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
// Every buffer has its capacity from flare_state_create. The sizes a build finds (pairs,
// atoms per environment class, rows, slices, slots) are formed on the device in a small
// layout record (d_layout) that the later kernels read; the host waits for the stream once,
// at the end, to read that record and the status words back.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "state.h"

namespace flare {
namespace {

constexpr int NT = 256;

// Layout record of a build (d_layout), formed on the device.
enum {
  LY_PAIRS = 0,      // listed pairs (nl_off[n])
  LY_COUNT = 1,      // [6] atoms per environment bucket
  LY_ROW0 = 7,       // [6] first row of each bucket inside its width class
  LY_ROWS1 = 13,     // padded rows of the 144-wide class
  LY_ROWSX = 14,     // padded rows of the 544-wide class
  LY_SLICES = 15,    // 32-row slices of both classes
  LY_SLOTS32 = 16,   // groups of 32 slots (the slice_base total)
  LY_FLAGS = 17,     // 1: more pairs than the capacity, 2: more slots than the capacity
  LY_BUILD = 18,     // the build's own status word (input and consistency checks)
  LY_STATUS = 19,    // the caller-visible status word raised since it was last read
  LY_N = 20
};
constexpr int BUILD_ASYMMETRIC = 256;   // a pair without its reverse (internal error)
constexpr int BUILD_OVERFLOW = 512;     // the int32 prefix of the pair counts overflowed

__device__ inline int floor_div(int u, int n) { return u >= 0 ? u / n : -((-u + n - 1) / n); }

// Caller order: wrap into the cell, bin, one 64-byte record per atom, bin counts; the
// positions themselves are kept (xb) as the reference of the per-step displacements.
__global__ __launch_bounds__(NT) void k_wrap_bin(int n, const double* __restrict__ x,
                                                 const double* __restrict__ y,
                                                 const double* __restrict__ z,
                                                 const int32_t* __restrict__ species,
                                                 const int* __restrict__ cell_off, int n_cell,
                                                 const CellGrid* __restrict__ grids,
                                                 CallerRec* __restrict__ rec, double* __restrict__ xb,
                                                 int* __restrict__ bin_count, int* __restrict__ status) {
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
  double wv[3], ov[3];
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
    wv[ax] = p[ax] - kl;
    ov[ax] = -kl;
    int bi = (int)floor(wv[ax] * g.inv_h[ax]);
    b[ax] = bi < 0 ? 0 : (bi >= g.nb[ax] ? g.nb[ax] - 1 : bi);
  }
  CallerRec r;
  r.wx = wv[0];
  r.wy = wv[1];
  r.wz = wv[2];
  r.ox = ov[0];
  r.oy = ov[1];
  r.oz = ov[2];
  r.bin = g.bin_base + (b[2] * g.nb[1] + b[1]) * g.nb[0] + b[0];
  r.cell = lo;
  r.pad0 = r.pad1 = 0;
  rec[a] = r;
  xb[a] = p[0];
  xb[(size_t)n + a] = p[1];
  xb[2 * (size_t)n + a] = p[2];
  atomicAdd(&bin_count[r.bin], 1);
}

__global__ __launch_bounds__(NT) void k_bin_scatter(int n, const CallerRec* __restrict__ rec,
                                                    const int* __restrict__ start,
                                                    int* __restrict__ fill,
                                                    int* __restrict__ sorted) {
  const int a = blockIdx.x * NT + threadIdx.x;
  if (a >= n) return;
  const int b = rec[a].bin;
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

// Internal order: one caller record (a 64-byte line) per atom, gathered in bin order; the
// species rides in w.w, so that a neighbour's position and species are one load.
__global__ __launch_bounds__(NT) void k_to_internal(int n, const int* __restrict__ sorted,
                                                    const CallerRec* __restrict__ rec,
                                                    const int32_t* __restrict__ species,
                                                    int* __restrict__ perm, int* __restrict__ inv_perm,
                                                    int* __restrict__ sp,
                                                    int* __restrict__ sid, int* __restrict__ bin,
                                                    double4* __restrict__ w, float4* __restrict__ wf,
                                                    double* __restrict__ off) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const int a = sorted[i];
  perm[i] = a;
  inv_perm[a] = i;
  const int s = species[a];
  const int sc = (s < 0 || s >= NS) ? 0 : s;
  sp[i] = sc;
  const CallerRec r = rec[a];
  sid[i] = r.cell;
  bin[i] = r.bin;
  w[i] = make_double4(r.wx, r.wy, r.wz, (double)sc);
  wf[i] = make_float4((float)r.wx, (float)r.wy, (float)r.wz, (float)sc);
  off[i] = r.ox;
  off[(size_t)n + i] = r.oy;
  off[2 * (size_t)n + i] = r.oz;
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
// H2/Pt(111) cell at r_list 4.7 A, whose largest count is 28). The filling pass also marks
// every pair's reverse as not found yet (-1), and does nothing when the pairs exceed the
// capacity (layout flag).
constexpr int PAIR_CACHE = 32;

template <bool FILL>
__global__ __launch_bounds__(NT) void k_pairs(int n, const CellGrid* __restrict__ grids,
                                              const int* __restrict__ sid,
                                              const int* __restrict__ bin,
                                              const double4* __restrict__ w,
                                              const float4* __restrict__ wf,
                                              const int* __restrict__ bstart, double rl2, float lo2,
                                              float hi2,
                                              int* __restrict__ cnt_out,
                                              int* __restrict__ envmask,
                                              int* __restrict__ bucket, int* __restrict__ blk,
                                              int nblk, const int* __restrict__ nl_off,
                                              int* __restrict__ nl_j, int32_t* __restrict__ nl_s,
                                              int* __restrict__ nl_rev, int2* __restrict__ cache,
                                              const int* __restrict__ layout) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * NT + threadIdx.x;
  int key_out = -1;
  if (FILL) {
    if (layout[LY_FLAGS]) return;
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
      nl_rev[p] = -1;
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
    const float4 wif = wf[i];
    int cnt = 0, mask = 0;
    long long o = FILL ? nl_off[i] : 0;
    for (int oz = -g.K[2]; oz <= g.K[2]; ++oz) {
      const int uz = bz + oz;
      const int sz = floor_div(uz, g.nb[2]);
      const int cz = uz - sz * g.nb[2];
      const double tz = (double)sz * g.L[2];
      const float tzf = (float)tz;
      for (int oy = -g.K[1]; oy <= g.K[1]; ++oy) {
        const int uy = by + oy;
        const int sy = floor_div(uy, g.nb[1]);
        const int cy = uy - sy * g.nb[1];
        const double ty = (double)sy * g.L[1];
        const float tyf = (float)ty;
        // the atoms of bin bb (image shift sx along x) in order, four positions per step: the
        // FP32 copies decide every candidate whose FP32 distance is outside [lo2, hi2) (the
        // band holds the FP32 error, so the decision is the FP64 one), the FP64 test the rest
        auto scan_bin = [&](int j0, int j1, int sx) {
          const double tx = (double)sx * g.L[0];
          const float txf = (float)tx;
          const bool zero_shift = (sx == 0) && (sy == 0) && (sz == 0);
          for (int j4 = j0; j4 < j1; j4 += 4) {
            float4 wq[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) wq[u] = j4 + u < j1 ? wf[j4 + u] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int j = j4 + u;
              if (j >= j1) break;
              const float fx = (wq[u].x - wif.x) + txf;
              const float fy = (wq[u].y - wif.y) + tyf;
              const float fz = (wq[u].z - wif.z) + tzf;
              const float r2f = fx * fx + fy * fy + fz * fz;
              bool in = r2f < lo2;
              if (!in && r2f < hi2) {
                const double4 wd = w[j];
                const double dx = (wd.x - wx) + tx;
                const double dy = (wd.y - wy) + ty;
                const double dz = (wd.z - wz) + tz;
                in = dx * dx + dy * dy + dz * dz < rl2;
              }
              if (in && !(zero_shift && j == i)) {
                if (FILL) {
                  nl_j[o + cnt] = j;
                  nl_s[o + cnt] = pack_shift(sx, sy, sz);
                  nl_rev[o + cnt] = -1;
                } else if (cnt < PAIR_CACHE) {
                  cache[(size_t)cnt * n + i] = make_int2(j, pack_shift(sx, sy, sz));
                }
                mask |= 1 << (int)wq[u].w;
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
      const int b = bucket_of((int)wi.w, mask);
      bucket[i] = b;
      if (b >= 0) key_out = row_key(b, cnt);
    }
  }
  if (!FILL) block_key_counts(key_out, blk, nblk);
}

// The per-atom counts are non-negative and each is below 2^31, so their int32 prefix sum
// has run past 2^31 - 1 exactly when one of its entries is negative.
__global__ __launch_bounds__(NT) void k_off_check(int n, const int* __restrict__ nl_off, int* __restrict__ status) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i <= n && nl_off[i] < 0) atomicOr(status, BUILD_OVERFLOW);
}

// Sizes after the counting pass: pairs, atoms per bucket, the rows of every bucket padded to
// the 128-row tile (144-wide buckets first, then the mixed ones), 32-row slices.
__global__ void k_layout_rows(int n, const int* __restrict__ nl_off, const int* __restrict__ blk_scan, int nblk,
                              long long max_pairs, const int* __restrict__ build_status, int* __restrict__ layout) {
  if (threadIdx.x != 0) return;
  const int pairs = nl_off[n];
  int flags = 0;
  if ((*build_status & BUILD_OVERFLOW) || pairs < 0 || (long long)pairs > max_pairs) flags |= 1;
  int r1 = 0, rx = 0;
  for (int b = 0; b < NBUCKET; ++b) {
    const int c = blk_scan[(size_t)(b + 1) * NCK * nblk] - blk_scan[(size_t)b * NCK * nblk];
    const int padded = (c + TILE_ROWS - 1) / TILE_ROWS * TILE_ROWS;
    layout[LY_COUNT + b] = c;
    if (b < 4) {
      layout[LY_ROW0 + b] = r1;
      r1 += padded;
    } else {
      layout[LY_ROW0 + b] = rx;
      rx += padded;
    }
  }
  layout[LY_PAIRS] = pairs;
  layout[LY_ROWS1] = r1;
  layout[LY_ROWSX] = rx;
  layout[LY_SLICES] = (r1 + rx) / 32;
  layout[LY_FLAGS] = flags;
}

// For every pair p = (i, j, s) find q = (j, i, -s) in j's list and keep the positions of
// the two inside their lists: rev[p] = q - nl_off[j], rev[q] = p - nl_off[i]. The list is
// symmetric because the FP64 distance test gives the same value for both orders (negating
// a rounded difference is exact). Only pairs with i <= j search (and write both entries);
// for a pair of an atom with its own image (i == j) both threads write the same two
// values; rev holds -1 from the filling pass, so a pair left without a partner shows in
// the slot pass.
// One thread per pair: a work-group takes the pairs of NT consecutive atoms, finds each
// pair's atom by bisection in the group's offsets (in LDS), then scans j's list.
__global__ __launch_bounds__(NT) void k_reverse(int n, const int* __restrict__ nl_off,
                                                const int* __restrict__ nl_j,
                                                const int32_t* __restrict__ nl_s,
                                                int* __restrict__ rev, const int* __restrict__ layout) {
  if (layout[LY_FLAGS]) return;
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
    const int q0 = nl_off[j], q1 = nl_off[j + 1];
    // four entries per step, their loads issued together
    for (int q = q0; q < q1 && found < 0; q += 4) {
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
      rev[p] = found - q0;
      rev[found] = p - offs[lo];
    }
  }
}

// Rows of each bucket in key order (see row_key); the rank among equal keys follows the
// internal index (block scan of the key counts, then the rank inside the block).
__global__ __launch_bounds__(NT) void k_assign_rows(int n, const int* __restrict__ bucket,
                                                    const int* __restrict__ cnt,
                                                    const int* __restrict__ blk_scan, int nblk,
                                                    const int* __restrict__ layout, int* __restrict__ row_of,
                                                    int* __restrict__ aor1, int* __restrict__ aorx) {
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
  const int row = layout[LY_ROW0 + b] + (blk_scan[(size_t)key * nblk + blockIdx.x] -
                                         blk_scan[(size_t)b * NCK * nblk]) + rank;
  row_of[i] = row;
  if (b < 4) aor1[row] = i;
  else aorx[row] = i;
}

// Row R of atom i: 144-wide rows R = row_of[i], mixed rows R = rows1 + row_of[i].
__device__ inline int global_row(int b, int r, int rows1) { return b < 4 ? r : rows1 + r; }

// Per-row copies of the atom's pair count and cell (padding rows: 0, 0), over the row
// capacity; rows past the build's rows are left alone.
__global__ __launch_bounds__(NT) void k_row_meta(int row_cap, const int* __restrict__ layout,
                                                 const int* __restrict__ aor1, const int* __restrict__ aorx,
                                                 const int* __restrict__ cnt, const int* __restrict__ sid,
                                                 int* __restrict__ cnt_row, int* __restrict__ sid_row) {
  const int R = blockIdx.x * NT + threadIdx.x;
  const int rows1 = layout[LY_ROWS1], rows = rows1 + layout[LY_ROWSX];
  if (R >= rows || R >= row_cap) return;
  const int i = R < rows1 ? aor1[R] : aorx[R - rows1];
  cnt_row[R] = i >= 0 ? cnt[i] : 0;
  sid_row[R] = i >= 0 ? sid[i] : 0;
}

// Row of every atom in caller order and the slot of its first pair in internal order (-1:
// no listed pair, no row).
__global__ __launch_bounds__(NT) void k_atom_rows(int n, const int* __restrict__ bucket,
                                                  const int* __restrict__ row_of, const int* __restrict__ layout,
                                                  const int* __restrict__ perm, const int* __restrict__ slice_base,
                                                  int* __restrict__ row_caller, int* __restrict__ slot0) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const int b = bucket[i];
  const int R = b < 0 ? -1 : global_row(b, row_of[i], layout[LY_ROWS1]);
  row_caller[perm[i]] = R;
  slot0[i] = R < 0 ? -1 : slot_of(slice_base, R, 0);
}

// Length of each 32-row slice: the largest pair count of its rows (padding rows count 0);
// zero for the slices past the build's, so that the prefix over the capacity ends at the
// build's total.
__global__ __launch_bounds__(NT) void k_slice_len(int slice_cap, const int* __restrict__ layout,
                                                  const int* __restrict__ cnt_row, int* __restrict__ slice_len) {
  const int S = blockIdx.x * NT + threadIdx.x;
  if (S >= slice_cap) return;
  int m = 0;
  if (S < layout[LY_SLICES])
    for (int r = 0; r < 32; ++r) m = max(m, cnt_row[S * 32 + r]);
  slice_len[S] = m;
}

__global__ void k_layout_slots(const int* __restrict__ slice_base, int slice_cap, long long slot_cap,
                               int* __restrict__ layout) {
  if (threadIdx.x != 0) return;
  const int groups = slice_base[slice_cap];
  layout[LY_SLOTS32] = groups;
  if ((long long)groups * 32 > slot_cap) layout[LY_FLAGS] |= 2;
}

// The sliced pair layout in one pass, a work-group per 32-row slice: thread (h, l) of 8 x 32
// takes the slots (slice_base[S] + k) * 32 + l for k = h, h + 8, ... of row R = 32 S + l, so
// every store is coalesced and the gathers of eight positions of a row are in flight at
// once. A slot of a listed pair p = (i, j, s) gets i, j, the fixed part of the pair vector
// (w_j - w_i) + s*L (FP64, stored FP32, neighbour species as the sign of .w) and the slot of
// its reverse pair: slot0[j] + 32 rev[p], rev[p] being the reverse pair's position in j's
// list. Per pair this gathers two things of the neighbour, w[j] and slot0[j]. Every other
// slot of the slice is padding: pointing at itself, its geometry zero (for every step of
// the list's life).
__global__ __launch_bounds__(NT) void k_slots(const int* __restrict__ layout, const int* __restrict__ aor1,
                                              const int* __restrict__ aorx, const int* __restrict__ nl_off,
                                              const int* __restrict__ nl_j, const int32_t* __restrict__ nl_s,
                                              const int* __restrict__ nl_rev, const int* __restrict__ slot0,
                                              const int* __restrict__ slice_base, const double4* __restrict__ w,
                                              const int* __restrict__ sid, const CellGrid* __restrict__ grids,
                                              int* __restrict__ slot_atom, int* __restrict__ slot_j,
                                              int* __restrict__ slot_rev, float4* __restrict__ slot_d0,
                                              float4* __restrict__ geom,
                                              int* __restrict__ status) {
#pragma clang fp contract(off)
  if (layout[LY_FLAGS]) return;
  const int S = blockIdx.x;
  if (S >= layout[LY_SLICES]) return;
  const int rows1 = layout[LY_ROWS1];
  const int l = threadIdx.x & 31, h = threadIdx.x >> 5;
  const int R = S * 32 + l;
  const int i = R < rows1 ? aor1[R] : aorx[R - rows1];
  const int base = slice_base[S], len = slice_base[S + 1] - base;
  int p0 = 0, own = 0;
  double4 wi = make_double4(0.0, 0.0, 0.0, 0.0);
  double L[3] = {0.0, 0.0, 0.0};
  if (i >= 0) {
    p0 = nl_off[i];
    own = nl_off[i + 1] - p0;
    wi = w[i];
    const CellGrid* g = grids + sid[i];
    L[0] = g->L[0];
    L[1] = g->L[1];
    L[2] = g->L[2];
  }
  for (int k = h; k < len; k += NT / 32) {
    const int slot = (base + k) * 32 + l;
    if (k < own) {
      const int p = p0 + k;
      const int j = nl_j[p];
      const int q = nl_rev[p];
      int sx, sy, sz;
      unpack_shift(nl_s[p], sx, sy, sz);
      const int sj = slot0[j];
      const double4 wj = w[j];
      int rs = slot;
      if (q < 0) atomicOr(status, BUILD_ASYMMETRIC);
      else rs = sj + 32 * q;
      const double dx = (wj.x - wi.x) + (double)sx * L[0];
      const double dy = (wj.y - wi.y) + (double)sy * L[1];
      const double dz = (wj.z - wi.z) + (double)sz * L[2];
      slot_atom[slot] = i;
      slot_j[slot] = j;
      slot_rev[slot] = rs;
      slot_d0[slot] = make_float4((float)dx, (float)dy, (float)dz, wj.w != 0.0 ? 1.f : -1.f);
    } else {
      slot_atom[slot] = -1;
      slot_j[slot] = 0;
      slot_rev[slot] = slot;            // padding slots point at themselves
      slot_d0[slot] = make_float4(0.f, 0.f, 0.f, 0.f);
      geom[slot] = make_float4(0.f, 0.f, 0.f, 0.f);   // the per-step geometry skips padding
    }
  }
}

// End of a build: the build's status word and the caller-visible one (which is moved to
// the host here and cleared, so that no flag of the ended interval is lost) into the layout.
__global__ void k_layout_status(int* __restrict__ status, int* __restrict__ layout) {
  if (threadIdx.x == 0) {
    layout[LY_BUILD] = status[1];
    layout[LY_STATUS] = status[0];
    status[0] = 0;
  }
}

// The fills of a build in one launch: up to ten (array, count, value) segments, every
// work-item striding over each of them.
struct ClearSeg {
  int* p;
  long long n;
  int v;
};
struct ClearArgs {
  ClearSeg seg[10];
  int nseg;
};
__global__ __launch_bounds__(NT) void k_clear(ClearArgs a) {
  const long long t = (long long)blockIdx.x * NT + threadIdx.x;
  const long long stride = (long long)gridDim.x * NT;
  for (int k = 0; k < a.nseg; ++k) {
    int* __restrict__ p = a.seg[k].p;
    const long long n = a.seg[k].n;
    const int v = a.seg[k].v;
    for (long long i = t; i < n; i += stride) p[i] = v;
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

int list_key_count() { return NKEY; }
int list_pair_cache() { return PAIR_CACHE; }
int list_layout_words() { return LY_N; }

int build_list(flare_state* s, const double* x, const double* y, const double* z,
               const int32_t* species) {
  const int n = s->n_atoms;
  hipStream_t st = s->stream;
  const int nc = s->n_struct;
  const int nbins = s->n_bins;
  const int nblk = grid_of(n);
  // reduction tasks: contiguous internal ranges of one cell, at most 2048 atoms each (one
  // work-group per task); cell c owns tasks [first_task[c], first_task[c + 1])
  s->tasks.clear();
  s->first_task.assign(nc + 1, 0);
  for (int c = 0; c < nc; ++c) {
    s->first_task[c] = (int)s->tasks.size();
    const int a = s->struct_off[c], b = s->struct_off[c + 1];
    if (a == b) s->tasks.push_back({c, a, a});
    for (int k = a; k < b; k += 2048) s->tasks.push_back({c, k, std::min(b, k + 2048)});
  }
  s->first_task[nc] = (int)s->tasks.size();
  if ((int)s->tasks.size() > s->task_cap) {
    set_error("more reduction tasks than the state holds");
    return FLARE_E_CAPACITY;
  }
  // the per-cell host data through the pinned stage: grids, offsets, tasks, task ranges
  char* hs = s->h_stage;
  const size_t b_grid = nc * sizeof(CellGrid), b_off = (nc + 1) * sizeof(int);
  const size_t b_task = s->tasks.size() * sizeof(RedTask), b_first = (nc + 1) * sizeof(int);
  std::memcpy(hs, s->grids.data(), b_grid);
  std::memcpy(hs + b_grid, s->struct_off.data(), b_off);
  std::memcpy(hs + b_grid + b_off, s->tasks.data(), b_task);
  std::memcpy(hs + b_grid + b_off + b_task, s->first_task.data(), b_first);
  HIPCHK(hipMemcpyAsync(s->d_grids, hs, b_grid, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(s->d_struct_off, hs + b_grid, b_off, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(s->d_tasks, hs + b_grid + b_off, b_task, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(s->d_first_task, hs + b_grid + b_off + b_task, b_first, hipMemcpyHostToDevice, st));
  // the build checks its inputs in a word of its own (d_status[1]); the caller-visible
  // word d_status[0] keeps what the per-step calls raised until k_layout_status moves it
  int* bst = s->d_status + 1;
  {
    // everything the build starts from: its status word and layout record, the bin
    // counters, no atom in any row, zero energies, variances and norms (atoms without a
    // listed pair keep them)
    ClearArgs c{};
    auto seg = [&](int* p, long long cnt, int v) { c.seg[c.nseg++] = ClearSeg{p, cnt, v}; };
    seg(bst, 1, 0);
    seg(s->d_layout, LY_N, 0);
    seg(s->bin_count, (long long)nbins + 1, 0);
    seg(s->bin_fill, (long long)nbins + 1, 0);
    seg(s->atom_of_row1, (long long)s->row_cap + 1, -1);
    seg(s->atom_of_rowx, (long long)s->row_cap + 1, -1);
    seg(reinterpret_cast<int*>(s->e_int), n, 0);
    seg(reinterpret_cast<int*>(s->v_int), n, 0);
    seg(reinterpret_cast<int*>(s->nrm), n, 0);
    long long longest = 1;
    for (int k = 0; k < c.nseg; ++k) longest = std::max(longest, c.seg[k].n);
    k_clear<<<(int)std::min<long long>(grid_of(longest), 2048), NT, 0, st>>>(c);
  }
  if (n > 0)
    k_wrap_bin<<<grid_of(n), NT, 0, st>>>(n, x, y, z, species, s->d_struct_off, nc, s->d_grids, s->crec, s->xb,
                                          s->bin_count, bst);
  scan_exclusive(s->bin_count, s->bin_start, nbins, s->scan_scratch, st);
  if (n > 0) {
    k_bin_scatter<<<grid_of(n), NT, 0, st>>>(n, s->crec, s->bin_start, s->bin_fill, s->sorted);
    k_bin_sort<<<grid_of(nbins), NT, 0, st>>>(nbins, s->bin_start, s->sorted);
    k_to_internal<<<grid_of(n), NT, 0, st>>>(n, s->sorted, s->crec, species, s->perm, s->inv_perm, s->sp, s->sid, s->bin, s->w, s->wf,
                                             s->off);
  }
  const double rl2 = s->r_list * s->r_list;
  // Band of the FP32 first test. Wrapped coordinates lie in [0, W] (W the largest box side),
  // image shifts are at most K box sides (K the largest stencil half-width), u = 2^-24. A
  // candidate near the list radius has every FP32 pair-vector component within
  // e = u ((3 + K) W + 2 r_list) of the FP64 one, so the FP32 |Delta|^2 is within
  // e (2 sqrt(3) r_list + 3 e) + 4 u r_list^2 of the FP64 value; the band is twice that.
  double wmax = 0.0;
  int kmax = 1;
  for (const CellGrid& g : s->grids)
    for (int ax = 0; ax < 3; ++ax) {
      wmax = std::max(wmax, g.L[ax]);
      kmax = std::max(kmax, g.K[ax]);
    }
  const double u32 = std::ldexp(1.0, -24);
  const double e32 = u32 * ((3.0 + kmax) * wmax + 2.0 * s->r_list);
  const double band = 2.0 * (e32 * (2.0 * std::sqrt(3.0) * s->r_list + 3.0 * e32) + 4.0 * u32 * rl2);
  const float lo2 = std::nextafter((float)(rl2 - band), -INFINITY);
  const float hi2 = std::nextafter((float)(rl2 + band), INFINITY);
  if (n > 0)
    k_pairs<false><<<nblk, NT, 0, st>>>(n, s->d_grids, s->sid, s->bin, s->w, s->wf, s->bin_start, rl2, lo2, hi2,
                                         s->nl_cnt,
                                         s->envmask, s->bucket, s->blk_bucket, nblk, nullptr, nullptr, nullptr,
                                         nullptr, s->pair_cache, nullptr);
  scan_exclusive(s->nl_cnt, s->nl_off, n, s->scan_scratch, st);
  scan_exclusive(s->blk_bucket, s->blk_bucket_scan, NKEY * nblk, s->scan_scratch, st);
  k_off_check<<<grid_of(n + 1), NT, 0, st>>>(n, s->nl_off, bst);
  k_layout_rows<<<1, 64, 0, st>>>(n, s->nl_off, s->blk_bucket_scan, nblk, s->max_pairs, bst, s->d_layout);
  if (n > 0) {
    k_pairs<true><<<nblk, NT, 0, st>>>(n, s->d_grids, s->sid, s->bin, s->w, s->wf, s->bin_start, rl2, lo2, hi2,
                                        nullptr,
                                        nullptr, nullptr, nullptr, nblk, s->nl_off, s->nl_j, s->nl_s, s->nl_rev,
                                        s->pair_cache, s->d_layout);
    k_reverse<<<nblk, NT, 0, st>>>(n, s->nl_off, s->nl_j, s->nl_s, s->nl_rev, s->d_layout);
    k_assign_rows<<<nblk, NT, 0, st>>>(n, s->bucket, s->nl_cnt, s->blk_bucket_scan, nblk, s->d_layout, s->row_of,
                                        s->atom_of_row1, s->atom_of_rowx);
  }
  k_row_meta<<<grid_of(s->row_cap), NT, 0, st>>>(s->row_cap, s->d_layout, s->atom_of_row1, s->atom_of_rowx,
                                                  s->nl_cnt, s->sid, s->cnt_row, s->sid_row);
  k_slice_len<<<grid_of(s->slice_cap), NT, 0, st>>>(s->slice_cap, s->d_layout, s->cnt_row, s->slice_len);
  scan_exclusive(s->slice_len, s->slice_base, s->slice_cap, s->scan_scratch, st);
  k_layout_slots<<<1, 64, 0, st>>>(s->slice_base, s->slice_cap, s->slot_cap, s->d_layout);
  if (n > 0)
    k_atom_rows<<<nblk, NT, 0, st>>>(n, s->bucket, s->row_of, s->d_layout, s->perm, s->slice_base, s->row_caller,
                                      s->slot0);
  k_slots<<<s->slice_cap, NT, 0, st>>>(s->d_layout, s->atom_of_row1, s->atom_of_rowx, s->nl_off, s->nl_j, s->nl_s,
                                       s->nl_rev, s->slot0, s->slice_base, s->w, s->sid, s->d_grids, s->slot_atom,
                                       s->slot_j, s->slot_rev, s->slot_d0, s->geom, bst);
  k_layout_status<<<1, 64, 0, st>>>(s->d_status, s->d_layout);
  HIPCHK(hipMemcpyAsync(s->h_info, s->d_layout, LY_N * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));      // the build's one wait
  const int* L = s->h_info;
  s->flags_at_build = L[LY_STATUS];
  s->flags_pending |= L[LY_STATUS];
  const int flags = L[LY_BUILD];
  if (flags & FLARE_FLAG_SPECIES) {
    set_error("species index outside [0, n_species)");
    return FLARE_E_SPECIES;
  }
  if (flags & FLARE_FLAG_NONFINITE) {
    set_error("non-finite position");
    return FLARE_E_NONFINITE;
  }
  if (L[LY_FLAGS] & 1) {
    set_error((flags & BUILD_OVERFLOW) || L[LY_PAIRS] < 0
                  ? std::string("list needs more than 2^31 pairs")
                  : "list needs " + std::to_string(L[LY_PAIRS]) + " pairs, state holds " +
                        std::to_string(s->max_pairs));
    return FLARE_E_CAPACITY;
  }
  if (L[LY_FLAGS] & 2) {
    set_error("sliced pair layout needs " + std::to_string(32LL * L[LY_SLOTS32]) + " slots, state holds " +
              std::to_string(s->slot_cap));
    return FLARE_E_CAPACITY;
  }
  if (flags & BUILD_ASYMMETRIC) {
    set_error("internal: neighbour list is not symmetric");
    return FLARE_E_HIP;
  }
  s->n_pairs = L[LY_PAIRS];
  for (int b = 0; b < NBUCKET; ++b) {
    s->bucket_count[b] = L[LY_COUNT + b];
    s->bucket_row0[b] = L[LY_ROW0 + b];
  }
  s->rows1 = L[LY_ROWS1];
  s->rowsx = L[LY_ROWSX];
  s->n_slices = L[LY_SLICES];
  s->n_slots = 32LL * L[LY_SLOTS32];
  return FLARE_OK;
}

}  // namespace flare
