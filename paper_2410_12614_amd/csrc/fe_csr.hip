// Global assembly A^g = L D L^T into CSR (Section 3.3).
//
// Symbolic phases (once per dof map):
//   COUNT: dof -> (cell, local index) adjacency by counting sort, every
//          adjacency list sorted so the order is deterministic; per row, the
//          dofs of all incident cells are sorted (bitonic, in LDS) and
//          de-duplicated to give the row length; an inclusive scan gives
//          row_ptr.
//   FILL:  the same per-row sort writes col_idx; then every local entry
//          (K, i, j) gets its position inside CSR row dof(K, i) as a 16-bit
//          rank (binary search of dof(K, j) in that row).
// Numeric phase (every call):
//   the cell kernels write the local matrices of all forms to the
//   workspace; one wave per CSR row then sums, in the fixed order of the
//   sorted adjacency list (cell ascending, then local row), the local rows
//   A_K(i, :) of the incident cells into an LDS window at their ranks and
//   writes the row once, coalesced.  No atomics touch values, so the result
//   is bitwise repeatable.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "fe_cell_kernel.h"
#include "fe_internal.h"

#include <map>
#include <mutex>
#include <vector>

namespace fe {
namespace {

struct PlanHeader {
  int32_t status;
  int32_t magic;
  int64_t n_cells, n_dofs;
  int32_t n_phi, pad;
  int64_t nnz, max_deg, max_len;
  int32_t ntasks;  // fused schedule: number of owner tasks (0 = not built)
  int32_t ntiles;
  int32_t span;    // CSR entries per task of the schedule
  int32_t elt;     // bytes per value of the forms it was built for (record layout)
};
constexpr int32_t PLAN_MAGIC = 0x46455043;  // "FEPC"

struct PlanLayout {
  size_t off_adj_ptr, off_cursor, off_adj, off_rank, off_srank, off_scan, off_tasks, off_lanes,
      total;
  size_t scan_blocks;
  int64_t tasks_max, tiles_max;
  int sstride;  // entries per pair of the schedule-order table
};

// Schedule-order rank rows hold a lane's four outputs per row tile in lane
// order, padded to a multiple of four entries so that every lane reads its
// four with one aligned 8-byte load.  With the single-precision output
// layout (rows 4 kb + r) entries past n_phi rounded up to four are padding
// only and are not stored; the FP64 layout (rows kb + 4 r) keeps whole
// 16-row tiles.
int sched_stride(int n_phi, bool f64rows) {
  return f64rows ? (n_phi + 15) / 16 * 16 : (n_phi + 3) / 4 * 4;
}

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int SCAN_TILE = 2048;  // elements per scan block (256 threads x 8)

PlanLayout plan_layout(int64_t n_cells, int n_phi, int64_t n_dofs, bool f64rows) {
  PlanLayout P;
  size_t off = 256;
  P.off_adj_ptr = off;
  off = a256(off + sizeof(int64_t) * (n_dofs + 1));
  P.off_cursor = off;
  off = a256(off + sizeof(int64_t) * n_dofs);
  P.off_adj = off;
  off = a256(off + sizeof(int64_t) * (size_t)n_cells * n_phi);
  P.sstride = sched_stride(n_phi, f64rows);
  P.off_rank = off;  // [n_cells][n_phi][n_phi]
  off = a256(off + sizeof(uint16_t) * (size_t)n_cells * n_phi * n_phi);
  P.off_srank = off;  // the same ranks in fused-schedule order (LDS offsets)
  off = a256(off + sizeof(uint16_t) * (size_t)n_cells * n_phi * P.sstride);
  P.scan_blocks = (size_t)(n_dofs + 1 + SCAN_TILE - 1) / SCAN_TILE;
  P.off_scan = off;
  off = a256(off + sizeof(int64_t) * (P.scan_blocks + 1));
  // Fused schedule.  A task holds at least FUSED_SPAN / 2 entries unless the
  // next row did not fit (then the next task holds more than FUSED_SPAN / 2)
  // or it closed on its tile cap, so for meshes whose rows have at most 32
  // incident pairs the number of tasks is below 4 nnz / SPAN + pairs / 32 + 2
  // with nnz <= pairs * n_phi; every task adds at most one partial tile.  A
  // schedule that does not fit is not used (the numeric phase then gathers).
  const int64_t pairs = n_cells * n_phi;
  P.tasks_max = std::min<int64_t>(n_dofs, 4 * pairs * n_phi / FUSED_SPAN + pairs / 32 + 2);
  P.tiles_max = (pairs + 15) / 16 + P.tasks_max;
  P.off_tasks = off;
  off = a256(off + sizeof(FusedTask) * P.tasks_max);
  P.off_lanes = off;
  off = a256(off + sizeof(FusedLane) * 16 * P.tiles_max);
  P.total = off;
  return P;
}

// Row-ownership schedule of the fused numeric path (host, once per dof map).
// Rows are packed in order into tasks of at most SPAN CSR entries (FUSED_SPAN,
// or FUSED_SPAN_BOX for hexahedral forms) and
// FUSED_TILE_MAX tiles of 16 (cell, local index) pairs.  Among the feasible
// ends of a task holding at least SPAN / 2 entries, the one whose pairs
// fill their tiles best is taken (then the longest), since idle lanes of a
// partial tile cost as much as busy ones.  The task's pairs are then dealt
// into tiles (below); lanes of one tile holding the same row carry
// increasing round numbers in adjacency order.  Returns false when a row is
// too long or has too many pairs, or the bounds of the layout would be
// exceeded.
bool build_fused_schedule(const std::vector<int64_t> &rp, const std::vector<int64_t> &ap,
                          const std::vector<int64_t> &adj, int64_t n_rows, int SPAN,
                          const PlanLayout &P, std::vector<FusedTask> &tasks,
                          std::vector<FusedLane> &lanes) {
  tasks.clear();
  lanes.clear();
  constexpr int64_t PAIRS_MAX = 16 * FUSED_TILE_MAX;
  int64_t r = 0, p0 = 0;
  while (r < n_rows) {
    const int64_t r0 = r;
    int64_t span = 0, npairs = 0;
    int64_t best_end = -1, best_pairs = 0, best_span = 0;
    while (r < n_rows) {
      const int64_t len = rp[r + 1] - rp[r], deg = ap[r + 1] - ap[r];
      if (len > SPAN || deg > PAIRS_MAX) return false;
      if (r > r0 && (span + len > SPAN || npairs + deg > PAIRS_MAX)) break;
      span += len;
      npairs += deg;
      ++r;
      if (2 * span >= SPAN) {
        // fill fraction npairs / (16 ceil(npairs / 16)), compared exactly
        const int64_t tiles = (npairs + 15) / 16, btiles = (best_pairs + 15) / 16;
        bool better = best_end < 0;
        if (!better) {
          const int64_t lhs = npairs * btiles, rhs = best_pairs * tiles;
          better = lhs > rhs || (lhs == rhs && span > best_span);
        }
        if (better) {
          best_end = r;
          best_pairs = npairs;
          best_span = span;
        }
      }
    }
    if (best_end > 0) {
      r = best_end;
      npairs = best_pairs;
    }
    const int64_t nr = r - r0;
    FusedTask tk;
    tk.r0 = (int32_t)r0;
    tk.t0 = (int32_t)(lanes.size() / 16);
    tk.base = rp[r0];
    tk.span = (int32_t)(rp[r] - rp[r0]);
    tk.p0 = (int32_t)p0;
    p0 += npairs;
    // Deal the pairs into nt tiles: the k-th of the d pairs of a row goes to
    // tile floor(k nt / d) or the next one with room, rows of many pairs
    // first, so every row is spread evenly and a tile holds few lanes of one
    // row (each repeat costs a scatter round).  Tiles stay in order along
    // every row, so each row's pairs keep their adjacency (cell ascending)
    // order; when that cannot be kept, the rows are swept instead, one pair
    // per row per sweep, filling tile after tile.
    const int nt = (int)((npairs + 15) / 16);
    std::vector<std::vector<int64_t>> tiles(nt);  // adjacency positions
    bool even = true;
    {
      std::vector<int64_t> order(nr);
      for (int64_t q = 0; q < nr; ++q) order[q] = q;
      std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
        return ap[r0 + x + 1] - ap[r0 + x] > ap[r0 + y + 1] - ap[r0 + y];
      });
      for (int64_t oi = 0; oi < nr && even; ++oi) {
        const int64_t g = r0 + order[oi], d = ap[g + 1] - ap[g];
        int last = 0;
        for (int64_t k = 0; k < d; ++k) {
          int t = std::max<int>(last, (int)(k * nt / d));
          while (t < nt && tiles[t].size() >= 16) ++t;
          if (t == nt) {
            even = false;
            break;
          }
          tiles[t].push_back(ap[g] + k);
          last = t;
        }
      }
    }
    if (!even) {
      for (auto &v : tiles) v.clear();
      std::vector<int64_t> cursor(nr, 0);
      int64_t left = npairs;
      for (int t = 0; t < nt; ++t)
        while (tiles[t].size() < 16 && left > 0)
          for (int64_t q = 0; q < nr && tiles[t].size() < 16; ++q) {
            const int64_t g = r0 + q;
            if (cursor[q] < ap[g + 1] - ap[g]) {
              tiles[t].push_back(ap[g] + cursor[q]++);
              --left;
            }
          }
    }
    int32_t pre = 0;  // real lanes before each tile, one byte per tile
    for (int t = 0, acc = 0; t < nt; ++t) {
      pre |= acc << (8 * t);
      acc += (int)tiles[t].size();
    }
    tk.pre = pre;
    for (int t = 0; t < nt; ++t) {
      // a tile's lanes in row order, then adjacency order within a row
      std::vector<int64_t> &v = tiles[t];
      std::sort(v.begin(), v.end());
      uint8_t maxr = 0;
      const size_t first = lanes.size();
      int64_t prev_row = -1;
      uint8_t rnd = 0;
      for (int64_t pos : v) {
        // row of adjacency position pos: the rows are ascending in pos
        const int64_t g = std::upper_bound(ap.begin() + r0, ap.begin() + r + 1, pos) - ap.begin() - 1;
        rnd = (g == prev_row) ? (uint8_t)(rnd + 1) : (uint8_t)0;
        prev_row = g;
        const int64_t ent = adj[pos];
        FusedLane L;
        L.cell = (int32_t)(ent >> ADJ_BITS);
        L.j = (uint8_t)(ent & ADJ_MASK);
        L.rowoff = (uint16_t)(rp[g] - rp[r0]);
        L.round = rnd;
        maxr = std::max(maxr, rnd);
        lanes.push_back(L);
      }
      // idle lanes take round 15, which no busy lane of a tile that has idle
      // lanes reaches (at most 15 busy lanes: rounds 0..14)
      for (size_t u = v.size(); u < 16; ++u) {
        FusedLane L;
        L.cell = -1;
        L.j = 0;
        L.rowoff = 0;
        L.round = 15;
        lanes.push_back(L);
      }
      // every lane also carries the tile's last round
      for (size_t u = first; u < lanes.size(); ++u) lanes[u].round |= (uint8_t)(maxr << 4);
    }
    tk.nt = nt;
    tasks.push_back(tk);
    if ((int64_t)tasks.size() > P.tasks_max || (int64_t)(lanes.size() / 16) > P.tiles_max) return false;
  }
  return true;
}

fe_status launch_fused(const FusedLaunch &a) {
  switch (a.L[0]->prec) {
    case FE_FP64: return launch_fused_fp64(a);
    case FE_FP32: return launch_fused_fp32(a);
    case FE_FP16_ACC32: return launch_fused_fp16(a);
    case FE_BF16_ACC32: return launch_fused_bf16(a);
    case FE_SPLITFP16_ACC32: return launch_fused_split(a);
  }
  return FE_EUNSUPPORTED;
}

// ---------------------------------------------------------------- kernels
__global__ void k_fill_i64(int64_t *x, int64_t n, int64_t v) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    x[t] = v;
}

__global__ void k_degree(const int32_t *dofmap, int64_t n_entries, int64_t n_dofs,
                         int64_t *deg /* [n_dofs+1], counts at g+1 */, int32_t *status) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_entries;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = dofmap[e];
    if (g < 0 || g >= n_dofs) {
      atomicOr(status, STATUS_BAD_DOF);
      continue;
    }
    atomicAdd((unsigned long long *)&deg[g + 1], 1ull);
  }
}

// Inclusive scan of x[0..n) in tiles of SCAN_TILE: per-tile scan + tile totals.
__global__ void k_scan_tiles(int64_t *x, int64_t n, int64_t *tile_sum) {
  __shared__ int64_t part[256];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * 8;
  int64_t v[8], run = 0;
  for (int e = 0; e < 8; ++e) {
    const int64_t idx = base + e;
    v[e] = idx < n ? x[idx] : 0;
    run += v[e];
    v[e] = run;
  }
  part[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int64_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  const int64_t prefix = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
  for (int e = 0; e < 8; ++e) {
    const int64_t idx = base + e;
    if (idx < n) x[idx] = v[e] + prefix;
  }
  if (threadIdx.x == 255) tile_sum[blockIdx.x] = part[255];
}

// Exclusive scan of the tile totals in one workgroup of SCAN_TOT threads:
// each thread sums a contiguous chunk, the chunk sums are scanned in LDS,
// then every thread writes its chunk's exclusive prefixes.
constexpr int SCAN_TOT = 1024;
__global__ __launch_bounds__(SCAN_TOT) void k_scan_totals(int64_t *tile_sum, int64_t nt) {
  __shared__ int64_t part[SCAN_TOT];
  const int64_t chunk = (nt + SCAN_TOT - 1) / SCAN_TOT;
  const int64_t t0 = (int64_t)threadIdx.x * chunk, t1 = min(nt, t0 + chunk);
  int64_t run = 0;
  for (int64_t t = t0; t < t1; ++t) run += tile_sum[t];
  part[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < SCAN_TOT; off <<= 1) {
    const int64_t add = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  run = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t v = tile_sum[t];
    tile_sum[t] = run;
    run += v;
  }
}

__global__ void k_scan_add(int64_t *x, int64_t n, const int64_t *tile_off) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  const int64_t add = tile_off[blockIdx.x];
  for (int e = threadIdx.x; e < SCAN_TILE; e += blockDim.x) {
    const int64_t idx = base + e;
    if (idx < n) x[idx] += add;
  }
}

__global__ void k_fill_adj(const int32_t *dofmap, int64_t n_cells, int n_phi, int64_t n_dofs,
                           const int64_t *adj_ptr, int64_t *cursor, int64_t *adj) {
  const int64_t n = n_cells * n_phi;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = dofmap[e];
    if (g < 0 || g >= n_dofs) continue;
    const int64_t K = e / n_phi, i = e - K * n_phi;
    const unsigned long long p = atomicAdd((unsigned long long *)&cursor[g], 1ull);
    adj[adj_ptr[g] + (int64_t)p] = (K << ADJ_BITS) + i;
  }
}

// Insertion sort of every adjacency list (lists are short: cells around a dof).
__global__ void k_sort_adj(const int64_t *adj_ptr, int64_t *adj, int64_t n_dofs,
                           int64_t *max_deg) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_dofs) return;
  const int64_t a0 = adj_ptr[g], a1 = adj_ptr[g + 1];
  for (int64_t a = a0 + 1; a < a1; ++a) {
    const int64_t v = adj[a];
    int64_t b = a - 1;
    while (b >= a0 && adj[b] > v) {
      adj[b + 1] = adj[b];
      --b;
    }
    adj[b + 1] = v;
  }
  atomicMax((unsigned long long *)max_deg, (unsigned long long)(a1 - a0));
}

// One workgroup per row: gather the dofs of every incident cell, bitonic sort
// in LDS, de-duplicate.  count mode: row length into rowlen[g+1]; fill mode:
// unique columns into col_idx[row_ptr[g] ...].
__global__ __launch_bounds__(256) void k_rows(const int32_t *dofmap, int n_phi,
                                              const int64_t *adj_ptr, const int64_t *adj,
                                              int64_t row0, int64_t n_rows, int64_t *rowlen,
                                              const int64_t *row_ptr, int32_t *col_idx,
                                              int64_t *max_len) {
  extern __shared__ int32_t buf[];
  __shared__ int32_t cnt[256];
  const int64_t g = row0 + blockIdx.x;
  if (g >= n_rows) return;
  const int64_t a0 = adj_ptr[g], a1 = adj_ptr[g + 1];
  const int n = (int)((a1 - a0) * n_phi);
  int npow = 1;
  while (npow < n) npow <<= 1;
  for (int t = threadIdx.x; t < npow; t += 256) {
    int32_t v = INT32_MAX;
    if (t < n) {
      const int64_t ent = adj[a0 + t / n_phi];
      v = dofmap[(ent >> ADJ_BITS) * n_phi + (t % n_phi)];
    }
    buf[t] = v;
  }
  __syncthreads();
  for (int k = 2; k <= npow; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < npow; t += 256) {
        const int ixj = t ^ j;
        if (ixj > t) {
          const int32_t a = buf[t], b = buf[ixj];
          const bool up = (t & k) == 0;
          if ((a > b) == up) {
            buf[t] = b;
            buf[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  // per-thread contiguous chunk of the sorted array
  const int chunk = (npow + 255) / 256;
  const int s0 = threadIdx.x * chunk;
  int local = 0;
  for (int t = s0; t < min(s0 + chunk, n); ++t)
    if (t == 0 || buf[t] != buf[t - 1]) ++local;
  cnt[threadIdx.x] = local;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int add = threadIdx.x >= off ? cnt[threadIdx.x - off] : 0;
    __syncthreads();
    cnt[threadIdx.x] += add;
    __syncthreads();
  }
  if (rowlen) {
    if (threadIdx.x == 0) {
      rowlen[g + 1] = cnt[255];
      atomicMax((unsigned long long *)max_len, (unsigned long long)cnt[255]);
    }
    return;
  }
  int pos = threadIdx.x > 0 ? cnt[threadIdx.x - 1] : 0;
  int32_t *out = col_idx + row_ptr[g];
  for (int t = s0; t < min(s0 + chunk, n); ++t)
    if (t == 0 || buf[t] != buf[t - 1]) out[pos++] = buf[t];
}

// One wave per local row (K, i): rank of every dof(K, j) inside CSR row dof(K, i).
__global__ __launch_bounds__(256) void k_ranks(const int32_t *dofmap, int64_t n_cells, int n_phi,
                                               const int64_t *row_ptr, const int32_t *col_idx,
                                               uint16_t *rank) {
  const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (e >= n_cells * n_phi) return;
  const int64_t K = e / n_phi;
  const int32_t g = dofmap[e];
  const int64_t r0 = row_ptr[g];
  const int64_t len = row_ptr[g + 1] - r0;
  const int32_t *row = col_idx + r0;
  for (int j = lane; j < n_phi; j += 64) {
    const int32_t h = dofmap[K * n_phi + j];
    int64_t lo = 0, hi = len;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (row[mid] < h) lo = mid + 1;
      else hi = mid;
    }
    rank[e * n_phi + j] = (uint16_t)lo;
  }
}

// Ranks in fused-schedule order: for the pair of schedule index p (tile
// column n of task tile t: p = p0 + pre[t] + n) and lane-order entry e
// (row tile mt = e/16, K-slot kb = e%16/4, output r = e%4 of the instruction,
// i.e. local row i = 16 mt + row(kb, r)), the LDS byte offset of the entry
// inside the owning wave's row buffer: rowoff + rank of dof(K, i) in row
// dof(K, j), or, for padding rows i >= n_phi, the private slot
// span + 16 kb + n of that lane.  One workgroup per task.
__global__ __launch_bounds__(64) void k_slot_ranks(const FusedTask *tasks, const FusedLane *lanes,
                                                   const uint16_t *rank, int n_phi, int sstride,
                                                   bool f64rows, int elt, int span, uint16_t *srank) {
  const FusedTask tk = tasks[blockIdx.x];
  const int nent = tk.nt * 16 * sstride;
  for (int u = threadIdx.x; u < nent; u += 64) {
    const int slot = u / sstride, e = u - slot * sstride;
    const FusedLane L = lanes[(size_t)tk.t0 * 16 + slot];
    if (L.cell < 0) continue;  // the pairs of a tile fill its first lanes
    const int n = slot & 15, mt = e >> 4, kb = (e & 15) >> 2, r = e & 3;
    const int pair = tk.p0 + ((tk.pre >> (8 * (slot >> 4))) & 0xff) + n;
    const int i = mt * 16 + (f64rows ? kb + 4 * r : 4 * kb + r);
    const int off = i < n_phi ? L.rowoff + rank[((size_t)L.cell * n_phi + L.j) * n_phi + i]
                              : span + 16 * kb + n;
    srank[(size_t)pair * sstride + e] = (uint16_t)(off * elt);
  }
}

// Numeric gather: NF forms, LDS window of W entries per form.  Each wave
// walks a block of consecutive CSR rows.  A row's incident local rows are
// visited in adjacency order (cell ascending, then local index), each whole
// (its n_phi <= 64 CH entries in chunks of 64 lanes); their loads are issued
// GROUP local rows at a time and the LDS additions then applied local row
// after local row, so every entry is summed in cell-ascending order.
// Software pipeline over the rows: while row g is summed, the ranks and
// values of row g + 1's first GROUP local rows and the extents and first
// adjacency entries of row g + 2 are in flight (extents, entries and values
// are three dependent memory round trips per row).
constexpr int GATHER_W = 512;
constexpr int GATHER_GROUP = 4;
constexpr int GATHER_CH = 8;     // chunks of the longest local row (n_phi <= 512)
constexpr int GATHER_ROWS = 32;  // consecutive rows per wave

// Ranks and values of the GROUP local rows whose adjacency entries lanes
// 0..GROUP-1 of `mine` hold (-1: none).  Ranks are raw positions in the row.
template <class T, int NF, int CH>
__device__ __forceinline__ void gather_group_load(int64_t mine, int lane, int n_phi,
                                                  const uint16_t *rank, const T *const *A,
                                                  int (&rk)[GATHER_GROUP][CH],
                                                  T (&v)[GATHER_GROUP][CH][NF]) {
#pragma unroll
  for (int u = 0; u < GATHER_GROUP; ++u) {
    const int lo = __shfl((int)(mine & 0xffffffff), u), hi = __shfl((int)(mine >> 32), u);
    const int64_t e = ((int64_t)hi << 32) | (uint32_t)lo;
    const size_t row = e < 0 ? 0 : (size_t)(e >> ADJ_BITS) * n_phi + (e & ADJ_MASK);
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
      const int j = 64 * ch + lane;
      rk[u][ch] = -1;
#pragma unroll
      for (int f = 0; f < NF; ++f) v[u][ch][f] = 0;
      if (e >= 0 && j < n_phi) {
        const size_t base = row * n_phi + j;
        rk[u][ch] = (int)rank[base];
#pragma unroll
        for (int f = 0; f < NF; ++f) v[u][ch][f] = A[f][base];
      }
    }
  }
}

// LDS additions of one group into the window [w0, w0 + wl), local row
// after local row.
template <class T, int NF, int CH, int W>
__device__ __forceinline__ void gather_group_add(const int (&rk)[GATHER_GROUP][CH],
                                                 const T (&v)[GATHER_GROUP][CH][NF], int w0, int wl,
                                                 T (*buf)[W]) {
#pragma unroll
  for (int u = 0; u < GATHER_GROUP; ++u)
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
      const int r = rk[u][ch] - w0;
      if (rk[u][ch] >= 0 && r >= 0 && r < wl) {
#pragma unroll
        for (int f = 0; f < NF; ++f) buf[f][r] += v[u][ch][f];
      }
    }
}

template <class T, int NF, int CH>
__global__ __launch_bounds__(256) void k_gather(const int64_t *adj_ptr, const int64_t *adj,
                                                const uint16_t *rank, const int64_t *row_ptr,
                                                int64_t n_rows, int n_phi,
                                                const T *A0, const T *A1, const T *A2,
                                                const T *A3, T *V0, T *V1, T *V2, T *V3) {
  constexpr int W = GATHER_W;
  constexpr int G = GATHER_GROUP;
  __shared__ T sbuf[4][NF][W];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t first = ((int64_t)blockIdx.x * 4 + wave) * GATHER_ROWS;
  if (first >= n_rows) return;
  const int64_t last = min(first + (int64_t)GATHER_ROWS, n_rows);
  T (*buf)[W] = sbuf[wave];
  const T *A[4] = {A0, A1, A2, A3};
  T *V[4] = {V0, V1, V2, V3};
  auto entries = [&](int64_t a, int64_t a_end) -> int64_t {
    return (lane < G && a + lane < a_end) ? adj[a + lane] : -1;
  };
  // row g: extents r0, r1, a0, a1 and its first group loaded (rk0, v0);
  // row g + 1: extents up to r2, a2 and its first entries ent1
  int64_t r0 = row_ptr[first], r1 = row_ptr[first + 1];
  int64_t a0 = adj_ptr[first], a1 = adj_ptr[first + 1];
  int rk0[G][CH];
  T v0[G][CH][NF];
  gather_group_load<T, NF, CH>(entries(a0, a1), lane, n_phi, rank, A, rk0, v0);
  int64_t r2 = r1, a2 = a1, ent1 = -1;
  if (first + 1 < last) {
    r2 = row_ptr[first + 2];
    a2 = adj_ptr[first + 2];
    ent1 = entries(a1, a2);
  }
  for (int64_t g = first; g < last; ++g) {
    // in flight during row g: row g + 1's first group, row g + 2's extents
    int rk1[G][CH];
    T v1[G][CH][NF];
    gather_group_load<T, NF, CH>(g + 1 < last ? ent1 : (int64_t)-1, lane, n_phi, rank, A, rk1, v1);
    int64_t r3 = r2, a3 = a2, ent2 = -1;
    if (g + 2 < last) {
      r3 = row_ptr[g + 3];
      a3 = adj_ptr[g + 3];
      ent2 = entries(a2, a3);
    }
    const int len = (int)(r1 - r0);
    for (int w0 = 0; w0 < len; w0 += W) {
      const int wl = min(W, len - w0);
      for (int r = lane; r < wl; r += 64)
#pragma unroll
        for (int f = 0; f < NF; ++f) buf[f][r] = 0;
      gather_group_add<T, NF, CH, W>(rk0, v0, w0, wl, buf);
      for (int64_t a = a0 + G; a < a1; a += G) {
        int rk[G][CH];
        T v[G][CH][NF];
        gather_group_load<T, NF, CH>(entries(a, a1), lane, n_phi, rank, A, rk, v);
        gather_group_add<T, NF, CH, W>(rk, v, w0, wl, buf);
      }
      for (int r = lane; r < wl; r += 64)
#pragma unroll
        for (int f = 0; f < NF; ++f) V[f][r0 + w0 + r] = buf[f][r];
    }
    r0 = r1;
    r1 = r2;
    r2 = r3;
    a0 = a1;
    a1 = a2;
    a2 = a3;
    ent1 = ent2;
#pragma unroll
    for (int u = 0; u < G; ++u)
#pragma unroll
      for (int ch = 0; ch < CH; ++ch) {
        rk0[u][ch] = rk1[u][ch];
#pragma unroll
        for (int f = 0; f < NF; ++f) v0[u][ch][f] = v1[u][ch][f];
      }
  }
}

// Numeric gather over a flat stream of local rows.  A wave owns FLAT_ROWS
// consecutive CSR rows; their incident local rows are consecutive in the
// adjacency, so the wave walks them as one stream in groups of FLAT_G,
// whatever row each belongs to.  The rows are cut into windows of at most
// W CSR entries (whole rows) kept in LDS; a group never straddles two
// windows.  Three stages overlap: the adjacency entries of group k + 2, the
// ranks and values of group k + 1 and the LDS additions of group k (local
// row after local row, so every entry is still summed in adjacency order,
// cell ascending).  A window is written out (coalesced) after its last
// group and cleared as it is read, so it starts at zero.  Every load is
// issued unconditionally (clamped addresses, out-of-range parts marked) so
// that the compiler's counts of memory operations in flight are exact.
// Rows must be at most W entries long (checked by the caller).
constexpr int FLAT_ROWS = 32;
constexpr int FLAT_G = 8;

struct FlatGroup {
  int a, n;       // first adjacency index (relative to the wave's first row) and count
  int r0, r1;     // the window's rows [r0, r1) (relative)
  bool valid, last;
};

template <class T, int NF, int CH, int W>
__global__ __launch_bounds__(256) void k_gather_flat(const int64_t *adj_ptr, const int64_t *adj,
                                                     const uint16_t *rank, const int64_t *row_ptr,
                                                     int64_t n_rows, int n_phi, const T *A0, const T *A1,
                                                     const T *A2, const T *A3, T *V0, T *V1, T *V2,
                                                     T *V3) {
  constexpr int G = FLAT_G;
  __shared__ T sbuf[4][NF][W];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t first = ((int64_t)blockIdx.x * 4 + wave) * FLAT_ROWS;
  if (first >= n_rows) return;
  const int nr = (int)min((int64_t)FLAT_ROWS, n_rows - first);
  T (*buf)[W] = sbuf[wave];
  const T *A[4] = {A0, A1, A2, A3};
  T *V[4] = {V0, V1, V2, V3};
  // lane l <= nr: the starts of row first + l in the CSR values and in the
  // adjacency, relative to row first's
  const int64_t rbase = row_ptr[first], abase = adj_ptr[first];
  const int64_t alast = adj_ptr[n_rows] - 1;  // the last adjacency entry (the mesh has cells)
  int rp = 0, ap = 0;
  if (lane <= nr) {
    rp = (int)(row_ptr[first + lane] - rbase);
    ap = (int)(adj_ptr[first + lane] - abase);
  }
  auto rp_of = [&](int r) { return __builtin_amdgcn_readlane(rp, r); };
  auto ap_of = [&](int r) { return __builtin_amdgcn_readlane(ap, r); };
  // the window starting at row r0: the rows whose entries fit W
  auto window_end = [&](int r0) {
    const unsigned long long m = __ballot(lane <= nr && lane > r0 && rp - rp_of(r0) <= W);
    return 63 - __builtin_clzll(m);
  };
  for (int t = lane; t < W; t += 64)
#pragma unroll
    for (int f = 0; f < NF; ++f) buf[f][t] = 0;

  // group cursor
  int cr0 = 0, cr1 = window_end(0), ca = 0, ca_end = ap_of(cr1);
  auto next_group = [&]() {
    FlatGroup g;
    g.valid = cr0 < nr;
    g.a = ca;
    g.n = g.valid ? min(G, ca_end - ca) : 0;
    g.r0 = cr0;
    g.r1 = cr1;
    g.last = g.valid && ca + g.n == ca_end;
    if (g.valid) {
      ca += g.n;
      if (ca == ca_end) {
        cr0 = cr1;
        if (cr0 < nr) {
          cr1 = window_end(cr0);
          ca_end = ap_of(cr1);
        }
      }
    }
    return g;
  };
  // adjacency entries of a group: lane u < G holds entry a + u (clamped to
  // the group; -1 marks lanes past it and invalid groups)
  auto load_entries = [&](const FlatGroup &g, int64_t &ent) {
    const int u = lane < G ? lane : 0;
    const int idx = g.n > 0 ? g.a + min(u, g.n - 1) : 0;
    // (the loaded value is used on both sides, so the load is not made
    // conditional on the lane)
    const int64_t e = adj[min(abase + idx, alast)];
    ent = e | ((g.valid && lane < g.n) ? (int64_t)0 : INT64_MIN);
  };
  // ranks and values of a group's local rows (rank -1: nothing to add)
  auto load_rows = [&](int64_t ent, int (&rk)[G][CH], T (&v)[G][CH][NF]) {
    const int64_t e0 = ((int64_t)__shfl((int)(ent >> 32), 0) << 32) | (uint32_t)__shfl((int)(ent & 0xffffffff), 0);
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int lo = __shfl((int)(ent & 0xffffffff), u), hi = __shfl((int)(ent >> 32), u);
      const int64_t e = ((int64_t)hi << 32) | (uint32_t)lo;
      const int64_t ec = e >= 0 ? e : (e0 >= 0 ? e0 : 0);  // a valid local row to read
      const size_t row = (size_t)(ec >> ADJ_BITS) * n_phi + (ec & ADJ_MASK);
#pragma unroll
      for (int ch = 0; ch < CH; ++ch) {
        const int j = 64 * ch + lane;
        const size_t base = row * n_phi + min(j, n_phi - 1);
        const int r = (int)rank[base];
        rk[u][ch] = r - ((e >= 0 && j < n_phi) ? 0 : 0x10000);
#pragma unroll
        for (int f = 0; f < NF; ++f) v[u][ch][f] = A[f][base];
      }
    }
  };
  // additions of a group into the window of rows [r0, r1)
  auto add_rows = [&](const FlatGroup &g, const int (&rk)[G][CH], const T (&v)[G][CH][NF]) {
    const int w0 = rp_of(g.r0);
#pragma unroll
    for (int u = 0; u < G; ++u) {
      if (u >= g.n) break;
      // the row of local row a + u: the last row starting at or before it
      const int ridx = __popcll(__ballot(lane <= nr && ap <= g.a + u)) - 1;
      const int off = rp_of(ridx) - w0;
#pragma unroll
      for (int ch = 0; ch < CH; ++ch)
        if (rk[u][ch] >= 0)
#pragma unroll
          for (int f = 0; f < NF; ++f) buf[f][off + rk[u][ch]] += v[u][ch][f];
    }
    if (g.last) {
      // the window's rows out, the window cleared
      const int span = rp_of(g.r1) - w0;
      const int64_t o = rbase + w0;
      for (int t = lane; t < span; t += 64)
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          V[f][o + t] = buf[f][t];
          buf[f][t] = 0;
        }
    }
  };

  // two register sets used in turn (no copies of loaded registers: a copy
  // would wait for the load): group g0's rows in set A, group g1's entries
  // in eB
  FlatGroup g0 = next_group(), g1 = next_group();
  int64_t eA, eB;
  load_entries(g0, eA);
  load_entries(g1, eB);
  int rkA[G][CH], rkB[G][CH];
  T vA[G][CH][NF], vB[G][CH][NF];
  load_rows(eA, rkA, vA);
  while (g0.valid) {
    const FlatGroup g2 = next_group();
    load_entries(g2, eA);
    load_rows(eB, rkB, vB);
    add_rows(g0, rkA, vA);
    if (!g1.valid) break;
    const FlatGroup g3 = next_group();
    load_entries(g3, eB);
    load_rows(eA, rkA, vA);
    add_rows(g1, rkB, vB);
    g0 = g2;
    g1 = g3;
  }
}

template <class T, int NF>
fe_status launch_gather(const int64_t *adj_ptr, const int64_t *adj, const uint16_t *rank,
                        const int64_t *row_ptr, int64_t n_rows, int n_phi, int64_t max_len,
                        void *const *A, void *const *V, hipStream_t s) {
  if (n_phi > 64 * GATHER_CH) return FE_EUNSUPPORTED;
  // the flat stream where the rows fit its window (and the local rows its
  // chunks)
  constexpr int FW = sizeof(T) * NF <= 4 ? 2048 : 1024;
  if (sizeof(T) * NF <= 8 && max_len <= FW && n_phi <= 128) {
    const int64_t waves = (n_rows + FLAT_ROWS - 1) / FLAT_ROWS;
    auto kern = n_phi <= 64 ? k_gather_flat<T, NF, 1, FW> : k_gather_flat<T, NF, 2, FW>;
    hipLaunchKernelGGL(kern, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, adj_ptr, adj, rank,
                       row_ptr, n_rows, n_phi, (const T *)A[0], (const T *)A[1], (const T *)A[2],
                       (const T *)A[3], (T *)V[0], (T *)V[1], (T *)V[2], (T *)V[3]);
    return hipGetLastError() == hipSuccess ? FE_OK : FE_EHIP;
  }
  const int64_t waves = (n_rows + GATHER_ROWS - 1) / GATHER_ROWS;
  const int64_t blocks = (waves + 3) / 4;
  auto kern = n_phi <= 64    ? k_gather<T, NF, 1>
              : n_phi <= 128 ? k_gather<T, NF, 2>
              : n_phi <= 192 ? k_gather<T, NF, 3>
              : n_phi <= 256 ? k_gather<T, NF, 4>
                             : k_gather<T, NF, 8>;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, s, adj_ptr, adj, rank,
                     row_ptr, n_rows, n_phi, (const T *)A[0], (const T *)A[1], (const T *)A[2],
                     (const T *)A[3], (T *)V[0], (T *)V[1], (T *)V[2], (T *)V[3]);
  return hipGetLastError() == hipSuccess ? FE_OK : FE_EHIP;
}

unsigned grid_for(int64_t n, int block) {
  int64_t b = (n + block - 1) / block;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 65536 * 4));
}

fe_status scan_inclusive(int64_t *x, int64_t n, int64_t *scratch, size_t tiles, hipStream_t s) {
  if (n <= 0) return FE_OK;
  const int64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
  if ((size_t)nt > tiles) return FE_EINVAL;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(256), 0, s, x, n, scratch);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(SCAN_TOT), 0, s, scratch, nt);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nt), dim3(256), 0, s, x, n, scratch);
  return hipGetLastError() == hipSuccess ? FE_OK : FE_EHIP;
}

bool sync_ok(hipStream_t s) { return hipStreamSynchronize(s) == hipSuccess; }

}  // namespace
}  // namespace fe

using namespace fe;

// compact: the workspace holds only what the fused path reads (no local
// matrices), and every form must take the fused path (the allocation-free
// entry point, whose workspace is the static scratch array below).
static fe_status assemble_csr(const fe_form_desc *forms, const void *const *form_bufs,
                              int32_t n_forms, const fe_mesh_view *m, int32_t phase,
                              fe_csr *mats, void *plan, size_t *plan_bytes,
                              void *workspace, size_t *ws_bytes, void *stream, bool compact) {
  if (!forms || n_forms < 1 || n_forms > 4 || !m) return FE_EINVAL;
  FormLayout L[4];
  for (int f = 0; f < n_forms; ++f) {
    fe_status st = compute_layout(&forms[f], &L[f]);
    if (st != FE_OK) return st;
    if (forms[f].cell != forms[0].cell || forms[f].degree != forms[0].degree) return FE_EINVAL;
    if ((forms[f].precision == FE_FP64) != (forms[0].precision == FE_FP64)) return FE_EINVAL;
    if (forms[f].geom_precision != forms[0].geom_precision) return FE_EINVAL;
  }
  if (m->n_cells < 0 || m->n_dofs < 1) return FE_EINVAL;
  if (m->n_dofs >= INT32_MAX) return FE_EOVERFLOW;
  const int n_phi = L[0].n_phi;
  const int64_t n_cells = m->n_cells, n_dofs = m->n_dofs;
  const size_t elt = (forms[0].precision == FE_FP64) ? 8 : 4;
  const PlanLayout P = plan_layout(n_cells, n_phi, n_dofs, forms[0].precision == FE_FP64);
  const size_t geo_offset = compact ? 0 : a256((size_t)n_forms * n_cells * n_phi * n_phi * elt);
  // per-form factor records of the fused path (FormGeo<double> is the larger)
  const size_t geo_bytes = a256(sizeof(FormGeo<double>) * (size_t)n_cells);
  // hexahedra: per-form per-point factors [n_cells][n_q_pad] (at most FP64)
  const size_t zpt_offset = geo_offset + (size_t)n_forms * geo_bytes;
  size_t zpt_bytes = 0;
  for (int f = 0; f < n_forms; ++f)
    if (L[f].box) zpt_bytes = std::max(zpt_bytes, a256((size_t)n_cells * L[f].n_q_pad * 8));
  // coefficient forms of the whole-cell kernel: the coefficient at the
  // points [n_cells][n_q_pad], its maximum per cell (FP32) and the cell
  // factors (32 bytes per cell), one region
  // shared by those forms (they run one after the other on the stream)
  const size_t zc_offset = zpt_offset + (size_t)n_forms * zpt_bytes;
  size_t zc_bytes = 0, zc_pts = 0;
  for (int f = 0; f < n_forms; ++f)
    if (forms[f].has_coeff && cellwise_eligible(L[f])) {
      zc_pts = std::max(zc_pts, a256((size_t)n_cells * L[f].n_q_pad * sizeof(float)));
      zc_bytes = zc_pts + a256((size_t)n_cells * sizeof(float)) + a256((size_t)n_cells * 32);
    }
  const size_t ws_need = std::max<size_t>(256, zc_offset + zc_bytes);
  const bool numeric = phase == FE_NUMERIC || phase == FE_NUMERIC_GATHER ||
                       phase == FE_NUMERIC_GEOMETRY || phase == FE_NUMERIC_FUSED ||
                       phase == FE_NUMERIC_LOCAL || phase == FE_NUMERIC_ASSEMBLE;
  if (!plan || (numeric && !workspace)) {
    if (!plan_bytes && !ws_bytes) return FE_EINVAL;
    if (plan_bytes) *plan_bytes = P.total;
    if (ws_bytes) *ws_bytes = ws_need;
    return FE_OK;
  }
  if (plan_bytes && *plan_bytes < P.total) return FE_ESIZE;
  if (!mats || !mats[0].row_ptr) return FE_EINVAL;
  if (n_cells > 0 && (!m->dofmap || !m->cell_coords)) return FE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  unsigned char *pb = (unsigned char *)plan;
  PlanHeader *hdr_d = (PlanHeader *)pb;
  int64_t *adj_ptr = (int64_t *)(pb + P.off_adj_ptr);
  int64_t *cursor = (int64_t *)(pb + P.off_cursor);
  int64_t *adj = (int64_t *)(pb + P.off_adj);
  uint16_t *rank = (uint16_t *)(pb + P.off_rank);
  int64_t *scan = (int64_t *)(pb + P.off_scan);
  int64_t *row_ptr = mats[0].row_ptr;

  if (phase == FE_SYMBOLIC_COUNT) {
    PlanHeader h;
    std::memset(&h, 0, sizeof(h));
    h.magic = PLAN_MAGIC;
    h.n_cells = n_cells;
    h.n_dofs = n_dofs;
    h.n_phi = n_phi;
    if (hipMemcpyAsync(hdr_d, &h, sizeof(h), hipMemcpyHostToDevice, s) != hipSuccess) return FE_EHIP;
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n_dofs + 1, 256)), dim3(256), 0, s, adj_ptr,
                       n_dofs + 1, (int64_t)0);
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n_dofs, 256)), dim3(256), 0, s, cursor, n_dofs,
                       (int64_t)0);
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n_dofs + 1, 256)), dim3(256), 0, s, row_ptr,
                       n_dofs + 1, (int64_t)0);
    if (n_cells > 0) {
      hipLaunchKernelGGL(k_degree, dim3(grid_for(n_cells * n_phi, 256)), dim3(256), 0, s, m->dofmap,
                         n_cells * n_phi, n_dofs, adj_ptr, &hdr_d->status);
      fe_status st = scan_inclusive(adj_ptr + 1, n_dofs, scan, P.scan_blocks, s);
      if (st != FE_OK) return st;
      hipLaunchKernelGGL(k_fill_adj, dim3(grid_for(n_cells * n_phi, 256)), dim3(256), 0, s,
                         m->dofmap, n_cells, n_phi, n_dofs, adj_ptr, cursor, adj);
      hipLaunchKernelGGL(k_sort_adj, dim3((unsigned)((n_dofs + 255) / 256)), dim3(256), 0, s,
                         adj_ptr, adj, n_dofs, &hdr_d->max_deg);
    }
    if (!sync_ok(s)) return FE_EHIP;
    if (hipMemcpy(&h, hdr_d, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return FE_EHIP;
    if (h.status & STATUS_BAD_DOF) return FE_EINVAL;
    const int64_t ncand = h.max_deg * n_phi;
    int64_t cap = 1;
    while (cap < ncand) cap <<= 1;
    if (cap > 32768) return FE_EUNSUPPORTED;
    const size_t smem = sizeof(int32_t) * (size_t)std::max<int64_t>(cap, 1);
    if (smem > 65536 && hipFuncSetAttribute((const void *)k_rows,
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)smem) != hipSuccess)
      return FE_EHIP;
    for (int64_t r0 = 0; r0 < n_dofs; r0 += (int64_t)1 << 30)
      hipLaunchKernelGGL(k_rows, dim3((unsigned)std::min<int64_t>(n_dofs - r0, (int64_t)1 << 30)),
                         dim3(256), smem, s, m->dofmap, n_phi, adj_ptr, adj, r0, n_dofs, row_ptr,
                         (const int64_t *)nullptr, (int32_t *)nullptr, &hdr_d->max_len);
    fe_status st = scan_inclusive(row_ptr + 1, n_dofs, scan, P.scan_blocks, s);
    if (st != FE_OK) return st;
    if (!sync_ok(s)) return FE_EHIP;
    int64_t nnz = 0;
    if (hipMemcpy(&nnz, row_ptr + n_dofs, sizeof(nnz), hipMemcpyDeviceToHost) != hipSuccess)
      return FE_EHIP;
    if (hipMemcpy(&h, hdr_d, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return FE_EHIP;
    h.nnz = nnz;
    if (hipMemcpy(hdr_d, &h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) return FE_EHIP;
    for (int f = 0; f < n_forms; ++f) {
      mats[f].n_rows = n_dofs;
      mats[f].nnz = nnz;
      mats[f].max_row_len = h.max_len;
    }
    if (h.max_len >= 65536) return FE_EOVERFLOW;
    return FE_OK;
  }

  PlanHeader h;
  if (phase == FE_SYMBOLIC_FILL) {
    if (!mats[0].col_idx) return FE_EINVAL;
    if (!sync_ok(s)) return FE_EHIP;
    if (hipMemcpy(&h, hdr_d, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return FE_EHIP;
    if (h.magic != PLAN_MAGIC || h.n_cells != n_cells || h.n_dofs != n_dofs || h.n_phi != n_phi)
      return FE_EINVAL;
    if (h.max_len >= 65536) return FE_EOVERFLOW;
    const int64_t ncand = h.max_deg * n_phi;
    int64_t cap = 1;
    while (cap < ncand) cap <<= 1;
    const size_t smem = sizeof(int32_t) * (size_t)std::max<int64_t>(cap, 1);
    if (smem > 65536 && hipFuncSetAttribute((const void *)k_rows,
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)smem) != hipSuccess)
      return FE_EHIP;
    for (int64_t r0 = 0; r0 < n_dofs; r0 += (int64_t)1 << 30)
      hipLaunchKernelGGL(k_rows, dim3((unsigned)std::min<int64_t>(n_dofs - r0, (int64_t)1 << 30)),
                         dim3(256), smem, s, m->dofmap, n_phi, adj_ptr, adj, r0, n_dofs,
                         (int64_t *)nullptr, (const int64_t *)row_ptr, mats[0].col_idx,
                         &hdr_d->max_len);
    if (n_cells > 0) {
      const int64_t ne = n_cells * n_phi;
      hipLaunchKernelGGL(k_ranks, dim3((unsigned)((ne + 3) / 4)), dim3(256), 0, s, m->dofmap,
                         n_cells, n_phi, (const int64_t *)row_ptr, mats[0].col_idx, rank);
    }
    if (hipGetLastError() != hipSuccess) return FE_EHIP;
    if (!sync_ok(s)) return FE_EHIP;
    // fused schedule (host): needs row_ptr and the sorted adjacency; built
    // only when one of the forms can take the fused path
    h.ntasks = 0;
    h.ntiles = 0;
    // task span: longer for hexahedral forms (all forms share the cell type)
    const int span = assembly_span(L, n_forms);
    h.span = span;
    h.elt = (int32_t)elt;
    bool any_fused = false;
    for (int f = 0; f < n_forms; ++f) any_fused = any_fused || fused_eligible(L[f]);
    if (any_fused && h.max_len <= span && n_cells > 0) {
      std::vector<int64_t> rp(n_dofs + 1), apv(n_dofs + 1), adjv((size_t)n_cells * n_phi);
      if (hipMemcpy(rp.data(), row_ptr, sizeof(int64_t) * rp.size(), hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(apv.data(), adj_ptr, sizeof(int64_t) * apv.size(), hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(adjv.data(), adj, sizeof(int64_t) * adjv.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return FE_EHIP;
      std::vector<FusedTask> tasks;
      std::vector<FusedLane> lanes;
      if (build_fused_schedule(rp, apv, adjv, n_dofs, span, P, tasks, lanes)) {
        if (hipMemcpy(pb + P.off_tasks, tasks.data(), sizeof(FusedTask) * tasks.size(),
                      hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(pb + P.off_lanes, lanes.data(), sizeof(FusedLane) * lanes.size(),
                      hipMemcpyHostToDevice) != hipSuccess)
          return FE_EHIP;
        h.ntasks = (int32_t)tasks.size();
        h.ntiles = (int32_t)(lanes.size() / 16);
        hipLaunchKernelGGL(k_slot_ranks, dim3((unsigned)tasks.size()), dim3(64), 0, s,
                           (const FusedTask *)(pb + P.off_tasks),
                           (const FusedLane *)(pb + P.off_lanes), (const uint16_t *)rank, n_phi,
                           P.sstride, forms[0].precision == FE_FP64, (int)elt, span,
                           (uint16_t *)(pb + P.off_srank));
        if (hipGetLastError() != hipSuccess || !sync_ok(s)) return FE_EHIP;
      }
    }
    if (hipMemcpy(hdr_d, &h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) return FE_EHIP;
    for (int f = 0; f < n_forms; ++f) {
      mats[f].schedule = h.ntasks;
      mats[f].schedule_span = h.ntasks > 0 ? span : 0;
      mats[f].schedule_elt = h.ntasks > 0 ? (int32_t)elt : 0;
    }
    return FE_OK;
  }

  if (!numeric) return FE_EINVAL;
  if (ws_bytes && *ws_bytes < ws_need) return FE_ESIZE;
  if (!mats[0].col_idx) return FE_EINVAL;
  for (int f = 0; f < n_forms; ++f)
    if (!form_bufs || !form_bufs[f] || !mats[f].values) return FE_EINVAL;
  if (n_cells == 0) return FE_OK;  // values of an empty pattern: nothing to write
  // The schedule's task span and record layout were fixed by the forms of the
  // FILL call: a schedule built for other forms (another value type, or a
  // span these forms' row buffers cannot hold) is not used.
  const bool sched_ok = mats[0].schedule > 0 && mats[0].schedule_span == assembly_span(L, n_forms) &&
                        mats[0].schedule_elt == (int32_t)elt;
  if ((phase == FE_NUMERIC_GEOMETRY || phase == FE_NUMERIC_FUSED) && mats[0].schedule > 0 && !sched_ok)
    return FE_EINVAL;
  // Forms whose tables fit on chip take the fused row-ownership path when the
  // FILL phase built its schedule; the others (coefficient forms, tables too
  // large) take the cell kernels and the row gather.
  bool on_fused[4] = {false, false, false, false};
  int n_fused = 0;
  // the halves of the gather path (LOCAL: cell kernels into the workspace,
  // ASSEMBLE: the row gather from it) take every form through the workspace
  const bool via_ws = phase == FE_NUMERIC_GATHER || phase == FE_NUMERIC_LOCAL ||
                      phase == FE_NUMERIC_ASSEMBLE;
  for (int f = 0; f < n_forms; ++f) {
    on_fused[f] = !via_ws && sched_ok && fused_eligible(L[f]);
    n_fused += on_fused[f] ? 1 : 0;
  }
  if ((phase == FE_NUMERIC_GEOMETRY || phase == FE_NUMERIC_FUSED || compact) && n_fused < n_forms)
    return FE_EUNSUPPORTED;
  {
    int fl[4], nf = 0;
    for (int f = 0; f < n_forms; ++f)
      if (on_fused[f]) fl[nf++] = f;
    // passes: two forms share one pass when they fit it together
    const FormLayout *pairL[2] = {&L[fl[0]], nf > 1 ? &L[fl[1]] : &L[fl[0]]};
    const bool pair = nf == 2 && fused_pair_fits(pairL) && !pairL[0]->box && !pairL[1]->box;
    for (int i = 0; i < nf; i += pair ? 2 : 1) {
      const int f = fl[i];
      FusedLaunch a;
      // the first fused form of each precision runs the geometry pass of all
      // fused forms of that precision
      a.geo_forms = 0;
      a.run_fused = phase != FE_NUMERIC_GEOMETRY;
      bool first = phase != FE_NUMERIC_FUSED;
      for (int e = 0; e < i; ++e) first = first && forms[fl[e]].precision != forms[f].precision;
      if (first)
        for (int e = i; e < nf; ++e)
          if (forms[fl[e]].precision == forms[f].precision) {
            a.geo_bufs[a.geo_forms] = (const unsigned char *)form_bufs[fl[e]];
            a.geo_nd[a.geo_forms] = L[fl[e]].nd;
            a.geo_out[a.geo_forms] = (unsigned char *)workspace + geo_offset + fl[e] * geo_bytes;
            a.geo_zpt[a.geo_forms] =
                L[fl[e]].box ? (unsigned char *)workspace + zpt_offset + fl[e] * zpt_bytes : nullptr;
            a.geo_L[a.geo_forms] = &L[fl[e]];
            ++a.geo_forms;
          }
      a.nforms = pair ? 2 : 1;
      // a pair runs the form with more derivative slabs first: the next
      // task's factors are then held only during the lighter form
      const bool swap = pair && L[fl[0]].ndt < L[fl[1]].ndt;
      for (int e = 0; e < a.nforms; ++e) {
        const int g = fl[i + (swap ? 1 - e : e)];
        a.L[e] = &L[g];
        a.form_buf[e] = (const unsigned char *)form_bufs[g];
        a.geo[e] = (unsigned char *)workspace + geo_offset + g * geo_bytes;
        a.zpt[e] = L[g].box ? (unsigned char *)workspace + zpt_offset + g * zpt_bytes : nullptr;
        a.values[e] = mats[g].values;
      }
      a.coords = m->cell_coords;
      a.n_cells = n_cells;
      a.tasks = (const FusedTask *)(pb + P.off_tasks);
      a.ntasks = mats[0].schedule;
      a.lanes = (const FusedLane *)(pb + P.off_lanes);
      a.srank = (const uint16_t *)(pb + P.off_srank);
      a.rstride = P.sstride;
      a.span = assembly_span(L, n_forms);
      a.stream = stream;
      fe_status st = launch_fused(a);
      if (st != FE_OK) return st;
    }
  }
  if (n_fused == n_forms) return FE_OK;
  // cell kernels into the workspace, then one row gather over these forms
  void *Aloc[4] = {nullptr, nullptr, nullptr, nullptr};
  void *V[4] = {nullptr, nullptr, nullptr, nullptr};
  const size_t stride = (size_t)n_cells * n_phi * n_phi * elt;
  int ng = 0;
  for (int f = 0; f < n_forms; ++f) {
    if (on_fused[f]) continue;
    Aloc[ng] = (unsigned char *)workspace + f * stride;
    V[ng] = mats[f].values;
    fe_mesh_view mv = *m;
    CellLaunch a;
    a.L = &L[f];
    a.form_buf = (const unsigned char *)form_bufs[f];
    a.status = (int32_t *)form_bufs[f];
    a.n_cells = n_cells;
    a.coords = mv.cell_coords;
    a.dofmap = mv.dofmap;
    a.n_dofs = n_dofs;
    a.coeff = forms[f].has_coeff ? mv.coeff : nullptr;
    if (forms[f].has_coeff && !mv.coeff) return FE_EINVAL;
    a.A_local = Aloc[ng];
    a.stream = stream;
    ++ng;
    if (phase == FE_NUMERIC_ASSEMBLE) continue;
    fe_status st;
    if (forms[f].has_coeff && cellwise_eligible(L[f])) {
      // coefficient forms in FP16: the whole-cell kernel after the
      // coefficient at the points
      CellwiseLaunch c;
      c.L = &L[f];
      c.form_buf = a.form_buf;
      c.status = a.status;
      c.n_cells = n_cells;
      c.coords = mv.cell_coords;
      c.dofmap = mv.dofmap;
      c.n_dofs = n_dofs;
      c.coeff = mv.coeff;
      c.zpt = (float *)((unsigned char *)workspace + zc_offset);
      c.zmax = (float *)((unsigned char *)workspace + zc_offset + zc_pts);
      c.rec = (unsigned char *)workspace + zc_offset + zc_pts + a256((size_t)n_cells * sizeof(float));
      c.A_local = (float *)Aloc[ng - 1];
      c.stream = stream;
      st = launch_cellwise_fp16(c);
    } else {
      st = launch_cell(a);
    }
    if (st != FE_OK) return st;
  }
  if (phase == FE_NUMERIC_LOCAL) return FE_OK;
  fe_status st = FE_EINVAL;
  if (elt == 8) {
    switch (ng) {
      case 1: st = launch_gather<double, 1>(adj_ptr, adj, rank, row_ptr, n_dofs, n_phi, mats[0].max_row_len, Aloc, V, s); break;
      case 2: st = launch_gather<double, 2>(adj_ptr, adj, rank, row_ptr, n_dofs, n_phi, mats[0].max_row_len, Aloc, V, s); break;
      case 3: st = launch_gather<double, 3>(adj_ptr, adj, rank, row_ptr, n_dofs, n_phi, mats[0].max_row_len, Aloc, V, s); break;
      case 4: st = launch_gather<double, 4>(adj_ptr, adj, rank, row_ptr, n_dofs, n_phi, mats[0].max_row_len, Aloc, V, s); break;
    }
  } else {
    switch (ng) {
      case 1: st = launch_gather<float, 1>(adj_ptr, adj, rank, row_ptr, n_dofs, n_phi, mats[0].max_row_len, Aloc, V, s); break;
      case 2: st = launch_gather<float, 2>(adj_ptr, adj, rank, row_ptr, n_dofs, n_phi, mats[0].max_row_len, Aloc, V, s); break;
      case 3: st = launch_gather<float, 3>(adj_ptr, adj, rank, row_ptr, n_dofs, n_phi, mats[0].max_row_len, Aloc, V, s); break;
      case 4: st = launch_gather<float, 4>(adj_ptr, adj, rank, row_ptr, n_dofs, n_phi, mats[0].max_row_len, Aloc, V, s); break;
    }
  }
  return st;
}

extern "C" fe_status fe_assemble_csr(const fe_form_desc *forms, const void *const *form_bufs,
                                     int32_t n_forms, const fe_mesh_view *m, int32_t phase,
                                     fe_csr *mats, void *plan, size_t *plan_bytes,
                                     void *workspace, size_t *ws_bytes, void *stream) {
  return assemble_csr(forms, form_bufs, n_forms, m, phase, mats, plan, plan_bytes, workspace,
                      ws_bytes, stream, false);
}

// ---------------------------------------- allocation-free numeric entry point
// The per-cell factor records (and per-point factors of hexahedral mass
// forms) of the fused path live in this file-scope array.  In host code its
// name is only a stand-in: the device address is asked from the runtime once
// per device and kept.
namespace {
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)16 << 20;
__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

fe_status scratch_address(void **out) {
  static std::mutex mu;
  static std::map<int, void *> addr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return FE_EHIP;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FE_EHIP;
    it = addr.emplace(dev, p).first;
  }
  *out = it->second;
  return FE_OK;
}
}  // namespace

extern "C" fe_status fe_assemble_csr_noalloc(const fe_form_desc *forms,
                                             const void *const *form_bufs, int32_t n_forms,
                                             const fe_mesh_view *m, fe_csr *mats, void *plan,
                                             void *stream) {
  void *ws = nullptr;
  fe_status st = scratch_address(&ws);
  if (st != FE_OK) return st;
  size_t cap = NOALLOC_SCRATCH_BYTES;
  return assemble_csr(forms, form_bufs, n_forms, m, FE_NUMERIC, mats, plan, nullptr, ws, &cap,
                      stream, true);
}

// ------------------------------------------------- vector assembly, actions
namespace fe {

VecPlanLayout vec_plan_layout(int64_t n_cells, int n_phi, int64_t n_dofs) {
  VecPlanLayout P;
  size_t off = 256;
  P.off_adj_ptr = off;
  off = a256(off + sizeof(int64_t) * (size_t)(n_dofs + 1));
  P.off_cursor = off;
  off = a256(off + sizeof(int64_t) * (size_t)n_dofs);
  P.off_adj = off;
  off = a256(off + sizeof(int64_t) * (size_t)std::max<int64_t>(1, n_cells * n_phi));
  P.scan_blocks = (size_t)(n_dofs + 1 + SCAN_TILE - 1) / SCAN_TILE;
  P.off_scan = off;
  off = a256(off + sizeof(int64_t) * (P.scan_blocks + 1));
  P.total = off;
  return P;
}

namespace {

// v^g = L b (Section 3.3): every dof sums the local-vector entries of its
// adjacency list, cell ascending, then i -- a fixed order, no atomics.  A
// plan built for another mesh is detected from its header (read before any
// offset derived from the mesh sizes is used) and reported through the
// status word; nothing is written then.
template <class T, int NF>
__global__ __launch_bounds__(256) void k_vgather(const VecPlanHeader *hdr, const int64_t *adj_ptr,
                                                 const int64_t *adj, int64_t n_cells,
                                                 int64_t n_dofs, int n_phi, int32_t *status,
                                                 const T *b0, const T *b1, T *out0, T *out1) {
  if (hdr->magic != VPLAN_MAGIC || hdr->n_cells != n_cells || hdr->n_dofs != n_dofs ||
      hdr->n_phi != n_phi) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(status, (int32_t)STATUS_BAD_DOF);
    return;
  }
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_dofs) return;
  T s0 = 0, s1 = 0;
  const int64_t a0 = adj_ptr[g], a1 = adj_ptr[g + 1];
  // four entries at a time: their loads are independent and in flight
  // together; the sums still run in list order
  for (int64_t a = a0; a < a1; a += 4) {
    int64_t idx[4];
    T v0[4], v1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t e = a + u < a1 ? adj[a + u] : -1;
      idx[u] = e < 0 ? -1 : (e >> ADJ_BITS) * n_phi + (e & ADJ_MASK);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      v0[u] = idx[u] < 0 ? (T)0 : b0[idx[u]];
      if (NF == 2) v1[u] = idx[u] < 0 ? (T)0 : b1[idx[u]];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (idx[u] < 0) break;
      s0 += v0[u];
      if (NF == 2) s1 += v1[u];
    }
  }
  out0[g] = s0;
  if (NF == 2) out1[g] = s1;
}

template <class T>
fe_status launch_vgather(const VecPlanHeader *hdr, const int64_t *adj_ptr, const int64_t *adj,
                         int64_t n_cells, int64_t n_dofs, int n_phi, int32_t *status,
                         const void *b0, const void *b1, void *out0, void *out1, hipStream_t s) {
  const unsigned blocks = (unsigned)((n_dofs + 255) / 256);
  if (b1)
    hipLaunchKernelGGL((k_vgather<T, 2>), dim3(blocks), dim3(256), 0, s, hdr, adj_ptr, adj,
                       n_cells, n_dofs, n_phi, status, (const T *)b0, (const T *)b1, (T *)out0,
                       (T *)out1);
  else
    hipLaunchKernelGGL((k_vgather<T, 1>), dim3(blocks), dim3(256), 0, s, hdr, adj_ptr, adj,
                       n_cells, n_dofs, n_phi, status, (const T *)b0, (const T *)nullptr,
                       (T *)out0, (T *)nullptr);
  return hipGetLastError() == hipSuccess ? FE_OK : FE_EHIP;
}

}  // namespace
}  // namespace fe

extern "C" fe_status fe_vector_plan(const fe_mesh_view *m, int32_t n_phi, void *plan,
                                    size_t *plan_bytes, void *stream) {
  if (!m || n_phi < 1 || n_phi > 256 || m->n_cells < 0 || m->n_dofs < 1) return FE_EINVAL;
  if (m->n_dofs >= INT32_MAX) return FE_EOVERFLOW;
  const int64_t n_cells = m->n_cells, n_dofs = m->n_dofs;
  const VecPlanLayout P = vec_plan_layout(n_cells, n_phi, n_dofs);
  if (!plan) {
    if (!plan_bytes) return FE_EINVAL;
    *plan_bytes = P.total;
    return FE_OK;
  }
  if (plan_bytes && *plan_bytes < P.total) return FE_ESIZE;
  if (n_cells > 0 && !m->dofmap) return FE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  unsigned char *pb = (unsigned char *)plan;
  VecPlanHeader *hdr_d = (VecPlanHeader *)pb;
  int64_t *adj_ptr = (int64_t *)(pb + P.off_adj_ptr);
  int64_t *cursor = (int64_t *)(pb + P.off_cursor);
  int64_t *adj = (int64_t *)(pb + P.off_adj);
  int64_t *scan = (int64_t *)(pb + P.off_scan);
  VecPlanHeader h;
  std::memset(&h, 0, sizeof(h));
  h.magic = VPLAN_MAGIC;
  h.n_cells = n_cells;
  h.n_dofs = n_dofs;
  h.n_phi = n_phi;
  if (hipMemcpyAsync(hdr_d, &h, sizeof(h), hipMemcpyHostToDevice, s) != hipSuccess) return FE_EHIP;
  hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n_dofs + 1, 256)), dim3(256), 0, s, adj_ptr,
                     n_dofs + 1, (int64_t)0);
  hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n_dofs, 256)), dim3(256), 0, s, cursor, n_dofs,
                     (int64_t)0);
  if (n_cells > 0) {
    hipLaunchKernelGGL(k_degree, dim3(grid_for(n_cells * n_phi, 256)), dim3(256), 0, s, m->dofmap,
                       n_cells * n_phi, n_dofs, adj_ptr, &hdr_d->status);
    fe_status st = scan_inclusive(adj_ptr + 1, n_dofs, scan, P.scan_blocks, s);
    if (st != FE_OK) return st;
    hipLaunchKernelGGL(k_fill_adj, dim3(grid_for(n_cells * n_phi, 256)), dim3(256), 0, s,
                       m->dofmap, n_cells, n_phi, n_dofs, adj_ptr, cursor, adj);
    hipLaunchKernelGGL(k_sort_adj, dim3((unsigned)((n_dofs + 255) / 256)), dim3(256), 0, s,
                       adj_ptr, adj, n_dofs, &hdr_d->max_deg);
  }
  if (!sync_ok(s)) return FE_EHIP;
  if (hipMemcpy(&h, hdr_d, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return FE_EHIP;
  if (h.status & STATUS_BAD_DOF) return FE_EINVAL;
  return FE_OK;
}

extern "C" fe_status fe_action_vjp(const fe_form_desc *f, const void *form_buf,
                                   const fe_mesh_view *m, const void *vplan, int32_t mode,
                                   const void *u, const void *v, void *y, void *grad_u,
                                   void *grad_coeff, void *workspace, size_t *ws_bytes,
                                   void *stream) {
  FormLayout L;
  fe_status st = compute_layout(f, &L);
  if (st != FE_OK) return st;
  if (L.act_nt == 0) return FE_EUNSUPPORTED;
  if (!m || m->n_cells < 0 || m->n_dofs < 1) return FE_EINVAL;
  if (mode != FE_ACTION && mode != FE_VJP) return FE_EINVAL;
  if (m->n_dofs >= INT32_MAX) return FE_EOVERFLOW;
  const int64_t n_cells = m->n_cells, n_dofs = m->n_dofs;
  const int n_phi = L.n_phi;
  const size_t elt = (L.prec == FE_FP64) ? 8 : 4;
  const bool gz = mode == FE_VJP && grad_coeff != nullptr;
  const size_t loc = a256(elt * (size_t)std::max<int64_t>(1, n_cells * n_phi));
  const size_t ws_need = loc * (gz ? 2 : 1);
  if (!workspace) {
    if (!ws_bytes) return FE_EINVAL;
    *ws_bytes = ws_need;
    return FE_OK;
  }
  if (ws_bytes && *ws_bytes < ws_need) return FE_ESIZE;
  if (!form_buf || !vplan) return FE_EINVAL;
  if (gz && !f->has_coeff) return FE_EINVAL;
  if (f->has_coeff && !m->coeff) return FE_EINVAL;
  if (mode == FE_ACTION && (!u || !y)) return FE_EINVAL;
  if (mode == FE_VJP && (!v || !grad_u || (gz && !u))) return FE_EINVAL;
  if (n_cells > 0 && (!m->dofmap || !m->cell_coords)) return FE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const VecPlanLayout P = vec_plan_layout(n_cells, n_phi, n_dofs);
  const unsigned char *pb = (const unsigned char *)vplan;
  const int64_t *adj_ptr = (const int64_t *)(pb + P.off_adj_ptr);
  const int64_t *adj = (const int64_t *)(pb + P.off_adj);
  unsigned char *wb = (unsigned char *)workspace;
  void *b0 = wb, *b1 = gz ? wb + loc : nullptr;
  void *out0 = mode == FE_ACTION ? y : grad_u;
  if (n_cells > 0) {
    ActionLaunch a;
    a.L = &L;
    a.form_buf = (const unsigned char *)form_buf;
    a.status = (int32_t *)form_buf;
    a.n_cells = n_cells;
    a.n_dofs = n_dofs;
    a.coords = m->cell_coords;
    a.dofmap = m->dofmap;
    a.coeff = f->has_coeff ? m->coeff : nullptr;
    // action on u; the adjoint acts on v (the forms are symmetric, so
    // A^T v = A v) and pairs it with u for the coefficient
    a.x0 = mode == FE_ACTION ? u : v;
    a.x1 = gz ? u : nullptr;
    a.geom = f->geom_precision;
    a.out0 = b0;
    a.out1 = b1;
    a.stream = stream;
    st = L.prec == FE_FP64 ? launch_action_fp64(a) : launch_action_fp32(a);
    if (st != FE_OK) return st;
  }
  const VecPlanHeader *hdr = (const VecPlanHeader *)vplan;
  int32_t *status = (int32_t *)form_buf;
  void *out1 = gz ? grad_coeff : nullptr;
  return L.prec == FE_FP64 ? launch_vgather<double>(hdr, adj_ptr, adj, n_cells, n_dofs, n_phi,
                                                    status, b0, b1, out0, out1, s)
                           : launch_vgather<float>(hdr, adj_ptr, adj, n_cells, n_dofs, n_phi,
                                                   status, b0, b1, out0, out1, s);
}
