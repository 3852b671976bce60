// Frontier phase of the analysis over a reverse graph grouped by source cell
// (K <= 64 inputs).
//
// The rows (c, u) of one cell under different inputs mostly meet the same
// targets: their images start from the same sample points.  The reverse graph
// therefore keeps one entry per (source cell c, target j) carrying the set of
// inputs u whose row (c, u) meets j as a 64-bit mask, instead of one entry per
// (row, target).  On a uniform Lorenz-type grid with 21 inputs this is a
// seventeenth of the entries.  The fixed point is the one the sweeps reach (the
// greatest fixed point of the monotone removal operator, Sec. 2.3); only the
// order of the removals differs.
//
//   controlled: row (c, u) is bad when OUT or when a target is removed; the
//     state is a bad-row mask per cell, and a cell dies when its mask is
//     full.  A step ORs the entry masks of the frontier's in-entries into
//     their cells' masks; the OR that completes a mask appends its cell.
//   nonleaving: row (c, u) lives while one of its targets does; the state is
//     a count of live reverse entries per row and of live rows per cell.  A
//     step decrements, per in-entry of a frontier cell and input bit, the
//     row's count, and for a count reaching zero the cell's, whose zero
//     appends the cell.
//
// Every removal is propagated exactly once.  A cell is appended once, when it
// dies, and flagged removed by the step that takes it from the frontier.
// Rows of cells already removed (by the sweeps) and edges to removed targets
// get no entry: the initial state accounts for those targets directly.
//
// Building the entries: a block takes whole cells and inserts their rows'
// (cell, target) keys into an LDS table, ORing each row's input bit into the
// key's mask.  One pass over the edges appends the block's entries to a
// staging area (k_cells_fill<STAGE>), counting them per target as it goes,
// and a scan and k_stage_scatter group them by target; when more entries come than the
// staging area holds, a first pass counts them per target (k_cells_count) and
// a second places them (k_cells_fill).
#include "gis_launch.h"

namespace gis {

namespace {

constexpr int kSlots = 2048;  // LDS hash slots of a block: (cell, target) keys
constexpr uint64_t kEmpty = ~0ull;
constexpr int kBatch = 8;     // targets loaded together

// Per block: distinct (local cell, target) keys of the block's rows and the
// OR of the input bits that met each.
struct CellTable {
  uint64_t key[kSlots];
  uint64_t mask[kSlots];
};

__device__ __forceinline__ uint64_t table_key(int32_t j, int cl) {
  return ((uint64_t)(uint32_t)j << 8) | (uint32_t)cl;
}

// Slot of key, inserting it if absent; -1 if the table is full.  The probe
// runs over the whole table, so an insertion fails only when the block has
// more than kSlots distinct keys, whatever the order of the insertions: the
// choice of the fallback below is the same in every pass over the block.
__device__ __forceinline__ int table_slot(CellTable& tb, uint64_t key) {
  uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 53) & (kSlots - 1);
  for (int p = 0; p < kSlots; ++p, h = (h + 1) & (kSlots - 1)) {
    uint64_t k = tb.key[h];
    if (k == key) return (int)h;
    if (k == kEmpty) {
      k = atomicCAS((unsigned long long*)&tb.key[h], (unsigned long long)kEmpty,
                    (unsigned long long)key);
      if (k == kEmpty || k == key) return (int)h;
    }
  }
  return -1;
}

__device__ __forceinline__ void table_clear(CellTable& tb) {
  for (int i = threadIdx.x; i < kSlots; i += blockDim.x) {
    tb.key[i] = kEmpty;
    tb.mask[i] = 0;
  }
}

// A block takes cpb = floor(256 / K) whole cells [g0, g0 + cpb), a thread
// per row.  Neighbouring lanes take different cells: the rows of one cell
// meet the same targets at the same time, and same-slot LDS atomics of one
// instruction serialise.
struct BlockRow {
  int cl, u;      // the thread's cell (local) and input
  int64_t c, r;   // its cell and row
  bool active;    // c < n_cells and c is present
};

__device__ __forceinline__ BlockRow block_row(const uint8_t* removed, int64_t n_cells, int32_t K,
                                              int32_t cpb, int64_t g0) {
  BlockRow b;
  const int t = threadIdx.x;
  b.cl = t % cpb;
  b.u = t / cpb;
  b.c = g0 + b.cl;
  b.r = b.c * K + b.u;
  b.active = t < cpb * K && b.c < n_cells && !removed[b.c];
  return b;
}

// Calls f(j, removed_j) for the targets of the thread's row in order, until
// f returns false.  Targets (and their removed flags, when any cell may be
// removed) are loaded kBatch at a time, so a row costs a memory latency per
// batch rather than per target.
template <typename F>
__device__ __forceinline__ void for_targets(const int64_t* row_ptr, const int32_t* col,
                                            const uint8_t* removed, bool any_removed,
                                            const BlockRow& b, F&& f) {
  if (!b.active) return;
  const int64_t a = row_ptr[b.r], e = row_ptr[b.r + 1];
  for (int64_t k = a; k < e; k += kBatch) {
    int32_t j[kBatch];
    bool rm[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) j[q] = k + q < e ? col[k + q] : -1;
#pragma unroll
    for (int q = 0; q < kBatch; ++q) rm[q] = any_removed && j[q] >= 0 && removed[j[q]] != 0;
#pragma unroll
    for (int q = 0; q < kBatch; ++q)
      if (j[q] >= 0 && !f(j[q], rm[q])) return;
  }
}

// Entry counts per target (deg, zero on entry): the distinct (cell, present
// target) pairs of each block, or (past kSlots of them) its present edges.
__global__ __launch_bounds__(256) void k_cells_count(const int64_t* row_ptr, const int32_t* col,
                                                     int64_t n_cells, int32_t K, int32_t cpb,
                                                     const uint8_t* removed, bool any_removed,
                                                     int32_t* deg) {
  __shared__ CellTable tb;
  __shared__ int s_over;
  const int t = threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * cpb;
  for (int64_t g0 = (int64_t)blockIdx.x * cpb; g0 < n_cells; g0 += stride) {
    table_clear(tb);
    if (t == 0) s_over = 0;
    __syncthreads();
    const BlockRow b = block_row(removed, n_cells, K, cpb, g0);
    for_targets(row_ptr, col, removed, any_removed, b, [&](int32_t j, bool rm) {
      if (rm || table_slot(tb, table_key(j, b.cl)) >= 0) return true;
      s_over = 1;
      return false;
    });
    __syncthreads();
    if (s_over == 0) {
      for (int i = t; i < kSlots; i += 256)
        if (tb.key[i] != kEmpty) atomicAdd(&deg[(int32_t)(tb.key[i] >> 8)], 1);
    } else {
      for_targets(row_ptr, col, removed, any_removed, b, [&](int32_t j, bool rm) {
        if (!rm) atomicAdd(&deg[j], 1);
        return true;
      });
    }
    __syncthreads();
  }
}

// Exclusive sum of v over the block (256 threads); *total gets the sum.
__device__ __forceinline__ int32_t block_exclusive_sum(int32_t v, int32_t* lds, int32_t& total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wid] = x;
  __syncthreads();
  int32_t before = 0;
  total = 0;
  for (int k = 0; k < 4; ++k) {
    before += k < wid ? lds[k] : 0;
    total += lds[k];
  }
  __syncthreads();
  return before + x - v;
}

// The analysis state with the first frontier (present cells already dead),
// and the entries: STAGE = false, at rptr[j] + (a slot counted down from
// deg[j]); STAGE = true, appended in any order to `stage` (one atomic per
// block; nothing is written past stage_cap, *n_staged still counts them).
template <int MODE, bool STAGE>
__global__ __launch_bounds__(256) void k_cells_fill(const int64_t* row_ptr, const int32_t* col,
                                                    const uint8_t* out, int64_t n_cells,
                                                    int32_t K, int32_t cpb,
                                                    const uint8_t* removed, bool any_removed,
                                                    const int64_t* rptr, int32_t* cursor,
                                                    int32_t* rsrc, uint64_t* rmask,
                                                    Staged* stage, int64_t stage_cap,
                                                    unsigned long long* n_staged,
                                                    uint32_t* rowstate, int32_t* good,
                                                    uint64_t* badmask, int32_t* front,
                                                    int32_t* count) {
  __shared__ CellTable tb;
  __shared__ int s_over;
  __shared__ uint8_t ok[256];
  __shared__ int32_t s_sum[4];
  __shared__ unsigned long long s_base;
  const int t = threadIdx.x;
  const uint64_t full = K == 64 ? ~0ull : ((1ull << K) - 1);
  const int64_t stride = (int64_t)gridDim.x * cpb;
  auto place = [&](int32_t j, int32_t c, uint64_t m) {
    const int32_t k = atomicSub(&cursor[j], 1);
    if (k <= 0) return;  // more entries than counted: never expected (no store out of range)
    rsrc[rptr[j] + k - 1] = c;
    rmask[rptr[j] + k - 1] = m;
  };
  for (int64_t g0 = (int64_t)blockIdx.x * cpb; g0 < n_cells; g0 += stride) {
    table_clear(tb);
    if (t == 0) s_over = 0;
    __syncthreads();
    const BlockRow b = block_row(removed, n_cells, K, cpb, g0);
    const uint64_t bit = 1ull << b.u;
    int32_t live = 0;  // distinct present targets: the entries carrying this row's bit
    bool hit_removed = false;
    for_targets(row_ptr, col, removed, any_removed, b, [&](int32_t j, bool rm) {
      if (rm) {
        hit_removed = true;
        return true;
      }
      const int sl = table_slot(tb, table_key(j, b.cl));
      if (sl < 0) {
        s_over = 1;
        return false;
      }
      if (MODE == GIS_ANALYSIS_NONLEAVING) {
        const uint64_t old = atomicOr((unsigned long long*)&tb.mask[sl], (unsigned long long)bit);
        if (!(old & bit)) ++live;
      } else {
        atomicOr((unsigned long long*)&tb.mask[sl], (unsigned long long)bit);
      }
      return true;
    });
    __syncthreads();
    const bool over = s_over != 0;
    if (over) {  // one entry per present edge
      live = 0;
      hit_removed = false;
      for_targets(row_ptr, col, removed, any_removed, b, [&](int32_t, bool rm) {
        if (rm) hit_removed = true;
        else ++live;
        return true;
      });
    }
    if (STAGE) {
      // this thread's entries: its table slots, or its row's present edges
      int32_t mine = 0;
      if (!over)
        for (int i = t; i < kSlots; i += 256) mine += tb.key[i] != kEmpty ? 1 : 0;
      else if (b.active)
        mine = live;
      int32_t total;
      const int32_t off = block_exclusive_sum(mine, s_sum, total);
      if (t == 0) s_base = atomicAdd(n_staged, (unsigned long long)total);
      __syncthreads();
      if ((int64_t)(s_base + total) <= stage_cap) {
        Staged* dst = stage + s_base + off;
        // (each written entry also counts toward its target's degree in
        // `cursor`, which the scan turns into the grouped offsets)
        if (!over) {
          for (int i = t; i < kSlots; i += 256) {
            const uint64_t key = tb.key[i];
            if (key != kEmpty) {
              *dst++ = Staged{(int32_t)(key >> 8), (int32_t)(g0 + (int64_t)(key & 255)),
                              tb.mask[i]};
              atomicAdd(&cursor[(int32_t)(key >> 8)], 1);
            }
          }
        } else {
          for_targets(row_ptr, col, removed, any_removed, b, [&](int32_t j, bool rm) {
            if (!rm) {
              *dst++ = Staged{j, (int32_t)b.c, bit};
              atomicAdd(&cursor[j], 1);
            }
            return true;
          });
        }
      }
    } else if (!over) {
      for (int i = t; i < kSlots; i += 256) {
        const uint64_t key = tb.key[i];
        if (key != kEmpty)
          place((int32_t)(key >> 8), (int32_t)(g0 + (int64_t)(key & 255)), tb.mask[i]);
      }
    } else {
      for_targets(row_ptr, col, removed, any_removed, b, [&](int32_t j, bool rm) {
        if (!rm) place(j, (int32_t)b.c, bit);
        return true;
      });
    }
    bool row_ok;
    if (MODE == GIS_ANALYSIS_NONLEAVING) {
      if (b.active) rowstate[b.r] = (uint32_t)live;
      row_ok = live > 0;
    } else {
      row_ok = b.active && !out[b.r] && !hit_removed;
    }
    if (t < cpb * K) ok[b.cl * K + b.u] = row_ok ? 1 : 0;
    __syncthreads();
    bool add = false;
    const int64_t cc = g0 + t;
    if (t < cpb && cc < n_cells && !removed[cc]) {
      if (MODE == GIS_ANALYSIS_NONLEAVING) {
        int32_t n = 0;
        for (int v = 0; v < K; ++v) n += ok[t * K + v];
        good[cc] = n;
        add = n == 0;
      } else {
        uint64_t bad = 0;
        for (int v = 0; v < K; ++v) bad |= (uint64_t)(ok[t * K + v] == 0) << v;
        badmask[cc] = bad;
        add = bad == full;
      }
    }
    append_block(add, (int32_t)cc, front, count);
    __syncthreads();
  }
}

// Staged entries (their counts per target taken by the staging pass): each
// entry at rptr[j] + (a slot counted down from deg[j]).
__global__ __launch_bounds__(256) void k_stage_scatter(const Staged* st, int64_t n,
                                                       const int64_t* rptr, int32_t* cursor,
                                                       int32_t* rsrc, uint64_t* rmask) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const Staged e = st[i];
    const int32_t k = atomicSub(&cursor[e.j], 1);
    if (k <= 0) continue;  // more entries than counted: never expected (no store out of range)
    rsrc[rptr[e.j] + k - 1] = e.c;
    rmask[rptr[e.j] + k - 1] = e.m;
  }
}

// Step s: a group of kGroup lanes per frontier cell walks its in-entries.
// The cells that die are collected in LDS.  While they are few (at most
// kLocal, a few passes of the block), the block follows them itself, for up
// to kDepth more generations, walking their in-entries the same way; the
// rest goes to the next step's frontier, spread over the whole grid, with
// one global atomic per block and pass (directly, one atomic each, past
// kList of them).  The thin tails of the removal chains then cost a launch
// per kDepth + 1 generations instead of one per generation.  Every dying
// cell is still visited exactly once, by this block or by a later step; only
// the order of the removals changes.
constexpr int kGroup = 16;
constexpr int kPer = 256 / kGroup;  // cells visited per pass of a block
constexpr int kList = 1024;
constexpr int kDepth = 16;
constexpr int kLocal = 4 * kPer;

template <int MODE>
__global__ __launch_bounds__(256) void k_cells_step(const int64_t* rptr, const int32_t* rsrc,
                                                    const uint64_t* rmask, int32_t K,
                                                    uint8_t* removed, uint64_t* badmask,
                                                    uint32_t* rowstate, int32_t* good,
                                                    const int32_t* front_in, int32_t* front_out,
                                                    int32_t* counts, int32_t s) {
  __shared__ int32_t s_list[2][kList];
  __shared__ int32_t s_n[2], s_base;
  if (blockIdx.x == 0 && threadIdx.x == 0) counts[(s + 2) % 3] = 0;
  int32_t* cnt_out = counts + (s + 1) % 3;
  const int32_t n = counts[s % 3];
  const uint64_t full = K == 64 ? ~0ull : ((1ull << K) - 1);
  const int t = threadIdx.x, sub = t % kGroup, slot = t / kGroup;
  auto push = [&](int32_t c, int o) {
    const int k = atomicAdd(&s_n[o], 1);
    if (k < kList) s_list[o][k] = c;
    else front_out[atomicAdd(cnt_out, 1)] = c;
  };
  // removes cell j and walks its in-entries; the cells that die go to list o
  auto visit = [&](int32_t j, int o) {
    if (sub == 0) removed[j] = 1;
    const int64_t b = rptr[j + 1];
    for (int64_t p = rptr[j] + sub; p < b; p += kGroup) {
      const int32_t c = rsrc[p];
      const uint64_t m = rmask[p];
      if (MODE == GIS_ANALYSIS_NONLEAVING) {
        for (uint64_t bits = m; bits; bits &= bits - 1) {
          const int u = __builtin_ctzll(bits);
          if (atomicSub(&rowstate[(int64_t)c * K + u], 1u) == 1u && atomicSub(&good[c], 1) == 1)
            push(c, o);
        }
      } else {
        const uint64_t old = atomicOr((unsigned long long*)&badmask[c], (unsigned long long)m);
        if (old != full && (old | m) == full) push(c, o);
      }
    }
  };
  for (int64_t i0 = (int64_t)blockIdx.x * kPer; i0 < n; i0 += (int64_t)gridDim.x * kPer) {
    if (t == 0) s_n[0] = 0;
    __syncthreads();
    const int64_t i = i0 + slot;
    if (i < n) visit(front_in[i], 0);
    __syncthreads();
    int cur = 0;
    for (int depth = 0; depth < kDepth; ++depth) {
      const int nl = s_n[cur];  // the same in every thread
      if (nl == 0 || nl > kLocal) break;
      if (t == 0) s_n[cur ^ 1] = 0;
      __syncthreads();
      for (int k0 = 0; k0 < nl; k0 += kPer)
        if (k0 + slot < nl) visit(s_list[cur][k0 + slot], cur ^ 1);
      __syncthreads();
      cur ^= 1;
    }
    const int32_t nl = s_n[cur] < kList ? s_n[cur] : kList;
    if (t == 0 && nl) s_base = atomicAdd(cnt_out, nl);
    __syncthreads();
    for (int k = t; k < nl; k += 256) front_out[s_base + k] = s_list[cur][k];
    __syncthreads();
  }
}

}  // namespace

namespace {

unsigned group_blocks(int64_t n_cells, int32_t cpb) {
  const int64_t groups = (n_cells + cpb - 1) / cpb;
  return (unsigned)(groups < 8192 ? (groups > 0 ? groups : 1) : 8192);
}

}  // namespace

int32_t cells_start(const int64_t* row_ptr, const int32_t* col, int64_t n_cells, int32_t K,
                    bool any_removed, const PruneWork& w, hipStream_t s) {
  if (K < 1 || K > 64) return GIS_E_INTERNAL;
  const int32_t cpb = 256 / K;
  hipLaunchKernelGGL(k_cells_count, dim3(group_blocks(n_cells, cpb)), dim3(256), 0, s, row_ptr,
                     col, n_cells, K, cpb, (const uint8_t*)w.removed, any_removed, w.rcur);
  GIS_LAUNCH_CHECK("k_cells_count");
  return scan_exclusive_i32(w.rcur, w.rptr, n_cells, w.rptr + n_cells, w.scan_tmp, s);
}

int32_t cells_scatter(const int64_t* row_ptr, const int32_t* col, const uint8_t* out,
                      int64_t n_cells, int32_t K, int32_t analysis, bool any_removed,
                      const PruneWork& w, hipStream_t s) {
  if (K < 1 || K > 64) return GIS_E_INTERNAL;
  int32_t rc;
  if ((rc = fill_i32(w.fcount, 0, 3, s))) return rc;
  const int32_t cpb = 256 / K;
  const unsigned nb = group_blocks(n_cells, cpb);
  if (analysis == GIS_ANALYSIS_NONLEAVING)
    hipLaunchKernelGGL((k_cells_fill<GIS_ANALYSIS_NONLEAVING, false>), dim3(nb), dim3(256), 0, s,
                       row_ptr, col, out, n_cells, K, cpb, (const uint8_t*)w.removed, any_removed,
                       (const int64_t*)w.rptr, w.rcur, w.rsrc, w.rmask, (Staged*)nullptr,
                       (int64_t)0, (unsigned long long*)nullptr, w.rowstate, w.good, w.badmask,
                       w.front, w.fcount);
  else
    hipLaunchKernelGGL((k_cells_fill<GIS_ANALYSIS_CONTROLLED, false>), dim3(nb), dim3(256), 0, s,
                       row_ptr, col, out, n_cells, K, cpb, (const uint8_t*)w.removed, any_removed,
                       (const int64_t*)w.rptr, w.rcur, w.rsrc, w.rmask, (Staged*)nullptr,
                       (int64_t)0, (unsigned long long*)nullptr, w.rowstate, w.good, w.badmask,
                       w.front, w.fcount);
  GIS_LAUNCH_CHECK("k_cells_fill");
  return GIS_OK;
}

int32_t cells_stage(const int64_t* row_ptr, const int32_t* col, const uint8_t* out,
                    int64_t n_cells, int32_t K, int32_t analysis, bool any_removed,
                    const PruneWork& w, Staged* stage, int64_t stage_cap,
                    unsigned long long* n_staged, hipStream_t s) {
  if (K < 1 || K > 64) return GIS_E_INTERNAL;
  int32_t rc;
  if ((rc = fill_i32(w.fcount, 0, 3, s))) return rc;
  if ((rc = fill_i64((int64_t*)n_staged, 0, 1, s))) return rc;
  const int32_t cpb = 256 / K;
  const unsigned nb = group_blocks(n_cells, cpb);
  if (analysis == GIS_ANALYSIS_NONLEAVING)
    hipLaunchKernelGGL((k_cells_fill<GIS_ANALYSIS_NONLEAVING, true>), dim3(nb), dim3(256), 0, s,
                       row_ptr, col, out, n_cells, K, cpb, (const uint8_t*)w.removed, any_removed,
                       (const int64_t*)nullptr, w.rcur, (int32_t*)nullptr,
                       (uint64_t*)nullptr, stage, stage_cap, n_staged, w.rowstate, w.good,
                       w.badmask, w.front, w.fcount);
  else
    hipLaunchKernelGGL((k_cells_fill<GIS_ANALYSIS_CONTROLLED, true>), dim3(nb), dim3(256), 0, s,
                       row_ptr, col, out, n_cells, K, cpb, (const uint8_t*)w.removed, any_removed,
                       (const int64_t*)nullptr, w.rcur, (int32_t*)nullptr,
                       (uint64_t*)nullptr, stage, stage_cap, n_staged, w.rowstate, w.good,
                       w.badmask, w.front, w.fcount);
  GIS_LAUNCH_CHECK("k_cells_fill");
  return GIS_OK;
}

int32_t cells_unstage(const Staged* stage, int64_t n_staged, int64_t n_cells, const PruneWork& w,
                      hipStream_t s) {
  const unsigned nb = (unsigned)((n_staged + 255) / 256 < 16384 ? (n_staged + 255) / 256 + 1 : 16384);
  // the degrees were counted in w.rcur by the staging pass
  int32_t rc;
  if ((rc = scan_exclusive_i32(w.rcur, w.rptr, n_cells, w.rptr + n_cells, w.scan_tmp, s)))
    return rc;
  hipLaunchKernelGGL(k_stage_scatter, dim3(nb), dim3(256), 0, s, stage, n_staged,
                     (const int64_t*)w.rptr, w.rcur, w.rsrc, w.rmask);
  GIS_LAUNCH_CHECK("k_stage_scatter");
  return GIS_OK;
}

int32_t cells_steps(int64_t n_cells, int32_t K, int32_t analysis, const PruneWork& w, int32_t t0,
                    int32_t count, hipStream_t s) {
  const unsigned nb = (unsigned)(w.front_blocks > 0 ? w.front_blocks : 2048);
  for (int32_t i = 0; i < count; ++i) {
    const int32_t t = t0 + i;
    const int32_t* cur = w.front + ((t & 1) ? n_cells : 0);
    int32_t* nxt = w.front + ((t & 1) ? 0 : n_cells);
    if (analysis == GIS_ANALYSIS_NONLEAVING)
      hipLaunchKernelGGL(k_cells_step<GIS_ANALYSIS_NONLEAVING>, dim3(nb), dim3(256), 0, s,
                         (const int64_t*)w.rptr, (const int32_t*)w.rsrc,
                         (const uint64_t*)w.rmask, K, w.removed, w.badmask, w.rowstate, w.good,
                         cur, nxt, w.fcount, t);
    else
      hipLaunchKernelGGL(k_cells_step<GIS_ANALYSIS_CONTROLLED>, dim3(nb), dim3(256), 0, s,
                         (const int64_t*)w.rptr, (const int32_t*)w.rsrc,
                         (const uint64_t*)w.rmask, K, w.removed, w.badmask, w.rowstate, w.good,
                         cur, nxt, w.fcount, t);
    GIS_LAUNCH_CHECK("k_cells_step");
  }
  return GIS_OK;
}

}  // namespace gis
