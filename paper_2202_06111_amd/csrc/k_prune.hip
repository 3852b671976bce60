// Graph analysis (Sec. 2.3) on the device.
//
// Both readings remove cells until a fixed point; the removed set is the least
// fixed point of a monotone operator, so any removal order reaches it:
//   controlled : row (c, u) is bad when it is OUT or one of its targets is
//                removed; a cell is removed when all its rows are bad;
//   nonleaving : row (c, u) is dead when all its targets are removed; a cell
//                is removed when all its rows are dead (a cell with no path
//                to a cycle of the input-union symbolic image, Definition 6).
// Two phases:
//   sweeps   : whole-graph passes, in place, until one removes nothing -- few
//              launches when the removal chains are short, and no reverse
//              graph to build; the nonleaving reading sweeps with a witness
//              target per cell (k_wsweep: one check per cell and sweep, each
//              cell's edges read at most once over the whole analysis), the
//              controlled one evaluates every row of the present cells;
//   frontier : for long chains, a breadth-first peel over the reverse CSR
//              (in-degree histogram -> offsets -> scatter), each step
//              propagating the cells removed in the step before through
//              per-row and per-cell counters (every removal once).
// The host runs a batch of sweeps and switches to the frontier phase when
// they have not converged.  The final pass writes kept flags and masks.
#include "gis_launch.h"

namespace gis {

namespace {

constexpr int kHash = 2048;        // LDS hash slots of the reverse-CSR kernels
constexpr int kProbe = 64;

inline unsigned grid_for(int64_t n, int64_t cap = 8192) {
  int64_t nb = (n + 255) / 256;
  if (nb < 1) nb = 1;
  if (nb > cap) nb = cap;
  return (unsigned)nb;
}

// Open-addressing hash of target ids in LDS; returns the slot of j or -1 if
// the probe sequence is full.  insert=false only looks j up.
__device__ __forceinline__ int lds_slot(int32_t* key, int32_t j, bool insert) {
  int h = (int)(((uint32_t)j * 2654435761u) >> 21) & (kHash - 1);
  for (int p = 0; p < kProbe; ++p, h = (h + 1) & (kHash - 1)) {
    int32_t k = key[h];
    if (k == j) return h;
    if (k == -1) {
      if (!insert) return -1;
      k = atomicCAS(&key[h], -1, j);
      if (k == -1 || k == j) return h;
    }
  }
  return -1;
}

// In-degree histogram.  A block takes 256 consecutive rows (thread = row);
// their targets overlap heavily (the inputs of one cell, neighbouring
// cells), so counts are first aggregated per distinct target in LDS and
// flushed with one global atomic per target.
__global__ __launch_bounds__(256) void k_indegree(const int64_t* row_ptr, const int32_t* col,
                                                  int64_t n_rows, int32_t* deg,
                                                  const int64_t* d_total, int64_t cap_edges) {
  if (d_total && *d_total > cap_edges) return;  // col was not written
  __shared__ int32_t key[kHash];
  __shared__ int32_t cnt[kHash];
  for (int i = threadIdx.x; i < kHash; i += 256) {
    key[i] = -1;
    cnt[i] = 0;
  }
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r < n_rows) {
    const int64_t e1 = row_ptr[r + 1];
    for (int64_t e = row_ptr[r]; e < e1; ++e) {
      const int32_t j = col[e];
      const int sl = lds_slot(key, j, true);
      if (sl >= 0) atomicAdd(&cnt[sl], 1);
      else atomicAdd(&deg[j], 1);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kHash; i += 256)
    if (key[i] >= 0) atomicAdd(&deg[key[i]], cnt[i]);
}

// Scatter of source rows into the reverse CSR, with the same blocks: each
// distinct target reserves one range for the block (one global atomic), and
// the block's edges fill it through LDS counters.
__global__ __launch_bounds__(256) void k_scatter(const int64_t* row_ptr, const int32_t* col,
                                                 int64_t n_rows, const int64_t* rptr,
                                                 int32_t* cursor, int32_t* rrow,
                                                 const int64_t* d_total, int64_t cap_edges) {
  if (d_total && *d_total > cap_edges) return;  // col was not written
  __shared__ int32_t key[kHash];
  __shared__ int32_t cnt[kHash];
  __shared__ int32_t base[kHash];
  for (int i = threadIdx.x; i < kHash; i += 256) {
    key[i] = -1;
    cnt[i] = 0;
  }
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = r < n_rows;
  const int64_t e0 = live ? row_ptr[r] : 0, e1 = live ? row_ptr[r + 1] : 0;
  for (int64_t e = e0; e < e1; ++e) {
    const int sl = lds_slot(key, col[e], true);
    if (sl >= 0) atomicAdd(&cnt[sl], 1);
  }
  __syncthreads();
  // cursors count down from the in-degree, so they end at zero (the state
  // the in-degree histogram of the next call starts from)
  for (int i = threadIdx.x; i < kHash; i += 256)
    if (key[i] >= 0) {
      base[i] = atomicSub(&cursor[key[i]], cnt[i]) - cnt[i];
      cnt[i] = 0;
    }
  __syncthreads();
  for (int64_t e = e0; e < e1; ++e) {
    const int32_t j = col[e];
    const int sl = lds_slot(key, j, false);
    const int32_t pos = sl >= 0 ? base[sl] + atomicAdd(&cnt[sl], 1) : atomicSub(&cursor[j], 1) - 1;
    rrow[rptr[j] + pos] = (int32_t)r;
  }
}

// Consistency of a caller-supplied CSR graph: row_ptr starts at 0, never
// decreases and ends at n_edges; every target is a cell id.
__global__ void k_check_graph(const int64_t* row_ptr, const int32_t* col, int64_t n_rows,
                              int64_t n_edges, int64_t n_cells, uint32_t* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t r = t; r < n_rows; r += stride) {
    const int64_t a = row_ptr[r], b = row_ptr[r + 1];
    if (a > b || a < 0 || b > n_edges) atomicOr(err, 1u);
  }
  if (t == 0 && (row_ptr[0] != 0 || row_ptr[n_rows] != n_edges)) atomicOr(err, 1u);
  for (int64_t e = t; e < n_edges; e += stride) {
    const int32_t j = col[e];
    if (j < 0 || (int64_t)j >= n_cells) atomicOr(err, 2u);
  }
}

// Removed flags as bytes (the sweeps update them in place), or packed 32 to
// a word for the read-only final pass: an eighth of the bytes, so that the
// flags of a large covering (4 MB for 32 M cells) stay in the L2 cache while
// every row looks up its targets'.
struct ByteFlags {
  const uint8_t* p;
  __device__ __forceinline__ bool operator[](int64_t j) const { return p[j] != 0; }
};
struct BitFlags {
  const uint32_t* w;
  __device__ __forceinline__ bool operator[](int64_t j) const {
    return ((w[j >> 5] >> (j & 31)) & 1u) != 0;
  }
};

// Packs removed bytes into words of 32 flags (bit i of word k: cell 32k + i).
__global__ __launch_bounds__(256) void k_pack_flags(const uint8_t* removed, int64_t n,
                                                    uint32_t* bits) {
  const int64_t words = (n + 31) / 32;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < words;
       k += (int64_t)gridDim.x * blockDim.x) {
    uint32_t v = 0;
    const int64_t c0 = 32 * k;
    if (c0 + 32 <= n && (((uintptr_t)(removed + c0)) & 15) == 0) {
      const uint4* q = (const uint4*)(removed + c0);
      const uint4 x = q[0], y = q[1];
      const uint32_t b[8] = {x.x, x.y, x.z, x.w, y.x, y.y, y.z, y.w};
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) v |= ((b[i] >> (8 * j)) & 0xffu ? 1u : 0u) << (4 * i + j);
    } else {
      for (int i = 0; i < 32 && c0 + i < n; ++i) v |= (removed[c0 + i] ? 1u : 0u) << i;
    }
    bits[k] = v;
  }
}

// Is row r good, given the removed flags of the cells?
//   controlled : not OUT and no target removed;
//   nonleaving : some target not removed.
// The targets are taken kBatch at a time: their ids are loaded together, then
// their flags together, so a row costs two memory latencies per batch rather
// than two per target.
constexpr int kBatch = 8;

template <int MODE, typename Flags>
__device__ __forceinline__ bool row_good(const int64_t* row_ptr, const int32_t* col,
                                         const uint8_t* out, Flags removed, int64_t r) {
  int64_t a = row_ptr[r];
  const int64_t b = row_ptr[r + 1];
  if (MODE == GIS_ANALYSIS_CONTROLLED && out[r]) return false;
  if (MODE != GIS_ANALYSIS_CONTROLLED) {
    // most rows of a kept cell meet a present cell first: one load decides them
    if (a < b && !removed[col[a]]) return true;
    ++a;
  }
  for (int64_t e = a; e < b; e += kBatch) {
    int32_t j[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) j[q] = e + q < b ? col[e + q] : -1;
    bool any_removed = false, any_present = false;
#pragma unroll
    for (int q = 0; q < kBatch; ++q)
      if (j[q] >= 0) {
        const bool rm = removed[j[q]];
        any_removed |= rm;
        any_present |= !rm;
      }
    if (MODE == GIS_ANALYSIS_CONTROLLED && any_removed) return false;
    if (MODE != GIS_ANALYSIS_CONTROLLED && any_present) return true;
  }
  return MODE == GIS_ANALYSIS_CONTROLLED;
}

// One sweep over every cell still present: a thread per row evaluates it,
// then a thread per cell removes the cell if none of its rows is good.  A
// block takes cpb = floor(256 / K) whole cells at a time.  Updates are made
// in place, so a sweep may already see removals of the same sweep; the
// result does not depend on that, because removal is monotone: a sweep that
// removes nothing has evaluated every cell against a constant set, which is
// then the fixed point.  `last` holds 1 + the index of the last sweep that
// removed a cell; sweep s starts only if sweep s-1 removed one.
template <int MODE>
__global__ __launch_bounds__(256) void k_sweep(const int64_t* row_ptr, const int32_t* col,
                                               const uint8_t* out, int64_t n_cells, int32_t K,
                                               int32_t cpb, uint8_t* removed, int32_t* last,
                                               int32_t s, const int64_t* d_total,
                                               int64_t cap_edges) {
  if (d_total && *d_total > cap_edges) return;  // col was not written
  if (s > 0 && *last < s) return;               // converged already
  __shared__ uint8_t ok[256];
  bool changed = false;
  const int t = threadIdx.x;
  // odd sweeps take the groups in reverse order (blocks start roughly in
  // index order), so removals propagate in place along both directions
  const int64_t groups = (n_cells + cpb - 1) / cpb;
  for (int64_t gi = blockIdx.x; gi < groups; gi += gridDim.x) {
    const int64_t g0 = ((s & 1) ? groups - 1 - gi : gi) * cpb;
    const int64_t c = g0 + t / K;
    bool good = false;
    if (t < cpb * K && c < n_cells && !removed[c])
      good = row_good<MODE>(row_ptr, col, out, ByteFlags{removed}, c * K + t % K);
    ok[t] = good ? 1 : 0;
    __syncthreads();
    if (t < cpb) {
      const int64_t cc = g0 + t;
      if (cc < n_cells && !removed[cc]) {
        bool any = false;
        for (int u = 0; u < K; ++u) any |= ok[t * K + u] != 0;
        if (!any) {
          removed[cc] = 1;
          changed = true;
        }
      }
    }
    __syncthreads();
  }
  if (__ballot(changed) && (t & 63) == 0) atomicMax(last, s + 1);
}

// ---- nonleaving: sweeps with a witness per cell.  A present cell stays
// present while some edge of its rows (all inputs together: the edges of
// rows c*K .. c*K+K-1 are one contiguous span of col) ends in a present
// cell.  Each present cell keeps the position and the id of such a target,
// its witness.  A sweep re-checks the witness only; when it has been
// removed, the cell looks for the next present target after it -- the
// targets before it were removed when they were passed, and removal is
// final -- and is removed when there is none.  Over a whole analysis each
// cell's span is read at most once, plus one witness check per sweep, and no
// reverse graph is built.  Sweep 0 (INIT) finds the first witnesses.
//
// A block takes 256 consecutive cells (odd sweeps go through the tiles in
// reverse order, so that removals propagate in place along both
// directions): a thread per cell checks the witness, the cells that need a
// new one are queued in LDS, and each wave then searches one queued cell's
// span 64 edges at a time (coalesced loads, one ballot per 64 edges).
//
// A witness at the start of the cell's span is recorded as position -1, and
// the span's bounds (row_ptr[c*K], row_ptr[(c+1)*K]) are read again only by
// a cell whose witness died: no per-cell copy of the span starts is kept.
template <bool INIT>
__global__ __launch_bounds__(256) void k_wsweep(const int64_t* row_ptr, const int32_t* col,
                                                int64_t n_cells, int32_t K,
                                                uint8_t* removed, int64_t* wpos, int32_t* wtgt,
                                                int32_t* last, int32_t s, const int64_t* d_total,
                                                int64_t cap_edges) {
  if (d_total && *d_total > cap_edges) return;  // col was not written
  if (!INIT && *last < s) return;                // sweep s-1 removed nothing: converged
  __shared__ int32_t q_cell[256];
  __shared__ int64_t q_from[256], q_end[256];
  __shared__ int32_t q_n;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  bool changed = false;
  const int64_t tiles = (n_cells + 255) / 256;
  for (int64_t ti = blockIdx.x; ti < tiles; ti += gridDim.x) {
    const int64_t tile = (s & 1) ? tiles - 1 - ti : ti;
    const int64_t c = tile * 256 + t;
    if (t == 0) q_n = 0;
    __syncthreads();
    if (c < n_cells && !removed[c]) {
      int64_t from = 0, end = 0;
      bool need;
      if (INIT) {
        const int64_t a = row_ptr[c * K];
        end = row_ptr[(c + 1) * K];
        from = a;
        need = true;
        if (a < end) {  // most cells: the first target is present
          const int32_t j = col[a];
          if (!removed[j]) {
            wpos[c] = -1;
            wtgt[c] = j;
            need = false;
          } else {
            from = a + 1;
          }
        }
      } else {
        need = removed[wtgt[c]] != 0;
        if (need) {
          const int64_t wp = wpos[c];
          from = (wp >= 0 ? wp : row_ptr[c * K]) + 1;
          end = row_ptr[(c + 1) * K];
        }
      }
      if (need) {
        const int k = atomicAdd(&q_n, 1);
        q_cell[k] = (int32_t)c;
        q_from[k] = from;
        q_end[k] = end;
      }
    }
    __syncthreads();
    const int nq = q_n;
    for (int k = wave; k < nq; k += 4) {
      const int32_t cq = q_cell[k];
      const int64_t from = q_from[k], end = q_end[k];
      int64_t pos = -1;
      int32_t jw = -1;
      for (int64_t p0 = from; p0 < end; p0 += 64) {
        const int64_t p = p0 + lane;
        int32_t j = -1;
        bool live = false;
        if (p < end) {
          j = col[p];
          live = removed[j] == 0;
        }
        const uint64_t m = __ballot(live);
        if (m) {  // wave-uniform
          const int f = __builtin_ctzll(m);
          pos = p0 + f;
          jw = __shfl(j, f, 64);
          break;
        }
      }
      if (lane == 0) {
        if (pos >= 0) {
          wpos[cq] = pos;
          wtgt[cq] = jw;
        } else {
          removed[cq] = 1;
          changed = true;
        }
      }
    }
    __syncthreads();
  }
  if (__ballot(changed) && lane == 0) atomicMax(last, s + 1);
}

// ---- frontier phase (long removal chains): a breadth-first peel over the
// reverse CSR.  It runs only after a synchronisation has shown the graph
// complete.  Step s takes the cells removed in step s-1 (list s & 1, length
// counts[s % 3]) and appends the cells it removes to the other list (length
// counts[(s+1) % 3]); the third count is cleared for the step after.
//
// controlled: a row turns bad when any target is removed, so a step marks
//   every in-row of the frontier bad with plain byte stores (idempotent, no
//   atomics) and flags its cell as a candidate; a second launch removes the
//   candidates whose rows are now all bad.  Row flags live at c * Kp + u
//   (Kp = K rounded up to 8) so that a cell's flags are whole 8-byte words.
// nonleaving: a row dies when its last present target is removed, which
//   needs a count per row; per-row and per-cell counters propagate each
//   removal exactly once, in one launch per step:
//   rowstate[r] = targets of r not yet removed, good[c] = rows of c alive.


// controlled, initial state: a row is bad when OUT; a cell with every row
// bad is removed; the first frontier is every removed cell (also those the
// sweeps removed, whose in-rows have not been marked).
__global__ __launch_bounds__(1024) void k_front_init_ctl(const uint8_t* out, int64_t n_cells, int32_t K, int32_t Kp,
                                 uint8_t* removed, uint8_t* rowbad, int32_t* front,
                                 int32_t* count) {
  for (int64_t c0 = (int64_t)blockIdx.x * blockDim.x; c0 < n_cells;
       c0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = c0 + threadIdx.x;
    bool rem = false;
    if (c < n_cells) {
      bool all = true;
      for (int32_t u = 0; u < K; ++u) {
        const bool bad = out[c * K + u] != 0;
        rowbad[c * Kp + u] = bad ? 1 : 0;
        all &= bad;
      }
      if (all) removed[c] = 1;
      rem = removed[c] != 0;
    }
    append_block(rem, (int32_t)c, front, count);
  }
}

// controlled, step s, first launch: a wave per frontier cell marks its
// in-rows bad and their cells as candidates.
__global__ __launch_bounds__(256) void k_front_mark_ctl(const int64_t* rptr, const int32_t* rrow,
                                                        int32_t K, int32_t Kp, uint8_t* rowbad,
                                                        uint8_t* cand, const int32_t* front_in,
                                                        int32_t* counts, int32_t s) {
  if (blockIdx.x == 0 && threadIdx.x == 0) counts[(s + 1) % 3] = 0;
  const int32_t n = counts[s % 3];
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < n;
       i += waves) {
    const int32_t c = front_in[i];
    const int64_t b = rptr[c], e = rptr[c + 1];
    for (int64_t p = b + lane; p < e; p += 64) {
      const int32_t r = rrow[p];
      const int32_t cell = r / K;
      uint8_t* f = rowbad + (int64_t)cell * Kp + (r - cell * K);
      if (*f) continue;
      *f = 1;
      cand[cell] = 1;
    }
  }
}

// controlled, step s, second launch: a candidate whose rows are all bad is
// removed and joins the next frontier (one counter atomic per wave).
__global__ __launch_bounds__(1024) void k_front_eval_ctl(int64_t n_cells, int32_t K, int32_t Kp, uint8_t* removed,
                                 const uint8_t* rowbad, uint8_t* cand, int32_t* front_out,
                                 int32_t* counts, int32_t s) {
  if (counts[s % 3] == 0) return;  // nothing was marked
  int32_t* cnt_out = counts + (s + 1) % 3;
  for (int64_t c0 = (int64_t)blockIdx.x * blockDim.x; c0 < n_cells;
       c0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = c0 + threadIdx.x;
    bool rem = false;
    if (c < n_cells && cand[c]) {
      cand[c] = 0;
      if (!removed[c]) {
        const uint64_t* wv = (const uint64_t*)(rowbad + c * Kp);
        bool all = true;
        for (int32_t u0 = 0; u0 < K; u0 += 8) {
          const int nb = K - u0 < 8 ? K - u0 : 8;
          const uint64_t m = nb == 8 ? 0x0101010101010101ull : ((1ull << (8 * nb)) - 1) & 0x0101010101010101ull;
          all &= (wv[u0 >> 3] & m) == m;
        }
        if (all) {
          removed[c] = 1;
          rem = true;
        }
      }
    }
    append_block(rem, (int32_t)c, front_out, cnt_out);
  }
}

// nonleaving, initial state: counters from the current removed flags (read
// only here), and the first frontier: the present cells without a live row.
// A block takes cpb whole cells, a thread per row, as in a sweep.
__device__ __forceinline__ int32_t live_targets(const int64_t* row_ptr, const int32_t* col,
                                                const uint8_t* removed, int64_t r) {
  const int64_t a = row_ptr[r], b = row_ptr[r + 1];
  int32_t alive = 0;
  for (int64_t e = a; e < b; e += kBatch) {
    int32_t j[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) j[q] = e + q < b ? col[e + q] : -1;
#pragma unroll
    for (int q = 0; q < kBatch; ++q) alive += (j[q] >= 0 && !removed[j[q]]) ? 1 : 0;
  }
  return alive;
}

__global__ __launch_bounds__(256) void k_front_init_nl(const int64_t* row_ptr, const int32_t* col,
                                                       int64_t n_cells, int32_t K, int32_t cpb,
                                                       const uint8_t* removed, uint32_t* rowstate,
                                                       int32_t* good, int32_t* front,
                                                       int32_t* count) {
  __shared__ uint8_t ok[256];
  const int t = threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * cpb;
  for (int64_t g0 = (int64_t)blockIdx.x * cpb; g0 < n_cells; g0 += stride) {
    const int64_t c = g0 + t / K;
    bool g = false;
    if (t < cpb * K && c < n_cells) {
      const int64_t r = c * K + t % K;
      const int32_t alive = removed[c] ? 0 : live_targets(row_ptr, col, removed, r);
      rowstate[r] = (uint32_t)alive;
      g = alive > 0;
    }
    ok[t] = g ? 1 : 0;
    __syncthreads();
    bool add = false;
    const int64_t cc = g0 + t;
    if (t < cpb && cc < n_cells) {
      int32_t n = 0;
      for (int u = 0; u < K; ++u) n += ok[t * K + u];
      good[cc] = n;
      add = n == 0 && !removed[cc];
    }
    append_block(add, (int32_t)cc, front, count);
    __syncthreads();
  }
}

// The same for K > 256: a thread per cell.
__global__ __launch_bounds__(256) void k_front_init_nl_wide(const int64_t* row_ptr, const int32_t* col, int64_t n_cells,
                                     int32_t K, const uint8_t* removed, uint32_t* rowstate,
                                     int32_t* good, int32_t* front, int32_t* count) {
  for (int64_t c0 = (int64_t)blockIdx.x * blockDim.x; c0 < n_cells;
       c0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = c0 + threadIdx.x;
    bool add = false;
    if (c < n_cells) {
      const bool present = !removed[c];
      int32_t n = 0;
      for (int32_t u = 0; u < K; ++u) {
        const int64_t r = c * K + u;
        const int32_t alive = present ? live_targets(row_ptr, col, removed, r) : 0;
        rowstate[r] = (uint32_t)alive;
        n += alive > 0 ? 1 : 0;
      }
      good[c] = n;
      add = n == 0 && present;
    }
    append_block(add, (int32_t)c, front, count);
  }
}

// nonleaving, step s: a block per frontier cell removes it and walks its
// in-rows; a row whose count reaches zero decrements its cell's count, and
// the cell whose count reaches zero joins the next frontier.
__global__ __launch_bounds__(256) void k_front_step_nl(const int64_t* rptr, const int32_t* rrow,
                                                       int32_t K, uint8_t* removed,
                                                       uint32_t* rowstate, int32_t* good,
                                                       const int32_t* front_in,
                                                       int32_t* front_out, int32_t* counts,
                                                       int32_t s) {
  if (blockIdx.x == 0 && threadIdx.x == 0) counts[(s + 2) % 3] = 0;
  int32_t* cnt_out = counts + (s + 1) % 3;
  const int32_t n = counts[s % 3];
  for (int32_t i = blockIdx.x; i < n; i += gridDim.x) {
    const int32_t c = front_in[i];
    if (threadIdx.x == 0) removed[c] = 1;
    const int64_t b = rptr[c], e = rptr[c + 1];
    for (int64_t p0 = b; p0 < e; p0 += blockDim.x) {
      const int64_t p = p0 + threadIdx.x;
      bool add = false;
      int32_t cell = 0;
      if (p < e) {
        const int32_t r = rrow[p];
        if (atomicSub(&rowstate[r], 1u) == 1u) {
          cell = r / K;
          add = atomicSub(&good[cell], 1) == 1;
        }
      }
      append_block(add, cell, front_out, cnt_out);
    }
  }
}

// kept flags, admissible-input masks and the kept count from the removed
// flags (rows evaluated against the final set).  Like a sweep, a block takes
// cpb = floor(256 / K) whole cells: a thread per row evaluates it, then a
// thread per (cell, mask word) assembles the word.
template <int MODE, typename Flags>
__global__ __launch_bounds__(256) void k_prune_final(const int64_t* row_ptr, const int32_t* col,
                                                     const uint8_t* out, int64_t n_cells,
                                                     int32_t K, int32_t cpb,
                                                     Flags removed, uint8_t* kept,
                                                     uint64_t* mask, int32_t W,
                                                     unsigned long long* nkept,
                                                     const int64_t* d_total, int64_t cap_edges,
                                                     const int32_t* last, int32_t sweeps,
                                                     const Job* jobs, int32_t n_jobs,
                                                     JobStats* stats, const uint8_t* level,
                                                     const int32_t* idx, const void* rowinfo,
                                                     int32_t frontier) {
  if (d_total && *d_total > cap_edges) return;  // col was not written
  if (sweeps > 0 && *last >= sweeps) return;     // the sweeps have not converged
  // after the frontier phase its state already tells which rows are good
  // (live-target counts per row; controlled: bad-row flags at c * Kp + u, or
  // a bad-row mask per cell); otherwise every row is evaluated against the
  // removed flags
  const int32_t Kp = (K + 7) & ~7;
  __shared__ uint64_t okw[5];  // the waves' good-row ballots (+ a zero word)
  __shared__ unsigned int grp_kept;
  __shared__ CoverIndex sci;   // covering index of job s_job, for the hole marking
  __shared__ int32_t s_job;
  const int t = threadIdx.x;
  if (t == 0) s_job = -1;
  unsigned long long mine = 0;
  // thread 0: kept cells of job kjob counted by this block so far (flushed to
  // the job's statistics when the job changes and at the end)
  unsigned long long kcnt = 0;
  int32_t kjob = -1;
  const int64_t stride = (int64_t)gridDim.x * cpb;
  for (int64_t g0 = (int64_t)blockIdx.x * cpb; g0 < n_cells; g0 += stride) {
    const int64_t c = g0 + t / K;
    bool good = false;
    if (t < cpb * K && c < n_cells && !removed[c]) {
      if (!rowinfo)
        good = row_good<MODE>(row_ptr, col, out, removed, c * K + t % K);
      else if (MODE == GIS_ANALYSIS_NONLEAVING)
        good = ((const uint32_t*)rowinfo)[c * K + t % K] > 0;
      else if (frontier == kCellFrontier)
        good = ((((const uint64_t*)rowinfo)[c] >> (t % K)) & 1) == 0;
      else
        good = ((const uint8_t*)rowinfo)[c * Kp + t % K] == 0;
    }
    const uint64_t bal = __ballot(good);
    if ((t & 63) == 0) okw[t >> 6] = bal;
    if (t == 0) {
      grp_kept = 0;
      okw[4] = 0;
    }
    // the group's job: one atomic for its kept count, and its covering index
    // staged in LDS for the hole marking, when the group lies in one job
    const int64_t glast = g0 + cpb - 1 < n_cells ? g0 + cpb - 1 : n_cells - 1;
    const bool need_job = stats || level;
    const int32_t jfirst = need_job ? job_of_cell(jobs, n_jobs, g0) : 0;
    const bool one_job = need_job && job_of_cell(jobs, n_jobs, glast) == jfirst;
    if (level && one_job && jfirst != s_job) stage_index(&sci, &jobs[jfirst].ci);
    __syncthreads();
    if (t == 0 && level && one_job) s_job = jfirst;
    if (t < cpb * W) {
      const int64_t cc = g0 + t / W;
      const int w = t % W;
      if (cc < n_cells) {
        const bool k = !removed[cc];
        // bits [p, p + nb) of the block's ballots: the cell's rows of word w
        const int p = (t / W) * K + w * 64;
        const int nb = K - w * 64 < 64 ? K - w * 64 : 64;
        const int q = p >> 6, sh = p & 63;
        uint64_t m = okw[q] >> sh;
        if (sh) m |= okw[q + 1] << (64 - sh);
        if (nb < 64) m &= (1ull << nb) - 1;
        mask[cc * W + w] = m;
        if (w == 0) {
          kept[cc] = k ? 1 : 0;
          mine += k;
          if (k && stats) {
            if (one_job) atomicAdd(&grp_kept, 1u);
            else atomicAdd(&stats[job_of_cell(jobs, n_jobs, cc)].n_kept, 1ull);
          }
          // a removed cell becomes a hole of its job's covering index, which
          // the boundary selection that follows reads
          if (!k && level) {
            const CoverIndex& ci = one_job ? sci : jobs[job_of_cell(jobs, n_jobs, cc)].ci;
            if (!ci.uniform) {
              const int64_t sl = cell_slot(ci, level, idx, cc);
              if (sl >= 0) ci.state[sl] = ST_HOLE;
            }
          }
        }
      }
    }
    __syncthreads();
    if (t == 0 && stats && one_job && grp_kept) {
      if (jfirst != kjob) {
        if (kcnt) atomicAdd(&stats[kjob].n_kept, kcnt);
        kjob = jfirst;
        kcnt = 0;
      }
      kcnt += grp_kept;
    }
  }
  if (t == 0 && kcnt) atomicAdd(&stats[kjob].n_kept, kcnt);
  for (int o = 32; o > 0; o >>= 1) mine += __shfl_down(mine, o, 64);
  if ((t & 63) == 0 && mine) atomicAdd(nkept, mine);
}


// The final pass in two launches (after sweeps, K <= 256): a thread per row
// evaluates it against the packed removed flags and a ballot per wave stores
// 64 rows' good flags (rowbits bit r = row r); then a thread per cell takes
// its kept flag, cuts its mask words out of the row bits, counts it and
// turns a removed cell into a hole of the covering index.  Rows are not
// grouped by cell, so no block synchronisation or staging is needed, and
// each wave keeps kRowsIlp rows' loads in flight: the first target of most
// rows decides them (non-leaving analysis), so their offsets, first targets
// and flags are fetched for all of them before any is decided.  With the
// build's first-target array (`first`, non-leaving analysis) a row's first
// target is one coalesced 4-byte load: the offsets and `col` are read only
// for the rows whose first target was removed (reading `col[row_ptr[r]]`
// instead touches every line of `col`, a row being a few dozen bytes of it).
constexpr int kRowsIlp = 4;

template <int MODE, typename Flags>
__global__ __launch_bounds__(256) void k_row_good(const int64_t* row_ptr, const int32_t* col,
                                                  const uint8_t* out, const int32_t* first,
                                                  int64_t n_rows, int32_t K, Flags removed,
                                                  uint64_t* rowbits, const int64_t* d_total,
                                                  int64_t cap_edges, const int32_t* last,
                                                  int32_t sweeps) {
  if (d_total && *d_total > cap_edges) return;  // col was not written
  if (sweeps > 0 && *last >= sweeps) return;     // the sweeps have not converged
  const int lane = threadIdx.x & 63;
  const int64_t words = (n_rows + 63) / 64;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t w0 = wave * kRowsIlp; w0 < words; w0 += waves * kRowsIlp) {
    int64_t r[kRowsIlp];
    bool good[kRowsIlp], done[kRowsIlp];
    if (MODE != GIS_ANALYSIS_CONTROLLED && first) {
      int32_t j[kRowsIlp];
#pragma unroll
      for (int q = 0; q < kRowsIlp; ++q) {
        r[q] = (w0 + q) * 64 + lane;
        // rows of removed cells need no test (their cells' masks are 0)
        const bool in = r[q] < n_rows && !removed[r[q] / K];
        j[q] = in ? first[r[q]] : -1;
        good[q] = false;
        done[q] = !in || j[q] < 0;  // a row with no target is not good
      }
#pragma unroll
      for (int q = 0; q < kRowsIlp; ++q)
        if (!done[q] && !removed[j[q]]) {
          good[q] = true;
          done[q] = true;
        }
#pragma unroll
      for (int q = 0; q < kRowsIlp; ++q)
        if (!done[q]) good[q] = row_good<MODE>(row_ptr, col, out, removed, r[q]);
#pragma unroll
      for (int q = 0; q < kRowsIlp; ++q) {
        const uint64_t m = __ballot(good[q]);
        if (lane == 0 && w0 + q < words) rowbits[w0 + q] = m;
      }
      continue;
    }
    int64_t a[kRowsIlp], b[kRowsIlp];
#pragma unroll
    for (int q = 0; q < kRowsIlp; ++q) {
      r[q] = (w0 + q) * 64 + lane;
      const bool in = r[q] < n_rows && !removed[r[q] / K];
      a[q] = in ? row_ptr[r[q]] : 0;
      b[q] = in ? row_ptr[r[q] + 1] : 0;
      good[q] = false;
      done[q] = !in;
    }
    if (MODE != GIS_ANALYSIS_CONTROLLED) {
      int32_t j[kRowsIlp];
#pragma unroll
      for (int q = 0; q < kRowsIlp; ++q) j[q] = !done[q] && a[q] < b[q] ? col[a[q]] : -1;
#pragma unroll
      for (int q = 0; q < kRowsIlp; ++q)
        if (j[q] >= 0 && !removed[j[q]]) {
          good[q] = true;
          done[q] = true;
        }
    }
#pragma unroll
    for (int q = 0; q < kRowsIlp; ++q)
      if (!done[q]) good[q] = row_good<MODE>(row_ptr, col, out, removed, r[q]);
#pragma unroll
    for (int q = 0; q < kRowsIlp; ++q) {
      const uint64_t m = __ballot(good[q]);
      if (lane == 0 && w0 + q < words) rowbits[w0 + q] = m;
    }
  }
}

template <typename Flags>
__global__ __launch_bounds__(256) void k_cell_masks(int64_t n_cells, int32_t K, Flags removed,
                                                    const uint64_t* rowbits, uint8_t* kept,
                                                    uint64_t* mask, int32_t W,
                                                    unsigned long long* nkept,
                                                    const int64_t* d_total, int64_t cap_edges,
                                                    const int32_t* last, int32_t sweeps,
                                                    const Job* jobs, int32_t n_jobs,
                                                    JobStats* stats, const uint8_t* level,
                                                    const int32_t* idx) {
  if (d_total && *d_total > cap_edges) return;
  if (sweeps > 0 && *last >= sweeps) return;
  const int lane = threadIdx.x & 63;
  // kept counts are accumulated over the grid-stride loop and added once per
  // wave at the end (an atomic per wave and iteration on the same two
  // counters serialised in L2: a millisecond per 10^7 cells); the wave's
  // cells come in increasing order, so its jobs do too
  unsigned long long mine = 0, jcnt = 0;
  int32_t wjob = -1;
  for (int64_t c0 = (int64_t)blockIdx.x * blockDim.x; c0 < n_cells;
       c0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = c0 + threadIdx.x;
    const bool live = c < n_cells;
    const bool k = live && !removed[c];
    mine += k ? 1 : 0;
    if (live) {
      kept[c] = k ? 1 : 0;
      for (int w = 0; w < W; ++w) {
        uint64_t m = 0;
        if (k) {
          const int64_t s0 = c * K + 64 * w;
          const int len = K - 64 * w < 64 ? K - 64 * w : 64;
          const int64_t i = s0 >> 6;
          const int sh = (int)(s0 & 63);
          m = rowbits[i] >> sh;
          if (sh && sh + len > 64) m |= rowbits[i + 1] << (64 - sh);
          if (len < 64) m &= (1ull << len) - 1;
        }
        mask[c * W + w] = m;
      }
      // a removed cell becomes a hole of its job's covering index, which the
      // boundary selection that follows reads
      if (!k && level) {
        const CoverIndex& ci = jobs[job_of_cell(jobs, n_jobs, c)].ci;
        if (!ci.uniform) {
          const int64_t sl = cell_slot(ci, level, idx, c);
          if (sl >= 0) ci.state[sl] = ST_HOLE;
        }
      }
    }
    // per-job kept counts: the wave's count joins its running count when
    // its cells lie in one job, which is flushed when the job changes
    const uint64_t bal = __ballot(k);
    if (stats && lane == 0 && bal) {
      const int64_t wc = c0 + (threadIdx.x & ~63);
      const int64_t wl = wc + 63 < n_cells ? wc + 63 : n_cells - 1;
      const int32_t j0 = job_of_cell(jobs, n_jobs, wc);
      if (job_of_cell(jobs, n_jobs, wl) == j0) {
        if (j0 != wjob) {
          if (jcnt) atomicAdd(&stats[wjob].n_kept, jcnt);
          wjob = j0;
          jcnt = 0;
        }
        jcnt += (unsigned long long)__popcll(bal);
      } else {
        for (uint64_t m = bal; m; m &= m - 1)
          atomicAdd(&stats[job_of_cell(jobs, n_jobs, wc + __builtin_ctzll(m))].n_kept, 1ull);
      }
    }
  }
  if (stats && lane == 0 && jcnt) atomicAdd(&stats[wjob].n_kept, jcnt);
  for (int o = 32; o > 0; o >>= 1) mine += __shfl_down(mine, o, 64);
  if (lane == 0 && mine) atomicAdd(nkept, mine);
}

// The same for K > 256 inputs: a thread per cell.
template <int MODE, typename Flags>
__global__ void k_prune_final_wide(const int64_t* row_ptr, const int32_t* col, const uint8_t* out,
                                   int64_t n_cells, int32_t K, Flags removed,
                                   uint8_t* kept, uint64_t* mask, int32_t W,
                                   unsigned long long* nkept, const int64_t* d_total,
                                   int64_t cap_edges, const int32_t* last, int32_t sweeps) {
  if (d_total && *d_total > cap_edges) return;
  if (sweeps > 0 && *last >= sweeps) return;
  unsigned long long mine = 0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells;
       c += (int64_t)gridDim.x * blockDim.x) {
    const bool k = !removed[c];
    kept[c] = k ? 1 : 0;
    mine += k;
    for (int w = 0; w < W; ++w) {
      uint64_t m = 0;
      if (k)
        for (int b = 0; b < 64 && w * 64 + b < K; ++b)
          m |= (uint64_t)row_good<MODE>(row_ptr, col, out, removed, c * K + w * 64 + b) << b;
      mask[c * W + w] = m;
    }
  }
  for (int o = 32; o > 0; o >>= 1) mine += __shfl_down(mine, o, 64);
  if ((threadIdx.x & 63) == 0 && mine) atomicAdd(nkept, mine);
}

// reverse CSR of a graph: in-degree histogram -> offsets -> scatter (the
// cursors count down to zero again)
int32_t reverse_csr(const int64_t* row_ptr, const int32_t* col, int64_t n_cells, int32_t K,
                    const PruneWork& w, hipStream_t s) {
  const int64_t n_rows = n_cells * K;
  const unsigned row_blocks = (unsigned)((n_rows + 255) / 256);
  int32_t rc;
  if (n_rows > 0) {
    hipLaunchKernelGGL(k_indegree, dim3(row_blocks), dim3(256), 0, s, row_ptr, col, n_rows, w.rcur,
                       w.d_total, w.cap_edges);
    GIS_LAUNCH_CHECK("k_indegree");
  }
  if ((rc = scan_exclusive_i32(w.rcur, w.rptr, n_cells, w.rptr + n_cells, w.scan_tmp, s)) != GIS_OK)
    return rc;
  if (n_rows > 0) {
    hipLaunchKernelGGL(k_scatter, dim3(row_blocks), dim3(256), 0, s, row_ptr, col, n_rows, w.rptr,
                       w.rcur, w.rrow, w.d_total, w.cap_edges);
    GIS_LAUNCH_CHECK("k_scatter");
  }
  return GIS_OK;
}

template <int MODE>
int32_t sweeps_mode(const int64_t* row_ptr, const int32_t* col, const uint8_t* out,
                    int64_t n_cells, int32_t K, const PruneWork& w, int32_t s0, int32_t count,
                    hipStream_t s) {
  const int32_t cpb = 256 / K;
  const int64_t groups = (n_cells + cpb - 1) / cpb;
  const int64_t cap = w.sweep_blocks > 0 ? w.sweep_blocks : 4096;
  const unsigned nb = (unsigned)(groups < cap ? (groups > 0 ? groups : 1) : cap);
  for (int32_t i = 0; i < count; ++i) {
    hipLaunchKernelGGL((k_sweep<MODE>), dim3(nb), dim3(256), 0, s, row_ptr, col, out, n_cells, K,
                       cpb, w.removed, w.last, s0 + i, w.d_total, w.cap_edges);
    GIS_LAUNCH_CHECK("k_sweep");
  }
  return GIS_OK;
}

int32_t frontier_steps(int32_t analysis, int64_t n_cells, int32_t K, const PruneWork& w,
                       int32_t t0, int32_t count, hipStream_t s) {
  const int32_t Kp = (K + 7) & ~7;
  const unsigned nb = (unsigned)(w.front_blocks > 0 ? w.front_blocks : 2048);
  for (int32_t i = 0; i < count; ++i) {
    const int32_t t = t0 + i;
    const int32_t* cur = w.front + ((t & 1) ? n_cells : 0);
    int32_t* nxt = w.front + ((t & 1) ? 0 : n_cells);
    if (analysis == GIS_ANALYSIS_NONLEAVING) {
      hipLaunchKernelGGL(k_front_step_nl, dim3(nb), dim3(256), 0, s, (const int64_t*)w.rptr,
                         (const int32_t*)w.rrow, K, w.removed, w.rowstate, w.good, cur, nxt,
                         w.fcount, t);
      GIS_LAUNCH_CHECK("k_front_step_nl");
    } else {
      hipLaunchKernelGGL(k_front_mark_ctl, dim3(nb), dim3(256), 0, s, (const int64_t*)w.rptr,
                         (const int32_t*)w.rrow, K, Kp, w.rowbad, w.cand, cur, w.fcount, t);
      GIS_LAUNCH_CHECK("k_front_mark_ctl");
      hipLaunchKernelGGL(k_front_eval_ctl, dim3((unsigned)((n_cells + 1023) / 1024 < 2048 ? (n_cells + 1023) / 1024 : 2048)), dim3(1024), 0, s,
                         n_cells, K, Kp, w.removed, (const uint8_t*)w.rowbad, w.cand, nxt,
                         w.fcount, t);
      GIS_LAUNCH_CHECK("k_front_eval_ctl");
    }
  }
  return GIS_OK;
}

int32_t frontier_init(int32_t analysis, const int64_t* row_ptr, const int32_t* col,
                      const uint8_t* out, int64_t n_cells, int32_t K, const PruneWork& w,
                      hipStream_t s) {
  int32_t rc;
  if ((rc = fill_i32(w.fcount, 0, 3, s))) return rc;
  if (analysis != GIS_ANALYSIS_NONLEAVING) {
    if ((rc = fill_u8(w.cand, 0, n_cells, s))) return rc;
    hipLaunchKernelGGL(k_front_init_ctl, dim3((unsigned)((n_cells + 1023) / 1024 < 2048 ? (n_cells + 1023) / 1024 : 2048)), dim3(1024), 0, s, out, n_cells, K,
                       (K + 7) & ~7, w.removed, w.rowbad, w.front, w.fcount);
    GIS_LAUNCH_CHECK("k_front_init_ctl");
    return GIS_OK;
  }
  if (K > 256) {
    hipLaunchKernelGGL(k_front_init_nl_wide, dim3(grid_for(n_cells)), dim3(256), 0, s, row_ptr,
                       col, n_cells, K, (const uint8_t*)w.removed, w.rowstate, w.good, w.front,
                       w.fcount);
    GIS_LAUNCH_CHECK("k_front_init_nl_wide");
    return GIS_OK;
  }
  const int32_t cpb = 256 / K;
  const int64_t groups = (n_cells + cpb - 1) / cpb;
  const unsigned nb = (unsigned)(groups < 8192 ? (groups > 0 ? groups : 1) : 8192);
  hipLaunchKernelGGL(k_front_init_nl, dim3(nb), dim3(256), 0, s, row_ptr, col, n_cells, K, cpb,
                     (const uint8_t*)w.removed, w.rowstate, w.good, w.front, w.fcount);
  GIS_LAUNCH_CHECK("k_front_init_nl");
  return GIS_OK;
}

template <int MODE>
int32_t final_mode(const int64_t* row_ptr, const int32_t* col, const uint8_t* out,
                   int64_t n_cells, int32_t K, const PruneWork& w, uint8_t* kept, uint64_t* mask,
                   int32_t W, unsigned long long* d_nkept, int32_t sweeps, const Job* jobs,
                   int32_t n_jobs, JobStats* stats, const uint8_t* level, const int32_t* idx,
                   const void* rowinfo, int32_t frontier, hipStream_t s) {
  // rows are evaluated against the flags packed 32 to a word when there is
  // room for them (w.rbits) and no frontier state gives the good rows
  const bool packed = w.rbits && n_cells <= w.rbits_cells && !rowinfo;
  if (packed) {
    hipLaunchKernelGGL(k_pack_flags, dim3(grid_for((n_cells + 31) / 32)), dim3(256), 0, s,
                       (const uint8_t*)w.removed, n_cells, w.rbits);
    GIS_LAUNCH_CHECK("k_pack_flags");
  }
  const ByteFlags bytes{(const uint8_t*)w.removed};
  const BitFlags bits{(const uint32_t*)w.rbits};
  const int64_t n_rows = n_cells * K;
  if (packed && K <= 256 && w.rowbits && n_rows <= w.rowbits_rows) {
    const int64_t words = (n_rows + 63) / 64;
    const int64_t waves = (words + kRowsIlp - 1) / kRowsIlp;
    const unsigned nb = (unsigned)((waves + 3) / 4 < 8192 ? (waves + 3) / 4 : 8192);
    hipLaunchKernelGGL((k_row_good<MODE, BitFlags>), dim3(nb), dim3(256), 0, s, row_ptr, col, out,
                       w.first, n_rows, K, bits, w.rowbits, w.d_total, w.cap_edges,
                       (const int32_t*)w.last, sweeps);
    GIS_LAUNCH_CHECK("k_row_good");
    hipLaunchKernelGGL((k_cell_masks<BitFlags>), dim3(grid_for(n_cells)), dim3(256), 0, s, n_cells,
                       K, bits, (const uint64_t*)w.rowbits, kept, mask, W, d_nkept, w.d_total,
                       w.cap_edges, (const int32_t*)w.last, sweeps, jobs, n_jobs, stats, level,
                       idx);
    GIS_LAUNCH_CHECK("k_cell_masks");
    return GIS_OK;
  }
  if (K <= 256) {
    const int32_t cpb = 256 / K;
    const int64_t groups = (n_cells + cpb - 1) / cpb;
    const unsigned nb = (unsigned)(groups < 4096 ? (groups > 0 ? groups : 1) : 4096);
    if (packed)
      hipLaunchKernelGGL((k_prune_final<MODE, BitFlags>), dim3(nb), dim3(256), 0, s, row_ptr, col,
                         out, n_cells, K, cpb, bits, kept, mask, W, d_nkept, w.d_total,
                         w.cap_edges, (const int32_t*)w.last, sweeps, jobs, n_jobs, stats, level,
                         idx, rowinfo, frontier);
    else
      hipLaunchKernelGGL((k_prune_final<MODE, ByteFlags>), dim3(nb), dim3(256), 0, s, row_ptr,
                         col, out, n_cells, K, cpb, bytes, kept, mask, W, d_nkept, w.d_total,
                         w.cap_edges, (const int32_t*)w.last, sweeps, jobs, n_jobs, stats, level,
                         idx, rowinfo, frontier);
    GIS_LAUNCH_CHECK("k_prune_final");
    return GIS_OK;
  } else {
    if (packed)
      hipLaunchKernelGGL((k_prune_final_wide<MODE, BitFlags>), dim3(grid_for(n_cells)), dim3(256),
                         0, s, row_ptr, col, out, n_cells, K, bits, kept, mask, W, d_nkept,
                         w.d_total, w.cap_edges, (const int32_t*)w.last, sweeps);
    else
      hipLaunchKernelGGL((k_prune_final_wide<MODE, ByteFlags>), dim3(grid_for(n_cells)),
                         dim3(256), 0, s, row_ptr, col, out, n_cells, K, bytes, kept, mask, W,
                         d_nkept, w.d_total, w.cap_edges, (const int32_t*)w.last, sweeps);
    GIS_LAUNCH_CHECK("k_prune_final_wide");
  }
  // per-job kept counts for the wide variant
  if (stats) return batch_count_kept_cells(jobs, n_jobs, n_cells, kept, stats, s);
  return GIS_OK;
}

}  // namespace

int32_t launch_check_graph(const int64_t* row_ptr, const int32_t* col, int64_t n_rows,
                           int64_t n_edges, int64_t n_cells, uint32_t* d_err, hipStream_t s) {
  int32_t rc = fill_u32(d_err, 0u, 1, s);
  if (rc != GIS_OK) return rc;
  hipLaunchKernelGGL(k_check_graph, dim3(grid_for(n_rows > n_edges ? n_rows : n_edges)), dim3(256),
                     0, s, row_ptr, col, n_rows, n_edges, n_cells, d_err);
  GIS_LAUNCH_CHECK("k_check_graph");
  return GIS_OK;
}

int32_t prune_sweeps(const int64_t* row_ptr, const int32_t* col, const uint8_t* out,
                     int64_t n_cells, int32_t K, int32_t analysis, const PruneWork& w,
                     int32_t first, int32_t count, hipStream_t s) {
  if (n_cells == 0 || count <= 0) return GIS_OK;
  if (analysis == GIS_ANALYSIS_NONLEAVING)
    return sweeps_mode<GIS_ANALYSIS_NONLEAVING>(row_ptr, col, out, n_cells, K, w, first, count, s);
  return sweeps_mode<GIS_ANALYSIS_CONTROLLED>(row_ptr, col, out, n_cells, K, w, first, count, s);
}

int32_t prune_wsweeps(const int64_t* row_ptr, const int32_t* col, int64_t n_cells, int32_t K,
                      const PruneWork& w, int32_t first, int32_t count, hipStream_t s) {
  if (n_cells == 0 || count <= 0) return GIS_OK;
  const int64_t tiles = (n_cells + 255) / 256;
  const int64_t cap = w.sweep_blocks > 0 ? w.sweep_blocks : 4096;
  const unsigned nb = (unsigned)(tiles < cap ? tiles : cap);
  for (int32_t i = 0; i < count; ++i) {
    const int32_t sw = first + i;
    if (sw == 0)
      hipLaunchKernelGGL(k_wsweep<true>, dim3(nb), dim3(256), 0, s, row_ptr, col, n_cells,
                         K, w.removed, w.wpos, w.wtgt, w.last, sw, w.d_total,
                         w.cap_edges);
    else
      hipLaunchKernelGGL(k_wsweep<false>, dim3(nb), dim3(256), 0, s, row_ptr, col, n_cells,
                         K, w.removed, w.wpos, w.wtgt, w.last, sw, w.d_total,
                         w.cap_edges);
    GIS_LAUNCH_CHECK("k_wsweep");
  }
  return GIS_OK;
}

int32_t prune_frontier_start(const int64_t* row_ptr, const int32_t* col, const uint8_t* out,
                             int64_t n_cells, int32_t K, int32_t analysis, const PruneWork& w,
                             hipStream_t s) {
  if (n_cells == 0) return GIS_OK;
  int32_t rc;
  if ((rc = reverse_csr(row_ptr, col, n_cells, K, w, s)) != GIS_OK) return rc;
  return frontier_init(analysis, row_ptr, col, out, n_cells, K, w, s);
}

int32_t prune_frontier_steps(const int64_t* row_ptr, const int32_t* col, int64_t n_cells, int32_t K,
                             int32_t analysis, const PruneWork& w, int32_t first, int32_t count,
                             hipStream_t s) {
  if (n_cells == 0 || count <= 0) return GIS_OK;
  (void)row_ptr;
  (void)col;
  return frontier_steps(analysis, n_cells, K, w, first, count, s);
}

int32_t prune_final(const int64_t* row_ptr, const int32_t* col, const uint8_t* out,
                    int64_t n_cells, int32_t K, int32_t analysis, const PruneWork& w,
                    uint8_t* kept, uint64_t* mask, int32_t mask_words,
                    unsigned long long* d_nkept, int32_t sweeps, const Job* jobs, int32_t n_jobs,
                    JobStats* stats, const uint8_t* level, const int32_t* idx, int32_t frontier,
                    hipStream_t s) {
  if (n_cells == 0) return GIS_OK;
  if (analysis == GIS_ANALYSIS_NONLEAVING)
    return final_mode<GIS_ANALYSIS_NONLEAVING>(
        row_ptr, col, out, n_cells, K, w, kept, mask, mask_words, d_nkept, sweeps, jobs, n_jobs,
        stats, level, idx, frontier ? (const void*)w.rowstate : nullptr, frontier, s);
  const void* info = frontier == kCellFrontier ? (const void*)w.badmask
                     : frontier                ? (const void*)w.rowbad
                                               : nullptr;
  return final_mode<GIS_ANALYSIS_CONTROLLED>(row_ptr, col, out, n_cells, K, w, kept, mask,
                                             mask_words, d_nkept, sweeps, jobs, n_jobs, stats,
                                             level, idx, info, frontier, s);
}

}  // namespace gis
