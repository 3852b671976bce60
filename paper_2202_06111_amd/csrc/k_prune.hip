// Graph analysis (Sec. 2.3) as a frontier computation on the device.
//
// Both readings remove cells until a fixed point; the removed set is the least
// fixed point of a monotone operator, so any removal order reaches it:
//   controlled : row (c, u) turns bad when it is OUT or one of its targets is
//                removed; a cell is removed when all its rows are bad;
//   nonleaving : row (c, u) dies when all its targets are removed; a cell is
//                removed when all its rows are dead (a cell with no path to a
//                cycle of the input-union symbolic image, Definition 6).
// Steps: in-degree histogram -> offsets -> scatter of source rows (reverse
// CSR) -> initial counts and first removals -> one persistent launch that
// drains a device work queue (a wave per removed cell, its lanes over the
// cell's in-rows) and stops by itself when no work is left in flight ->
// kept flags and admissible-input masks.
#include "gis_internal.h"

namespace gis {

namespace {

// qctl layout: one 128-byte line per counter, so waves polling `pending`
// do not contend with the increments of `alloc` and `head`
constexpr int Q_ALLOC = 0, Q_HEAD = 32, Q_PENDING = 64, Q_ERROR = 96, Q_WORDS = 128;
constexpr int32_t kSlotDone = -2;  // written into waiting slots once nothing is left
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
                                                  int64_t n_rows, int32_t* deg) {
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
                                                 int32_t* cursor, int32_t* rrow) {
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
  for (int i = threadIdx.x; i < kHash; i += 256)
    if (key[i] >= 0) {
      base[i] = atomicAdd(&cursor[key[i]], cnt[i]);
      cnt[i] = 0;
    }
  __syncthreads();
  for (int64_t e = e0; e < e1; ++e) {
    const int32_t j = col[e];
    const int sl = lds_slot(key, j, false);
    const int32_t pos = sl >= 0 ? base[sl] + atomicAdd(&cnt[sl], 1) : atomicAdd(&cursor[j], 1);
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

// bad bits of the controlled analysis: a row starts bad when it is OUT.
__global__ void k_badbits_init(const uint8_t* out, int64_t n_rows, uint32_t* bits) {
  const int64_t words = (n_rows + 31) / 32;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words;
       w += (int64_t)gridDim.x * blockDim.x) {
    uint32_t b = 0;
    for (int i = 0; i < 32; ++i) {
      const int64_t r = w * 32 + i;
      if (r < n_rows && out[r]) b |= 1u << i;
    }
    bits[w] = b;
  }
}

// Every piece of state the drain shares (row flags, cell counters, the queue
// and its counters) changes only through agent-scope atomics, so relaxed
// ordering suffices and no cache-wide fence is issued (on this GPU an
// acquire or release at agent scope invalidates or writes back an XCD's whole
// L2).  Termination needs only the modification order of `pending`: a cell's
// increment precedes the decrement of the item whose processing pushed it
// (same thread, same location), so `pending` stays >= 1 until every pushed
// cell has been processed.
__device__ __forceinline__ void push_removed(int32_t* queue, int32_t* qctl, int32_t cell) {
  __hip_atomic_fetch_add(&qctl[Q_PENDING], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int32_t slot =
      __hip_atomic_fetch_add(&qctl[Q_ALLOC], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&queue[slot], cell, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int MODE>
__global__ void k_prune_init(const int64_t* row_ptr, int64_t n_cells, int32_t K,
                             const uint32_t* bits, int32_t* alive, int32_t* good, int32_t* queue,
                             int32_t* qctl) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells;
       c += (int64_t)gridDim.x * blockDim.x) {
    int32_t g = 0;
    for (int32_t u = 0; u < K; ++u) {
      const int64_t r = c * K + u;
      if (MODE == GIS_ANALYSIS_CONTROLLED) {
        g += !((bits[r >> 5] >> (r & 31)) & 1u);
      } else {
        const int32_t deg = (int32_t)(row_ptr[r + 1] - row_ptr[r]);
        alive[r] = deg;
        g += deg > 0;
      }
    }
    good[c] = g;
    if (g == 0) push_removed(queue, qctl, (int32_t)c);
  }
}

// Persistent drain of the removal queue, one wave per block.  The loop
// skeleton has no lane-dependent branch: the queue counters are updated by
// atomics every lane executes (lane 0 contributes the increment, the others
// add 0), the claimed slot and the removed cell are read into scalar
// registers (readfirstlane), and every exit tests a scalar.  So all lanes of
// the wave run the same iterations; only the loop over a cell's in-rows is
// lane-divergent, and it has no early exit.  Exit conditions every wave
// reaches: the claimed slot is past the last possible slot, or it is still
// empty while nothing is in flight (no further removal can happen), or a
// wall-clock limit (sets the error word; never expected).
template <int MODE>
__global__ __launch_bounds__(64) void k_prune_run(const int64_t* rptr, const int32_t* rrow,
                                                  int64_t n_cells, int32_t K, uint32_t* bits,
                                                  int32_t* alive, int32_t* good, int32_t* queue,
                                                  int32_t* qctl) {
  const int lane = threadIdx.x;
  const int32_t one = lane == 0 ? 1 : 0;
  const uint64_t t0 = wall_clock64();
  const uint64_t limit = 60ull * 100000000ull;  // 60 s of the 100 MHz constant clock
  for (;;) {
    const int32_t i = __builtin_amdgcn_readfirstlane(
        __hip_atomic_fetch_add(&qctl[Q_HEAD], one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if ((int64_t)i >= n_cells) break;
    int32_t c = -1;
    for (uint32_t spin = 0;; ++spin) {
      c = __builtin_amdgcn_readfirstlane(
          __hip_atomic_load(&queue[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (c >= 0 || c == kSlotDone) break;
      if ((spin & 63) == 0) {  // rarely: a slot claimed after the sentinels were written
        const int32_t pend = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&qctl[Q_PENDING], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (pend == 0) break;
        if (wall_clock64() - t0 > limit) {
          __hip_atomic_fetch_or(&qctl[Q_ERROR], one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
      __builtin_amdgcn_s_sleep(2);
    }
    if (c < 0) break;
    const int64_t b = rptr[c], e = rptr[c + 1];
    for (int64_t p = b + lane; p < e; p += 64) {
      const int32_t r = rrow[p];
      bool died;
      if (MODE == GIS_ANALYSIS_CONTROLLED) {
        const uint32_t bit = 1u << (r & 31);
        died = !(atomicOr(&bits[r >> 5], bit) & bit);
      } else {
        died = atomicSub(&alive[r], 1) == 1;
      }
      if (died) {
        const int32_t cell = r / K;
        if (atomicSub(&good[cell], 1) == 1) push_removed(queue, qctl, cell);
      }
    }
    const int32_t before = __builtin_amdgcn_readfirstlane(__hip_atomic_fetch_add(
        &qctl[Q_PENDING], -one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (before == 1) {
      // nothing is in flight and nothing can be pushed any more: release the
      // waves waiting on claimed but empty slots
      const int32_t a0 = __builtin_amdgcn_readfirstlane(
          __hip_atomic_load(&qctl[Q_ALLOC], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      int64_t h = __builtin_amdgcn_readfirstlane(
          __hip_atomic_load(&qctl[Q_HEAD], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      h = h < n_cells ? h : n_cells;
      for (int64_t q = a0 + lane; q < h; q += 64)
        __hip_atomic_store(&queue[q], kSlotDone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <int MODE>
__global__ void k_prune_final(int64_t n_cells, int32_t K, const uint32_t* bits,
                              const int32_t* alive, const int32_t* good, uint8_t* kept,
                              uint64_t* mask, int32_t W, unsigned long long* nkept,
                              const int32_t* qctl, int32_t* err_out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *err_out = qctl[Q_ERROR];
  unsigned long long mine = 0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells;
       c += (int64_t)gridDim.x * blockDim.x) {
    const bool k = good[c] > 0;
    kept[c] = k ? 1 : 0;
    mine += k;
    for (int w = 0; w < W; ++w) {
      uint64_t m = 0;
      if (k) {
        for (int b = 0; b < 64 && w * 64 + b < K; ++b) {
          const int64_t r = c * K + w * 64 + b;
          const bool ok = MODE == GIS_ANALYSIS_CONTROLLED ? !((bits[r >> 5] >> (r & 31)) & 1u)
                                                           : alive[r] > 0;
          m |= (uint64_t)ok << b;
        }
      }
      mask[c * W + w] = m;
    }
  }
  for (int o = 32; o > 0; o >>= 1) mine += __shfl_down(mine, o, 64);
  if ((threadIdx.x & 63) == 0 && mine) atomicAdd(nkept, mine);
}

template <int MODE>
int32_t prune_mode(const int64_t* row_ptr, const int32_t* col, const uint8_t* out, int64_t n_cells,
                   int32_t K, int64_t n_edges, const PruneWork& w, uint8_t* kept, uint64_t* mask,
                   int32_t W, unsigned long long* d_nkept, hipStream_t s) {
  const int64_t n_rows = n_cells * K;
  int32_t rc;
  // reverse CSR
  const unsigned row_blocks = (unsigned)((n_rows + 255) / 256);
  if ((rc = fill_i32(w.rcur, 0, n_cells, s)) != GIS_OK) return rc;
  if (n_edges > 0) {
    hipLaunchKernelGGL(k_indegree, dim3(row_blocks), dim3(256), 0, s, row_ptr, col, n_rows, w.rcur);
    GIS_LAUNCH_CHECK("k_indegree");
  }
  if ((rc = scan_exclusive_i32(w.rcur, w.rptr, n_cells, w.rptr + n_cells, w.scan_tmp, s)) != GIS_OK)
    return rc;
  if ((rc = fill_i32(w.rcur, 0, n_cells, s)) != GIS_OK) return rc;
  if (n_edges > 0) {
    hipLaunchKernelGGL(k_scatter, dim3(row_blocks), dim3(256), 0, s, row_ptr, col, n_rows, w.rptr,
                       w.rcur, w.rrow);
    GIS_LAUNCH_CHECK("k_scatter");
  }
  // initial state
  if ((rc = fill_i32(w.qctl, 0, Q_WORDS, s)) != GIS_OK) return rc;
  if ((rc = fill_i32(w.queue, -1, n_cells, s)) != GIS_OK) return rc;
  if (MODE == GIS_ANALYSIS_CONTROLLED) {
    hipLaunchKernelGGL(k_badbits_init, dim3(grid_for((n_rows + 31) / 32)), dim3(256), 0, s, out,
                       n_rows, w.badbits);
    GIS_LAUNCH_CHECK("k_badbits_init");
  }
  hipLaunchKernelGGL((k_prune_init<MODE>), dim3(grid_for(n_cells)), dim3(256), 0, s, row_ptr,
                     n_cells, K, (const uint32_t*)w.badbits, w.alive, w.good, w.queue, w.qctl);
  GIS_LAUNCH_CHECK("k_prune_init");
  // persistent drain: one wave per block, two per SIMD
  const int64_t waves = n_cells < 2048 ? (n_cells > 0 ? n_cells : 1) : 2048;
  hipLaunchKernelGGL((k_prune_run<MODE>), dim3((unsigned)waves), dim3(64), 0, s,
                     (const int64_t*)w.rptr, (const int32_t*)w.rrow, n_cells, K, w.badbits,
                     w.alive, w.good, w.queue, w.qctl);
  GIS_LAUNCH_CHECK("k_prune_run");
  if ((rc = fill_u32((uint32_t*)d_nkept, 0u, 2, s)) != GIS_OK) return rc;
  hipLaunchKernelGGL((k_prune_final<MODE>), dim3(grid_for(n_cells)), dim3(256), 0, s, n_cells, K,
                     (const uint32_t*)w.badbits, (const int32_t*)w.alive, (const int32_t*)w.good,
                     kept, mask, W, d_nkept, (const int32_t*)w.qctl, w.err_out);
  GIS_LAUNCH_CHECK("k_prune_final");
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

int32_t launch_prune(const int64_t* row_ptr, const int32_t* col, const uint8_t* out,
                     int64_t n_cells, int32_t K, int64_t n_edges, int32_t analysis,
                     const PruneWork& w, uint8_t* kept, uint64_t* mask, int32_t mask_words,
                     unsigned long long* d_nkept, hipStream_t s) {
  if (analysis == GIS_ANALYSIS_NONLEAVING)
    return prune_mode<GIS_ANALYSIS_NONLEAVING>(row_ptr, col, out, n_cells, K, n_edges, w, kept, mask,
                                               mask_words, d_nkept, s);
  return prune_mode<GIS_ANALYSIS_CONTROLLED>(row_ptr, col, out, n_cells, K, n_edges, w, kept, mask,
                                             mask_words, d_nkept, s);
}

}  // namespace gis
