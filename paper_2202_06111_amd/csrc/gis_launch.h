// Host launchers of the analysis, covering-index, refinement and query
// translation units, and device helpers of the analysis kernels (the build
// kernel's unit does not include this header).
#pragma once

#include "gis_internal.h"

namespace gis {

// Appends v to list for every thread with add set, with one global atomic
// per block (a frontier list's counter is shared by the whole device, and
// per-wave atomics on it serialise).  Every thread of the block must call it
// the same number of times.
__device__ __forceinline__ void append_block(bool add, int32_t v, int32_t* list, int32_t* count) {
  __shared__ int32_t s_cnt, s_base;
  const uint64_t m = __ballot(add);
  const int lane = threadIdx.x & 63;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  int32_t woff = 0;
  if (lane == 0 && m) woff = atomicAdd(&s_cnt, (int32_t)__popcll(m));
  woff = __shfl(woff, 0, 64);
  __syncthreads();
  if (threadIdx.x == 0 && s_cnt) s_base = atomicAdd(count, s_cnt);
  __syncthreads();
  if (add) list[s_base + woff + __popcll(m & ((1ull << lane) - 1))] = v;
}

// k_prune.hip
struct PruneWork {
  uint8_t* removed;  // [n_cells] 0 on entry to the sweeps
  int32_t* last;     // 1 + index of the last sweep that removed a cell (0 on entry)
  // frontier phase
  int64_t* rptr;     // [n_cells + 1] reverse-CSR offsets
  int32_t* rrow;     // [cap_edges] in-rows per target cell
  int32_t* rcur;     // [n_cells] in-degree cursors: zero on entry, left zero
  uint32_t* rowstate;  // nonleaving: [n_rows] live targets per row
  int32_t* good;       // nonleaving: [n_cells] live rows per cell
  uint8_t* rowbad;     // controlled: [n_cells * Kp] bad-row flags (same memory as rowstate)
  uint8_t* cand;       // controlled: [n_cells] candidate flags (same memory as good)
  // cell-grouped frontier (K <= 64): one reverse entry per (source cell,
  // target) with the inputs whose rows meet the target as a bit mask
  int32_t* rsrc;       // [entries] source cells (same memory as rrow)
  uint64_t* rmask;     // [entries] input masks
  uint64_t* badmask;   // controlled: [n_cells] bad rows of each cell (same memory as rowstate)
  // nonleaving witness sweeps
  int64_t* wpos;       // [n_cells] position of the cell's witness edge (-1: the span's first)
  int32_t* wtgt;       // [n_cells] its target
  uint32_t* rbits;     // removed flags packed 32 to a word for the final pass, or null
  int64_t rbits_cells; // cells rbits has room for (the final pass packs only up to that)
  uint64_t* rowbits;   // good-row flags of the final pass, 64 rows a word, or null
  const int32_t* first;  // [rows] each row's first target (-1: none) from the build, or null
  int64_t rowbits_rows;  // rows rowbits has room for
  int32_t* front;      // [2 * n_cells] the two frontier lists
  int32_t* fcount;     // [3] rotating list lengths
  void* scan_tmp;
  int32_t sweep_blocks;    // grid cap of a sweep
  int32_t front_blocks;    // grid of a frontier step
  const int64_t* d_total;  // device edge total, or null: reverse-CSR kernels do no work
  int64_t cap_edges;       // when *d_total > cap_edges (col was not written)
};
// Flags an inconsistent CSR graph in *d_err (bit 0 offsets, bit 1 targets).
int32_t launch_check_graph(const int64_t* row_ptr, const int32_t* col, int64_t n_rows,
                           int64_t n_edges, int64_t n_cells, uint32_t* d_err, hipStream_t s);
// Sweeps first .. first+count-1 (K <= 256).  Converged when *last < first+count.
int32_t prune_sweeps(const int64_t* row_ptr, const int32_t* col, const uint8_t* out,
                     int64_t n_cells, int32_t K, int32_t analysis, const PruneWork& w,
                     int32_t first, int32_t count, hipStream_t s);
// nonleaving: witness sweeps first .. first+count-1; sweep 0 must come first
// in an analysis (it sets the first witnesses).  Converged when
// *last < first+count.
int32_t prune_wsweeps(const int64_t* row_ptr, const int32_t* col, int64_t n_cells, int32_t K,
                      const PruneWork& w, int32_t first, int32_t count, hipStream_t s);
// Reverse CSR, the counters from the current removed flags, and the first
// frontier (present cells without a good row); fcount[0] = its length.
int32_t prune_frontier_start(const int64_t* row_ptr, const int32_t* col, const uint8_t* out,
                             int64_t n_cells, int32_t K, int32_t analysis, const PruneWork& w,
                             hipStream_t s);
// Frontier steps first .. first+count-1; step t takes list t & 1 with length
// fcount[t % 3].  Done when fcount[(first+count) % 3] == 0.
int32_t prune_frontier_steps(const int64_t* row_ptr, const int32_t* col, int64_t n_cells, int32_t K,
                             int32_t analysis, const PruneWork& w, int32_t first, int32_t count,
                             hipStream_t s);
// kept flags, masks (mask_words per cell) and the kept count (added to
// *d_nkept, and per job to stats[j].n_kept when stats is set); with
// sweeps > 0, only if sweep sweeps-1 removed nothing.  With level (and idx)
// set and K <= 256 it also turns every removed cell into a hole of its
// job's covering index.  frontier: kRowFrontier or kCellFrontier when that
// frontier phase ran to its end, whose state then gives the good rows (K <=
// 256; no target is read); 0 when the sweeps converged.
constexpr int32_t kRowFrontier = 1, kCellFrontier = 2;
int32_t prune_final(const int64_t* row_ptr, const int32_t* col, const uint8_t* out,
                    int64_t n_cells, int32_t K, int32_t analysis, const PruneWork& w,
                    uint8_t* kept, uint64_t* mask, int32_t mask_words,
                    unsigned long long* d_nkept, int32_t sweeps, const Job* jobs, int32_t n_jobs,
                    JobStats* stats, const uint8_t* level, const int32_t* idx, int32_t frontier,
                    hipStream_t s);

// k_frontier.hip: the frontier phase over the cell-grouped reverse graph
// (1 <= K <= 64).  cells_start: the reverse-graph entry counts per target
// into rcur (zero on entry) and the reverse offsets rptr (entry total at
// rptr[n_cells]).  cells_scatter, once rsrc/rmask hold that many entries,
// fills them (rcur is left zero) and sets the analysis state from the current
// removed flags and the first frontier (fcount[0]).  cells_steps: frontier
// steps t0 .. t0+count-1, with the list conventions of prune_frontier_steps.
// any_removed: some removed flag may be set (otherwise they are not read).
int32_t cells_start(const int64_t* row_ptr, const int32_t* col, int64_t n_cells, int32_t K,
                    bool any_removed, const PruneWork& w, hipStream_t s);
int32_t cells_scatter(const int64_t* row_ptr, const int32_t* col, const uint8_t* out,
                      int64_t n_cells, int32_t K, int32_t analysis, bool any_removed,
                      const PruneWork& w, hipStream_t s);
// One pass instead of cells_start + cells_scatter: the state, the first
// frontier and the entries appended to `stage` (any order, up to stage_cap of
// them; *n_staged, cleared here, receives their number even past the cap,
// when nothing past it was written and the two-pass route must be taken),
// their counts per target added to w.rcur (zero on entry; clear it again
// before the two-pass route).  cells_unstage then scans the counts and
// places the entries.
struct Staged {
  int32_t j, c;  // target, source cell
  uint64_t m;    // input mask
};
int32_t cells_stage(const int64_t* row_ptr, const int32_t* col, const uint8_t* out,
                    int64_t n_cells, int32_t K, int32_t analysis, bool any_removed,
                    const PruneWork& w, Staged* stage, int64_t stage_cap,
                    unsigned long long* n_staged, hipStream_t s);
int32_t cells_unstage(const Staged* stage, int64_t n_staged, int64_t n_cells, const PruneWork& w,
                      hipStream_t s);
int32_t cells_steps(int64_t n_cells, int32_t K, int32_t analysis, const PruneWork& w, int32_t t0,
                    int32_t count, hipStream_t s);

// k_index.hip, job-batched: covering indexes of every job's cell list (the
// jobs' state arrays are cleared first by the caller).  Flags invalid lists in
// *d_err (bit 0: index out of range, bit 1: not canonical / duplicate,
// bit 2: overlapping cells).  Jobs whose ci.uniform is set only get checked.
struct BatchArgs {
  const Job* jobs;
  int32_t n_jobs;
  int32_t n;              // state dimension
  int32_t K;
  const uint8_t* level;   // global cell list
  const int32_t* idx;
  int64_t blocks[LK_KINDS];
};
// ... and the prefix counts of the jobs with index arrays: pfx_all receives
// total_slots + 1 values over the batch's concatenated state arrays state_all.
// Without `validate` the list is taken as valid (produced by the library)
// and no check is made.
int32_t batch_index_build(const BatchArgs& b, uint32_t* d_err, const uint8_t* state_all,
                          int64_t* pfx_all, int64_t total_slots, void* scan_tmp, bool validate,
                          hipStream_t s);
int32_t batch_mark_dropped(const BatchArgs& b, const uint8_t* kept, hipStream_t s);

// k_scc.hip: Definition 6 read literally.  Work arrays, [n_cells] each
// unless stated; best and left are adjacent ([n_jobs] each), h_best pinned
// host memory of [2 * n_jobs] and h_last of one word.
struct SccWork {
  int32_t *color, *comp, *size, *minid;
  uint32_t* rose;  // per cell: the colour sweep that last raised its colour
  uint8_t *rem, *bw, *loop, *inset;
  unsigned long long *best, *left;
  uint32_t* last;
  unsigned long long* h_best;
  uint32_t* h_last;
  int32_t* hint;  // host, per pass (trim, colour, backward, reach): sweeps needed, in and out
};
// removed: in, the non-leaving analysis' removed flags; out, 1 for every cell
// outside the largest component with a cycle and the cells with a path into
// it (per job of `jobs`, or one job when jobs is null).  Synchronises s.
int32_t largest_component_set(const int64_t* row_ptr, const int32_t* col, int64_t n_cells,
                              int32_t K, const Job* jobs, int32_t n_jobs, uint8_t* removed,
                              const SccWork& w, hipStream_t s);

// k_refine.hip, job-batched
// Boundary flags of the kept cells (Sec. 3.1.1) and, with flag_next, for
// jobs with a next layout, the next-covering flags (those arrays are zero on
// entry; batch_compact leaves them zero again).
int32_t batch_boundary(const BatchArgs& b, const uint8_t* kept, int32_t rule, uint8_t* boundary,
                       JobStats* stats, hipStream_t s, bool flag_next = true);
// Neighbourhood selection (Sec. 3.1.2) after batch_boundary without next
// flags: sel (zero on entry) gets the boundary cells and the nn (1..64) kept
// cells nearest to each, then the next-covering flags are set from sel.
int32_t batch_neighbours(const BatchArgs& b, const uint8_t* kept, const uint8_t* boundary,
                         int32_t nn, uint8_t* sel, JobStats* stats, hipStream_t s);
// Standard subdivision (Sec. 2.1): the next-covering flags of both halves of
// every kept cell across dimension `dim`, the next layouts being level 0 of
// the grid with twice the cells along `dim`; split[c] = 1 for the cells cut,
// stats[j].n_boundary counts them; kept cells not of level 0 or outside the
// grid are skipped and counted in *err (may be null).
int32_t batch_bisect(const BatchArgs& b, const uint8_t* kept, int32_t dim, uint8_t* split,
                     JobStats* stats, uint32_t* err, hipStream_t s);
// pos: exclusive scan of the batch's next-flag array; writes the new global
// cell list (up to cap) and each job's next_start / level_start.
int32_t batch_compact(const BatchArgs& b, const int64_t* pos, int64_t cap, uint8_t* level_out,
                      int32_t* idx_out, JobStats* stats, hipStream_t s);
int32_t batch_coarse(const BatchArgs& b, uint8_t* level, int32_t* idx, hipStream_t s);
// stats[j].n_kept = 0 for every job.
int32_t batch_clear_kept(JobStats* stats, int32_t n_jobs, hipStream_t s);
// Kept cells per job into stats[j].n_kept.
int32_t batch_count_kept(const BatchArgs& b, const uint8_t* kept, JobStats* stats, hipStream_t s);
// The same from the job table alone (any launch layout).
int32_t batch_count_kept_cells(const Job* jobs, int32_t n_jobs, int64_t n_cells,
                               const uint8_t* kept, JobStats* stats, hipStream_t s);

// k_index.hip: copies `bytes` (a multiple of 4) of device memory into
// host-coherent pinned memory, then stores seq into *host_flag.
int32_t publish(const void* src, void* host_dst, size_t bytes, uint32_t* host_flag, uint32_t seq,
                hipStream_t s);

// k_query.hip
int32_t launch_query(const CoverIndex& ci, const GridArgs& g, const uint8_t* kept,
                     const uint64_t* mask, int32_t mask_words, const double* states, int64_t n,
                     uint8_t* member, uint64_t* adm, hipStream_t s);

}  // namespace gis
