// Definition 6 read literally (Sec. 2.3): the vertices of the largest
// strongly connected component of the input-union symbolic image, plus every
// vertex with a path into it.  Only components with a cycle count (two or
// more cells, or one with an edge to itself); equally large components go to
// the one holding the smallest cell id; per job of a batch.
//
// Every component with a cycle lies in the non-leaving set (cells with an
// infinite path), which the caller has computed; the search starts from it,
// less the cells that a backward trim shows to lie on no cycle.
// Components come from max-colour propagation: each candidate cell starts
// with its own id as colour and takes the largest colour of a candidate
// predecessor until nothing changes, so colour(c) is the largest id that
// reaches c.  A cell whose colour is its own id is a root; the cells of its
// colour that reach it are its component.  Every round of the search takes
// the components of all roots out of the candidates; it ends for a job when
// its best component is larger than what is left of its candidates.  Then a
// backward search from the best component gives the set.
//
// All passes are in-place sweeps over the rows (one thread per row, the
// row's cell from row / K) to a fixed point, checked every few sweeps: each
// sweep that changes something records its number (numbers grow through a
// pass), a sweep whose predecessor changed nothing returns at once, and a
// batch whose last sweep changed nothing has converged.  Sweeps alternate
// between ascending and descending row order, so that a change travels far
// along paths of either direction within one sweep.  A colour sweep takes
// only the rows of cells whose colour rose in the previous sweep or in this
// one (the sweep number of each cell's last rise is kept): a colour that
// stays put has already been passed on.
#include "gis_launch.h"

namespace gis {

namespace {

__device__ __forceinline__ int32_t job_at(const Job* jobs, int32_t n_jobs, int64_t c) {
  return jobs ? job_of_cell(jobs, n_jobs, c) : 0;
}

__device__ __forceinline__ int64_t first_cell(const Job* jobs, int32_t j) {
  return jobs ? jobs[j].cell_off : 0;
}

// sweep s - 1 changed nothing: the pass has converged
__device__ __forceinline__ bool converged(const uint32_t* last, uint32_t sweep) {
  return sweep > 1 && *last < sweep - 1;
}

// candidates = the non-leaving cells; no component assigned yet
__global__ void k_scc_begin(int64_t n, const uint8_t* removed, uint8_t* rem, int32_t* comp) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x) {
    rem[c] = removed[c] ? 0 : 1;
    comp[c] = -1;
  }
}

// backward trim, one step: mark the candidates with a candidate predecessor
__global__ void k_scc_haspred(const int64_t* row_ptr, const int32_t* col, int64_t n_rows,
                              int32_t K, const uint8_t* rem, uint8_t* haspred,
                              const uint32_t* last, uint32_t sweep) {
  if (converged(last, sweep)) return;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = r / K;
    if (!rem[c]) continue;
    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e)
      if (rem[col[e]]) haspred[col[e]] = 1;
  }
}

// ... and drop the candidates without one (no cycle passes through them);
// the marks are cleared for the next sweep
__global__ void k_scc_trim(int64_t n, uint8_t* rem, uint8_t* haspred, uint32_t* last,
                           uint32_t sweep) {
  if (converged(last, sweep)) return;  // as k_scc_haspred of this sweep did
  bool changed = false;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x) {
    if (rem[c] && !haspred[c]) {
      rem[c] = 0;
      changed = true;
    }
    haspred[c] = 0;
  }
  const uint64_t m = __ballot(changed);  // one atomic per wave
  if (m && (threadIdx.x & 63) == 0) atomicMax(last, sweep);
}

// a round's start: own colours, cleared reach flags and tallies
__global__ void k_scc_round(int64_t n, const uint8_t* rem, int32_t* color, uint32_t* rose,
                            uint8_t* bw, int32_t* size, int32_t* minid, uint8_t* loop) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x) {
    color[c] = rem[c] ? (int32_t)c : -1;
    rose[c] = 0;
    bw[c] = 0;
    size[c] = 0;
    minid[c] = INT32_MAX;
    loop[c] = 0;
  }
}

// one sweep of max-colour propagation along the edges of candidate cells;
// rose[c] is the sweep that last raised colour[c] (0: its own id).
//
// A block takes 256 rows at a time.  The cells it raises are also queued in
// LDS, and while there are any (at most kColQ; the rest wait for the next
// sweep, which takes them through rose[]) the block passes their colours on
// itself, for up to kColDepth generations: a colour then travels that many
// more edges per launch.  Each step is a valid max-colour update, so the
// fixed point is the same.
constexpr int kColQ = 256;
constexpr int kColDepth = 16;

__global__ __launch_bounds__(256) void k_scc_color(const int64_t* row_ptr, const int32_t* col,
                                                   int64_t n_rows, int32_t K, const uint8_t* rem,
                                                   int32_t* color, uint32_t* rose,
                                                   uint32_t* last, uint32_t sweep) {
  if (converged(last, sweep)) return;
  __shared__ int32_t s_q[2][kColQ];
  __shared__ int32_t s_n[2];
  const int t = threadIdx.x;
  bool changed = false;
  // passes row r's colour cc on; raised cells go to list o
  auto pass_on = [&](int64_t r, int32_t cc, int o) {
    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
      const int32_t v = col[e];
      if (rem[v] && color[v] < cc && atomicMax(&color[v], cc) < cc) {
        rose[v] = sweep;
        changed = true;
        const int k = atomicAdd(&s_n[o], 1);
        if (k < kColQ) s_q[o][k] = v;
      }
    }
  };
  for (int64_t tile = blockIdx.x; tile * 256 < n_rows; tile += gridDim.x) {
    if (t == 0) s_n[0] = 0;
    __syncthreads();
    const int64_t q = tile * 256 + t;
    if (q < n_rows) {
      const int64_t r = (sweep & 1) ? q : n_rows - 1 - q;
      const int64_t c = r / K;
      if (rem[c] && rose[c] + 1 >= sweep) pass_on(r, color[c], 0);
    }
    __syncthreads();
    int cur = 0;
    for (int depth = 0; depth < kColDepth; ++depth) {
      const int n = s_n[cur] < kColQ ? s_n[cur] : kColQ;  // the same in every thread
      if (n == 0) break;
      if (t == 0) s_n[cur ^ 1] = 0;
      __syncthreads();
      for (int k = t; k < n * K; k += 256) {
        const int32_t v = s_q[cur][k / K];
        pass_on((int64_t)v * K + k % K, color[v], cur ^ 1);
      }
      __syncthreads();
      cur ^= 1;
    }
  }
  const uint64_t m = __ballot(changed);  // one atomic per wave
  if (m && (t & 63) == 0) atomicMax(last, sweep);
}

// roots: candidate cells whose colour is their own id
__global__ void k_scc_roots(int64_t n, const uint8_t* rem, const int32_t* color, uint8_t* bw) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x)
    bw[c] = rem[c] && color[c] == (int32_t)c ? 1 : 0;
}

// one sweep of the backward search inside each colour: a candidate cell with
// an edge to a marked cell of its own colour reaches that colour's root
__global__ void k_scc_back(const int64_t* row_ptr, const int32_t* col, int64_t n_rows, int32_t K,
                           const uint8_t* rem, const int32_t* color, uint8_t* bw, uint32_t* last,
                           uint32_t sweep) {
  if (converged(last, sweep)) return;
  bool changed = false;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_rows;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = (sweep & 1) ? q : n_rows - 1 - q;
    const int64_t c = r / K;
    if (!rem[c] || bw[c]) continue;
    const int32_t cc = color[c];
    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
      const int32_t v = col[e];
      if (bw[v] && color[v] == cc) {
        bw[c] = 1;
        changed = true;
        break;
      }
    }
  }
  const uint64_t m = __ballot(changed);  // one atomic per wave
  if (m && (threadIdx.x & 63) == 0) atomicMax(last, sweep);
}

// size and smallest id of every root's component; self-loops of roots
__global__ void k_scc_tally(const int64_t* row_ptr, const int32_t* col, int64_t n_rows, int32_t K,
                            const int32_t* color, const uint8_t* bw, int32_t* size, int32_t* minid,
                            uint8_t* loop) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = r / K;
    if (!bw[c]) continue;
    const int32_t root = color[c];
    if (r % K == 0) {
      atomicAdd(&size[root], 1);
      atomicMin(&minid[root], (int32_t)c);
    }
    if (root == (int32_t)c)
      for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e)
        if (col[e] == (int32_t)c) loop[c] = 1;
  }
}

// the round's components leave the candidates (each cell keeps its
// component's smallest id); each job's best component with a cycle is kept
// as the key (size, -smallest id within the job)
__global__ void k_scc_pick(int64_t n, const Job* jobs, int32_t n_jobs, uint8_t* rem,
                           const int32_t* color, const uint8_t* bw, const int32_t* size,
                           const int32_t* minid, const uint8_t* loop, int32_t* comp,
                           unsigned long long* best) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x) {
    if (!rem[c] || !bw[c]) continue;
    const int32_t root = color[c];
    comp[c] = minid[root];
    rem[c] = 0;
    if (root == (int32_t)c && (size[c] >= 2 || loop[c])) {
      const int32_t j = job_at(jobs, n_jobs, c);
      const uint32_t local = (uint32_t)(minid[c] - first_cell(jobs, j));
      const unsigned long long key =
          ((unsigned long long)(uint32_t)size[c] << 32) | (unsigned long long)(0xFFFFFFFFu - local);
      atomicMax(&best[j], key);
    }
  }
}

// candidates left per job
__global__ void k_scc_left(int64_t n, const Job* jobs, int32_t n_jobs, const uint8_t* rem,
                           unsigned long long* left) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x)
    if (rem[c]) atomicAdd(&left[job_at(jobs, n_jobs, c)], 1ull);
}

// the set starts as each job's best component
__global__ void k_scc_seed(int64_t n, const Job* jobs, int32_t n_jobs, const int32_t* comp,
                           const unsigned long long* best, uint8_t* inset) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = job_at(jobs, n_jobs, c);
    const unsigned long long k = best[j];
    const int64_t want = first_cell(jobs, j) + (int64_t)(0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull));
    inset[c] = k != 0 && comp[c] >= 0 && (int64_t)comp[c] == want ? 1 : 0;
  }
}

// one sweep of the backward search from the set over all cells
__global__ void k_scc_reach(const int64_t* row_ptr, const int32_t* col, int64_t n_rows, int32_t K,
                            uint8_t* inset, uint32_t* last, uint32_t sweep) {
  if (converged(last, sweep)) return;
  bool changed = false;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_rows;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = (sweep & 1) ? q : n_rows - 1 - q;
    const int64_t c = r / K;
    if (inset[c]) continue;
    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e)
      if (inset[col[e]]) {
        inset[c] = 1;
        changed = true;
        break;
      }
  }
  const uint64_t m = __ballot(changed);  // one atomic per wave
  if (m && (threadIdx.x & 63) == 0) atomicMax(last, sweep);
}

__global__ void k_scc_end(int64_t n, const uint8_t* inset, uint8_t* removed) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x)
    removed[c] = inset[c] ? 0 : 1;
}

unsigned blocks_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

// Runs `sweep(id)` for id = 1, 2, ... in batches until a batch's last sweep
// changed nothing (the sweeps after a sweep that changed nothing return at
// once, so a batch may overshoot cheaply); at most `bound` sweeps (then the
// pass did not converge: internal error).  The first batch is w.hint[pass]
// (what the same pass of the same round needed in the caller's last solve)
// plus a margin, so that most passes end at their first check; the pass
// leaves the sweeps it needed there.
template <typename F>
int32_t to_fixed_point(const SccWork& w, int pass, int64_t bound, hipStream_t s, F&& sweep) {
  int32_t rc = fill_u32(w.last, 0u, 1, s);
  if (rc) return rc;
  int32_t batch = w.hint[pass] + 4 > 8 ? w.hint[pass] + 4 : 8;
  for (int64_t done = 0;;) {
    for (int32_t i = 1; i <= batch; ++i)
      if ((rc = sweep((uint32_t)(done + i)))) return rc;
    GIS_HIP(hipMemcpyAsync(w.h_last, w.last, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    GIS_HIP(hipStreamSynchronize(s));
    done += batch;
    if (*w.h_last < (uint32_t)done) {
      w.hint[pass] = (int32_t)*w.h_last + 1;  // incl. the sweep that changed nothing
      return GIS_OK;
    }
    if (done > bound) {
      set_error("internal: a component search did not converge");
      return GIS_E_INTERNAL;
    }
    if (batch < 64) batch *= 2;
  }
}

}  // namespace

int32_t largest_component_set(const int64_t* row_ptr, const int32_t* col, int64_t n_cells,
                              int32_t K, const Job* jobs, int32_t n_jobs, uint8_t* removed,
                              const SccWork& w, hipStream_t s) {
  if (n_cells == 0) return GIS_OK;
  const int64_t n_rows = n_cells * K;
  const unsigned gc = blocks_for(n_cells), gr = blocks_for(n_rows);
  int32_t rc;
  if ((rc = fill_u32((uint32_t*)w.best, 0u, 2 * (int64_t)n_jobs, s))) return rc;
  hipLaunchKernelGGL(k_scc_begin, dim3(gc), dim3(256), 0, s, n_cells, removed, w.rem, w.comp);
  GIS_LAUNCH_CHECK("k_scc_begin");
  // backward trim: candidates with no candidate predecessor lie on no cycle;
  // dropping them layer by layer leaves the cycles and the cells between
  // them (the non-leaving set's transient cells would otherwise take one
  // search round per layer)
  if ((rc = fill_u8(w.bw, 0, n_cells, s))) return rc;
  rc = to_fixed_point(w, 0, n_cells + 1, s, [&](uint32_t id) -> int32_t {
    hipLaunchKernelGGL(k_scc_haspred, dim3(gr), dim3(256), 0, s, row_ptr, col, n_rows, K,
                       (const uint8_t*)w.rem, w.bw, (const uint32_t*)w.last, id);
    GIS_LAUNCH_CHECK("k_scc_haspred");
    hipLaunchKernelGGL(k_scc_trim, dim3(gc), dim3(256), 0, s, n_cells, w.rem, w.bw, w.last, id);
    GIS_LAUNCH_CHECK("k_scc_trim");
    return GIS_OK;
  });
  if (rc) return rc;
  for (int64_t round = 0;; ++round) {
    if (round > n_cells) {  // every round takes at least one component out
      set_error("internal: the component search did not end");
      return GIS_E_INTERNAL;
    }
    hipLaunchKernelGGL(k_scc_round, dim3(gc), dim3(256), 0, s, n_cells, (const uint8_t*)w.rem,
                       w.color, w.rose, w.bw, w.size, w.minid, w.loop);
    GIS_LAUNCH_CHECK("k_scc_round");
    rc = to_fixed_point(w, 1, n_cells + 1, s, [&](uint32_t id) -> int32_t {
      hipLaunchKernelGGL(k_scc_color, dim3(gr), dim3(256), 0, s, row_ptr, col, n_rows, K,
                         (const uint8_t*)w.rem, w.color, w.rose, w.last, id);
      GIS_LAUNCH_CHECK("k_scc_color");
      return GIS_OK;
    });
    if (rc) return rc;
    hipLaunchKernelGGL(k_scc_roots, dim3(gc), dim3(256), 0, s, n_cells, (const uint8_t*)w.rem,
                       (const int32_t*)w.color, w.bw);
    GIS_LAUNCH_CHECK("k_scc_roots");
    rc = to_fixed_point(w, 2, n_cells + 1, s, [&](uint32_t id) -> int32_t {
      hipLaunchKernelGGL(k_scc_back, dim3(gr), dim3(256), 0, s, row_ptr, col, n_rows, K,
                         (const uint8_t*)w.rem, (const int32_t*)w.color, w.bw, w.last, id);
      GIS_LAUNCH_CHECK("k_scc_back");
      return GIS_OK;
    });
    if (rc) return rc;
    hipLaunchKernelGGL(k_scc_tally, dim3(gr), dim3(256), 0, s, row_ptr, col, n_rows, K,
                       (const int32_t*)w.color, (const uint8_t*)w.bw, w.size, w.minid, w.loop);
    GIS_LAUNCH_CHECK("k_scc_tally");
    hipLaunchKernelGGL(k_scc_pick, dim3(gc), dim3(256), 0, s, n_cells, jobs, n_jobs, w.rem,
                       (const int32_t*)w.color, (const uint8_t*)w.bw, (const int32_t*)w.size,
                       (const int32_t*)w.minid, (const uint8_t*)w.loop, w.comp, w.best);
    GIS_LAUNCH_CHECK("k_scc_pick");
    if ((rc = fill_u32((uint32_t*)w.left, 0u, 2 * (int64_t)n_jobs, s))) return rc;
    hipLaunchKernelGGL(k_scc_left, dim3(gc), dim3(256), 0, s, n_cells, jobs, n_jobs,
                       (const uint8_t*)w.rem, w.left);
    GIS_LAUNCH_CHECK("k_scc_left");
    GIS_HIP(hipMemcpyAsync(w.h_best, w.best, sizeof(unsigned long long) * 2 * n_jobs,
                           hipMemcpyDeviceToHost, s));  // best and left are adjacent
    GIS_HIP(hipStreamSynchronize(s));
    // a job is done when nothing is left or its best component is larger
    // than all that is left (an equally large one could hold a smaller id)
    bool done = true;
    for (int32_t j = 0; j < n_jobs; ++j) {
      const unsigned long long left = w.h_best[n_jobs + j];
      done = done && (left == 0 || (w.h_best[j] >> 32) > left);
    }
    if (done) break;
  }
  hipLaunchKernelGGL(k_scc_seed, dim3(gc), dim3(256), 0, s, n_cells, jobs, n_jobs,
                     (const int32_t*)w.comp, (const unsigned long long*)w.best, w.inset);
  GIS_LAUNCH_CHECK("k_scc_seed");
  rc = to_fixed_point(w, 3, n_cells + 1, s, [&](uint32_t id) -> int32_t {
    hipLaunchKernelGGL(k_scc_reach, dim3(gr), dim3(256), 0, s, row_ptr, col, n_rows, K, w.inset,
                       w.last, id);
    GIS_LAUNCH_CHECK("k_scc_reach");
    return GIS_OK;
  });
  if (rc) return rc;
  hipLaunchKernelGGL(k_scc_end, dim3(gc), dim3(256), 0, s, n_cells, (const uint8_t*)w.inset,
                     removed);
  GIS_LAUNCH_CHECK("k_scc_end");
  return GIS_OK;
}

}  // namespace gis
