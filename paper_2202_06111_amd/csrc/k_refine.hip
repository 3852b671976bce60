// Boundary selection and subdivision (Sec. 3.1.1, Algorithm 1, Remark 1).
//
// A kept cell is a boundary cell when one of its probes -- a finest-level
// cell adjacent to it -- lies outside X or is not covered by a kept cell.
// This is Algorithm 1 with the enlargement delta taken below one finest cell
// width: the vertices of the enlarged cell fall in the 2^n diagonal corner
// neighbours (rule CORNERS), and adding Remark 1's edge points makes the probe
// set every adjacent finest cell (rule SHELL).  Probes are answered by walking
// the covering index in which dropped cells were turned into holes.
//
// The next covering is produced without sorting: every surviving cell (or the
// 2^n children of a boundary cell) sets a flag in a dense per-level array laid
// out like the covering index; a scan of the flags in level-major, row-major
// order is exactly the canonical numbering of the new cell list.
#include "gis_launch.h"

namespace gis {

namespace {

// Is finest cell k covered by a kept cell?  (k inside the grid)  A leaf's
// ancestors are all REFINED, so k is covered exactly when one of its
// ancestor slots is a LEAF; the slots of four levels are read together
// (independent loads) instead of one level after the other.
template <int N>
__device__ __forceinline__ bool covered(const CoverIndex& ci, const int64_t* k) {
  for (int L0 = 0; L0 <= ci.lmax; L0 += 4) {
    uint8_t st[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int L = L0 + q;
      st[q] = ST_NONE;
      if (L <= ci.lmax) {
        const int s = ci.lmax - L;
        int64_t lin = 0;
#pragma unroll
        for (int d = 0; d < N; ++d) lin = lin * ci.dims[L][d] + (k[d] >> s);
        st[q] = ci.state[ci.off[L] + lin];
      }
    }
    bool leaf = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) leaf |= st[q] == ST_LEAF;
    if (leaf) return true;
  }
  return false;
}

// Number of probes of a kept cell whose finest-level box has side w - 2:
// CORNERS the 2^n diagonal neighbours, SHELL every cell of the surface of the
// box enlarged by one (w per side), split into 2n faces: face (d, side) has
// coordinate d on that side, the coordinates before d strictly inside and the
// ones after d anywhere, so no surface cell is counted twice.
template <int N>
__device__ __forceinline__ int64_t probe_count(int32_t rule, int64_t w) {
  if (rule == GIS_BOUNDARY_CORNERS) return (int64_t)1 << N;
  int64_t total = 0;
#pragma unroll
  for (int d = 0; d < N; ++d) {
    int64_t f = 2;
#pragma unroll
    for (int e = 0; e < N; ++e)
      if (e != d) f *= e < d ? w - 2 : w;
    total += f;
  }
  return total;
}

// Finest-level coordinates of probe p of the cell whose enlarged box is
// [lo, lo + w - 1] per dimension.
template <int N>
__device__ __forceinline__ void probe_coords(int32_t rule, const int64_t* lo, int64_t w, int64_t p,
                                             int64_t* k) {
  if (rule == GIS_BOUNDARY_CORNERS) {
#pragma unroll
    for (int d = 0; d < N; ++d) k[d] = lo[d] + (((p >> (N - 1 - d)) & 1) ? w - 1 : 0);
    return;
  }
#pragma unroll
  for (int d = 0; d < N; ++d) {
    int64_t f = 1;
#pragma unroll
    for (int e = 0; e < N; ++e)
      if (e != d) f *= e < d ? w - 2 : w;
    if (p < 2 * f) {
      const bool hi = p >= f;
      int64_t q = hi ? p - f : p;
      k[d] = lo[d] + (hi ? w - 1 : 0);
      const int first = d == 0 ? 1 : 0;  // the slowest remaining dimension takes the rest of q
#pragma unroll
      for (int e = N - 1; e >= 0; --e) {
        if (e == d) continue;
        const int64_t base = lo[e] + (e < d ? 1 : 0);
        if (e == first) {
          k[e] = base + q;
        } else {
          const int64_t r = e < d ? w - 2 : w;
          k[e] = base + q % r;
          q /= r;
        }
      }
      return;
    }
    p -= 2 * f;
  }
}

// A wave decides cpw = 64 / fan cells (lane i < cpw owns cell i of the
// wave), and the probes of those cells are shared out over all 64 lanes: a
// coarse cell next to finely refined ones has thousands of probes, a
// finest-level cell 3^n - 1.  Lane i takes probes i, i + 64, ... of the
// wave's concatenated probe list and skips the probes of cells already found
// to be boundary cells.  Each 256-cell block of the cell layout is split
// over fan launch blocks, so small coverings still fill the device.
template <int N>
__global__ __launch_bounds__(256) void k_boundary(BatchArgs b, const uint8_t* kept, int32_t rule,
                                                  uint8_t* boundary, JobStats* stats, int32_t fan,
                                                  bool flag_next) {
  __shared__ CoverIndex ci;
  __shared__ int64_t s_first[256];  // first probe of each thread's cell in its wave's list
  __shared__ int64_t s_lo[N][256];
  __shared__ int64_t s_w[256];
  __shared__ uint8_t s_bnd[256];
  const int64_t cb = blockIdx.x / fan;  // block of the cell layout
  const int32_t jb = job_of_block(b.jobs, b.n_jobs, LK_CELLS, cb);
  const Job& J = b.jobs[jb];
  stage_index(&ci, &J.ci);
  const int tid = threadIdx.x, lane = tid & 63, w0 = tid & ~63;
  const int cpw = 64 / fan;
  const int64_t c = (cb - J.blk[LK_CELLS]) * 256 + (blockIdx.x % fan) * (4 * cpw) + (tid >> 6) * cpw +
                    lane;
  const bool live = lane < cpw && c < J.n_cells;
  const int64_t gc = J.cell_off + c;
  const bool kp = live && kept[gc] != 0;
  int64_t np = 0;
  if (kp) {
    const int s = ci.lmax - b.level[gc];
    const int64_t w = ((int64_t)1 << s) + 2;
#pragma unroll
    for (int d = 0; d < N; ++d) s_lo[d][tid] = ((int64_t)b.idx[gc * N + d] << s) - 1;
    s_w[tid] = w;
    np = probe_count<N>(rule, w);
  }
  // exclusive scan of the probe counts over the wave
  int64_t incl = np;
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  const int64_t total = __shfl(incl, 63, 64);
  s_first[tid] = incl - np;
  s_bnd[tid] = 0;
  __syncthreads();
  int64_t Nf[N];
#pragma unroll
  for (int d = 0; d < N; ++d) Nf[d] = ci.dims[ci.lmax][d];
  for (int64_t i = lane; i < total; i += 64) {
    // owner: the last lane of the wave whose first probe is <= i
    int lo_l = 0, hi_l = 63;
    while (lo_l < hi_l) {
      const int mid = (lo_l + hi_l + 1) >> 1;
      if (s_first[w0 + mid] <= i) lo_l = mid; else hi_l = mid - 1;
    }
    const int o = w0 + lo_l;
    if (s_bnd[o]) continue;
    int64_t lo[N], k[N];
#pragma unroll
    for (int d = 0; d < N; ++d) lo[d] = s_lo[d][o];
    probe_coords<N>(rule, lo, s_w[o], i - s_first[o], k);
    bool outside = false;
#pragma unroll
    for (int d = 0; d < N; ++d) outside |= k[d] < 0 || k[d] >= Nf[d];
    if (outside || !covered<N>(ci, k)) s_bnd[o] = 1;
  }
  __syncthreads();
  const bool bnd = kp && s_bnd[tid] != 0;
  if (live) {
    boundary[gc] = bnd ? 1 : 0;
    // the next covering: the cell itself, or its 2^n children if it is a
    // boundary cell (jobs that stopped have no flag array)
    const CoverIndex& next = J.next;
    if (flag_next && kept[gc] && next.state) {
      const int L = b.level[gc];
      if (!bnd) {
        int64_t lin = 0;
#pragma unroll
        for (int d = 0; d < N; ++d) lin = lin * next.dims[L][d] + b.idx[gc * N + d];
        next.state[next.off[L] + lin] = 1;
      } else {
        for (int ch = 0; ch < (1 << N); ++ch) {
          int64_t lin = 0;
#pragma unroll
          for (int d = 0; d < N; ++d)
            lin = lin * next.dims[L + 1][d] +
                  (2 * (int64_t)b.idx[gc * N + d] + ((ch >> (N - 1 - d)) & 1));
          next.state[next.off[L + 1] + lin] = 1;
        }
      }
    }
  }
  const uint64_t m = __ballot(bnd);  // one atomic per wave (blocks never straddle jobs)
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(&stats[jb].n_boundary, (unsigned long long)__popcll(m));
}

// Neighbourhood of the boundary cells (Sec. 3.1.2): the nn kept cells whose
// centres lie nearest to a boundary cell's centre (Euclidean distance in
// state units, the cell itself not counted, equal distances ordered by cell
// id) are selected for subdivision with it.  sel is zero on entry; every
// boundary cell and each of its neighbours get sel = 1 (plain stores of 1:
// no race matters).
//
// A wave takes one boundary cell at a time and keeps its best nn candidates
// sorted across its lanes (lane l holds rank l).  Candidates are the kept
// cells meeting a box of finest-level cells around the cell, enumerated slot
// by slot in the covering index (every kept cell is the LEAF slot of its own
// level, so each is met once).  Every cell whose centre lies within distance
// D of the cell's centre meets the box, D being the distance from the centre
// to the nearest side of the box that is not a side of X; when the nn-th
// candidate lies within D the list is final, otherwise the box grows.
// Distances: centre offsets are integers on the grid of half the finest
// width, scaled by that width, squared and summed dimension by dimension in
// FP64 (the same operations in the same order for every pair).
template <int N>
__global__ __launch_bounds__(256) void k_neighbours(BatchArgs b, const uint8_t* kept,
                                                    const uint8_t* boundary, int32_t nn,
                                                    uint8_t* sel) {
  __shared__ CoverIndex ci;
  const int32_t jb = job_of_block(b.jobs, b.n_jobs, LK_CELLS, blockIdx.x);
  const Job& J = b.jobs[jb];
  stage_index(&ci, &J.ci);
  const int lane = threadIdx.x & 63;
  const int64_t c0 = (blockIdx.x - J.blk[LK_CELLS]) * 256 + (threadIdx.x & ~63);
  const int64_t mine = c0 + lane;
  const bool isb = mine < J.n_cells && kept[J.cell_off + mine] && boundary[J.cell_off + mine];
  uint64_t todo = __ballot(isb);
  const int lmax = ci.lmax;
  double hw[N];
  int64_t Nf[N];
#pragma unroll
  for (int d = 0; d < N; ++d) {
    hw[d] = ldexp(J.grid.w0[d], -(lmax + 1));
    Nf[d] = ci.dims[lmax][d];
  }
  const double kInf = INFINITY;
  while (todo) {
    const int src = __builtin_ctzll(todo);
    todo &= todo - 1;
    const int64_t gb = J.cell_off + c0 + src;
    const int Lb = b.level[gb];
    const int sb = lmax - Lb;
    int64_t ib[N], cb[N];  // index, centre on the half-finest grid
#pragma unroll
    for (int d = 0; d < N; ++d) {
      ib[d] = b.idx[gb * N + d];
      cb[d] = (2 * ib[d] + 1) << sb;
    }
    if (lane == 0) sel[gb] = 1;
    double md2 = kInf;    // this lane's rank in the candidate list
    int64_t mid = -1;
    for (int64_t r = 1;; r = 2 * r + 1) {
      md2 = kInf;
      mid = -1;
      int64_t lo[N], hi[N];
      bool all_clipped = true;
      double dlim = kInf;  // squared distance within which every centre is in the box
#pragma unroll
      for (int d = 0; d < N; ++d) {
        const int64_t l0 = (ib[d] << sb) - r, h0 = ((ib[d] + 1) << sb) - 1 + r;
        lo[d] = l0 < 0 ? 0 : l0;
        hi[d] = h0 > Nf[d] - 1 ? Nf[d] - 1 : h0;
        if (l0 >= 0) {
          const double t = (double)(cb[d] - 2 * lo[d]) * hw[d];
          dlim = t * t < dlim ? t * t : dlim;
        }
        if (h0 <= Nf[d] - 1) {
          const double t = (double)(2 * (hi[d] + 1) - cb[d]) * hw[d];
          dlim = t * t < dlim ? t * t : dlim;
        }
        all_clipped &= l0 < 0 && h0 > Nf[d] - 1;
      }
      for (int L = 0; L <= lmax; ++L) {
        const int s = lmax - L;
        int64_t blo[N], ext[N], count = 1;
#pragma unroll
        for (int d = 0; d < N; ++d) {
          blo[d] = lo[d] >> s;
          ext[d] = (hi[d] >> s) - blo[d] + 1;
          count *= ext[d];
        }
        for (int64_t k0 = 0; k0 < count; k0 += 64) {
          const int64_t k = k0 + lane;
          bool valid = false;
          double d2 = kInf;
          int64_t id = -1;
          if (k < count) {
            int64_t rem = k, kk[N];
#pragma unroll
            for (int d = N - 1; d >= 0; --d) {
              kk[d] = blo[d] + rem % ext[d];
              rem /= ext[d];
            }
            int64_t lin = 0;
#pragma unroll
            for (int d = 0; d < N; ++d) lin = lin * ci.dims[L][d] + kk[d];
            // a kept cell: a LEAF slot of the index (removed cells are
            // holes), or, on a full level-0 grid without index arrays, a
            // cell whose kept flag is set
            bool leaf;
            if (ci.uniform) {
              id = J.cell_off + lin;
              leaf = kept[id] != 0;
            } else {
              const int64_t slot = ci.off[L] + lin;
              leaf = ci.state[slot] == ST_LEAF;
              id = J.cell_off + (int64_t)((uint64_t)ci.pfx[slot] & 0xffffffffull) - ci.pbase;
            }
            if (leaf) {
              if (id != gb) {
                valid = true;
                d2 = 0.0;
#pragma unroll
                for (int d = 0; d < N; ++d) {
                  const double t = (double)(((2 * kk[d] + 1) << s) - cb[d]) * hw[d];
                  d2 = d2 + t * t;
                }
              }
            }
          }
          // insert the lanes' candidates one by one (wave-uniform loop)
          for (uint64_t cand = __ballot(valid); cand; cand &= cand - 1) {
            const int q = __builtin_ctzll(cand);
            const double cd = __shfl(d2, q, 64);
            const int64_t cid = __shfl(id, q, 64);
            const bool less = lane < nn && (md2 < cd || (md2 == cd && mid < cid && mid >= 0));
            const int pos = __popcll(__ballot(less));
            if (pos < nn) {
              const double up_d = __shfl_up(md2, 1, 64);
              const int64_t up_i = __shfl_up(mid, 1, 64);
              if (lane > pos && lane < nn) {
                md2 = up_d;
                mid = up_i;
              } else if (lane == pos) {
                md2 = cd;
                mid = cid;
              }
            }
          }
        }
      }
      // done when the list is full and its last entry lies within dlim, or
      // the box already spans the whole grid
      const double last = __shfl(md2, nn - 1, 64);
      const int64_t last_id = __shfl(mid, nn - 1, 64);
      if (all_clipped || (last_id >= 0 && last <= dlim)) break;
    }
    if (lane < nn && mid >= 0) sel[mid] = 1;
  }
}

// Next-covering flags from the selection: a selected kept cell sets the
// flags of its 2^n children, any other kept cell its own; stats[j].n_selected
// counts the selected cells.
template <int N>
__global__ __launch_bounds__(256) void k_mark_next(BatchArgs b, const uint8_t* kept,
                                                   const uint8_t* sel, JobStats* stats) {
  const int32_t jb = job_of_block(b.jobs, b.n_jobs, LK_CELLS, blockIdx.x);
  const Job& J = b.jobs[jb];
  const int64_t c = (blockIdx.x - J.blk[LK_CELLS]) * 256 + threadIdx.x;
  const int64_t gc = J.cell_off + c;
  const bool live = c < J.n_cells && kept[gc];
  const uint64_t m = __ballot(live && sel[gc]);  // one atomic per wave (blocks never straddle jobs)
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(&stats[jb].n_selected, (unsigned long long)__popcll(m));
  const CoverIndex& next = J.next;
  if (!live || !next.state) return;
  const int L = b.level[gc];
  if (!sel[gc]) {
    int64_t lin = 0;
#pragma unroll
    for (int d = 0; d < N; ++d) lin = lin * next.dims[L][d] + b.idx[gc * N + d];
    next.state[next.off[L] + lin] = 1;
    return;
  }
  for (int ch = 0; ch < (1 << N); ++ch) {
    int64_t lin = 0;
#pragma unroll
    for (int d = 0; d < N; ++d)
      lin = lin * next.dims[L + 1][d] + (2 * (int64_t)b.idx[gc * N + d] + ((ch >> (N - 1 - d)) & 1));
    next.state[next.off[L + 1] + lin] = 1;
  }
}

// Standard subdivision (Sec. 2.1): every kept cell of a level-0 covering is
// halved across dimension `dim`.  The halves are level-0 cells of the grid
// on which the next covering's flag array is laid out (the current grid with
// twice the cells along `dim`); each sets its flag there, and the scan of the
// flags numbers them canonically, as for the adaptive subdivision.  A kept
// cell not of level 0 or outside the grid sets no flag and is counted in
// *err (when err is given).
__global__ void k_bisect(BatchArgs b, const uint8_t* kept, int32_t dim, uint8_t* split,
                         JobStats* stats, uint32_t* err) {
  const int32_t jb = job_of_block(b.jobs, b.n_jobs, LK_CELLS, blockIdx.x);
  const Job& J = b.jobs[jb];
  const int64_t c = (blockIdx.x - J.blk[LK_CELLS]) * blockDim.x + threadIdx.x;
  const bool live = c < J.n_cells;
  const int64_t gc = J.cell_off + c;
  bool cut = live && kept[gc] != 0;
  if (cut) {
    const CoverIndex& next = J.next;
    bool ok = b.level[gc] == 0;
    int64_t lin = 0, stride = 1;
    for (int d = 0; d < b.n; ++d) {
      const int64_t halves = d == dim ? 2 : 1;
      const int64_t k = (int64_t)b.idx[gc * b.n + d] * halves;
      ok = ok && k >= 0 && k + halves - 1 < next.dims[0][d];
      lin = lin * next.dims[0][d] + k;
      if (d > dim) stride *= next.dims[0][d];
    }
    if (ok && next.state) {
      next.state[next.off[0] + lin] = 1;           // lower half
      next.state[next.off[0] + lin + stride] = 1;  // upper half
    }
    if (!ok) {
      if (err) atomicAdd(err, 1u);
      cut = false;
    }
  }
  if (live) split[gc] = cut ? 1 : 0;
  const uint64_t m = __ballot(cut);  // one atomic per wave (blocks never straddle jobs)
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(&stats[jb].n_boundary, (unsigned long long)__popcll(m));
}

// pos: exclusive scan of the batch's flag array (jobs' arrays back to back).
// Clears every flag it consumes, so the array is zero for the next call.
// Also records each job's first new cell and the new cells before each of
// its levels (from the threads at the first slot of the job and of each level).
__global__ void k_compact(BatchArgs b, const int64_t* pos, int64_t cap, uint8_t* level_out,
                          int32_t* idx_out, JobStats* stats) {
  const int32_t jb = job_of_block(b.jobs, b.n_jobs, LK_NEXT, blockIdx.x);
  const Job& J = b.jobs[jb];
  const CoverIndex& next = J.next;
  const int64_t sl = (blockIdx.x - J.blk[LK_NEXT]) * blockDim.x + threadIdx.x;
  if (!next.state || sl >= next.off[next.lmax + 1]) return;
  int L = 0;
  while (sl >= next.off[L + 1]) ++L;
  if (sl == next.off[L]) {
    stats[jb].level_start[L] = pos[J.next_off + sl];
    if (L == 0) stats[jb].next_start = pos[J.next_off + sl];
  }
  if (!next.state[sl]) return;
  next.state[sl] = 0;
  const int64_t p = pos[J.next_off + sl];
  if (p >= cap) return;
  int64_t rem = sl - next.off[L];
  level_out[p] = (uint8_t)L;
  for (int d = next.n - 1; d >= 0; --d) {
    idx_out[p * next.n + d] = (int32_t)(rem % next.dims[L][d]);
    rem /= next.dims[L][d];
  }
}

__global__ void k_coarse(BatchArgs b, uint8_t* level, int32_t* idx) {
  const int32_t jb = job_of_block(b.jobs, b.n_jobs, LK_CELLS, blockIdx.x);
  const Job& J = b.jobs[jb];
  const int64_t c = (blockIdx.x - J.blk[LK_CELLS]) * blockDim.x + threadIdx.x;
  if (c >= J.n_cells) return;
  const int64_t gc = J.cell_off + c;
  int64_t rem = c;
  level[gc] = 0;
  for (int d = J.grid.n - 1; d >= 0; --d) {
    idx[gc * J.grid.n + d] = (int32_t)(rem % J.grid.n0[d]);
    rem /= J.grid.n0[d];
  }
}

__global__ void k_count_kept(BatchArgs b, const uint8_t* kept, JobStats* stats) {
  const int32_t jb = job_of_block(b.jobs, b.n_jobs, LK_CELLS, blockIdx.x);
  const Job& J = b.jobs[jb];
  const int64_t c = (blockIdx.x - J.blk[LK_CELLS]) * blockDim.x + threadIdx.x;
  // one atomic per wave (a block never straddles two jobs)
  const uint64_t m = __ballot(c < J.n_cells && kept[J.cell_off + c]);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(&stats[jb].n_kept, (unsigned long long)__popcll(m));
}

__global__ void k_count_kept_cells(const Job* jobs, int32_t n_jobs, int64_t n_cells,
                                   const uint8_t* kept, JobStats* stats) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells;
       c += (int64_t)gridDim.x * blockDim.x)
    if (kept[c]) atomicAdd(&stats[job_of_cell(jobs, n_jobs, c)].n_kept, 1ull);
}

__global__ void k_clear_kept(JobStats* stats, int32_t n_jobs) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n_jobs) stats[j].n_kept = 0;
}

}  // namespace

int32_t batch_clear_kept(JobStats* stats, int32_t n_jobs, hipStream_t s) {
  if (n_jobs <= 0) return GIS_OK;
  hipLaunchKernelGGL(k_clear_kept, dim3((unsigned)((n_jobs + 255) / 256)), dim3(256), 0, s, stats,
                     n_jobs);
  GIS_LAUNCH_CHECK("k_clear_kept");
  return GIS_OK;
}

int32_t batch_count_kept_cells(const Job* jobs, int32_t n_jobs, int64_t n_cells,
                               const uint8_t* kept, JobStats* stats, hipStream_t s) {
  if (n_cells == 0) return GIS_OK;
  int64_t nb = (n_cells + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_count_kept_cells, dim3((unsigned)nb), dim3(256), 0, s, jobs, n_jobs, n_cells,
                     kept, stats);
  GIS_LAUNCH_CHECK("k_count_kept_cells");
  return GIS_OK;
}

#define GIS_DIM_SWITCH(N_, CALL)                                   \
  switch (N_) {                                                    \
    case 1: CALL(1); break;                                        \
    case 2: CALL(2); break;                                        \
    case 3: CALL(3); break;                                        \
    case 4: CALL(4); break;                                        \
    default: set_error("unsupported dimension"); return GIS_E_UNSUPPORTED; \
  }

int32_t batch_boundary(const BatchArgs& b, const uint8_t* kept, int32_t rule, uint8_t* boundary,
                       JobStats* stats, hipStream_t s, bool flag_next) {
  if (b.blocks[LK_CELLS] == 0) return GIS_OK;
  // lanes per cell: enough waves for about four per SIMD (1024 SIMDs)
  int32_t fan = 1;
  while (fan < 16 && b.blocks[LK_CELLS] * 4 * fan < 4096) fan *= 2;
#define GIS_CALL(N) hipLaunchKernelGGL(k_boundary<N>, dim3((unsigned)(b.blocks[LK_CELLS] * fan)), dim3(256), 0, s, b, kept, rule, boundary, stats, fan, flag_next)
  GIS_DIM_SWITCH(b.n, GIS_CALL)
#undef GIS_CALL
  GIS_LAUNCH_CHECK("k_boundary");
  return GIS_OK;
}

int32_t batch_neighbours(const BatchArgs& b, const uint8_t* kept, const uint8_t* boundary,
                         int32_t nn, uint8_t* sel, JobStats* stats, hipStream_t s) {
  if (b.blocks[LK_CELLS] == 0) return GIS_OK;
  if (nn < 1 || nn > 64) {
    set_error("neighbourhood size must be 1..64");
    return GIS_E_UNSUPPORTED;
  }
#define GIS_CALL(N) hipLaunchKernelGGL(k_neighbours<N>, dim3((unsigned)b.blocks[LK_CELLS]), dim3(256), 0, s, b, kept, boundary, nn, sel)
  GIS_DIM_SWITCH(b.n, GIS_CALL)
#undef GIS_CALL
  GIS_LAUNCH_CHECK("k_neighbours");
#define GIS_CALL(N) hipLaunchKernelGGL(k_mark_next<N>, dim3((unsigned)b.blocks[LK_CELLS]), dim3(256), 0, s, b, kept, sel, stats)
  GIS_DIM_SWITCH(b.n, GIS_CALL)
#undef GIS_CALL
  GIS_LAUNCH_CHECK("k_mark_next");
  return GIS_OK;
}

int32_t batch_bisect(const BatchArgs& b, const uint8_t* kept, int32_t dim, uint8_t* split,
                     JobStats* stats, uint32_t* err, hipStream_t s) {
  if (b.blocks[LK_CELLS] == 0) return GIS_OK;
  hipLaunchKernelGGL(k_bisect, dim3((unsigned)b.blocks[LK_CELLS]), dim3(256), 0, s, b, kept, dim,
                     split, stats, err);
  GIS_LAUNCH_CHECK("k_bisect");
  return GIS_OK;
}

int32_t batch_compact(const BatchArgs& b, const int64_t* pos, int64_t cap, uint8_t* level_out,
                      int32_t* idx_out, JobStats* stats, hipStream_t s) {
  if (b.blocks[LK_NEXT] > 0) {
    hipLaunchKernelGGL(k_compact, dim3((unsigned)b.blocks[LK_NEXT]), dim3(256), 0, s, b, pos, cap,
                       level_out, idx_out, stats);
    GIS_LAUNCH_CHECK("k_compact");
  }
  return GIS_OK;
}

int32_t batch_coarse(const BatchArgs& b, uint8_t* level, int32_t* idx, hipStream_t s) {
  if (b.blocks[LK_CELLS] == 0) return GIS_OK;
  hipLaunchKernelGGL(k_coarse, dim3((unsigned)b.blocks[LK_CELLS]), dim3(256), 0, s, b, level, idx);
  GIS_LAUNCH_CHECK("k_coarse");
  return GIS_OK;
}

int32_t batch_count_kept(const BatchArgs& b, const uint8_t* kept, JobStats* stats, hipStream_t s) {
  if (b.blocks[LK_CELLS] == 0) return GIS_OK;
  hipLaunchKernelGGL(k_count_kept, dim3((unsigned)b.blocks[LK_CELLS]), dim3(256), 0, s, b, kept,
                     stats);
  GIS_LAUNCH_CHECK("k_count_kept");
  return GIS_OK;
}

}  // namespace gis
