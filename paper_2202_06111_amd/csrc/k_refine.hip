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
#include "gis_internal.h"

namespace gis {

namespace {

inline unsigned grid_for(int64_t n) {
  int64_t nb = (n + 255) / 256;
  if (nb < 1) nb = 1;
  if (nb > 8192) nb = 8192;
  return (unsigned)nb;
}

// Is finest cell k covered by a kept cell?  (k inside the grid)
template <int N>
__device__ __forceinline__ bool covered(const CoverIndex& ci, const int64_t* k) {
  for (int L = 0; L <= ci.lmax; ++L) {
    const int s = ci.lmax - L;
    int64_t lin = 0;
#pragma unroll
    for (int d = 0; d < N; ++d) lin = lin * ci.dims[L][d] + (k[d] >> s);
    const uint8_t st = ci.state[ci.off[L] + lin];
    if (st == ST_LEAF) return true;
    if (st != ST_REFINED) return false;
  }
  return false;
}

template <int N>
__global__ void k_boundary(CoverIndex ci, const uint8_t* level, const int32_t* idx,
                           int64_t n_cells, const uint8_t* kept, int32_t rule, uint8_t* boundary) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells;
       c += (int64_t)gridDim.x * blockDim.x) {
    if (!kept[c]) {
      boundary[c] = 0;
      continue;
    }
    const int s = ci.lmax - level[c];
    int64_t lo[N], hi[N], k[N], Nf[N];
#pragma unroll
    for (int d = 0; d < N; ++d) {
      lo[d] = ((int64_t)idx[c * N + d] << s) - 1;
      hi[d] = ((int64_t)idx[c * N + d] + 1) << s;
      k[d] = lo[d];
      Nf[d] = ci.dims[ci.lmax][d];
    }
    bool bnd = false;
    if (rule == GIS_BOUNDARY_CORNERS) {
      for (int q = 0; q < (1 << N) && !bnd; ++q) {
        bool outside = false;
#pragma unroll
        for (int d = 0; d < N; ++d) {
          k[d] = ((q >> (N - 1 - d)) & 1) ? hi[d] : lo[d];
          outside |= k[d] < 0 || k[d] >= Nf[d];
        }
        bnd = outside || !covered<N>(ci, k);
      }
    } else {
      // every cell of the box [lo, hi] that is on its surface; the interior of
      // the last dimension is skipped when all other coordinates are inside
      for (;;) {
        bool outside = false, inner = true;
#pragma unroll
        for (int d = 0; d < N; ++d) {
          outside |= k[d] < 0 || k[d] >= Nf[d];
          if (d < N - 1) inner &= k[d] != lo[d] && k[d] != hi[d];
        }
        if (outside || !covered<N>(ci, k)) {
          bnd = true;
          break;
        }
        if (inner && k[N - 1] == lo[N - 1]) {
          k[N - 1] = hi[N - 1];
          continue;
        }
        int d = N - 1;
        while (d >= 0 && k[d] == hi[d]) {
          k[d] = lo[d];
          --d;
        }
        if (d < 0) break;
        ++k[d];
      }
    }
    boundary[c] = bnd ? 1 : 0;
  }
}

template <int N>
__global__ void k_next_flags(CoverIndex next, const uint8_t* level, const int32_t* idx,
                             int64_t n_cells, const uint8_t* kept, const uint8_t* boundary) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells;
       c += (int64_t)gridDim.x * blockDim.x) {
    if (!kept[c]) continue;
    const int L = level[c];
    if (!boundary[c]) {
      int64_t lin = 0;
#pragma unroll
      for (int d = 0; d < N; ++d) lin = lin * next.dims[L][d] + idx[c * N + d];
      next.state[next.off[L] + lin] = 1;
      continue;
    }
    for (int ch = 0; ch < (1 << N); ++ch) {
      int64_t lin = 0;
#pragma unroll
      for (int d = 0; d < N; ++d)
        lin = lin * next.dims[L + 1][d] + (2 * (int64_t)idx[c * N + d] + ((ch >> (N - 1 - d)) & 1));
      next.state[next.off[L + 1] + lin] = 1;
    }
  }
}

__global__ void k_compact(CoverIndex next, const int64_t* pos, int64_t cap, uint8_t* level_out,
                          int32_t* idx_out) {
  const int64_t total = next.off[next.lmax + 1];
  for (int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; sl < total;
       sl += (int64_t)gridDim.x * blockDim.x) {
    if (!next.state[sl]) continue;
    const int64_t p = pos[sl];
    if (p >= cap) continue;
    int L = 0;
    while (sl >= next.off[L + 1]) ++L;
    int64_t rem = sl - next.off[L];
    level_out[p] = (uint8_t)L;
    for (int d = next.n - 1; d >= 0; --d) {
      idx_out[p * next.n + d] = (int32_t)(rem % next.dims[L][d]);
      rem /= next.dims[L][d];
    }
  }
}

__global__ void k_level_starts(CoverIndex next, const int64_t* pos, int64_t* out) {
  const int L = threadIdx.x;
  if (L <= next.lmax) out[L] = pos[next.off[L]];
}

__global__ void k_coarse(GridArgs g, int64_t total, uint8_t* level, int32_t* idx) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < total;
       c += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = c;
    level[c] = 0;
    for (int d = g.n - 1; d >= 0; --d) {
      idx[c * g.n + d] = (int32_t)(rem % g.n0[d]);
      rem /= g.n0[d];
    }
  }
}

}  // namespace

int32_t launch_boundary(const CoverIndex& ci, const GridArgs& g, const uint8_t* level,
                        const int32_t* idx, int64_t n_cells, const uint8_t* kept, int32_t rule,
                        uint8_t* boundary, hipStream_t s) {
  (void)g;
  if (n_cells == 0) return GIS_OK;
  switch (ci.n) {
    case 1: hipLaunchKernelGGL(k_boundary<1>, dim3(grid_for(n_cells)), dim3(256), 0, s, ci, level, idx, n_cells, kept, rule, boundary); break;
    case 2: hipLaunchKernelGGL(k_boundary<2>, dim3(grid_for(n_cells)), dim3(256), 0, s, ci, level, idx, n_cells, kept, rule, boundary); break;
    case 3: hipLaunchKernelGGL(k_boundary<3>, dim3(grid_for(n_cells)), dim3(256), 0, s, ci, level, idx, n_cells, kept, rule, boundary); break;
    case 4: hipLaunchKernelGGL(k_boundary<4>, dim3(grid_for(n_cells)), dim3(256), 0, s, ci, level, idx, n_cells, kept, rule, boundary); break;
    default: set_error("unsupported dimension"); return GIS_E_UNSUPPORTED;
  }
  GIS_LAUNCH_CHECK("k_boundary");
  return GIS_OK;
}

int32_t launch_next_flags(const CoverIndex& next, const uint8_t* level, const int32_t* idx,
                          int64_t n_cells, const uint8_t* kept, const uint8_t* boundary,
                          hipStream_t s) {
  int32_t rc = fill_u8(next.state, 0, next.off[next.lmax + 1], s);
  if (rc != GIS_OK || n_cells == 0) return rc;
  switch (next.n) {
    case 1: hipLaunchKernelGGL(k_next_flags<1>, dim3(grid_for(n_cells)), dim3(256), 0, s, next, level, idx, n_cells, kept, boundary); break;
    case 2: hipLaunchKernelGGL(k_next_flags<2>, dim3(grid_for(n_cells)), dim3(256), 0, s, next, level, idx, n_cells, kept, boundary); break;
    case 3: hipLaunchKernelGGL(k_next_flags<3>, dim3(grid_for(n_cells)), dim3(256), 0, s, next, level, idx, n_cells, kept, boundary); break;
    case 4: hipLaunchKernelGGL(k_next_flags<4>, dim3(grid_for(n_cells)), dim3(256), 0, s, next, level, idx, n_cells, kept, boundary); break;
    default: set_error("unsupported dimension"); return GIS_E_UNSUPPORTED;
  }
  GIS_LAUNCH_CHECK("k_next_flags");
  return GIS_OK;
}

int32_t launch_compact(const CoverIndex& next, const int64_t* pos, int64_t cap, uint8_t* level_out,
                       int32_t* idx_out, hipStream_t s) {
  const int64_t total = next.off[next.lmax + 1];
  if (total == 0) return GIS_OK;
  hipLaunchKernelGGL(k_compact, dim3(grid_for(total)), dim3(256), 0, s, next, pos, cap, level_out,
                     idx_out);
  GIS_LAUNCH_CHECK("k_compact");
  return GIS_OK;
}

int32_t launch_level_starts(const CoverIndex& next, const int64_t* pos, int64_t* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_level_starts, dim3(1), dim3(64), 0, s, next, pos, out);
  GIS_LAUNCH_CHECK("k_level_starts");
  return GIS_OK;
}

int32_t launch_coarse(const GridArgs& g, uint8_t* level, int32_t* idx, hipStream_t s) {
  int64_t total = 1;
  for (int d = 0; d < g.n; ++d) total *= g.n0[d];
  hipLaunchKernelGGL(k_coarse, dim3(grid_for(total)), dim3(256), 0, s, g, total, level, idx);
  GIS_LAUNCH_CHECK("k_coarse");
  return GIS_OK;
}

}  // namespace gis
