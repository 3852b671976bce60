// Covering index: the cells of a covering (Sec. 2.1) held as one dense
// row-major state array per level -- LEAF where a cell of the list sits,
// REFINED above a leaf, HOLE where a region of X has no cell, NONE below a
// leaf or a hole -- plus prefix counts of leaves and holes in slot order.
// Since the slot order (level, then row-major) is the canonical cell order,
// the leaves of any run of slots along the last dimension are cells with
// consecutive ids, and two prefix values give a run's leaves and holes.  This
// turns "which cells meet this box" into a few loads per row of the box and
// level, and "is this finest cell covered" into a walk over at most lmax + 1
// levels, with no search structure to build (the role the paper gives an
// R*-tree, Sec. 2.4).
#include "gis_launch.h"

namespace gis {

namespace {

template <typename T>
__global__ void k_fill(T* p, T v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename T>
int32_t fill(T* p, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return GIS_OK;
  int64_t nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL((k_fill<T>), dim3((unsigned)nb), dim3(256), 0, s, p, v, n);
  GIS_LAUNCH_CHECK("k_fill");
  return GIS_OK;
}

// Copies `words` 32-bit words from device memory to host-coherent pinned
// memory, then publishes seq in the host flag (after a system-scope fence):
// a host spinning on the flag sees the words once it sees seq.
__global__ void k_publish(const uint32_t* src, uint32_t* dst, int32_t words, uint32_t* flag,
                          uint32_t seq) {
  for (int32_t i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence_system();
    __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

__global__ void k_zero_ranges(ZeroRanges z) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int r = 0; r < z.n; ++r)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < z.words[r]; i += stride)
      z.p[r][i] = 0u;
}

// Segment blockIdx.y of a gather, copied in the widest unit that both of its
// addresses allow.
template <typename T>
__device__ __forceinline__ void copy_units(const uint8_t* src, uint8_t* dst, int64_t bytes) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nu = bytes / (int64_t)sizeof(T);
  for (int64_t i = t; i < nu; i += stride) ((T*)dst)[i] = ((const T*)src)[i];
  for (int64_t i = nu * (int64_t)sizeof(T) + t; i < bytes; i += stride) dst[i] = src[i];
}

__global__ void k_gather(Gather g) {
  const int k = blockIdx.y;
  if (k >= g.n) return;
  const uint8_t* src = g.src[k];
  uint8_t* dst = g.dst[k];
  const uintptr_t al = (uintptr_t)src | (uintptr_t)dst;
  if ((al & 15) == 0) copy_units<uint4>(src, dst, g.bytes[k]);
  else if ((al & 7) == 0) copy_units<uint64_t>(src, dst, g.bytes[k]);
  else if ((al & 3) == 0) copy_units<uint32_t>(src, dst, g.bytes[k]);
  else copy_units<uint8_t>(src, dst, g.bytes[k]);
}

__global__ void k_max_level(const uint8_t* level, int64_t n, uint32_t* out) {
  uint32_t m = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m = level[i] > m ? level[i] : m;
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t w = __shfl_down(m, o, 64);
    m = w > m ? w : m;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

// Range and canonical-order checks; LEAF entries for jobs with index arrays.
__global__ void k_leaves(BatchArgs b, uint32_t* err) {
  const int32_t jb = job_of_block(b.jobs, b.n_jobs, LK_CELLS, blockIdx.x);
  const Job& J = b.jobs[jb];
  const int64_t c = (blockIdx.x - J.blk[LK_CELLS]) * blockDim.x + threadIdx.x;
  if (c >= J.n_cells) return;
  const int64_t gc = J.cell_off + c;
  const int64_t slot = cell_slot(J.ci, b.level, b.idx, gc);
  if (slot < 0) {
    atomicOr(err, 1u);
    return;
  }
  if (c > 0) {
    // canonical order = strictly increasing (level, row-major index) = slot order
    const int64_t pslot = cell_slot(J.ci, b.level, b.idx, gc - 1);
    if (pslot >= 0 && pslot >= slot) atomicOr(err, 2u);
  }
  if (!J.ci.uniform) J.ci.state[slot] = ST_LEAF;
}

// Marks every ancestor of every leaf REFINED; an ancestor that is itself a
// leaf means two cells overlap.
__global__ void k_ancestors(BatchArgs b, uint32_t* err) {
  const int32_t jb = job_of_block(b.jobs, b.n_jobs, LK_CELLS, blockIdx.x);
  const Job& J = b.jobs[jb];
  const int64_t c = (blockIdx.x - J.blk[LK_CELLS]) * blockDim.x + threadIdx.x;
  if (c >= J.n_cells || J.ci.uniform) return;
  const int64_t gc = J.cell_off + c;
  if (cell_slot(J.ci, b.level, b.idx, gc) < 0) return;  // reported by k_leaves
  int L = b.level[gc];
  int64_t k[kMaxDim];
  for (int d = 0; d < J.ci.n; ++d) k[d] = b.idx[gc * J.ci.n + d];
  while (L > 0) {
    --L;
    int64_t lin = 0;
    for (int d = 0; d < J.ci.n; ++d) {
      k[d] >>= 1;
      lin = lin * J.ci.dims[L][d] + k[d];
    }
    const int64_t slot = J.ci.off[L] + lin;
    if (J.ci.state[slot] == ST_LEAF) {
      atomicOr(err, 4u);
      break;
    }
    J.ci.state[slot] = ST_REFINED;
  }
}

// For lists known to be valid (the library's own): LEAF for every cell and
// REFINED for its ancestors in one pass, no checks.  Cells sharing an
// ancestor write the same value; a valid list has no cell inside another.
__global__ void k_leaves_up(BatchArgs b) {
  const int32_t jb = job_of_block(b.jobs, b.n_jobs, LK_CELLS, blockIdx.x);
  const Job& J = b.jobs[jb];
  const int64_t c = (blockIdx.x - J.blk[LK_CELLS]) * blockDim.x + threadIdx.x;
  if (c >= J.n_cells || J.ci.uniform) return;
  const int64_t gc = J.cell_off + c;
  int L = b.level[gc];
  int64_t k[kMaxDim];
  int64_t lin = 0;
  for (int d = 0; d < J.ci.n; ++d) {
    k[d] = b.idx[gc * J.ci.n + d];
    lin = lin * J.ci.dims[L][d] + k[d];
  }
  J.ci.state[J.ci.off[L] + lin] = ST_LEAF;
  while (L > 0) {
    --L;
    lin = 0;
    for (int d = 0; d < J.ci.n; ++d) {
      k[d] >>= 1;
      lin = lin * J.ci.dims[L][d] + k[d];
    }
    J.ci.state[J.ci.off[L] + lin] = ST_REFINED;
  }
}

// NONE slots at level 0, or below a REFINED parent, are holes.
__global__ void k_holes(BatchArgs b) {
  const int32_t jb = job_of_block(b.jobs, b.n_jobs, LK_SLOTS, blockIdx.x);
  const Job& J = b.jobs[jb];
  const CoverIndex& ci = J.ci;
  if (ci.uniform) return;
  const int64_t s = (blockIdx.x - J.blk[LK_SLOTS]) * blockDim.x + threadIdx.x;
  if (s >= ci.off[ci.lmax + 1] || ci.state[s] != ST_NONE) return;
  int L = 0;
  while (s >= ci.off[L + 1]) ++L;
  if (L == 0) {
    ci.state[s] = ST_HOLE;
    return;
  }
  int64_t rem = s - ci.off[L];
  int64_t k[kMaxDim];
  for (int d = ci.n - 1; d >= 0; --d) {
    k[d] = rem % ci.dims[L][d];
    rem /= ci.dims[L][d];
  }
  int64_t plin = 0;
  for (int d = 0; d < ci.n; ++d) plin = plin * ci.dims[L - 1][d] + (k[d] >> 1);
  if (ci.state[ci.off[L - 1] + plin] == ST_REFINED) ci.state[s] = ST_HOLE;
}

__global__ void k_mark_dropped(BatchArgs b, const uint8_t* kept) {
  const int32_t jb = job_of_block(b.jobs, b.n_jobs, LK_CELLS, blockIdx.x);
  const Job& J = b.jobs[jb];
  const int64_t c = (blockIdx.x - J.blk[LK_CELLS]) * blockDim.x + threadIdx.x;
  if (c >= J.n_cells || J.ci.uniform) return;
  const int64_t gc = J.cell_off + c;
  if (kept[gc]) return;
  const int64_t slot = cell_slot(J.ci, b.level, b.idx, gc);
  if (slot >= 0) J.ci.state[slot] = ST_HOLE;
}

inline unsigned grid_for(int64_t n) {
  int64_t nb = (n + 255) / 256;
  if (nb < 1) nb = 1;
  if (nb > 8192) nb = 8192;
  return (unsigned)nb;
}

}  // namespace

int32_t fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) { return fill(p, v, n, s); }
int32_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) { return fill(p, v, n, s); }
int32_t fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s) { return fill(p, v, n, s); }
int32_t fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s) { return fill(p, v, n, s); }

int32_t zero_ranges(const ZeroRanges& z, hipStream_t s) {
  int64_t most = 0;
  for (int r = 0; r < z.n; ++r) most = z.words[r] > most ? z.words[r] : most;
  if (most == 0) return GIS_OK;
  int64_t nb = (most + 255) / 256;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(k_zero_ranges, dim3((unsigned)nb), dim3(256), 0, s, z);
  GIS_LAUNCH_CHECK("k_zero_ranges");
  return GIS_OK;
}

int32_t gather_copy(const Gather& g, hipStream_t s) {
  int64_t most = 0;
  for (int k = 0; k < g.n; ++k) most = g.bytes[k] > most ? g.bytes[k] : most;
  if (most == 0 || g.n <= 0) return GIS_OK;
  int64_t nb = (most / 16 + 255) / 256;
  if (nb < 1) nb = 1;
  if (nb > 2048) nb = 2048;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)nb, (unsigned)g.n), dim3(256), 0, s, g);
  GIS_LAUNCH_CHECK("k_gather");
  return GIS_OK;
}

int32_t max_level(const uint8_t* level, int64_t n_cells, uint32_t* d_out, hipStream_t s) {
  int32_t rc = fill_u32(d_out, 0u, 1, s);
  if (rc != GIS_OK || n_cells == 0) return rc;
  hipLaunchKernelGGL(k_max_level, dim3(grid_for(n_cells)), dim3(256), 0, s, level, n_cells, d_out);
  GIS_LAUNCH_CHECK("k_max_level");
  return GIS_OK;
}

int32_t batch_index_build(const BatchArgs& b, uint32_t* d_err, const uint8_t* state_all,
                          int64_t* pfx_all, int64_t total_slots, void* scan_tmp, bool validate,
                          hipStream_t s) {
  if (!validate) {
    if (b.blocks[LK_CELLS] > 0) {
      hipLaunchKernelGGL(k_leaves_up, dim3((unsigned)b.blocks[LK_CELLS]), dim3(256), 0, s, b);
      GIS_LAUNCH_CHECK("k_leaves_up");
    }
    if (b.blocks[LK_SLOTS] > 0) {
      hipLaunchKernelGGL(k_holes, dim3((unsigned)b.blocks[LK_SLOTS]), dim3(256), 0, s, b);
      GIS_LAUNCH_CHECK("k_holes");
    }
    if (total_slots > 0) return scan_leaf_hole(state_all, pfx_all, total_slots, scan_tmp, s);
    return GIS_OK;
  }
  int32_t rc = fill_u32(d_err, 0u, 1, s);
  if (rc != GIS_OK) return rc;
  if (b.blocks[LK_CELLS] > 0) {
    hipLaunchKernelGGL(k_leaves, dim3((unsigned)b.blocks[LK_CELLS]), dim3(256), 0, s, b, d_err);
    GIS_LAUNCH_CHECK("k_leaves");
    hipLaunchKernelGGL(k_ancestors, dim3((unsigned)b.blocks[LK_CELLS]), dim3(256), 0, s, b, d_err);
    GIS_LAUNCH_CHECK("k_ancestors");
  }
  if (b.blocks[LK_SLOTS] > 0) {
    hipLaunchKernelGGL(k_holes, dim3((unsigned)b.blocks[LK_SLOTS]), dim3(256), 0, s, b);
    GIS_LAUNCH_CHECK("k_holes");
  }
  if (total_slots > 0) return scan_leaf_hole(state_all, pfx_all, total_slots, scan_tmp, s);
  return GIS_OK;
}

int32_t batch_mark_dropped(const BatchArgs& b, const uint8_t* kept, hipStream_t s) {
  if (b.blocks[LK_CELLS] == 0) return GIS_OK;
  hipLaunchKernelGGL(k_mark_dropped, dim3((unsigned)b.blocks[LK_CELLS]), dim3(256), 0, s, b, kept);
  GIS_LAUNCH_CHECK("k_mark_dropped");
  return GIS_OK;
}

int32_t publish(const void* src, void* host_dst, size_t bytes, uint32_t* host_flag, uint32_t seq,
                hipStream_t s) {
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(256), 0, s, (const uint32_t*)src,
                     (uint32_t*)host_dst, (int32_t)((bytes + 3) / 4), host_flag, seq);
  GIS_LAUNCH_CHECK("k_publish");
  return GIS_OK;
}

}  // namespace gis
