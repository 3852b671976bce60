// Internal declarations of libgis: kernel argument blocks, the covering
// index, device helpers and the host-side launchers of each translation unit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "gis.h"

namespace gis {

constexpr int kMaxDim = 4;
constexpr int kMaxLevels = 24;
constexpr int kRowBlock = 256;      // rows per block of the image / emit kernels
constexpr int kScanBlock = 256;     // threads of the scan kernels
constexpr int kScanItems = 8;       // items per thread of the scan kernels

// Covering-index states of a (level, multi-index) slot.
enum : uint8_t { ST_NONE = 0, ST_LEAF = 1, ST_REFINED = 2, ST_HOLE = 3 };

// Vector field parameters, the RK4 substep constants and the sizes.
struct SysArgs {
  int32_t kind, n, m, nsub;
  double h, h2, h6;     // substep, half substep, substep / 6 (computed on the host)
  double p[24];
};

// State box and level-0 widths.
struct GridArgs {
  int32_t n;
  int32_t n0[kMaxDim];
  double lo[kMaxDim], hi[kMaxDim];
  double w0[kMaxDim];   // (hi - lo) / n0
};

// Dense per-level index of a covering: for every level L <= lmax a row-major
// array of states (and of cell ids where the state is LEAF).
struct CoverIndex {
  int32_t n, lmax;
  int32_t uniform;                       // 1: full level-0 grid, no arrays needed
  int32_t dims[kMaxLevels][kMaxDim];     // n0_d << L
  int64_t off[kMaxLevels + 1];           // offset of level L in state/id
  uint8_t* state;
  int32_t* id;
};

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ int64_t lin_index(const int32_t* dims, const int64_t* k, int n) {
  int64_t lin = 0;
  for (int d = 0; d < n; ++d) lin = lin * dims[d] + k[d];
  return lin;
}

// ---------------------------------------------------------------- error handling
void set_error(const std::string& msg);
int32_t hip_fail(hipError_t e, const char* what);

#define GIS_HIP(expr)                                  \
  do {                                                 \
    hipError_t _e = (expr);                            \
    if (_e != hipSuccess) return gis::hip_fail(_e, #expr); \
  } while (0)

#define GIS_LAUNCH_CHECK(what)                         \
  do {                                                 \
    hipError_t _e = hipGetLastError();                 \
    if (_e != hipSuccess) return gis::hip_fail(_e, what); \
  } while (0)

// ---------------------------------------------------------------- workspace
// A growable device buffer owned by a context.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};
int32_t ensure(DevBuf& b, size_t bytes);
void release(DevBuf& b);

// HIP events bracketing the image kernels (created once per context).
struct KernelTimer {
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  bool ok = false;
};

// ---------------------------------------------------------------- launchers
// k_scan.hip
// Exclusive prefix sum of n int64 values into out[0..n) and the total into
// *d_total.  tmp must hold scan_tmp_bytes(n).
size_t scan_tmp_bytes(int64_t n);
int32_t scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* d_total,
                           void* tmp, hipStream_t s);
// Same for uint8 flags (0/1) -> int64 positions.
int32_t scan_exclusive_u8(const uint8_t* in, int64_t* out, int64_t n, int64_t* d_total, void* tmp,
                          hipStream_t s);
int32_t scan_exclusive_i32(const int32_t* in, int64_t* out, int64_t n, int64_t* d_total, void* tmp,
                           hipStream_t s);

// k_index.hip
// Builds the covering index of a canonical cell list; flags invalid lists in
// *d_err (bit 0: index out of range, bit 1: not canonical / duplicate,
// bit 2: overlapping cells).
int32_t index_build(CoverIndex& ci, const GridArgs& g, const uint8_t* level, const int32_t* idx,
                    int64_t n_cells, uint32_t* d_err, hipStream_t s);
int32_t index_mark_dropped(const CoverIndex& ci, const uint8_t* level, const int32_t* idx,
                           int64_t n_cells, const uint8_t* kept, hipStream_t s);
int32_t max_level(const uint8_t* level, int64_t n_cells, uint32_t* d_out, hipStream_t s);
int32_t fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
int32_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
int32_t fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s);
int32_t fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s);

// k_build.hip
struct BuildArgs {
  SysArgs sys;
  GridArgs grid;
  CoverIndex ci;
  const double* u;        // K x m
  int32_t K;
  int32_t samples;        // GIS_SAMPLES_*
  int32_t fast_out;
  const uint8_t* level;
  const int32_t* idx;
  int64_t n_rows;
  double band[kMaxDim];   // FP32 recheck band
  // outputs
  int32_t* rng;           // [n_rows * 2n] closed ranges on the finest grid (lo, hi per dim)
  int32_t* cnt;           // [n_rows] edge counts
  uint8_t* out;           // [n_rows] OUT flags
  int64_t* bsum;          // [n_blocks] edge count per block of kRowBlock rows
  int64_t* recheck;       // [n_rows] rows queued for the FP64 recheck
  int64_t* n_recheck;     // device counter
};
int32_t launch_count(const BuildArgs& a, int32_t precision, hipStream_t s);
int32_t launch_recheck(const BuildArgs& a, hipStream_t s);
struct EmitArgs {
  CoverIndex ci;
  int32_t n;
  int64_t n_rows;
  const int32_t* rng;
  const int32_t* cnt;
  const int64_t* bscan;   // exclusive scan of bsum
  const int64_t* total;   // device total edges
  int64_t cap_edges;
  int64_t* row_ptr;
  int32_t* col;
};
int32_t launch_emit(const EmitArgs& a, hipStream_t s);
int32_t launch_images(const BuildArgs& a, int32_t precision, double* d_images, hipStream_t s);
int32_t launch_calibrate(const BuildArgs& a, unsigned long long* d_maxerr, hipStream_t s);
int32_t count_out(const uint8_t* out, int64_t n, unsigned long long* d_count, hipStream_t s);

// k_prune.hip
struct PruneWork {
  int64_t* rptr;     // [n_cells + 1]
  int32_t* rrow;     // [n_edges] in-rows per target cell
  int32_t* rcur;     // [n_cells] scatter cursors / in-degrees
  int32_t* good;     // [n_cells]
  int32_t* alive;    // [n_rows] remaining kept targets (non-leaving analysis)
  uint32_t* badbits; // [ceil(n_rows / 32)] (controlled analysis)
  int32_t* queue;    // [n_cells]
  int32_t* qctl;     // [4]: alloc, head, pending, error
  void* scan_tmp;
};
// Flags an inconsistent CSR graph in *d_err (bit 0 offsets, bit 1 targets).
int32_t launch_check_graph(const int64_t* row_ptr, const int32_t* col, int64_t n_rows,
                           int64_t n_edges, int64_t n_cells, uint32_t* d_err, hipStream_t s);
int32_t launch_prune(const int64_t* row_ptr, const int32_t* col, const uint8_t* out,
                     int64_t n_cells, int32_t K, int64_t n_edges, int32_t analysis,
                     const PruneWork& w, uint8_t* kept, uint64_t* mask, int32_t mask_words,
                     unsigned long long* d_nkept, hipStream_t s);

// k_refine.hip
int32_t launch_boundary(const CoverIndex& ci, const GridArgs& g, const uint8_t* level,
                        const int32_t* idx, int64_t n_cells, const uint8_t* kept, int32_t rule,
                        uint8_t* boundary, hipStream_t s);
// Dense "present" flags of the next covering over levels 0..lmax+1 (layout of
// `next`), then compaction into a canonical cell list.
int32_t launch_next_flags(const CoverIndex& next, const uint8_t* level, const int32_t* idx,
                          int64_t n_cells, const uint8_t* kept, const uint8_t* boundary,
                          hipStream_t s);
int32_t launch_compact(const CoverIndex& next, const int64_t* pos, int64_t cap, uint8_t* level_out,
                       int32_t* idx_out, hipStream_t s);
int32_t launch_coarse(const GridArgs& g, uint8_t* level, int32_t* idx, hipStream_t s);
// out[L] = pos[first slot of level L] for L <= next.lmax
int32_t launch_level_starts(const CoverIndex& next, const int64_t* pos, int64_t* out,
                            hipStream_t s);

// k_query.hip
int32_t launch_query(const CoverIndex& ci, const GridArgs& g, const uint8_t* kept,
                     const uint64_t* mask, int32_t mask_words, const double* states, int64_t n,
                     uint8_t* member, uint64_t* adm, hipStream_t s);

}  // namespace gis
