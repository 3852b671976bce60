// Internal declarations of libgis shared by every translation unit: kernel
// argument blocks, the covering index, device helpers, the scan, fill, copy and
// build launchers.  The other units' launchers are declared in gis_launch.h.
// Under hipRTC (runtime-compiled user fields, __HIPCC_RTC__) only the device
// part is seen: argument blocks, job table and device helpers.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#endif

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
// array of states, and prefix counts of its leaves and holes.
struct CoverIndex {
  int32_t n, lmax;
  int32_t uniform;                       // 1: full level-0 grid, no arrays needed
  int32_t dims[kMaxLevels][kMaxDim];     // n0_d << L
  int64_t off[kMaxLevels + 1];           // offset of level L in state / pfx
  int64_t pbase;          // leaves before the job's first slot (see pfx)
  uint8_t* state;
  // [slots + 1] over the slots in canonical order (level, then row-major):
  // (number of LEAF slots before it) | (number of HOLE slots before it) << 32,
  // counted from the start of the batch's index.  A run of slots holds
  // pfx[b+1] - pfx[a] leaves and holes, and its leaves have the consecutive
  // local ids (pfx[a] & 0xffffffff) - pbase, ...
  int64_t* pfx;
};

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ int64_t lin_index(const int32_t* dims, const int64_t* k, int n) {
  int64_t lin = 0;
  for (int d = 0; d < n; ++d) lin = lin * dims[d] + k[d];
  return lin;
}

#ifndef __HIPCC_RTC__
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
// Grows b to at least `bytes` (contents are lost when it grows; *fresh is
// set then).
int32_t ensure(DevBuf& b, size_t bytes, bool* fresh = nullptr);
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
// Exclusive scan of packed (leaf, hole << 32) indicators of index states into
// out[0..n], out[n] = total.
int32_t scan_leaf_hole(const uint8_t* state, int64_t* out, int64_t n, void* tmp, hipStream_t s);

// k_index.hip
int32_t max_level(const uint8_t* level, int64_t n_cells, uint32_t* d_out, hipStream_t s);
int32_t fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
int32_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
int32_t fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s);
int32_t fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s);
// Up to four buffers cleared by one launch (sizes in 32-bit words).
struct ZeroRanges {
  uint32_t* p[4];
  int64_t words[4];
  int n;
};
int32_t zero_ranges(const ZeroRanges& z, hipStream_t s);
// Up to six device-to-device copies in one launch (any alignment).
constexpr int kGatherSegs = 6;
struct Gather {
  const uint8_t* src[kGatherSegs];
  uint8_t* dst[kGatherSegs];
  int64_t bytes[kGatherSegs];
  int n;
};
int32_t gather_copy(const Gather& g, hipStream_t s);
#endif  // __HIPCC_RTC__

// ---------------------------------------------------------------- jobs
// A batch runs several independent solves (jobs) through the same launches.
// Cells and rows are numbered globally, job after job (row = global cell * K
// + input), so the graph of a batch is the disjoint union of the jobs'
// graphs.  Each launch pads only its grid: every block belongs to one job,
// found by a binary search over the jobs' first-block offsets for that kind
// of launch, so all job parameters are wave-uniform.
enum LaunchKind { LK_ROWS = 0, LK_CELLS = 1, LK_SLOTS = 2, LK_NEXT = 3, LK_KINDS = 4 };

struct Job {
  SysArgs sys;
  GridArgs grid;
  CoverIndex ci;          // index of the job's current covering
  CoverIndex next;        // layout (and flag array) of the next covering
  const double* u;        // K x m inputs
  int64_t n_cells;        // cells of the current covering
  int64_t cell_off;       // global id of the job's first cell
  int64_t next_off;       // offset of the job's flags in the batch's next-flag array
  int64_t blk[LK_KINDS];  // first launch block of the job, per launch kind
  double band[kMaxDim];   // FP32 recheck band
};

// Per-job counters, read back once per phase.
struct JobStats {
  unsigned long long n_out, n_kept, n_boundary, n_recheck, n_selected;
  int64_t n_edges;
  int64_t next_start;                   // first new cell of the job (global position)
  int64_t level_start[kMaxLevels + 1];  // new cells before each level (global position)
};

__device__ __forceinline__ int32_t job_of_block(const Job* jobs, int32_t n_jobs, int kind,
                                                int64_t b) {
  int32_t lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (jobs[mid].blk[kind] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Copies a job's covering index into LDS (all threads of the block take
// part).  Kernels then walk the index from LDS: reading it through the job
// table in global memory would make the compiler reload it after every
// global store, since it cannot rule out aliasing.
__device__ __forceinline__ void stage_index(CoverIndex* dst, const CoverIndex* src) {
  const int words = (int)(sizeof(CoverIndex) / 4);
  for (int i = threadIdx.x; i < words; i += blockDim.x)
    ((int32_t*)dst)[i] = ((const int32_t*)src)[i];
  __syncthreads();
}

// Slot of global cell gc in its job's covering index ci; -1 if its level or
// multi-index is out of range.
__device__ __forceinline__ int64_t cell_slot(const CoverIndex& ci, const uint8_t* level,
                                             const int32_t* idx, int64_t gc) {
  const int L = level[gc];
  if (L > ci.lmax) return -1;
  int64_t lin = 0;
  for (int d = 0; d < ci.n; ++d) {
    const int32_t v = idx[gc * ci.n + d];
    if (v < 0 || v >= ci.dims[L][d]) return -1;
    lin = lin * ci.dims[L][d] + v;
  }
  return ci.off[L] + lin;
}

// Job owning a global cell (binary search over the jobs' cell offsets).
__device__ __forceinline__ int32_t job_of_cell(const Job* jobs, int32_t n_jobs, int64_t cell) {
  int32_t lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (jobs[mid].cell_off <= cell) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Job owning a global row (binary search over the jobs' row offsets).
__device__ __forceinline__ int32_t job_of_row(const Job* jobs, int32_t n_jobs, int32_t K,
                                              int64_t row) {
  int32_t lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (jobs[mid].cell_off * K <= row) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------- k_build.hip
struct BuildArgs {
  const Job* jobs;
  int32_t n_jobs;
  int32_t K;
  int32_t samples;        // GIS_SAMPLES_*
  int32_t fast_out;
  int32_t kind, n, m;     // system kind, state and input dimensions shared by the batch
  int32_t all_uniform;    // every job's covering is its full level-0 grid
  int64_t n_blocks;       // launch blocks (LK_ROWS)
  int64_t total_rows;
  const uint8_t* level;   // global cell list
  const int32_t* idx;
  // outputs of k_build, indexed by global row
  uint8_t* out;           // [rows] OUT flags
  int64_t* row_ptr;       // [rows + 1]
  int32_t* col;           // [cap_edges]
  int32_t* first;         // [rows] each row's first target (-1: none), or null
  int64_t cap_edges;
  uint64_t* lb;           // [n_blocks] look-back words (tagged with `epoch`)
  uint32_t* ticket;       // block ticket: 0 before the launch, reset to 0 by the last block
  uint32_t epoch;         // 1 .. 2^24-1, different from every word left in lb
  int64_t* d_total;       // edge total of the batch
  unsigned long long* n_recheck;  // rows the FP32 test sent to FP64
  uint32_t* err;          // bit 8: a look-back wait reached its time limit
  JobStats* stats;        // per-job n_edges, n_out, n_recheck (accumulated)
  const void* user;       // host: the context's compiled user field (kind GIS_SYS_USER)
};
#ifndef __HIPCC_RTC__
// Symbolic image of the batch's coverings into (row_ptr, col, out); col is
// written only if the edge total fits in cap_edges.
int32_t launch_build(const BuildArgs& a, int32_t precision, hipStream_t s);
int32_t launch_images(const BuildArgs& a, int32_t precision, double* d_images, hipStream_t s);
// The library's FP64 exponential (the CSTR field's), elementwise.
int32_t launch_exp(const double* d_x, int64_t n, double* d_y, hipStream_t s);
// max |y32 - y64| per job and dimension over the rows of every stride-th
// launch block of each job (all rows when stride <= 1).
int32_t launch_calibrate(const BuildArgs& a, unsigned long long* d_maxerr, int64_t stride,
                         hipStream_t s);
// Writes the calibrated band into the device job table for every (job,
// dimension) whose band is not positive there: max(8 maxerr, floor_rel w),
// w the finest cell width of the job's current covering.
int32_t launch_band(Job* d_jobs, int32_t n_jobs, int32_t n, const unsigned long long* d_maxerr,
                    double floor_rel, hipStream_t s);
#endif  // __HIPCC_RTC__

}  // namespace gis
