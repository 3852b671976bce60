// gis_prune_static: the graph analysis of gis_prune without any device
// allocation, for callers that cannot allocate (code under HIP graph
// capture, tight serving loops).  Its workspace is the file-scope device
// array `scratch` below, one copy per GPU, held until the process ends.
//
// The analysis runs by sweeps only (witness sweeps for the non-leaving
// reading, row sweeps for the controlled one), which need a few bytes per
// cell and no reverse graph; the host checks convergence after each batch.
// Every call on a GPU shares that GPU's array: calls that overlap in time on
// one GPU (two host threads, or two streams) race on it and must not be made.
#include <mutex>

#include "gis_launch.h"

namespace gis {
namespace {

constexpr int64_t kStaticCells = (int64_t)1 << 21;  // largest n_cells accepted
constexpr size_t kAlign = 256;
constexpr size_t al(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Layout: counters, removed flags [n], witness
// positions [n], witness targets [n], removed flags packed 32 to a word.
struct StaticCounters {
  int32_t last;                 // 1 + index of the last sweep that removed a cell
  uint32_t err;                 // graph check flags
  unsigned long long n_kept;    // kept cells
};
constexpr size_t kOffRemoved = al(sizeof(StaticCounters));
constexpr size_t kOffWpos = kOffRemoved + al((size_t)kStaticCells);
constexpr size_t kOffWtgt = kOffWpos + al(8 * (size_t)kStaticCells);
constexpr size_t kOffBits = kOffWtgt + al(4 * (size_t)kStaticCells);
constexpr size_t kScratchBytes = kOffBits + al((size_t)kStaticCells / 8);  // about 26 MiB

}  // namespace
}  // namespace gis

static __device__ __align__(256) uint8_t scratch[gis::kScratchBytes];

namespace gis {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint8_t* g_ptr[kMaxDevices] = {};

// The array's device address on the current device (looked up once per
// device; host code never passes `scratch` itself to a kernel).
int32_t scratch_ptr(uint8_t** out) {
  int dev = -1;
  GIS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index out of range");
    return GIS_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    GIS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_ptr[dev] = (uint8_t*)p;
  }
  *out = g_ptr[dev];
  return GIS_OK;
}

int32_t inval(const char* m) {
  set_error(m);
  return GIS_E_INVAL;
}

}  // namespace
}  // namespace gis

using namespace gis;

extern "C" int32_t gis_prune_static(const gis_graph* graph, int64_t n_cells, int32_t K,
                                    int32_t analysis, uint8_t* d_kept, uint64_t* d_mask,
                                    int64_t* n_kept, void* stream) {
  if (!graph) return inval("graph is required");
  if (analysis != GIS_ANALYSIS_CONTROLLED && analysis != GIS_ANALYSIS_NONLEAVING)
    return inval("gis_prune_static: analysis must be controlled or nonleaving");
  if (n_cells < 0 || K < 1) return inval("invalid sizes");
  if (K > 256) return inval("gis_prune_static: at most 256 inputs");
  if (n_cells > kStaticCells) {
    set_error("gis_prune_static: more than 2^21 cells (the static workspace's limit)");
    return GIS_E_CAPACITY;
  }
  if (graph->n_rows != n_cells * K) return inval("graph rows != n_cells * K");
  if (n_cells > 0 && (!d_kept || !d_mask || !graph->row_ptr || !graph->out ||
                      (graph->n_edges > 0 && !graph->col)))
    return inval("buffers missing");
  if (n_cells == 0) {
    if (n_kept) *n_kept = 0;
    return GIS_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  uint8_t* base = nullptr;
  int32_t rc;
  if ((rc = scratch_ptr(&base))) return rc;
  StaticCounters* cnt = (StaticCounters*)base;
  StaticCounters h{};
  // counters to zero (a fill kernel, no memset), then the graph check
  if ((rc = fill_u32((uint32_t*)cnt, 0u, (int64_t)(sizeof(StaticCounters) / 4), s))) return rc;
  if ((rc = launch_check_graph(graph->row_ptr, graph->col, graph->n_rows, graph->n_edges, n_cells,
                               &cnt->err, s)))
    return rc;
  GIS_HIP(hipMemcpyAsync(&h, cnt, sizeof h, hipMemcpyDeviceToHost, s));
  GIS_HIP(hipStreamSynchronize(s));
  if (h.err & 1u) return inval("graph row offsets are inconsistent");
  if (h.err & 2u) return inval("graph targets are not cell ids");

  PruneWork w{};
  w.removed = base + kOffRemoved;
  w.last = &cnt->last;
  w.wpos = (int64_t*)(base + kOffWpos);
  w.wtgt = (int32_t*)(base + kOffWtgt);
  w.rbits = (uint32_t*)(base + kOffBits);
  w.rbits_cells = kStaticCells;
  w.sweep_blocks = 4096;
  if ((rc = fill_u8(w.removed, 0, n_cells, s))) return rc;
  // sweeps in batches until one removes nothing; each sweep that does not
  // converge removes a cell, so n_cells + 1 sweeps always suffice
  constexpr int32_t kBatch = 16;
  bool converged = false;
  for (int64_t done = 0; !converged; done += kBatch) {
    if (done > n_cells + kBatch) {
      set_error("internal: the sweeps did not converge");
      return GIS_E_INTERNAL;
    }
    rc = analysis == GIS_ANALYSIS_NONLEAVING
             ? prune_wsweeps(graph->row_ptr, graph->col, n_cells, K, w, (int32_t)done, kBatch, s)
             : prune_sweeps(graph->row_ptr, graph->col, graph->out, n_cells, K, analysis, w,
                            (int32_t)done, kBatch, s);
    if (rc) return rc;
    GIS_HIP(hipMemcpyAsync(&h, cnt, sizeof h, hipMemcpyDeviceToHost, s));
    GIS_HIP(hipStreamSynchronize(s));
    converged = h.last < done + kBatch;
  }
  if ((rc = prune_final(graph->row_ptr, graph->col, graph->out, n_cells, K, analysis, w, d_kept,
                        d_mask, (K + 63) / 64, &cnt->n_kept, 0, nullptr, 0, nullptr, nullptr,
                        nullptr, 0, s)))
    return rc;
  GIS_HIP(hipMemcpyAsync(&h, cnt, sizeof h, hipMemcpyDeviceToHost, s));
  GIS_HIP(hipStreamSynchronize(s));
  if (n_kept) *n_kept = (int64_t)h.n_kept;
  return GIS_OK;
}
