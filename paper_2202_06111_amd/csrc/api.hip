// C ABI of libgis (declared in include/gis.h): argument checks, device
// workspace, and the host-side sequencing of the kernels of one iteration of
// the GIS loop (Sec. 2 and Sec. 3.1): build the symbolic image, analyse it,
// select boundary cells and subdivide them.
#include <math.h>
#include <string.h>

#include <string>
#include <utility>

#include "gis_internal.h"

namespace gis {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int32_t hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? GIS_E_NOMEM : GIS_E_HIP;
}

int32_t ensure(DevBuf& b, size_t bytes) {
  if (bytes <= b.bytes && b.ptr) return GIS_OK;
  release(b);
  size_t want = bytes + bytes / 4 + 256;
  hipError_t e = hipMalloc(&b.ptr, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.ptr = nullptr;
    b.bytes = 0;
    set_error("device allocation of " + std::to_string(want) + " bytes failed");
    return GIS_E_NOMEM;
  }
  b.bytes = want;
  return GIS_OK;
}

void release(DevBuf& b) {
  if (b.ptr) (void)hipFree(b.ptr);
  b.ptr = nullptr;
  b.bytes = 0;
}

// Device counters shared by the kernels of one call; read back in one copy.
struct Counters {
  int64_t total_edges;
  int64_t n_recheck;
  unsigned long long n_out;
  unsigned long long n_kept[2];
  uint32_t err;
  uint32_t maxlevel;
  int64_t n_next;
  unsigned long long maxerr[kMaxDim];
  int32_t qctl[4];
  int64_t level_start[kMaxLevels + 1];   // new cells before each level (subdivision)
};

}  // namespace gis

using namespace gis;

struct gis_ctx {
  int device = 0;
  DevBuf counters;
  Counters* h_counters = nullptr;   // pinned
  DevBuf rng, cnt, bsum, bscan, recheck, scan_tmp;
  DevBuf idx_state, idx_id, next_state, pos;
  DevBuf rptr, rrow, rcur, good, alive, badbits, queue;
  DevBuf bnd;
  // cell lists and graph of the solve loop
  DevBuf lvA, ixA, lvB, ixB, row_ptr, col, out, kept, mask;
  DevBuf ubuf;
  gis::KernelTimer timer;
};

struct gis_solution {
  int device = 0;
  GridArgs grid{};
  CoverIndex ci{};
  int32_t K = 0, W = 0;
  int64_t n_cells = 0;
  DevBuf level, idx, kept, mask, state, id;
  gis_solve_info info{};
};

namespace gis {
namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

int32_t inval(const std::string& m) {
  set_error(m);
  return GIS_E_INVAL;
}

int32_t check_system(const gis_system* s) {
  if (!s) return inval("system is NULL");
  if (s->n < 1 || s->n > kMaxDim) return inval("state dimension must be 1..4");
  if (s->m < 1 || s->m > 2) return inval("input dimension must be 1..2");
  if (s->nsub < 1) return inval("nsub must be >= 1");
  if (!(s->dt > 0.0) || !isfinite(s->dt)) return inval("dt must be finite and > 0");
  switch (s->kind) {
    case GIS_SYS_LINEAR: break;
    case GIS_SYS_VDP: if (s->n != 2 || s->m != 1) return inval("VDP needs n=2, m=1"); break;
    case GIS_SYS_LORENZ: if (s->n != 3 || s->m != 1) return inval("LORENZ needs n=3, m=1"); break;
    case GIS_SYS_VDP2: if (s->n != 4 || s->m != 2) return inval("VDP2 needs n=4, m=2"); break;
    default: return inval("unknown system kind");
  }
  return GIS_OK;
}

int32_t check_grid(const gis_grid* g, int n) {
  if (!g) return inval("grid is NULL");
  if (g->n != n) return inval("grid dimension differs from the system's");
  for (int d = 0; d < n; ++d) {
    if (g->n0[d] < 1) return inval("coarse cell counts must be >= 1");
    if (!(g->lo[d] < g->hi[d]) || !isfinite(g->lo[d]) || !isfinite(g->hi[d]))
      return inval("state box needs finite lo < hi");
  }
  return GIS_OK;
}

int32_t check_opts(const gis_opts* o) {
  if (!o) return inval("opts is NULL");
  if (o->samples != GIS_SAMPLES_LATTICE3 && o->samples != GIS_SAMPLES_CORNERS_CENTER)
    return inval("unknown sample scheme");
  if (o->precision != GIS_PREC_FP64 && o->precision != GIS_PREC_FP32_RECHECK)
    return inval("unknown precision");
  if (o->boundary_rule != GIS_BOUNDARY_SHELL && o->boundary_rule != GIS_BOUNDARY_CORNERS)
    return inval("unknown boundary rule");
  if (o->analysis != GIS_ANALYSIS_CONTROLLED && o->analysis != GIS_ANALYSIS_NONLEAVING)
    return inval("unknown analysis");
  return GIS_OK;
}

SysArgs make_sys(const gis_system* s) {
  SysArgs a{};
  a.kind = s->kind;
  a.n = s->n;
  a.m = s->m;
  a.nsub = s->nsub;
  a.h = s->dt / (double)s->nsub;
  a.h2 = 0.5 * a.h;
  a.h6 = a.h / 6.0;
  for (int i = 0; i < 24; ++i) a.p[i] = s->params[i];
  return a;
}

GridArgs make_grid(const gis_grid* g) {
  GridArgs a{};
  a.n = g->n;
  for (int d = 0; d < g->n; ++d) {
    a.n0[d] = g->n0[d];
    a.lo[d] = g->lo[d];
    a.hi[d] = g->hi[d];
    a.w0[d] = (g->hi[d] - g->lo[d]) / (double)g->n0[d];
  }
  return a;
}

int64_t prod_n0(const GridArgs& g) {
  int64_t t = 1;
  for (int d = 0; d < g.n; ++d) t *= g.n0[d];
  return t;
}

// Layout of a covering index with levels 0..lmax.
int32_t layout_index(CoverIndex& ci, const GridArgs& g, int lmax) {
  if (lmax < 0 || lmax >= kMaxLevels) return inval("too many refinement levels");
  ci.n = g.n;
  ci.lmax = lmax;
  ci.off[0] = 0;
  for (int L = 0; L <= lmax; ++L) {
    int64_t t = 1;
    for (int d = 0; d < g.n; ++d) {
      const int64_t Nd = (int64_t)g.n0[d] << L;
      if (Nd >= (int64_t)1 << 30) {
        set_error("finest grid exceeds 2^30 cells per dimension");
        return GIS_E_UNSUPPORTED;
      }
      ci.dims[L][d] = (int32_t)Nd;
      t *= Nd;
    }
    if (t > ((int64_t)1 << 36)) {
      set_error("dense covering index would exceed 64 GiB");
      return GIS_E_UNSUPPORTED;
    }
    ci.off[L + 1] = ci.off[L] + t;
  }
  return GIS_OK;
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

int32_t sync_counters(gis_ctx* ctx, hipStream_t s) {
  GIS_HIP(hipMemcpyAsync(ctx->h_counters, ctx->counters.ptr, sizeof(Counters),
                         hipMemcpyDeviceToHost, s));
  GIS_HIP(hipStreamSynchronize(s));
  return GIS_OK;
}

Counters* dcnt(gis_ctx* ctx) { return (Counters*)ctx->counters.ptr; }

int32_t zero_counters(gis_ctx* ctx, hipStream_t s) {
  return fill_u32((uint32_t*)ctx->counters.ptr, 0u, (int64_t)(sizeof(Counters) / 4), s);
}

// Finds the finest level of a cell list (synchronises).
int32_t list_lmax(gis_ctx* ctx, const uint8_t* level, int64_t n_cells, int* lmax, hipStream_t s) {
  int32_t rc = zero_counters(ctx, s);
  if (rc) return rc;
  if ((rc = max_level(level, n_cells, &dcnt(ctx)->maxlevel, s))) return rc;
  if ((rc = sync_counters(ctx, s))) return rc;
  *lmax = (int)ctx->h_counters->maxlevel;
  return GIS_OK;
}

// Builds (or, for the full level-0 grid, only checks) the covering index of
// a cell list in the context's index buffers.  With `validate` it
// synchronises to report an invalid list; lists the library produced itself
// are canonical by construction and skip that round trip.
int32_t prepare_index(gis_ctx* ctx, const GridArgs& g, const uint8_t* level, const int32_t* idx,
                      int64_t n_cells, int lmax, bool want_arrays, CoverIndex& ci, hipStream_t s,
                      bool validate = true) {
  int32_t rc = layout_index(ci, g, lmax);
  if (rc) return rc;
  ci.uniform = (!want_arrays && lmax == 0 && n_cells == prod_n0(g)) ? 1 : 0;
  ci.state = nullptr;
  ci.id = nullptr;
  if (!ci.uniform) {
    const int64_t total = ci.off[lmax + 1];
    if ((rc = ensure(ctx->idx_state, (size_t)total))) return rc;
    if ((rc = ensure(ctx->idx_id, (size_t)total * 4))) return rc;
    ci.state = (uint8_t*)ctx->idx_state.ptr;
    ci.id = (int32_t*)ctx->idx_id.ptr;
  }
  if ((rc = index_build(ci, g, level, idx, n_cells, &dcnt(ctx)->err, s))) return rc;
  if (!validate) return GIS_OK;
  if ((rc = sync_counters(ctx, s))) return rc;
  const uint32_t e = ctx->h_counters->err;
  if (e & 1u) return inval("a cell's level or multi-index is out of range");
  if (e & 2u) return inval("cells are not in canonical order (level, row-major index) or repeat");
  if (e & 4u) return inval("cells overlap (a cell contains another)");
  return GIS_OK;
}

struct Graph {
  int64_t* row_ptr;
  int32_t* col;
  uint8_t* out;
  int64_t cap_edges;
  int64_t n_edges, n_out, n_recheck;
  float ms_image, ms_recheck;   // with opts.timing
};


BuildArgs make_build_args(gis_ctx* ctx, const gis_system* sys, const gis_grid* grid,
                          const double* d_u, int32_t K, const CoverIndex& ci, const uint8_t* level,
                          const int32_t* idx, int64_t n_cells, const gis_opts* o) {
  BuildArgs a{};
  a.sys = make_sys(sys);
  a.grid = make_grid(grid);
  a.ci = ci;
  a.u = d_u;
  a.K = K;
  a.samples = o ? o->samples : GIS_SAMPLES_LATTICE3;
  a.fast_out = o ? o->fast_out : 0;
  a.level = level;
  a.idx = idx;
  a.n_rows = n_cells * K;
  for (int d = 0; d < kMaxDim; ++d) a.band[d] = o ? o->band[d] : 0.0;
  a.rng = (int32_t*)ctx->rng.ptr;
  a.cnt = (int32_t*)ctx->cnt.ptr;
  a.bsum = (int64_t*)ctx->bsum.ptr;
  a.recheck = (int64_t*)ctx->recheck.ptr;
  a.n_recheck = &dcnt(ctx)->n_recheck;
  return a;
}

// count -> (recheck) -> scan -> emit; `col` may be too small (then only the
// counts are valid).  Synchronises.
int32_t run_build(gis_ctx* ctx, const gis_system* sys, const gis_grid* grid, const double* d_u,
                  int32_t K, const CoverIndex& ci, const uint8_t* level, const int32_t* idx,
                  int64_t n_cells, const gis_opts* o, Graph& gr, hipStream_t s) {
  const int64_t n_rows = n_cells * K;
  const int64_t nb = (n_rows + kRowBlock - 1) / kRowBlock;
  int32_t rc;
  if ((rc = ensure(ctx->rng, (size_t)n_rows * 2 * sys->n * 4 + 16))) return rc;
  if ((rc = ensure(ctx->cnt, (size_t)n_rows * 4 + 16))) return rc;
  if ((rc = ensure(ctx->bsum, (size_t)nb * 8 + 16))) return rc;
  if ((rc = ensure(ctx->bscan, (size_t)nb * 8 + 16))) return rc;
  if ((rc = ensure(ctx->scan_tmp, scan_tmp_bytes(nb > n_cells ? nb : n_cells + 1)))) return rc;
  if (o->precision == GIS_PREC_FP32_RECHECK && (rc = ensure(ctx->recheck, (size_t)n_rows * 8 + 16)))
    return rc;
  if ((rc = zero_counters(ctx, s))) return rc;
  BuildArgs a = make_build_args(ctx, sys, grid, d_u, K, ci, level, idx, n_cells, o);
  a.out = gr.out;
  KernelTimer& tm = ctx->timer;
  const bool timing = o->timing && tm.ok;
  if (timing) GIS_HIP(hipEventRecord(tm.ev[0], s));
  if ((rc = launch_count(a, o->precision, s))) return rc;
  if (timing) GIS_HIP(hipEventRecord(tm.ev[1], s));
  if (o->precision == GIS_PREC_FP32_RECHECK && (rc = launch_recheck(a, s))) return rc;
  if (timing) GIS_HIP(hipEventRecord(tm.ev[2], s));
  if ((rc = scan_exclusive_i64((const int64_t*)ctx->bsum.ptr, (int64_t*)ctx->bscan.ptr, nb,
                               &dcnt(ctx)->total_edges, ctx->scan_tmp.ptr, s)))
    return rc;
  EmitArgs e{};
  e.ci = ci;
  e.n = sys->n;
  e.n_rows = n_rows;
  e.rng = a.rng;
  e.cnt = a.cnt;
  e.bscan = (const int64_t*)ctx->bscan.ptr;
  e.total = &dcnt(ctx)->total_edges;
  e.cap_edges = gr.cap_edges;
  e.row_ptr = gr.row_ptr;
  e.col = gr.col;
  if ((rc = launch_emit(e, s))) return rc;
  if ((rc = count_out(gr.out, n_rows, &dcnt(ctx)->n_out, s))) return rc;
  if ((rc = sync_counters(ctx, s))) return rc;
  gr.n_edges = ctx->h_counters->total_edges;
  gr.n_out = (int64_t)ctx->h_counters->n_out;
  gr.n_recheck = ctx->h_counters->n_recheck;
  gr.ms_image = gr.ms_recheck = 0.f;
  if (timing) {
    GIS_HIP(hipEventElapsedTime(&gr.ms_image, tm.ev[0], tm.ev[1]));
    GIS_HIP(hipEventElapsedTime(&gr.ms_recheck, tm.ev[1], tm.ev[2]));
  }
  if (n_rows == 0) {  // row_ptr[0] = 0 for an empty graph
    if ((rc = fill_i64(gr.row_ptr, 0, 1, s))) return rc;
  }
  return GIS_OK;
}

// Re-runs only the emitter after col was grown.
int32_t rerun_emit(gis_ctx* ctx, int n, const CoverIndex& ci, int64_t n_rows, Graph& gr,
                   hipStream_t s) {
  EmitArgs e{};
  e.ci = ci;
  e.n = n;
  e.n_rows = n_rows;
  e.rng = (const int32_t*)ctx->rng.ptr;
  e.cnt = (const int32_t*)ctx->cnt.ptr;
  e.bscan = (const int64_t*)ctx->bscan.ptr;
  e.total = &dcnt(ctx)->total_edges;
  e.cap_edges = gr.cap_edges;
  e.row_ptr = gr.row_ptr;
  e.col = gr.col;
  return launch_emit(e, s);
}

int32_t run_prune(gis_ctx* ctx, const int64_t* row_ptr, const int32_t* col, const uint8_t* out,
                  int64_t n_cells, int32_t K, int64_t n_edges, int32_t analysis, uint8_t* kept,
                  uint64_t* mask, int64_t* n_kept, hipStream_t s) {
  const int64_t n_rows = n_cells * K;
  const int32_t W = (K + 63) / 64;
  int32_t rc;
  if ((rc = ensure(ctx->rptr, (size_t)(n_cells + 1) * 8))) return rc;
  if ((rc = ensure(ctx->rrow, (size_t)n_edges * 4 + 16))) return rc;
  if ((rc = ensure(ctx->rcur, (size_t)n_cells * 4 + 16))) return rc;
  if ((rc = ensure(ctx->good, (size_t)n_cells * 4 + 16))) return rc;
  if ((rc = ensure(ctx->queue, (size_t)n_cells * 4 + 16))) return rc;
  if ((rc = ensure(ctx->scan_tmp, scan_tmp_bytes(n_cells + 1)))) return rc;
  if (analysis == GIS_ANALYSIS_NONLEAVING) {
    if ((rc = ensure(ctx->alive, (size_t)n_rows * 4 + 16))) return rc;
  } else if ((rc = ensure(ctx->badbits, (size_t)((n_rows + 31) / 32) * 4 + 16))) {
    return rc;
  }
  if ((rc = zero_counters(ctx, s))) return rc;
  PruneWork w{};
  w.rptr = (int64_t*)ctx->rptr.ptr;
  w.rrow = (int32_t*)ctx->rrow.ptr;
  w.rcur = (int32_t*)ctx->rcur.ptr;
  w.good = (int32_t*)ctx->good.ptr;
  w.alive = (int32_t*)ctx->alive.ptr;
  w.badbits = (uint32_t*)ctx->badbits.ptr;
  w.queue = (int32_t*)ctx->queue.ptr;
  w.qctl = dcnt(ctx)->qctl;
  w.scan_tmp = ctx->scan_tmp.ptr;
  if ((rc = launch_prune(row_ptr, col, out, n_cells, K, n_edges, analysis, w, kept, mask, W,
                         dcnt(ctx)->n_kept, s)))
    return rc;
  if ((rc = sync_counters(ctx, s))) return rc;
  if (ctx->h_counters->qctl[3]) {
    set_error("prune work queue did not drain within its time limit");
    return GIS_E_INTERNAL;
  }
  if (n_kept) *n_kept = (int64_t)ctx->h_counters->n_kept[0];
  return GIS_OK;
}

// Boundary selection + next covering.  `ci` is the index of the current list
// with its arrays built.  Writes the new list to (lv_out, ix_out) if cap
// allows.  Synchronises.
int32_t run_subdivide(gis_ctx* ctx, const GridArgs& g, CoverIndex& ci, const uint8_t* level,
                      const int32_t* idx, int64_t n_cells, const uint8_t* kept, int32_t rule,
                      uint8_t* boundary, uint8_t* lv_out, int32_t* ix_out, int64_t cap,
                      int64_t* n_new, int* new_lmax, int64_t* n_boundary, hipStream_t s) {
  int32_t rc;
  if ((rc = index_mark_dropped(ci, level, idx, n_cells, kept, s))) return rc;
  if ((rc = launch_boundary(ci, g, level, idx, n_cells, kept, rule, boundary, s))) return rc;
  CoverIndex next{};
  if ((rc = layout_index(next, g, ci.lmax + 1))) return rc;
  const int64_t total = next.off[next.lmax + 1];
  if ((rc = ensure(ctx->next_state, (size_t)total + 16))) return rc;
  if ((rc = ensure(ctx->pos, (size_t)(total + 1) * 8))) return rc;
  if ((rc = ensure(ctx->scan_tmp, scan_tmp_bytes(total)))) return rc;
  next.state = (uint8_t*)ctx->next_state.ptr;
  if ((rc = launch_next_flags(next, level, idx, n_cells, kept, boundary, s))) return rc;
  int64_t* pos = (int64_t*)ctx->pos.ptr;
  if ((rc = zero_counters(ctx, s))) return rc;
  if ((rc = scan_exclusive_u8(next.state, pos, total, &dcnt(ctx)->n_next, ctx->scan_tmp.ptr, s)))
    return rc;
  if ((rc = launch_compact(next, pos, cap, lv_out, ix_out, s))) return rc;
  if ((rc = count_out(boundary, n_cells, &dcnt(ctx)->n_out, s))) return rc;
  // new cells before each level start -> the finest level present
  if ((rc = launch_level_starts(next, pos, dcnt(ctx)->level_start, s))) return rc;
  if ((rc = sync_counters(ctx, s))) return rc;
  *n_new = ctx->h_counters->n_next;
  *n_boundary = (int64_t)ctx->h_counters->n_out;
  const int64_t* h_pos = ctx->h_counters->level_start;
  int lm = 0;
  for (int L = 0; L <= next.lmax; ++L) {
    const int64_t end = L < next.lmax ? h_pos[L + 1] : *n_new;
    if (end > h_pos[L]) lm = L;
  }
  *new_lmax = lm;
  if (*n_new > cap) {
    set_error("output cell list capacity too small");
    return GIS_E_CAPACITY;
  }
  return GIS_OK;
}

}  // namespace
}  // namespace gis

// ====================================================================== ABI
extern "C" {

const char* gis_last_error(void) { return g_err.c_str(); }
const char* gis_version(void) { return "gis-mi355x 0.1 (gfx950)"; }

int32_t gis_ctx_create(int32_t device, gis_ctx** out) {
  if (!out) return inval("out is NULL");
  *out = nullptr;
  int count = 0;
  GIS_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return inval("no such device");
  DeviceGuard g(device);
  gis_ctx* c = new gis_ctx();
  c->device = device;
  int32_t rc = ensure(c->counters, sizeof(Counters));
  if (rc) {
    delete c;
    return rc;
  }
  hipError_t e = hipHostMalloc((void**)&c->h_counters, sizeof(Counters), hipHostMallocDefault);
  if (e != hipSuccess) {
    release(c->counters);
    delete c;
    return hip_fail(e, "hipHostMalloc");
  }
  c->timer.ok = true;
  for (int i = 0; i < 3; ++i)
    if (hipEventCreate(&c->timer.ev[i]) != hipSuccess) c->timer.ok = false;
  *out = c;
  return GIS_OK;
}

void gis_ctx_destroy(gis_ctx* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();
  DevBuf* bufs[] = {&c->counters, &c->rng, &c->cnt, &c->bsum, &c->bscan, &c->recheck,
                    &c->scan_tmp, &c->idx_state, &c->idx_id, &c->next_state, &c->pos, &c->rptr,
                    &c->rrow, &c->rcur, &c->good, &c->alive, &c->badbits, &c->queue, &c->bnd,
                    &c->lvA, &c->ixA, &c->lvB, &c->ixB, &c->row_ptr, &c->col, &c->out,
                    &c->kept, &c->mask, &c->ubuf};
  for (DevBuf* b : bufs) release(*b);
  if (c->h_counters) (void)hipHostFree(c->h_counters);
  for (int i = 0; i < 3; ++i)
    if (c->timer.ev[i]) (void)hipEventDestroy(c->timer.ev[i]);
  delete c;
}

int32_t gis_build_graph(gis_ctx* ctx, const gis_system* sys, const gis_grid* grid,
                        const double* d_u, int32_t K, const gis_cells* cells, const gis_opts* opts,
                        gis_graph* graph, void* stream) {
  if (!ctx) return inval("ctx is NULL");
  int32_t rc;
  if ((rc = check_system(sys)) || (rc = check_grid(grid, sys->n)) || (rc = check_opts(opts)))
    return rc;
  if (!cells || !graph || !d_u || K < 1) return inval("cells, graph, inputs and K >= 1 are required");
  if (cells->n_cells < 0 || (cells->n_cells > 0 && (!cells->level || !cells->idx)))
    return inval("invalid cell list");
  if (cells->n_cells * (int64_t)K >= ((int64_t)1 << 31)) {
    set_error("more than 2^31 - 1 rows");
    return GIS_E_UNSUPPORTED;
  }
  if (opts->precision == GIS_PREC_FP32_RECHECK)
    for (int d = 0; d < sys->n; ++d)
      if (!(opts->band[d] > 0.0)) return inval("FP32 recheck needs band[d] > 0 (see gis_calibrate_band)");
  const int64_t n_rows = cells->n_cells * K;
  if (!graph->row_ptr || (n_rows > 0 && !graph->out) || (graph->cap_edges > 0 && !graph->col))
    return inval("graph buffers missing");
  DeviceGuard g(ctx->device);
  hipStream_t s = as_stream(stream);
  const GridArgs ga = make_grid(grid);
  int lmax = 0;
  if ((rc = list_lmax(ctx, cells->level, cells->n_cells, &lmax, s))) return rc;
  CoverIndex ci{};
  if ((rc = prepare_index(ctx, ga, cells->level, cells->idx, cells->n_cells, lmax, false, ci, s)))
    return rc;
  Graph gr{graph->row_ptr, graph->col, graph->out, graph->cap_edges, 0, 0, 0, 0.f, 0.f};
  if ((rc = run_build(ctx, sys, grid, d_u, K, ci, cells->level, cells->idx, cells->n_cells, opts,
                      gr, s)))
    return rc;
  graph->n_rows = n_rows;
  graph->n_edges = gr.n_edges;
  graph->n_out = gr.n_out;
  graph->n_recheck = gr.n_recheck;
  if (gr.n_edges > graph->cap_edges) {
    set_error("col capacity too small; n_edges holds the needed capacity");
    return GIS_E_CAPACITY;
  }
  return GIS_OK;
}

int32_t gis_prune(gis_ctx* ctx, const gis_graph* graph, int64_t n_cells, int32_t K,
                  int32_t analysis, uint8_t* d_kept, uint64_t* d_mask, int64_t* n_kept,
                  void* stream) {
  if (!ctx || !graph) return inval("ctx and graph are required");
  if (analysis != GIS_ANALYSIS_CONTROLLED && analysis != GIS_ANALYSIS_NONLEAVING)
    return inval("unknown analysis");
  if (n_cells < 0 || K < 1) return inval("invalid sizes");
  if (graph->n_rows != n_cells * K) return inval("graph rows != n_cells * K");
  if (n_cells * (int64_t)K >= ((int64_t)1 << 31)) {
    set_error("more than 2^31 - 1 rows");
    return GIS_E_UNSUPPORTED;
  }
  if (n_cells > 0 && (!d_kept || !d_mask || !graph->row_ptr || !graph->out ||
                      (graph->n_edges > 0 && !graph->col)))
    return inval("buffers missing");
  if (n_cells == 0) {
    if (n_kept) *n_kept = 0;
    return GIS_OK;
  }
  DeviceGuard g(ctx->device);
  hipStream_t s = as_stream(stream);
  int32_t rc;
  if ((rc = zero_counters(ctx, s))) return rc;
  if ((rc = launch_check_graph(graph->row_ptr, graph->col, graph->n_rows, graph->n_edges, n_cells,
                               &dcnt(ctx)->err, s)))
    return rc;
  if ((rc = sync_counters(ctx, s))) return rc;
  if (ctx->h_counters->err & 1u) return inval("graph row offsets are inconsistent");
  if (ctx->h_counters->err & 2u) return inval("graph targets are not cell ids");
  return run_prune(ctx, graph->row_ptr, graph->col, graph->out, n_cells, K, graph->n_edges,
                   analysis, d_kept, d_mask, n_kept, s);
}

int32_t gis_subdivide(gis_ctx* ctx, const gis_grid* grid, const gis_cells* in,
                      const uint8_t* d_kept, int32_t boundary_rule, uint8_t* d_boundary,
                      gis_cells* out, void* stream) {
  if (!ctx || !grid || !in || !out) return inval("ctx, grid, in and out are required");
  if (grid->n < 1 || grid->n > kMaxDim) return inval("grid dimension must be 1..4");
  int32_t rc;
  if ((rc = check_grid(grid, grid->n))) return rc;
  if (boundary_rule != GIS_BOUNDARY_SHELL && boundary_rule != GIS_BOUNDARY_CORNERS)
    return inval("unknown boundary rule");
  if (in->n_cells < 0 || (in->n_cells > 0 && (!in->level || !in->idx || !d_kept)))
    return inval("invalid input cell list");
  if (out->cap > 0 && (!out->level || !out->idx)) return inval("output buffers missing");
  DeviceGuard g(ctx->device);
  hipStream_t s = as_stream(stream);
  if (in->n_cells == 0) {
    out->n_cells = 0;
    return GIS_OK;
  }
  const GridArgs ga = make_grid(grid);
  int lmax = 0;
  if ((rc = list_lmax(ctx, in->level, in->n_cells, &lmax, s))) return rc;
  CoverIndex ci{};
  if ((rc = prepare_index(ctx, ga, in->level, in->idx, in->n_cells, lmax, true, ci, s))) return rc;
  uint8_t* bnd = d_boundary;
  if (!bnd) {
    if ((rc = ensure(ctx->bnd, (size_t)in->n_cells))) return rc;
    bnd = (uint8_t*)ctx->bnd.ptr;
  }
  int64_t n_new = 0, n_b = 0;
  int new_lmax = 0;
  rc = run_subdivide(ctx, ga, ci, in->level, in->idx, in->n_cells, d_kept, boundary_rule, bnd,
                     out->level, out->idx, out->cap, &n_new, &new_lmax, &n_b, s);
  out->n_cells = n_new;
  return rc;
}

int32_t gis_solve(gis_ctx* ctx, const gis_system* sys, const gis_grid* grid, const double* d_u,
                  int32_t K, int32_t rounds, const gis_opts* opts, gis_solution** out_sol,
                  void* stream) {
  if (!ctx || !out_sol) return inval("ctx and out are required");
  *out_sol = nullptr;
  int32_t rc;
  if ((rc = check_system(sys)) || (rc = check_grid(grid, sys->n)) || (rc = check_opts(opts)))
    return rc;
  if (!d_u || K < 1) return inval("inputs and K >= 1 are required");
  if (rounds < 0 || rounds >= GIS_MAX_ROUNDS) return inval("rounds must be 0..31");
  DeviceGuard dg(ctx->device);
  hipStream_t s = as_stream(stream);
  const GridArgs ga = make_grid(grid);
  const int n = sys->n;
  const int32_t W = (K + 63) / 64;
  gis_opts o = *opts;
  gis_solve_info info{};
  info.n = n;
  info.K = K;
  info.mask_words = W;

  hipEvent_t ev[4];
  for (int i = 0; i < 4; ++i) GIS_HIP(hipEventCreate(&ev[i]));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 4; ++i) (void)hipEventDestroy(e[i]);
    }
  } evg{ev};

  // round-0 covering: the full coarse grid
  int64_t n_cells = prod_n0(ga);
  if (n_cells * (int64_t)K >= ((int64_t)1 << 31)) {
    set_error("more than 2^31 - 1 rows");
    return GIS_E_UNSUPPORTED;
  }
  if ((rc = ensure(ctx->lvA, (size_t)n_cells + 16)) || (rc = ensure(ctx->ixA, (size_t)n_cells * n * 4 + 16)))
    return rc;
  if ((rc = launch_coarse(ga, (uint8_t*)ctx->lvA.ptr, (int32_t*)ctx->ixA.ptr, s))) return rc;
  int lmax = 0;

  // FP32 recheck band: calibrate on the coarse covering when not given
  if (o.precision == GIS_PREC_FP32_RECHECK) {
    bool need = false;
    for (int d = 0; d < n; ++d) need |= !(o.band[d] > 0.0);
    if (need) {
      gis_cells cc{n_cells, n_cells, (uint8_t*)ctx->lvA.ptr, (int32_t*)ctx->ixA.ptr};
      double band[kMaxDim] = {0, 0, 0, 0};
      const double floor_rel = 1e-5 * ldexp(1.0, -rounds);
      if ((rc = gis_calibrate_band(ctx, sys, grid, d_u, K, &cc, o.samples, 8.0, floor_rel, band, stream)))
        return rc;
      for (int d = 0; d < n; ++d)
        if (!(o.band[d] > 0.0)) o.band[d] = band[d];
    }
  }
  for (int d = 0; d < n; ++d) info.band[d] = o.precision == GIS_PREC_FP32_RECHECK ? o.band[d] : 0.0;

  bool cur_is_A = true;
  int64_t n_kept = 0;
  CoverIndex ci{};
  for (int r = 0; r <= rounds; ++r) {
    uint8_t* lv = (uint8_t*)(cur_is_A ? ctx->lvA.ptr : ctx->lvB.ptr);
    int32_t* ix = (int32_t*)(cur_is_A ? ctx->ixA.ptr : ctx->ixB.ptr);
    gis_round_stats& st = info.rounds[r];
    float ms_sub = 0.f;
    if (r > 0) {
      // subdivide the previous round's kept boundary cells
      const int64_t cap = n_kept << n;
      DevBuf& lvN = cur_is_A ? ctx->lvB : ctx->lvA;
      DevBuf& ixN = cur_is_A ? ctx->ixB : ctx->ixA;
      if ((rc = ensure(lvN, (size_t)cap + 16)) || (rc = ensure(ixN, (size_t)cap * n * 4 + 16))) return rc;
      if ((rc = ensure(ctx->bnd, (size_t)n_cells + 16))) return rc;
      if (ci.uniform) {  // the boundary walk needs the index arrays
        if ((rc = prepare_index(ctx, ga, lv, ix, n_cells, lmax, true, ci, s, false))) return rc;
      }
      GIS_HIP(hipEventRecord(ev[3], s));
      int64_t n_new = 0, n_b = 0;
      int new_lmax = 0;
      if ((rc = run_subdivide(ctx, ga, ci, lv, ix, n_cells, (const uint8_t*)ctx->kept.ptr,
                              o.boundary_rule, (uint8_t*)ctx->bnd.ptr, (uint8_t*)lvN.ptr,
                              (int32_t*)ixN.ptr, cap, &n_new, &new_lmax, &n_b, s)))
        return rc;
      info.rounds[r - 1].n_boundary = n_b;
      cur_is_A = !cur_is_A;
      lv = (uint8_t*)lvN.ptr;
      ix = (int32_t*)ixN.ptr;
      n_cells = n_new;
      lmax = new_lmax;
      if (n_cells == 0) break;
      if (n_cells * (int64_t)K >= ((int64_t)1 << 31)) {
        set_error("more than 2^31 - 1 rows");
        return GIS_E_UNSUPPORTED;
      }
    }
    // build
    const int64_t n_rows = n_cells * K;
    GIS_HIP(hipEventRecord(ev[0], s));
    if ((rc = prepare_index(ctx, ga, lv, ix, n_cells, lmax, false, ci, s, r == 0))) return rc;
    if ((rc = ensure(ctx->row_ptr, (size_t)(n_rows + 1) * 8)) || (rc = ensure(ctx->out, (size_t)n_rows + 16)))
      return rc;
    if (ctx->col.bytes < 16 && (rc = ensure(ctx->col, (size_t)n_rows * 4 * 8))) return rc;
    Graph gr{(int64_t*)ctx->row_ptr.ptr, (int32_t*)ctx->col.ptr, (uint8_t*)ctx->out.ptr,
             (int64_t)(ctx->col.bytes / 4), 0, 0, 0, 0.f, 0.f};
    if ((rc = run_build(ctx, sys, grid, d_u, K, ci, lv, ix, n_cells, &o, gr, s))) return rc;
    if (gr.n_edges > gr.cap_edges) {
      if ((rc = ensure(ctx->col, (size_t)gr.n_edges * 4))) return rc;
      gr.col = (int32_t*)ctx->col.ptr;
      gr.cap_edges = (int64_t)(ctx->col.bytes / 4);
      if ((rc = rerun_emit(ctx, n, ci, n_rows, gr, s))) return rc;
    }
    GIS_HIP(hipEventRecord(ev[1], s));
    // prune
    if ((rc = ensure(ctx->kept, (size_t)n_cells + 16)) || (rc = ensure(ctx->mask, (size_t)n_cells * W * 8 + 16)))
      return rc;
    if ((rc = run_prune(ctx, gr.row_ptr, gr.col, gr.out, n_cells, K, gr.n_edges, o.analysis,
                        (uint8_t*)ctx->kept.ptr, (uint64_t*)ctx->mask.ptr, &n_kept, s)))
      return rc;
    GIS_HIP(hipEventRecord(ev[2], s));
    GIS_HIP(hipEventSynchronize(ev[2]));  // run_prune synchronised: returns at once
    float ms_b = 0.f, ms_p = 0.f;
    GIS_HIP(hipEventElapsedTime(&ms_b, ev[0], ev[1]));
    GIS_HIP(hipEventElapsedTime(&ms_p, ev[1], ev[2]));
    if (r > 0) {
      GIS_HIP(hipEventElapsedTime(&ms_sub, ev[3], ev[0]));
      info.rounds[r - 1].ms_subdivide = ms_sub;
    }
    st.n_cells = n_cells;
    st.n_rows = n_rows;
    st.n_edges = gr.n_edges;
    st.n_out = gr.n_out;
    st.n_kept = n_kept;
    st.n_recheck = gr.n_recheck;
    st.max_level = lmax;
    st.ms_build = ms_b;
    st.ms_prune = ms_p;
    st.ms_image = gr.ms_image;
    st.ms_recheck = gr.ms_recheck;
    info.n_rounds = r + 1;
    if (n_kept == 0) break;
  }

  // result handle
  gis_solution* sol = new gis_solution();
  sol->device = ctx->device;
  sol->grid = ga;
  sol->K = K;
  sol->W = W;
  const int64_t nc = n_cells;
  sol->n_cells = nc;
  info.n_cells = nc;
  info.n_kept = nc > 0 ? n_kept : 0;
  sol->info = info;
  auto fail = [&](int32_t code) {
    gis_solution_free(sol);
    return code;
  };
  const uint8_t* lv = (const uint8_t*)(cur_is_A ? ctx->lvA.ptr : ctx->lvB.ptr);
  const int32_t* ix = (const int32_t*)(cur_is_A ? ctx->ixA.ptr : ctx->ixB.ptr);
  if ((rc = ensure(sol->level, (size_t)nc + 16)) || (rc = ensure(sol->idx, (size_t)nc * n * 4 + 16)) ||
      (rc = ensure(sol->kept, (size_t)nc + 16)) || (rc = ensure(sol->mask, (size_t)nc * W * 8 + 16)))
    return fail(rc);
  if (nc > 0) {
    if (hipMemcpyAsync(sol->level.ptr, lv, nc, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(sol->idx.ptr, ix, nc * n * 4, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(sol->kept.ptr, ctx->kept.ptr, nc, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(sol->mask.ptr, ctx->mask.ptr, nc * W * 8, hipMemcpyDeviceToDevice, s) != hipSuccess) {
      set_error("copy of the solution failed");
      return fail(GIS_E_HIP);
    }
    sol->ci = ci;
    if (!ci.uniform) {
      const int64_t total = ci.off[ci.lmax + 1];
      if ((rc = ensure(sol->state, (size_t)total + 16)) || (rc = ensure(sol->id, (size_t)total * 4 + 16)))
        return fail(rc);
      if (hipMemcpyAsync(sol->state.ptr, ci.state, total, hipMemcpyDeviceToDevice, s) != hipSuccess ||
          hipMemcpyAsync(sol->id.ptr, ci.id, total * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        set_error("copy of the covering index failed");
        return fail(GIS_E_HIP);
      }
      sol->ci.state = (uint8_t*)sol->state.ptr;
      sol->ci.id = (int32_t*)sol->id.ptr;
    }
  } else {
    sol->ci = ci;
    sol->ci.uniform = 0;
  }
  if (hipStreamSynchronize(s) != hipSuccess) {
    set_error("stream synchronisation failed");
    return fail(GIS_E_HIP);
  }
  *out_sol = sol;
  return GIS_OK;
}

int32_t gis_solution_info(const gis_solution* sol, gis_solve_info* info) {
  if (!sol || !info) return inval("sol and info are required");
  *info = sol->info;
  return GIS_OK;
}

int32_t gis_solution_export(const gis_solution* sol, gis_cells* cells, uint8_t* d_kept,
                            uint64_t* d_mask, void* stream) {
  if (!sol || !cells) return inval("sol and cells are required");
  if (cells->cap < sol->n_cells) {
    cells->n_cells = sol->n_cells;
    set_error("cell capacity too small");
    return GIS_E_CAPACITY;
  }
  const int64_t nc = sol->n_cells;
  cells->n_cells = nc;
  if (nc == 0) return GIS_OK;
  if (!cells->level || !cells->idx || !d_kept || !d_mask) return inval("buffers missing");
  DeviceGuard g(sol->device);
  hipStream_t s = as_stream(stream);
  GIS_HIP(hipMemcpyAsync(cells->level, sol->level.ptr, nc, hipMemcpyDeviceToDevice, s));
  GIS_HIP(hipMemcpyAsync(cells->idx, sol->idx.ptr, nc * sol->grid.n * 4, hipMemcpyDeviceToDevice, s));
  GIS_HIP(hipMemcpyAsync(d_kept, sol->kept.ptr, nc, hipMemcpyDeviceToDevice, s));
  GIS_HIP(hipMemcpyAsync(d_mask, sol->mask.ptr, nc * sol->W * 8, hipMemcpyDeviceToDevice, s));
  return GIS_OK;
}

void gis_solution_free(gis_solution* sol) {
  if (!sol) return;
  DeviceGuard g(sol->device);
  (void)hipDeviceSynchronize();
  release(sol->level);
  release(sol->idx);
  release(sol->kept);
  release(sol->mask);
  release(sol->state);
  release(sol->id);
  delete sol;
}

static int32_t query_common(const gis_solution* sol, const double* d_states, int64_t n,
                            uint8_t* member, uint64_t* adm, void* stream) {
  if (!sol) return inval("sol is NULL");
  if (n < 0 || (n > 0 && !d_states)) return inval("invalid states");
  if (n == 0) return GIS_OK;
  DeviceGuard g(sol->device);
  if (sol->n_cells == 0) {  // empty covering: nothing is a member
    hipStream_t s = as_stream(stream);
    if (member) return fill_u8(member, 0, n, s);
    return fill_i64((int64_t*)adm, 0, n * sol->W, s);
  }
  return launch_query(sol->ci, sol->grid, (const uint8_t*)sol->kept.ptr,
                      (const uint64_t*)sol->mask.ptr, sol->W, d_states, n, member, adm,
                      as_stream(stream));
}

int32_t gis_query_membership(const gis_solution* sol, const double* d_states, int64_t n,
                             uint8_t* d_member, void* stream) {
  if (n > 0 && !d_member) return inval("d_member is NULL");
  return query_common(sol, d_states, n, d_member, nullptr, stream);
}

int32_t gis_query_admissible(const gis_solution* sol, const double* d_states, int64_t n,
                             uint64_t* d_mask_out, void* stream) {
  if (n > 0 && !d_mask_out) return inval("d_mask_out is NULL");
  return query_common(sol, d_states, n, nullptr, d_mask_out, stream);
}

int32_t gis_images(gis_ctx* ctx, const gis_system* sys, const gis_grid* grid, const double* d_u,
                   int32_t K, const gis_cells* cells, int32_t samples, int32_t precision,
                   double* d_images, void* stream) {
  if (!ctx) return inval("ctx is NULL");
  int32_t rc;
  if ((rc = check_system(sys)) || (rc = check_grid(grid, sys->n))) return rc;
  if (!cells || !d_u || K < 1 || (cells->n_cells > 0 && !d_images)) return inval("missing arguments");
  if (samples != GIS_SAMPLES_LATTICE3 && samples != GIS_SAMPLES_CORNERS_CENTER)
    return inval("unknown sample scheme");
  if (precision != GIS_PREC_FP64 && precision != GIS_PREC_FP32_RECHECK) return inval("unknown precision");
  DeviceGuard g(ctx->device);
  gis_opts o{};
  o.samples = samples;
  CoverIndex ci{};
  BuildArgs a = make_build_args(ctx, sys, grid, d_u, K, ci, cells->level, cells->idx,
                                cells->n_cells, &o);
  return launch_images(a, precision, d_images, as_stream(stream));
}

int32_t gis_calibrate_band(gis_ctx* ctx, const gis_system* sys, const gis_grid* grid,
                           const double* d_u, int32_t K, const gis_cells* cells, int32_t samples,
                           double safety, double floor_rel, double* band_out, void* stream) {
  if (!ctx || !band_out) return inval("ctx and band_out are required");
  int32_t rc;
  if ((rc = check_system(sys)) || (rc = check_grid(grid, sys->n))) return rc;
  if (!cells || !d_u || K < 1) return inval("missing arguments");
  if (samples != GIS_SAMPLES_LATTICE3 && samples != GIS_SAMPLES_CORNERS_CENTER)
    return inval("unknown sample scheme");
  DeviceGuard g(ctx->device);
  hipStream_t s = as_stream(stream);
  gis_opts o{};
  o.samples = samples;
  CoverIndex ci{};
  if ((rc = zero_counters(ctx, s))) return rc;
  BuildArgs a = make_build_args(ctx, sys, grid, d_u, K, ci, cells->level, cells->idx,
                                cells->n_cells, &o);
  if ((rc = launch_calibrate(a, dcnt(ctx)->maxerr, s))) return rc;
  if ((rc = sync_counters(ctx, s))) return rc;
  const GridArgs ga = make_grid(grid);
  for (int d = 0; d < sys->n; ++d) {
    double e;
    memcpy(&e, &ctx->h_counters->maxerr[d], 8);
    const double fl = floor_rel * ga.w0[d];
    const double b = safety * e;
    band_out[d] = b > fl ? b : fl;
  }
  return GIS_OK;
}

}  // extern "C"
