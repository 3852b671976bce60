// Graph construction kernels: symbolic image of a covering (Sec. 2.2,
// Definition 1) as CSR rows, one row per (cell, input).
//
//   count   : per row, the images of the sample points (nsub RK4 substeps),
//             their bounding box, the closed index range of finest-level
//             cells it meets, the OUT flag and the row's edge count; one
//             int64 edge total per block of kRowBlock rows.
//   recheck : FP64 redo of the rows the FP32 count kernel could not decide.
//   emit    : block-local scan of the counts plus the block offset -> row_ptr;
//             the row's target ids are enumerated into an LDS tile and copied
//             to col[] with coalesced stores.
//
// Cell ids follow the canonical order of the covering (level, then row-major
// index), so enumerating the covering index level by level, row-major inside
// each level, yields every row's targets in ascending order with no sort and
// no duplicates.
#include <float.h>
#include <math.h>

#include "dynamics.h"
#include "gis_internal.h"

namespace gis {

namespace {

constexpr int kTile = 8192;  // LDS tile of the emitter (int32 ids, 32 KiB)

// ------------------------------------------------------------------ cover logic
// Position of v on the finest grid, clamped to [-2, N + 2] (the clamp keeps
// the integer conversion defined and never changes a clamped range).
__device__ __forceinline__ double grid_pos(double v, double lo, double hs, int32_t N) {
  double t = (v - lo) / hs;
  t = t < -2.0 ? -2.0 : t;
  t = t > (double)N + 2.0 ? (double)N + 2.0 : t;
  return t;
}

template <int N>
struct Ranges {
  int32_t lo[N], hi[N];     // closed range R
  int32_t ilo[N], ihi[N];   // interior range (R when the interior range is empty)
  bool empty, iempty, outx;
};

template <int N>
__device__ __forceinline__ Ranges<N> ranges_of(const GridArgs& g, const CoverIndex& ci,
                                               const double* bl, const double* bh) {
  Ranges<N> r;
  r.empty = r.iempty = r.outx = false;
  const int L = ci.lmax;
#pragma unroll
  for (int d = 0; d < N; ++d) {
    const int32_t Nd = ci.dims[L][d];
    const double hs = ldexp(g.w0[d], -L);
    const double ta = grid_pos(bl[d], g.lo[d], hs, Nd);
    const double tb = grid_pos(bh[d], g.lo[d], hs, Nd);
    int32_t rlo = (int32_t)ceil(ta) - 1, rhi = (int32_t)floor(tb);
    int32_t ilo = (int32_t)floor(ta), ihi = (int32_t)ceil(tb) - 1;
    rlo = rlo < 0 ? 0 : rlo;
    rhi = rhi > Nd - 1 ? Nd - 1 : rhi;
    ilo = ilo < 0 ? 0 : ilo;
    ihi = ihi > Nd - 1 ? Nd - 1 : ihi;
    if (ilo > ihi) {
      ilo = rlo;
      ihi = rhi;
    }
    r.lo[d] = rlo;
    r.hi[d] = rhi;
    r.ilo[d] = ilo;
    r.ihi[d] = ihi;
    r.empty |= rlo > rhi;
    r.iempty |= ilo > ihi;
    r.outx |= (bl[d] < g.lo[d]) || (bh[d] > g.hi[d]);
  }
  return r;
}

// Visits the slots of the covering index met by the finest-level box
// [lo, hi], level by level (coarse to fine), row-major inside a level:
// f(level, slot, state) returns false to stop early.  Below level 0 only the
// children of REFINED slots can hold leaves or holes, so each level is
// restricted to the box spanned by the children of the REFINED slots seen one
// level up, and the walk ends at the first level without a REFINED slot.  The
// visiting order (level-major, row-major) is the canonical id order.
template <int N, typename F>
__device__ __forceinline__ void walk_levels(const CoverIndex& ci, const int32_t* lo,
                                            const int32_t* hi, F&& f) {
  int32_t plo[N], phi[N];  // REFINED bounding box one level up
  for (int L = 0; L <= ci.lmax; ++L) {
    const int s = ci.lmax - L;
    int32_t blo[N], bhi[N], k[N], nlo[N], nhi[N];
    bool empty = false;
#pragma unroll
    for (int d = 0; d < N; ++d) {
      blo[d] = lo[d] >> s;
      bhi[d] = hi[d] >> s;
      if (L > 0) {
        blo[d] = blo[d] > 2 * plo[d] ? blo[d] : 2 * plo[d];
        bhi[d] = bhi[d] < 2 * phi[d] + 1 ? bhi[d] : 2 * phi[d] + 1;
      }
      empty |= blo[d] > bhi[d];
      k[d] = blo[d];
      nlo[d] = 0x7fffffff;
      nhi[d] = -1;
    }
    if (empty) return;
    bool refined = false;
    const int64_t base = ci.off[L];
    for (;;) {
      int64_t lin = 0;
#pragma unroll
      for (int d = 0; d < N; ++d) lin = lin * ci.dims[L][d] + k[d];
      const uint8_t st = ci.state[base + lin];
      if (!f(L, base + lin, st)) return;
      if (st == ST_REFINED) {
        refined = true;
#pragma unroll
        for (int d = 0; d < N; ++d) {
          nlo[d] = k[d] < nlo[d] ? k[d] : nlo[d];
          nhi[d] = k[d] > nhi[d] ? k[d] : nhi[d];
        }
      }
      int d = N - 1;
      while (d >= 0 && k[d] == bhi[d]) {
        k[d] = blo[d];
        --d;
      }
      if (d < 0) break;
      ++k[d];
    }
    if (!refined) return;
#pragma unroll
    for (int d = 0; d < N; ++d) {
      plo[d] = nlo[d];
      phi[d] = nhi[d];
    }
  }
}

template <int N>
__device__ __forceinline__ bool has_hole(const CoverIndex& ci, const Ranges<N>& r) {
  if (ci.uniform || r.iempty) return false;
  bool hole = false;
  walk_levels<N>(ci, r.ilo, r.ihi, [&](int, int64_t, uint8_t st) {
    if (st == ST_HOLE) {
      hole = true;
      return false;
    }
    return true;
  });
  return hole;
}

template <int N>
__device__ __forceinline__ int32_t count_targets(const CoverIndex& ci, const Ranges<N>& r) {
  if (r.empty) return 0;
  if (ci.uniform) {
    int32_t c = 1;
#pragma unroll
    for (int d = 0; d < N; ++d) c *= r.hi[d] - r.lo[d] + 1;
    return c;
  }
  int32_t c = 0;
  walk_levels<N>(ci, r.lo, r.hi, [&](int, int64_t, uint8_t st) {
    c += st == ST_LEAF;
    return true;
  });
  return c;
}

// Writes the cover decision of global row g of job J; returns its edge count.
template <int N>
__device__ __forceinline__ int32_t decide_row(const BuildArgs& a, const Job& J,
                                              const CoverIndex& ci, int64_t g, bool finite,
                                              const double* bl, const double* bh) {
  int32_t count = 0;
  bool out = true;
  int32_t* rg = a.rng + g * (2 * N);
  if (finite) {
    const Ranges<N> rr = ranges_of<N>(J.grid, ci, bl, bh);
    out = rr.outx || has_hole<N>(ci, rr);
    count = count_targets<N>(ci, rr);
    if (a.fast_out && out) count = 0;
#pragma unroll
    for (int d = 0; d < N; ++d) {
      rg[2 * d] = rr.lo[d];
      rg[2 * d + 1] = rr.hi[d];
    }
  }
  a.cnt[g] = count;
  a.out[g] = out ? 1 : 0;
  return count;
}

// Bounding box of the sample images of local row lr of job J, in precision R.
template <int KIND, int N, typename R>
__device__ __forceinline__ bool row_bbox(const BuildArgs& a, const Job& J, const Rk4Consts<R>& kc,
                                         int64_t lr, R* bl, R* bh) {
  const int64_t c = lr / a.K;
  const int32_t j = (int32_t)(lr - c * a.K);
  const int64_t gc = J.cell_off + c;
  const int level = a.level[gc];
  int32_t ci[N];
#pragma unroll
  for (int d = 0; d < N; ++d) ci[d] = a.idx[gc * N + d];
  const int m = J.sys.m;
  R u[2];
  u[0] = R(J.u[(int64_t)j * m]);
  u[1] = m > 1 ? R(J.u[(int64_t)j * m + 1]) : R(0);
  bool finite = true;
#pragma unroll
  for (int d = 0; d < N; ++d) {
    bl[d] = R(INFINITY);
    bh[d] = R(-INFINITY);
  }
  const int S = num_samples(a.samples, N);
  for (int q = 0; q < S; ++q) {
    int k[N];
    double xd[N];
    sample_offsets<N>(a.samples, q, k);
    sample_point<N>(J.grid, level, ci, k, xd);
    R x[N];
#pragma unroll
    for (int d = 0; d < N; ++d) x[d] = R(xd[d]);
    rk4<KIND, N, R>(kc, m, J.sys.nsub, x, u);
#pragma unroll
    for (int d = 0; d < N; ++d) {
      finite &= isfinite(x[d]);
      bl[d] = x[d] < bl[d] ? x[d] : bl[d];
      bh[d] = x[d] > bh[d] ? x[d] : bh[d];
    }
  }
  return finite;
}

__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t* lds) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  int64_t t = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += lds[w];
  return t;
}

// ------------------------------------------------------------------ kernels
// One thread per (cell, input) row; a block never straddles two jobs.
template <int KIND, int N>
__global__ __launch_bounds__(kRowBlock) void k_count_f64(BuildArgs a) {
  __shared__ int64_t lds[kRowBlock / 64];
  __shared__ CoverIndex ci;
  const int32_t jb = job_of_block(a.jobs, a.n_jobs, LK_ROWS, blockIdx.x);
  const Job& J = a.jobs[jb];
  stage_index(&ci, &J.ci);
  const int64_t lr = (blockIdx.x - J.blk[LK_ROWS]) * kRowBlock + threadIdx.x;
  int64_t mine = 0;
  if (lr < J.n_cells * a.K) {
    const Rk4Consts<double> kc = make_consts<double>(J.sys);
    double bl[N], bh[N];
    const bool finite = row_bbox<KIND, N, double>(a, J, kc, lr, bl, bh);
    mine = decide_row<N>(a, J, ci, J.cell_off * a.K + lr, finite, bl, bh);
  }
  const int64_t t = block_sum_i64(mine, lds);
  if (threadIdx.x == 0) a.bsum[blockIdx.x] = t;
}

// FP32 images; a row is decided from its FP32 box only when every decision
// taken from a box extreme (the finest-grid position's floor/ceil, the
// comparisons with lo and hi) is the same anywhere within band[d] of it.
// Since |y32 - y64| <= band[d] holds for every sample image, and min/max are
// 1-Lipschitz, the FP64 box extremes then lead to the same decisions.
// Other rows are queued for the FP64 recheck kernel.
template <int KIND, int N>
__global__ __launch_bounds__(kRowBlock) void k_count_f32(BuildArgs a) {
  __shared__ int64_t lds[kRowBlock / 64];
  __shared__ CoverIndex ci;
  const int32_t jb = job_of_block(a.jobs, a.n_jobs, LK_ROWS, blockIdx.x);
  const Job& J = a.jobs[jb];
  stage_index(&ci, &J.ci);
  const int64_t lr = (blockIdx.x - J.blk[LK_ROWS]) * kRowBlock + threadIdx.x;
  int64_t mine = 0;
  if (lr < J.n_cells * a.K) {
    const int64_t g = J.cell_off * a.K + lr;
    const Rk4Consts<float> kc = make_consts<float>(J.sys);
    float bl[N], bh[N];
    bool safe = row_bbox<KIND, N, float>(a, J, kc, lr, bl, bh);
    double dl[N], dh[N];
    const int L = ci.lmax;
#pragma unroll
    for (int d = 0; d < N; ++d) {
      dl[d] = (double)bl[d];
      dh[d] = (double)bh[d];
      const double hs = ldexp(J.grid.w0[d], -L);
      const double eps = J.band[d];
      const double ta = (dl[d] - J.grid.lo[d]) / hs;
      const double tb = (dh[d] - J.grid.lo[d]) / hs;
      const double tola = eps / hs + 1e-9 * (fabs(ta) + 1.0);
      const double tolb = eps / hs + 1e-9 * (fabs(tb) + 1.0);
      safe &= fabs(ta - rint(ta)) > tola;
      safe &= fabs(tb - rint(tb)) > tolb;
      safe &= fabs(dh[d] - J.grid.hi[d]) > eps;
    }
    if (safe) {
      mine = decide_row<N>(a, J, ci, g, true, dl, dh);
    } else {
      const unsigned long long slot = atomicAdd((unsigned long long*)a.n_recheck, 1ull);
      a.recheck[slot] = g;
      a.cnt[g] = 0;
      atomicAdd(&a.stats[jb].n_recheck, 1ull);
    }
  }
  const int64_t t = block_sum_i64(mine, lds);
  if (threadIdx.x == 0) a.bsum[blockIdx.x] = t;
}

template <int KIND, int N>
__global__ __launch_bounds__(kRowBlock) void k_recheck(BuildArgs a) {
  const int64_t n = *a.n_recheck;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = a.recheck[i];
    const int32_t jb = job_of_row(a.jobs, a.n_jobs, a.K, g);
    const Job& J = a.jobs[jb];
    const int64_t lr = g - J.cell_off * a.K;
    const Rk4Consts<double> kc = make_consts<double>(J.sys);
    double bl[N], bh[N];
    const bool finite = row_bbox<KIND, N, double>(a, J, kc, lr, bl, bh);
    const int32_t c = decide_row<N>(a, J, J.ci, g, finite, bl, bh);
    if (c)
      atomicAdd((unsigned long long*)&a.bsum[J.blk[LK_ROWS] + lr / kRowBlock],
                (unsigned long long)c);
  }
}

template <int KIND, int N, typename R>
__global__ __launch_bounds__(kRowBlock) void k_images(BuildArgs a, double* out) {
  const int32_t jb = job_of_block(a.jobs, a.n_jobs, LK_ROWS, blockIdx.x);
  const Job& J = a.jobs[jb];
  const int64_t lr = (blockIdx.x - J.blk[LK_ROWS]) * kRowBlock + threadIdx.x;
  if (lr >= J.n_cells * a.K) return;
  const int64_t g = J.cell_off * a.K + lr;
  const Rk4Consts<R> kc = make_consts<R>(J.sys);
  const int64_t c = lr / a.K;
  const int32_t j = (int32_t)(lr - c * a.K);
  const int64_t gc = J.cell_off + c;
  int32_t ci[N];
#pragma unroll
  for (int d = 0; d < N; ++d) ci[d] = a.idx[gc * N + d];
  const int m = J.sys.m;
  R u[2];
  u[0] = R(J.u[(int64_t)j * m]);
  u[1] = m > 1 ? R(J.u[(int64_t)j * m + 1]) : R(0);
  const int S = num_samples(a.samples, N);
  for (int q = 0; q < S; ++q) {
    int k[N];
    double xd[N];
    sample_offsets<N>(a.samples, q, k);
    sample_point<N>(J.grid, a.level[gc], ci, k, xd);
    R x[N];
#pragma unroll
    for (int d = 0; d < N; ++d) x[d] = R(xd[d]);
    rk4<KIND, N, R>(kc, m, J.sys.nsub, x, u);
#pragma unroll
    for (int d = 0; d < N; ++d) out[(g * S + q) * N + d] = (double)x[d];
  }
}

// max |y32 - y64| per dimension (bit patterns of non-negative doubles order
// like the values, so an integer atomicMax works).
template <int KIND, int N>
__global__ __launch_bounds__(kRowBlock) void k_calibrate(BuildArgs a, unsigned long long* maxerr) {
  const int32_t jb = job_of_block(a.jobs, a.n_jobs, LK_ROWS, blockIdx.x);
  const Job& J = a.jobs[jb];
  const int64_t lr = (blockIdx.x - J.blk[LK_ROWS]) * kRowBlock + threadIdx.x;
  double e[N];
#pragma unroll
  for (int d = 0; d < N; ++d) e[d] = 0.0;
  if (lr < J.n_cells * a.K) {
    const Rk4Consts<double> k64 = make_consts<double>(J.sys);
    const Rk4Consts<float> k32 = make_consts<float>(J.sys);
    const int64_t c = lr / a.K;
    const int32_t j = (int32_t)(lr - c * a.K);
    const int64_t gc = J.cell_off + c;
    int32_t ci[N];
#pragma unroll
    for (int d = 0; d < N; ++d) ci[d] = a.idx[gc * N + d];
    const int m = J.sys.m;
    double u64[2];
    float u32[2];
    u64[0] = J.u[(int64_t)j * m];
    u64[1] = m > 1 ? J.u[(int64_t)j * m + 1] : 0.0;
    u32[0] = (float)u64[0];
    u32[1] = (float)u64[1];
    const int S = num_samples(a.samples, N);
    for (int q = 0; q < S; ++q) {
      int k[N];
      double xd[N];
      float xf[N];
      sample_offsets<N>(a.samples, q, k);
      sample_point<N>(J.grid, a.level[gc], ci, k, xd);
#pragma unroll
      for (int d = 0; d < N; ++d) xf[d] = (float)xd[d];
      rk4<KIND, N, double>(k64, m, J.sys.nsub, xd, u64);
      rk4<KIND, N, float>(k32, m, J.sys.nsub, xf, u32);
#pragma unroll
      for (int d = 0; d < N; ++d) {
        double diff = fabs((double)xf[d] - xd[d]);
        if (!(diff <= DBL_MAX)) diff = DBL_MAX;  // non-finite images force the largest band
        e[d] = diff > e[d] ? diff : e[d];
      }
    }
  }
#pragma unroll
  for (int d = 0; d < N; ++d) {
    double v = e[d];
    for (int o = 32; o > 0; o >>= 1) {
      const double w = __shfl_down(v, o, 64);
      v = w > v ? w : v;
    }
    if ((threadIdx.x & 63) == 0)
      atomicMax(&maxerr[jb * kMaxDim + d], (unsigned long long)__double_as_longlong(v));
  }
}

// ------------------------------------------------------------------ emit
template <int N>
__global__ __launch_bounds__(kRowBlock) void k_emit(EmitArgs a) {
  __shared__ int32_t tile[kTile];
  __shared__ int64_t wsum[kRowBlock / 64];
  __shared__ CoverIndex ci;
  const int32_t jb = job_of_block(a.jobs, a.n_jobs, LK_ROWS, blockIdx.x);
  const Job& J = a.jobs[jb];
  stage_index(&ci, &J.ci);
  const int64_t lr = (blockIdx.x - J.blk[LK_ROWS]) * kRowBlock + threadIdx.x;
  const bool live = lr < J.n_cells * a.K;
  const int64_t g = J.cell_off * a.K + lr;
  const int32_t c = live ? a.cnt[g] : 0;
  // block-exclusive scan of the counts
  int64_t x = c;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  int64_t before = 0, total = 0;
  for (int w = 0; w < kRowBlock / 64; ++w) {
    before += w < wid ? wsum[w] : 0;
    total += wsum[w];
  }
  const int64_t off = before + x - c;
  const int64_t base = a.bscan[blockIdx.x];
  if (live) a.row_ptr[g] = base + off;
  if (live && g == a.total_rows - 1) a.row_ptr[a.total_rows] = base + off + c;
  if (base + total > a.cap_edges) return;  // capacity miss: col is not written
  const bool staged = total <= kTile;
  if (c > 0) {
    const int32_t* rg = a.rng + g * (2 * N);
    int32_t lo[N], hi[N];
#pragma unroll
    for (int d = 0; d < N; ++d) {
      lo[d] = rg[2 * d];
      hi[d] = rg[2 * d + 1];
    }
    int32_t* dst = staged ? tile + off : a.col + base + off;
    const int32_t id0 = (int32_t)J.cell_off;
    int32_t w = 0;
    if (ci.uniform) {
      int32_t k[N];
#pragma unroll
      for (int d = 0; d < N; ++d) k[d] = lo[d];
      for (;;) {
        int32_t lin = 0;
#pragma unroll
        for (int d = 0; d < N; ++d) lin = lin * ci.dims[0][d] + k[d];
        if (w < c) dst[w++] = id0 + lin;
        int d = N - 1;
        while (d >= 0 && k[d] == hi[d]) {
          k[d] = lo[d];
          --d;
        }
        if (d < 0) break;
        ++k[d];
      }
    } else {
      walk_levels<N>(ci, lo, hi, [&](int, int64_t slot, uint8_t st) {
        if (st == ST_LEAF && w < c) dst[w++] = id0 + ci.id[slot];
        return true;
      });
    }
  }
  if (staged) {
    __syncthreads();
    for (int64_t i = threadIdx.x; i < total; i += kRowBlock) a.col[base + i] = tile[i];
  }
}

__global__ void k_job_edges(const Job* jobs, int32_t n_jobs, int32_t K, const int64_t* row_ptr,
                            JobStats* stats) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_jobs) return;
  const int64_t r0 = jobs[j].cell_off * K, r1 = (jobs[j].cell_off + jobs[j].n_cells) * K;
  stats[j].n_edges = r1 > r0 ? row_ptr[r1] - row_ptr[r0] : 0;
}

__global__ void k_count_out(const uint8_t* out, int64_t n, unsigned long long* cnt) {
  unsigned long long mine = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    mine += out[i];
  for (int o = 32; o > 0; o >>= 1) mine += __shfl_down(mine, o, 64);
  if ((threadIdx.x & 63) == 0 && mine) atomicAdd(cnt, mine);
}

// ------------------------------------------------------------------ dispatch
template <template <int, int> class Launcher, typename... Args>
int32_t dispatch_sys(int kind, int n, Args&&... args) {
  switch (kind) {
    case GIS_SYS_VDP:
      if (n == 2) return Launcher<GIS_SYS_VDP, 2>::run(args...);
      break;
    case GIS_SYS_LORENZ:
      if (n == 3) return Launcher<GIS_SYS_LORENZ, 3>::run(args...);
      break;
    case GIS_SYS_VDP2:
      if (n == 4) return Launcher<GIS_SYS_VDP2, 4>::run(args...);
      break;
    case GIS_SYS_LINEAR:
      if (n == 1) return Launcher<GIS_SYS_LINEAR, 1>::run(args...);
      if (n == 2) return Launcher<GIS_SYS_LINEAR, 2>::run(args...);
      if (n == 3) return Launcher<GIS_SYS_LINEAR, 3>::run(args...);
      if (n == 4) return Launcher<GIS_SYS_LINEAR, 4>::run(args...);
      break;
  }
  set_error("unsupported system kind / dimension");
  return GIS_E_UNSUPPORTED;
}

template <int KIND, int N>
struct CountF64 {
  static int32_t run(const BuildArgs& a, hipStream_t s) {
    if (a.n_blocks == 0) return GIS_OK;
    hipLaunchKernelGGL((k_count_f64<KIND, N>), dim3((unsigned)a.n_blocks), dim3(kRowBlock), 0, s, a);
    GIS_LAUNCH_CHECK("k_count_f64");
    return GIS_OK;
  }
};
template <int KIND, int N>
struct CountF32 {
  static int32_t run(const BuildArgs& a, hipStream_t s) {
    if (a.n_blocks == 0) return GIS_OK;
    hipLaunchKernelGGL((k_count_f32<KIND, N>), dim3((unsigned)a.n_blocks), dim3(kRowBlock), 0, s, a);
    GIS_LAUNCH_CHECK("k_count_f32");
    return GIS_OK;
  }
};
template <int KIND, int N>
struct Recheck {
  static int32_t run(const BuildArgs& a, hipStream_t s) {
    if (a.n_blocks == 0) return GIS_OK;
    const unsigned nb = a.n_blocks < 2048 ? (unsigned)a.n_blocks : 2048u;
    hipLaunchKernelGGL((k_recheck<KIND, N>), dim3(nb), dim3(kRowBlock), 0, s, a);
    GIS_LAUNCH_CHECK("k_recheck");
    return GIS_OK;
  }
};
template <int KIND, int N>
struct Images {
  static int32_t run(const BuildArgs& a, int32_t precision, double* out, hipStream_t s) {
    if (a.n_blocks == 0) return GIS_OK;
    if (precision == GIS_PREC_FP32_RECHECK)
      hipLaunchKernelGGL((k_images<KIND, N, float>), dim3((unsigned)a.n_blocks), dim3(kRowBlock), 0, s, a, out);
    else
      hipLaunchKernelGGL((k_images<KIND, N, double>), dim3((unsigned)a.n_blocks), dim3(kRowBlock), 0, s, a, out);
    GIS_LAUNCH_CHECK("k_images");
    return GIS_OK;
  }
};
template <int KIND, int N>
struct Calibrate {
  static int32_t run(const BuildArgs& a, unsigned long long* maxerr, hipStream_t s) {
    if (a.n_blocks == 0) return GIS_OK;
    hipLaunchKernelGGL((k_calibrate<KIND, N>), dim3((unsigned)a.n_blocks), dim3(kRowBlock), 0, s, a, maxerr);
    GIS_LAUNCH_CHECK("k_calibrate");
    return GIS_OK;
  }
};

template <int N>
int32_t emit_n(const EmitArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_emit<N>), dim3((unsigned)a.n_blocks), dim3(kRowBlock), 0, s, a);
  GIS_LAUNCH_CHECK("k_emit");
  return GIS_OK;
}

}  // namespace

int32_t launch_count(const BuildArgs& a, int32_t precision, hipStream_t s) {
  if (precision == GIS_PREC_FP32_RECHECK) return dispatch_sys<CountF32>(a.kind, a.n, a, s);
  return dispatch_sys<CountF64>(a.kind, a.n, a, s);
}

int32_t launch_recheck(const BuildArgs& a, hipStream_t s) {
  return dispatch_sys<Recheck>(a.kind, a.n, a, s);
}

int32_t launch_images(const BuildArgs& a, int32_t precision, double* d_images, hipStream_t s) {
  return dispatch_sys<Images>(a.kind, a.n, a, precision, d_images, s);
}

int32_t launch_calibrate(const BuildArgs& a, unsigned long long* d_maxerr, hipStream_t s) {
  return dispatch_sys<Calibrate>(a.kind, a.n, a, d_maxerr, s);
}

int32_t launch_emit(const EmitArgs& a, hipStream_t s) {
  if (a.n_blocks == 0) return GIS_OK;
  switch (a.n) {
    case 1: return emit_n<1>(a, s);
    case 2: return emit_n<2>(a, s);
    case 3: return emit_n<3>(a, s);
    case 4: return emit_n<4>(a, s);
  }
  set_error("unsupported dimension");
  return GIS_E_UNSUPPORTED;
}

int32_t launch_job_edges(const Job* jobs, int32_t n_jobs, int32_t K, const int64_t* row_ptr,
                         JobStats* stats, hipStream_t s) {
  if (n_jobs == 0) return GIS_OK;
  hipLaunchKernelGGL(k_job_edges, dim3((n_jobs + 63) / 64), dim3(64), 0, s, jobs, n_jobs, K,
                     row_ptr, stats);
  GIS_LAUNCH_CHECK("k_job_edges");
  return GIS_OK;
}

int32_t count_out(const uint8_t* out, int64_t n, unsigned long long* d_count, hipStream_t s) {
  if (n == 0) return GIS_OK;
  int64_t nb = (n + 255) / 256;
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_count_out, dim3((unsigned)nb), dim3(256), 0, s, out, n, d_count);
  GIS_LAUNCH_CHECK("k_count_out");
  return GIS_OK;
}

}  // namespace gis
