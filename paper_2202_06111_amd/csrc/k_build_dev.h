// Graph construction: the symbolic image of a covering (Sec. 2.2,
// Definition 1) as CSR rows, one row per (cell, input), in one pass.  The
// device part: k_build.hip instantiates these kernels for the built-in fields
// and launches them; the runtime compiler instantiates them for a user field
// (rtc.hip).
//
// k_build, one thread per row, a block of kRowBlock consecutive rows:
//   1. images of the sample points (nsub RK4 substeps) and their bounding box,
//      in FP64, or in FP32 with the row redone in FP64 when a decision taken
//      from its box is not safe within the recheck band;
//   2. the closed index range of finest-level cells the box meets, the OUT
//      flag, and the row's edge count from a walk of the covering index (the
//      first few target ids are kept in LDS for step 5);
//   3. a block-wide exclusive scan of the counts;
//   4. the block's global edge offset by decoupled look-back: blocks take
//      their index from an atomic ticket, publish their edge total, and the
//      first wave sums the totals of the blocks before it 64 at a time until
//      it meets one that has published its inclusive prefix;
//   5. row_ptr, and the target ids: on full level-0 grids written into an LDS
//      tile and copied to col with coalesced stores, tile by tile; on
//      refined coverings stored by each row directly (consecutive rows' ids
//      are adjacent in col, so the L2 cache merges them into whole lines; a
//      tile measured 8% slower there, coupled Van der Pol round 2, while on
//      the uniform Lorenz-type grid direct stores were 40% slower).
//
// Cell ids follow the canonical order of the covering (level, then row-major
// index), so enumerating the covering index level by level, row-major inside
// each level, yields every row's targets in ascending order with no sort and
// no duplicates.
#pragma once

#ifndef __HIPCC_RTC__
#include <float.h>
#include <math.h>
#else
#define DBL_MAX 1.7976931348623157e308
#define INFINITY __builtin_huge_valf()
#endif

#include "dynamics.h"
#include "gis_internal.h"

namespace gis {
namespace kbuild {

constexpr int kTile = 4096;   // LDS staging tile of the emitter (int32 ids, 16 KiB)
// Runs of target ids kept in LDS per row between count and emit: 16 for
// three- and four-dimensional fields (their finer boxes have more runs; on
// the coupled Van der Pol last round 16 instead of 8 saved 1% of the FP32
// build and 4% of the FP64 one), 8 for smaller ones, whose kernels also
// keep the emit's staging area in LDS.
template <int N>
constexpr int cache_runs() {
  return N > 2 ? 16 : 8;
}
constexpr int kStage = 512;   // ids a wave stages in LDS per coalesced store pass (refined coverings)

// Orders one wave's LDS writes before its lanes' later reads (and reads
// before later writes): the wave's memory operations at wavefront scope, no
// block barrier.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Look-back words: the launch's epoch in bits 40-63, a status in bits 38-39
// and an edge total in bits 0-37.  A word written by an earlier launch
// carries another epoch and reads as "not yet published".
constexpr uint64_t kLbAgg = 1ull << 38;   // the block's own total
constexpr uint64_t kLbInc = 2ull << 38;   // total of this block and all before it
constexpr uint64_t kLbVal = (1ull << 38) - 1;
__device__ __forceinline__ uint32_t lb_status(uint64_t w, uint32_t epoch) {
  return (uint32_t)(w >> 40) == epoch ? (uint32_t)(w >> 38) & 3u : 0u;
}

// ------------------------------------------------------------------ cover logic
// Position t = (v - lo) / hs of v on the finest grid, clamped to [-2, N + 2]
// (the clamp keeps the integer conversion defined and never changes a
// clamped range).
__device__ __forceinline__ double clamp_pos(double t, int32_t N) {
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
    const double ta = clamp_pos((bl[d] - g.lo[d]) / hs, Nd);
    const double tb = clamp_pos((bh[d] - g.lo[d]) / hs, Nd);
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

// Visits the runs of index slots met by the finest-level box [lo, hi]: for
// every level L (coarse to fine) and every row of the box at that level (all
// coordinates but the last fixed, row-major), the slots a .. b of that row
// between the box's first and last column.  Per run f(p0, p1, inner, q0, q1)
// gets the prefix counts P[a] and P[b+1] and, when the row lies in the
// interior box [ilo, ihi] (and `interior` is set), the prefix counts at that
// box's first column and one past its last; f returns false to stop.
// Level-major, row-major order is the canonical id order, so the leaves come
// out ascending.  The cost is one call per row of the box and level, whatever
// the box's width and however the covering is refined inside it; the loads
// of kRuns runs are issued together.  The walk ends after a level whose slots
// in the box are all leaves or holes: the slots below a leaf or a hole hold
// neither, so the finer levels would add nothing (a row of a coarse cell
// whose box lies in a coarse region stops after a few runs instead of
// visiting every row of its box at the finest level).
constexpr int kRuns = 2;
constexpr int64_t kLo32 = 0xffffffffll;  // the leaf half of a prefix word

template <int N, typename F>
__device__ __forceinline__ void walk_runs(const CoverIndex& ci, const int32_t* lo,
                                          const int32_t* hi, const int32_t* ilo,
                                          const int32_t* ihi, bool interior, F&& f) {
  // the index lives in global memory; its pointer comes from the block's
  // LDS copy of the index description, so say so (global loads instead of
  // flat ones, whose waits would also hold the LDS traffic of the walk)
  const int64_t __attribute__((address_space(1)))* P =
      (const int64_t __attribute__((address_space(1)))*)ci.pfx;
  for (int L = 0; L <= ci.lmax; ++L) {
    const int s = ci.lmax - L;
    // the box and its interior at this level; the rows of the box (all
    // coordinates but the last) are enumerated by an odometer k, and a
    // pointer to the row's first slot follows it by additions: jump[d] is
    // the pointer's move when the odometer's carry stops at coordinate d
    // (d increments, the coordinates after it wrap back to the box's start)
    int32_t blo[N], bhi[N], il[N], ih[N], k[N];
    int64_t st[N];
#pragma unroll
    for (int d = 0; d < N; ++d) {
      blo[d] = lo[d] >> s;
      bhi[d] = hi[d] >> s;
      il[d] = ilo[d] >> s;
      ih[d] = ihi[d] >> s;
      k[d] = blo[d];
    }
    st[N - 1] = 1;
#pragma unroll
    for (int d = N - 2; d >= 0; --d) st[d] = st[d + 1] * ci.dims[L][d + 1];
    int64_t row = ci.off[L];
    int64_t nrows = 1;
    int64_t slots = bhi[N - 1] - blo[N - 1] + 1;  // slots of the box at this level
    int64_t jump[N] = {};
    int64_t back = 0;  // the moves that wrap the coordinates after d
#pragma unroll
    for (int d = N - 2; d >= 0; --d) {
      jump[d] = st[d] - back;
      back += (int64_t)(bhi[d] - blo[d]) * st[d];
    }
#pragma unroll
    for (int d = 0; d < N - 1; ++d) {
      row += (int64_t)blo[d] * st[d];
      nrows *= bhi[d] - blo[d] + 1;
    }
    slots *= nrows;
    const int64_t __attribute__((address_space(1)))* rp = P + row;
    // the four prefix words of a run, relative to its row's first slot
    const int32_t o0 = blo[N - 1], o1 = bhi[N - 1] + 1, o2 = il[N - 1], o3 = ih[N - 1] + 1;
    int64_t settled = 0;  // leaves and holes among the slots
    for (int64_t t = 0; t < nrows; t += kRuns) {
      // kRuns rows of the box; past its last row the odometer has wrapped to
      // the first, so every address below stays inside the box's runs and
      // the loads need no guard
      int64_t p0[kRuns], p1[kRuns], q0[kRuns], q1[kRuns];
      bool in[kRuns];
#pragma unroll
      for (int q = 0; q < kRuns; ++q) {
        bool inner = interior;
#pragma unroll
        for (int d = 0; d < N - 1; ++d) inner &= k[d] >= il[d] && k[d] <= ih[d];
        in[q] = inner;
        p0[q] = rp[o0];
        p1[q] = rp[o1];
        q0[q] = rp[o2];
        q1[q] = rp[o3];
        int64_t mv = jump[0];
        bool carry = true;
#pragma unroll
        for (int d = N - 2; d >= 0; --d) {
          const bool wrap = carry && k[d] == bhi[d];
          if (d > 0) mv = carry && !wrap ? jump[d] : mv;
          k[d] = wrap ? blo[d] : k[d] + (carry ? 1 : 0);
          carry = wrap;
        }
        // (a full wrap, past the box's last row, moves back to its first)
        rp += carry ? -back : mv;
      }
#pragma unroll
      for (int q = 0; q < kRuns; ++q) {
        if (t + q < nrows) {
          settled += ((p1[q] & kLo32) - (p0[q] & kLo32)) + ((p1[q] >> 32) - (p0[q] >> 32));
          if (!f(p0[q], p1[q], in[q], in[q] ? q0[q] : 0, in[q] ? q1[q] : 0)) return;
        }
      }
    }
    if (settled == slots) return;
  }
}

// Input j of job J (m components, the second 0 when m = 1).  The input array
// is in global memory, but its pointer is read from the job table, so the
// loads are told so (global loads instead of flat ones).
__device__ __forceinline__ void job_input(const Job& J, int32_t j, double* u) {
  const double __attribute__((address_space(1)))* U =
      (const double __attribute__((address_space(1)))*)J.u;
  const int m = J.sys.m;
  u[0] = U[(int64_t)j * m];
  u[1] = m > 1 ? U[(int64_t)j * m + 1] : 0.0;
}

// Bounding box of the sample images of the row (local cell c, input j) of
// job J, in precision R.
template <int KIND, int N, typename R>
__device__ __forceinline__ bool row_bbox(const BuildArgs& a, const Job& J, const Rk4Consts<R>& kc,
                                         int64_t c, int32_t j, R* bl, R* bh) {
  const int64_t gc = J.cell_off + c;
  const int level = a.level[gc];
  int32_t ci[N];
#pragma unroll
  for (int d = 0; d < N; ++d) ci[d] = a.idx[gc * N + d];
  const int m = J.sys.m;
  double ud[2];
  job_input(J, j, ud);
  const R u[2] = {R(ud[0]), R(ud[1])};
  bool finite = true;
#pragma unroll
  for (int d = 0; d < N; ++d) {
    bl[d] = R(INFINITY);
    bh[d] = R(-INFINITY);
  }
  const int S = num_samples(a.samples, N);
  // one sample at a time: advancing two in lockstep (independent chains)
  // raised the four-dimensional kernel's registers from 114 to 139 and its
  // occupancy from 4 to 3 waves per SIMD, 9% slower on the coupled Van der
  // Pol system's last round
  constexpr int P = 1;
  for (int q0 = 0; q0 < S; q0 += P) {
    const int np = S - q0 < P ? S - q0 : P;
    R x[P][N];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      int k[N];
      double xd[N];
      sample_offsets<N>(a.samples, q0 + (i < np ? i : 0), k);
      sample_point<N>(J.grid, level, ci, k, xd);
#pragma unroll
      for (int d = 0; d < N; ++d) x[i][d] = R(xd[d]);
    }
    if (np == P) rk4_multi<KIND, N, P, R>(kc, m, J.sys.nsub, x, u);
    else rk4<KIND, N, R>(kc, m, J.sys.nsub, x[0], u);
#pragma unroll
    for (int i = 0; i < P; ++i)
      if (i < np) {
#pragma unroll
        for (int d = 0; d < N; ++d) {
          // min/max instructions: they differ from compare-and-select only
          // for NaN (the row is then decided by `finite`) and in the sign of
          // a zero (which changes no cover decision: (-0) - lo == (+0) - lo)
          finite &= isfinite(x[i][d]);
          bl[d] = vmin(x[i][d], bl[d]);
          bh[d] = vmax(x[i][d], bh[d]);
        }
      }
  }
  return finite;
}


// Decisions of a row whose FP32 box is [fl, fh] (fh >= fl): safe when every
// decision taken from a box extreme (the finest-grid position's floor/ceil,
// the comparisons with lo and hi) is the same anywhere within band[d] of it.
// Since |y32 - y64| <= band[d] holds for every sample image, and min/max are
// 1-Lipschitz, the FP64 box extremes then lead to the same decisions.
// epsr[d] = band[d] / hs_d, the band in finest cell widths, and invh[d] =
// 1 / hs_d (the same for the whole block).  The positions are taken with the
// reciprocal, not divided: they are within a few ulp of the cover step's
// exact quotients, far inside the 1e-9 relative slack of the tolerances, so
// a row found safe here is safe for the exact positions too.
template <int N>
__device__ __forceinline__ bool band_safe(const Job& J, const double* epsr, const double* invh,
                                          const float* fl, const float* fh) {
  bool safe = true;
#pragma unroll
  for (int d = 0; d < N; ++d) {
    const double dl = (double)fl[d], dh = (double)fh[d];
    const double ta = (dl - J.grid.lo[d]) * invh[d];
    const double tb = (dh - J.grid.lo[d]) * invh[d];
    const double tola = epsr[d] + 1e-9 * (fabs(ta) + 1.0);
    const double tolb = epsr[d] + 1e-9 * (fabs(tb) + 1.0);
    safe &= fabs(ta - rint(ta)) > tola;
    safe &= fabs(tb - rint(tb)) > tolb;
    safe &= fabs(dh - J.grid.hi[d]) > J.band[d];
  }
  return safe;
}

// FP64 image of sample q of local row lr (one RK4 trajectory).
template <int KIND, int N>
__device__ __forceinline__ void sample_image(const BuildArgs& a, const Job& J,
                                             const Rk4Consts<double>& kc, int64_t lr, int q,
                                             double* x) {
  const int64_t c = (int64_t)((uint32_t)lr / (uint32_t)a.K);
  const int32_t j = (int32_t)(lr - c * a.K);
  const int64_t gc = J.cell_off + c;
  const int level = a.level[gc];
  int32_t ci[N];
#pragma unroll
  for (int d = 0; d < N; ++d) ci[d] = a.idx[gc * N + d];
  const int m = J.sys.m;
  double u[2];
  job_input(J, j, u);
  int k[N];
  sample_offsets<N>(a.samples, q, k);
  sample_point<N>(J.grid, level, ci, k, x);
  rk4<KIND, N, double>(kc, m, J.sys.nsub, x, u);
}

// The FP64 redo of the rows of a wave whose FP32 box the band test could not
// decide (lanes in `pend`), done by the whole wave: the S samples of a row
// are spread over a group of G lanes (G the power of two >= S, at most 64;
// 64 / G rows at a time), each lane images its samples, and the group's
// min/max and finiteness are reduced across its lanes and handed to the
// row's lane.  The same images and the same exact min/max as the row's own
// sequential FP64 pass, for about a seventeenth of the wave's instructions
// on a row of 17 samples: flagged rows are rare (a few per thousand), so a
// wave rarely has more than one, and imaging it sample after sample kept
// the other 63 lanes idle for a whole row's images.
template <int KIND, int N>
__device__ __forceinline__ void redo_rows_fp64(const BuildArgs& a, const Job& J, int64_t lr,
                                               uint64_t pend, double* bl, double* bh,
                                               bool& finite) {
  const int lane = threadIdx.x & 63;
  const int S = num_samples(a.samples, N);
  const int G = S <= 8 ? 8 : S <= 16 ? 16 : S <= 32 ? 32 : 64;
  const int R = 64 / G;  // rows per pass
  const Rk4Consts<double> kc = make_consts<double>(J.sys);
  const int grp = lane / G, q0 = lane % G;
  while (pend) {  // wave-uniform
    // this pass's rows: the R lowest pending lanes (-1: none)
    int src = -1;
    uint64_t p = pend;
    for (int g = 0; g < R; ++g) {
      const int f = p ? __builtin_ctzll(p) : -1;
      if (g == grp) src = f;
      if (p) p &= p - 1;
    }
    double lo[N], hi[N];
    bool fin = true;
#pragma unroll
    for (int d = 0; d < N; ++d) {
      lo[d] = __builtin_huge_val();
      hi[d] = -__builtin_huge_val();
    }
    const int64_t rlr = __shfl(lr, src < 0 ? 0 : src, 64);
    if (src >= 0) {
      for (int q = q0; q < S; q += G) {
        double x[N];
        sample_image<KIND, N>(a, J, kc, rlr, q, x);
#pragma unroll
        for (int d = 0; d < N; ++d) {
          fin &= isfinite(x[d]);
          lo[d] = vmin(x[d], lo[d]);
          hi[d] = vmax(x[d], hi[d]);
        }
      }
    }
    // reduce within each group of G lanes
    for (int o = G >> 1; o > 0; o >>= 1) {
#pragma unroll
      for (int d = 0; d < N; ++d) {
        lo[d] = vmin(__shfl_xor(lo[d], o, 64), lo[d]);
        hi[d] = vmax(__shfl_xor(hi[d], o, 64), hi[d]);
      }
      fin &= __shfl_xor((int)fin, o, 64) != 0;
    }
    // hand each group's result to its row's lane
    for (int g = 0; g < R; ++g) {
      const int f = __shfl(src, g * G, 64);  // the row group g imaged (wave-uniform)
      if (f < 0) break;
#pragma unroll
      for (int d = 0; d < N; ++d) {
        const double vl = __shfl(lo[d], g * G, 64), vh = __shfl(hi[d], g * G, 64);
        if (lane == f) {
          bl[d] = vl;
          bh[d] = vh;
        }
      }
      const bool vf = __shfl((int)fin, g * G, 64) != 0;
      if (lane == f) finite = vf;
      pend &= ~(1ull << f);
    }
  }
}

// Edge count of a row; *hole is set when a hole of the covering meets the
// interior range, *first to the local id of its first target (when it has one).  Per run of index slots the prefix counts give the leaves
// (ids consecutive from the first) and, on rows of the interior box, the holes
// between the interior columns.  The first cache_runs<N>() runs that hold leaves are
// kept as (first local id, length) pairs with stride kRowBlock from `cache`
// (length 0 after the last one), so that the emit need not walk the index
// again for rows with no more runs than that.
template <int N, bool UNI>
__device__ __forceinline__ int32_t count_targets(const CoverIndex& ci, const Ranges<N>& r,
                                                 int2* cache, bool* hole, int32_t* first) {
  *hole = false;
  if (r.empty) return 0;
  if (UNI || ci.uniform) {
    int32_t c = 1, lin = 0;
#pragma unroll
    for (int d = 0; d < N; ++d) {
      c *= r.hi[d] - r.lo[d] + 1;
      lin = lin * ci.dims[0][d] + r.lo[d];
    }
    *first = lin;
    return c;
  }
  int32_t c = 0, nr = 0;
  bool h = false;
  walk_runs<N>(ci, r.lo, r.hi, r.ilo, r.ihi, true,
               [&](int64_t p0, int64_t p1, bool inner, int64_t q0, int64_t q1) {
                 const int32_t nl = (int32_t)((p1 & kLo32) - (p0 & kLo32));
                 if (nl > 0) {
                   if (nr == 0) *first = (int32_t)((p0 & kLo32) - ci.pbase);
                   if (nr < cache_runs<N>())
                     cache[nr * kRowBlock] = make_int2((int32_t)((p0 & kLo32) - ci.pbase), nl);
                   ++nr;
                   c += nl;
                 }
                 h |= inner && (q1 >> 32) != (q0 >> 32);
                 return true;
               });
  if (nr < cache_runs<N>()) cache[nr * kRowBlock] = make_int2(0, 0);
  else if (nr > cache_runs<N>()) cache[0] = make_int2(0, -1);  // too many runs: walk again
  *hole = h;
  return c;
}

// Targets p0 .. p1-1 of a row (0-based positions in its ascending target
// list) as global ids into dst[0 .. p1-p0).
template <int N, bool UNI>
__device__ __forceinline__ void emit_targets(const CoverIndex& ci, const int32_t* lo,
                                             const int32_t* hi, int32_t /*count*/,
                                             const int2* cache, int32_t id0, int32_t p0,
                                             int32_t p1, int32_t* dst) {
  if (UNI || ci.uniform) {
    // position -> multi-index in the box, last dimension fastest; ids along
    // the last dimension are consecutive, so the id is recomputed only when
    // a slower coordinate moves
    int32_t k[N];
#pragma unroll
    for (int d = 0; d < N; ++d) k[d] = lo[d];
    if (p0 > 0) {  // only rows that straddle a tile boundary divide
      int32_t rem = p0;
#pragma unroll
      for (int d = N - 1; d >= 0; --d) {
        const int32_t w = hi[d] - lo[d] + 1;
        k[d] += rem % w;
        rem /= w;
      }
    }
    auto lin_of = [&]() {
      int32_t lin = 0;
#pragma unroll
      for (int d = 0; d < N; ++d) lin = lin * ci.dims[0][d] + k[d];
      return id0 + lin;
    };
    int32_t id = lin_of();
    for (int32_t p = p0; p < p1;) {
      // the rest of the current run along the last dimension
      const int32_t run = hi[N - 1] - k[N - 1] + 1;
      const int32_t q1 = p1 - p < run ? p1 : p + run;
      for (; p < q1; ++p) dst[p - p0] = id++;
      if (p >= p1) break;
      if constexpr (N > 1) {  // (with one dimension the run always reaches p1)
        // next position of the box odometer (unrolled: a runtime index
        // would put k in scratch memory); p < p1, so it does not wrap
        k[N - 1] = lo[N - 1];
        bool carry = true;
#pragma unroll
        for (int d = N - 2; d >= 0; --d) {
          if (carry) {
            if (d > 0 && k[d] == hi[d]) {
              k[d] = lo[d];
            } else {
              ++k[d];
              carry = false;
            }
          }
        }
        id = lin_of();
      } else {
        break;
      }
    }
    return;
  }
  if constexpr (UNI) return;
  if (cache[0].y >= 0) {  // the row's runs are cached
    int32_t w = 0;        // position of the run's first leaf in the row's list
    for (int k = 0; k < cache_runs<N>() && w < p1; ++k) {
      const int2 run = cache[k * kRowBlock];
      if (run.y == 0) break;
      const int32_t i0 = p0 > w ? p0 - w : 0;
      const int32_t i1 = p1 - w < run.y ? p1 - w : run.y;
      for (int32_t i = i0; i < i1; ++i) dst[w + i - p0] = id0 + run.x + i;
      w += run.y;
    }
    return;
  }
  int32_t w = 0;  // position of the run's first leaf in the row's list
  walk_runs<N>(ci, lo, hi, lo, hi, false, [&](int64_t v0, int64_t v1, bool, int64_t, int64_t) {
    const int32_t nl = (int32_t)((v1 & kLo32) - (v0 & kLo32));
    const int32_t first = id0 + (int32_t)((v0 & kLo32) - ci.pbase);
    const int32_t i0 = p0 > w ? p0 - w : 0;
    const int32_t i1 = p1 - w < nl ? p1 - w : nl;
    for (int32_t i = i0; i < i1; ++i) dst[w + i - p0] = first + i;
    w += nl;
    return w < p1;
  });
}

// UNI: every job of the launch is a full level-0 grid (no index walk is
// compiled in, which keeps the register count, and so the occupancy, of the
// image loop higher).
template <int KIND, int N, bool F32, bool UNI>
//
// At least four waves per SIMD: the FP32 variant of four-dimensional fields
// would otherwise take 140 VGPRs (three waves) for the registers of the
// wave-wide FP64 redo; bounded at 128, the compiler spills two doubles.
__global__ __launch_bounds__(kRowBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_build(
    BuildArgs a) {
  __shared__ CoverIndex ci;
  __shared__ int32_t tile[UNI ? kTile : 1];
  __shared__ int2 cache[UNI ? 1 : cache_runs<N>() * kRowBlock];
  __shared__ int32_t stage[UNI || N > 2 ? 1 : kStage * (kRowBlock / 64)];
  __shared__ int64_t wsum[kRowBlock / 64];
  __shared__ int64_t s_prefix;
  __shared__ double s_epsr[F32 ? N : 1], s_invh[F32 ? N : 1];
  __shared__ uint32_t s_bid, s_out, s_rchk;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) {
    const uint32_t t = atomicAdd(a.ticket, 1u);
    // every other block has its ticket: reset the counter for the next launch
    if (t == (uint32_t)a.n_blocks - 1)
      __hip_atomic_store(a.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_bid = t;
    s_out = 0;
    s_rchk = 0;
  }
  __syncthreads();
  const int64_t bid = s_bid;
  const int32_t jb = job_of_block(a.jobs, a.n_jobs, LK_ROWS, bid);
  const Job& J = a.jobs[jb];
  if constexpr (F32) {
    // the recheck band in finest cell widths, per dimension
    if (tid < N) {
      const double hs = ldexp(J.grid.w0[tid], -J.ci.lmax);
      s_epsr[tid] = J.band[tid] / hs;
      s_invh[tid] = 1.0 / hs;
    }
  }
  stage_index(&ci, &J.ci);
  // ---- 1-2: images, box, cover decision, count
  const int64_t lr = (bid - J.blk[LK_ROWS]) * kRowBlock + tid;
  const bool live = lr < J.n_cells * a.K;
  const int64_t g = J.cell_off * a.K + lr;
  // the row's cell and input (a job has fewer than 2^31 rows: 32-bit division)
  const int64_t lc = (int64_t)((uint32_t)lr / (uint32_t)a.K);
  const int32_t lj = (int32_t)(lr - lc * a.K);
  int32_t lo[N], hi[N];
  int32_t c = 0, first = 0;
#pragma unroll
  for (int d = 0; d < N; ++d) lo[d] = hi[d] = 0;
  double bl[N], bh[N];
  bool finite = false;
  if constexpr (F32) {
    // FP32 images; the rows the band test cannot decide are redone in FP64
    // by the whole wave, which overwrites their boxes.  The FP32 box is
    // widened to FP64 (exactly) before the redo, so that only one copy of
    // the box is live across it.
    float fl[N], fh[N];
#pragma unroll
    for (int d = 0; d < N; ++d) fl[d] = fh[d] = 0.f;
    if (live) {
      const Rk4Consts<float> kc = make_consts<float>(J.sys);
      const bool fin32 = row_bbox<KIND, N, float>(a, J, kc, lc, lj, fl, fh);
      finite = fin32 && band_safe<N>(J, s_epsr, s_invh, fl, fh);
    }
#pragma unroll
    for (int d = 0; d < N; ++d) {
      bl[d] = (double)fl[d];
      bh[d] = (double)fh[d];
    }
    const uint64_t pend = __ballot(live && !finite);
    if (pend) {
      redo_rows_fp64<KIND, N>(a, J, lr, pend, bl, bh, finite);
      if (lane == 0) atomicAdd(&s_rchk, (uint32_t)__popcll(pend));
    }
  }
  if (live) {
    if constexpr (!F32) {
      const Rk4Consts<double> kd = make_consts<double>(J.sys);
      finite = row_bbox<KIND, N, double>(a, J, kd, lc, lj, bl, bh);
    }
    bool out = true;
    if (finite) {
      const Ranges<N> rr = ranges_of<N>(J.grid, ci, bl, bh);
      bool hole;
      c = count_targets<N, UNI>(ci, rr, UNI ? cache : cache + tid, &hole, &first);
      out = rr.outx || hole;
      if (a.fast_out && out) c = 0;
#pragma unroll
      for (int d = 0; d < N; ++d) {
        lo[d] = rr.lo[d];
        hi[d] = rr.hi[d];
      }
    }
    a.out[g] = out ? 1 : 0;
    if (out) atomicAdd(&s_out, 1u);
  }

  // ---- 3: block-exclusive scan of the counts
  int64_t x = c;
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  int64_t before = 0, T = 0;
  for (int w = 0; w < kRowBlock / 64; ++w) {
    before += w < wid ? wsum[w] : 0;
    T += wsum[w];
  }
  const int64_t off = before + x - c;

  // ---- 4: decoupled look-back (first wave; control flow wave-uniform)
  if (wid == 0) {
    const uint64_t tag = (uint64_t)a.epoch << 40;
    int64_t prefix = 0;
    if (bid == 0) {
      if (lane == 0)
        __hip_atomic_store(&a.lb[0], tag | kLbInc | (uint64_t)T, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    } else {
      if (lane == 0)
        __hip_atomic_store(&a.lb[bid], tag | kLbAgg | (uint64_t)T, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      const uint64_t t0 = wall_clock64();
      int64_t top = bid - 1;  // lane i looks at block top - i
      for (;;) {
        const int64_t q = top - lane;
        uint64_t w = 0;
        for (uint32_t spin = 0;; ++spin) {
          w = q >= 0 ? __hip_atomic_load(&a.lb[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                     : tag | kLbInc;
          if (__ballot(lb_status(w, a.epoch) == 0) == 0) break;
          if ((spin & 255) == 255 && wall_clock64() - t0 > 10ull * 100000000ull) {
            // never expected: record it and leave with a wrong prefix (the
            // capacity test below keeps every store in bounds)
            if (lane == 0) atomicOr(a.err, 256u);
            w = tag | kLbInc;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        const uint64_t inc = __ballot(lb_status(w, a.epoch) == 2);
        const int first = inc ? __builtin_ctzll(inc) : 64;
        int64_t v = lane <= first ? (int64_t)(w & kLbVal) : 0;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        prefix += v;
        if (inc) break;
        top -= 64;
      }
      if (lane == 0) {
        if ((uint64_t)(prefix + T) > kLbVal) atomicOr(a.err, 512u);  // beyond 2^38 edges
        __hip_atomic_store(&a.lb[bid], tag | kLbInc | ((uint64_t)(prefix + T) & kLbVal),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (lane == 0) {
      s_prefix = prefix;
      if (bid == a.n_blocks - 1) *a.d_total = prefix + T;
      atomicAdd((unsigned long long*)&a.stats[jb].n_edges, (unsigned long long)T);
      if (s_out) atomicAdd(&a.stats[jb].n_out, (unsigned long long)s_out);
      if (s_rchk) {
        atomicAdd(&a.stats[jb].n_recheck, (unsigned long long)s_rchk);
        atomicAdd(a.n_recheck, (unsigned long long)s_rchk);
      }
    }
  }
  __syncthreads();
  const int64_t prefix = s_prefix;

  // ---- 5: row offsets, first targets and target ids
  if (live) a.row_ptr[g] = prefix + off;
  if (live && a.first) a.first[g] = c > 0 ? (int32_t)J.cell_off + first : -1;
  if (live && g == a.total_rows - 1) a.row_ptr[a.total_rows] = prefix + off + c;
  if (prefix + T > a.cap_edges) return;  // capacity miss: col is not written
  const int32_t id0 = (int32_t)J.cell_off;
  if constexpr (!UNI && N > 2) {
    // rows of three- and four-dimensional fields write their own targets:
    // staging them (below) was slower there (their kernels are at the
    // register limit already)
    if (c > 0) emit_targets<N, UNI>(ci, lo, hi, c, cache + tid, id0, 0, c, a.col + prefix + off);
    return;
  }
  if constexpr (!UNI) {
    // The wave's rows own one contiguous range of col.  It is written in
    // chunks of kStage ids: each lane puts its ids of the chunk into the
    // wave's LDS area, then the wave stores the chunk with consecutive lanes
    // on consecutive ids (a row writing its own ids would spread each store
    // instruction over the 64 rows' ranges).  Only the wave synchronises.
    // A wave holding a row with more runs than the LDS cache keeps writes
    // its rows' targets directly, as the rows of larger fields do: that row
    // would walk the index again for every chunk it spans.
    if (__ballot(c > 0 && !ci.uniform && cache[tid].y < 0)) {
      if (c > 0) emit_targets<N, UNI>(ci, lo, hi, c, cache + tid, id0, 0, c, a.col + prefix + off);
      return;
    }
    const int64_t wbeg = __shfl(off, 0, 64), wend = __shfl(off + c, 63, 64);
    int32_t* ws = stage + wid * kStage;
    for (int64_t ch = wbeg; ch < wend; ch += kStage) {  // wave-uniform
      const int64_t ce = ch + kStage < wend ? ch + kStage : wend;
      const int64_t r0 = off > ch ? off : ch, r1 = off + c < ce ? off + c : ce;
      if (r0 < r1)
        emit_targets<N, UNI>(ci, lo, hi, c, cache + tid, id0, (int32_t)(r0 - off),
                             (int32_t)(r1 - off), ws + (r0 - ch));
      wave_sync();
      for (int64_t i = lane; i < ce - ch; i += 64) a.col[prefix + ch + i] = ws[i];
      wave_sync();
    }
    return;
  }
  for (int64_t w0 = 0; w0 < T; w0 += kTile) {
    const int64_t w1 = T < w0 + kTile ? T : w0 + kTile;
    const int64_t s0 = off > w0 ? off : w0;
    const int64_t s1 = off + c < w1 ? off + c : w1;
    if (s0 < s1)
      emit_targets<N, UNI>(ci, lo, hi, c, UNI ? cache : cache + tid, id0, (int32_t)(s0 - off),
                           (int32_t)(s1 - off), tile + (s0 - w0));
    __syncthreads();
    for (int64_t i = tid; i < w1 - w0; i += kRowBlock) a.col[prefix + w0 + i] = tile[i];
    __syncthreads();
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
  double ud[2];
  job_input(J, j, ud);
  const R u[2] = {R(ud[0]), R(ud[1])};
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
__global__ __launch_bounds__(kRowBlock) void k_calibrate(BuildArgs a, unsigned long long* maxerr,
                                                        int64_t stride) {
  const int32_t jb = job_of_block(a.jobs, a.n_jobs, LK_ROWS, blockIdx.x);
  const Job& J = a.jobs[jb];
  const int64_t lb = blockIdx.x - J.blk[LK_ROWS];
  if (lb % stride != 0) return;  // sample whole blocks: every lane of a wave does work
  const int64_t lr = lb * kRowBlock + threadIdx.x;
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
    job_input(J, j, u64);
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

}  // namespace kbuild
}  // namespace gis
