/*
 * gis.h -- C ABI of the MI355X (gfx950) graph-construction path of the
 * graph-based invariant set (GIS) algorithm of Decardi-Nelson and Liu,
 * "An efficient implementation of graph-based invariant set algorithm for
 * constrained nonlinear dynamical systems", arXiv 2202.06111.
 *
 * Problem (Sec. 2, Eq. 1): a discrete-time system x+ = f(x, u) with a closed
 * state box X = prod_d [lo_d, hi_d] and a finite sampled input set
 * U = {u_0 .. u_{K-1}}.  Here f is nsub classical RK4 substeps of one of the
 * built-in vector fields over a sampling interval dt.
 *
 * Covering (Sec. 2.1): cells are closed boxes; a cell of level L has the
 * multi-index i (0 <= i_d < n0_d 2^L) and the box
 *   [lo_d + i_d w_{L,d}, lo_d + (i_d + 1) w_{L,d}],  w_{L,d} = ((hi_d - lo_d) / n0_d) 2^-L.
 * A cell list is in canonical order: ascending level, then ascending
 * row-major multi-index (dimension 0 slowest); a cell's position in the list
 * is its id.  Cells of one list never overlap.
 *
 * Symbolic image (Sec. 2.2, Eqs. 2-3, Definition 1): one row per
 * (cell, input), row = cell * K + input.  The image F(B_i) under input u is
 * approximated by the bounding box of the images of the cell's sample points
 * (3^n lattice points or 2^n corners + centre).  The row's edges are the ids
 * of every cell whose closed box meets that bounding box, ascending.  A row is
 * OUT when the box leaves X, when some image is not finite, or when the box's
 * interior meets a part of X that no cell of the list covers.
 *
 * Graph analysis (Sec. 2.3), two readings:
 *   GIS_ANALYSIS_CONTROLLED  keep the largest cell set K in which every cell
 *     has an input whose row is not OUT and whose edges all end in K;
 *   GIS_ANALYSIS_NONLEAVING  keep the cells with an infinite admissible path
 *     in the input-union symbolic image (Definitions 5-6): iterated removal of
 *     cells none of whose edges ends in the kept set.
 *   GIS_ANALYSIS_LARGEST_SCC  Definition 6 read literally: the largest
 *     strongly connected component of the input-union symbolic image that
 *     holds a cycle (two or more cells, or one cell with an edge to itself),
 *     plus every cell with a path into it; of equally large components the
 *     one holding the smallest cell id; nothing if the graph has no cycle.
 *     Mask bit u: row (cell, u) has an edge into the kept set.
 * The admissible-input mask of a kept cell has bit u set when row (cell, u)
 * satisfies the analysis' condition at the fixed point.
 *
 * Adaptive subdivision (Sec. 3.1.1, Algorithm 1, Remark 1): a kept cell is a
 * boundary cell when a finest-level cell adjacent to it lies outside X or is
 * not covered by a kept cell (GIS_BOUNDARY_SHELL: all adjacent cells, which
 * includes Remark 1's edge points; GIS_BOUNDARY_CORNERS: the 2^n diagonal
 * corners only, Algorithm 1 as printed).  The next covering holds the 2^n
 * children of every boundary cell and every other kept cell.
 *
 * Standard subdivision (Sec. 2.1): every kept cell of a level-0 covering is
 * halved across one dimension, which cycles from one iteration to the next
 * (dimension 0 first).  The halves are the level-0 cells of the grid with
 * twice as many cells along that dimension (same X); the widths
 * (hi_d - lo_d) / (2 n0_d) are exactly half of (hi_d - lo_d) / n0_d, so the
 * geometry is that of the halved cells.
 *
 * Conventions for every function below:
 *  - Return value: a gis_status code; on failure gis_last_error() gives a
 *    message (thread-local).  Outputs are unspecified after a failure.
 *  - Pointers named d_* are device memory of the context's device, owned by
 *    the caller; the library never frees them.  Structs are host memory.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *    it; functions that report counts to the host synchronise it.
 *  - Arrays are dense and row-major; int64 sizes.
 */
#ifndef GIS_H
#define GIS_H

#ifndef __HIPCC_RTC__  /* the library's runtime-compiled fields define the types themselves */
#include <stdint.h>
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GIS_OK = 0,
  GIS_E_INVAL = 1,        /* invalid argument or invalid cell list */
  GIS_E_NOMEM = 2,        /* device allocation failed */
  GIS_E_HIP = 3,          /* HIP runtime error */
  GIS_E_CAPACITY = 4,     /* a caller buffer is too small; the needed size is reported */
  GIS_E_UNSUPPORTED = 5,  /* valid request outside the library's limits */
  GIS_E_INTERNAL = 6      /* a device-side consistency check failed */
} gis_status;

enum { GIS_SYS_LINEAR = 0, GIS_SYS_VDP = 1, GIS_SYS_LORENZ = 2, GIS_SYS_VDP2 = 3,
       GIS_SYS_CSTR = 4, GIS_SYS_USER = 5 };
enum { GIS_SAMPLES_LATTICE3 = 1, GIS_SAMPLES_CORNERS_CENTER = 2 };
enum { GIS_PREC_FP64 = 1, GIS_PREC_FP32_RECHECK = 2 };
enum { GIS_BOUNDARY_SHELL = 1, GIS_BOUNDARY_CORNERS = 2 };
enum { GIS_ANALYSIS_CONTROLLED = 1, GIS_ANALYSIS_NONLEAVING = 2, GIS_ANALYSIS_LARGEST_SCC = 3 };
enum { GIS_SUBDIVIDE_BOUNDARY = 0, GIS_SUBDIVIDE_BISECT = 1 };

/* Vector field g of x' = g(x, u); f = nsub RK4 substeps of length dt/nsub.
 *  LINEAR (n <= 4, m <= 2): g = A x + B u, A = params[4d + j], B = params[16 + 2d + k]
 *  VDP    (n = 2, m = 1):   g = (x2, mu (1 - x1^2) x2 - x1 + u),          mu = params[0]
 *  LORENZ (n = 3, m = 1):   g = (s (x2 - x1), x1 (r - x3) - x2 + u, x1 x2 - b x3),
 *                           s, r, b = params[0..2]
 *  VDP2   (n = 4, m = 2):   state (x1, v1, x2, v2),
 *                           vi' = (1 - xi^2) vi - xi + c (xj - xi) + ui, c = params[0]
 *  CSTR   (n = 2, m = 1):   the reactor of Sec. 4.1 (Eq. 4), state (cA, T), input Tc,
 *                           r = k0 exp(-(E/R) / T) cA,
 *                           g = (q/V (cAf - cA) - r,
 *                                q/V (Tf - T) + (-dH)/(rho cp) r + UA/(V rho cp) (Tc - T)),
 *                           params[0..6] = q/V, cAf, Tf, E/R, k0, -dH/(rho cp), UA/(V rho cp);
 *                           exp is the library's own (Cody-Waite reduction, degree-13
 *                           Taylor polynomial, exact 2^k scaling; within 1 ulp), so FP64
 *                           images are reproducible bit for bit
 *  USER   (n <= 4, m <= 2): the context's runtime-compiled field (gis_set_user_field) */
typedef struct gis_system {
  int32_t kind, n, m, nsub;
  double dt;
  double params[32];
} gis_system;

/* Closed state box X and its coarse partition (n0_d level-0 cells per dimension). */
typedef struct gis_grid {
  int32_t n;
  int32_t n0[4];
  double lo[4], hi[4];
} gis_grid;

typedef struct gis_opts {
  int32_t samples;        /* GIS_SAMPLES_* */
  int32_t precision;      /* GIS_PREC_*: FP64 images, or FP32 images with an FP64 recheck of
                             every row whose FP32 box extreme lies within band[d] of a
                             finest-level face or of the border of X */
  int32_t boundary_rule;  /* GIS_BOUNDARY_* */
  int32_t analysis;       /* GIS_ANALYSIS_* */
  int32_t fast_out;       /* nonzero: OUT rows get no edges.  The controlled analysis gives
                             the same kept set and masks either way (an OUT row never keeps
                             its cell); the other analyses count an OUT row's edges, so
                             fast_out requires analysis GIS_ANALYSIS_CONTROLLED
                             (GIS_E_INVAL otherwise) */
  int32_t timing;         /* HIP-event timings in gis_round_stats: 1 the build kernel (ms_image),
                             2 also the phases (ms_build, ms_prune, ms_subdivide); 0 none */
  int32_t subdivision;    /* GIS_SUBDIVIDE_*: gis_solve refines the 2^n children of the
                             boundary cells (BOUNDARY, 0), or halves every kept cell across
                             the cycled dimension (BISECT; boundary_rule is then unused) */
  int32_t check_band;     /* nonzero (FP32 path of gis_solve / gis_solve_batch): each round
                             also measures the largest |FP32 image - FP64 image| over every
                             sample of every row (gis_round_stats.max_err_all) and fails
                             with GIS_E_INTERNAL if it exceeds the round's band; costs
                             about one more image pass per round */
  int32_t neighbours;     /* N of the neighbourhood selection (Sec. 3.1.2, Figure 5): with
                             GIS_SUBDIVIDE_BOUNDARY, the N kept cells whose centres lie
                             nearest to each boundary cell's centre (Euclidean distance in
                             state units, the cell itself not counted, equal distances by
                             cell id) are subdivided with it; 0: boundary cells only
                             (0..64) */
  int32_t reserved;       /* 0 */
  double band[4];         /* absolute recheck band per dimension; 0 = gis_solve calibrates
                             it on each round's covering before that round's build:
                             band = max(8 e, 1e-5 w_finest), e the largest |FP32 - FP64|
                             image difference over every row of the covering, or over an
                             evenly strided sample of about 2^20 rows of larger coverings
                             (gis_calibrate_band takes every row) */
} gis_opts;

/* A cell list in device memory. */
typedef struct gis_cells {
  int64_t n_cells;   /* number of cells (output of gis_subdivide) */
  int64_t cap;       /* capacity in cells of level[] and idx[] */
  uint8_t* level;    /* d [cap] */
  int32_t* idx;      /* d [cap * n], cell-major */
} gis_cells;

/* The symbolic image as CSR over rows (cell * K + input). */
typedef struct gis_graph {
  int64_t n_rows;     /* out: n_cells * K */
  int64_t n_edges;    /* out: number of edges (needed capacity on GIS_E_CAPACITY) */
  int64_t n_out;      /* out: number of OUT rows */
  int64_t n_recheck;  /* out: rows recomputed in FP64 by the FP32 path */
  int64_t cap_edges;  /* in: capacity of col[] */
  int64_t* row_ptr;   /* d [n_rows + 1] */
  int32_t* col;       /* d [cap_edges] */
  uint8_t* out;       /* d [n_rows] */
} gis_graph;

typedef struct gis_ctx gis_ctx;
typedef struct gis_solution gis_solution;

typedef struct gis_round_stats {
  int64_t n_cells, n_rows, n_edges, n_out, n_kept, n_boundary, n_recheck;
  int32_t max_level, reserved;
  double ms_build, ms_prune, ms_subdivide;   /* device time between HIP events (opts.timing 2) */
  double ms_image;    /* the one-pass build kernel: images, boxes, cover, FP64 recheck of the
                         rows that need it, CSR emit (opts.timing) */
  double ms_recheck;  /* 0: the recheck runs inside the build kernel */
  double ms_host;       /* host time of the round outside synchronisations (launches, bookkeeping) */
  double ms_host_wait;  /* host time blocked in the round's synchronisations */
  double band[4];       /* FP32 path: recheck band of the round per dimension */
  double max_err[4];    /* FP32 path, calibrated band: largest |FP32 - FP64| image difference
                           over the calibration sample of the round's covering */
  double max_err_all[4];  /* with opts.check_band: the same over every row (0 otherwise) */
  int64_t n_selected;   /* cells subdivided after the round: the boundary cells and their
                           neighbourhood (opts.neighbours), or the halved cells */
} gis_round_stats;

#define GIS_MAX_ROUNDS 32

typedef struct gis_solve_info {
  int32_t n_rounds;        /* rounds actually run (<= requested + 1) */
  int32_t n, K, mask_words;
  int32_t n0[4];           /* cells per dimension of the final covering's grid: the coarse
                              grid's, doubled along each dimension a bisection cut */
  int64_t n_cells, n_kept; /* final covering and kept set */
  double band[4];          /* recheck band used (FP32 path) */
  gis_round_stats rounds[GIS_MAX_ROUNDS];
} gis_solve_info;

/* ---- context: device workspace, reusable across calls, one stream at a time ---- */
int32_t gis_ctx_create(int32_t device, gis_ctx** out);
void gis_ctx_destroy(gis_ctx* ctx);

/* Schedule parameters of a context.  They change launch shapes and where the
 * host checks for convergence, never results (the analysis reaches the same
 * fixed point in any order, Sec. 2.3).  Defaults in brackets; gis_autotune
 * picks them by timing. */
typedef struct gis_tuning {
  int32_t first_sweeps;    /* analysis sweeps enqueued with a round before its convergence
                              check [16]; later rounds enqueue what the previous round
                              needed plus a margin, at most this many (1..256) */
  int32_t sweep_batch;     /* sweeps between later checks [8] (1..256) */
  int64_t sweep_edges;     /* graphs with more edges (or K > 256) skip the sweeps and run
                              the frontier phase [8388608] (>= 0) */
  int32_t frontier_batch;  /* frontier steps between checks [16] (1..256) */
  int32_t sweep_blocks;    /* grid cap of a sweep launch [4096] (1..65536) */
  int32_t front_blocks;    /* grid of a frontier step, 4 waves per block [2048] (1..65536) */
  int32_t use_graphs;      /* nonzero: a round's analysis launch sequence is captured as a
                              HIP graph at its second sighting and replayed later [0] */
  int32_t edge_hint;       /* edges per row assumed for the first build of a solve, which
                              sizes the edge buffer (0: 2^(n+1)); too small a value costs
                              one rebuild of that round, never a wrong result (0..4096) */
  int32_t row_frontier;    /* nonzero: the frontier phase keeps one reverse entry per (row,
                              target) also for K <= 64 inputs, instead of one per (source
                              cell, target) with an input mask [0] (0..1) */
  int32_t wit_sweeps;      /* non-leaving analysis: at most this many witness sweeps (a
                              present target kept per cell and re-checked each sweep; any
                              graph size, sweep_edges does not apply) before the frontier
                              phase takes over; 0: the row sweeps and frontier phase of the
                              controlled analysis instead [256] (0..4096) */
} gis_tuning;

/* Reads / replaces the context's schedule parameters.  GIS_E_INVAL when a
 * field is out of range (nothing is changed then). */
int32_t gis_get_tuning(const gis_ctx* ctx, gis_tuning* out);
int32_t gis_set_tuning(gis_ctx* ctx, const gis_tuning* tuning);

/* Autotuner: chooses the context's schedule parameters for one problem by
 * timing whole gis_solve calls of it (arguments as for gis_solve).  Starting
 * from the current parameters it tries, one field at a time, a few values
 * per field and keeps a value when the median wall time of `repeats` solves
 * (1..16, each trial after two untimed solves) drops by more than 2%.  Every trial must reproduce the first trial's
 * kept-cell count (GIS_E_INTERNAL otherwise).  The chosen parameters are set
 * on ctx and returned in *best (may be NULL), their median time in *best_ms
 * (may be NULL).  Synchronises; allocates like gis_solve. */
int32_t gis_autotune(gis_ctx* ctx, const gis_system* sys, const gis_grid* grid,
                     const double* d_u, int32_t K, int32_t rounds, const gis_opts* opts,
                     int32_t repeats, gis_tuning* best, double* best_ms, void* stream);

/* Symbolic image of a covering (Sec. 2.2, Definition 1).  d_u: K x m inputs
 * (FP64).  Fills row_ptr, out and, when cap_edges suffices, col; synchronises
 * to report n_edges, n_out and n_recheck.  GIS_E_CAPACITY: n_edges holds the
 * needed capacity, row_ptr and out are valid, col is not. */
int32_t gis_build_graph(gis_ctx* ctx, const gis_system* sys, const gis_grid* grid,
                        const double* d_u, int32_t K, const gis_cells* cells,
                        const gis_opts* opts, gis_graph* graph, void* stream);

/* Graph analysis (Sec. 2.3) of a graph from gis_build_graph.  d_kept [n_cells]
 * (1 = kept), d_mask [n_cells * ceil(K/64)] admissible inputs (bit u of word
 * u/64).  Synchronises to report *n_kept (may be NULL). */
int32_t gis_prune(gis_ctx* ctx, const gis_graph* graph, int64_t n_cells, int32_t K,
                  int32_t analysis, uint8_t* d_kept, uint64_t* d_mask, int64_t* n_kept,
                  void* stream);

/* gis_prune for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * kept flags, masks and count as gis_prune, computed by sweeps only in a
 * static device workspace of about 26 MiB per GPU, held until the process
 * ends; no context.  It runs on the current device, which must be the device
 * of `stream` and of the buffers.  Analysis GIS_ANALYSIS_CONTROLLED or
 * GIS_ANALYSIS_NONLEAVING (GIS_E_INVAL otherwise), K <= 256 (GIS_E_INVAL),
 * n_cells <= 2^21 (GIS_E_CAPACITY beyond).  Calls no hipMalloc/hipFree.
 * Every call on a GPU shares its workspace: calls that overlap in time on
 * one GPU race and must not be made.  Synchronises. */
int32_t gis_prune_static(const gis_graph* graph, int64_t n_cells, int32_t K, int32_t analysis,
                         uint8_t* d_kept, uint64_t* d_mask, int64_t* n_kept, void* stream);

/* Boundary selection and subdivision (Sec. 3.1.1), with the neighbourhood of
 * the boundary cells (Sec. 3.1.2) when neighbours > 0 (0..64, GIS_E_INVAL
 * beyond): the boundary cells and the `neighbours` kept cells nearest to each
 * are split into their 2^n children.  d_boundary [in->n_cells] receives the
 * boundary flags (may be NULL).  Synchronises; out->n_cells is the new cell
 * count, GIS_E_CAPACITY if it exceeds out->cap (nothing written). */
int32_t gis_subdivide(gis_ctx* ctx, const gis_grid* grid, const gis_cells* in,
                      const uint8_t* d_kept, int32_t boundary_rule, int32_t neighbours,
                      uint8_t* d_boundary, gis_cells* out, void* stream);

/* Standard subdivision (Sec. 2.1): halves every kept cell of `in` across
 * dimension `dim` (0 <= dim < n).  Every kept cell must be a level-0 cell of
 * `grid` (GIS_E_INVAL otherwise); the list's order does not matter and the
 * cells that are not kept are ignored.  *grid_out receives the grid of the
 * halves (grid with n0[dim] doubled, at most 2^30); out receives the halves as
 * its level-0 cells in canonical order (2 per kept cell, duplicates of `in`
 * merged).  Synchronises; GIS_E_CAPACITY if out->cap is too small
 * (out->n_cells then holds the count needed). */
int32_t gis_bisect(gis_ctx* ctx, const gis_grid* grid, const gis_cells* in, const uint8_t* d_kept,
                   int32_t dim, gis_grid* grid_out, gis_cells* out, void* stream);

/* The iteration loop: coarse covering -> build -> prune, then `rounds` times
 * subdivide -> build -> prune (opts->subdivision: boundary cells or every kept
 * cell); stops early when nothing is kept.  The result
 * stays on the device in a library-owned handle (free with gis_solution_free). */
int32_t gis_solve(gis_ctx* ctx, const gis_system* sys, const gis_grid* grid, const double* d_u,
                  int32_t K, int32_t rounds, const gis_opts* opts, gis_solution** out,
                  void* stream);
/* A batch of independent solves run through the same launches (one launch
 * per kernel for all jobs and all refinement levels): the jobs share the
 * system kind and dimensions, K and the options; each has its own system
 * parameters, time step, state box, coarse grid and inputs (d_u: K x m).
 * out_sols[j] receives job j's solution, identical to what gis_solve returns
 * for that job alone. */
typedef struct gis_job {
  gis_system sys;
  gis_grid grid;
  const double* d_u;
} gis_job;
int32_t gis_solve_batch(gis_ctx* ctx, int32_t n_jobs, const gis_job* jobs, int32_t K,
                        int32_t rounds, const gis_opts* opts, gis_solution** out_sols,
                        void* stream);

int32_t gis_solution_info(const gis_solution* sol, gis_solve_info* info);
/* Copies the final covering, kept flags and masks into caller buffers
 * (cells->cap >= n_cells; d_kept [n_cells]; d_mask [n_cells * mask_words]). */
int32_t gis_solution_export(const gis_solution* sol, gis_cells* cells, uint8_t* d_kept,
                            uint64_t* d_mask, void* stream);
void gis_solution_free(gis_solution* sol);

/* Point queries on a solution: d_states [n x dim] FP64.  Membership: 1 if the
 * state lies in X and in a kept cell (a state on a face belongs to the cell
 * above it, the upper border of X to the last cell).  Admissible: the mask of
 * that cell, 0 words otherwise; d_mask_out [n x mask_words]. */
int32_t gis_query_membership(const gis_solution* sol, const double* d_states, int64_t n,
                             uint8_t* d_member, void* stream);
int32_t gis_query_admissible(const gis_solution* sol, const double* d_states, int64_t n,
                             uint64_t* d_mask_out, void* stream);

/* Sample images of every row for parity checks: d_images [n_cells*K x S x n]
 * FP64 (FP32 results widened when precision is GIS_PREC_FP32_RECHECK). */
int32_t gis_images(gis_ctx* ctx, const gis_system* sys, const gis_grid* grid, const double* d_u,
                   int32_t K, const gis_cells* cells, int32_t samples, int32_t precision,
                   double* d_images, void* stream);

/* Recheck band for the FP32 path from the largest |FP32 image - FP64 image|
 * per dimension over every sample of every row of a covering:
 * band_out[d] = max(floor_rel * w_finest_d, safety * that largest difference),
 * w_finest_d the cell width of the covering's finest level.  Synchronises. */
int32_t gis_calibrate_band(gis_ctx* ctx, const gis_system* sys, const gis_grid* grid,
                           const double* d_u, int32_t K, const gis_cells* cells, int32_t samples,
                           double safety, double floor_rel, double* band_out, void* stream);

/* The vector field of systems of kind GIS_SYS_USER in this context: the
 * problem statement (Eq. 1) takes f as given, so the caller may supply g of
 * x' = g(x, u) as code, which the library compiles at run time (hipRTC, about
 * a second) together with its own graph-construction kernels -- the same RK4
 * operation order, sample points, cover logic, recheck and emit as for the
 * built-in fields.  `body` is C++ for the device that sets dx[0 .. n-1] from
 * x[0 .. n-1], u[0 .. m-1] and p[0 .. 23] (gis_system.params), all of type R
 * (double for FP64 images, float for FP32 ones); fmaT(a, b, c) (fused
 * multiply-add) and expT(v) (the library's exp, see GIS_SYS_CSTR) may be
 * called, and locals declared.  Compiled with -ffp-contract=off: FP64 images
 * are reproducible bit for bit when the body uses only IEEE operations
 * (+ - * /, fmaT) and expT.  The field replaces the context's previous one;
 * systems of kind GIS_SYS_USER must have its n (1..4) and m (1..2)
 * (GIS_E_INVAL at the call otherwise, and when no field is set).  With ctx
 * NULL the body is only compiled, for gfx950, needing no device.  GIS_E_INVAL
 * if it does not compile (the compiler's messages in gis_last_error()).
 * Synchronises the context's device. */
int32_t gis_set_user_field(gis_ctx* ctx, const char* body, int32_t n, int32_t m);

/* The library's FP64 exponential, the one in the CSTR field (Sec. 4.1,
 * Eq. 4), applied elementwise for parity checks: d_y[i] = exp(d_x[i]),
 * d_x and d_y device arrays of n doubles (they may be the same array), on
 * the current device.  Overflow gives +inf, underflow 0 (through the
 * subnormals), NaN stays NaN.  Synchronises. */
int32_t gis_exp(const double* d_x, int64_t n, double* d_y, void* stream);

const char* gis_last_error(void);
const char* gis_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GIS_H */
