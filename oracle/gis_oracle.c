/*
 * gis_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 CPU implementation of one iteration
 * loop of the graph-based invariant set (GIS) algorithm of Decardi-Nelson and
 * Liu, "An efficient implementation of graph-based invariant set algorithm
 * for constrained nonlinear dynamical systems" (arXiv 2202.06111):
 *   cell coverings (Sec. 2.1), the symbolic image built from one-step images
 *   of the cells (Sec. 2.2, Eqs. 2-3, Definition 1), pruning of cells whose
 *   images leave the covering (Sec. 2.3) and boundary-only subdivision
 *   (Sec. 3.1.1, Algorithm 1, Remark 1).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or
 * helper with the HIP library; the two meet only through the caller's
 * inputs.  Every floating-point step is IEEE binary64 with round-to-nearest;
 * the file must be compiled with -ffp-contract=off and without fast-math so
 * that the only fused operations are the explicit fma() calls written here.
 *
 * Readings of the paper that it takes (the paper leaves these open):
 *  - F(B_i) is approximated by the axis-aligned bounding box of the images of
 *    a fixed set of sample points of B_i under every sampled input
 *    (the paper does not say how the one-step image is formed, Sec. 2.4).
 *  - The discrete-time map of Eq. (1) is nsub classical RK4 substeps of the
 *    ODE over the sampling interval dt, in the fixed operation order of
 *    rk4_substep() below.
 *  - Cells are closed (Sec. 2.1), so a bounding box that only touches a cell
 *    face still produces an edge (Definition 1).
 *  - A (cell, input) image that leaves the state box X, or that covers a part
 *    of X no longer covered by any current cell, is flagged OUT: such an input
 *    cannot keep the cell (zero out-degree argument of Sec. 2.3).
 *  - Pruning keeps the greatest set K of cells such that every cell of K has
 *    an input whose image is not OUT and whose edges all end in K.
 *  - Boundary cells: the delta -> 0+ limit of Algorithm 1, evaluated on the
 *    finest-level index grid; rule 1 ("shell") probes every finest cell
 *    adjacent to the cell, which includes the edge points of Remark 1; rule 2
 *    ("corners") probes the 2^n diagonal corners only (Algorithm 1 as
 *    printed).
 *  - Subdivision splits each boundary cell into its 2^n children, and with a
 *    neighbourhood size N > 0 also the N kept cells nearest to each boundary
 *    cell (Sec. 3.1.2): distances between cell centres in state units, the
 *    cell itself not counted, equal distances ordered by cell id.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- system kinds and sample schemes (the oracle's own numbering) ---- */
enum { OR_LINEAR = 0, OR_VDP = 1, OR_LORENZ = 2, OR_VDP2 = 3, OR_CSTR = 4, OR_USER = 5 };
enum { OR_LATTICE3 = 1, OR_CORNERS_CENTER = 2 };
enum { OR_SHELL = 1, OR_CORNERS = 2 };

typedef struct {
  int32_t kind, n, m, nsub;
  double dt;
  double p[32];
} or_system;

typedef struct {
  int32_t n;
  int32_t n0[4];
  double lo[4], hi[4];
} or_grid;

/* ------------------------------------------------------------------ */
/* exp(x) for the Arrhenius factor of the CSTR model (Sec. 4.1).        */
/* ------------------------------------------------------------------ */
/* The C library's exp is not the same function on every platform, so the
 * oracle fixes its own: Cody-Waite reduction x = k ln2 + r with k the
 * nearest integer to x / ln2 (ties to even) and ln2 split into its double
 * rounding plus the remainder, |r| <= ln2 / 2; exp(r) by the Taylor
 * polynomial of degree 13 (the first omitted term is below 5e-18 there),
 * evaluated by Horner's rule with fused multiply-adds from the highest
 * coefficient; then the exact scaling by 2^k.  Within 1 ulp of exp. */
static const double EXP_INV_LN2 = 0x1.71547652b82fep+0;
static const double EXP_LN2_HI = 0x1.62e42fefa39efp-1;
static const double EXP_LN2_LO = 0x1.abc9e3b39803fp-56;
static const double EXP_TAYLOR[14] = {  /* 1/j!, rounded to nearest */
    0x1.0000000000000p+0, 0x1.0000000000000p+0, 0x1.0000000000000p-1, 0x1.5555555555555p-3,
    0x1.5555555555555p-5, 0x1.1111111111111p-7, 0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13,
    0x1.a01a01a01a01ap-16, 0x1.71de3a556c734p-19, 0x1.27e4fb7789f5cp-22, 0x1.ae64567f544e4p-26,
    0x1.1eed8eff8d898p-29, 0x1.6124613a86d09p-33};

double or_exp(double x) {
  if (x != x) return x;              /* NaN */
  if (x > 709.79) return HUGE_VAL;   /* beyond the largest double */
  if (x < -745.2) return 0.0;        /* below half the smallest subnormal */
  const double k = rint(x * EXP_INV_LN2);
  double r = fma(-k, EXP_LN2_HI, x);
  r = fma(-k, EXP_LN2_LO, r);
  double p = EXP_TAYLOR[13];
  for (int j = 12; j >= 0; --j) p = fma(p, r, EXP_TAYLOR[j]);
  return ldexp(p, (int)k);
}

void or_exp_vec(const double* x, int64_t n, double* y) {
  for (int64_t i = 0; i < n; ++i) y[i] = or_exp(x[i]);
}

/* ------------------------------------------------------------------ */
/* A field given as code by the caller (Eq. 1 takes f as input): the     */
/* Python side compiles its body as C into a library of its own and      */
/* installs the function here.                                           */
/* ------------------------------------------------------------------ */
typedef void (*or_user_fn)(const double* p, const double* x, const double* u, double* dx);
static or_user_fn g_user_field = 0;

void or_set_user_field(or_user_fn f) { g_user_field = f; }

/* ------------------------------------------------------------------ */
/* Vector field f of the ODE whose RK4 discretisation is Eq. (1).      */
/* ------------------------------------------------------------------ */
static void field(const or_system* s, const double* x, const double* u, double* dx) {
  const double* p = s->p;
  switch (s->kind) {
    case OR_LINEAR: {
      /* dx_d = sum_k B[d][k] u_k + sum_j A[d][j] x_j, A = p[0..16) row-major
       * with stride 4, B = p[16..24) row-major with stride 2. */
      for (int d = 0; d < s->n; ++d) {
        double acc = 0.0;
        for (int k = 0; k < s->m; ++k) acc = fma(p[16 + 2 * d + k], u[k], acc);
        for (int j = 0; j < s->n; ++j) acc = fma(p[4 * d + j], x[j], acc);
        dx[d] = acc;
      }
      break;
    }
    case OR_VDP: {
      /* x1' = x2 ;  x2' = mu (1 - x1^2) x2 - x1 + u */
      const double mu = p[0];
      dx[0] = x[1];
      dx[1] = fma(mu * fma(-x[0], x[0], 1.0), x[1], u[0] - x[0]);
      break;
    }
    case OR_LORENZ: {
      /* x1' = sigma (x2 - x1) ; x2' = x1 (rho - x3) - x2 + u ;
       * x3' = x1 x2 - beta x3 */
      const double sigma = p[0], rho = p[1], beta = p[2];
      dx[0] = sigma * (x[1] - x[0]);
      dx[1] = fma(x[0], rho - x[2], u[0] - x[1]);
      dx[2] = fma(x[0], x[1], -(beta * x[2]));
      break;
    }
    case OR_VDP2: {
      /* state (x1, v1, x2, v2); xi'' = (1 - xi^2) xi' - xi + c (xj - xi) + ui */
      const double c = p[0];
      dx[0] = x[1];
      dx[1] = fma(fma(-x[0], x[0], 1.0), x[1], fma(c, x[2] - x[0], u[0] - x[0]));
      dx[2] = x[3];
      dx[3] = fma(fma(-x[2], x[2], 1.0), x[3], fma(c, x[0] - x[2], u[1] - x[2]));
      break;
    }
    case OR_CSTR: {
      /* Eq. (4), state (cA, T), input Tc:
       *   cA' = q/V (cAf - cA) - k0 exp(-(E/R) / T) cA
       *   T'  = q/V (Tf - T) + (-dH / (rho cp)) k0 exp(-(E/R) / T) cA
       *         + UA / (V rho cp) (Tc - T)
       * p = (q/V, cAf, Tf, E/R, k0, -dH/(rho cp), UA/(V rho cp)). */
      const double e = or_exp(-(p[3] / x[1]));
      const double rate = (p[4] * e) * x[0];
      dx[0] = fma(p[0], p[1] - x[0], -rate);
      dx[1] = fma(p[0], p[2] - x[1], fma(p[5], rate, p[6] * (u[0] - x[1])));
      break;
    }
    case OR_USER:
      if (g_user_field) {
        g_user_field(p, x, u, dx);
        break;
      }
      for (int d = 0; d < s->n; ++d) dx[d] = NAN;
      break;
    default:
      for (int d = 0; d < s->n; ++d) dx[d] = NAN;
  }
}

/* One classical fourth-order Runge-Kutta substep of length h. */
static void rk4_substep(const or_system* s, double h, double* x, const double* u) {
  const int n = s->n;
  const double h2 = 0.5 * h, h6 = h / 6.0;
  double k1[4], k2[4], k3[4], k4[4], y[4];
  field(s, x, u, k1);
  for (int d = 0; d < n; ++d) y[d] = fma(h2, k1[d], x[d]);
  field(s, y, u, k2);
  for (int d = 0; d < n; ++d) y[d] = fma(h2, k2[d], x[d]);
  field(s, y, u, k3);
  for (int d = 0; d < n; ++d) y[d] = fma(h, k3[d], x[d]);
  field(s, y, u, k4);
  for (int d = 0; d < n; ++d) {
    double a = k1[d] + k4[d];
    double b = k2[d] + k3[d];
    a = fma(2.0, b, a);
    x[d] = fma(h6, a, x[d]);
  }
}

/* x+ = f(x, u) of Eq. (1): nsub RK4 substeps over one sampling interval. */
void or_step(const or_system* s, const double* x0, const double* u, double* xout) {
  const double h = s->dt / (double)s->nsub;
  double x[4];
  for (int d = 0; d < s->n; ++d) x[d] = x0[d];
  for (int q = 0; q < s->nsub; ++q) rk4_substep(s, h, x, u);
  for (int d = 0; d < s->n; ++d) xout[d] = x[d];
}

/* ------------------------------------------------------------------ */
/* Geometry of the covering (Sec. 2.1)                                 */
/* ------------------------------------------------------------------ */
static double width(const or_grid* g, int d, int level) {
  return ldexp((g->hi[d] - g->lo[d]) / (double)g->n0[d], -level);
}

int32_t or_num_samples(int32_t scheme, int32_t n) {
  if (scheme == OR_LATTICE3) {
    int32_t s = 1;
    for (int d = 0; d < n; ++d) s *= 3;
    return s;
  }
  if (scheme == OR_CORNERS_CENTER) return (1 << n) + 1;
  return 0;
}

/* Offsets k_d in {0,1,2} (lower face, centre, upper face) of sample q. */
static void sample_offsets(int32_t scheme, int n, int q, int* k) {
  if (scheme == OR_LATTICE3) {
    for (int d = n - 1; d >= 0; --d) { k[d] = q % 3; q /= 3; }
  } else if (q == (1 << n)) {
    for (int d = 0; d < n; ++d) k[d] = 1;
  } else {
    for (int d = 0; d < n; ++d) k[d] = 2 * ((q >> (n - 1 - d)) & 1);
  }
}

/* Coordinate of sample q of the cell (level, idx): lo + (2 i + k) * (h / 2). */
static void sample_point(const or_grid* g, int32_t scheme, int level, const int32_t* idx,
                         int q, double* x) {
  int k[4];
  sample_offsets(scheme, g->n, q, k);
  for (int d = 0; d < g->n; ++d)
    x[d] = fma((double)(2 * (int64_t)idx[d] + k[d]), 0.5 * width(g, d, level), g->lo[d]);
}

/* Images of every sample of every (cell, input) row: out[(row*S + q)*n + d].
 * Rows are ordered cell-major: row = cell * K + input. */
void or_images(const or_system* s, const or_grid* g, int32_t scheme, const uint8_t* level,
               const int32_t* idx, int64_t n_cells, const double* u, int32_t K, double* out) {
  const int n = g->n, S = or_num_samples(scheme, n);
  for (int64_t c = 0; c < n_cells; ++c)
    for (int32_t j = 0; j < K; ++j)
      for (int q = 0; q < S; ++q) {
        double x[4];
        sample_point(g, scheme, level[c], idx + c * n, q, x);
        or_step(s, x, u + (int64_t)j * s->m, out + (((c * K + j) * S) + q) * n);
      }
}

/* Bounding box of the sample images of one (cell, input) row.
 * Returns 0 if some image coordinate is not finite. */
static int row_bbox(const or_system* s, const or_grid* g, int32_t scheme, int level,
                    const int32_t* idx, const double* u, double* a, double* b) {
  const int n = g->n, S = or_num_samples(scheme, n);
  int finite = 1;
  for (int d = 0; d < n; ++d) { a[d] = INFINITY; b[d] = -INFINITY; }
  for (int q = 0; q < S; ++q) {
    double x[4], y[4];
    sample_point(g, scheme, level, idx, q, x);
    or_step(s, x, u, y);
    for (int d = 0; d < n; ++d) {
      if (!isfinite(y[d])) finite = 0;
      if (y[d] < a[d]) a[d] = y[d];
      if (y[d] > b[d]) b[d] = y[d];
    }
  }
  return finite;
}

/* Position of v on the finest grid of spacing hs, clamped to [-2, N+2]
 * (the clamp only keeps the integer conversion defined; it never changes a
 * clamped range below). */
static double grid_pos(double v, double lo, double hs, int64_t N) {
  double t = (v - lo) / hs;
  if (t < -2.0) t = -2.0;
  if (t > (double)N + 2.0) t = (double)N + 2.0;
  return t;
}

/* Index ranges on the finest grid (cells of N per dimension, spacing hs)
 * covered by the box [a, b]:
 *   R  : closed cells meeting [a,b] (touching counts, Definition 1)
 *   Ri : cells whose interior meets the open box; if empty, R.
 * Returns OUT_X: the box leaves the closed state box X. */
int32_t or_cover(const or_grid* g, int32_t Lstar, const double* a, const double* b,
                 int64_t* R, int64_t* Ri) {
  int out = 0;
  for (int d = 0; d < g->n; ++d) {
    const int64_t N = (int64_t)g->n0[d] << Lstar;
    const double hs = width(g, d, Lstar);
    const double ta = grid_pos(a[d], g->lo[d], hs, N);
    const double tb = grid_pos(b[d], g->lo[d], hs, N);
    int64_t rlo = (int64_t)ceil(ta) - 1, rhi = (int64_t)floor(tb);
    int64_t ilo = (int64_t)floor(ta), ihi = (int64_t)ceil(tb) - 1;
    if (rlo < 0) rlo = 0;
    if (rhi > N - 1) rhi = N - 1;
    if (ilo < 0) ilo = 0;
    if (ihi > N - 1) ihi = N - 1;
    if (ilo > ihi) { ilo = rlo; ihi = rhi; }
    R[2 * d] = rlo; R[2 * d + 1] = rhi;
    Ri[2 * d] = ilo; Ri[2 * d + 1] = ihi;
    if (a[d] < g->lo[d] || b[d] > g->hi[d]) out = 1;
  }
  return out;
}

/* ------------------------------------------------------------------ */
/* Owner map: which current cell contains each finest-level cell.      */
/* ------------------------------------------------------------------ */
static int64_t finest_count(const or_grid* g, int Lstar) {
  int64_t t = 1;
  for (int d = 0; d < g->n; ++d) t *= (int64_t)g->n0[d] << Lstar;
  return t;
}

static int64_t finest_lin(const or_grid* g, int Lstar, const int64_t* k) {
  int64_t lin = 0;
  for (int d = 0; d < g->n; ++d) lin = lin * ((int64_t)g->n0[d] << Lstar) + k[d];
  return lin;
}

int32_t or_max_level(const uint8_t* level, int64_t n_cells) {
  int32_t L = 0;
  for (int64_t c = 0; c < n_cells; ++c) if (level[c] > L) L = level[c];
  return L;
}

/* Fills owner[finest cell] with the index of the cell containing it, or -1.
 * Cells with keep != NULL && keep[c] == 0 are left out.  Returns -1 if two
 * cells overlap or a cell lies outside the grid, else 0. */
static int build_owner(const or_grid* g, int Lstar, const uint8_t* level, const int32_t* idx,
                       int64_t n_cells, const uint8_t* keep, int32_t* owner) {
  const int n = g->n;
  const int64_t total = finest_count(g, Lstar);
  for (int64_t k = 0; k < total; ++k) owner[k] = -1;
  for (int64_t c = 0; c < n_cells; ++c) {
    if (keep && !keep[c]) continue;
    const int sh = Lstar - level[c];
    if (sh < 0) return -1;
    int64_t lo[4], hi[4], k[4];
    for (int d = 0; d < n; ++d) {
      if (idx[c * n + d] < 0 || (int64_t)idx[c * n + d] >= ((int64_t)g->n0[d] << level[c])) return -1;
      lo[d] = (int64_t)idx[c * n + d] << sh;
      hi[d] = lo[d] + ((int64_t)1 << sh) - 1;
      k[d] = lo[d];
    }
    for (;;) {
      const int64_t lin = finest_lin(g, Lstar, k);
      if (owner[lin] != -1) return -1;
      owner[lin] = (int32_t)c;
      int d = n - 1;
      while (d >= 0 && k[d] == hi[d]) { k[d] = lo[d]; --d; }
      if (d < 0) break;
      ++k[d];
    }
  }
  return 0;
}

static int cmp_i32(const void* x, const void* y) {
  const int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
  return (a > b) - (a < b);
}

/* Edges and OUT flag of one row given its bounding box. Writes the ascending
 * distinct owners of the finest cells of the closed range into tmp, returns
 * the edge count; *out_flag receives the OUT decision. */
static int64_t row_edges(const or_grid* g, int Lstar, const int32_t* owner, int finite,
                         const double* a, const double* b, int32_t* tmp, int64_t tmp_cap,
                         int* out_flag) {
  const int n = g->n;
  if (!finite) { *out_flag = 1; return 0; }
  int64_t R[8], Ri[8], k[4];
  int out = or_cover(g, Lstar, a, b, R, Ri);
  /* hole test: a finest cell of the interior range owned by no current cell */
  int empty = 0;
  for (int d = 0; d < n; ++d) if (Ri[2 * d] > Ri[2 * d + 1]) empty = 1;
  if (!out && !empty) {
    for (int d = 0; d < n; ++d) k[d] = Ri[2 * d];
    for (;;) {
      if (owner[finest_lin(g, Lstar, k)] < 0) { out = 1; break; }
      int d = n - 1;
      while (d >= 0 && k[d] == Ri[2 * d + 1]) { k[d] = Ri[2 * d]; --d; }
      if (d < 0) break;
      ++k[d];
    }
  }
  *out_flag = out;
  empty = 0;
  for (int d = 0; d < n; ++d) if (R[2 * d] > R[2 * d + 1]) empty = 1;
  if (empty) return 0;
  int64_t cnt = 0;
  for (int d = 0; d < n; ++d) k[d] = R[2 * d];
  for (;;) {
    const int32_t o = owner[finest_lin(g, Lstar, k)];
    if (o >= 0) {
      if (cnt >= tmp_cap) return -1;
      tmp[cnt++] = o;
    }
    int d = n - 1;
    while (d >= 0 && k[d] == R[2 * d + 1]) { k[d] = R[2 * d]; --d; }
    if (d < 0) break;
    ++k[d];
  }
  qsort(tmp, (size_t)cnt, sizeof(int32_t), cmp_i32);
  int64_t u = 0;
  for (int64_t i = 0; i < cnt; ++i)
    if (u == 0 || tmp[u - 1] != tmp[i]) tmp[u++] = tmp[i];
  return u;
}

/* Symbolic image (Definition 1) of the covering given as a cell list.
 * rows: the row indices (cell*K + input) to evaluate, or NULL for all rows in
 * order.  Outputs per evaluated row i: cnt[i] edges, out[i] flag; the edge
 * targets of all rows, ascending within a row, go to *col_out, a buffer this
 * function allocates (release it with or_free).
 * fast_out != 0 drops the edges of OUT rows.
 * Returns the total number of edges, or -1 on an invalid covering, -2 on
 * memory exhaustion. */
int64_t or_build(const or_system* s, const or_grid* g, int32_t scheme, const uint8_t* level,
                 const int32_t* idx, int64_t n_cells, const double* u, int32_t K,
                 int32_t fast_out, const int64_t* rows, int64_t n_rows, int64_t* cnt,
                 uint8_t* out, int32_t** col_out) {
  const int n = g->n;
  const int Lstar = or_max_level(level, n_cells);
  const int64_t total = finest_count(g, Lstar);
  int32_t* owner = (int32_t*)malloc(sizeof(int32_t) * (size_t)total);
  const int64_t tmp_cap = 1 << 24;
  int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)tmp_cap);
  int64_t written = 0, cap_col = 1024;
  int32_t* col = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap_col);
  *col_out = NULL;
  if (!owner || !tmp || !col) { free(owner); free(tmp); free(col); return -2; }
  if (build_owner(g, Lstar, level, idx, n_cells, NULL, owner) != 0) {
    free(owner); free(tmp); free(col); return -1;
  }
  if (!rows) n_rows = n_cells * K;
  for (int64_t i = 0; i < n_rows; ++i) {
    const int64_t r = rows ? rows[i] : i;
    const int64_t c = r / K;
    const int32_t j = (int32_t)(r % K);
    double a[4], b[4];
    const int finite = row_bbox(s, g, scheme, level[c], idx + c * n, u + (int64_t)j * s->m, a, b);
    int of = 0;
    int64_t e = row_edges(g, Lstar, owner, finite, a, b, tmp, tmp_cap, &of);
    if (e < 0) { free(owner); free(tmp); free(col); return -2; }
    if (fast_out && of) e = 0;
    cnt[i] = e;
    out[i] = (uint8_t)of;
    if (written + e > cap_col) {
      while (written + e > cap_col) cap_col *= 2;
      int32_t* grown = (int32_t*)realloc(col, sizeof(int32_t) * (size_t)cap_col);
      if (!grown) { free(owner); free(tmp); free(col); return -2; }
      col = grown;
    }
    for (int64_t q = 0; q < e; ++q) col[written + q] = tmp[q];
    written += e;
  }
  free(owner);
  free(tmp);
  *col_out = col;
  return written;
}

void or_free(void* p) { free(p); }

/* Bounding boxes of selected rows (for parity of the image stage). */
void or_bboxes(const or_system* s, const or_grid* g, int32_t scheme, const uint8_t* level,
               const int32_t* idx, const double* u, int32_t K, const int64_t* rows, int64_t n_rows,
               double* a, double* b, uint8_t* finite) {
  const int n = g->n;
  for (int64_t i = 0; i < n_rows; ++i) {
    const int64_t c = rows[i] / K;
    const int32_t j = (int32_t)(rows[i] % K);
    finite[i] = (uint8_t)row_bbox(s, g, scheme, level[c], idx + c * n, u + (int64_t)j * s->m,
                                  a + i * n, b + i * n);
  }
}

/* ------------------------------------------------------------------ */
/* Graph analysis (Sec. 2.3), two readings, both as plain synchronous   */
/* sweeps K_{t+1} = {c in K_t : exists u with good_t(c, u)} from K_0 =  */
/* every cell until nothing changes.                                     */
/*  analysis 1 (controlled invariance): good(c,u) <=> the row is not OUT */
/*    and every edge of the row ends in K_t; K* is the largest cell set  */
/*    in which each cell has an input keeping its whole image inside.    */
/*  analysis 2 (non-leaving cells, Definitions 5-6): good(c,u) <=> some  */
/*    edge of the row ends in K_t; K* is the set of vertices of the      */
/*    input-union symbolic image with an infinite admissible path.       */
/* mask(c) = {u : good*(c,u)} for c in K*, else empty.                   */
/* ------------------------------------------------------------------ */
static int row_good(int32_t analysis, const int64_t* row_ptr, const int32_t* col,
                    const uint8_t* out, const uint8_t* kept, int64_t r) {
  if (analysis == 2) {
    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e)
      if (kept[col[e]]) return 1;
    return 0;
  }
  if (out[r]) return 0;
  for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e)
    if (!kept[col[e]]) return 0;
  return 1;
}

int32_t or_prune(const int64_t* row_ptr, const int32_t* col, const uint8_t* out, int64_t n_cells,
                 int32_t K, int32_t analysis, uint8_t* kept, uint64_t* mask, int32_t mask_words) {
  uint8_t* next = (uint8_t*)malloc((size_t)(n_cells > 0 ? n_cells : 1));
  for (int64_t c = 0; c < n_cells; ++c) kept[c] = 1;
  int32_t sweeps = 0;
  for (;;) {
    int changed = 0;
    for (int64_t c = 0; c < n_cells; ++c) {
      next[c] = 0;
      if (!kept[c]) continue;
      for (int32_t j = 0; j < K && !next[c]; ++j)
        if (row_good(analysis, row_ptr, col, out, kept, c * K + j)) next[c] = 1;
      if (!next[c]) changed = 1;
    }
    if (!changed) break;
    memcpy(kept, next, (size_t)n_cells);
    ++sweeps;
  }
  for (int64_t c = 0; c < n_cells; ++c) {
    for (int w = 0; w < mask_words; ++w) mask[c * mask_words + w] = 0;
    if (!kept[c]) continue;
    for (int32_t j = 0; j < K; ++j)
      if (row_good(analysis, row_ptr, col, out, kept, c * K + j))
        mask[c * mask_words + j / 64] |= (uint64_t)1 << (j % 64);
  }
  free(next);
  return sweeps;
}

/* ------------------------------------------------------------------ */
/* Boundary selection (Sec. 3.1.1, Algorithm 1, Remark 1), in the limit */
/* of a vanishing enlargement, on the finest-level index grid.          */
/* ------------------------------------------------------------------ */
int32_t or_boundary(const or_grid* g, const uint8_t* level, const int32_t* idx, int64_t n_cells,
                    const uint8_t* kept, int32_t rule, uint8_t* boundary) {
  const int n = g->n;
  const int Lstar = or_max_level(level, n_cells);
  const int64_t total = finest_count(g, Lstar);
  int32_t* owner = (int32_t*)malloc(sizeof(int32_t) * (size_t)total);
  if (!owner) return -2;
  if (build_owner(g, Lstar, level, idx, n_cells, kept, owner) != 0) { free(owner); return -1; }
  for (int64_t c = 0; c < n_cells; ++c) {
    boundary[c] = 0;
    if (!kept[c]) continue;
    const int sh = Lstar - level[c];
    int64_t lo[4], hi[4], k[4];
    for (int d = 0; d < n; ++d) {
      lo[d] = ((int64_t)idx[c * n + d] << sh) - 1;
      hi[d] = (((int64_t)idx[c * n + d] + 1) << sh);
      k[d] = lo[d];
    }
    for (;;) {
      int on_shell = 0, on_corner = 1, outside = 0;
      for (int d = 0; d < n; ++d) {
        if (k[d] == lo[d] || k[d] == hi[d]) on_shell = 1; else on_corner = 0;
        if (k[d] < 0 || k[d] >= ((int64_t)g->n0[d] << Lstar)) outside = 1;
      }
      const int probe = (rule == OR_CORNERS) ? on_corner : on_shell;
      if (probe && (outside || owner[finest_lin(g, Lstar, k)] < 0)) { boundary[c] = 1; break; }
      int d = n - 1;
      while (d >= 0 && k[d] == hi[d]) { k[d] = lo[d]; --d; }
      if (d < 0) break;
      ++k[d];
    }
  }
  free(owner);
  return 0;
}

/* canonical order: level, then row-major multi-index (dimension 0 slowest) */
static int g_sort_n;
static int cmp_cell(const void* x, const void* y) {
  const int32_t* a = (const int32_t*)x;
  const int32_t* b = (const int32_t*)y;
  for (int d = 0; d <= g_sort_n; ++d) {
    if (a[d] != b[d]) return a[d] < b[d] ? -1 : 1;
  }
  return 0;
}

/* Next covering: the 2^n children of every boundary cell plus every other
 * kept cell, in canonical order. Returns the new cell count (or the needed
 * count if it exceeds cap; nothing is written then). */
int64_t or_subdivide(const or_grid* g, const uint8_t* level, const int32_t* idx, int64_t n_cells,
                     const uint8_t* kept, const uint8_t* boundary, uint8_t* level_out,
                     int32_t* idx_out, int64_t cap) {
  const int n = g->n;
  int64_t cnt = 0;
  for (int64_t c = 0; c < n_cells; ++c)
    if (kept[c]) cnt += boundary[c] ? (1 << n) : 1;
  if (cnt > cap) return cnt;
  int32_t* rec = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cnt > 0 ? cnt : 1) * (n + 1));
  int64_t w = 0;
  for (int64_t c = 0; c < n_cells; ++c) {
    if (!kept[c]) continue;
    if (!boundary[c]) {
      rec[w * (n + 1)] = level[c];
      for (int d = 0; d < n; ++d) rec[w * (n + 1) + 1 + d] = idx[c * n + d];
      ++w;
      continue;
    }
    for (int ch = 0; ch < (1 << n); ++ch) {
      rec[w * (n + 1)] = level[c] + 1;
      for (int d = 0; d < n; ++d)
        rec[w * (n + 1) + 1 + d] = 2 * idx[c * n + d] + ((ch >> (n - 1 - d)) & 1);
      ++w;
    }
  }
  g_sort_n = n;
  qsort(rec, (size_t)cnt, sizeof(int32_t) * (n + 1), cmp_cell);
  for (int64_t i = 0; i < cnt; ++i) {
    level_out[i] = (uint8_t)rec[i * (n + 1)];
    for (int d = 0; d < n; ++d) idx_out[i * n + d] = rec[i * (n + 1) + 1 + d];
  }
  free(rec);
  return cnt;
}

/* ------------------------------------------------------------------ */
/* Neighbourhood of the boundary cells (Sec. 3.1.2, Figure 5): for each  */
/* boundary cell, the N kept cells whose centres lie nearest to its      */
/* centre, by brute force over every kept cell.                          */
/* ------------------------------------------------------------------ */
typedef struct {
  double d2;
  int64_t id;
} or_nb;

static int cmp_nb(const void* x, const void* y) {
  const or_nb* a = (const or_nb*)x;
  const or_nb* b = (const or_nb*)y;
  if (a->d2 != b->d2) return a->d2 < b->d2 ? -1 : 1;
  return a->id < b->id ? -1 : (a->id > b->id ? 1 : 0);
}

/* Squared Euclidean distance (state units) between the centres of cells a
 * and b.  The centre of a level-L cell with index i lies at
 * lo + (2 i + 1) w_L / 2; on the grid of half the finest width every centre
 * is an integer point, so the difference of two centres is formed exactly
 * there, then scaled by that half width, squared and summed over the
 * dimensions in order.  */
static double centre_d2(const or_grid* g, int Lstar, const uint8_t* level, const int32_t* idx,
                        int64_t a, int64_t b) {
  double s = 0.0;
  for (int d = 0; d < g->n; ++d) {
    const int64_t ca = (2 * (int64_t)idx[a * g->n + d] + 1) << (Lstar - level[a]);
    const int64_t cb = (2 * (int64_t)idx[b * g->n + d] + 1) << (Lstar - level[b]);
    const double t = (double)(ca - cb) * width(g, d, Lstar + 1);
    s = s + t * t;
  }
  return s;
}

/* sel[c] = 1 for every boundary cell (kept and boundary[c]) and for the N
 * kept cells nearest to some boundary cell (the cell itself not counted;
 * equal distances ordered by cell id); 0 otherwise.  Returns 0, or -2 when
 * out of memory. */
int32_t or_neighbours(const or_grid* g, const uint8_t* level, const int32_t* idx, int64_t n_cells,
                      const uint8_t* kept, const uint8_t* boundary, int32_t N, uint8_t* sel) {
  const int Lstar = or_max_level(level, n_cells);
  or_nb* cand = (or_nb*)malloc(sizeof(or_nb) * (size_t)(n_cells > 0 ? n_cells : 1));
  if (!cand) return -2;
  for (int64_t c = 0; c < n_cells; ++c) sel[c] = (kept[c] && boundary[c]) ? 1 : 0;
  for (int64_t b = 0; b < n_cells && N > 0; ++b) {
    if (!(kept[b] && boundary[b])) continue;
    int64_t m = 0;
    for (int64_t j = 0; j < n_cells; ++j) {
      if (j == b || !kept[j]) continue;
      cand[m].d2 = centre_d2(g, Lstar, level, idx, b, j);
      cand[m].id = j;
      ++m;
    }
    qsort(cand, (size_t)m, sizeof(or_nb), cmp_nb);
    for (int64_t k = 0; k < m && k < N; ++k) sel[cand[k].id] = 1;
  }
  free(cand);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Queries on a pruned covering: membership of a state in the kept set  */
/* and the admissible-input mask of the cell containing it.             */
/* ------------------------------------------------------------------ */
int32_t or_query(const or_grid* g, const uint8_t* level, const int32_t* idx, int64_t n_cells,
                 const uint8_t* kept, const uint64_t* mask, int32_t mask_words, const double* x,
                 int64_t n_states, uint8_t* member, uint64_t* adm) {
  const int n = g->n;
  const int Lstar = or_max_level(level, n_cells);
  const int64_t total = finest_count(g, Lstar);
  int32_t* owner = (int32_t*)malloc(sizeof(int32_t) * (size_t)total);
  if (!owner) return -2;
  if (build_owner(g, Lstar, level, idx, n_cells, kept, owner) != 0) { free(owner); return -1; }
  for (int64_t i = 0; i < n_states; ++i) {
    member[i] = 0;
    for (int w = 0; w < mask_words; ++w) adm[i * mask_words + w] = 0;
    int inside = 1;
    int64_t k[4];
    for (int d = 0; d < n; ++d) {
      const double v = x[i * n + d];
      if (!(v >= g->lo[d] && v <= g->hi[d])) { inside = 0; break; }
      const int64_t N = (int64_t)g->n0[d] << Lstar;
      int64_t kd = (int64_t)floor((v - g->lo[d]) / width(g, d, Lstar));
      if (kd > N - 1) kd = N - 1;
      k[d] = kd;
    }
    if (!inside) continue;
    const int32_t o = owner[finest_lin(g, Lstar, k)];
    if (o < 0) continue;
    member[i] = 1;
    for (int w = 0; w < mask_words; ++w) adm[i * mask_words + w] = mask[(int64_t)o * mask_words + w];
  }
  free(owner);
  return 0;
}
