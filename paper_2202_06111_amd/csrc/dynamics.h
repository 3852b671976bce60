// Device-side dynamics: the built-in vector fields, the RK4 discretisation
// x+ = f(x, u) of Eq. (1) and the sample points of a cell.
//
// The FP64 instantiation is the reference arithmetic of the library: every
// operation is IEEE binary64 round-to-nearest, the only fused operations are
// the explicit fma() calls below, and the translation unit is compiled with
// -ffp-contract=off, so the results are reproducible operation by operation.
// The FP32 instantiation runs the same operation sequence in binary32 with
// the constants rounded to nearest; its results only steer which rows need
// the FP64 recheck.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#include "gis_internal.h"

namespace gis {

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Minimum and maximum as single VALU instructions.  fmin/fmax compile to the
// same instructions preceded by a copy of each operand that quiets signalling
// NaNs (the compiler cannot see that loop-carried values are already quiet),
// three extra instructions per coordinate and sample.  A NaN image is decided
// by the caller's finiteness test either way.
__device__ __forceinline__ double vmin(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double vmax(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ float vmin(float a, float b) {
  float r;
  asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ float vmax(float a, float b) {
  float r;
  asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// exp(x) for the Arrhenius factor of the CSTR field (Sec. 4.1).  The device
// library's exp is not bound to any particular rounding, so the library fixes
// its own: Cody-Waite reduction x = k ln2 + r with k = rint(x / ln2) (ties to
// even) and ln2 split into its rounding plus the remainder, |r| <= ln2 / 2;
// exp(r) by its Taylor polynomial of degree 13 (the first omitted term is
// below 5e-18 there) in Horner form with fused multiply-adds from the highest
// coefficient; then the exact scaling by 2^k.  Every step is one correctly
// rounded IEEE operation, so the FP64 result does not depend on the machine;
// it is within 1 ulp of exp.  The FP32 instantiation runs the same sequence
// with binary32 constants (ln2 split at binary32) and binary32 limits.
template <typename R>
struct ExpConsts;
template <>
struct ExpConsts<double> {
  static constexpr double inv_ln2 = 0x1.71547652b82fep+0;
  static constexpr double ln2_hi = 0x1.62e42fefa39efp-1;
  static constexpr double ln2_lo = 0x1.abc9e3b39803fp-56;
  static constexpr double over = 709.79;   // beyond the largest finite value
  static constexpr double under = -745.2;  // below half the smallest subnormal
};
template <>
struct ExpConsts<float> {
  static constexpr float inv_ln2 = 0x1.715476p+0f;
  static constexpr float ln2_hi = 0x1.62e430p-1f;
  static constexpr float ln2_lo = -0x1.05c610p-29f;
  static constexpr float over = 88.73f;
  static constexpr float under = -103.98f;
};

// 1/j!, j = 0..13, rounded to nearest binary64.
__device__ constexpr double kExpTaylor[14] = {
    0x1.0000000000000p+0, 0x1.0000000000000p+0, 0x1.0000000000000p-1, 0x1.5555555555555p-3,
    0x1.5555555555555p-5, 0x1.1111111111111p-7, 0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13,
    0x1.a01a01a01a01ap-16, 0x1.71de3a556c734p-19, 0x1.27e4fb7789f5cp-22, 0x1.ae64567f544e4p-26,
    0x1.1eed8eff8d898p-29, 0x1.6124613a86d09p-33};

__device__ __forceinline__ double rintT(double v) { return __builtin_rint(v); }
__device__ __forceinline__ float rintT(float v) { return __builtin_rintf(v); }
__device__ __forceinline__ double ldexpT(double v, int e) { return __builtin_ldexp(v, e); }
__device__ __forceinline__ float ldexpT(float v, int e) { return __builtin_ldexpf(v, e); }

template <typename R>
__device__ __forceinline__ R expT(R x) {
  using C = ExpConsts<R>;
  if (x != x) return x;
  if (x > C::over) return R(__builtin_huge_val());
  if (x < C::under) return R(0);
  const R k = rintT(x * C::inv_ln2);
  R r = fmaT(-k, C::ln2_hi, x);
  r = fmaT(-k, C::ln2_lo, r);
  R p = R(kExpTaylor[13]);
#pragma unroll
  for (int j = 12; j >= 0; --j) p = fmaT(p, r, R(kExpTaylor[j]));
  return ldexpT(p, (int)k);
}

// The field of kind GIS_SYS_USER: the caller's code, compiled at run time
// (rtc.hip defines it in the runtime-compiled program; the static library
// never instantiates it).  p: parameters, x: state, u: input, dx: g(x, u).
template <typename R>
__device__ void user_field(const R* p, const R* x, const R* u, R* dx);

// Vector field g(x, u) of x' = g(x, u).  N is the state dimension; m (inputs)
// is only a runtime value for the linear field.
template <int KIND, int N, typename R>
__device__ __forceinline__ void field(const R* __restrict__ p, int m, const R* x, const R* u, R* dx) {
  if constexpr (KIND == GIS_SYS_LINEAR) {
#pragma unroll
    for (int d = 0; d < N; ++d) {
      R acc = R(0);
      for (int k = 0; k < m; ++k) acc = fmaT(p[16 + 2 * d + k], u[k], acc);
#pragma unroll
      for (int j = 0; j < N; ++j) acc = fmaT(p[4 * d + j], x[j], acc);
      dx[d] = acc;
    }
  } else if constexpr (KIND == GIS_SYS_VDP) {
    dx[0] = x[1];
    dx[1] = fmaT(p[0] * fmaT(-x[0], x[0], R(1)), x[1], u[0] - x[0]);
  } else if constexpr (KIND == GIS_SYS_LORENZ) {
    dx[0] = p[0] * (x[1] - x[0]);
    dx[1] = fmaT(x[0], p[1] - x[2], u[0] - x[1]);
    dx[2] = fmaT(x[0], x[1], -(p[2] * x[2]));
  } else if constexpr (KIND == GIS_SYS_USER) {
    user_field<R>(p, x, u, dx);
  } else if constexpr (KIND == GIS_SYS_CSTR) {
    // Eq. (4), state (cA, T), input Tc; p = (q/V, cAf, Tf, E/R, k0,
    // -dH/(rho cp), UA/(V rho cp)); the reaction rate k0 exp(-(E/R)/T) cA
    // enters both equations.
    const R e = expT<R>(-(p[3] / x[1]));
    const R rate = (p[4] * e) * x[0];
    dx[0] = fmaT(p[0], p[1] - x[0], -rate);
    dx[1] = fmaT(p[0], p[2] - x[1], fmaT(p[5], rate, p[6] * (u[0] - x[1])));
  } else {  // GIS_SYS_VDP2, state (x1, v1, x2, v2)
    dx[0] = x[1];
    dx[1] = fmaT(fmaT(-x[0], x[0], R(1)), x[1], fmaT(p[0], x[2] - x[0], u[0] - x[0]));
    dx[2] = x[3];
    dx[3] = fmaT(fmaT(-x[2], x[2], R(1)), x[3], fmaT(p[0], x[0] - x[2], u[1] - x[2]));
  }
}

// Substep constants and parameters in the working precision.
template <typename R>
struct Rk4Consts {
  R h, h2, h6;
  R p[24];
};

template <typename R>
__device__ __forceinline__ Rk4Consts<R> make_consts(const SysArgs& s) {
  Rk4Consts<R> c;
  c.h = R(s.h);
  c.h2 = R(s.h2);
  c.h6 = R(s.h6);
#pragma unroll
  for (int i = 0; i < 24; ++i) c.p[i] = R(s.p[i]);
  return c;
}

// nsub classical RK4 substeps, in place.
template <int KIND, int N, typename R>
__device__ __forceinline__ void rk4(const Rk4Consts<R>& c, int m, int nsub, R* x, const R* u) {
  for (int q = 0; q < nsub; ++q) {
    R k1[N], k2[N], k3[N], k4[N], y[N];
    field<KIND, N, R>(c.p, m, x, u, k1);
#pragma unroll
    for (int d = 0; d < N; ++d) y[d] = fmaT(c.h2, k1[d], x[d]);
    field<KIND, N, R>(c.p, m, y, u, k2);
#pragma unroll
    for (int d = 0; d < N; ++d) y[d] = fmaT(c.h2, k2[d], x[d]);
    field<KIND, N, R>(c.p, m, y, u, k3);
#pragma unroll
    for (int d = 0; d < N; ++d) y[d] = fmaT(c.h, k3[d], x[d]);
    field<KIND, N, R>(c.p, m, y, u, k4);
#pragma unroll
    for (int d = 0; d < N; ++d) {
      R s = k1[d] + k4[d];
      R t = k2[d] + k3[d];
      s = fmaT(R(2), t, s);
      x[d] = fmaT(c.h6, s, x[d]);
    }
  }
}

// The same for P independent states advanced in lockstep: the P dependency
// chains interleave, which hides arithmetic latency at low occupancy.  Each
// state sees exactly the operation sequence of rk4().
template <int KIND, int N, int P, typename R>
__device__ __forceinline__ void rk4_multi(const Rk4Consts<R>& c, int m, int nsub, R (*x)[N],
                                          const R* u) {
  for (int q = 0; q < nsub; ++q) {
    R k1[P][N], k2[P][N], k3[P][N], k4[P][N], y[P][N];
#pragma unroll
    for (int i = 0; i < P; ++i) field<KIND, N, R>(c.p, m, x[i], u, k1[i]);
#pragma unroll
    for (int i = 0; i < P; ++i)
#pragma unroll
      for (int d = 0; d < N; ++d) y[i][d] = fmaT(c.h2, k1[i][d], x[i][d]);
#pragma unroll
    for (int i = 0; i < P; ++i) field<KIND, N, R>(c.p, m, y[i], u, k2[i]);
#pragma unroll
    for (int i = 0; i < P; ++i)
#pragma unroll
      for (int d = 0; d < N; ++d) y[i][d] = fmaT(c.h2, k2[i][d], x[i][d]);
#pragma unroll
    for (int i = 0; i < P; ++i) field<KIND, N, R>(c.p, m, y[i], u, k3[i]);
#pragma unroll
    for (int i = 0; i < P; ++i)
#pragma unroll
      for (int d = 0; d < N; ++d) y[i][d] = fmaT(c.h, k3[i][d], x[i][d]);
#pragma unroll
    for (int i = 0; i < P; ++i) field<KIND, N, R>(c.p, m, y[i], u, k4[i]);
#pragma unroll
    for (int i = 0; i < P; ++i)
#pragma unroll
      for (int d = 0; d < N; ++d) {
        R s = k1[i][d] + k4[i][d];
        R t = k2[i][d] + k3[i][d];
        s = fmaT(R(2), t, s);
        x[i][d] = fmaT(c.h6, s, x[i][d]);
      }
  }
}

__host__ __device__ constexpr int ipow3(int n) { return n <= 0 ? 1 : 3 * ipow3(n - 1); }

__device__ __forceinline__ int num_samples(int scheme, int n) {
  return scheme == GIS_SAMPLES_LATTICE3 ? ipow3(n) : (1 << n) + 1;
}

// Offset k_d in {0, 1, 2} (lower face, centre, upper face) of sample q:
// LATTICE3 enumerates base-3 digits with dimension 0 most significant;
// CORNERS_CENTER enumerates the corners by bits (dimension 0 most
// significant) and puts the centre last.
template <int N>
__device__ __forceinline__ void sample_offsets(int scheme, int q, int* k) {
  if (scheme == GIS_SAMPLES_LATTICE3) {
#pragma unroll
    for (int d = N - 1; d >= 0; --d) {
      k[d] = q % 3;
      q /= 3;
    }
  } else if (q == (1 << N)) {
#pragma unroll
    for (int d = 0; d < N; ++d) k[d] = 1;
  } else {
#pragma unroll
    for (int d = 0; d < N; ++d) k[d] = 2 * ((q >> (N - 1 - d)) & 1);
  }
}

// Sample coordinates (FP64): lo_d + (2 i_d + k_d) * (w_{L,d} / 2).
template <int N>
__device__ __forceinline__ void sample_point(const GridArgs& g, int level, const int32_t* i,
                                             const int* k, double* x) {
#pragma unroll
  for (int d = 0; d < N; ++d) {
    const double half = 0.5 * ldexp(g.w0[d], -level);
    // 2 i + k < 2^32 for every index below 2^31 - 1: one exact u32 -> f64 conversion
    x[d] = __builtin_fma((double)(2u * (uint32_t)i[d] + (uint32_t)k[d]), half, g.lo[d]);
  }
}

}  // namespace gis
