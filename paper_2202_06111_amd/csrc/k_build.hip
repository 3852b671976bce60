// Launchers of the graph-construction kernels (k_build_dev.h) for the
// built-in fields, and the small kernels of the build phase (the library's
// exponential, the recheck band).  Fields of kind GIS_SYS_USER go to the
// runtime-compiled kernels of rtc.hip.
#include <float.h>
#include <math.h>

#include "k_build_dev.h"
#include "gis_internal.h"
#include "gis_rtc.h"

namespace gis {

namespace {

using kbuild::k_build;
using kbuild::k_images;
using kbuild::k_calibrate;

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
    case GIS_SYS_CSTR:
      if (n == 2) return Launcher<GIS_SYS_CSTR, 2>::run(args...);
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
struct Build {
  static int32_t run(const BuildArgs& a, int32_t precision, hipStream_t s) {
    if (a.n_blocks == 0) return GIS_OK;
    const dim3 g((unsigned)a.n_blocks), b(kRowBlock);
    if (precision == GIS_PREC_FP32_RECHECK) {
      if (a.all_uniform) hipLaunchKernelGGL((k_build<KIND, N, true, true>), g, b, 0, s, a);
      else hipLaunchKernelGGL((k_build<KIND, N, true, false>), g, b, 0, s, a);
    } else {
      if (a.all_uniform) hipLaunchKernelGGL((k_build<KIND, N, false, true>), g, b, 0, s, a);
      else hipLaunchKernelGGL((k_build<KIND, N, false, false>), g, b, 0, s, a);
    }
    GIS_LAUNCH_CHECK("k_build");
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
  static int32_t run(const BuildArgs& a, unsigned long long* maxerr, int64_t stride, hipStream_t s) {
    if (a.n_blocks == 0) return GIS_OK;
    hipLaunchKernelGGL((k_calibrate<KIND, N>), dim3((unsigned)a.n_blocks), dim3(kRowBlock), 0, s, a,
                       maxerr, stride < 1 ? (int64_t)1 : stride);
    GIS_LAUNCH_CHECK("k_calibrate");
    return GIS_OK;
  }
};

}  // namespace

int32_t launch_build(const BuildArgs& a, int32_t precision, hipStream_t s) {
  if (a.kind == GIS_SYS_USER) return user_launch_build(a, precision, s);
  return dispatch_sys<Build>(a.kind, a.n, a, precision, s);
}

int32_t launch_images(const BuildArgs& a, int32_t precision, double* d_images, hipStream_t s) {
  if (a.kind == GIS_SYS_USER) return user_launch_images(a, precision, d_images, s);
  return dispatch_sys<Images>(a.kind, a.n, a, precision, d_images, s);
}

namespace {
__global__ void k_exp(const double* __restrict__ x, int64_t n, double* __restrict__ y) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step)
    y[i] = expT<double>(x[i]);
}
}  // namespace

int32_t launch_exp(const double* d_x, int64_t n, double* d_y, hipStream_t s) {
  if (n <= 0) return GIS_OK;
  const int64_t blocks = (n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192;
  hipLaunchKernelGGL(k_exp, dim3((unsigned)blocks), dim3(256), 0, s, d_x, n, d_y);
  GIS_LAUNCH_CHECK("k_exp");
  return GIS_OK;
}

int32_t launch_calibrate(const BuildArgs& a, unsigned long long* d_maxerr, int64_t stride,
                         hipStream_t s) {
  if (a.kind == GIS_SYS_USER) return user_launch_calibrate(a, d_maxerr, stride, s);
  return dispatch_sys<Calibrate>(a.kind, a.n, a, d_maxerr, stride, s);
}

namespace {
// Recheck band of each (job, dimension) not given by the caller: eight times
// the calibrated FP32 error, at least floor_rel of the finest cell width of
// the job's current covering.
__global__ void k_band(Job* jobs, int32_t n_jobs, int32_t n, const unsigned long long* maxerr,
                       double floor_rel) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_jobs * n) return;
  const int j = t / n, d = t - j * n;
  if (jobs[j].band[d] > 0.0) return;
  const double e = __longlong_as_double((long long)maxerr[j * kMaxDim + d]);
  const double fl = floor_rel * ldexp(jobs[j].grid.w0[d], -jobs[j].ci.lmax);
  jobs[j].band[d] = 8.0 * e > fl ? 8.0 * e : fl;
}
}  // namespace

int32_t launch_band(Job* d_jobs, int32_t n_jobs, int32_t n, const unsigned long long* d_maxerr,
                    double floor_rel, hipStream_t s) {
  const int t = n_jobs * n;
  if (t <= 0) return GIS_OK;
  hipLaunchKernelGGL(k_band, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, d_jobs, n_jobs, n,
                     d_maxerr, floor_rel);
  GIS_LAUNCH_CHECK("k_band");
  return GIS_OK;
}

}  // namespace gis
