// Runtime-compiled vector fields (kind GIS_SYS_USER): the caller's code for
// g(x, u) of x' = g(x, u) -- the f of Eq. (1) is the problem's input -- is
// compiled with hipRTC together with the library's own graph-construction
// kernels (k_build_dev.h, embedded here at build time), so a user field runs
// exactly the kernels of the built-in ones: the same RK4 operation order, the
// same sample points, cover logic, FP32 recheck and CSR emit.
//
// One program per (body, n, m, device architecture): k_build in its four
// variants (FP32 or FP64 images, uniform or refined covering), the parity
// kernel k_images (both precisions) and the band calibration k_calibrate.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <memory>
#include <string>
#include <vector>

#include "gis_internal.h"
#include "gis_rtc.h"

namespace gis {

namespace {

#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wc23-extensions"
const char kSrcGis[] = {
#embed "../../include/gis.h"
    , 0};
const char kSrcInternal[] = {
#embed "gis_internal.h"
    , 0};
const char kSrcDynamics[] = {
#embed "dynamics.h"
    , 0};
const char kSrcBuild[] = {
#embed "k_build_dev.h"
    , 0};
#pragma clang diagnostic pop

// hipRTC's runtime header declares the fixed-width integer types inside its
// own namespace; the library's headers use them unqualified.
const char kPrelude[] = R"(
typedef __hip_internal::int8_t int8_t;
typedef __hip_internal::uint8_t uint8_t;
typedef __hip_internal::int16_t int16_t;
typedef __hip_internal::uint16_t uint16_t;
typedef __hip_internal::int32_t int32_t;
typedef __hip_internal::uint32_t uint32_t;
typedef __hip_internal::int64_t int64_t;
typedef __hip_internal::uint64_t uint64_t;
#include "k_build_dev.h"
namespace gis {
template <typename R>
__device__ void user_field(const R* p, const R* x, const R* u, R* dx) {
#line 1 "user field"
)";
const char kEpilogue[] = "\n}\n}  // namespace gis\n";

std::string kernel_name(const char* kernel, int n, const char* rest) {
  return std::string("gis::kbuild::") + kernel + "<" + std::to_string(GIS_SYS_USER) + ", " +
         std::to_string(n) + rest + ">";
}

const char* const kBuildVariants[4] = {", false, false", ", false, true", ", true, false",
                                       ", true, true"};

int32_t rtc_fail(hiprtcResult r, const char* what) {
  set_error(std::string(what) + ": " + hiprtcGetErrorString(r));
  return GIS_E_HIP;
}

}  // namespace

void UserField::unload() {
  if (module) {
    int prev = 0;
    const bool have = hipGetDevice(&prev) == hipSuccess;
    if (hipSetDevice(device) == hipSuccess) (void)hipModuleUnload(module);
    if (have) (void)hipSetDevice(prev);
    module = nullptr;
  }
}

int32_t user_field_compile(const char* body, int32_t n, int32_t m, int device, UserField** out) {
  if (!body) {
    set_error("user field body is NULL");
    return GIS_E_INVAL;
  }
  if (n < 1 || n > kMaxDim || m < 1 || m > 2) {
    set_error("user field: n must be 1..4 and m 1..2");
    return GIS_E_INVAL;
  }
  // the device's architecture, or gfx950 for a compile-only check
  std::string arch = "gfx950";
  if (device >= 0) {
    hipDeviceProp_t prop;
    GIS_HIP(hipGetDeviceProperties(&prop, device));
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
  }
  const std::string src = std::string(kPrelude) + body + kEpilogue;
  const char* headers[4] = {kSrcGis, kSrcInternal, kSrcDynamics, kSrcBuild};
  const char* names[4] = {"gis.h", "gis_internal.h", "dynamics.h", "k_build_dev.h"};
  hiprtcProgram prog;
  hiprtcResult r = hiprtcCreateProgram(&prog, src.c_str(), "gis_user_field.hip", 4, headers, names);
  if (r != HIPRTC_SUCCESS) return rtc_fail(r, "hiprtcCreateProgram");
  std::unique_ptr<hiprtcProgram, void (*)(hiprtcProgram*)> guard(
      &prog, [](hiprtcProgram* p) { (void)hiprtcDestroyProgram(p); });
  std::vector<std::string> exprs;
  for (int v = 0; v < 4; ++v) exprs.push_back(kernel_name("k_build", n, kBuildVariants[v]));
  exprs.push_back(kernel_name("k_images", n, ", float"));
  exprs.push_back(kernel_name("k_images", n, ", double"));
  exprs.push_back(kernel_name("k_calibrate", n, ""));
  for (const std::string& e : exprs)
    if ((r = hiprtcAddNameExpression(prog, e.c_str())) != HIPRTC_SUCCESS)
      return rtc_fail(r, "hiprtcAddNameExpression");
  // the static library's flags: IEEE operations only where written (no
  // contraction), no packed FP32 instructions
  const std::string arch_opt = "--offload-arch=" + arch;
  const char* opts[] = {arch_opt.c_str(), "-O3", "-std=c++17", "-ffp-contract=off",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
  if (r != HIPRTC_SUCCESS) {
    size_t ls = 0;
    std::string log;
    if (hiprtcGetProgramLogSize(prog, &ls) == HIPRTC_SUCCESS && ls > 1) {
      log.resize(ls);
      (void)hiprtcGetProgramLog(prog, &log[0]);
      log.resize(ls - 1);
    }
    set_error("user field does not compile:\n" + log);
    return GIS_E_INVAL;
  }
  auto uf = std::make_unique<UserField>();
  uf->n = n;
  uf->m = m;
  uf->device = device;
  uf->body = body;
  std::vector<std::string> lowered(exprs.size());
  for (size_t i = 0; i < exprs.size(); ++i) {
    const char* ln = nullptr;
    if ((r = hiprtcGetLoweredName(prog, exprs[i].c_str(), &ln)) != HIPRTC_SUCCESS)
      return rtc_fail(r, "hiprtcGetLoweredName");
    lowered[i] = ln;
  }
  if (out) *out = nullptr;
  if (device < 0) return GIS_OK;  // compile-only check
  size_t code_bytes = 0;
  if ((r = hiprtcGetCodeSize(prog, &code_bytes)) != HIPRTC_SUCCESS)
    return rtc_fail(r, "hiprtcGetCodeSize");
  std::vector<char> code(code_bytes);
  if ((r = hiprtcGetCode(prog, code.data())) != HIPRTC_SUCCESS) return rtc_fail(r, "hiprtcGetCode");
  GIS_HIP(hipModuleLoadData(&uf->module, code.data()));
  for (int v = 0; v < 4; ++v) GIS_HIP(hipModuleGetFunction(&uf->build[v], uf->module, lowered[v].c_str()));
  GIS_HIP(hipModuleGetFunction(&uf->images[0], uf->module, lowered[4].c_str()));
  GIS_HIP(hipModuleGetFunction(&uf->images[1], uf->module, lowered[5].c_str()));
  GIS_HIP(hipModuleGetFunction(&uf->calibrate, uf->module, lowered[6].c_str()));
  if (!out) return GIS_OK;
  *out = uf.release();
  return GIS_OK;
}

namespace {

int32_t check_user(const BuildArgs& a, const UserField*& uf) {
  uf = static_cast<const UserField*>(a.user);
  if (!uf) {
    set_error("system kind GIS_SYS_USER, but no user field is set in this context");
    return GIS_E_INVAL;
  }
  if (uf->n != a.n || uf->m != a.m) {
    set_error("the user field was compiled for n = " + std::to_string(uf->n) + ", m = " +
              std::to_string(uf->m) + "; the system has n = " + std::to_string(a.n) +
              ", m = " + std::to_string(a.m));
    return GIS_E_INVAL;
  }
  return GIS_OK;
}

}  // namespace

int32_t user_launch_build(const BuildArgs& a, int32_t precision, hipStream_t s) {
  const UserField* uf;
  int32_t rc;
  if ((rc = check_user(a, uf))) return rc;
  if (a.n_blocks == 0) return GIS_OK;
  const int v = (precision == GIS_PREC_FP32_RECHECK ? 2 : 0) + (a.all_uniform ? 1 : 0);
  BuildArgs arg = a;
  void* params[] = {&arg};
  GIS_HIP(hipModuleLaunchKernel(uf->build[v], (unsigned)a.n_blocks, 1, 1, kRowBlock, 1, 1, 0, s,
                                params, nullptr));
  return GIS_OK;
}

int32_t user_launch_images(const BuildArgs& a, int32_t precision, double* d_images, hipStream_t s) {
  const UserField* uf;
  int32_t rc;
  if ((rc = check_user(a, uf))) return rc;
  if (a.n_blocks == 0) return GIS_OK;
  BuildArgs arg = a;
  double* outp = d_images;
  void* params[] = {&arg, &outp};
  GIS_HIP(hipModuleLaunchKernel(uf->images[precision == GIS_PREC_FP32_RECHECK ? 0 : 1],
                                (unsigned)a.n_blocks, 1, 1, kRowBlock, 1, 1, 0, s, params, nullptr));
  return GIS_OK;
}

int32_t user_launch_calibrate(const BuildArgs& a, unsigned long long* d_maxerr, int64_t stride,
                              hipStream_t s) {
  const UserField* uf;
  int32_t rc;
  if ((rc = check_user(a, uf))) return rc;
  if (a.n_blocks == 0) return GIS_OK;
  BuildArgs arg = a;
  unsigned long long* me = d_maxerr;
  int64_t st = stride < 1 ? 1 : stride;
  void* params[] = {&arg, &me, &st};
  GIS_HIP(hipModuleLaunchKernel(uf->calibrate, (unsigned)a.n_blocks, 1, 1, kRowBlock, 1, 1, 0, s,
                                params, nullptr));
  return GIS_OK;
}

}  // namespace gis
