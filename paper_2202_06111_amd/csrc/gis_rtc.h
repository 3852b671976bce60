// Runtime-compiled user fields (rtc.hip): one hipRTC program per field with
// the graph-construction kernels instantiated for kind GIS_SYS_USER.
#pragma once

#include <string>

#include "gis_internal.h"

namespace gis {

struct UserField {
  int32_t n = 0, m = 0;
  int device = -1;
  std::string body;
  hipModule_t module = nullptr;
  hipFunction_t build[4] = {};   // [2 * FP32 images + uniform covering]
  hipFunction_t images[2] = {};  // float, double
  hipFunction_t calibrate = nullptr;
  void unload();
  ~UserField() { unload(); }
};

// Compiles `body` (the field's code, see gis_set_user_field) with the build
// kernels for `device`'s architecture and loads the module there; device < 0
// compiles for gfx950 only, to check the body (*out is then NULL).
int32_t user_field_compile(const char* body, int32_t n, int32_t m, int device, UserField** out);

// The launchers of k_build.hip for kind GIS_SYS_USER (a.user is the field).
int32_t user_launch_build(const BuildArgs& a, int32_t precision, hipStream_t s);
int32_t user_launch_images(const BuildArgs& a, int32_t precision, double* d_images, hipStream_t s);
int32_t user_launch_calibrate(const BuildArgs& a, unsigned long long* d_maxerr, int64_t stride,
                              hipStream_t s);

}  // namespace gis
