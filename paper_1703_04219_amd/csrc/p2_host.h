// Host-side internals shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "p2_kernels.h"

namespace p2host {

// Text of the last failure on this thread (parafac2_last_error).
std::string& last_error();

// Record a failure message and return code.
int fail(int code, const char* fmt, ...);

}  // namespace p2host

#define P2_HIP_TRY(expr)                                                                   \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return p2host::fail(P2_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));             \
  } while (0)

// Fixed (V, H) of a projection model, in the model's workspace.
struct parafac2_model {
  int64_t J = 0;
  int R = 0, LDV = 0;
  hipStream_t stream = nullptr;
  unsigned char* ws = nullptr;
  size_t oV = 0, oH = 0, oN3 = 0, oN3p = 0, oVtV = 0, oHtH = 0, oMap = 0, total = 0;
  p2::PolarParams pp{};

  const float* V() const { return reinterpret_cast<const float*>(ws + oV); }
  const double* H() const { return reinterpret_cast<const double*>(ws + oH); }
  const double* N3() const { return reinterpret_cast<const double*>(ws + oN3); }
  const double* N3p() const { return reinterpret_cast<const double*>(ws + oN3p); }
};
