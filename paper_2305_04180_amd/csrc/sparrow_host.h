// sparrow_host.h -- host-side helpers shared by the library's translation
// units: the thread-local last-error message behind sparrow_last_error() and
// the HIP_TRY early return.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/sparrow.h"

namespace sp {

// Record msg as the calling thread's last error and return code.
int fail(int code, const std::string& msg);

}  // namespace sp

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return ::sp::fail(SPARROW_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)
