// Internal declarations of libcptr (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "setup.h"

namespace cptr {

void set_last_error(const std::string &msg);

#define CPTR_HIP_TRY(expr)                                                          \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      throw ::cptr::Error{CPTR_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

}  // namespace cptr
