// Shared host-side helpers: error reporting across the C ABI and HIP checks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>
#include <string>

#include "litho.h"

namespace litho {

// Records the reason of the last failure on this thread (read by litho_last_error).
void set_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();
const char *last_error();

}  // namespace litho

#define LITHO_HIP_TRY(expr)                                                      \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      litho::set_error("%s failed: %s", #expr, hipGetErrorString(e_));          \
      return LITHO_E_HIP;                                                        \
    }                                                                            \
  } while (0)

#define LITHO_TRY(expr)          \
  do {                           \
    int rc_ = (expr);            \
    if (rc_ != LITHO_OK) return rc_; \
  } while (0)
