// Shared definitions of libpepsenv (host and device).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

namespace pe {

// Status codes mirror peps_status of include/peps_env.h.
enum : int {
  ST_OK = 0, ST_INVALID = -1, ST_OOM = -2, ST_HIP = -3, ST_NOT_CONVERGED = -4, ST_NONFINITE = -5, ST_UNSUPPORTED = -6
};

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define PE_HIP(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      throw ::pe::Error(::pe::ST_HIP, std::string(#x) + ": " + hipGetErrorString(e_));  \
  } while (0)
#define PE_REQUIRE(cond, msg)                                  \
  do {                                                         \
    if (!(cond)) throw ::pe::Error(::pe::ST_INVALID, (msg));   \
  } while (0)

// Element types of device buffers.
enum DType : int { DT_F64 = 0, DT_F32 = 1 };
inline size_t dtype_size(int dt) { return dt == DT_F64 ? 8 : 4; }

}  // namespace pe
