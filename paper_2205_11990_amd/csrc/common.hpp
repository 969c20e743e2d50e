// Shared host/device helpers for the MPS Vlasov-Poisson library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

namespace mpsv {

// Error carried from deep inside the engine up to the C-ABI, which turns it
// into a status code and a thread-local message.  Never crosses the ABI.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

enum : int { kOk = 0, kEinval = -1, kEnomem = -2, kEnumeric = -3, kEdevice = -4 };

#define MPSV_HIP(call)                                                         \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      throw ::mpsv::Error(::mpsv::kEdevice,                                    \
                          std::string(#call) + ": " + hipGetErrorString(e_));  \
  } while (0)

#define MPSV_CHECK(cond, code, msg)                                            \
  do {                                                                         \
    if (!(cond)) throw ::mpsv::Error((code), (msg));                           \
  } while (0)

// Launch-time check of a kernel launch (configuration errors).
#define MPSV_LAUNCHED() MPSV_HIP(hipGetLastError())

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// A strided view of a (batched) matrix: element (b, i, j) lives at
// p[b*bs + i*rs + j*cs].  All strides are in elements.
struct MatView {
  double* p;
  long rs, cs, bs;
};
struct CMatView {
  const double* p;
  long rs, cs, bs;
};

inline MatView row_major(double* p, long ld) { return MatView{p, ld, 1, 0}; }
inline CMatView crow_major(const double* p, long ld) { return CMatView{p, ld, 1, 0}; }

}  // namespace mpsv
