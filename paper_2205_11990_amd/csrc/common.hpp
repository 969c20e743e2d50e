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

// ---- lock-step instances
//
// A batch of instances of one problem shape keeps every device buffer of
// instance i exactly i * stride bytes after instance 0's copy: each chunk of
// its arenas is allocated once for all instances, `stride` bytes per
// instance.  The engine issues each step's launches once, for instance 0's
// addresses, and every launch covers the instances of the current Lanes:
// instance z of the launch is instance `first + z`, and a kernel shifts each
// of its pointer arguments by InstOff::of(blockIdx.z) bytes (the GEMM folds
// the instance into its batch index).  Outside a batch there is one
// instance and no shift.
struct Lanes {
  int n = 1;         // instances covered by a launch
  long first = 0;    // bytes: offset of the launch's instance 0
  long stride = 0;   // bytes between consecutive instances
  // the problem's choice of kernel for reflector applications on tall
  // blocks (mps_problem.tall_apply): it goes with the lanes so that every
  // thread issuing one engine's launches makes the same choice
  int tall_apply = 0;
};
// The calling thread's current lanes (one instance, no shift by default).
Lanes& lanes();
// Sets the calling thread's lanes for its lifetime, restoring them after.
class LanesScope {
 public:
  explicit LanesScope(const Lanes& l) : saved_(lanes()) { lanes() = l; }
  ~LanesScope() { lanes() = saved_; }
  LanesScope(const LanesScope&) = delete;
  LanesScope& operator=(const LanesScope&) = delete;

 private:
  Lanes saved_;
};

// Kernel-side view of the lanes of one launch.
struct InstOff {
  long first, stride;
  __host__ __device__ long of(long z) const { return first + z * stride; }
};
inline InstOff inst_off() { return InstOff{lanes().first, lanes().stride}; }
inline int inst_count() { return lanes().n; }

// Page-locked host buffer that only grows (released with its owner): the
// read-backs of all lock-step instances land in it as one transfer.
class PinnedBuf {
 public:
  PinnedBuf() = default;
  ~PinnedBuf() {
    if (p_) (void)hipHostFree(p_);
  }
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  void* get(size_t bytes) {
    if (bytes > cap_) {
      if (p_) (void)hipHostFree(p_);
      p_ = nullptr;
      cap_ = 0;
      MPSV_HIP(hipHostMalloc(&p_, bytes, hipHostMallocDefault));
      cap_ = bytes;
    }
    return p_;
  }

 private:
  void* p_ = nullptr;
  size_t cap_ = 0;
};

// `bytes` bytes at d of every instance of the calling thread's lanes into
// h (instance i's at h + i * bytes) on stream s: one strided transfer.
void lanes_d2h(hipStream_t s, void* h, const void* d, size_t bytes);

template <class T>
__host__ __device__ inline T* shifted(T* p, long off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(p) + off);
}
template <class T>
__host__ __device__ inline const T* shifted(const T* p, long off) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + off);
}
__host__ __device__ inline MatView shifted(MatView v, long off) {
  v.p = shifted(v.p, off);
  return v;
}
__host__ __device__ inline CMatView shifted(CMatView v, long off) {
  v.p = shifted(v.p, off);
  return v;
}

}  // namespace mpsv
