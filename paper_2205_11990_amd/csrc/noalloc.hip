// Device scratch of the allocation-free entry point (mpsb_svd_truncate_noalloc
// in include/mps_blocks.h): a file-scope device array, one copy per GPU,
// held until the process ends.  Host code never uses the array's name as an
// address: its device address is looked up once per device with
// hipGetSymbolAddress and kept.
#include <mutex>

#include "noalloc.hpp"

namespace mpsv {

namespace {

static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

}  // namespace

double* noalloc_scratch() {
  int dev = -1;
  MPSV_HIP(hipGetDevice(&dev));
  MPSV_CHECK(dev >= 0 && dev < kMaxDevices, kEinval, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    // the current device is `dev`: its own copy of the array
    void* p = nullptr;
    MPSV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    MPSV_CHECK(p != nullptr, kEdevice, "no device address for the scratch array");
    g_ptr[dev] = static_cast<double*>(p);
  }
  return g_ptr[dev];
}

}  // namespace mpsv
