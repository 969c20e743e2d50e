// Optional per-kernel-class timing with HIP events on the launching stream.
// Off by default; when on, every launch of an instrumented kernel is
// bracketed by two events and its nominal FLOP/byte count is recorded.
#pragma once
#include "common.hpp"

namespace mpsv {

enum KClass : int {
  kClsGemm = 0,
  kClsQrPanel = 1,
  kClsJacobi = 2,
  kClsOther = 3,
  kClsQrApply = 4,
  kClsQrWy = 5,  // compact-WY reflector application (HBM-bound streams of Y)
  kClsCount = 6
};

bool prof_enabled();
void prof_enable(bool on);  // enabling clears previous records
// Returns an opaque slot (or -1 when disabled); call prof_end with it.  The
// counts given to prof_end are per instance; a launch over several
// lock-step instances (Lanes) records them times the instance count.
int prof_begin(hipStream_t s);
void prof_end(hipStream_t s, int slot, int cls, double flops, double bytes);
// Synchronises the device and sums the records of class `cls`.
void prof_read(int cls, long* launches, double* ms, double* flops,
               double* bytes);
// The FLOPs of class `cls` recorded inside a truncated SVD (its
// preconditioning QRs, reflector applications and GEMM): the SVD's own record
// already counts the nominal work of the whole decomposition, so a sum over
// classes subtracts these.
double prof_nested_flops(int cls);

// Marks the calling thread's launches as nested in a truncated SVD for its
// lifetime (the SVD's own record is taken outside it).
class ProfNested {
 public:
  ProfNested();
  ~ProfNested();
  ProfNested(const ProfNested&) = delete;
  ProfNested& operator=(const ProfNested&) = delete;
};

}  // namespace mpsv
