// One-sided Jacobi SVD of small matrices on one workgroup (see jacobi.hip).
#pragma once
#include "common.hpp"

namespace mpsv {

constexpr size_t kJacobiMaxLds = 150 * 1024;
constexpr int kJacobiMaxCols = 128;

// LDS bytes of the column pass (and of V when keep_v).
size_t jacobi_lds_bytes(int mb, int c, bool keep_v);

// B: mb x c row-major (ldb), read only.  Outputs (device): Vt (D x c),
// USs (mb x D, leading dimension D), sigbuf (>= 2c doubles: sorted values
// first), perm (c ints), info (5 doubles: D, discarded, sweeps, converged,
// rounds).  When keep_v is false, rotlog (>= 2 * max_sweeps * (c+1) *
// (c/2+1) doubles) and rflag (>= max_sweeps * (c+1) ints, zeroed) hold the
// rotation log replayed by the second pass.
void jacobi_svd(hipStream_t s, const double* B, int mb, int c, long ldb,
                int cap, double tol, int max_sweeps, double* rotlog, int* rflag,
                double* Vt, double* USs, double* sigbuf, int* perm,
                double* info, bool keep_v);

}  // namespace mpsv
