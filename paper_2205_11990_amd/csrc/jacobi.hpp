// One-sided Jacobi SVD of small matrices on one workgroup (see jacobi.hip).
#pragma once
#include "common.hpp"

namespace mpsv {

constexpr size_t kJacobiMaxLds = 150 * 1024;
constexpr int kJacobiMaxCols = 128;

// LDS bytes of the column pass (and of the rotations when keep_v).
size_t jacobi_lds_bytes(int k, int c, bool keep_v);

// One-sided Jacobi on the columns of Xr^T, where Xr (k x k, row-major,
// leading dimension ldx, k <= 128, read only) is the triangular factor of
// X (mode 0) or of X^T (mode 1).  Outputs (device, leading dimension D for
// the k x D arrays):
//   mode 0: out1 = Vt (D x k) right singular vectors of Xr,
//           out2 = (k x D) left singular vectors times sigma;
//   mode 1: out1 = (k x D) right singular vectors of Xr times sigma,
//           out2 = (k x D) left singular vectors of Xr.
// sigbuf (>= 2k doubles: sorted values first), perm (k ints), info (5
// doubles: D, discarded, sweeps, converged, rounds).  When keep_v is false,
// rotlog (>= max_sweeps * (k+1) * (k+2) doubles) and rflag
// (>= max_sweeps * (k+1) ints) hold the rotation log replayed by the
// second pass.
void jacobi_svd(hipStream_t s, const double* Xr, int k, int c, long ldx,
                int mode, int cap, double tol, int max_sweeps, double* rotlog,
                int* rflag, double* out1, double* out2, double* sigbuf,
                int* perm, double* info, bool keep_v);

}  // namespace mpsv
