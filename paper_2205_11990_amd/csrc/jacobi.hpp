// One-sided Jacobi SVD of small matrices on one workgroup (see jacobi.hip).
#pragma once
#include "common.hpp"

namespace mpsv {

constexpr size_t kJacobiMaxLds = 150 * 1024;
constexpr int kJacobiMaxCols = 128;

// LDS bytes of the kernel for a k x k factor.
size_t jacobi_lds_bytes(int k);

// One-sided Jacobi on the columns of Xr^T, where Xr (k x k, row-major,
// leading dimension ldx, k <= 128, read only) is a triangular factor R of
// the matrix X being decomposed (X = Q R).  The columns converge to the
// right singular vectors of X times its singular values.  Outputs (device):
// Vt (D x k, the kept right singular vectors as rows), sigbuf (>= 2k
// doubles: sorted values first), perm (k ints), info (5 doubles: D,
// discarded weight, sweeps, converged, rounds).
void jacobi_svd(hipStream_t s, const double* Xr, int k, long ldx, int cap,
                double tol, int max_sweeps, double* Vt, double* sigbuf,
                int* perm, double* info);

}  // namespace mpsv
