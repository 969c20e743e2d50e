// One-sided Jacobi SVD of small matrices on one workgroup (see jacobi.hip).
#pragma once
#include "common.hpp"

namespace mpsv {

constexpr size_t kJacobiMaxLds = 150 * 1024;
constexpr int kJacobiOneWgCols = 128;  // one workgroup up to here
constexpr int kJacobiMaxCols = 256;    // four workgroups up to here

// How a k x k factor is decomposed: 0 on one workgroup, else log2 of the
// number of workgroups sharing it.
int jacobi_split(int k);

// LDS bytes of the kernel for a k x k factor.
size_t jacobi_lds_bytes(int k);

// Device workspace (doubles) the kernel needs beyond its outputs: zero up
// to kJacobiOneWgCols columns, the exchange area of the workgroups
// above.
size_t jacobi_ws_doubles(int k);

// One-sided Jacobi on the columns of Xr^T, where Xr (k x k, row-major,
// leading dimension ldx, k <= 256, read only) is a triangular factor R of
// the matrix X being decomposed (X = Q R).  The columns converge to the
// right singular vectors of X times its singular values.  Outputs (device):
// Vt (D x k, the kept right singular vectors as rows), sigbuf (>= 2k
// doubles: sorted values first), perm (k ints), info (6 doubles: D,
// discarded weight, sweeps, converged, steps, 1 if the workgroups
// failed to meet).  ws: jacobi_ws_doubles(k) doubles of device workspace.
void jacobi_svd(hipStream_t s, const double* Xr, int k, long ldx, int cap,
                double tol, int max_sweeps, double* Vt, double* sigbuf,
                int* perm, double* info, double* ws);

}  // namespace mpsv
