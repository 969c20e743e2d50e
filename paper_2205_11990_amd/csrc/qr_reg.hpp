// Householder QR with the matrix held in the registers of one workgroup
// (see qr_reg.hip).
#pragma once
#include "common.hpp"

namespace mpsv {

// Largest shapes the one-workgroup factorisation holds on chip.
bool qr_reg_fits(int m, int n);
// Widest panel qr_reg_factor takes for m rows (m <= 2048).
int qr_reg_panel_cols(int m);

// Householder QR of A (m x n, row-major, leading dimension lda, read only
// unless R aliases it).  Writes R (min(m,n) x n, zeros below the diagonal,
// leading dimension ldr), the reflectors V (column-major m x k, V[j*m + i],
// unit diagonal, zeros above) and tau (k); A = H_0 ... H_{k-1} [R; 0] with
// H_j = I - tau_j v_j v_j^T (LAPACK sign conventions).
void qr_reg_factor(hipStream_t s, const double* A, long lda, int m, int n,
                   double* R, long ldr, double* V, double* tau);

// Y (m x p, row-major, leading dimension ldy) <- Q Y (trans = false) or
// Q^T Y (trans = true), Q = H_0 ... H_{k-1} from qr_reg_factor (V has m
// rows).  Columns are spread over as many workgroups as needed; m <= 2048.
void qr_reg_apply(hipStream_t s, const double* V, const double* tau, int m,
                  int k, double* Y, long ldy, int p, bool trans);

}  // namespace mpsv
