// Householder QR with the matrix held in the registers of one workgroup
// (see qr_reg.hip).
#pragma once
#include "common.hpp"

namespace mpsv {

// Largest shapes the one-workgroup factorisation holds on chip.
bool qr_reg_fits(int m, int n);
// Widest panel qr_reg_factor takes for m rows (m <= 2048).
int qr_reg_panel_cols(int m);

// Householder QR of A (m x n, element (i, j) at A.p[i*A.rs + j*A.cs], read
// only unless R aliases it with the same strides).  Writes R (min(m,n) x n,
// zeros below the diagonal, element (i, j) at R.p[i*R.rs + j*R.cs]), the
// reflectors V (column-major m x k, V[j*m + i], unit diagonal, zeros above)
// and tau (k); A = H_0 ... H_{k-1} [R; 0] with H_j = I - tau_j v_j v_j^T
// (LAPACK sign conventions).  Strided views let callers factor a transpose
// or write R^T without a copy.
void qr_reg_factor(hipStream_t s, CMatView A, int m, int n, MatView R,
                   double* V, double* tau);

// Yout <- Q Yin (trans = false) or Q^T Yin (trans = true), Q = H_0 ... H_{k-1}
// from qr_reg_factor (V has m rows); both blocks m x p with element (i, j)
// at p[i*rs + j*cs]; rows >= rows_in of Yin are taken as zero (not read).
// Yout may alias Yin with the same strides.  Columns are spread over as
// many workgroups as needed; m <= 2048.
void qr_reg_apply(hipStream_t s, const double* V, const double* tau, int m,
                  int k, CMatView Yin, int rows_in, MatView Yout, int p,
                  bool trans);

// Groups of up to four 16-column panels (at most 64 reflectors over m
// rows) applied as one compact-WY block Q_g = H_0 ... H_{k-1} = I - V T V^T
// (the compact-WY mode's factorisation of blocks over 512 rows).  The
// group's reflectors are stored panel after panel: panel t (reflectors
// 16 t .. 16 t + 15) column-major over its own m - 16 t rows (it starts at
// row 16 t of the group; unit diagonal, zeros above), at offset
// qr_group_voff(m, t); tau holds the k scalars in order.
long qr_group_voff(int m, int t);
// T of the group: 64 x 64 row-major, upper triangular, zero past k.
void qr_wy_group_t(hipStream_t s, const double* V, const double* tau, int m, int k,
                   double* T);
// Yout <- Q_g Yin (trans = false) or Q_g^T Yin (m x p blocks, any strides;
// rows >= rows_in of Yin taken as zero).  Yout may alias Yin with the same
// strides.
void qr_wy_group_apply(hipStream_t s, const double* V, const double* T, int m, int k,
                       CMatView Yin, int rows_in, MatView Yout, int p, bool trans);

// Row-chunked factorisation of a tall panel (the first step of a TSQR): A
// (m x n) is cut into chunks of `rows` rows (the last one may be shorter;
// rows >= n, rows <= 2048, n <= qr_reg_panel_cols(rows)), each factored on
// its own workgroup of one launch.  Chunk c writes its R (min(rows_c, n) x
// n) at rows [c n, c n + min(rows_c, n)) of S, its reflectors (rows_c long,
// V[j*rows_c + i]) at V + c*rows*n and tau at tau + c*n.
void qr_reg_factor_chunks(hipStream_t s, CMatView A, int m, int n, int rows,
                          MatView S, double* V, double* tau);

// Y <- Q_c Y or Q_c^T Y on every chunk c of rows of Y (m x p, in place), with
// the reflectors of qr_reg_factor_chunks (k per chunk, same rows).
void qr_reg_apply_chunks(hipStream_t s, const double* V, const double* tau,
                         int m, int k, int rows, MatView Y, int p, bool trans);

}  // namespace mpsv
