// Small data-movement kernels of the MPS engine (host wrappers).
#pragma once
#include "common.hpp"

namespace mpsv {

// out[j][i][k] = in[i][j][k] for i < d0, j < d1, k < inner  (swap two outer dims)
void swap01(hipStream_t s, const double* in, int d0, int d1, long inner,
            double* out);

// dst (rows x cols, ldd) = alpha * src (rows x cols, lds)
void copy2d(hipStream_t s, int rows, int cols, double alpha, const double* src,
            long lds, double* dst, long ldd);

// out[a][b] = in[a][0][b] + in[a][1][b]  for an l x 2 x r core
void sum_physical(hipStream_t s, const double* in, int l, int r, double* out);

// out (rows x len) = diag(g(d)) in, g(x) = x or, with `inverse`, 1/x and 0
// for x <= d[0] * 1e-200 (d: device, sorted descending; in may equal out)
void scale_rows(hipStream_t s, const double* in, int rows, long len,
                const double* d, bool inverse, double* out);

// A (n x n, row-major) = the identity
void identity(hipStream_t s, double* A, int n);

// out[b][t][a] = in[a][t][b]: an l x 2 x r core read from the right
void reverse_core(hipStream_t s, const double* in, int l, int r, double* out);

// Chain-order vector of a sequential ordering (x bits, then v bits; a
// dimension with rx / rv set has its least significant bit first) ->
// F[i*Nv + j].
void chain_to_grid(hipStream_t s, const double* in, int Lx, int Lv, bool rx,
                   bool rv, double* out);

// Embed an operator/core of one dimension into the interleaved chain:
// A has shape (l, P, r) with P = 2 (MPS core) or 4 (MPO core, (o,i) pairs).
// mode 0 (A-major): out[(a, c), P, (b, c)]  -- fused index a*d + c
// mode 1 (A-minor): out[(c, a), P, (c, b)]  -- fused index c*l + a
void kron_embed(hipStream_t s, const double* A, int l, int P, int r, int d,
                int mode, double* out);

// Diagonal MPO from an MPS core (SI, Dot Product):
// W[a][o][i][b] = scale * E[a][i][b] * delta(o, i)
void diag_mpo_site(hipStream_t s, const double* E, int l, int r, double scale,
                   double* W);

// Wmat[(o*wr + b')][(b*2 + i)] = W[b][o][i][b']   ((2wr) x (2wl))
void mpo_left_matrix(hipStream_t s, const double* W, int wl, int wr,
                     double* Wmat);

// Interleaved chain vector (x1 v1 x2 v2 ... MSB first) -> F[i*Nv + j].
void deinterleave(hipStream_t s, const double* in, int L, double* out);

// flag[0] += number of non-finite entries among n values (flag is int)
void count_nonfinite(hipStream_t s, const double* x, long n, int* flag);

// out[0] = sum x_i^2 * scale
void sum_squares(hipStream_t s, const double* x, long n, double scale,
                 double* out);

// Pair an MPS core A (l x 2 x r) with a weight core W (c x 2 x d) site by
// site: out[(a,c)][t][(b,e)] = A[a][t][b] W[c][t][e] (sum_bit false), or
// out[(a,c)][(b,e)] = sum_t A[a][t][b] W[c][t][e] (sum_bit true); fused
// bonds a-major.
void pair_cores(hipStream_t s, const double* A, int l, int r, const double* W,
                int c, int d, bool sum_bit, double* out);

// Local drift and temperature from the moments n = <1,f>, P = <v,f>,
// H = <v^2/2, f> on nx points: v0 = P / n, T = 2 H / n - v0^2 (both 0 where
// n = 0).
void dougherty_fields(hipStream_t s, const double* n, const double* P,
                      const double* H, long nx, double* v0, double* T);

void fill(hipStream_t s, double* x, long n, double v);
// dst[0:n] = src[0:n] (device buffers of the current lanes' instances)
void copy_doubles(hipStream_t s, double* dst, const double* src, long n);
void fill_int(hipStream_t s, int* x, long n, int v);

}  // namespace mpsv
