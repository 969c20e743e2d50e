// One-sided (Hestenes) Jacobi SVD of a small matrix on one workgroup of
// 1024 threads.  The matrix handed in is X (m x c, m <= c) or the triangular
// factor R (c x c) of a tall X; the rotations act on the columns of its
// transpose B = X^T (or R^T), whose k = min(m, c) columns converge to
// v_i sigma_i while the accumulated rotations converge to U.  Working on the
// transpose of the triangular factor needs far fewer sweeps than working on
// the factor itself (about 9 against 22 on the matrices of the compression
// sweep).
//
// Columns are orthogonalised pairwise in the cyclic round-robin ordering:
// each round pairs all c columns into disjoint pairs; a group of G lanes
// (G a power of two <= 64) owns one pair, accumulates the three inner
// products over its rows, reduces them with cross-lane shuffles, and
// applies the rotation.  The columns live in LDS with an odd leading
// dimension so that the groups of one wave hit distinct banks.
//
// When the accumulated rotations V (c x c) fit in LDS next to B they are
// updated in the same pass.  Otherwise (c > ~96) the rotation of every
// pair slot is logged to global memory and a second kernel replays the log
// on V held in LDS; this keeps both passes on-chip.
//
// On exit: singular values are the column norms, sorted descending (ties by
// index), the truncation rank D follows the rule min(cap, smallest D' whose
// relative discarded weight is <= tol) (eq. 5 with the i = D+1 reading),
// Vt (D x c) holds the kept right singular vectors (normalised columns) and
// USs (k x D) the columns u_i sigma_i (accumulated rotations times sigma).
#include <cmath>

#include "jacobi.hpp"

namespace mpsv {

namespace {

constexpr int JT = 1024;
constexpr int G = 16;    // lanes per column pair (one DPP row)
constexpr int RPT = 8;   // rows per lane: 16 * 8 = 128 rows

struct Pairing {
  int cc, np;
};

__device__ inline Pairing make_pairing(int c) {
  Pairing P;
  P.cc = c + (c & 1);
  P.np = P.cc / 2;
  return P;
}

__device__ inline void pair_of(int r, int k, int cc, int& p, int& q) {
  if (k == 0) {
    p = cc - 1;
    q = r;
  } else {
    p = (r + k) % (cc - 1);
    q = (r - k + cc - 1) % (cc - 1);
  }
}

template <int CTRL>
__device__ inline double dpp(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over an aligned group of 16 lanes (one DPP row); every lane gets it.
__device__ inline double sum16(double v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  return v;
}

// 1/x from the hardware estimate refined by two Newton steps.
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// Rutishauser's rotation that orthogonalises columns with Gram [[a,g],[g,b]].
__device__ inline void rotation(double a, double b, double g, double& cs,
                                double& sn) {
  const double z = (b - a) * rcp_nr(2.0 * g);
  const double az = fabs(z);
  double t;
  if (z == 0.0) t = 1.0;
  else if (az > 1e150) t = 0.5 * rcp_nr(z);
  else t = copysign(rcp_nr(az + sqrt(fma(z, z, 1.0))), z);
  cs = rcp_nr(sqrt(fma(t, t, 1.0)));
  sn = cs * t;
}

__device__ inline void rotate_cols(double* __restrict__ xp, double* __restrict__ yp,
                                   int n, int lig, double cs, double sn) {
  double x[RPT], y[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = lig + G * r;
    x[r] = (i < n) ? xp[i] : 0.0;
    y[r] = (i < n) ? yp[i] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = lig + G * r;
    if (i < n) {
      xp[i] = cs * x[r] - sn * y[r];
      yp[i] = sn * x[r] + cs * y[r];
    }
  }
}

__device__ inline double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < JT / 64; ++i) t += red[i];
  return t;
}

// info: [0] D, [1] discarded weight, [2] sweeps, [3] converged, [4] rounds
// Xr: k x c row-major triangular factor (c == k); the Jacobi columns are
// its rows: A[j][i] = Xr[j][i], j < k, i < c.  Outputs by mode:
//   mode 0 (factor of X):   out1 = Vt (D x c), rows A_d / sigma_d
//                           out2 = (k x D) J[:, d] sigma_d   (= U_R Sigma)
//   mode 1 (factor of X^T): out1 = (k x D) A_d               (= U Sigma)
//                           out2 = (k x D) J[:, d]           (V = Q' J)
__global__ __launch_bounds__(JT) void jacobi_cols_kernel(
    const double* __restrict__ Xr, int k, int c, long ldx, int keep_v, int mode,
    double* __restrict__ rotlog, int* __restrict__ rflag, int max_sweeps,
    int cap, double tol, double* __restrict__ Vt, double* __restrict__ USs,
    double* __restrict__ sigbuf, int* __restrict__ perm_out,
    double* __restrict__ info) {
  extern __shared__ double smem[];
  __shared__ double red[JT / 64];
  __shared__ int sweep_any;
  __shared__ int round_any[2];
  __shared__ int Dsh;
  const int tid = threadIdx.x;
  const int nrow = c, ncol = k;            // Jacobi matrix A = Xr^T: c x k
  const int lda = nrow | 1, ldv = ncol | 1;
  double* A = smem;                        // A[j*lda + i], j < k, i < c
  double* V = smem + (long)ncol * lda;     // accumulated rotations (keep_v)

  for (long e = tid; e < (long)ncol * nrow; e += JT) {
    const long j = e / nrow, i = e % nrow;
    A[j * lda + i] = Xr[j * ldx + i];
  }
  if (keep_v)
    for (long e = tid; e < (long)ncol * ncol; e += JT) {
      const long j = e / ncol, i = e % ncol;
      V[j * ldv + i] = (i == j) ? 1.0 : 0.0;
    }
  __syncthreads();
  double part = 0.0;
  for (long e = tid; e < (long)ncol * nrow; e += JT) {
    const long j = e / nrow, i = e % nrow;
    const double x = A[j * lda + i];
    part += x * x;
  }
  const double normF2 = block_sum(part, red);
  const double abs_floor = 1e-30 * normF2;
  const double eps = 1e-14;

  const Pairing P = make_pairing(ncol);
  const int kk = tid / G, lig = tid % G;   // pair slot of this lane group
  int sweep = 0, converged = 0, rounds = 0;
  if (tid == 0) round_any[0] = round_any[1] = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) sweep_any = 0;
    __syncthreads();
    for (int r = 0; r < P.cc - 1; ++r, ++rounds) {
      int p = 0, q = 0;
      if (kk < P.np) pair_of(r, kk, P.cc, p, q);
      if (kk < P.np && p < ncol && q < ncol) {
        double* ap = A + (long)p * lda;
        double* aq = A + (long)q * lda;
        double x[RPT], y[RPT];
#pragma unroll
        for (int rr = 0; rr < RPT; ++rr) {
          const int i = lig + G * rr;
          x[rr] = (i < nrow) ? ap[i] : 0.0;
          y[rr] = (i < nrow) ? aq[i] : 0.0;
        }
        double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
        for (int rr = 0; rr < RPT; ++rr) {
          a = fma(x[rr], x[rr], a);
          b = fma(y[rr], y[rr], b);
          g = fma(x[rr], y[rr], g);
        }
        a = sum16(a);
        b = sum16(b);
        g = sum16(g);
        double cs = 1.0, sn = 0.0;
        const bool rot = g != 0.0 && fabs(g) > eps * sqrt(a * b) && fabs(g) > abs_floor;
        if (rot) {
          rotation(a, b, g, cs, sn);
#pragma unroll
          for (int rr = 0; rr < RPT; ++rr) {
            const int i = lig + G * rr;
            if (i < nrow) {
              ap[i] = cs * x[rr] - sn * y[rr];
              aq[i] = sn * x[rr] + cs * y[rr];
            }
          }
          if (keep_v)
            rotate_cols(V + (long)p * ldv, V + (long)q * ldv, ncol, lig, cs, sn);
          if (lig == 0) {
            sweep_any = 1;
            round_any[rounds & 1] = 1;
          }
        }
        if (!keep_v && lig == 0) {
          rotlog[(2L * rounds) * P.np + 2 * kk] = cs;
          rotlog[(2L * rounds) * P.np + 2 * kk + 1] = sn;
        }
      }
      __syncthreads();
      if (tid == 0) {
        if (!keep_v) rflag[rounds] = round_any[rounds & 1];
        round_any[rounds & 1] = 0;
      }
    }
    __syncthreads();
    if (sweep_any == 0) {
      converged = 1;
      ++sweep;
      break;
    }
    __syncthreads();
  }

  // singular values = column norms (scratch half of sigbuf), rank-sorted
  for (int j = tid; j < ncol; j += JT) {
    double s2 = 0.0;
    const double* aj = A + (long)j * lda;
    for (int i = 0; i < nrow; ++i) s2 += aj[i] * aj[i];
    sigbuf[ncol + j] = sqrt(s2);
  }
  __syncthreads();
  for (int j = tid; j < ncol; j += JT) {
    const double sj = sigbuf[ncol + j];
    int rank = 0;
    for (int q = 0; q < ncol; ++q) {
      const double sq = sigbuf[ncol + q];
      rank += (sq > sj || (sq == sj && q < j)) ? 1 : 0;
    }
    perm_out[rank] = j;
    sigbuf[rank] = sj;
  }
  __syncthreads();
  const int kmax = ncol;
  if (tid == 0) {
    double tot = 0.0;
    for (int i = 0; i < ncol; ++i) tot += sigbuf[i] * sigbuf[i];
    const int capd = cap < kmax ? cap : kmax;
    int D;
    if (tot <= 0.0) {
      D = 1;
    } else if (tol <= 0.0) {
      D = capd;
    } else {
      // smallest D' >= 1 whose discarded tail (summed from the smallest
      // value) is <= tol^2
      double acc = 0.0;
      int best = kmax;
      for (int Dp = kmax - 1; Dp >= 1; --Dp) {
        acc += sigbuf[Dp] * sigbuf[Dp] / tot;
        if (acc <= tol * tol) best = Dp; else break;
      }
      D = best < capd ? best : capd;
    }
    if (D < 1) D = 1;
    double disc2 = 0.0;
    for (int i = D; i < ncol; ++i) disc2 += sigbuf[i] * sigbuf[i];
    Dsh = D;
    info[0] = (double)D;
    info[1] = (tot > 0.0) ? sqrt(disc2 / tot) : 0.0;
    info[2] = (double)sweep;
    info[3] = (double)converged;
    info[4] = (double)rounds;
  }
  __syncthreads();
  const int D = Dsh;
  if (mode == 0) {
    // Vt[d][i] = A[perm d][i] / sigma_d   (right singular vectors)
    for (long e = tid; e < (long)D * nrow; e += JT) {
      const long d = e / nrow, i = e % nrow;
      const double sd = sigbuf[d];
      Vt[e] = (sd > 0.0) ? A[(long)perm_out[d] * lda + i] / sd : 0.0;
    }
  } else {
    // out1[i][d] = A[perm d][i]   (left singular vectors times sigma)
    for (long e = tid; e < (long)nrow * D; e += JT) {
      const long i = e / D, d = e % D;
      Vt[e] = A[(long)perm_out[d] * lda + i];
    }
  }
  if (keep_v)
    for (long e = tid; e < (long)ncol * D; e += JT) {
      const long i = e / D, d = e % D;
      const double v = V[(long)perm_out[d] * ldv + i];
      USs[e] = (mode == 0) ? v * sigbuf[d] : v;
    }
}

constexpr int kReplayChunk = 16;   // rounds of the log staged in LDS at once

// Replays the logged rotations on J = I (c x c in LDS) and writes
// USs[i][d] = J[i][perm d] * sigma_d.
__global__ __launch_bounds__(JT) void jacobi_replay_kernel(
    int c, int mode, const double* __restrict__ rotlog,
    const int* __restrict__ rflag, const int* __restrict__ perm,
    const double* __restrict__ info, const double* __restrict__ sig,
    double* __restrict__ USs) {
  extern __shared__ double smem[];
  __shared__ int fl[kReplayChunk];
  const int tid = threadIdx.x;
  const int ldv = c | 1;
  double* V = smem;
  const Pairing P = make_pairing(c);
  double* L = smem + (long)c * ldv;  // kReplayChunk * 2 * np doubles
  for (long e = tid; e < (long)c * c; e += JT) {
    const long j = e / c, i = e % c;
    V[j * ldv + i] = (i == j) ? 1.0 : 0.0;
  }
  const int k = tid / G, lig = tid % G;
  const int rounds = (int)info[4];
  for (int r0 = 0; r0 < rounds; r0 += kReplayChunk) {
    const int nr = rounds - r0 < kReplayChunk ? rounds - r0 : kReplayChunk;
    __syncthreads();
    for (long e = tid; e < (long)nr * 2 * P.np; e += JT)
      L[e] = rotlog[(long)r0 * 2 * P.np + e];
    if (tid < nr) fl[tid] = rflag[r0 + tid];
    __syncthreads();
    for (int t = 0; t < nr; ++t) {
      if (fl[t] == 0) continue;  // uniform across the workgroup
      const int r = (r0 + t) % (P.cc - 1);
      if (k < P.np) {
        int p, q;
        pair_of(r, k, P.cc, p, q);
        const double cs = L[(long)t * 2 * P.np + 2 * k];
        const double sn = L[(long)t * 2 * P.np + 2 * k + 1];
        if (p < c && q < c && !(cs == 1.0 && sn == 0.0))
          rotate_cols(V + (long)p * ldv, V + (long)q * ldv, c, lig, cs, sn);
      }
      __syncthreads();
    }
  }
  __syncthreads();
  const int D = (int)info[0];
  for (long e = tid; e < (long)c * D; e += JT) {
    const long i = e / D, d = e % D;
    const double v = V[(long)perm[d] * ldv + i];
    USs[e] = (mode == 0) ? v * sig[d] : v;
  }
}

bool g_attr = false;

}  // namespace

size_t jacobi_lds_bytes(int k, int c, bool keep_v) {
  size_t a = (size_t)k * (size_t)(c | 1);
  size_t v = keep_v ? (size_t)k * (size_t)(k | 1) : 0;
  return (a + v) * sizeof(double);
}

void jacobi_svd(hipStream_t s, const double* Xr, int k, int c, long ldx,
                int mode, int cap, double tol, int max_sweeps, double* rotlog,
                int* rflag, double* out1, double* out2, double* sigbuf,
                int* perm, double* info, bool keep_v) {
  if (!g_attr) {
    MPSV_HIP(hipFuncSetAttribute((const void*)jacobi_cols_kernel,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)kJacobiMaxLds));
    MPSV_HIP(hipFuncSetAttribute((const void*)jacobi_replay_kernel,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)kJacobiMaxLds));
    g_attr = true;
  }
  const size_t lds = jacobi_lds_bytes(k, c, keep_v);
  MPSV_CHECK(lds <= kJacobiMaxLds && c <= kJacobiMaxCols && k <= c, kEinval,
             "Jacobi SVD: matrix does not fit on chip");
  hipLaunchKernelGGL(jacobi_cols_kernel, dim3(1), dim3(JT), lds, s, Xr, k, c,
                     ldx, keep_v ? 1 : 0, mode, rotlog, rflag, max_sweeps, cap,
                     tol, out1, out2, sigbuf, perm, info);
  MPSV_LAUNCHED();
  if (!keep_v) {
    const size_t lv = ((size_t)k * (size_t)(k | 1) +
                       (size_t)kReplayChunk * (k + 2)) * sizeof(double);
    hipLaunchKernelGGL(jacobi_replay_kernel, dim3(1), dim3(JT), lv, s, k, mode,
                       rotlog, rflag, perm, info, sigbuf, out2);
    MPSV_LAUNCHED();
  }
}

}  // namespace mpsv
