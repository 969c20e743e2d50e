// One-sided (Hestenes) Jacobi SVD of a small square triangular factor on
// one workgroup of 1024 threads.  The rotations act on the columns of
// B = R^T; they converge to v_i sigma_i, the right singular vectors of the
// matrix R came from, scaled by its singular values.  Working on the
// transpose of the triangular factor needs far fewer sweeps than working on
// the factor itself (about 9 against 22 on the matrices of the compression
// sweep).  The rotations themselves are not accumulated: the caller forms
// the left factor as X V (one GEMM), so the kernel keeps only B on chip.
//
// Columns are orthogonalised pairwise in the cyclic round-robin ordering:
// each round pairs all columns into disjoint pairs; a group of 16 lanes (one
// DPP row) owns one pair, accumulates the three inner products over its
// rows, reduces them with row-local DPP moves and applies the rotation.
// The columns live in LDS with an odd leading dimension so that the groups
// of one wave hit distinct banks.
//
// On exit: singular values are the column norms, sorted descending (ties by
// index), the truncation rank D follows the rule min(cap, smallest D' whose
// relative discarded weight is <= tol) (eq. 5 with the i = D+1 reading), and
// Vt (D x k) holds the kept right singular vectors (normalised columns).
#include <cmath>
#include <mutex>

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
// Xr: k x k row-major triangular factor; the Jacobi columns are its rows:
// A[j][i] = Xr[j][i].  Output Vt[d][i] = A[perm d][i] / sigma_d.
__global__ __launch_bounds__(JT) void jacobi_cols_kernel(
    const double* __restrict__ Xr, int k, long ldx, int max_sweeps, int cap,
    double tol, double* __restrict__ Vt, double* __restrict__ sigbuf,
    int* __restrict__ perm_out, double* __restrict__ info) {
  extern __shared__ double smem[];
  __shared__ double red[JT / 64];
  __shared__ int sweep_any;
  __shared__ int Dsh;
  const int tid = threadIdx.x;
  const int nrow = k, ncol = k;            // Jacobi matrix A = Xr^T
  const int lda = nrow | 1;
  double* A = smem;                        // A[j*lda + i]

  for (long e = tid; e < (long)ncol * nrow; e += JT) {
    const long j = e / nrow, i = e % nrow;
    A[j * lda + i] = Xr[j * ldx + i];
  }
  __syncthreads();
  double part = 0.0;
  for (long e = tid; e < (long)ncol * nrow; e += JT) {
    const long j = e / nrow, i = e % nrow;
    const double x = A[j * lda + i];
    part += x * x;
  }
  const double normF2 = block_sum(part, red);
  // Columns whose squared norm is below `negl` (sigma below 1e-15 of the
  // Frobenius norm) are numerical zeros: they are never rotated (rotating
  // them against the others only stirs rounding noise and can stall the
  // convergence to a linear rate), and their singular vectors are returned
  // as zero rows, so that the kept rows of Vt are orthonormal and X V_D is
  // a projection that misses at most that noise.
  const double negl = 1e-30 * normF2;
  // A pair is rotated when its cosine |g| / (|a_p| |a_q|) exceeds eps.  The
  // iteration stops after the first sweep in which no cosine exceeded conv
  // (its rotations are still applied).  Cyclic Jacobi converges
  // quadratically: once every rotation angle of a sweep is below conv, the
  // rotations that follow the visit of a pair can restore at most about
  // 2k conv^2 < 3e-14 of its cosine, so the extra sweep that would only
  // confirm convergence is skipped.  The threshold also tolerates pairs that
  // stagnate at rounding level near the numerical null space.
  const double eps = 1e-14, conv = 1e-8;

  const Pairing P = make_pairing(ncol);
  const int kk = tid / G, lig = tid % G;   // pair slot of this lane group
  int sweep = 0, converged = 0, rounds = 0;
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
        const bool rot = g != 0.0 && fabs(g) > eps * sqrt(a) * sqrt(b) && fmin(a, b) > negl;
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
          if (lig == 0 && fabs(g) > conv * sqrt(a) * sqrt(b)) sweep_any = 1;
        }
      }
      __syncthreads();
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
  // Vt[d][i] = A[perm d][i] / sigma_d   (right singular vectors)
  for (long e = tid; e < (long)D * nrow; e += JT) {
    const long d = e / nrow, i = e % nrow;
    const double sd = sigbuf[d];
    Vt[e] = (sd * sd > negl) ? A[(long)perm_out[d] * lda + i] / sd : 0.0;
  }
}

}  // namespace

size_t jacobi_lds_bytes(int k) {
  return (size_t)k * (size_t)(k | 1) * sizeof(double);
}

void jacobi_svd(hipStream_t s, const double* Xr, int k, long ldx, int cap,
                double tol, int max_sweeps, double* Vt, double* sigbuf,
                int* perm, double* info) {
  static std::once_flag once;
  std::call_once(once, [] {
    MPSV_HIP(hipFuncSetAttribute((const void*)jacobi_cols_kernel,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)kJacobiMaxLds));
  });
  const size_t lds = jacobi_lds_bytes(k);
  MPSV_CHECK(lds <= kJacobiMaxLds && k <= kJacobiMaxCols && k >= 1, kEinval,
             "Jacobi SVD: matrix does not fit on chip");
  hipLaunchKernelGGL(jacobi_cols_kernel, dim3(1), dim3(JT), lds, s, Xr, k, ldx,
                     max_sweeps, cap, tol, Vt, sigbuf, perm, info);
  MPSV_LAUNCHED();
}

}  // namespace mpsv
