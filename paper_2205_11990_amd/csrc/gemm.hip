// FP64 general strided batched GEMM on the CDNA4 matrix cores.
//
//   C[b] = alpha * A[b] (M x K) * B[b] (K x N) + beta * C[b]
//
// Every operand is a strided view (row stride, column stride, batch stride),
// so transposes, sub-blocks and the fused-bond reshapes of MPS cores are
// expressed without copies.  Tiles of 64 x 64 x 16 are staged through LDS;
// each of the 4 waves owns a 32 x 32 sub-tile computed by 2 x 2
// v_mfma_f64_16x16x4f64 accumulators (64-wide wavefronts).
#include <algorithm>

#include "gemm.hpp"
#include "prof.hpp"
#include "tune.hpp"

namespace mpsv {

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;

// Products with few rows and a short contraction, FP64: the MPO factor W
// (at most 48 x 48, shared by every batch entry) times many blocks.  They
// are bound by streaming B and C, and the 64 x 64 tiles of the matrix-core
// kernel would stay mostly empty.  One thread per column of one batch
// entry keeps the MM sums in registers and reads W from LDS (every lane the
// same word); loads of B and stores of C run along the columns.  Each
// output sums its K products in order, k = 0 .. K-1, whatever the instance
// count.
constexpr int SM_MAX = 48;
template <int MM>
__global__ __launch_bounds__(NT) void gemm_small_kernel(
    int M, int N, int K, double alpha, const double* __restrict__ A, long ars, long acs,
    const double* __restrict__ B, long brs, long bcs, long bbs, double beta,
    double* __restrict__ C, long crs, long ccs, long cbs, int nb, InstOff io) {
  __shared__ double Ws[MM * SM_MAX];
  {
    const long o_ = io.of(blockIdx.z);
    A = shifted(A, o_);
    B = shifted(B, o_);
    C = shifted(C, o_);
  }
  for (int e = threadIdx.x; e < MM * K; e += NT) {
    const int m = e / K, k = e - m * K;
    Ws[m * SM_MAX + k] = (m < M) ? A[(long)m * ars + (long)k * acs] : 0.0;
  }
  __syncthreads();
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= (long)nb * N) return;
  const int b = (int)(t / N), n = (int)(t - (long)b * N);
  const double* bp = B + (long)b * bbs + (long)n * bcs;
  double* cp = C + (long)b * cbs + (long)n * ccs;
  double acc[MM];
#pragma unroll
  for (int m = 0; m < MM; ++m) acc[m] = 0.0;
  // eight loads of B in flight before their products (a state alone has
  // too few waves to hide one load per step)
  int k = 0;
  for (; k + 8 <= K; k += 8) {
    double z[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) z[u] = bp[(long)(k + u) * brs];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int m = 0; m < MM; ++m) acc[m] = fma(Ws[m * SM_MAX + k + u], z[u], acc[m]);
  }
  for (; k < K; ++k) {
    const double z = bp[(long)k * brs];
#pragma unroll
    for (int m = 0; m < MM; ++m) acc[m] = fma(Ws[m * SM_MAX + k], z, acc[m]);
  }
#pragma unroll
  for (int m = 0; m < MM; ++m)
    if (m < M) {
      double* o = cp + (long)m * crs;
      *o = (beta == 0.0) ? alpha * acc[m] : fma(beta, *o, alpha * acc[m]);
    }
}

// blockIdx.z = batch * nsplit + split; split covers K range
// [split*kchunk, min(K, (split+1)*kchunk)).
__global__ __launch_bounds__(NT) void gemm_f64_kernel(
    int M, int N, int K, double alpha, const double* __restrict__ A, long ars,
    long acs, long abs_, const double* __restrict__ B, long brs, long bcs,
    long bbs, double beta, double* __restrict__ C, long crs, long ccs, long cbs,
    int a_kfast, int b_nfast, int nsplit, int kchunk, int zper, InstOff io) {
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // blockIdx.z = instance * zper + batch * nsplit + split
  const long o_ = io.of(blockIdx.z / zper);
  A = shifted(A, o_);
  B = shifted(B, o_);
  C = shifted(C, o_);
  const int zb = blockIdx.z % zper;
  const long bz = zb / nsplit;
  const int split = zb % nsplit;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  A += bz * abs_;
  B += bz * bbs;
  C += bz * cbs + (long)split * M * N * (nsplit > 1 ? 1 : 0);
  const int kbeg = split * kchunk;
  const int kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;

  dbl4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int q = 0; q < (BM * BK) / NT; ++q) {
      int e = tid + q * NT;
      int r, k;
      if (a_kfast) { r = e / BK; k = e % BK; } else { k = e / BM; r = e % BM; }
      int gr = m0 + r, gk = k0 + k;
      As[k][r] = (gr < M && gk < kend) ? A[(long)gr * ars + (long)gk * acs] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < (BN * BK) / NT; ++q) {
      int e = tid + q * NT;
      int c, k;
      if (b_nfast) { k = e / BN; c = e % BN; } else { c = e / BK; k = e % BK; }
      int gc = n0 + c, gk = k0 + k;
      Bs[k][c] = (gc < N && gk < kend) ? B[(long)gk * brs + (long)gc * bcs] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a0 = As[kr][wm * 32 + (lane & 15)];
      double a1 = As[kr][wm * 32 + 16 + (lane & 15)];
      double b0 = Bs[kr][wn * 32 + (lane & 15)];
      double b1 = Bs[kr][wn * 32 + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }

  // D layout of the 16x16 f64 block: lane l, item r -> row 4*r + l/16, col l%16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gr = m0 + wm * 32 + i * 16 + 4 * r + (lane >> 4);
        int gc = n0 + wn * 32 + j * 16 + (lane & 15);
        if (gr < M && gc < N) {
          double* cp = C + (long)gr * crs + (long)gc * ccs;
          double v = alpha * acc[i][j][r];
          *cp = (beta == 0.0) ? v : v + beta * (*cp);
        }
      }
}

// Large tiles for the big contractions (the MPO x MPS products of the
// field term at bond cap 128): a 128 x 128 output tile per workgroup of 256
// threads, four waves in a 2 x 2 arrangement, each owning 64 x 64 = 4 x 4
// blocks of v_mfma_f64_16x16x4f64 (16 accumulators, 64 doubles per lane).
// K advances in steps of 16 through two LDS buffers: the global loads of
// step t + 1 are in flight while the matrix cores work on step t, and one
// barrier per step separates the buffers.  AK: A's k index is contiguous
// (row-major A); BNF: B's n index is contiguous (row-major B); the loads of
// each thread walk the contiguous index.  TN = 64 gives 128 x 64 output
// tiles (each wave 64 x 32, 4 x 2 blocks): twice the tiles of a product, for
// shapes whose 128 x 128 tiles leave the last round of compute units mostly
// idle.  Every output sums its K products in the same order on the same
// instruction in all three tilings (64 x 64, 128 x 128, 128 x 64), so they
// give the same bits.
constexpr int TB = 128, TK = 16, TLD = TB + 2;

template <int AK, int BNF, int TN = 128>
__global__ __launch_bounds__(NT, 2) void gemm_f64_t128_kernel(
    int M, int N, int K, double alpha, const double* __restrict__ A, long ars,
    long acs, long abs_, const double* __restrict__ B, long brs, long bcs,
    long bbs, double beta, double* __restrict__ C, long crs, long ccs, long cbs,
    int nsplit, int kchunk, int zper, InstOff io) {
  static_assert(TN == 128 || TN == 64, "tile width 128 or 64");
  constexpr int PB = TN / 16;        // B values each thread stages per step
  constexpr int TPC = TK / PB;       // threads per column of a k-major B tile
  constexpr int NJ = TN / 32;        // 16-wide blocks per wave along n
  __shared__ double As[2][TK][TLD];
  __shared__ double Bs[2][TK][TN + 2];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const long o_ = io.of(blockIdx.z / zper);
  A = shifted(A, o_);
  B = shifted(B, o_);
  C = shifted(C, o_);
  const int zb = blockIdx.z % zper;
  const long bz = zb / nsplit;
  const int split = zb % nsplit;
  const int m0 = blockIdx.y * TB, n0 = blockIdx.x * TN;
  A += bz * abs_;
  B += bz * bbs;
  C += bz * cbs + (long)split * M * N * (nsplit > 1 ? 1 : 0);
  const int kbeg = split * kchunk;
  const int kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
  const int nt = (kend - kbeg + TK - 1) / TK;

  // each thread stages 8 values of A and 8 of B per step: along the
  // contiguous index of its operand, 8 consecutive elements
  //   A k-fast: row ra = tid / 2, k = (tid % 2) * 8 + e; else k = tid / 16,
  //   row = (tid % 16) * 8 + e.  B n-fast: k = tid / 16, col = (tid % 16) * 8
  //   + e; else col = tid / 2, k = (tid % 2) * 8 + e.
  double ra[8], rb[PB];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      int r, k;
      if (AK) { r = tid >> 1; k = ((tid & 1) << 3) + e; }
      else { k = tid >> 4; r = ((tid & 15) << 3) + e; }
      const int gr = m0 + r, gk = k0 + k;
      ra[e] = (gr < M && gk < kend) ? A[(long)gr * ars + (long)gk * acs] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < PB; ++e) {
      int c, k;
      if (BNF) { k = tid >> 4; c = (tid & 15) * PB + e; }
      else { c = tid / TPC; k = (tid % TPC) * PB + e; }
      const int gc = n0 + c, gk = k0 + k;
      rb[e] = (gc < N && gk < kend) ? B[(long)gk * brs + (long)gc * bcs] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      if (AK) As[buf][((tid & 1) << 3) + e][tid >> 1] = ra[e];
      else As[buf][tid >> 4][((tid & 15) << 3) + e] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < PB; ++e) {
      if (BNF) Bs[buf][tid >> 4][(tid & 15) * PB + e] = rb[e];
      else Bs[buf][(tid % TPC) * PB + e][tid / TPC] = rb[e];
    }
  };

  dbl4 acc[4][NJ];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  if (nt > 0) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  for (int t = 0; t < nt; ++t) {
    const int buf = t & 1;
    if (t + 1 < nt) load(kbeg + (t + 1) * TK);
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a[4], b[NJ];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[buf][kr][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < NJ; ++j) b[j] = Bs[buf][kr][wn * (TN / 2) + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (t + 1 < nt) store(buf ^ 1);
    __syncthreads();
  }

  // D layout of the 16x16 f64 block: lane l, item r -> row 4*r + l/16, col l%16
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = m0 + wm * 64 + i * 16 + 4 * r + (lane >> 4);
        const int gc = n0 + wn * (TN / 2) + j * 16 + (lane & 15);
        if (gr < M && gc < N) {
          double* cp = C + (long)gr * crs + (long)gc * ccs;
          const double v = alpha * acc[i][j][r];
          *cp = (beta == 0.0) ? v : v + beta * (*cp);
        }
      }
}

// Reduced-precision contraction variants (the MPS problem's precision modes
// 1 and 2): the FP64 operands are rounded as they are staged in LDS, to
// FP32 (MODE 1) or to BF16 (MODE 2: to FP32, then to the nearest BF16, ties
// to even), the products are accumulated in FP32 on the matrix cores
// (v_mfma_f32_16x16x4f32, or v_mfma_f32_16x16x16bf16 whose BF16 products
// are exact in FP32), and the result is stored as FP64.  Same tiling and
// views as gemm_f64_kernel.
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));

// x rounded to the nearest BF16 (ties to even), as a float; finite inputs
__device__ inline float round_bf16(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

template <int MODE>
__device__ inline float stage(double x) {
  if constexpr (MODE == 2) return round_bf16((float)x);
  else return (float)x;
}

template <int MODE>
__global__ __launch_bounds__(NT) void gemm_f32acc_kernel(
    int M, int N, int K, double alpha, const double* __restrict__ A, long ars,
    long acs, long abs_, const double* __restrict__ B, long brs, long bcs,
    long bbs, double beta, double* __restrict__ C, long crs, long ccs, long cbs,
    int a_kfast, int b_nfast, int nsplit, int kchunk, int zper, InstOff io) {
  __shared__ float As[BK][BM + 1];
  __shared__ float Bs[BK][BN + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // blockIdx.z = instance * zper + batch * nsplit + split
  const long o_ = io.of(blockIdx.z / zper);
  A = shifted(A, o_);
  B = shifted(B, o_);
  C = shifted(C, o_);
  const int zb = blockIdx.z % zper;
  const long bz = zb / nsplit;
  const int split = zb % nsplit;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  A += bz * abs_;
  B += bz * bbs;
  C += bz * cbs + (long)split * M * N * (nsplit > 1 ? 1 : 0);
  const int kbeg = split * kchunk;
  const int kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;

  flt4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = flt4{0.0f, 0.0f, 0.0f, 0.0f};

  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int q = 0; q < (BM * BK) / NT; ++q) {
      int e = tid + q * NT;
      int r, k;
      if (a_kfast) { r = e / BK; k = e % BK; } else { k = e / BM; r = e % BM; }
      int gr = m0 + r, gk = k0 + k;
      As[k][r] = (gr < M && gk < kend) ? stage<MODE>(A[(long)gr * ars + (long)gk * acs]) : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < (BN * BK) / NT; ++q) {
      int e = tid + q * NT;
      int c, k;
      if (b_nfast) { k = e / BN; c = e % BN; } else { c = e / BK; k = e % BK; }
      int gc = n0 + c, gk = k0 + k;
      Bs[k][c] = (gc < N && gk < kend) ? stage<MODE>(B[(long)gk * brs + (long)gc * bcs]) : 0.0f;
    }
    __syncthreads();
    if constexpr (MODE == 2) {
      // one 16 x 16 x 16 step: lane l holds k = 4 (l / 16) + q, q < 4, of
      // row (A) or column (B) l % 16, as the high halves of the staged floats
      static_assert(BK == 16, "one BF16 MFMA step per tile");
      bf16x4 a0, a1, b0, b1;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kr = 4 * (lane >> 4) + q;
        a0[q] = (short)(__float_as_uint(As[kr][wm * 32 + (lane & 15)]) >> 16);
        a1[q] = (short)(__float_as_uint(As[kr][wm * 32 + 16 + (lane & 15)]) >> 16);
        b0[q] = (short)(__float_as_uint(Bs[kr][wn * 32 + (lane & 15)]) >> 16);
        b1[q] = (short)(__float_as_uint(Bs[kr][wn * 32 + 16 + (lane & 15)]) >> 16);
      }
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b1, acc[1][1], 0, 0, 0);
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        const int kr = kk + (lane >> 4);
        const float a0 = As[kr][wm * 32 + (lane & 15)];
        const float a1 = As[kr][wm * 32 + 16 + (lane & 15)];
        const float b0 = Bs[kr][wn * 32 + (lane & 15)];
        const float b1 = Bs[kr][wn * 32 + 16 + (lane & 15)];
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // D layout of the 16x16 f32 block: lane l, item r -> row 4*(l/16) + r,
  // col l%16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gr = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        int gc = n0 + wn * 32 + j * 16 + (lane & 15);
        if (gr < M && gc < N) {
          double* cp = C + (long)gr * crs + (long)gc * ccs;
          double v = alpha * (double)acc[i][j][r];
          *cp = (beta == 0.0) ? v : v + beta * (*cp);
        }
      }
}

// C[b] = alpha * sum_s P[b*nsplit + s] + beta * C[b]
__global__ void splitk_reduce_kernel(int M, int N, int nsplit, double alpha,
                                     const double* __restrict__ P, double beta,
                                     double* __restrict__ C, long crs, long ccs,
                                     long cbs, InstOff io) {
  const long o_ = io.of(blockIdx.z);
  P = shifted(P, o_);
  C = shifted(C, o_);
  const long b = blockIdx.y;
  const long MN = (long)M * N;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < MN;
       e += (long)gridDim.x * blockDim.x) {
    double acc = 0.0;
    const double* pp = P + b * nsplit * MN + e;
    for (int q = 0; q < nsplit; ++q) acc += pp[q * MN];
    const long i = e / N, j = e % N;
    double* cp = C + b * cbs + i * crs + j * ccs;
    *cp = (beta == 0.0) ? alpha * acc : alpha * acc + beta * (*cp);
  }
}

}  // namespace

void gemm(hipStream_t s, int M, int N, int K, double alpha, CMatView A,
          CMatView B, double beta, MatView C, int batch, int prec, Arena* ws) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K <= 0) {
    // C = beta * C
    scale_matrix(s, M, N, beta, C, batch);
    return;
  }
  const int a_kfast = (A.cs == 1) ? 1 : 0;
  const int b_nfast = (B.cs == 1) ? 1 : 0;
  const int ninst = inst_count();
  if (prec == 0 && M <= SM_MAX && K <= SM_MAX && A.bs == 0 && (long)batch * N >= 4 * NT) {
    // a small shared factor times many columns: the streaming kernel
    const int slot = prof_begin(s);
    const long cols = (long)batch * N;
    const dim3 grid(ceil_div(cols, NT), 1, ninst);
    if (M <= 16)
      hipLaunchKernelGGL(gemm_small_kernel<16>, grid, dim3(NT), 0, s, M, N, K, alpha, A.p, A.rs,
                         A.cs, B.p, B.rs, B.cs, B.bs, beta, C.p, C.rs, C.cs, C.bs, batch,
                         inst_off());
    else
      hipLaunchKernelGGL(gemm_small_kernel<SM_MAX>, grid, dim3(NT), 0, s, M, N, K, alpha, A.p,
                         A.rs, A.cs, B.p, B.rs, B.cs, B.bs, beta, C.p, C.rs, C.cs, C.bs, batch,
                         inst_off());
    MPSV_LAUNCHED();
    prof_end(s, slot, kClsGemm, 2.0 * M * N * (double)K * batch,
             8.0 * ((double)M * K + ((double)K * N + 2.0 * M * N) * batch));
    return;
  }
  // split K when the output alone (in 64 x 64 tiles) cannot fill the chip;
  // the partial products live in the caller's workspace (none given: no
  // split).  The choice ignores lock-step instances, so that every instance
  // sums in the order a stand-alone state does.
  const long tiles64 = (long)ceil_div(N, BN) * ceil_div(M, BM);
  int nsplit = 1;
  if (ws && K >= 4 * BK * 4 && tiles64 * batch < 256) {
    long want = 512 / (tiles64 * batch);
    long maxk = K / (4 * BK);
    const long fit = (long)(ws->max_alloc_bytes() / sizeof(double)) /
                     std::max(1L, (long)batch * M * N);
    nsplit = (int)std::max(1L, std::min(std::min(std::min(want, maxk), 64L), fit));
  }
  // FP64 products with at least two 128 x 128 tiles per compute unit take
  // the large tiles, unless the launch-shape table says otherwise for this
  // shape and instance count (both tiles give the same bits: each output
  // sums its K products in the same order on the same matrix-core
  // instruction)
  bool big = prec == 0 && nsplit == 1 && M >= TB && N >= TB && K >= TK &&
             (long)ceil_div(N, TB) * ceil_div(M, TB) * batch >= 512;
  // tiling: 0 = 64 x 64, 1 = 128 x 128, 2 = 128 x 64
  TunePick tp{big ? 1 : 0, -1};
  if (prec == 0 && nsplit == 1) {
    const TuneKey key{{kTuneGemmTile, M, N, K, 4 * batch + 2 * a_kfast + b_nfast,
                       tune_inst_class(ninst)}};
    tp = tune_pick(s, key, big ? 1 : 0, 7u);
    big = tp.value != 0;
  }
  const bool half = big && tp.value == 2;
  const int tm = big ? TB : BM, tn = big ? (half ? TB / 2 : TB) : BN;
  const int kchunk = (nsplit > 1) ? ceil_div(ceil_div(K, nsplit), BK) * BK : K;
  if (nsplit > 1) nsplit = ceil_div(K, kchunk);
  const int bmax = std::max(1, 65535 / (nsplit * ninst));
  for (int b0 = 0; b0 < batch; b0 += bmax) {
    int nb = batch - b0 < bmax ? batch - b0 : bmax;
    const int zper = nb * nsplit;
    dim3 grid(ceil_div(N, tn), ceil_div(M, tm), zper * ninst);
    const int slot = prof_begin(s);
    if (big && nsplit == 1) {
      auto k = half ? (a_kfast ? (b_nfast ? gemm_f64_t128_kernel<1, 1, 64> : gemm_f64_t128_kernel<1, 0, 64>)
                               : (b_nfast ? gemm_f64_t128_kernel<0, 1, 64> : gemm_f64_t128_kernel<0, 0, 64>))
                    : (a_kfast ? (b_nfast ? gemm_f64_t128_kernel<1, 1> : gemm_f64_t128_kernel<1, 0>)
                               : (b_nfast ? gemm_f64_t128_kernel<0, 1> : gemm_f64_t128_kernel<0, 0>));
      hipLaunchKernelGGL(k, grid, dim3(NT), 0, s, M, N, K, alpha,
                         A.p + (long)b0 * A.bs, A.rs, A.cs, A.bs,
                         B.p + (long)b0 * B.bs, B.rs, B.cs, B.bs, beta,
                         C.p + (long)b0 * C.bs, C.rs, C.cs, C.bs, 1, K, zper,
                         inst_off());
      MPSV_LAUNCHED();
    } else if (nsplit == 1) {
      hipLaunchKernelGGL(prec == 2 ? gemm_f32acc_kernel<2>
                         : prec == 1 ? gemm_f32acc_kernel<1> : gemm_f64_kernel, grid,
                         dim3(NT), 0, s, M, N, K, alpha,
                         A.p + (long)b0 * A.bs, A.rs, A.cs, A.bs,
                         B.p + (long)b0 * B.bs, B.rs, B.cs, B.bs, beta,
                         C.p + (long)b0 * C.bs, C.rs, C.cs, C.bs, a_kfast,
                         b_nfast, 1, K, zper, inst_off());
      MPSV_LAUNCHED();
    } else {
      ArenaScope sc(*ws);
      double* P = ws->alloc((size_t)nb * nsplit * M * N);
      hipLaunchKernelGGL(prec == 2 ? gemm_f32acc_kernel<2>
                         : prec == 1 ? gemm_f32acc_kernel<1> : gemm_f64_kernel, grid,
                         dim3(NT), 0, s, M, N, K, 1.0,
                         A.p + (long)b0 * A.bs, A.rs, A.cs, A.bs,
                         B.p + (long)b0 * B.bs, B.rs, B.cs, B.bs, 0.0, P,
                         (long)N, 1L, (long)nsplit * M * N, a_kfast, b_nfast,
                         nsplit, kchunk, zper, inst_off());
      MPSV_LAUNCHED();
      const long MN = (long)M * N;
      int blocks = ceil_div(MN, 256);
      if (blocks > 1024) blocks = 1024;
      hipLaunchKernelGGL(splitk_reduce_kernel, dim3(blocks, nb, ninst), dim3(256), 0,
                         s, M, N, nsplit, alpha, P, beta,
                         C.p + (long)b0 * C.bs, C.rs, C.cs, C.bs, inst_off());
      MPSV_LAUNCHED();
    }
    prof_end(s, slot, kClsGemm, 2.0 * M * N * (double)K * nb,
             8.0 * ((double)M * K + (double)K * N + 2.0 * M * N) * nb);
  }
  tune_end(s, tp.slot);
}

namespace {
__global__ void scale_matrix_kernel(int M, int N, double beta, double* C,
                                    long rs, long cs, long bs, InstOff io) {
  C = shifted(C, io.of(blockIdx.z));
  long b = blockIdx.y;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)M * N;
       e += (long)gridDim.x * blockDim.x) {
    long i = e / N, j = e % N;
    double* p = C + b * bs + i * rs + j * cs;
    *p = (beta == 0.0) ? 0.0 : beta * (*p);
  }
}
}  // namespace

void scale_matrix(hipStream_t s, int M, int N, double beta, MatView C,
                  int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  long tot = (long)M * N;
  int blocks = ceil_div(tot, 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(scale_matrix_kernel, dim3(blocks, batch, inst_count()), dim3(256), 0,
                     s, M, N, beta, C.p, C.rs, C.cs, C.bs, inst_off());
  MPSV_LAUNCHED();
}

}  // namespace mpsv
