// Householder QR (SI, "Canonicalization and Compression": the left sweep
// and the triangular preconditioning of the SVD) with the matrix held in the
// registers of one workgroup.
//
// Factorisation: 16 waves; wave w holds the columns j = w + 16 b (b < CPW)
// and lane l of every wave the rows i = l + 64 a (a < RPL), so each column
// lives inside one wave and the products v^T A of a reflector with the
// columns are wave-local sums: no LDS partial tables, one barrier per
// column.  For column j the owning wave forms the reflector (LAPACK dlarfg
// conventions: beta = -sign(alpha) |x|, tau = (beta - alpha) / beta,
// v = x / (alpha - beta), v_j = 1) and publishes v in LDS (double
// buffered); after the barrier every wave updates its columns right of j.
// The reflectors go to global memory, column-major, for later application.
//
// Application: Q Y or Q^T Y for a block of columns Y; each wave owns CPW
// columns and streams the reflectors from L2, several steps ahead of their
// use, with the reflector scalars held in lane registers.  Up to 256 rows
// the reflectors are applied four at a time as compact-WY blocks (one
// cross-lane reduction per block instead of one per reflector).  There is
// no dependency between columns, so the kernel has no barrier and spreads
// over as many workgroups as the column count allows.  Panels of a wider matrix are
// factored one after the other with the trailing columns updated by the
// same application kernel (blocked right-looking QR without a T factor).
#include <algorithm>
#include <cmath>
#include <mutex>

#include "prof.hpp"
#include "qr_reg.hpp"
#include "tune.hpp"
#include "wave.hpp"

namespace mpsv {

// Row chunks of a tall block handled by the workgroups y of one launch:
// chunk y is rows [y * rows, min((y + 1) * rows, m)); its reflectors start
// at V + y * rows * kstride and tau + y * kstride.  One chunk ({m, k}) is
// the plain single-block case.
struct Chunks {
  int rows;
  int kstride;
};

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int FT = 1024;  // factorisation workgroup: 16 waves
constexpr int AT = 256;   // application workgroup: 4 waves

// 1 / x from the hardware reciprocal estimate refined by two Newton steps
// (e = 1 - x y, y <- y + y e), within about one unit in the last place;
// shorter than the correctly rounded division on the reflector's critical
// path.  x is finite and non-zero where it is used.
__device__ __forceinline__ double recip(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

template <int N>
__device__ __forceinline__ void sums_any(double (&p)[N]) {
  if constexpr (N == 1 || N == 2 || N == 4 || N == 8) {
    wave::sums<N>(p);
  } else {
    constexpr int M = N <= 4 ? 4 : 8;
    double q[M];
#pragma unroll
    for (int i = 0; i < M; ++i) q[i] = i < N ? p[i] : 0.0;
    wave::sums<M>(q);
#pragma unroll
    for (int i = 0; i < N; ++i) p[i] = q[i];
  }
}

// Columns 16 B .. 16 B + 15 of the factorisation (register column B).
template <int CPW, int RPL, int B>
__device__ __forceinline__ void factor_block(double (&x)[RPL][CPW], int w,
                                             int l, int m, int k, double* vb,
                                             double* tb, double* __restrict__ V,
                                             double* __restrict__ tau) {
  constexpr int NB = CPW - B;  // register columns that can still change
  for (int t = 0; t < 16; ++t) {
    const int j = 16 * B + t;
    if (j >= k) return;  // uniform over the workgroup
    const int buf = j & 1;
    double* vj = vb + buf * 64 * RPL;
    if (w == t) {
      double s2 = 0.0, xa = 0.0;
      const int aj = j >> 6;
#pragma unroll
      for (int a = 0; a < RPL; ++a) {
        const int i = l + 64 * a;
        const double xi = x[a][B];
        if (i > j) s2 = fma(xi, xi, s2);
        if (a == aj) xa = xi;
      }
      s2 = wave::sum64(s2);
      const double alpha = wave::read_lane(xa, j & 63);
      double tj = 0.0, beta = alpha, scal = 0.0;
      if (s2 > 0.0) {
        beta = -copysign(sqrt(fma(alpha, alpha, s2)), alpha);
        tj = (beta - alpha) * recip(beta);
        scal = recip(alpha - beta);
      }
      // The reflector goes to global memory now, or (32 rows per lane,
      // where the row addresses would not fit in registers) stays below the
      // diagonal of its column and is written out with R at the end.
#pragma unroll
      for (int a = 0; a < RPL; ++a) {
        const int i = l + 64 * a;
        const double v = (i > j) ? x[a][B] * scal : (i == j ? 1.0 : 0.0);
        vj[i] = v;
        if constexpr (RPL < 32) {
          if (i < m) V[(long)j * m + i] = v;
          x[a][B] = (i == j) ? beta : (i > j ? 0.0 : x[a][B]);
        } else {
          x[a][B] = (i == j) ? beta : (i > j ? v : x[a][B]);
        }
      }
      if (l == 0) {
        tb[buf] = tj;
        tau[j] = tj;
      }
    }
    wave::lds_barrier();
    const double tj = tb[buf];
    if (tj != 0.0) {
      // the reflector is kept in registers unless the rows need 32 per
      // lane; then it is streamed from LDS in chunks of 8 rows (the empty
      // asm statements keep the compiler from hoisting all the loads)
      constexpr bool kVReg = RPL < 32;
      constexpr int CH = kVReg ? RPL : 8;
      double v[kVReg ? RPL : 1];
      if constexpr (kVReg) {
#pragma unroll
        for (int a = 0; a < RPL; ++a) v[a] = vj[l + 64 * a];
      }
      double p[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) p[q] = 0.0;
#pragma unroll
      for (int a0 = 0; a0 < RPL; a0 += CH) {
        double vc[CH];
#pragma unroll
        for (int i = 0; i < CH; ++i) vc[i] = kVReg ? v[a0 + i] : vj[l + 64 * (a0 + i)];
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
          for (int i = 0; i < CH; ++i) p[q] = fma(vc[i], x[a0 + i][B + q], p[q]);
        if constexpr (!kVReg) __asm__ volatile("" ::: "memory");
      }
      // register column B of this wave is column j itself (w == t) or
      // already finished (w < t); both hold reflectors below the diagonal
      if (w <= t) p[0] = 0.0;
      sums_any<NB>(p);
#pragma unroll
      for (int q = 0; q < NB; ++q) p[q] *= tj;
#pragma unroll
      for (int a0 = 0; a0 < RPL; a0 += CH) {
        double vc[CH];
#pragma unroll
        for (int i = 0; i < CH; ++i) vc[i] = kVReg ? v[a0 + i] : vj[l + 64 * (a0 + i)];
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
          for (int i = 0; i < CH; ++i) x[a0 + i][B + q] = fma(-vc[i], p[q], x[a0 + i][B + q]);
        if constexpr (!kVReg) __asm__ volatile("" ::: "memory");
      }
    }
  }
  if constexpr (B + 1 < CPW)
    factor_block<CPW, RPL, B + 1>(x, w, l, m, k, vb, tb, V, tau);
}

template <int CPW, int RPL>
__global__ __launch_bounds__(FT) void qr_reg_factor_kernel(
    CMatView A, int m, int n, MatView R, double* __restrict__ V,
    double* __restrict__ tau, Chunks ch, InstOff io) {
  __shared__ double vb[2 * 64 * RPL];
  __shared__ double tb[2];
  {
    const long o_ = io.of(blockIdx.z);
    A = shifted(A, o_);
    R = shifted(R, o_);
    V = shifted(V, o_);
    tau = shifted(tau, o_);
  }
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  // workgroup y factors rows [y * ch.rows, ...) of A on its own; its R
  // block goes n rows further down R, its reflectors to its own slots
  const int cb = blockIdx.y;
  const int row0 = cb * ch.rows;
  m = min(ch.rows, m - row0);
  A.p += (long)row0 * A.rs;
  R.p += (long)cb * n * R.rs;
  V += (long)cb * ch.rows * n;
  tau += (long)cb * n;
  const int k = m < n ? m : n;
  double x[RPL][CPW];
#pragma unroll
  for (int a = 0; a < RPL; ++a)
#pragma unroll
    for (int b = 0; b < CPW; ++b) {
      const int i = l + 64 * a, j = w + 16 * b;
      x[a][b] = (i < m && j < n) ? A.p[(long)i * A.rs + (long)j * A.cs] : 0.0;
    }
  factor_block<CPW, RPL, 0>(x, w, l, m, k, vb, tb, V, tau);
  // every wave has passed the first barrier, so A (which R may alias) has
  // been read completely
#pragma unroll
  for (int b = 0; b < CPW; ++b) {
    const int j = w + 16 * b;
    if (j >= n) continue;
#pragma unroll
    for (int a = 0; a < RPL; ++a) {
      const int i = l + 64 * a;
      if (i < k) R.p[(long)i * R.rs + (long)j * R.cs] = (i <= j) ? x[a][b] : 0.0;
      if (RPL == 32 && j < k && i < m)
        V[(long)j * m + i] = (i > j) ? x[a][b] : (i == j ? 1.0 : 0.0);
    }
  }
}

// Factorisation with a column per DPP row: group g (16 lanes) holds the
// columns c = g + 64 s (s < CPG), lane l of the group the rows l + 16 a
// (a < RPT).  The products v^T A of a reflector with a column are then
// reduced over 16 lanes only (row-local DPP moves), four columns per wave
// at once, which needs fewer cross-lane instructions per column than the
// wave-per-column layout when the rows fit in 16 * RPT <= 256.
template <int CPG, int RPT>
__global__ __launch_bounds__(FT) void qr_g16_factor_kernel(
    CMatView A, int m, int n, MatView R, double* __restrict__ V,
    double* __restrict__ tau, InstOff io) {
  __shared__ double vb[2 * 16 * RPT];
  __shared__ double tb[2];
  {
    const long o_ = io.of(blockIdx.z);
    A = shifted(A, o_);
    R = shifted(R, o_);
    V = shifted(V, o_);
    tau = shifted(tau, o_);
  }
  const int tid = threadIdx.x, g = tid >> 4, lig = tid & 15;
  const int k = m < n ? m : n;
  double x[CPG][RPT];
#pragma unroll
  for (int c = 0; c < CPG; ++c)
#pragma unroll
    for (int a = 0; a < RPT; ++a) {
      const int i = lig + 16 * a, j = g + 64 * c;
      x[c][a] = (i < m && j < n) ? A.p[(long)i * A.rs + (long)j * A.cs] : 0.0;
    }
  for (int j = 0; j < k; ++j) {
    const int og = j & 63, os = j >> 6, buf = j & 1;
    double* vj = vb + buf * 16 * RPT;
    if (g == og) {  // the 16 lanes owning column j (register column os)
#pragma unroll
      for (int c = 0; c < CPG; ++c) {
        if (c != os) continue;
        double s2 = 0.0, xa = 0.0;
        const int aj = j >> 4;
#pragma unroll
        for (int a = 0; a < RPT; ++a) {
          const int i = lig + 16 * a;
          if (i > j) s2 = fma(x[c][a], x[c][a], s2);
          if (a == aj) xa = x[c][a];
        }
        s2 = wave::sum16(s2);
        const double alpha = wave::read_lane(xa, ((g & 3) << 4) + (j & 15));
        double tj = 0.0, beta = alpha, scal = 0.0;
        if (s2 > 0.0) {
          beta = -copysign(sqrt(fma(alpha, alpha, s2)), alpha);
          tj = (beta - alpha) * recip(beta);
          scal = recip(alpha - beta);
        }
        double* Vj = V + (long)j * m;
#pragma unroll
        for (int a = 0; a < RPT; ++a) {
          const int i = lig + 16 * a;
          const double v = (i > j) ? x[c][a] * scal : (i == j ? 1.0 : 0.0);
          vj[i] = v;
          if (i < m) Vj[i] = v;
          x[c][a] = (i == j) ? beta : (i > j ? 0.0 : x[c][a]);
        }
        if (lig == 0) {
          tb[buf] = tj;
          tau[j] = tj;
        }
      }
    }
    wave::lds_barrier();
    const double tj = tb[buf];
    if (tj != 0.0) {
      double v[RPT];
#pragma unroll
      for (int a = 0; a < RPT; ++a) v[a] = vj[lig + 16 * a];
#pragma unroll
      for (int c = 0; c < CPG; ++c) {
        const int col = g + 64 * c;
        if (col > j && col < n) {  // uniform over the group
          // four independent partial sums shorten the dependency chain
          double d[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int a = 0; a < RPT; ++a) d[a & 3] = fma(v[a], x[c][a], d[a & 3]);
          const double f = tj * wave::sum16((d[0] + d[1]) + (d[2] + d[3]));
#pragma unroll
          for (int a = 0; a < RPT; ++a) x[c][a] = fma(-v[a], f, x[c][a]);
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CPG; ++c) {
    const int j = g + 64 * c;
    if (j >= n) continue;
#pragma unroll
    for (int a = 0; a < RPT; ++a) {
      const int i = lig + 16 * a;
      if (i < k) R.p[(long)i * R.rs + (long)j * R.cs] = (i <= j) ? x[c][a] : 0.0;
    }
  }
}

// Blocked factorisation with panels of eight columns, for m <= 64 * RPL
// rows and n <= 128 columns.  Wave w holds the columns 8w .. 8w+7 (lane
// l the rows l + 64 a).  Panel p is factored by wave p alone, without
// barriers (its reflectors update the rest of the panel in registers); it
// then publishes the eight reflectors in LDS and every wave to its right
// applies them to its own columns.  The wave that owns the next panel
// applies them first and factors its panel straight away, so one barrier
// per panel suffices and the other waves' updates overlap the next panel.
template <int RPL>
__device__ __forceinline__ void blk_factor_panel(double (&x)[RPL][8], int p,
                                                 int l, int k, double* vb,
                                                 double* tb,
                                                 double* __restrict__ tau);

template <int RPL, int B>
__device__ __forceinline__ void blk_factor_col(double (&x)[RPL][8], int p,
                                               int l, int k, double* vb,
                                               double* tb,
                                               double* __restrict__ tau) {
  const int j = 8 * p + B;
  if (j >= k) return;
  double s2 = 0.0, xa = 0.0;
  const int aj = j >> 6;
#pragma unroll
  for (int a = 0; a < RPL; ++a) {
    const int i = l + 64 * a;
    if (i > j) s2 = fma(x[a][B], x[a][B], s2);
    if (a == aj) xa = x[a][B];
  }
  s2 = wave::sum64(s2);
  const double alpha = wave::read_lane(xa, j & 63);
  double tj = 0.0, beta = alpha, scal = 0.0;
  if (s2 > 0.0) {
    beta = -copysign(sqrt(fma(alpha, alpha, s2)), alpha);
    tj = (beta - alpha) * recip(beta);
    scal = recip(alpha - beta);
  }
  double v[RPL];
#pragma unroll
  for (int a = 0; a < RPL; ++a) {
    const int i = l + 64 * a;
    v[a] = (i > j) ? x[a][B] * scal : (i == j ? 1.0 : 0.0);
    vb[B * 64 * RPL + i] = v[a];
    // LAPACK storage: beta on the diagonal, the reflector below
    x[a][B] = (i == j) ? beta : (i > j ? v[a] : x[a][B]);
  }
  if (l == 0) {
    tb[B] = tj;
    tau[j] = tj;
  }
  if constexpr (B < 7) {
    if (tj != 0.0) {
      constexpr int NB = 7 - B;
      double d[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < RPL; ++a) acc = fma(v[a], x[a][B + 1 + q], acc);
        d[q] = acc;
      }
      sums_any<NB>(d);
      if constexpr (RPL >= 4) {
        // reread the reflector (this wave's own LDS writes) rather than
        // keep it live across the reduction
        __asm__ volatile("" ::: "memory");
#pragma unroll
        for (int a = 0; a < RPL; ++a) v[a] = vb[B * 64 * RPL + l + 64 * a];
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const double f = tj * d[q];
#pragma unroll
        for (int a = 0; a < RPL; ++a) x[a][B + 1 + q] = fma(-v[a], f, x[a][B + 1 + q]);
      }
    }
    blk_factor_col<RPL, B + 1>(x, p, l, k, vb, tb, tau);
  }
}

template <int RPL>
__device__ __forceinline__ void blk_factor_panel(double (&x)[RPL][8], int p,
                                                 int l, int k, double* vb,
                                                 double* tb,
                                                 double* __restrict__ tau) {
  blk_factor_col<RPL, 0>(x, p, l, k, vb, tb, tau);
}

template <int RPL>
__device__ __forceinline__ void blk_apply_panel(double (&x)[RPL][8], int p,
                                                int l, int k, const double* vb,
                                                const double* tb) {
#pragma unroll 1
  for (int b = 0; b < 8; ++b) {
    if (8 * p + b >= k) break;
    const double tj = tb[b];
    if (tj == 0.0) continue;
    double v[RPL];
#pragma unroll
    for (int a = 0; a < RPL; ++a) v[a] = vb[b * 64 * RPL + l + 64 * a];
    double d[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < RPL; ++a) acc = fma(v[a], x[a][c], acc);
      d[c] = acc;
    }
    wave::sums<8>(d);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double f = tj * d[c];
#pragma unroll
      for (int a = 0; a < RPL; ++a) x[a][c] = fma(-v[a], f, x[a][c]);
    }
  }
}

template <int RPL>
__global__ __launch_bounds__(FT) void qr_blk_factor_kernel(
    CMatView A, int m, int n, MatView R, double* __restrict__ V,
    double* __restrict__ tau, InstOff io) {
  __shared__ double vb[2 * 8 * 64 * RPL];
  __shared__ double tb[2 * 8];
  {
    const long o_ = io.of(blockIdx.z);
    A = shifted(A, o_);
    R = shifted(R, o_);
    V = shifted(V, o_);
    tau = shifted(tau, o_);
  }
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int k = m < n ? m : n;
  const int npan = (k + 7) / 8;
  double x[RPL][8];
#pragma unroll
  for (int a = 0; a < RPL; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int i = l + 64 * a, j = 8 * w + b;
      x[a][b] = (i < m && j < n) ? A.p[(long)i * A.rs + (long)j * A.cs] : 0.0;
    }
  for (int p = 0; p < npan; ++p) {
    double* vbp = vb + (p & 1) * 8 * 64 * RPL;
    double* tbp = tb + (p & 1) * 8;
    if (w == p) blk_factor_panel<RPL>(x, p, l, k, vbp, tbp, tau);
    wave::lds_barrier();
    if (w > p) blk_apply_panel<RPL>(x, p, l, k, vbp, tbp);
  }
  // every wave has passed the first barrier, so A (which R may alias) has
  // been read completely
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const int j = 8 * w + b;
    if (j >= n) continue;
#pragma unroll
    for (int a = 0; a < RPL; ++a) {
      const int i = l + 64 * a;
      if (i < k) R.p[(long)i * R.rs + (long)j * R.cs] = (i <= j) ? x[a][b] : 0.0;
      if (j < k && i < m) V[(long)j * m + i] = (i > j) ? x[a][b] : (i == j ? 1.0 : 0.0);
    }
  }
}

template <int CPW, int RPL>
__global__ __launch_bounds__(AT) void qr_reg_apply_kernel(
    const double* __restrict__ V, const double* __restrict__ tau, int m, int k,
    CMatView Yin, int rows_in, MatView Yout, int p, int trans, Chunks ch,
    InstOff io) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  {
    const long o_ = io.of(blockIdx.z);
    V = shifted(V, o_);
    tau = shifted(tau, o_);
    Yin = shifted(Yin, o_);
    Yout = shifted(Yout, o_);
  }
  // workgroup row y applies the reflectors of chunk y to rows
  // [y * ch.rows, ...) (see qr_reg_factor_chunks)
  {
    const int cb = blockIdx.y;
    const int row0 = cb * ch.rows;
    const int mc = min(ch.rows, m - row0);
    V += (long)cb * ch.rows * ch.kstride;
    tau += (long)cb * ch.kstride;
    k = min(k, mc);
    rows_in = min(rows_in - row0, mc);
    m = mc;
    Yin.p += (long)row0 * Yin.rs;
    Yout.p += (long)row0 * Yout.rs;
  }
  const int c0 = (blockIdx.x * (AT / 64) + w) * CPW;
  if (c0 >= p) return;  // whole wave; the kernel has no barrier
  double y[RPL][CPW];
#pragma unroll
  for (int a = 0; a < RPL; ++a)
#pragma unroll
    for (int b = 0; b < CPW; ++b) {
      const int i = l + 64 * a;
      y[a][b] = (i < rows_in && c0 + b < p)
                    ? Yin.p[(long)i * Yin.rs + (long)(c0 + b) * Yin.cs] : 0.0;
    }
  // the scalars of all k <= 128 reflectors in two lane registers, read by
  // lane index in the loop (no memory round trip per reflector)
  const double ta = (l < k) ? tau[l] : 0.0;
  const double tb = (l + 64 < k) ? tau[l + 64] : 0.0;
  if constexpr (RPL <= 4) {
    // Blocks of four reflectors as one compact-WY product (forward
    // accumulation of the triangular factor): Q_B = H_j0 H_j0+1 H_j0+2
    // H_j0+3 = I - V T V^T with T upper triangular, T_ii = tau_i and
    // T_{<i,i} = -tau_i T_{<i,<i} (V_{<i}^T v_i).  Q Y applies the blocks
    // last to first as Y - V (T (V^T Y)), Q^T Y first to last as
    // Y - V (T^T (V^T Y)).  The products V^T Y and the six V^T V entries
    // of a block are reduced across the wave together, so a block costs
    // one reduction instead of four dependent ones.  Reflectors past k
    // enter as zero with tau = 0 (the identity).  Blocks are loaded PB
    // ahead into a register ring; rows past m read row m - 1 and are
    // zeroed when the block is used (no branch around the loads).
    constexpr int BK = 4;
    constexpr int PB = RPL <= 2 ? 2 : 1;
    constexpr int NR = BK * CPW + 6;
    constexpr int NRP = (NR + 3) / 4 * 4;
    const int nb = (k + BK - 1) / BK;
    auto roff = [&](int a) { return (long)min(l + 64 * a, m - 1); };
    auto blk = [&](int t) { return trans ? t : nb - 1 - t; };
    double ring[PB][BK][RPL];
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int B = blk(min(q, nb - 1));
#pragma unroll
      for (int i = 0; i < BK; ++i) {
        const long j = min(BK * B + i, k - 1);
#pragma unroll
        for (int a = 0; a < RPL; ++a) ring[q][i][a] = V[j * m + roff(a)];
      }
    }
    for (int t0 = 0; t0 < nb; t0 += PB) {
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        const int t = t0 + q;
        if (t >= nb) break;  // uniform
        const int B = blk(t);
        double v[BK][RPL];
        double tq[BK];
#pragma unroll
        for (int i = 0; i < BK; ++i) {
          const int j = BK * B + i;
          const bool ok = j < k;
#pragma unroll
          for (int a = 0; a < RPL; ++a)
            v[i][a] = (ok && l + 64 * a < m) ? ring[q][i][a] : 0.0;
          const double tj = wave::read_lane(j < 64 ? ta : tb, j & 63);
          tq[i] = ok ? tj : 0.0;
        }
        {
          const int Bn = blk(min(t + PB, nb - 1));
#pragma unroll
          for (int i = 0; i < BK; ++i) {
            const long j = min(BK * Bn + i, k - 1);
#pragma unroll
            for (int a = 0; a < RPL; ++a) ring[q][i][a] = V[j * m + roff(a)];
          }
        }
        // r = [V^T y (BK x CPW), v0.v1, v0.v2, v0.v3, v1.v2, v1.v3, v2.v3, 0..]
        double r[NRP];
#pragma unroll
        for (int e = 0; e < NRP; ++e) r[e] = 0.0;
#pragma unroll
        for (int a = 0; a < RPL; ++a) {
#pragma unroll
          for (int i = 0; i < BK; ++i)
#pragma unroll
            for (int b = 0; b < CPW; ++b) r[i * CPW + b] = fma(v[i][a], y[a][b], r[i * CPW + b]);
          r[BK * CPW + 0] = fma(v[0][a], v[1][a], r[BK * CPW + 0]);
          r[BK * CPW + 1] = fma(v[0][a], v[2][a], r[BK * CPW + 1]);
          r[BK * CPW + 2] = fma(v[0][a], v[3][a], r[BK * CPW + 2]);
          r[BK * CPW + 3] = fma(v[1][a], v[2][a], r[BK * CPW + 3]);
          r[BK * CPW + 4] = fma(v[1][a], v[3][a], r[BK * CPW + 4]);
          r[BK * CPW + 5] = fma(v[2][a], v[3][a], r[BK * CPW + 5]);
        }
        wave::sums<NRP>(r);
        const double g01 = r[BK * CPW + 0], g02 = r[BK * CPW + 1], g03 = r[BK * CPW + 2];
        const double g12 = r[BK * CPW + 3], g13 = r[BK * CPW + 4], g23 = r[BK * CPW + 5];
        const double T00 = tq[0], T11 = tq[1], T22 = tq[2], T33 = tq[3];
        const double T01 = -tq[1] * (T00 * g01);
        const double T12 = -tq[2] * (T11 * g12);
        const double T02 = -tq[2] * fma(T00, g02, T01 * g12);
        const double T23 = -tq[3] * (T22 * g23);
        const double T13 = -tq[3] * fma(T11, g13, T12 * g23);
        const double T03 = -tq[3] * fma(T00, g03, fma(T01, g13, T02 * g23));
#pragma unroll
        for (int b = 0; b < CPW; ++b) {
          const double w0 = r[0 * CPW + b], w1 = r[1 * CPW + b];
          const double w2 = r[2 * CPW + b], w3 = r[3 * CPW + b];
          double u0, u1, u2, u3;
          if (trans) {
            u0 = T00 * w0;
            u1 = fma(T01, w0, T11 * w1);
            u2 = fma(T02, w0, fma(T12, w1, T22 * w2));
            u3 = fma(T03, w0, fma(T13, w1, fma(T23, w2, T33 * w3)));
          } else {
            u0 = fma(T00, w0, fma(T01, w1, fma(T02, w2, T03 * w3)));
            u1 = fma(T11, w1, fma(T12, w2, T13 * w3));
            u2 = fma(T22, w2, T23 * w3);
            u3 = T33 * w3;
          }
#pragma unroll
          for (int a = 0; a < RPL; ++a)
            y[a][b] -= fma(v[0][a], u0, fma(v[1][a], u1, fma(v[2][a], u2, v[3][a] * u3)));
        }
      }
    }
  } else if constexpr (RPL <= 16) {
    // reflectors in flight: a ring of PF register slots, slot q holding the
    // reflector of step s0 + q and refilled with that of step s0 + q + PF as
    // soon as it is consumed, so each load has PF steps to arrive.  The loads
    // are unconditional (rows past m read row m - 1, steps past k the last
    // reflector) so that no branch makes the compiler wait for all of them;
    // rows past m are zeroed when a reflector is used.
    constexpr int PF = RPL <= 2 ? 8 : (RPL <= 4 ? 4 : 2);
    auto roff = [&](int a) { return (long)min(l + 64 * a, m - 1); };
    double ring[PF][RPL];
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int sq = min(q, k - 1);
      const long j = trans ? sq : k - 1 - sq;
#pragma unroll
      for (int a = 0; a < RPL; ++a) ring[q][a] = V[j * m + roff(a)];
    }
    for (int s0 = 0; s0 < k; s0 += PF) {
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int s = s0 + q;
        if (s >= k) break;  // uniform
        double v[RPL];
#pragma unroll
        for (int a = 0; a < RPL; ++a) v[a] = (l + 64 * a < m) ? ring[q][a] : 0.0;
        {
          const int sn = min(s + PF, k - 1);
          const long jn = trans ? sn : k - 1 - sn;
#pragma unroll
          for (int a = 0; a < RPL; ++a) ring[q][a] = V[jn * m + roff(a)];
        }
        const int j = trans ? s : k - 1 - s;
        const double tj = wave::read_lane(j < 64 ? ta : tb, j & 63);
        if (tj == 0.0) continue;
        double d[CPW];
#pragma unroll
        for (int b = 0; b < CPW; ++b) {
          double acc = 0.0;
#pragma unroll
          for (int a = 0; a < RPL; ++a) acc = fma(v[a], y[a][b], acc);
          d[b] = acc;
        }
        wave::sums<CPW>(d);
#pragma unroll
        for (int b = 0; b < CPW; ++b) {
          const double f = tj * d[b];
#pragma unroll
          for (int a = 0; a < RPL; ++a) y[a][b] = fma(-v[a], f, y[a][b]);
        }
      }
    }
  } else {
    // many rows per lane: one reflector ahead (the registers hold no more)
    double vn[RPL];
    {
      const int j = trans ? 0 : k - 1;
#pragma unroll
      for (int a = 0; a < RPL; ++a) {
        const int i = l + 64 * a;
        vn[a] = (i < m) ? V[(long)j * m + i] : 0.0;
      }
    }
    for (int s = 0; s < k; ++s) {
      const int j = trans ? s : k - 1 - s;
      double v[RPL];
#pragma unroll
      for (int a = 0; a < RPL; ++a) v[a] = vn[a];
      if (s + 1 < k) {
        const int jn = trans ? s + 1 : k - 2 - s;
#pragma unroll
        for (int a = 0; a < RPL; ++a) {
          const int i = l + 64 * a;
          vn[a] = (i < m) ? V[(long)jn * m + i] : 0.0;
        }
      }
      const double tj = wave::read_lane(j < 64 ? ta : tb, j & 63);
      if (tj == 0.0) continue;
      double d[CPW];
#pragma unroll
      for (int b = 0; b < CPW; ++b) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < RPL; ++a) acc = fma(v[a], y[a][b], acc);
        d[b] = acc;
      }
      wave::sums<CPW>(d);
#pragma unroll
      for (int b = 0; b < CPW; ++b) {
        const double f = tj * d[b];
#pragma unroll
        for (int a = 0; a < RPL; ++a) y[a][b] = fma(-v[a], f, y[a][b]);
      }
    }
  }
#pragma unroll
  for (int a = 0; a < RPL; ++a)
#pragma unroll
    for (int b = 0; b < CPW; ++b) {
      const int i = l + 64 * a;
      if (i < m && c0 + b < p) Yout.p[(long)i * Yout.rs + (long)(c0 + b) * Yout.cs] = y[a][b];
    }
}

// Reflector application with the reflectors shared by the waves of a
// workgroup through LDS (rows of 257 to 2048, one reflector at a time).
// Blocks of RB reflectors are loaded once per workgroup, coalesced, into one
// of two LDS buffers while the other is applied; each of the LT / 64 waves
// carries CPW columns and reads every reflector from LDS instead of
// streaming its own copy from L2.  Column by column the arithmetic is that
// of qr_reg_apply_kernel's one-reflector path (the same products in the same
// order, the same cross-lane sums), so the two kernels give the same bits.
// Every wave takes part in the loads and barriers, also one whose columns
// lie past p.
//
// With STAGE the block of Y the workgroup owns (its LT / 64 * CPW adjacent
// columns) also moves through LDS, RC rows at a time: loaded row by row,
// coalesced, and handed to the waves column by column (and back the same way
// at the end).  A row-major Y read column by column, one column per wave,
// touches a different cache line in every lane; staged, each row of the
// block is one contiguous read.
constexpr int LT = 512;  // 8 waves
constexpr int RC = 512;  // rows of Y per staging pass

template <int RPL>
constexpr int lds_block() { return RPL >= 16 ? 4 : 8; }

template <int CPW, int RPL, bool STAGE>
constexpr size_t lds_apply_bytes() {
  const size_t refl = (size_t)2 * lds_block<RPL>() * 64 * RPL;
  const size_t stage = STAGE ? (size_t)RC * ((LT / 64) * CPW + 1) : 0;
  return (refl > stage ? refl : stage) * sizeof(double);
}

template <int CPW, int RPL, bool STAGE>
__global__ __launch_bounds__(LT) void qr_lds_apply_kernel(
    const double* __restrict__ V, const double* __restrict__ tau, int m, int k,
    CMatView Yin, int rows_in, MatView Yout, int p, int trans, Chunks ch,
    InstOff io) {
  constexpr int R = 64 * RPL;             // rows of one reflector slot
  constexpr int RB = lds_block<RPL>();    // reflectors per block
  constexpr int PER = RB * R / LT;        // values each thread stages per block
  static_assert(RB * R % LT == 0, "block must divide over the workgroup");
  extern __shared__ double vs[];          // [2][RB][R]
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  {
    const long o_ = io.of(blockIdx.z);
    V = shifted(V, o_);
    tau = shifted(tau, o_);
    Yin = shifted(Yin, o_);
    Yout = shifted(Yout, o_);
  }
  {
    const int cb = blockIdx.y;
    const int row0 = cb * ch.rows;
    const int mc = min(ch.rows, m - row0);
    V += (long)cb * ch.rows * ch.kstride;
    tau += (long)cb * ch.kstride;
    k = min(k, mc);
    rows_in = min(rows_in - row0, mc);
    m = mc;
    Yin.p += (long)row0 * Yin.rs;
    Yout.p += (long)row0 * Yout.rs;
  }
  const int c0 = (blockIdx.x * (LT / 64) + w) * CPW;
  const bool active = c0 < p;
  // the workgroup's columns and the row pitch of a staging pass
  constexpr int NC = (LT / 64) * CPW;
  constexpr int LDY = NC + 1;
  const int cw = blockIdx.x * NC;
  double y[RPL][CPW];
  if constexpr (STAGE) {
#pragma unroll
    for (int r0 = 0; r0 < 64 * RPL; r0 += RC) {
      for (int e = tid; e < RC * NC; e += LT) {
        const int rr = e / NC, cc = e % NC;
        const int i = r0 + rr, c = cw + cc;
        vs[rr * LDY + cc] = (i < rows_in && c < p)
                                ? Yin.p[(long)i * Yin.rs + (long)c * Yin.cs] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int a = 0; a < RPL; ++a)
        if (64 * a >= r0 && 64 * a < r0 + RC)
#pragma unroll
          for (int b = 0; b < CPW; ++b)
            y[a][b] = vs[(l + 64 * a - r0) * LDY + w * CPW + b];
      __syncthreads();
    }
  } else {
#pragma unroll
    for (int a = 0; a < RPL; ++a)
#pragma unroll
      for (int b = 0; b < CPW; ++b) {
        const int i = l + 64 * a;
        y[a][b] = (active && i < rows_in && c0 + b < p)
                      ? Yin.p[(long)i * Yin.rs + (long)(c0 + b) * Yin.cs] : 0.0;
      }
  }
  const double ta = (l < k) ? tau[l] : 0.0;
  const double tb = (l + 64 < k) ? tau[l + 64] : 0.0;
  const int nb = (k + RB - 1) / RB;
  double st[PER];
  // element e of block t: reflector step t * RB + e / R, row e % R (rows
  // past m and steps past k stage zeros)
  auto fetch = [&](int t) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + q * LT;
      const int r = e % R;
      const int sidx = t * RB + e / R;
      const long j = trans ? sidx : k - 1 - sidx;
      st[q] = (sidx < k && r < m) ? V[j * m + r] : 0.0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < PER; ++q) vs[(long)buf * RB * R + tid + q * LT] = st[q];
  };
  fetch(0);
  stash(0);
  __syncthreads();
  for (int t = 0; t < nb; ++t) {
    const int buf = t & 1;
    if (t + 1 < nb) fetch(t + 1);
    if (active) {
      for (int i = 0; i < RB; ++i) {
        const int sidx = t * RB + i;
        if (sidx >= k) break;  // uniform
        const int j = trans ? sidx : k - 1 - sidx;
        const double tj = wave::read_lane(j < 64 ? ta : tb, j & 63);
        if (tj == 0.0) continue;
        const double* vp = vs + ((long)buf * RB + i) * R + l;
        double v[RPL];
#pragma unroll
        for (int a = 0; a < RPL; ++a) v[a] = vp[64 * a];
        double d[CPW];
#pragma unroll
        for (int b = 0; b < CPW; ++b) {
          double acc = 0.0;
#pragma unroll
          for (int a = 0; a < RPL; ++a) acc = fma(v[a], y[a][b], acc);
          d[b] = acc;
        }
        wave::sums<CPW>(d);
#pragma unroll
        for (int b = 0; b < CPW; ++b) {
          const double f = tj * d[b];
#pragma unroll
          for (int a = 0; a < RPL; ++a) y[a][b] = fma(-v[a], f, y[a][b]);
        }
      }
    }
    // buffer buf ^ 1 was last read before the previous barrier
    if (t + 1 < nb) stash(buf ^ 1);
    __syncthreads();
  }
  if constexpr (STAGE) {
    // the last barrier above ends every read of the reflector buffers
#pragma unroll
    for (int r0 = 0; r0 < 64 * RPL; r0 += RC) {
#pragma unroll
      for (int a = 0; a < RPL; ++a)
        if (64 * a >= r0 && 64 * a < r0 + RC)
#pragma unroll
          for (int b = 0; b < CPW; ++b)
            vs[(l + 64 * a - r0) * LDY + w * CPW + b] = y[a][b];
      __syncthreads();
      for (int e = tid; e < RC * NC; e += LT) {
        const int rr = e / NC, cc = e % NC;
        const int i = r0 + rr, c = cw + cc;
        if (i < m && c < p) Yout.p[(long)i * Yout.rs + (long)c * Yout.cs] = vs[rr * LDY + cc];
      }
      __syncthreads();
    }
    return;
  }
  if (!active) return;
#pragma unroll
  for (int a = 0; a < RPL; ++a)
#pragma unroll
    for (int b = 0; b < CPW; ++b) {
      const int i = l + 64 * a;
      if (i < m && c0 + b < p) Yout.p[(long)i * Yout.rs + (long)(c0 + b) * Yout.cs] = y[a][b];
    }
}

// Application of up to 16 reflectors in compact-WY form on the matrix
// cores, for tall blocks (the trailing updates of 16-column panels):
//   Q = H_0 ... H_{k-1} = I - V T V^T,  T upper triangular (k x k),
//   T_jj = tau_j,  T_{<j,j} = -tau_j T_{<j,<j} (V_{<j}^T v_j),
// Q^T Y = Y - V T^T (V^T Y),  Q Y = Y - V T (V^T Y).
// A workgroup of four waves owns 64 columns of Y (16 per wave) and streams
// the rows twice, 128 at a time, the reflectors through LDS (loaded
// coalesced along each reflector), Y straight from memory (16 adjacent
// columns per row, the loads of 32 rows issued before the matrix-core steps
// that use them).  Pass 1 accumulates W = V^T Y and the Gram matrix V^T V
// with v_mfma_f64_16x16x4f64; wave 0 forms T from the Gram matrix and tau
// (one lane per row of T) and every wave W' = T^T W (or T W); pass 2
// subtracts V W' (four matrix-core steps per 16 rows).  Small register and
// LDS footprints keep four workgroups on a compute unit.  It reads each element of Y twice
// and writes it once, whatever k, and fills the chip when many lock-step
// instances share the launch; one state alone does better with the
// one-reflector-at-a-time kernels (more workgroups, shorter chains), so the
// problem chooses (mps_problem.tall_apply) and the choice never depends on
// the instance count.
constexpr int WY_T = 256;     // 4 waves
constexpr int WY_RC = 128;    // rows per chunk
constexpr int WY_LD = 17;     // LDS pitch of a 16-wide row

__global__ __launch_bounds__(WY_T) void qr_wy_apply_kernel(
    const double* __restrict__ V, const double* __restrict__ tau, int m, int k,
    CMatView Yin, int rows_in, MatView Yout, int p, int trans, Chunks ch,
    InstOff io) {
  __shared__ double Vs[WY_RC * WY_LD];
  __shared__ double Gs[16 * WY_LD];     // the Gram matrix V^T V (from wave 0)
  __shared__ double Ts[16 * WY_LD];     // T
  __shared__ double Wsh[4][16 * WY_LD]; // per wave: its block of V^T Y
  {
    const long o_ = io.of(blockIdx.z);
    V = shifted(V, o_);
    tau = shifted(tau, o_);
    Yin = shifted(Yin, o_);
    Yout = shifted(Yout, o_);
  }
  {
    const int cb = blockIdx.y;
    const int row0 = cb * ch.rows;
    const int mc = min(ch.rows, m - row0);
    V += (long)cb * ch.rows * ch.kstride;
    tau += (long)cb * ch.kstride;
    k = min(k, mc);
    rows_in = min(rows_in - row0, mc);
    m = mc;
    Yin.p += (long)row0 * Yin.rs;
    Yout.p += (long)row0 * Yout.rs;
  }
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int lr = l & 15, lk = l >> 4;
  const int col = blockIdx.x * 64 + w * 16 + lr;  // this lane's column (B and D)
  const bool colok = col < p;
  double* Wl = Wsh[w];
  // stage reflector rows [i0, i0 + WY_RC) (zeros past m and past k)
  // (all eight loads of a thread issued before the first store)
  auto stage = [&](int i0) {
    double v[WY_RC * 16 / WY_T];
#pragma unroll
    for (int it = 0; it < WY_RC * 16 / WY_T; ++it) {
      const int e = tid + it * WY_T;
      const int j = e / WY_RC, r = e % WY_RC;
      const int i = i0 + r;
      const bool ok = j < k && i < m;
      const double x = V[ok ? (long)j * m + i : 0];
      v[it] = ok ? x : 0.0;
    }
#pragma unroll
    for (int it = 0; it < WY_RC * 16 / WY_T; ++it) {
      const int e = tid + it * WY_T;
      Vs[(e % WY_RC) * WY_LD + e / WY_RC] = v[it];
    }
  };
  dbl4 accW = {0.0, 0.0, 0.0, 0.0}, accG = {0.0, 0.0, 0.0, 0.0};
  for (int i0 = 0; i0 < m; i0 += WY_RC) {
    __syncthreads();
    stage(i0);
    __syncthreads();
    const int nrow = min(WY_RC, m - i0);
    // 32 rows per group: the 8 loads of Y are issued before the 16
    // matrix-core steps that use them (rows past m load and stage zeros)
    for (int r32 = 0; r32 < nrow; r32 += 32) {
      double bb[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int i = i0 + r32 + 4 * q + lk;
        const bool ok = colok && i < rows_in;
        const double y = Yin.p[ok ? (long)i * Yin.rs + (long)col * Yin.cs : 0];
        bb[q] = ok ? y : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        // A = V^T (row j = lr, k index = chunk row); B = Y rows (k, col)
        const double a = Vs[(r32 + 4 * q + lk) * WY_LD + lr];
        accW = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb[q], accW, 0, 0, 0);
        // the Gram matrix: B = V rows, the same element as A
        accG = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, accG, 0, 0, 0);
      }
    }
  }
  // D layout: lane l, item r -> row 4 r + lk, column lr (every wave has the
  // same Gram matrix; wave 0's is kept)
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (w == 0) Gs[(4 * r + lk) * WY_LD + lr] = accG[r];
    Wl[(4 * r + lk) * WY_LD + lr] = accW[r];
  }
  __syncthreads();
  // T by wave 0, one lane per row, column after column; each lane reads
  // back only the entries of its own row
  if (w == 0 && l < 16) {
    const int row = l;
    for (int c = 0; c < 16; ++c) {
      const double tc = (c < k) ? tau[c] : 0.0;
      double v = 0.0;
      if (row == c) {
        v = tc;
      } else if (row < c) {
        double acc = 0.0;
        for (int q = row; q < c; ++q) acc = fma(Ts[row * WY_LD + q], Gs[q * WY_LD + c], acc);
        v = -tc * acc;
      }
      Ts[row * WY_LD + c] = v;
    }
  }
  __syncthreads();
  // W' = T^T W (trans) or T W, as the B operand of pass 2:
  // step s takes W'[4 s + lk][lr]
  double bw[4];
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) {
    const int row = 4 * s4 + lk;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const double tq = trans ? Ts[q * WY_LD + row] : Ts[row * WY_LD + q];
      acc = fma(tq, Wl[q * WY_LD + lr], acc);
    }
    bw[s4] = acc;
  }
  // pass 2: Y -= V W', two tiles of 16 rows per group of 32
  for (int i0 = 0; i0 < m; i0 += WY_RC) {
    __syncthreads();
    stage(i0);
    __syncthreads();
    const int nrow = min(WY_RC, m - i0);
    for (int r32 = 0; r32 < nrow; r32 += 32) {
      double yy[2][4];
#pragma unroll
      for (int tt = 0; tt < 2; ++tt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + r32 + 16 * tt + 4 * r + lk;
          const bool ok = colok && i < rows_in;
          const double y = Yin.p[ok ? (long)i * Yin.rs + (long)col * Yin.cs : 0];
          yy[tt][r] = ok ? y : 0.0;
        }
#pragma unroll
      for (int tt = 0; tt < 2; ++tt) {
        dbl4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          // A[row][kk] = V[chunk row r32 + 16 tt + lr][4 s + lk]
          const double a = Vs[(r32 + 16 * tt + lr) * WY_LD + 4 * s4 + lk];
          d = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bw[s4], d, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + r32 + 16 * tt + 4 * r + lk;
          if (colok && i < m) Yout.p[(long)i * Yout.rs + (long)col * Yout.cs] = yy[tt][r] - d[r];
        }
      }
    }
  }
}

// Groups of up to four 16-column panels of a tall block applied as one
// compact-WY block, Q_g = H_0 ... H_{k-1} = I - V T V^T (k <= 64), in the
// compact-WY mode: the trailing columns of the block are read and written
// once per 64 reflectors instead of once per 16.  The group's reflectors
// are kept panel after panel: panel t (reflectors 16 t .. 16 t + 15,
// starting at row 16 t of the group's m rows) column-major over its own
// m - 16 t rows, unit diagonal and zeros above, at offset
// group_voff(m, t); the rows above 16 t are zero and are not stored.
constexpr int WG_T = 256;   // 4 waves
constexpr int WG_RC = 64;   // rows per staged chunk
constexpr int WG_P1 = 72;   // LDS pitch of V read along the reflectors
constexpr int WG_P2 = 68;   // LDS pitch of V read down the rows

__host__ __device__ inline long group_voff(int m, int t) {
  return 16L * ((long)t * m - 8L * t * (t - 1));
}

// Rows [i0, i0 + WG_RC) of the group's m x 64 reflector matrix, as 16
// values per thread (zeros past m, above each panel's first row and past
// k): thread tid takes reflector 16 t + (tid >> 4) of panel t = it & 3 and
// row 16 (it >> 2) + (tid & 15), so a wave reads 16 consecutive rows of 4
// reflectors (128 bytes each).  All 16 loads are issued before any is
// used; group_store puts them into LDS (pitch P) once they have arrived.
__device__ inline void group_load(double (&v)[16], const double* __restrict__ V, int m,
                                  int k, int i0, int tid) {
  const int rl = tid & 15, jj = tid >> 4;
#pragma unroll
  for (int it = 0; it < 16; ++it) {
    const int t = it & 3, j = 16 * t + jj;
    const int i = i0 + 16 * (it >> 2) + rl;
    // every lane loads (element 0 where the value is zero), so no branch
    // separates the loads
    const bool ok = j < k && i < m && i >= 16 * t;
    const long idx = ok ? group_voff(m, t) + (long)jj * (m - 16 * t) + (i - 16 * t) : 0;
    const double x = V[idx];
    v[it] = ok ? x : 0.0;
  }
}

template <int P>
__device__ inline void group_store(double* Vs, const double (&v)[16], int tid) {
  const int rl = tid & 15, jj = tid >> 4;
#pragma unroll
  for (int it = 0; it < 16; ++it) Vs[(16 * (it >> 2) + rl) * P + 16 * (it & 3) + jj] = v[it];
}

// T of one group (one workgroup per instance).  The Gram matrix G = V^T V
// on the matrix cores: its ten blocks of the upper block triangle, each
// wave taking 16 rows of every staged chunk (two chunks of reflector rows
// in flight), the four partial sums added through LDS.  Then T by blocks
// of 16: the diagonal blocks T_bb by the recurrence T_jj = tau_j,
// T_{<j,j} = -tau_j T_{<j,<j} (V_{<j}^T v_j) within the block (one wave
// per block, one lane per row; a lane reads only its own row), and block
// column J from the ones before it, T_{<J,J} = -T_{<J,<J} G_{<J,J} T_JJ
// (the product of the first J blocks' reflectors with block J's), on the
// matrix cores.  T is written whole (64 x 64, row-major, zeros below the
// diagonal and past k).
__global__ __launch_bounds__(WG_T) void qr_wy_group_t_kernel(
    const double* __restrict__ V, const double* __restrict__ tau, int m, int k,
    double* __restrict__ T, InstOff io) {
  __shared__ double Vs[WG_RC * WG_P1];  // staged reflector rows, later T (pitch 65)
  __shared__ double Gs[64 * 65];
  __shared__ double Ys[4][16 * 17];
  {
    const long o_ = io.of(blockIdx.z);
    V = shifted(V, o_);
    tau = shifted(tau, o_);
    T = shifted(T, o_);
  }
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int lr = l & 15, lk = l >> 4;
  // the ten blocks (a, b), a <= b, of the upper block triangle (V is zero
  // past k, and so are those blocks)
  dbl4 acc[10];
#pragma unroll
  for (int x = 0; x < 10; ++x) acc[x] = dbl4{0.0, 0.0, 0.0, 0.0};
  auto gram_chunk = [&]() {
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4) {
      const double* row = Vs + (16 * w + 4 * q4 + lk) * WG_P1 + lr;
      double a[4];
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) a[bb] = row[16 * bb];
      int x = 0;
#pragma unroll
      for (int a0 = 0; a0 < 4; ++a0)
#pragma unroll
        for (int bb = a0; bb < 4; ++bb, ++x)
          acc[x] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[a0], a[bb], acc[x], 0, 0, 0);
    }
  };
  double va[16], vb[16];
  group_load(va, V, m, k, 0, tid);
  if (WG_RC < m) group_load(vb, V, m, k, WG_RC, tid);
  for (int i0 = 0; i0 < m; i0 += 2 * WG_RC) {
    __syncthreads();
    group_store<WG_P1>(Vs, va, tid);
    __syncthreads();
    if (i0 + 2 * WG_RC < m) group_load(va, V, m, k, i0 + 2 * WG_RC, tid);
    gram_chunk();
    if (i0 + WG_RC < m) {
      __syncthreads();
      group_store<WG_P1>(Vs, vb, tid);
      __syncthreads();
      if (i0 + 3 * WG_RC < m) group_load(vb, V, m, k, i0 + 3 * WG_RC, tid);
      gram_chunk();
    }
  }
  // D layout: item r of lane (lk, lr) is row 4 r + lk, column lr of a
  // block; the waves' partial sums are added in turn
  for (int ww = 0; ww < 4; ++ww) {
    if (w == ww) {
      int x = 0;
#pragma unroll
      for (int a0 = 0; a0 < 4; ++a0)
#pragma unroll
        for (int bb = a0; bb < 4; ++bb, ++x)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            double* g = &Gs[(16 * a0 + 4 * r + lk) * 65 + 16 * bb + lr];
            *g = (ww == 0 ? 0.0 : *g) + acc[x][r];
          }
    }
    __syncthreads();
  }
  double* Ts = Vs;  // pitch 65
  for (int e = tid; e < 64 * 64; e += WG_T) Ts[(e >> 6) * 65 + (e & 63)] = 0.0;
  __syncthreads();
  // diagonal blocks: wave w takes block w, lane lr its row
  if (lk == 0) {
    const int b0 = 16 * w, row = b0 + lr;
    for (int c = 0; c < 16; ++c) {
      const int j = b0 + c;
      const double tc = (j < k) ? tau[j] : 0.0;
      double v = 0.0;
      if (lr == c) {
        v = tc;
      } else if (lr < c && j < k) {
        double a0 = 0.0, a1 = 0.0;
        int q = row;
        for (; q + 1 < j; q += 2) {
          a0 = fma(Ts[row * 65 + q], Gs[q * 65 + j], a0);
          a1 = fma(Ts[row * 65 + q + 1], Gs[(q + 1) * 65 + j], a1);
        }
        if (q < j) a0 = fma(Ts[row * 65 + q], Gs[q * 65 + j], a0);
        v = -tc * (a0 + a1);
      }
      Ts[row * 65 + j] = v;
    }
  }
  __syncthreads();
  // block columns: wave i < J forms T_iJ = -(sum_{l=i}^{J-1} T_il G_lJ) T_JJ
  for (int J = 1; J < 4; ++J) {
    if (w < J) {
      dbl4 y = {0.0, 0.0, 0.0, 0.0};
      for (int lb = w; lb < J; ++lb)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
          y = __builtin_amdgcn_mfma_f64_16x16x4f64(
              Ts[(16 * w + lr) * 65 + 16 * lb + 4 * s4 + lk],
              Gs[(16 * lb + 4 * s4 + lk) * 65 + 16 * J + lr], y, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) Ys[w][(4 * r + lk) * 17 + lr] = y[r];
    }
    __syncthreads();
    if (w < J) {
      dbl4 t = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
        t = __builtin_amdgcn_mfma_f64_16x16x4f64(
            Ys[w][lr * 17 + 4 * s4 + lk], Ts[(16 * J + 4 * s4 + lk) * 65 + 16 * J + lr], t, 0,
            0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) Ts[(16 * w + 4 * r + lk) * 65 + 16 * J + lr] = -t[r];
    }
    __syncthreads();
  }
  for (int e = tid; e < 64 * 64; e += WG_T) T[e] = Ts[(e >> 6) * 65 + (e & 63)];
}

// Yout <- Q_g^T Yin (trans) or Q_g Yin = Yin - V T' (V^T Yin), T' = T^T or
// T.  A workgroup of four waves owns 64 columns (16 per wave) and streams
// the rows twice, 64 at a time, the reflectors staged through LDS with a
// row pitch chosen for each pass's reads (two lanes per bank pair, the
// least 64 lanes of doubles allow); the next chunk's rows of
// Y and of the reflectors are loaded while the current chunk is on the
// matrix cores.  Pass 1 accumulates W = V^T Y (64 x 16 per wave, four
// 16 x 16 blocks); T' W comes from T staged through LDS with the blocks of
// W as B operands; pass 2 subtracts V (T' W) sixteen rows at a time.
__global__ __launch_bounds__(WG_T) void qr_wy_group_apply_kernel(
    const double* __restrict__ V, const double* __restrict__ T, int m, int k,
    CMatView Yin, int rows_in, MatView Yout, int p, int trans, InstOff io) {
  __shared__ double Vs[WG_RC * WG_P1];
  {
    const long o_ = io.of(blockIdx.z);
    V = shifted(V, o_);
    T = shifted(T, o_);
    Yin = shifted(Yin, o_);
    Yout = shifted(Yout, o_);
  }
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int lr = l & 15, lk = l >> 4;
  const int col = blockIdx.x * 64 + w * 16 + lr;
  const bool colok = col < p;
  const double* yin = Yin.p + (long)(colok ? col : 0) * Yin.cs;
  double* yout = Yout.p + (long)(colok ? col : 0) * Yout.cs;
  // pass 1: element e of a chunk's Y registers is row 4 e + lk
  // (loads of rows and columns outside Y read its element (0, 0) and are
  // replaced by zeros: no branch between the loads)
  auto load_y1 = [&](double (&y)[16], int i0) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int i = i0 + 4 * e + lk;
      const bool ok = colok && i < rows_in;
      const double x = yin[(long)(ok ? i : 0) * Yin.rs];
      y[e] = ok ? x : 0.0;
    }
  };
  dbl4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = dbl4{0.0, 0.0, 0.0, 0.0};
  double vn[16], yn[16];
  group_load(vn, V, m, k, 0, tid);
  load_y1(yn, 0);
  for (int i0 = 0; i0 < m; i0 += WG_RC) {
    double bb[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) bb[e] = yn[e];
    __syncthreads();
    group_store<WG_P1>(Vs, vn, tid);
    __syncthreads();
    if (i0 + WG_RC < m) {
      group_load(vn, V, m, k, i0 + WG_RC, tid);
      load_y1(yn, i0 + WG_RC);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const double* row = Vs + (4 * q + lk) * WG_P1 + lr;
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(row[16 * b], bb[q], acc[b], 0, 0, 0);
      // at most four steps' LDS operands in flight (register budget)
      if ((q & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
  }
  // T' W: block bo of the result takes the blocks bi of W on T's nonzero
  // side (bi <= bo for T^T, bi >= bo for T); the B operand of step s of
  // block bi is item s of acc[bi]
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += WG_T) Vs[(e >> 6) * 65 + (e & 63)] = T[e];
  // the first chunk of pass 2 in flight meanwhile
  auto load_y2 = [&](double (&y)[16], int i0) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int i = i0 + 16 * (e >> 2) + 4 * (e & 3) + lk;
      const bool ok = colok && i < rows_in;
      const double x = yin[(long)(ok ? i : 0) * Yin.rs];
      y[e] = ok ? x : 0.0;
    }
  };
  group_load(vn, V, m, k, 0, tid);
  load_y2(yn, 0);
  __syncthreads();
  dbl4 wp[4];
#pragma unroll
  for (int bo = 0; bo < 4; ++bo) {
    wp[bo] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
      if (trans ? bi <= bo : bi >= bo) {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int jr = 16 * bo + lr, kq = 16 * bi + 4 * s4 + lk;
          const double a = trans ? Vs[kq * 65 + jr] : Vs[jr * 65 + kq];
          wp[bo] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, acc[bi][s4], wp[bo], 0, 0, 0);
        }
      }
    }
  }
  // pass 2: Y -= V (T' W); step u of a 16-row tile takes reflectors
  // 4 u .. 4 u + 3, its B operand item u & 3 of wp[u >> 2]; element e of a
  // chunk's Y registers is row 16 (e >> 2) + 4 (e & 3) + lk
  for (int i0 = 0; i0 < m; i0 += WG_RC) {
    double yy[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) yy[e] = yn[e];
    __syncthreads();
    group_store<WG_P2>(Vs, vn, tid);
    __syncthreads();
    if (i0 + WG_RC < m) {
      group_load(vn, V, m, k, i0 + WG_RC, tid);
      load_y2(yn, i0 + WG_RC);
    }
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
      if (i0 + 16 * tt < m) {
        dbl4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 0; u < 16; ++u)
          d = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[(16 * tt + lr) * WG_P2 + 4 * u + lk],
                                                   wp[u >> 2][u & 3], d, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + 16 * tt + 4 * r + lk;
          if (colok && i < m) yout[(long)i * Yout.rs] = yy[4 * tt + r] - d[r];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

int rows_per_lane(int m) {
  int r = 1;
  while (64 * r < m) r *= 2;
  return r;
}

int cols_per_wave(int n) {
  int c = 1;
  while (16 * c < n) c *= 2;
  return c;
}

template <int CPW, int RPL>
void launch_factor(hipStream_t s, CMatView A, int m, int n, MatView R,
                   double* V, double* tau, Chunks ch, int nchunks) {
  hipLaunchKernelGGL((qr_reg_factor_kernel<CPW, RPL>), dim3(1, nchunks, inst_count()),
                     dim3(FT), 0, s, A, m, n, R, V, tau, ch, inst_off());
}

template <int CPW, int RPL>
void launch_apply(hipStream_t s, const double* V, const double* tau, int m,
                  int k, CMatView Yin, int rows_in, MatView Yout, int p,
                  int trans, Chunks ch, int nchunks) {
  const int per_block = (AT / 64) * CPW;
  hipLaunchKernelGGL((qr_reg_apply_kernel<CPW, RPL>),
                     dim3(ceil_div(p, per_block), nchunks, inst_count()), dim3(AT), 0, s,
                     V, tau, m, k, Yin, rows_in, Yout, p, trans, ch, inst_off());
}

template <int CPW, int RPL, bool STAGE>
void launch_lds_apply(hipStream_t s, const double* V, const double* tau, int m,
                      int k, CMatView Yin, int rows_in, MatView Yout, int p,
                      int trans, Chunks ch, int nchunks) {
  static std::once_flag once;
  std::call_once(once, [] {
    MPSV_HIP(hipFuncSetAttribute((const void*)qr_lds_apply_kernel<CPW, RPL, STAGE>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds_apply_bytes<CPW, RPL, STAGE>()));
  });
  const int per_block = (LT / 64) * CPW;
  const size_t lds = lds_apply_bytes<CPW, RPL, STAGE>();
  hipLaunchKernelGGL((qr_lds_apply_kernel<CPW, RPL, STAGE>),
                     dim3(ceil_div(p, per_block), nchunks, inst_count()), dim3(LT), lds, s,
                     V, tau, m, k, Yin, rows_in, Yout, p, trans, ch, inst_off());
}

}  // namespace

// The register budget of 16 waves per CU is 128 VGPRs: at most 32 matrix
// elements per lane, 16 when the rows need 16 per lane (the reflector and
// its prefetch take the rest), and one column of 32 rows per lane with the
// reflector read from LDS.
static int elems_per_lane(int rpl) { return rpl == 16 ? 16 : 32; }

bool qr_reg_fits(int m, int n) {
  if (m < 1 || n < 1 || m > 2048 || n > 128) return false;
  const int rpl = rows_per_lane(m), cpw = cols_per_wave(n);
  return rpl * cpw <= elems_per_lane(rpl);
}

int qr_reg_panel_cols(int m) {
  const int rpl = rows_per_lane(m);
  return 16 * std::min(8, elems_per_lane(rpl) / rpl);
}

void qr_reg_factor(hipStream_t s, CMatView A, int m, int n, MatView R,
                   double* V, double* tau) {
  MPSV_CHECK(qr_reg_fits(m, n), kEinval, "qr_reg_factor: shape does not fit");
  const int rpl = rows_per_lane(m), cpw = cols_per_wave(n);
  const int slot = prof_begin(s);
  // column-per-row layout where the rows fit (16 * RPT >= m, <= 32 values)
  int rpt = 2;
  while (16 * rpt < m) rpt *= 2;
  const int cpg = n <= 64 ? 1 : 2;
  // measured fastest per shape: column-per-row layout up to 64 rows,
  // eight-column wave panels up to 128 rows, wave-per-column layout above
  const bool g16 = m <= 64 && n <= 128;
  const bool blk = !g16 && m <= 128 && n <= 128;
#define MPSV_G(C, Rr)                                                   \
  if (g16 && cpg == C && rpt == Rr)                                     \
    hipLaunchKernelGGL((qr_g16_factor_kernel<C, Rr>), dim3(1, 1, inst_count()), \
                       dim3(FT), 0, s, A, m, n, R, V, tau, inst_off()); else
#define MPSV_F(C, Rr)                                                   \
  if (cpw == C && rpl == Rr) launch_factor<C, Rr>(s, A, m, n, R, V, tau, Chunks{m, n}, 1); else
  if (blk)
    hipLaunchKernelGGL((qr_blk_factor_kernel<2>), dim3(1, 1, inst_count()), dim3(FT), 0, s,
                       A, m, n, R, V, tau, inst_off());
  else
  MPSV_G(1, 2) MPSV_G(1, 4) MPSV_G(2, 2) MPSV_G(2, 4)
  MPSV_F(1, 1) MPSV_F(2, 1) MPSV_F(4, 1) MPSV_F(8, 1)
  MPSV_F(1, 2) MPSV_F(2, 2) MPSV_F(4, 2) MPSV_F(8, 2)
  MPSV_F(1, 4) MPSV_F(2, 4) MPSV_F(4, 4) MPSV_F(8, 4)
  MPSV_F(1, 8) MPSV_F(2, 8) MPSV_F(4, 8)
  MPSV_F(1, 16) MPSV_F(1, 32)
  throw Error(kEinval, "qr_reg_factor: no kernel for this shape");
#undef MPSV_F
#undef MPSV_G
  MPSV_LAUNCHED();
  const int k = m < n ? m : n;
  // nominal GEQRF flops, 2 m n^2 - 2 n^3 / 3 (n = k columns reduced) plus
  // the update of the n - k columns right of a wide block
  prof_end(s, slot, kClsQrPanel,
           2.0 * m * (double)k * k - 2.0 * k * (double)k * k / 3.0 +
               4.0 * (double)(n - k) * k * (m - k / 2.0),
           8.0 * (2.0 * m * n + (double)m * k));
}

// Variant of a reflector application: columns per wave (1, 2 or 4) of the
// register-streaming kernel, 8 + columns per wave (1, or 2 up to 1024 rows)
// of the kernel that shares the reflectors through LDS, or 16 + columns per
// wave of the same kernel with Y staged through LDS as well; the built-in
// rule, or the launch-shape table's choice for this shape and instance
// count.  Every
// choice gives the same bits: each column's products and reductions are
// the same whichever wave and kernel carry it.
// Reflector applications that take the compact-WY matrix-core kernel: when
// the problem asks for it (carried with the lanes of its launches), tall
// blocks (more than 512 rows per chunk), at most 16 reflectors, at least 32
// columns.  The choice depends on the problem and the shape, never on the
// number of lock-step instances.
static bool wy_shape(int rows, int k, int p) {
  return lanes().tall_apply == 1 && rows > 512 && k <= 16 && p >= 32;
}

static void launch_wy(hipStream_t s, const double* V, const double* tau, int m, int k,
                      CMatView Yin, int rows_in, MatView Yout, int p, int tr, Chunks ch,
                      int nchunks) {
  hipLaunchKernelGGL(qr_wy_apply_kernel, dim3(ceil_div(p, 64), nchunks, inst_count()),
                     dim3(WY_T), 0, s, V, tau, m, k, Yin, rows_in, Yout, p, tr, ch,
                     inst_off());
  MPSV_LAUNCHED();
}

static TunePick apply_cols(hipStream_t s, int rows, int k, int p, int nch, int tr, int rpl) {
  const int dflt = (p >= 128 && rpl < 32) ? 2 : 1;
  uint32_t allowed = 1u << 1;
  if (rpl < 32) allowed |= 1u << 2;
  if (rpl <= 8) allowed |= 1u << 4;
  // reflectors shared through LDS (values 8 + columns per wave), 257 to
  // 2048 rows
  if (rpl >= 8) allowed |= (1u << 9) | (1u << 17);
  if (rpl >= 8 && rpl < 32) allowed |= (1u << 10) | (1u << 18);
  const TuneKey key{{kTuneApplyCols, rows, k, p, 2 * nch + tr, tune_inst_class(inst_count())}};
  return tune_pick(s, key, dflt, allowed);
}

void qr_reg_apply(hipStream_t s, const double* V, const double* tau, int m,
                  int k, CMatView Yin, int rows_in, MatView Yout, int p,
                  bool trans) {
  if (p <= 0 || k <= 0) return;
  MPSV_CHECK(m >= 1 && m <= 2048 && k <= m && k <= 128, kEinval,
             "qr_reg_apply: bad shape");
  const int rpl = rows_per_lane(m);
  const int tr = trans ? 1 : 0;
  if (wy_shape(m, k, p)) {
    // (the kernel's out-of-range lanes load element (0, 0) of Yin)
    MPSV_CHECK(rows_in >= 1, kEinval, "qr_reg_apply: no input rows");
    const int slot = prof_begin(s);
    launch_wy(s, V, tau, m, k, Yin, rows_in, Yout, p, tr, Chunks{m, k}, 1);
    // algorithmic bytes: Y read twice and written once, the reflectors
    // read twice
    prof_end(s, slot, kClsQrWy, 4.0 * p * (double)k * (m - (k - 1) / 2.0),
             8.0 * (3.0 * m * p + 2.0 * (double)m * k));
    return;
  }
  const TunePick tp = apply_cols(s, m, k, p, 1, tr, rpl);
  const int cpw = tp.value;
  const int slot = prof_begin(s);
#define MPSV_A(C, Rr)                                                   \
  if (cpw == C && rpl == Rr) launch_apply<C, Rr>(s, V, tau, m, k, Yin, rows_in, Yout, p, tr, Chunks{m, k}, 1); else
#define MPSV_L(C, Rr)                                                   \
  if (cpw == 8 + C && rpl == Rr) launch_lds_apply<C, Rr, false>(s, V, tau, m, k, Yin, rows_in, Yout, p, tr, Chunks{m, k}, 1); else
#define MPSV_S(C, Rr)                                                   \
  if (cpw == 16 + C && rpl == Rr) launch_lds_apply<C, Rr, true>(s, V, tau, m, k, Yin, rows_in, Yout, p, tr, Chunks{m, k}, 1); else
  MPSV_A(1, 1) MPSV_A(2, 1) MPSV_A(4, 1) MPSV_A(1, 2) MPSV_A(2, 2) MPSV_A(4, 2)
  MPSV_A(1, 4) MPSV_A(2, 4) MPSV_A(4, 4) MPSV_A(1, 8) MPSV_A(2, 8) MPSV_A(4, 8)
  MPSV_A(1, 16) MPSV_A(2, 16) MPSV_A(1, 32)
  MPSV_L(1, 8) MPSV_L(2, 8) MPSV_L(1, 16) MPSV_L(2, 16) MPSV_L(1, 32)
  MPSV_S(1, 8) MPSV_S(2, 8) MPSV_S(1, 16) MPSV_S(2, 16) MPSV_S(1, 32)
  throw Error(kEinval, "qr_reg_apply: no kernel for this shape");
#undef MPSV_S
#undef MPSV_L
#undef MPSV_A
  MPSV_LAUNCHED();
  // k reflectors of decreasing length applied to p columns
  prof_end(s, slot, kClsQrApply, 4.0 * p * (double)k * (m - (k - 1) / 2.0),
           8.0 * (2.0 * m * p + (double)m * k));
  tune_end(s, tp.slot);
}

long qr_group_voff(int m, int t) { return group_voff(m, t); }

void qr_wy_group_t(hipStream_t s, const double* V, const double* tau, int m, int k,
                   double* T) {
  MPSV_CHECK(k >= 1 && k <= 64 && k <= m, kEinval, "qr_wy_group_t: bad shape");
  const int slot = prof_begin(s);
  hipLaunchKernelGGL(qr_wy_group_t_kernel, dim3(1, 1, inst_count()), dim3(WG_T), 0, s, V,
                     tau, m, k, T, inst_off());
  MPSV_LAUNCHED();
  // the Gram matrix's upper block triangle (10 of 16 blocks for four
  // panels) and the recurrence; V read once, T written
  const int np = (k + 15) / 16;
  prof_end(s, slot, kClsQrWy, 2.0 * m * 256.0 * np * (np + 1) / 2.0 + k * (double)k * k / 3.0,
           8.0 * ((double)m * k + 64.0 * 64.0));
}

void qr_wy_group_apply(hipStream_t s, const double* V, const double* T, int m, int k,
                       CMatView Yin, int rows_in, MatView Yout, int p, bool trans) {
  if (p <= 0 || k <= 0) return;
  MPSV_CHECK(k <= 64 && k <= m && rows_in >= 1, kEinval, "qr_wy_group_apply: bad shape");
  rows_in = std::min(rows_in, m);
  const int slot = prof_begin(s);
  hipLaunchKernelGGL(qr_wy_group_apply_kernel, dim3(ceil_div(p, 64), 1, inst_count()),
                     dim3(WG_T), 0, s, V, T, m, k, Yin, rows_in, Yout, p, trans ? 1 : 0,
                     inst_off());
  MPSV_LAUNCHED();
  // the two products with V (k reflectors of decreasing length) and T' W;
  // algorithmic bytes: Y read twice and written once, the reflectors read
  // twice
  prof_end(s, slot, kClsQrWy,
           4.0 * p * (double)k * (m - (k - 1) / 2.0) + 2.0 * (double)k * k * p,
           8.0 * (3.0 * m * p + 2.0 * (double)m * k));
}

void qr_reg_factor_chunks(hipStream_t s, CMatView A, int m, int n, int rows,
                          MatView S, double* V, double* tau) {
  const int nch = (m + rows - 1) / rows;
  MPSV_CHECK(rows >= n && rows <= 2048 && n <= qr_reg_panel_cols(rows) &&
                 qr_reg_fits(rows, n),
             kEinval, "qr_reg_factor_chunks: shape does not fit");
  const int rpl = rows_per_lane(rows), cpw = cols_per_wave(n);
  const int slot = prof_begin(s);
  const Chunks ch{rows, n};
#define MPSV_F(C, Rr)                                                   \
  if (cpw == C && rpl == Rr) launch_factor<C, Rr>(s, A, m, n, S, V, tau, ch, nch); else
  MPSV_F(1, 1) MPSV_F(2, 1) MPSV_F(4, 1) MPSV_F(8, 1)
  MPSV_F(1, 2) MPSV_F(2, 2) MPSV_F(4, 2) MPSV_F(8, 2)
  MPSV_F(1, 4) MPSV_F(2, 4) MPSV_F(4, 4) MPSV_F(8, 4)
  MPSV_F(1, 8) MPSV_F(2, 8) MPSV_F(4, 8)
  MPSV_F(1, 16) MPSV_F(1, 32)
  throw Error(kEinval, "qr_reg_factor_chunks: no kernel for this shape");
#undef MPSV_F
  MPSV_LAUNCHED();
  prof_end(s, slot, kClsQrPanel,
           2.0 * m * (double)n * n - 2.0 * nch * n * (double)n * n / 3.0,
           8.0 * 3.0 * m * n);
}

void qr_reg_apply_chunks(hipStream_t s, const double* V, const double* tau,
                         int m, int k, int rows, MatView Y, int p, bool trans) {
  if (p <= 0 || k <= 0) return;
  const int nch = (m + rows - 1) / rows;
  MPSV_CHECK(rows >= k && rows <= 2048 && k <= 128, kEinval,
             "qr_reg_apply_chunks: bad shape");
  const int rpl = rows_per_lane(rows);
  const int tr = trans ? 1 : 0;
  if (wy_shape(rows, k, p)) {
    const int slot = prof_begin(s);
    launch_wy(s, V, tau, m, k, CMatView{Y.p, Y.rs, Y.cs, 0}, m, Y, p, tr, Chunks{rows, k}, nch);
    prof_end(s, slot, kClsQrWy, 4.0 * p * (double)k * m,
             8.0 * (3.0 * m * p + 2.0 * (double)m * k));
    return;
  }
  const TunePick tp = apply_cols(s, rows, k, p, nch, tr, rpl);
  const int cpw = tp.value;
  const int slot = prof_begin(s);
  const Chunks ch{rows, k};
  const CMatView Yin{Y.p, Y.rs, Y.cs, 0};
#define MPSV_A(C, Rr)                                                   \
  if (cpw == C && rpl == Rr) launch_apply<C, Rr>(s, V, tau, m, k, Yin, m, Y, p, tr, ch, nch); else
#define MPSV_L(C, Rr)                                                   \
  if (cpw == 8 + C && rpl == Rr) launch_lds_apply<C, Rr, false>(s, V, tau, m, k, Yin, m, Y, p, tr, ch, nch); else
#define MPSV_S(C, Rr)                                                   \
  if (cpw == 16 + C && rpl == Rr) launch_lds_apply<C, Rr, true>(s, V, tau, m, k, Yin, m, Y, p, tr, ch, nch); else
  MPSV_A(1, 1) MPSV_A(2, 1) MPSV_A(4, 1) MPSV_A(1, 2) MPSV_A(2, 2) MPSV_A(4, 2)
  MPSV_A(1, 4) MPSV_A(2, 4) MPSV_A(4, 4) MPSV_A(1, 8) MPSV_A(2, 8) MPSV_A(4, 8)
  MPSV_A(1, 16) MPSV_A(2, 16) MPSV_A(1, 32)
  MPSV_L(1, 8) MPSV_L(2, 8) MPSV_L(1, 16) MPSV_L(2, 16) MPSV_L(1, 32)
  MPSV_S(1, 8) MPSV_S(2, 8) MPSV_S(1, 16) MPSV_S(2, 16) MPSV_S(1, 32)
  throw Error(kEinval, "qr_reg_apply_chunks: no kernel for this shape");
#undef MPSV_S
#undef MPSV_L
#undef MPSV_A
  MPSV_LAUNCHED();
  prof_end(s, slot, kClsQrApply, 4.0 * p * (double)k * m, 8.0 * (2.0 * m * p + (double)m * k));
  tune_end(s, tp.slot);
}

}  // namespace mpsv
