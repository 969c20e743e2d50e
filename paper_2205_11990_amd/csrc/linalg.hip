// FP64 factorisations for the compression sweeps (SI, "Canonicalization and
// Compression"): blocked Householder QR and one-sided Jacobi SVD.
//
// QR: right-looking blocked Householder with register-resident panels
// (qr_reg.hip).  Blocks of at most 2048 rows are factored panel by panel on
// one workgroup each, the trailing columns updated by the reflector
// application kernel.  Taller blocks factor each 16-column panel as a TSQR:
// row chunks of at most 2048 rows factored side by side in one launch, then
// the stacked triangular factors; the trailing columns take the chunk
// reflectors and then those of the stacked factor on the chunk-top rows.
//
// SVD: X (m x c) is first reduced to its c x c triangular factor when tall,
// then one-sided (Hestenes) Jacobi with the cyclic round-robin ordering is
// run by one workgroup, columns and accumulated rotations held in LDS when
// they fit.  Singular values are the final column norms; sorting and the
// truncation rule (cap chi, relative discarded weight tol, eq. 5) are
// evaluated on the device.
#include <algorithm>
#include <optional>
#include <cmath>
#include <cstdlib>
#include <mutex>

#include "gemm.hpp"
#include "jacobi.hpp"
#include "linalg.hpp"
#include "prof.hpp"
#include "qr_reg.hpp"

namespace mpsv {

namespace {

constexpr int NT = 256;
constexpr size_t kJacobiLds = 144 * 1024;

LinalgStats g_stats;
int g_max_sweeps = 60;

// Extra QR factorisations of the triangular factor before the Jacobi
// sweeps, after the first one of X (tuning knob, MPSV_SVD_PRECOND_QR in the
// environment, 0..6; default 2: B^T, then B).
int svd_precondition_qrs() {
  static const int n = [] {
    const char* e = std::getenv("MPSV_SVD_PRECOND_QR");
    return e ? std::max(0, std::min(6, std::atoi(e))) : 2;
  }();
  return n;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the workgroup; every thread receives the total.
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) t += red[i];
  return t;
}

__global__ void extract_r_kernel(const double* A, int k, int n, long ld,
                                 MatView R, InstOff io) {
  const long o_ = io.of(blockIdx.z);
  A = shifted(A, o_);
  R = shifted(R, o_);
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)k * n;
       e += (long)gridDim.x * blockDim.x) {
    long i = e / n, j = e % n;
    R.p[i * R.rs + j * R.cs] = (j >= i) ? A[i * ld + j] : 0.0;
  }
}

// out[0:rows, 0:cols] = in (rows < rows_in), 0 (rows >= rows_in); any strides
__global__ void copy_view_kernel(CMatView in, int rows_in, MatView out,
                                 int rows, int cols, InstOff io) {
  const long o_ = io.of(blockIdx.z);
  in = shifted(in, o_);
  out = shifted(out, o_);
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
       e < (long)rows * cols; e += (long)gridDim.x * blockDim.x) {
    const long i = e / cols, j = e % cols;
    out.p[i * out.rs + j * out.cs] = (i < rows_in) ? in.p[i * in.rs + j * in.cs] : 0.0;
  }
}

__global__ void fill_rows_zero_kernel(double* X, int r0, int r1, int nc,
                                      long ld, InstOff io) {
  X = shifted(X, io.of(blockIdx.z));
  long tot = (long)(r1 - r0) * nc;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    long i = r0 + e / nc, j = e % nc;
    X[i * ld + j] = 0.0;
  }
}

// One-sided Jacobi SVD of B (mb x c, row-major, leading dimension ldb).
// Working copies are column-major: W[j*mb + i] (= B J) and J[j*c + i].
// info[0] = D, info[1] = discarded weight, info[2] = sweeps, info[3] = 1 if
// converged.
__global__ __launch_bounds__(NT) void jacobi_svd_kernel(
    const double* __restrict__ B, int mb, int c, long ldb, double* Wg,
    double* Jg, int use_lds, int cap, double tol, int max_sweeps, double* Vt,
    double* USs, long ldus_rows_limit, double* sig_out, double* info,
    InstOff io) {
  {
    const long o_ = io.of(blockIdx.z);
    B = shifted(B, o_);
    if (Wg) Wg = shifted(Wg, o_);
    if (Jg) Jg = shifted(Jg, o_);
    Vt = shifted(Vt, o_);
    USs = shifted(USs, o_);
    sig_out = shifted(sig_out, o_);
    info = shifted(info, o_);
  }
  extern __shared__ double smem[];
  __shared__ double red[NT / 64];
  __shared__ int rotated;
  __shared__ int Dsh;
  const int tid = threadIdx.x;
  double* W = use_lds ? smem : Wg;
  double* J = use_lds ? smem + (long)mb * c : Jg;

  for (long e = tid; e < (long)mb * c; e += NT) {
    long j = e / mb, i = e % mb;
    W[e] = B[i * ldb + j];
  }
  for (long e = tid; e < (long)c * c; e += NT) {
    long j = e / c, i = e % c;
    J[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  double part = 0.0;
  for (long e = tid; e < (long)mb * c; e += NT) part += W[e] * W[e];
  const double normF2 = block_sum(part, red);
  const double abs_floor = 1e-32 * normF2;
  const double eps = 1e-15;

  const int cc = c + (c & 1);
  const int np = cc / 2;
  int G = 1;
  while (G < 64 && G * 2 * np <= NT) G *= 2;
  const int ngroups = NT / G;
  const int grp = tid / G, lig = tid % G;

  int sweep = 0;
  int converged = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < cc - 1; ++r) {
      for (int k = grp; k < np; k += ngroups) {
        int p, q;
        if (k == 0) {
          p = cc - 1;
          q = r;
        } else {
          p = (r + k) % (cc - 1);
          q = (r - k + cc - 1) % (cc - 1);
        }
        if (p >= c || q >= c) continue;
        double* wp = W + (long)p * mb;
        double* wq = W + (long)q * mb;
        double a = 0.0, b = 0.0, g = 0.0;
        for (int i = lig; i < mb; i += G) {
          double x = wp[i], y = wq[i];
          a += x * x;
          b += y * y;
          g += x * y;
        }
        for (int o = G >> 1; o > 0; o >>= 1) {
          a += __shfl_xor(a, o, 64);
          b += __shfl_xor(b, o, 64);
          g += __shfl_xor(g, o, 64);
        }
        if (g != 0.0 && fabs(g) > eps * sqrt(a * b) && fabs(g) > abs_floor) {
          const double z = (b - a) / (2.0 * g);
          const double t = (z == 0.0) ? 1.0 : copysign(1.0, z) / (fabs(z) + hypot(1.0, z));
          const double cs = 1.0 / sqrt(1.0 + t * t);
          const double sn = cs * t;
          for (int i = lig; i < mb; i += G) {
            double x = wp[i], y = wq[i];
            wp[i] = cs * x - sn * y;
            wq[i] = sn * x + cs * y;
          }
          double* jp = J + (long)p * c;
          double* jq = J + (long)q * c;
          for (int i = lig; i < c; i += G) {
            double x = jp[i], y = jq[i];
            jp[i] = cs * x - sn * y;
            jq[i] = sn * x + cs * y;
          }
          if (lig == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    if (rotated == 0) {
      converged = 1;
      ++sweep;
      break;
    }
    __syncthreads();
  }

  // singular values = column norms, sorted descending (ties by index);
  // the norms go to the scratch half of sig_out first
  for (int j = tid; j < c; j += NT) {
    double s2 = 0.0;
    const double* wj = W + (long)j * mb;
    for (int i = 0; i < mb; ++i) s2 += wj[i] * wj[i];
    sig_out[c + j] = sqrt(s2);  // scratch half of sig_out (length 2c)
  }
  __syncthreads();
  __threadfence_block();
  int* perm = (int*)(sig_out + 2 * c);  // int scratch after the values
  for (int j = tid; j < c; j += NT) {
    const double sj = sig_out[c + j];
    int rank = 0;
    for (int k = 0; k < c; ++k) {
      double sk = sig_out[c + k];
      rank += (sk > sj || (sk == sj && k < j)) ? 1 : 0;
    }
    perm[rank] = j;
    sig_out[rank] = sj;
  }
  __syncthreads();
  __threadfence_block();
  const int kmax = mb < c ? mb : c;
  if (tid == 0) {
    double tot = 0.0;
    for (int i = 0; i < c; ++i) tot += sig_out[i] * sig_out[i];
    int D = kmax;
    int capd = cap < kmax ? cap : kmax;
    double disc2 = 0.0;
    if (tol <= 0.0) {
      D = capd;  // the cap alone decides, whatever the values (a zero block too)
    } else if (tot <= 0.0) {
      D = 1;
    } else {
      // smallest D' >= 1 with sum_{i >= D'} t_i <= tol^2, tail summed from the end
      double tail = 0.0;
      for (int i = c - 1; i >= kmax; --i) tail += sig_out[i] * sig_out[i] / tot;
      // walk down from kmax accumulating the tail (values beyond kmax are
      // the numerically zero columns of a wide matrix)
      int best = kmax;
      double acc = tail;
      for (int Dp = kmax - 1; Dp >= 1; --Dp) {
        acc += sig_out[Dp] * sig_out[Dp] / tot;
        if (acc <= tol * tol) best = Dp; else break;
      }
      D = best;
      if (D > capd) D = capd;
    }
    if (D < 1) D = 1;
    for (int i = D; i < c; ++i) disc2 += sig_out[i] * sig_out[i];
    Dsh = D;
    info[0] = (double)D;
    info[1] = (tot > 0.0) ? sqrt(disc2 / tot) : 0.0;
    info[2] = (double)sweep;
    info[3] = (double)converged;
  }
  __syncthreads();
  const int D = Dsh;
  // Vt[d][i] = J[i][perm[d]]
  for (long e = tid; e < (long)D * c; e += NT) {
    long d = e / c, i = e % c;
    Vt[e] = J[(long)perm[d] * c + i];
  }
  // USs[i][d] = W[i][perm[d]] for i < min(mb, limit)
  const int rows = (int)(mb < ldus_rows_limit ? mb : ldus_rows_limit);
  for (long e = tid; e < (long)rows * D; e += NT) {
    long i = e / D, d = e % D;
    USs[e] = W[(long)perm[d] * mb + i];
  }
}

// Chunk-top rows of a TSQR panel: stacked row t of T (t < srows) is row
// (t / jb) * crows + t % jb of X (leading dimension ld); gathered into T
// (srows x nc, row-major) or scattered back.
__global__ void chunk_tops_kernel(double* X, long ld, int crows, int jb,
                                  int srows, int nc, double* T, int gather,
                                  InstOff io) {
  const long o_ = io.of(blockIdx.z);
  X = shifted(X, o_);
  T = shifted(T, o_);
  const long total = (long)srows * nc;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int t = (int)(e / nc), c = (int)(e % nc);
    const long row = (long)(t / jb) * crows + t % jb;
    if (gather) T[e] = X[row * ld + c];
    else X[row * ld + c] = T[e];
  }
}

std::once_flag g_attr_once;
void set_attrs() {
  std::call_once(g_attr_once, [] {
    MPSV_HIP(hipFuncSetAttribute((const void*)jacobi_svd_kernel,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)kJacobiLds));
  });
}

}  // namespace

LinalgStats& linalg_stats() { return g_stats; }

void SvdOutcomes::begin() {
  MPSV_CHECK(ring_ != nullptr, kEinval, "SVD outcome ring not bound");
  rec_ = Record{};
  on_ = true;
}

double* SvdOutcomes::reserve(double* disc, long disc_stride, bool split) {
  const int slot = rec_.used++;
  if (disc) {
    rec_.disc.push_back({disc, slot});
    rec_.disc_stride.push_back(disc_stride);
  }
  rec_.split.push_back(split ? 1 : 0);
  return ring_ + (long)slot * kInfoWords;
}

void SvdOutcomes::end(hipStream_t s) {
  if (!on_) return;
  on_ = false;
  if (rec_.used == 0) return;
  // the used slots of every lock-step instance, one row per instance
  const int ni = inst_count();
  const size_t row = (size_t)rec_.used * kInfoWords;
  double* h = (double*)host_.get(row * (size_t)ni * sizeof(double));
  lanes_d2h(s, h, ring_, row * sizeof(double));
  MPSV_HIP(hipStreamSynchronize(s));
  int code = 0;
  std::string msg;
  for (int inst = 0; inst < ni; ++inst) {
    const double* hi = h + row * inst;
    for (int i = 0; i < rec_.used; ++i) {
      const double* w = hi + (long)i * kInfoWords;
      g_stats.jacobi_sweeps += (long)w[2];
      if (code) continue;
      if (rec_.split[i] && w[5] != 0.0) {
        code = kEdevice;
        msg = "Jacobi SVD: the workgroups did not meet in time";
      } else if (w[3] == 0.0) {
        code = kEnumeric;
        msg = "Jacobi SVD did not converge within " + std::to_string(g_max_sweeps) +
              " sweeps";
      }
      if (code && ni > 1) msg = "instance " + std::to_string(inst) + ": " + msg;
    }
    for (size_t t = 0; t < rec_.disc.size(); ++t)
      rec_.disc[t].first[inst * rec_.disc_stride[t]] =
          hi[(long)rec_.disc[t].second * kInfoWords + 1];
  }
  rec_ = Record{};
  if (code) throw Error(code, msg);
}

SvdOutcomes::Record SvdOutcomes::take() {
  Record r = rec_;
  on_ = false;
  rec_ = Record{};
  return r;
}

void SvdOutcomes::resume(const Record& r) {
  MPSV_CHECK(ring_ != nullptr && r.used <= kSlots, kEinval,
             "deferred SVD record without its slots");
  rec_ = r;
  on_ = true;
}

void SvdOutcomes::cancel(hipStream_t s) noexcept {
  if (!on_) return;
  on_ = false;
  (void)hipStreamSynchronize(s);
  rec_ = Record{};
}

void set_jacobi_max_sweeps(int n) { g_max_sweeps = n < 1 ? 1 : n; }
int jacobi_max_sweeps() { return g_max_sweeps; }

void extract_r(hipStream_t s, const double* A, int k, int n, long ld,
               MatView R) {
  if (k <= 0 || n <= 0) return;
  int blocks = std::min(1024, ceil_div((long)k * n, 256));
  hipLaunchKernelGGL(extract_r_kernel, dim3(blocks, 1, inst_count()), dim3(256), 0, s, A, k, n,
                     ld, R, inst_off());
  MPSV_LAUNCHED();
}

void chunk_tops(hipStream_t s, double* X, long ld, int crows, int jb, int srows,
                int nc, double* T, bool gather) {
  if (srows <= 0 || nc <= 0) return;
  int blocks = std::min(1024, ceil_div((long)srows * nc, 256));
  hipLaunchKernelGGL(chunk_tops_kernel, dim3(blocks, 1, inst_count()), dim3(256), 0, s, X, ld,
                     crows, jb, srows, nc, T, gather ? 1 : 0, inst_off());
  MPSV_LAUNCHED();
}

void copy_view(hipStream_t s, CMatView in, int rows_in, MatView out, int rows,
               int cols) {
  if (rows <= 0 || cols <= 0) return;
  int blocks = std::min(1024, ceil_div((long)rows * cols, 256));
  hipLaunchKernelGGL(copy_view_kernel, dim3(blocks, 1, inst_count()), dim3(256), 0, s, in,
                     rows_in, out, rows, cols, inst_off());
  MPSV_LAUNCHED();
}

__global__ void fill_ints_kernel(int* x, long n, InstOff io) {
  x = shifted(x, io.of(blockIdx.z));
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
       e += (long)gridDim.x * blockDim.x)
    x[e] = 0;
}

static void fill_ints(hipStream_t s, int* x, long n) {
  if (n <= 0) return;
  int blocks = std::min(1024, ceil_div(n, 256));
  hipLaunchKernelGGL(fill_ints_kernel, dim3(blocks, 1, inst_count()), dim3(256), 0, s, x, n, inst_off());
  MPSV_LAUNCHED();
}

__global__ void transpose_kernel(const double* A, int rows, int cols, long lda,
                                 double* B, long ldb, InstOff io) {
  const long o_ = io.of(blockIdx.z);
  A = shifted(A, o_);
  B = shifted(B, o_);
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
       e < (long)rows * cols; e += (long)gridDim.x * blockDim.x) {
    const long i = e % rows, j = e / rows;   // consecutive threads: rows of A
    B[j * ldb + i] = A[i * lda + j];
  }
}

// B (cols x rows, ldb) = A^T for A rows x cols (lda)
static void transpose(hipStream_t s, const double* A, int rows, int cols,
                      long lda, double* B, long ldb) {
  if (rows <= 0 || cols <= 0) return;
  int blocks = std::min(1024, ceil_div((long)rows * cols, 256));
  hipLaunchKernelGGL(transpose_kernel, dim3(blocks, 1, inst_count()), dim3(256), 0, s, A, rows,
                     cols, lda, B, ldb, inst_off());
  MPSV_LAUNCHED();
}

__global__ void copy_rows_kernel(const double* A, long n, double* B, InstOff io) {
  const long o_ = io.of(blockIdx.z);
  A = shifted(A, o_);
  B = shifted(B, o_);
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
       e += (long)gridDim.x * blockDim.x)
    B[e] = A[e];
}

// B[0:rows, :] = A (rows x cols, both contiguous with leading dim cols)
static void copy_rows(hipStream_t s, const double* A, int rows, int cols,
                      double* B) {
  const long n = (long)rows * cols;
  if (n <= 0) return;
  int blocks = std::min(1024, ceil_div(n, 256));
  hipLaunchKernelGGL(copy_rows_kernel, dim3(blocks, 1, inst_count()), dim3(256), 0, s, A, n, B, inst_off());
  MPSV_LAUNCHED();
}

static void fill_rows_zero(hipStream_t s, double* X, int r0, int r1, int nc,
                           long ld) {
  if (r1 <= r0 || nc <= 0) return;
  int blocks = std::min(1024, ceil_div((long)(r1 - r0) * nc, 256));
  hipLaunchKernelGGL(fill_rows_zero_kernel, dim3(blocks, 1, inst_count()), dim3(256), 0, s, X,
                     r0, r1, nc, ld, inst_off());
  MPSV_LAUNCHED();
}

// Panel groups of the compact-WY mode: blocks of more than 512 rows whose
// register panels are 16 columns wide, with more than one panel left.
constexpr int kGroupCols = 64;
static bool group_panels(int rows, int ncols) {
  return lanes().tall_apply == 1 && rows > 512 && qr_reg_panel_cols(rows) == 16 &&
         ncols > 16;
}

void qr_factor(hipStream_t s, Arena& ws, double* A, int m, int n, long ld,
               QrFactor& f, MatView R) {
  set_attrs();
  f.m = m;
  f.n = n;
  f.k = std::min(m, n);
  f.panels.clear();
  g_stats.qr_calls++;
  // one register panel with a separate R: written straight there, A
  // untouched
  const bool single = m <= 2048 && n <= qr_reg_panel_cols(m);
  for (int k0 = 0; k0 < f.k;) {
    const int rows = m - k0;
    double* P = A + (long)k0 * ld + k0;
    QrPanel pn;
    pn.k0 = k0;
    if (rows <= 2048 && group_panels(rows, n - k0)) {
      // compact-WY mode: up to four 16-column panels factored in turn, each
      // updating only the group's columns right of it; the group's
      // reflectors then reach the trailing columns as one block
      const int kg = std::min(kGroupCols, n - k0);
      const int np = ceil_div(kg, 16);
      pn.jb = kg;
      pn.reg = true;
      pn.grp = np;
      pn.V = ws.alloc((size_t)qr_group_voff(rows, np));
      pn.tau = ws.alloc((size_t)kGroupCols);
      pn.T = ws.alloc((size_t)kGroupCols * kGroupCols);
      for (int t = 0; t < np; ++t) {
        const int c0 = 16 * t, jb = std::min(16, kg - c0), r = rows - c0;
        double* Pt = P + (long)c0 * ld + c0;
        double* Vp = pn.V + qr_group_voff(rows, t);
        qr_reg_factor(s, CMatView{Pt, ld, 1, 0}, r, jb, MatView{Pt, ld, 1, 0}, Vp,
                      pn.tau + c0);
        const int nin = kg - c0 - jb;
        if (nin > 0)
          qr_reg_apply(s, Vp, pn.tau + c0, r, jb, CMatView{Pt + jb, ld, 1, 0}, r,
                       MatView{Pt + jb, ld, 1, 0}, nin, true);
      }
      qr_wy_group_t(s, pn.V, pn.tau, rows, kg, pn.T);
      const int n2 = n - k0 - kg;
      if (n2 > 0)
        qr_wy_group_apply(s, pn.V, pn.T, rows, kg, CMatView{P + kg, ld, 1, 0}, rows,
                          MatView{P + kg, ld, 1, 0}, n2, true);
      f.panels.push_back(pn);
      k0 += kg;
      continue;
    }
    if (rows <= 2048) {
      // register-resident panel; the trailing columns are updated by the
      // reflector-application kernel
      const int jb = std::min(qr_reg_panel_cols(rows), n - k0);
      const int kk = std::min(rows, jb);
      pn.jb = kk;
      pn.reg = true;
      pn.V = ws.alloc((size_t)rows * kk);
      pn.tau = ws.alloc((size_t)kk);
      const MatView Rout = (single && R.p) ? R : MatView{P, ld, 1, 0};
      qr_reg_factor(s, CMatView{P, ld, 1, 0}, rows, jb, Rout, pn.V, pn.tau);
      const int n2 = n - k0 - jb;
      if (n2 > 0)
        qr_reg_apply(s, pn.V, pn.tau, rows, kk, CMatView{P + jb, ld, 1, 0}, rows,
                     MatView{P + jb, ld, 1, 0}, n2, true);
      f.panels.push_back(pn);
      k0 += jb;
      continue;
    }
    // TSQR panel: row chunks, each factored on its own workgroup, their
    // triangular factors stacked (chunk c at rows c*jb) and factored again;
    // the panel's R lands in the panel's top rows.  Chunks of at most 512
    // rows take 32-column panels (half the panels, and launches, of the
    // 16-column panels that 2048-row chunks allow) while the stacked
    // factors still fit one register panel (at most 16 chunks).
    int chunk_max = 512, jb = 32;
    if ((rows + chunk_max - 1) / chunk_max * jb > 512) {
      chunk_max = 2048;
      jb = qr_reg_panel_cols(2048);
    }
    jb = std::min(jb, f.k - k0);
    const int nch = (rows + chunk_max - 1) / chunk_max;
    const int crows = (rows + nch - 1) / nch;
    const int last = rows - (nch - 1) * crows;
    pn.jb = jb;
    pn.crows = crows;
    pn.srows = (nch - 1) * jb + std::min(last, jb);
    pn.V = ws.alloc((size_t)nch * crows * jb);
    pn.tau = ws.alloc((size_t)nch * jb);
    pn.Vt = ws.alloc((size_t)pn.srows * jb);
    pn.taut = ws.alloc((size_t)jb);
    {
      ArenaScope sc(ws);
      double* S = ws.alloc((size_t)nch * jb * jb);
      qr_reg_factor_chunks(s, CMatView{P, ld, 1, 0}, rows, jb, crows,
                           MatView{S, jb, 1, 0}, pn.V, pn.tau);
      qr_reg_factor(s, CMatView{S, jb, 1, 0}, pn.srows, jb, MatView{P, ld, 1, 0},
                    pn.Vt, pn.taut);
    }
    const int n2 = n - k0 - jb;
    if (n2 > 0) {
      // trailing columns: Q^T = Q_top^T diag(Q_c^T)
      qr_reg_apply_chunks(s, pn.V, pn.tau, rows, jb, crows,
                          MatView{P + jb, ld, 1, 0}, n2, true);
      ArenaScope sc(ws);
      double* T = ws.alloc((size_t)pn.srows * n2);
      chunk_tops(s, P + jb, ld, crows, jb, pn.srows, n2, T, true);
      qr_reg_apply(s, pn.Vt, pn.taut, pn.srows, jb, CMatView{T, n2, 1, 0},
                   pn.srows, MatView{T, n2, 1, 0}, n2, true);
      chunk_tops(s, P + jb, ld, crows, jb, pn.srows, n2, T, false);
    }
    f.panels.push_back(pn);
    k0 += jb;
  }
  if (R.p && !single) extract_r(s, A, f.k, n, ld, R);
}

void qr_factor_view(hipStream_t s, Arena& ws, CMatView A, int m, int n,
                    QrFactor& f, MatView R) {
  if (m <= 2048 && n <= qr_reg_panel_cols(m)) {
    set_attrs();
    f.m = m;
    f.n = n;
    f.k = std::min(m, n);
    f.panels.clear();
    g_stats.qr_calls++;
    QrPanel pn;
    pn.k0 = 0;
    pn.jb = f.k;
    pn.reg = true;
    pn.V = ws.alloc((size_t)m * f.k);
    pn.tau = ws.alloc((size_t)f.k);
    qr_reg_factor(s, A, m, n, R, pn.V, pn.tau);
    f.panels.push_back(pn);
    return;
  }
  double* C = ws.alloc((size_t)m * n);
  copy_view(s, A, m, MatView{C, n, 1, 0}, m, n);
  qr_factor(s, ws, C, m, n, n, f, R);
}

void qr_apply_q_view(hipStream_t s, Arena& ws, const QrFactor& f, CMatView Yin,
                     int rows_in, MatView Yout, int nc) {
  if (nc <= 0) return;
  if (f.panels.size() == 1 && f.panels[0].reg) {
    const QrPanel& pn = f.panels[0];
    if (pn.grp)
      qr_wy_group_apply(s, pn.V, pn.T, f.m, pn.jb, Yin, rows_in, Yout, nc, false);
    else
      qr_reg_apply(s, pn.V, pn.tau, f.m, pn.jb, Yin, rows_in, Yout, nc, false);
    return;
  }
  if (Yout.cs != 1) {
    // panelled Q into a strided output: through a row-major buffer
    ArenaScope sc(ws);
    double* T = ws.alloc((size_t)f.m * nc);
    copy_view(s, Yin, rows_in, MatView{T, nc, 1, 0}, f.m, nc);
    qr_apply_q(s, ws, f, T, nc, nc);
    copy_view(s, CMatView{T, nc, 1, 0}, f.m, Yout, f.m, nc);
    return;
  }
  if (Yin.p != Yout.p || Yin.rs != Yout.rs || Yin.cs != Yout.cs || rows_in < f.m)
    copy_view(s, Yin, rows_in, Yout, f.m, nc);
  qr_apply_q(s, ws, f, Yout.p, nc, Yout.rs);
}

void qr_apply_q(hipStream_t s, Arena& ws, const QrFactor& f, double* X, int nc,
                long ldx) {
  if (nc <= 0) return;
  for (int p = (int)f.panels.size() - 1; p >= 0; --p) {
    const QrPanel& pn = f.panels[p];
    const int rows = f.m - pn.k0;
    double* X2 = X + (long)pn.k0 * ldx;
    if (pn.grp) {
      qr_wy_group_apply(s, pn.V, pn.T, rows, pn.jb, CMatView{X2, ldx, 1, 0}, rows,
                        MatView{X2, ldx, 1, 0}, nc, false);
      continue;
    }
    if (pn.reg) {
      qr_reg_apply(s, pn.V, pn.tau, rows, pn.jb, CMatView{X2, ldx, 1, 0}, rows,
                   MatView{X2, ldx, 1, 0}, nc, false);
      continue;
    }
    // TSQR panel: Q = diag(Q_c) Q_top, the stacked factor acting on the
    // chunk-top rows
    ArenaScope sc(ws);
    double* T = ws.alloc((size_t)pn.srows * nc);
    chunk_tops(s, X2, ldx, pn.crows, pn.jb, pn.srows, nc, T, true);
    qr_reg_apply(s, pn.Vt, pn.taut, pn.srows, pn.jb, CMatView{T, nc, 1, 0},
                 pn.srows, MatView{T, nc, 1, 0}, nc, false);
    chunk_tops(s, X2, ldx, pn.crows, pn.jb, pn.srows, nc, T, false);
    qr_reg_apply_chunks(s, pn.V, pn.tau, rows, pn.jb, pn.crows,
                        MatView{X2, ldx, 1, 0}, nc, false);
  }
}

int svd_truncate(hipStream_t s, Arena& ws, double* X, int m, int c, long ldx,
                 int cap, double tol, double* Vt, double* US, double* sig,
                 double* discarded, SvdOutcomes* out, long disc_stride) {
  set_attrs();
  g_stats.svd_calls++;
  MPSV_CHECK(m >= 1 && c >= 1, kEinval, "svd_truncate: empty matrix");
  ArenaScope sc(ws);
  // the launches of the decomposition are nested in its record (the
  // Jacobi launch, which carries the nominal work of the whole SVD)
  std::optional<ProfNested> nest;
  nest.emplace();
  // the kernels write their outcome words to device memory: a slot of the
  // lane's deferred record, or a block of the workspace read back below
  const int k0 = std::min(m, c);
  const bool defer = tol <= 0.0 && out && out->deferring();
  MPSV_CHECK(defer || inst_count() == 1, kEinval,
             "lock-step instances need fixed-rank truncations (tol = 0)");
  double* info = defer ? out->reserve(discarded, disc_stride,
                                      k0 <= kJacobiMaxCols && jacobi_split(k0) > 0)
                       : ws.alloc(SvdOutcomes::kInfoWords);
  double* sigbuf = ws.alloc((size_t)3 * std::max(m, c) + 8);
  const int k = std::min(m, c);
  // Preconditioning: Jacobi runs on the transpose of a triangular factor
  // B obtained by a chain of QR factorisations, first of X (m >= c) or of
  // X^T (m < c), then alternately of B^T and B, until
  //   X = L_1 ... L_p  B  (R_1 ... R_q)^T,   B upper triangular (k x k).
  // Jacobi on B^T gives W Sigma (W: right singular vectors of B), so
  //   V = R_1 (... (R_q W)),   U Sigma = L_1 (... (L_p (B W))) = X V.
  // Each extra pair of factorisations moves B closer to diagonal and saves
  // Jacobi sweeps.  The rotations are never accumulated, and U Sigma of the
  // kept values is formed as X V_D by one GEMM (X is read, not modified).
  const bool onchip = k <= kJacobiMaxCols;
  const int mode = (m >= c) ? 0 : 1;
  QrFactor qf;  // used by the large-matrix path
  std::vector<QrFactor> Lf, Rf;
  Lf.reserve(4);
  Rf.reserve(4);
  double* Rk = nullptr;
  double* Wt = nullptr;
  int slot = -1;
  if (onchip) {
    // B is kept row-major k x k in Bk; the factorisations read it (or its
    // transpose) through strided views and write the next B in place of a
    // second buffer, so no transposes or copies are launched.
    bool upper;
    double* Bk = ws.alloc((size_t)k * k);
    double* Bn = ws.alloc((size_t)k * k);
    if (mode == 0) {
      // read through a view: X itself stays intact for U Sigma = X V below
      Lf.emplace_back();
      qr_factor_view(s, ws, CMatView{X, ldx, 1, 0}, m, c, Lf.back(),
                     MatView{Bk, k, 1, 0});
      upper = true;
    } else {
      // X^T = Q1 R1 read through a transposed view; B = R1^T (lower)
      Rf.emplace_back();
      qr_factor_view(s, ws, CMatView{X, 1, ldx, 0}, c, m, Rf.back(),
                     MatView{Bk, 1, k, 0});
      upper = false;
    }
    // the Jacobi kernel takes any square factor, upper or lower triangular
    int extra = svd_precondition_qrs();
    while (extra > 0) {
      if (upper) {
        // B = R: R^T = Q' R'  ->  B = R'^T Q'^T; write R'^T
        Rf.emplace_back();
        qr_factor_view(s, ws, CMatView{Bk, 1, k, 0}, k, k, Rf.back(),
                       MatView{Bn, 1, k, 0});
        upper = false;
      } else {
        // B lower: B = Q' R'
        Lf.emplace_back();
        qr_factor_view(s, ws, CMatView{Bk, k, 1, 0}, k, k, Lf.back(),
                       MatView{Bn, k, 1, 0});
        upper = true;
      }
      std::swap(Bk, Bn);
      --extra;
    }
    Rk = Bk;
    Wt = ws.alloc((size_t)k * k);
    int* perm = ws.alloc_int((size_t)k);
    const size_t jws = jacobi_ws_doubles(k);
    double* jw = jws ? ws.alloc(jws) : nullptr;
    nest.reset();
    slot = prof_begin(s);
    jacobi_svd(s, Rk, k, k, cap, tol, g_max_sweeps, Wt, sigbuf, perm, info, jw);
  } else {
    // large matrices: unpreconditioned Jacobi on the columns, in global memory
    const bool tall = m > c;
    const double* B = X;
    long ldb = ldx;
    int mb = m;
    if (tall) {
      double* R = ws.alloc((size_t)c * c);
      qr_factor(s, ws, X, m, c, ldx, qf, MatView{R, c, 1, 0});
      B = R;
      ldb = c;
      mb = c;
    }
    const size_t need = ((size_t)mb * c + (size_t)c * c) * sizeof(double);
    const int use_lds = need <= kJacobiLds ? 1 : 0;
    double* Wg = use_lds ? nullptr : ws.alloc((size_t)mb * c);
    double* Jg = use_lds ? nullptr : ws.alloc((size_t)c * c);
    nest.reset();
    slot = prof_begin(s);
    hipLaunchKernelGGL(jacobi_svd_kernel, dim3(1, 1, inst_count()), dim3(NT),
                       use_lds ? need : 0, s, B, mb, c, ldb, Wg, Jg, use_lds, cap,
                       tol, g_max_sweeps, Vt, US, (long)mb, sigbuf, info,
                       inst_off());
    MPSV_LAUNCHED();
  }
  {
    // nominal SVD flops of the factored m x c matrix, 6 m n^2 + 20 n^3
    const double mm = std::max(m, c), nn = std::min(m, c);
    prof_end(s, slot, kClsJacobi, 6.0 * mm * nn * nn + 20.0 * nn * nn * nn,
             8.0 * (2.0 * m * c + 2.0 * nn * nn));
  }
  nest.emplace();
  int D;
  if (defer) {
    // fixed rank: the kernels keep min(cap, k) whatever the values
    D = cap < k ? cap : k;
  } else {
    // the rank read-back: into the lane's page-locked words when there is
    // a lane record
    double hs[SvdOutcomes::kInfoWords];
    double* h = out ? out->host_words(SvdOutcomes::kInfoWords) : hs;
    MPSV_HIP(hipMemcpyAsync(h, shifted(info, lanes().first),
                            SvdOutcomes::kInfoWords * sizeof(double),
                            hipMemcpyDeviceToHost, s));
    MPSV_HIP(hipStreamSynchronize(s));
    D = (int)h[0];
    if (discarded) *discarded = h[1];
    g_stats.jacobi_sweeps += (long)h[2];
    if (onchip && jacobi_split(k) > 0 && h[5] != 0.0)
      throw Error(kEdevice, "Jacobi SVD: the workgroups did not meet in time");
    if (h[3] == 0.0)
      throw Error(kEnumeric, "Jacobi SVD did not converge within " +
                                 std::to_string(g_max_sweeps) + " sweeps");
  }
  if (sig) copy_rows(s, sigbuf, 1, k, sig);
  if (onchip) {
    // V = R_1 (... (R_q W_D)) (c x D): the first application reads W_D = Wt^T
    // through a view, the last writes V^T straight into Vt; rows beyond the
    // k of the triangular factor enter as zeros
    CMatView in{Wt, 1, k, 0};
    double* Y = ws.alloc((size_t)c * D);
    for (int i = (int)Rf.size() - 1; i >= 0; --i) {
      const MatView out = (i == 0) ? MatView{Vt, 1, c, 0} : MatView{Y, D, 1, 0};
      qr_apply_q_view(s, ws, Rf[i], in, k, out, D);
      in = CMatView{Y, D, 1, 0};
    }
    if (Rf.empty()) copy_view(s, in, k, MatView{Vt, 1, c, 0}, c, D);
    // U Sigma = X V_D (m x D) by one GEMM from the untouched X: the
    // projection of X on the kept right singular vectors, the same product
    // as L_1 (... (L_p (B W_D))) without applying the left reflectors (the
    // left factorisations only serve as preconditioners)
    gemm(s, m, D, c, 1.0, CMatView{X, ldx, 1, 0}, CMatView{Vt, 1, c, 0}, 0.0,
         MatView{US, D, 1, 0}, 1, 0, &ws);
  } else if (m > c) {
    // US rows [0, c) hold U_R Sigma (leading dimension D): US = Q [U_R Sigma; 0]
    fill_rows_zero(s, US, c, m, D, D);
    qr_apply_q(s, ws, qf, US, D, D);
  }
  return D;
}

}  // namespace mpsv
