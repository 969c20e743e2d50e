// Data-movement kernels of the MPS engine: block copies for direct sums
// (SI, Addition), Kronecker embedding of one-dimension operators into the
// interleaved chain, diagonal MPOs (SI, Dot Product), bit permutations and
// reductions.  All are memory-bound grid-stride loops.
#include <algorithm>
#include <cmath>

#include "mps_kernels.hpp"

namespace mpsv {

Lanes& lanes() {
  static thread_local Lanes l;
  return l;
}

void lanes_d2h(hipStream_t s, void* h, const void* d, size_t bytes) {
  const int ni = inst_count();
  const void* src = shifted(d, lanes().first);
  if (ni == 1) {
    MPSV_HIP(hipMemcpyAsync(h, src, bytes, hipMemcpyDeviceToHost, s));
    return;
  }
  MPSV_CHECK((size_t)lanes().stride >= bytes, kEinval, "lanes_d2h: rows overlap");
  MPSV_HIP(hipMemcpy2DAsync(h, bytes, src, (size_t)lanes().stride, bytes, (size_t)ni,
                            hipMemcpyDeviceToHost, s));
}

namespace {

inline int grid_for(long n) {
  long b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
}

#define GRID_STRIDE(e, n)                                                  \
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (n);      \
       e += (long)gridDim.x * blockDim.x)

// out[j][i][k] = in[i][j][k]: block row y is the pair t = j d0 + i, the
// inner index runs along x (coalesced on both sides)
__global__ void swap01_kernel(const double* in, int d0, int d1, long inner,
                              double* out, InstOff io) {
  const long o_ = io.of(blockIdx.z);
  in = shifted(in, o_);
  out = shifted(out, o_);
  const int t = blockIdx.y, i = t % d0, j = t / d0;
  const double* src = in + ((long)i * d1 + j) * inner;
  double* dst = out + (long)t * inner;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < inner;
       k += (long)gridDim.x * blockDim.x)
    dst[k] = src[k];
}

__global__ void copy2d_kernel(int rows, int cols, double alpha,
                              const double* src, long lds, double* dst,
                              long ldd, InstOff io) {
  const long o_ = io.of(blockIdx.z);
  src = shifted(src, o_);
  dst = shifted(dst, o_);
  const long n = (long)rows * cols;
  GRID_STRIDE(e, n) {
    long i = e / cols, j = e % cols;
    dst[i * ldd + j] = alpha * src[i * lds + j];
  }
}

__global__ void sum_physical_kernel(const double* in, int l, int r,
                                    double* out, InstOff io) {
  const long o_ = io.of(blockIdx.z);
  in = shifted(in, o_);
  out = shifted(out, o_);
  const long n = (long)l * r;
  GRID_STRIDE(e, n) {
    long a = e / r, b = e % r;
    out[e] = in[(a * 2) * r + b] + in[(a * 2 + 1) * r + b];
  }
}

// out[a][t] = in[a][t] * g(d[a]) over rows a < rows, t < len; g(x) = x, or
// for `inverse` 1/x with 0 where x <= d[0] * 1e-200 (d sorted descending, so
// d[0] is the largest value: a zero of a rank-deficient cut gets 0)
__global__ void scale_rows_kernel(const double* in, int rows, long len,
                                  const double* d, int inverse, double* out,
                                  InstOff io) {
  const long o_ = io.of(blockIdx.z);
  in = shifted(in, o_);
  d = shifted(d, o_);
  out = shifted(out, o_);
  const long n = (long)rows * len;
  const double floor = d[0] * 1e-200;
  GRID_STRIDE(e, n) {
    const double x = d[e / len];
    const double g = inverse ? (x > floor ? 1.0 / x : 0.0) : x;
    out[e] = in[e] * g;
  }
}

__global__ void identity_kernel(double* A, int n, InstOff io) {
  A = shifted(A, io.of(blockIdx.z));
  const long total = (long)n * n;
  GRID_STRIDE(e, total) A[e] = (e / n == e % n) ? 1.0 : 0.0;
}

// out[b][t][a] = in[a][t][b] for an l x 2 x r core
__global__ void reverse_core_kernel(const double* in, int l, int r,
                                    double* out, InstOff io) {
  const long o_ = io.of(blockIdx.z);
  in = shifted(in, o_);
  out = shifted(out, o_);
  const long n = 2L * l * r;
  GRID_STRIDE(e, n) {
    const long a = e % l, t = (e / l) % 2, b = e / (2L * l);
    out[e] = in[(a * 2 + t) * r + b];
  }
}

// Chain-order vector of a sequential ordering -> F[i * Nv + j]: the chain
// position of (i, j) is the x bits then the v bits, each most significant
// first, or least significant first for a reversed dimension.
__global__ void chain_to_grid_kernel(const double* in, int Lx, int Lv, int rx,
                                     int rv, double* out, InstOff io) {
  const long o_ = io.of(blockIdx.z);
  in = shifted(in, o_);
  out = shifted(out, o_);
  const long n = 1L << (Lx + Lv);
  GRID_STRIDE(e, n) {
    const long i = e >> Lv, j = e & ((1L << Lv) - 1);
    long ci = i, cj = j;
    if (rx) {
      ci = 0;
      for (int k = 0; k < Lx; ++k) ci |= ((i >> k) & 1L) << (Lx - 1 - k);
    }
    if (rv) {
      cj = 0;
      for (int k = 0; k < Lv; ++k) cj |= ((j >> k) & 1L) << (Lv - 1 - k);
    }
    out[e] = in[(ci << Lv) | cj];
  }
}

__global__ void kron_embed_kernel(const double* A, int l, int P, int r, int d,
                                  int mode, double* out, InstOff io) {
  const long o_ = io.of(blockIdx.z);
  A = shifted(A, o_);
  out = shifted(out, o_);
  // out shape (l*d) x P x (r*d); write all entries (zeros off the identity)
  const long L = (long)l * d, R = (long)r * d;
  const long n = L * P * R;
  GRID_STRIDE(e, n) {
    long col = e % R;
    long t = e / R;
    long p = t % P;
    long row = t / P;
    long a, c1, b, c2;
    if (mode == 0) {
      a = row / d; c1 = row % d; b = col / d; c2 = col % d;
    } else {
      c1 = row / l; a = row % l; c2 = col / r; b = col % r;
    }
    out[e] = (c1 == c2) ? A[(a * P + p) * r + b] : 0.0;
  }
}

__global__ void diag_mpo_kernel(const double* E, int l, int r, double scale,
                                double* W, InstOff io) {
  const long o_ = io.of(blockIdx.z);
  E = shifted(E, o_);
  W = shifted(W, o_);
  const long n = (long)l * 4 * r;
  GRID_STRIDE(e, n) {
    long b = e % r;
    long t = e / r;
    long i = t % 2;
    long o = (t / 2) % 2;
    long a = t / 4;
    W[e] = (o == i) ? scale * E[(a * 2 + i) * r + b] : 0.0;
  }
}

__global__ void mpo_left_matrix_kernel(const double* W, int wl, int wr,
                                       double* Wmat, InstOff io) {
  const long o_ = io.of(blockIdx.z);
  W = shifted(W, o_);
  Wmat = shifted(Wmat, o_);
  const long n = (long)2 * wr * 2 * wl;
  GRID_STRIDE(e, n) {
    long col = e % (2 * wl);   // (b, i)
    long row = e / (2 * wl);   // (o, b')
    long b = col / 2, i = col % 2;
    long o = row / wr, bp = row % wr;
    Wmat[e] = W[((b * 2 + o) * 2 + i) * wr + bp];
  }
}

__global__ void deinterleave_kernel(const double* in, int L, double* out,
                                    InstOff io) {
  const long o_ = io.of(blockIdx.z);
  in = shifted(in, o_);
  out = shifted(out, o_);
  const long N = 1L << L;
  const long n = N * N;
  GRID_STRIDE(e, n) {
    long i = e / N, j = e % N;
    long idx = 0;
    for (int k = 0; k < L; ++k) {
      long xb = (i >> (L - 1 - k)) & 1;
      long vb = (j >> (L - 1 - k)) & 1;
      idx = (idx << 2) | (xb << 1) | vb;
    }
    out[e] = in[idx];
  }
}

__global__ void count_nonfinite_kernel(const double* x, long n, int* flag,
                                       InstOff io) {
  const long o_ = io.of(blockIdx.z);
  x = shifted(x, o_);
  flag = shifted(flag, o_);
  int bad = 0;
  GRID_STRIDE(e, n) {
    if (!isfinite(x[e])) bad = 1;
  }
  if (bad) atomicAdd(flag, 1);
}

__global__ void sum_squares_kernel(const double* x, long n, double scale,
                                   double* out, InstOff io) {
  const long o_ = io.of(blockIdx.z);
  x = shifted(x, o_);
  out = shifted(out, o_);
  __shared__ double red[256];
  double acc = 0.0;
  for (long e = threadIdx.x; e < n; e += blockDim.x) acc += x[e] * x[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = scale * red[0];
}

__global__ void fill_kernel(double* x, long n, double v, InstOff io) {
  x = shifted(x, io.of(blockIdx.z));
  GRID_STRIDE(e, n) x[e] = v;
}
__global__ void pair_cores_kernel(const double* A, int l, int r, const double* W,
                                  int c, int d, int sum_bit, double* out,
                                  InstOff io) {
  const long o_ = io.of(blockIdx.z);
  A = shifted(A, o_);
  W = shifted(W, o_);
  out = shifted(out, o_);
  const long R = (long)r * d;
  const long n = (long)l * c * (sum_bit ? 1 : 2) * R;
  GRID_STRIDE(e, n) {
    const long col = e % R;
    const long b = col / d, ee = col % d;
    long t = e / R;
    if (sum_bit) {
      const long a = t / c, cc = t % c;
      out[e] = A[(a * 2) * r + b] * W[(cc * 2) * d + ee] +
               A[(a * 2 + 1) * r + b] * W[(cc * 2 + 1) * d + ee];
    } else {
      const long bit = t % 2;
      t /= 2;
      const long a = t / c, cc = t % c;
      out[e] = A[(a * 2 + bit) * r + b] * W[(cc * 2 + bit) * d + ee];
    }
  }
}

__global__ void dougherty_fields_kernel(const double* n, const double* P,
                                        const double* H, long nx, double* v0,
                                        double* T, InstOff io) {
  const long o_ = io.of(blockIdx.z);
  n = shifted(n, o_);
  P = shifted(P, o_);
  H = shifted(H, o_);
  v0 = shifted(v0, o_);
  T = shifted(T, o_);
  GRID_STRIDE(e, nx) {
    const double m = n[e];
    const double u = (m != 0.0) ? P[e] / m : 0.0;
    v0[e] = u;
    T[e] = (m != 0.0) ? 2.0 * H[e] / m - u * u : 0.0;
  }
}

__global__ void copy_doubles_kernel(double* dst, const double* src, long n,
                                    InstOff io) {
  const long o_ = io.of(blockIdx.z);
  dst = shifted(dst, o_);
  src = shifted(src, o_);
  GRID_STRIDE(e, n) dst[e] = src[e];
}
__global__ void fill_int_kernel(int* x, long n, int v, InstOff io) {
  x = shifted(x, io.of(blockIdx.z));
  GRID_STRIDE(e, n) x[e] = v;
}

}  // namespace

void swap01(hipStream_t s, const double* in, int d0, int d1, long inner,
            double* out) {
  long n = (long)d0 * d1 * inner;
  if (n <= 0) return;
  MPSV_CHECK((long)d0 * d1 <= 65535, kEinval, "swap01: too many index pairs");
  const int gx = std::min(64, ceil_div(inner, 256));
  hipLaunchKernelGGL(swap01_kernel, dim3(gx, d0 * d1, inst_count()), dim3(256), 0, s, in, d0,
                     d1, inner, out, inst_off());
  MPSV_LAUNCHED();
}

void copy2d(hipStream_t s, int rows, int cols, double alpha, const double* src,
            long lds, double* dst, long ldd) {
  long n = (long)rows * cols;
  if (n <= 0) return;
  hipLaunchKernelGGL(copy2d_kernel, dim3(grid_for(n), 1, inst_count()), dim3(256), 0, s, rows,
                     cols, alpha, src, lds, dst, ldd, inst_off());
  MPSV_LAUNCHED();
}

void sum_physical(hipStream_t s, const double* in, int l, int r, double* out) {
  long n = (long)l * r;
  hipLaunchKernelGGL(sum_physical_kernel, dim3(grid_for(n), 1, inst_count()), dim3(256), 0, s,
                     in, l, r, out, inst_off());
  MPSV_LAUNCHED();
}

void scale_rows(hipStream_t s, const double* in, int rows, long len,
                const double* d, bool inverse, double* out) {
  const long n = (long)rows * len;
  if (n <= 0) return;
  hipLaunchKernelGGL(scale_rows_kernel, dim3(grid_for(n), 1, inst_count()), dim3(256), 0, s, in,
                     rows, len, d, inverse ? 1 : 0, out, inst_off());
  MPSV_LAUNCHED();
}

void identity(hipStream_t s, double* A, int n) {
  const long total = (long)n * n;
  if (total <= 0) return;
  hipLaunchKernelGGL(identity_kernel, dim3(grid_for(total), 1, inst_count()), dim3(256), 0, s, A, n, inst_off());
  MPSV_LAUNCHED();
}

void reverse_core(hipStream_t s, const double* in, int l, int r, double* out) {
  const long n = 2L * l * r;
  hipLaunchKernelGGL(reverse_core_kernel, dim3(grid_for(n), 1, inst_count()), dim3(256), 0, s,
                     in, l, r, out, inst_off());
  MPSV_LAUNCHED();
}

void chain_to_grid(hipStream_t s, const double* in, int Lx, int Lv, bool rx,
                   bool rv, double* out) {
  const long n = 1L << (Lx + Lv);
  hipLaunchKernelGGL(chain_to_grid_kernel, dim3(grid_for(n), 1, inst_count()), dim3(256), 0, s,
                     in, Lx, Lv, rx ? 1 : 0, rv ? 1 : 0, out, inst_off());
  MPSV_LAUNCHED();
}

void kron_embed(hipStream_t s, const double* A, int l, int P, int r, int d,
                int mode, double* out) {
  long n = (long)l * d * P * r * d;
  hipLaunchKernelGGL(kron_embed_kernel, dim3(grid_for(n), 1, inst_count()), dim3(256), 0, s, A,
                     l, P, r, d, mode, out, inst_off());
  MPSV_LAUNCHED();
}

void diag_mpo_site(hipStream_t s, const double* E, int l, int r, double scale,
                   double* W) {
  long n = (long)l * 4 * r;
  hipLaunchKernelGGL(diag_mpo_kernel, dim3(grid_for(n), 1, inst_count()), dim3(256), 0, s, E, l,
                     r, scale, W, inst_off());
  MPSV_LAUNCHED();
}

void mpo_left_matrix(hipStream_t s, const double* W, int wl, int wr,
                     double* Wmat) {
  long n = (long)4 * wl * wr;
  hipLaunchKernelGGL(mpo_left_matrix_kernel, dim3(grid_for(n), 1, inst_count()), dim3(256), 0, s,
                     W, wl, wr, Wmat, inst_off());
  MPSV_LAUNCHED();
}

void deinterleave(hipStream_t s, const double* in, int L, double* out) {
  long n = 1L << (2 * L);
  hipLaunchKernelGGL(deinterleave_kernel, dim3(grid_for(n), 1, inst_count()), dim3(256), 0, s,
                     in, L, out, inst_off());
  MPSV_LAUNCHED();
}

void count_nonfinite(hipStream_t s, const double* x, long n, int* flag) {
  if (n <= 0) return;
  hipLaunchKernelGGL(count_nonfinite_kernel, dim3(grid_for(n), 1, inst_count()), dim3(256), 0,
                     s, x, n, flag, inst_off());
  MPSV_LAUNCHED();
}

void sum_squares(hipStream_t s, const double* x, long n, double scale,
                 double* out) {
  hipLaunchKernelGGL(sum_squares_kernel, dim3(1, 1, inst_count()), dim3(256), 0, s, x, n, scale,
                     out, inst_off());
  MPSV_LAUNCHED();
}

void fill(hipStream_t s, double* x, long n, double v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n), 1, inst_count()), dim3(256), 0, s, x, n, v, inst_off());
  MPSV_LAUNCHED();
}

void pair_cores(hipStream_t s, const double* A, int l, int r, const double* W,
                int c, int d, bool sum_bit, double* out) {
  const long n = (long)l * c * (sum_bit ? 1 : 2) * r * d;
  if (n <= 0) return;
  hipLaunchKernelGGL(pair_cores_kernel, dim3(grid_for(n), 1, inst_count()), dim3(256), 0,
                     s, A, l, r, W, c, d, sum_bit ? 1 : 0, out, inst_off());
  MPSV_LAUNCHED();
}

void dougherty_fields(hipStream_t s, const double* n, const double* P,
                      const double* H, long nx, double* v0, double* T) {
  if (nx <= 0) return;
  hipLaunchKernelGGL(dougherty_fields_kernel, dim3(grid_for(nx), 1, inst_count()),
                     dim3(256), 0, s, n, P, H, nx, v0, T, inst_off());
  MPSV_LAUNCHED();
}

void copy_doubles(hipStream_t s, double* dst, const double* src, long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(copy_doubles_kernel, dim3(grid_for(n), 1, inst_count()), dim3(256), 0,
                     s, dst, src, n, inst_off());
  MPSV_LAUNCHED();
}

void fill_int(hipStream_t s, int* x, long n, int v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_int_kernel, dim3(grid_for(n), 1, inst_count()), dim3(256), 0, s, x, n,
                     v, inst_off());
  MPSV_LAUNCHED();
}

}  // namespace mpsv
