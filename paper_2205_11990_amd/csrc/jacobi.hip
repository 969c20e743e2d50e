// One-sided (Hestenes) Jacobi SVD of a small square triangular factor on
// one workgroup.  The rotations act on the columns of B = R^T; they
// converge to v_i sigma_i, the right singular vectors of the matrix R came
// from, scaled by its singular values.  Working on the transpose of the
// triangular factor needs far fewer sweeps than working on the factor
// itself (about 9 against 22 on the matrices of the compression sweep).
// The rotations themselves are not accumulated: the caller forms the left
// factor as X V (one GEMM), so the kernel keeps only B on chip.
//
// Layout: the columns are held in registers.  A node is an aligned group of
// NL lanes (8 above 32 columns, 16 below); it owns two columns (a, b),
// NL * RPT rows each, RPT per lane.  Each step orthogonalises the pair of
// every node at once (inner products reduced with DPP moves inside the
// group), then columns move between nodes.  With 8-lane nodes a 128-column
// factor takes 8 waves (two per SIMD) and the per-pair work of a step (the
// reduction, the angle, the moves) is shared by 16 rows per lane: a sweep
// at 128 columns takes 0.093 ms against 0.104 with 16-lane nodes and 0.104
// with 4-lane nodes (one wave per SIMD, no latency hiding).
//
// Ordering: a hypercube ordering of the N = 2^d nodes that meets every pair
// exactly once per sweep in 2N - 1 steps, built recursively: pair all
// columns inside each half-cube, exchange one column per node across the
// top dimension so that every node holds one column of each half, then
// let the second columns walk through the cube along a Gray code (one
// dimension per step), which brings every column of one half next to every
// column of the other.  The low log2(64 / NL) node bits select lanes
// inside a wave, so moves along those dimensions are lane permutations
// (ds_swizzle / ds_bpermute through the LDS crossbar, which leaves the
// vector ALU free); only moves along the wave bits go through LDS memory,
// with a barrier.  At 128 columns and 8-lane nodes 112 of the 126 moves of
// a sweep stay inside the waves.
//
// Squared column norms are carried with the columns and updated with each
// rotation.  Columns below 1e-15 of the Frobenius norm are numerical zeros
// and are never rotated.
//
// From 129 to 256 columns the matrix no longer fits in one compute unit:
// four workgroups of 32 nodes each hold a quarter of the 128 nodes (rows up
// to 256, 16 per lane), and the two top cube dimensions join them.  Only
// six moves per sweep cross them; they go through global memory, with a
// rendezvous of all workgroups on release/acquire flags at device scope.
// Each wait is bounded; a rendezvous that times out ends every workgroup
// and is reported instead of a result.  The end-of-sweep decision sums all
// workgroups' convergence flags, so all of them run the same sweeps.
//
// On exit: singular values are the column norms, sorted descending (ties by
// index), the truncation rank D follows the rule min(cap, smallest D' whose
// relative discarded weight is <= tol) (eq. 5 with the i = D+1 reading), and
// Vt (D x k) holds the kept right singular vectors (normalised columns).
#include <cmath>
#include <cstdlib>
#include <mutex>

#include "jacobi.hpp"
#include "mps_kernels.hpp"
#include "wave.hpp"

namespace mpsv {

namespace {

constexpr int MAXT = 1024;  // 64 nodes of 16 lanes

// Rotation that orthogonalises columns with Gram [[a,g],[g,b]] (Rutishauser's
// formulas): t = tan(theta) is the smaller root of t^2 + 2 z t - 1 = 0 with
// z = (b - a) / (2g), cs = 1 / sqrt(1 + t^2), sn = cs t.  The rotation is
// orthogonal whatever t is, so t comes from the hardware estimates (about
// 5e-8 relative, which only leaves a residual cosine of that order times
// the one removed, cleaned up by the following sweeps); cs must satisfy
// cs^2 + sn^2 = 1 to rounding and is refined by two Newton steps.  No
// branch: for |z| beyond 1e154, z^2 overflows and t becomes 0, an angle
// below 1e-154 that would not change a double anyway (the rotation test
// keeps |z| far below that).
__device__ inline void rotation(double a, double b, double g, double& cs,
                                double& sn) {
  const double z = (b - a) * __builtin_amdgcn_rcp(2.0 * g);
  const double az = fabs(z);
  const double t =
      copysign(__builtin_amdgcn_rcp(az + __builtin_amdgcn_sqrt(fma(z, z, 1.0))), z);
  const double w = fma(t, t, 1.0);
  double y = __builtin_amdgcn_rsq(w);
  y = fma(y, 0.5 * fma(-w * y, y, 1.0), y);
  y = fma(y, 0.5 * fma(-w * y, y, 1.0), y);
  cs = y;
  sn = y * t;
}

// Value of the same lane in the DPP row (node) row ^ (1 << DIM), DIM < 2:
// a lane permutation through the LDS crossbar (no LDS memory, no VALU
// issue slots): ds_swizzle with xor mask 16 inside each half-wave, or
// ds_bpermute to lane ^ 32.
template <int DIM>
__device__ inline int row_swap(int v) {
  if constexpr (DIM == 0) {
    // bit mode: and_mask 0x1f, or_mask 0, xor_mask 0x10
    return __builtin_amdgcn_ds_swizzle(v, 0x401F);
  } else {
    const int lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    return __builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, v);
  }
}

template <int DIM>
__device__ inline double row_swap(double v) {
  const int lo = row_swap<DIM>(__double2loint(v));
  const int hi = row_swap<DIM>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// A column travelling between nodes: data, squared norm and column index.
template <int RPT>
struct Col {
  double v[RPT];
  double n;
  int id;
};

// Value of lane (lane ^ LX) for LX in {4, 8, 16, 32}: ds_swizzle in bit mode
// (and mask 0x1f, xor mask LX) inside each half-wave, ds_bpermute across
// the halves.  Both go through the LDS crossbar and leave the vector ALU
// free.
template <int LX>
__device__ inline int lane_swap(int v) {
  static_assert(LX == 4 || LX == 8 || LX == 16 || LX == 32, "lane xor 4 .. 32");
  if constexpr (LX < 32) {
    return __builtin_amdgcn_ds_swizzle(v, 0x1F | (LX << 10));
  } else {
    const int lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    return __builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, v);
  }
}

template <int LX>
__device__ inline double lane_swap(double v) {
  const int lo = lane_swap<LX>(__double2loint(v));
  const int hi = lane_swap<LX>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

template <int LX, int RPT>
__device__ inline void swap_lanes(const Col<RPT>& send, Col<RPT>& recv) {
#pragma unroll
  for (int r = 0; r < RPT; ++r) recv.v[r] = lane_swap<LX>(send.v[r]);
  recv.n = lane_swap<LX>(send.n);
  recv.id = lane_swap<LX>(send.id);
}

// Sum over the NL lanes of a node (aligned groups of 4, 8 or 16 lanes).
template <int NL>
__device__ inline double node_sum(double v) {
  if constexpr (NL == 16) return wave::sum16(v);
  else if constexpr (NL == 8) return wave::sum8(v);
  else return wave::sum4(v);
}

// The column `send` of node x goes to node x ^ (1 << dim); returns the one
// arriving from there.  Nodes of NL lanes: the low log2(64 / NL) node bits
// select lanes of one wave (lane xor NL << dim, through the crossbar); the
// others select waves, and the column passes through the LDS buffer `xb`
// (one barrier).
template <int RPT, int NL>
__device__ inline void exchange(const Col<RPT>& send, Col<RPT>& recv, int dim,
                                int x, int lig, int N, int& par, double* xb,
                                double* xn, int* xi) {
  if (dim == 0) {
    swap_lanes<NL, RPT>(send, recv);
    return;
  }
  if (dim == 1) {
    swap_lanes<2 * NL, RPT>(send, recv);
    return;
  }
  if constexpr (NL <= 8) {
    if (dim == 2) {
      swap_lanes<4 * NL, RPT>(send, recv);
      return;
    }
  }
  if constexpr (NL == 4) {
    if (dim == 3) {
      swap_lanes<32, RPT>(send, recv);
      return;
    }
  }
  const int pb = par;
  par ^= 1;
  double* dst = xb + (long)(pb * N + x) * RPT * NL;
#pragma unroll
  for (int r = 0; r < RPT; ++r) dst[r * NL + lig] = send.v[r];
  if (lig == 0) {
    xn[pb * 64 + x] = send.n;
    xi[pb * 64 + x] = send.id;
  }
  __syncthreads();
  const int y = x ^ (1 << dim);
  const double* src = xb + (long)(pb * N + y) * RPT * NL;
#pragma unroll
  for (int r = 0; r < RPT; ++r) recv.v[r] = src[r * NL + lig];
  recv.n = xn[pb * 64 + y];
  recv.id = xi[pb * 64 + y];
}

// info: [0] D, [1] discarded weight, [2] sweeps, [3] converged, [4] steps
// Xr: k x k row-major triangular factor; the Jacobi columns are its rows.
// Output Vt[d][i] = column perm(d) / sigma_d.  Nodes of NL lanes, RPT rows
// per lane (NL * RPT >= k).
template <int RPT, int NL>
__global__ __launch_bounds__(64 * NL) void jacobi_hc_kernel(
    const double* __restrict__ Xr, int k, long ldx, int d, int max_sweeps,
    int cap, double tol, double* __restrict__ Vt, double* __restrict__ sigbuf,
    int* __restrict__ perm_out, double* __restrict__ info, InstOff io) {
  static_assert(NL == 4 || NL == 8 || NL == 16, "nodes of 4, 8 or 16 lanes");
  {
    const long o_ = io.of(blockIdx.z);
    Xr = shifted(Xr, o_);
    Vt = shifted(Vt, o_);
    sigbuf = shifted(sigbuf, o_);
    perm_out = shifted(perm_out, o_);
    info = shifted(info, o_);
  }
  extern __shared__ double smem[];
  __shared__ double red[MAXT / 64];
  __shared__ double xn[2 * 64];
  __shared__ int xi[2 * 64];
  __shared__ int sweep_any;
  __shared__ int Dsh;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int x = tid / NL, lig = tid % NL;
  const int N = 1 << d;

  // node x starts with columns 2x and 2x+1; indices >= k are zero padding
  Col<RPT> A, B;
  A.id = 2 * x;
  B.id = 2 * x + 1;
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = lig + NL * r;
    A.v[r] = (A.id < k && i < k) ? Xr[(long)A.id * ldx + i] : 0.0;
    B.v[r] = (B.id < k && i < k) ? Xr[(long)B.id * ldx + i] : 0.0;
    sa = fma(A.v[r], A.v[r], sa);
    sb = fma(B.v[r], B.v[r], sb);
  }
  A.n = node_sum<NL>(sa);
  B.n = node_sum<NL>(sb);
  // Frobenius norm of the whole matrix; the columns are scaled to unit
  // Frobenius norm (undone on the singular values at the end), so that the
  // products below neither overflow nor underflow
  double part = (lig == 0) ? A.n + B.n : 0.0;
  part = wave::sum64(part);
  if ((tid & 63) == 0) red[tid >> 6] = part;
  __syncthreads();
  double normF2 = 0.0;
  for (int w = 0; w < nthr / 64; ++w) normF2 += red[w];
  const double scale = normF2 > 0.0 ? 1.0 / sqrt(normF2) : 1.0;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    A.v[r] *= scale;
    B.v[r] *= scale;
  }
  A.n *= scale * scale;
  B.n *= scale * scale;
  const double negl = 1e-30;
  // A pair is rotated when its cosine |g| / (|a| |b|) exceeds eps.  The
  // iteration stops after the first sweep in which no cosine exceeded conv
  // (its rotations are still applied).  Cyclic Jacobi converges
  // quadratically: once every rotation angle of a sweep is below conv, the
  // rotations that follow the visit of a pair can restore at most about
  // 2k conv^2 < 3e-14 of its cosine, so the sweep that would only confirm
  // convergence is skipped.  The threshold also tolerates pairs that
  // stagnate at rounding level near the numerical null space.
  const double eps2 = 1e-28, conv2 = 1e-16;

  // One step on the pair (P, Q) of every node.  The update is skipped by
  // the whole wave when none of its nodes rotates (a scalar branch); inside
  // it, nodes that do not rotate apply cs = 1, sn = 0, which leaves their
  // columns and norms exactly unchanged.  Squared norms follow the rotation
  // by formula; where one of them falls below 1e-8 of the pair's total (its
  // rounding error could then exceed 1e-8 of it) the norms are recomputed.
  auto pair_step = [&](Col<RPT>& P, Col<RPT>& Q) __attribute__((always_inline)) {
    // four independent partial sums shorten the dependency chain
    double gp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < RPT; ++r) gp[r & 3] = fma(P.v[r], Q.v[r], gp[r & 3]);
    const double g = node_sum<NL>((gp[0] + gp[1]) + (gp[2] + gp[3]));
    const double ab = P.n * Q.n, g2 = g * g;
    const bool rot = g2 > eps2 * ab && fmin(P.n, Q.n) > negl;
    if (__builtin_amdgcn_ballot_w64(rot) == 0) return;
    double cs, sn;
    rotation(P.n, Q.n, g, cs, sn);
    cs = rot ? cs : 1.0;
    sn = rot ? sn : 0.0;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const double u = P.v[r], v = Q.v[r];
      P.v[r] = cs * u - sn * v;
      Q.v[r] = sn * u + cs * v;
    }
    // the new squared norms of the rotated pair, exact in exact arithmetic
    // for the cs, sn applied
    const double c2 = cs * cs, s2 = sn * sn, csg = 2.0 * cs * sn * g;
    const double na = fma(c2, P.n, fma(s2, Q.n, -csg));
    const double nb = fma(s2, P.n, fma(c2, Q.n, csg));
    if (rot && fmin(na, nb) < 1e-8 * (P.n + Q.n)) {
      double sa2 = 0.0, sb2 = 0.0;
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        sa2 = fma(P.v[r], P.v[r], sa2);
        sb2 = fma(Q.v[r], Q.v[r], sb2);
      }
      P.n = node_sum<NL>(sa2);
      Q.n = node_sum<NL>(sb2);
    } else {
      P.n = na;
      Q.n = nb;
    }
    if (rot && lig == 0 && g2 > conv2 * ab) sweep_any = 1;
  };

  double* xb = smem;
  int par = 0;
  int sweep = 0, converged = 0, steps = 0;
  Col<RPT> R;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) sweep_any = 0;
    __syncthreads();
    pair_step(A, B);
    ++steps;
    for (int l = 1; l <= d; ++l) {
      // across dimension l-1: nodes of the lower half give b, those of the
      // upper half give a, so afterwards a holds lower-half columns and b
      // upper-half columns everywhere
      const int dim = l - 1;
      const bool up = (x >> dim) & 1;
      exchange<RPT, NL>(up ? A : B, R, dim, x, lig, N, par, xb, xn, xi);
      if (up) A = R; else B = R;
      pair_step(A, B);
      ++steps;
      // the b columns walk along a Gray code over the l lower dimensions;
      // two moves per iteration let B and R trade roles without copies
      const int last = (1 << l) - 1;
      int t = 1;
      for (; t + 1 <= last; t += 2) {
        exchange<RPT, NL>(B, R, __builtin_ctz(t), x, lig, N, par, xb, xn, xi);
        pair_step(A, R);
        exchange<RPT, NL>(R, B, __builtin_ctz(t + 1), x, lig, N, par, xb, xn, xi);
        pair_step(A, B);
        steps += 2;
      }
      if (t == last) {
        exchange<RPT, NL>(B, R, __builtin_ctz(t), x, lig, N, par, xb, xn, xi);
        B = R;
        pair_step(A, B);
        ++steps;
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

  // columns back into LDS by index: M[j][i], odd leading dimension
  __syncthreads();
  const int lda = k | 1;
  double* M = smem;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = lig + NL * r;
    if (i < k) {
      if (A.id < k) M[(long)A.id * lda + i] = A.v[r] / scale;
      if (B.id < k) M[(long)B.id * lda + i] = B.v[r] / scale;
    }
  }
  {
    // exact final norms, in the units of the input
    double sa2 = 0.0, sb2 = 0.0;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      sa2 = fma(A.v[r], A.v[r], sa2);
      sb2 = fma(B.v[r], B.v[r], sb2);
    }
    sa2 = node_sum<NL>(sa2);
    sb2 = node_sum<NL>(sb2);
    const double inv = 1.0 / scale;
    if (lig == 0) {
      if (A.id < k) sigbuf[k + A.id] = sqrt(sa2) * inv;
      if (B.id < k) sigbuf[k + B.id] = sqrt(sb2) * inv;
    }
  }
  __syncthreads();
  // rank-sort the singular values (ties by index)
  for (int j = tid; j < k; j += nthr) {
    const double sj = sigbuf[k + j];
    int rank = 0;
    for (int q = 0; q < k; ++q) {
      const double sq = sigbuf[k + q];
      rank += (sq > sj || (sq == sj && q < j)) ? 1 : 0;
    }
    perm_out[rank] = j;
    sigbuf[rank] = sj;
  }
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int i = 0; i < k; ++i) tot += sigbuf[i] * sigbuf[i];
    const int capd = cap < k ? cap : k;
    int D;
    if (tol <= 0.0) {
      D = capd;  // the cap alone decides, whatever the values (a zero block too)
    } else if (tot <= 0.0) {
      D = 1;
    } else {
      // smallest D' >= 1 whose discarded tail (summed from the smallest
      // value) is <= tol^2
      double acc = 0.0;
      int best = k;
      for (int Dp = k - 1; Dp >= 1; --Dp) {
        acc += sigbuf[Dp] * sigbuf[Dp] / tot;
        if (acc <= tol * tol) best = Dp; else break;
      }
      D = best < capd ? best : capd;
    }
    if (D < 1) D = 1;
    double disc2 = 0.0;
    for (int i = D; i < k; ++i) disc2 += sigbuf[i] * sigbuf[i];
    Dsh = D;
    info[0] = (double)D;
    info[1] = (tot > 0.0) ? sqrt(disc2 / tot) : 0.0;
    info[2] = (double)sweep;
    info[3] = (double)converged;
    info[4] = (double)steps;
  }
  __syncthreads();
  const int D = Dsh;
  // Vt[d][i] = column perm(d) / sigma_d; numerical zeros give zero rows
  for (long e = tid; e < (long)D * k; e += nthr) {
    const long dd = e / k, i = e % k;
    const double sd = sigbuf[dd];
    Vt[e] = (sd * sd > negl * normF2) ? M[(long)perm_out[dd] * lda + i] / sd : 0.0;
  }
}

// ------------------------------------------ several workgroups (k <= 256)

constexpr int kMaxWgs = 8;                       // most workgroups of a split
constexpr long kSpinLimit = 1L << 22;            // polls per wait, ~1 s

// A split Jacobi: 2^NLOG nodes over 2^GLOG workgroups, RPT rows per lane.
template <int NLOG, int GLOG, int RPT>
struct Split {
  static constexpr int wgs = 1 << GLOG;
  static constexpr int local = NLOG - GLOG;       // node bits inside a workgroup
  static constexpr int nodes = 1 << local;        // nodes per workgroup
  static constexpr int threads = 16 * nodes;
  static constexpr int col = 16 * RPT;            // doubles per column
  static constexpr int stride = col + 16;         // padded LDS column slot
  static constexpr int slots = wgs * 2 * nodes;   // exchange slots
  static_assert(local >= 2, "lane-row bits stay inside the workgroup");
  static_assert(wgs <= kMaxWgs, "too many workgroups");
};

// Global exchange area of the workgroups (see jacobi_ws_doubles); the
// slots alternate with the parity of the rendezvous number.
struct MultiWs {
  double* xg;   // [wg][parity][node][col] outgoing columns
  double* xn;   // [wg][parity][node] their squared norms
  double* val;  // [wg][parity] rendezvous payload
  int* xi;      // [wg][parity][node] their indices
  int* flags;   // [wg] last rendezvous published (zeroed before the launch)
};

__device__ inline void flag_publish(int* f, int v) {
  __hip_atomic_store(f, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int flag_read(int* f) {
  return __hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Rendezvous number `e` of all workgroups: every thread's earlier global
// stores become visible to the others, `mine` is published and the sum of
// all workgroups' values, taken in workgroup order (the same in each), is
// returned in `total`.  False, for the whole workgroup, when another
// workgroup does not arrive within the spin limit.  Since every workgroup
// waits for all others at each rendezvous, a slot written at rendezvous e
// has been read by everyone before any workgroup passes e + 1.
__device__ bool meet_all(const MultiWs& w, int wgs, int wg, int e, double mine,
                         double& total, int* sh_ok, double* sh_val) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    w.val[wg * 2 + (e & 1)] = mine;
    flag_publish(w.flags + wg, e);
    int ok = 1;
    for (int q = 0; q < wgs && ok; ++q) {
      if (q == wg) continue;
      long spins = 0;
      while (flag_read(w.flags + q) < e) {
        if (++spins > kSpinLimit) {
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(8);
      }
    }
    double t = 0.0;
    for (int q = 0; q < wgs && ok; ++q)
      t += (q == wg) ? mine : w.val[q * 2 + (e & 1)];
    *sh_ok = ok;
    *sh_val = t;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  total = *sh_val;
  return *sh_ok != 0;
}

// A value chosen by a per-lane condition.  Taking the operands by value
// makes both loads happen, so that a choice between two register-resident
// arrays never becomes a choice between their addresses (which would move
// the arrays to scratch memory).
__device__ inline double pick(bool c, double a, double b) { return c ? a : b; }
__device__ inline int pick(bool c, int a, int b) { return c ? a : b; }

// Info: [0] D, [1] discarded weight, [2] sweeps, [3] converged, [4] steps,
// [5] 1 if a rendezvous timed out.  Same inputs and outputs as
// jacobi_hc_kernel; launched as exactly S::wgs workgroups of S::threads
// threads.  Node bits 0-1 are lane rows, 2..local-1 waves, the rest the
// workgroup.
template <int NLOG, int GLOG, int RPT>
__global__ __launch_bounds__(16 << (NLOG - GLOG)) void jacobi_multi_kernel(
    const double* __restrict__ Xr, int k, long ldx, int max_sweeps, int cap,
    double tol, double* __restrict__ Vt, double* __restrict__ sigbuf,
    int* __restrict__ perm_out, double* __restrict__ info, MultiWs w,
    InstOff io) {
  using S = Split<NLOG, GLOG, RPT>;
  {
    // the workgroups of instance z meet in that instance's exchange area
    const long o_ = io.of(blockIdx.z);
    Xr = shifted(Xr, o_);
    Vt = shifted(Vt, o_);
    sigbuf = shifted(sigbuf, o_);
    perm_out = shifted(perm_out, o_);
    info = shifted(info, o_);
    w.xg = shifted(w.xg, o_);
    w.xn = shifted(w.xn, o_);
    w.val = shifted(w.val, o_);
    w.xi = shifted(w.xi, o_);
    w.flags = shifted(w.flags, o_);
  }
  constexpr int kMultiWgs = S::wgs;
  constexpr int kMultiLog = GLOG;
  constexpr int kMultiNodes = S::nodes;
  constexpr int kMultiLocal = S::local;
  constexpr int kMultiT = S::threads;
  constexpr int kMultiCol = S::col;
  constexpr int kMultiStride = S::stride;
  extern __shared__ double smem[];
  __shared__ double red[kMultiT / 64];
  __shared__ double lxn[kMultiNodes];
  __shared__ int lxi[kMultiNodes];
  __shared__ int sweep_any;
  __shared__ int sh_ok;
  __shared__ double sh_val;
  __shared__ int Dsh;
  const int wg = blockIdx.x;
  const int tid = threadIdx.x;
  const int x = tid >> 4, lig = tid & 15;
  const int gx = wg * kMultiNodes + x;
  int epoch = 0;

  Col<RPT> A, B;
  A.id = 2 * gx;
  B.id = 2 * gx + 1;
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = lig + 16 * r;
    A.v[r] = (A.id < k && i < k) ? Xr[(long)A.id * ldx + i] : 0.0;
    B.v[r] = (B.id < k && i < k) ? Xr[(long)B.id * ldx + i] : 0.0;
    sa = fma(A.v[r], A.v[r], sa);
    sb = fma(B.v[r], B.v[r], sb);
  }
  A.n = wave::sum16(sa);
  B.n = wave::sum16(sb);
  double part = (lig == 0) ? A.n + B.n : 0.0;
  part = wave::sum64(part);
  if ((tid & 63) == 0) red[tid >> 6] = part;
  __syncthreads();
  double mine = 0.0;
  for (int v = 0; v < kMultiT / 64; ++v) mine += red[v];
  double normF2 = 0.0;
  bool ok = meet_all(w, kMultiWgs, wg, ++epoch, mine, normF2, &sh_ok, &sh_val);
  const double scale = normF2 > 0.0 ? 1.0 / sqrt(normF2) : 1.0;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    A.v[r] *= scale;
    B.v[r] *= scale;
  }
  A.n *= scale * scale;
  B.n *= scale * scale;
  const double negl = 1e-30;
  const double eps2 = 1e-28, conv2 = 1e-16;

  auto pair_step = [&]() __attribute__((always_inline)) {
    double gp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < RPT; ++r) gp[r & 3] = fma(A.v[r], B.v[r], gp[r & 3]);
    const double g = wave::sum16((gp[0] + gp[1]) + (gp[2] + gp[3]));
    const double ab = A.n * B.n, g2 = g * g;
    const bool rot = g2 > eps2 * ab && fmin(A.n, B.n) > negl;
    // skipped by the whole wave when none of its nodes rotates; nodes that
    // do not rotate apply cs = 1, sn = 0 (no change)
    if (__builtin_amdgcn_ballot_w64(rot) == 0) return;
    double cs, sn;
    rotation(A.n, B.n, g, cs, sn);
    cs = rot ? cs : 1.0;
    sn = rot ? sn : 0.0;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const double u = A.v[r], v = B.v[r];
      A.v[r] = cs * u - sn * v;
      B.v[r] = sn * u + cs * v;
    }
    const double c2 = cs * cs, s2 = sn * sn, csg = 2.0 * cs * sn * g;
    const double na = fma(c2, A.n, fma(s2, B.n, -csg));
    const double nb = fma(s2, A.n, fma(c2, B.n, csg));
    if (rot && fmin(na, nb) < 1e-8 * (A.n + B.n)) {
      double sa2 = 0.0, sb2 = 0.0;
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        sa2 = fma(A.v[r], A.v[r], sa2);
        sb2 = fma(B.v[r], B.v[r], sb2);
      }
      A.n = wave::sum16(sa2);
      B.n = wave::sum16(sb2);
    } else {
      A.n = na;
      B.n = nb;
    }
    if (rot && lig == 0 && g2 > conv2 * ab) sweep_any = 1;
  };

  double* xb = smem;
  // Column a where `up`, else column b, of node gx goes to node
  // gx ^ (1 << dim) and is replaced by the one arriving from there.  The
  // choice can differ between lanes and waves, so it is made element by
  // element and every thread sends and receives in the same phase; the
  // columns never leave the registers except through the exchange buffer.
  auto send = [&](double* dst, double* dn, int* di, bool up)
      __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < RPT; ++r) dst[r * 16 + lig] = pick(up, A.v[r], B.v[r]);
    if (lig == 0) {
      *dn = pick(up, A.n, B.n);
      *di = pick(up, A.id, B.id);
    }
  };
  auto receive = [&](const double* src, const double* sn, const int* si,
                     bool up) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const double rcv = src[r * 16 + lig];
      A.v[r] = pick(up, rcv, A.v[r]);
      B.v[r] = pick(up, B.v[r], rcv);
    }
    const double rn = *sn;
    const int ri = *si;
    A.n = pick(up, rn, A.n);
    A.id = pick(up, ri, A.id);
    B.n = pick(up, B.n, rn);
    B.id = pick(up, B.id, ri);
  };
  auto move = [&](int dim, bool up) __attribute__((always_inline)) -> bool {
    if (dim <= 1) {
      // lane rows of one wave: a permutation through the LDS crossbar
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const double snd = pick(up, A.v[r], B.v[r]);
        const double rcv = dim == 0 ? row_swap<0>(snd) : row_swap<1>(snd);
        A.v[r] = pick(up, rcv, A.v[r]);
        B.v[r] = pick(up, B.v[r], rcv);
      }
      const double sn = pick(up, A.n, B.n);
      const int si = pick(up, A.id, B.id);
      const double rn = dim == 0 ? row_swap<0>(sn) : row_swap<1>(sn);
      const int ri = dim == 0 ? row_swap<0>(si) : row_swap<1>(si);
      A.n = pick(up, rn, A.n);
      A.id = pick(up, ri, A.id);
      B.n = pick(up, B.n, rn);
      B.id = pick(up, B.id, ri);
      return true;
    }
    if (dim < kMultiLocal) {
      // waves of one workgroup: through LDS
      const int y = x ^ (1 << dim);
      wave::lds_barrier();  // the previous move's reads are done
      send(xb + x * kMultiStride, lxn + x, lxi + x, up);
      wave::lds_barrier();
      receive(xb + y * kMultiStride, lxn + y, lxi + y, up);
      return true;
    }
    // node x of this workgroup and node x of workgroup wg ^ (1 << (dim - 5)),
    // through global memory
    const int e = epoch + 1;
    const int pw = wg ^ (1 << (dim - kMultiLocal));
    const long mine_s = (long)(wg * 2 + (e & 1)) * kMultiNodes + x;
    const long theirs = (long)(pw * 2 + (e & 1)) * kMultiNodes + x;
    send(w.xg + mine_s * kMultiCol, w.xn + mine_s, w.xi + mine_s, up);
    double unused;
    if (!meet_all(w, kMultiWgs, wg, ++epoch, 0.0, unused, &sh_ok, &sh_val)) return false;
    receive(w.xg + theirs * kMultiCol, w.xn + theirs, w.xi + theirs, up);
    return true;
  };

  int sweep = 0, converged = 0, steps = 0;
  for (; ok && sweep < max_sweeps; ++sweep) {
    if (tid == 0) sweep_any = 0;
    __syncthreads();
    pair_step();
    ++steps;
    for (int l = 1; ok && l <= kMultiLocal + kMultiLog; ++l) {
      // across dimension l-1 the lower node gives b and the upper node a,
      // so that a holds lower-half columns and b upper-half columns
      // everywhere; then the b columns walk along a Gray code
      const int dim = l - 1;
      ok = move(dim, (gx >> dim) & 1);
      pair_step();
      ++steps;
      for (int t = 1; ok && t < (1 << l); ++t) {
        ok = move(__builtin_ctz(t), false);
        pair_step();
        ++steps;
      }
    }
    if (!ok) break;
    __syncthreads();
    double any = 0.0;
    ok = meet_all(w, kMultiWgs, wg, ++epoch, sweep_any ? 1.0 : 0.0, any, &sh_ok, &sh_val);
    if (!ok) break;
    if (any == 0.0) {
      converged = 1;
      ++sweep;
      break;
    }
    __syncthreads();
  }

  // exact final norms in the units of the input, published to the others
  {
    double sa2 = 0.0, sb2 = 0.0;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      sa2 = fma(A.v[r], A.v[r], sa2);
      sb2 = fma(B.v[r], B.v[r], sb2);
    }
    sa2 = wave::sum16(sa2);
    sb2 = wave::sum16(sb2);
    const double inv = 1.0 / scale;
    if (ok && lig == 0) {
      if (A.id < k) sigbuf[k + A.id] = sqrt(sa2) * inv;
      if (B.id < k) sigbuf[k + B.id] = sqrt(sb2) * inv;
    }
  }
  double unused_total;
  if (ok) ok = meet_all(w, kMultiWgs, wg, ++epoch, 0.0, unused_total, &sh_ok, &sh_val);
  if (!ok) {
    if (tid == 0) {
      info[3] = 0.0;
      info[5] = 1.0;
    }
    return;
  }
  // every workgroup ranks all k values the same way
  double* sv = smem;                  // k values
  double* sorted = smem + 256;        // k sorted values
  int* rk = (int*)(smem + 512);       // rank of each column
  __syncthreads();
  for (int j = tid; j < k; j += kMultiT) sv[j] = sigbuf[k + j];
  __syncthreads();
  for (int j = tid; j < k; j += kMultiT) {
    const double sj = sv[j];
    int rank = 0;
    for (int q = 0; q < k; ++q) {
      const double sq = sv[q];
      rank += (sq > sj || (sq == sj && q < j)) ? 1 : 0;
    }
    rk[j] = rank;
    sorted[rank] = sj;
  }
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int i = 0; i < k; ++i) tot += sorted[i] * sorted[i];
    const int capd = cap < k ? cap : k;
    int D;
    if (tol <= 0.0) {
      D = capd;  // the cap alone decides, whatever the values (a zero block too)
    } else if (tot <= 0.0) {
      D = 1;
    } else {
      double acc = 0.0;
      int best = k;
      for (int Dp = k - 1; Dp >= 1; --Dp) {
        acc += sorted[Dp] * sorted[Dp] / tot;
        if (acc <= tol * tol) best = Dp; else break;
      }
      D = best < capd ? best : capd;
    }
    if (D < 1) D = 1;
    Dsh = D;
    if (wg == 0) {
      double disc2 = 0.0;
      for (int i = D; i < k; ++i) disc2 += sorted[i] * sorted[i];
      info[0] = (double)D;
      info[1] = (tot > 0.0) ? sqrt(disc2 / tot) : 0.0;
      info[2] = (double)sweep;
      info[3] = (double)converged;
      info[4] = (double)steps;
      info[5] = 0.0;
    }
  }
  __syncthreads();
  const int D = Dsh;
  if (wg == 0) {
    for (int j = tid; j < k; j += kMultiT) {
      sigbuf[j] = sorted[j];
      perm_out[rk[j]] = j;
    }
  }
  // Vt[d][i] = column perm(d) / sigma_d, written by the node holding it
  const double inv = 1.0 / scale;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int id = pick(c == 0, A.id, B.id);
    if (id >= k) continue;
    const int d = rk[id];
    if (d >= D) continue;
    const double sd = sorted[d];
    const double f = (sd * sd > negl * normF2) ? inv / sd : 0.0;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = lig + 16 * r;
      if (i < k) Vt[(long)d * k + i] = pick(c == 0, A.v[r], B.v[r]) * f;
    }
  }
}

// One-workgroup layout for k columns: 2^d nodes of nl lanes, rpt rows per
// lane (nl * rpt = 32, 64 or 128 rows).  Above 32 columns nodes are
// narrower than a 16-lane row: with nl lanes the per-pair work of a step
// (the reduction, the rotation angle, the column moves) is shared by
// 128 / nl rows per lane, fewer waves share each SIMD, and log2(64 / nl)
// node bits stay inside a wave.  MPSV_JACOBI_NODE_LANES (4, 8 or 16)
// overrides the default for timing.
struct Shape {
  int d, nodes, rpt, nl;
};

Shape shape_of(int k) {
  static const int lanes = [] {
    const char* e = std::getenv("MPSV_JACOBI_NODE_LANES");
    const int v = e ? std::atoi(e) : 8;
    return (v == 4 || v == 16) ? v : 8;
  }();
  Shape s;
  s.d = 2;
  while ((1 << s.d) * 2 < k) ++s.d;
  s.nodes = 1 << s.d;
  const int rows = k <= 32 ? 32 : (k <= 64 ? 64 : 128);
  s.nl = k <= 32 ? 16 : lanes;
  s.rpt = rows / s.nl;
  return s;
}

}  // namespace

namespace {

// Split chosen for k columns: 0 = one workgroup (jacobi_hc_kernel), else
// log2 of the workgroups.  Up to 128 columns one workgroup unless
// MPSV_JACOBI_SPLIT128 asks for 1 (2 workgroups) or 2 (4); above, four
// workgroups unless MPSV_JACOBI_SPLIT256 asks for 3 (8).
int split_of(int k) {
  static const int s128 = [] {
    const char* e = std::getenv("MPSV_JACOBI_SPLIT128");
    const int v = e ? std::atoi(e) : 0;
    return (v == 1 || v == 2) ? v : 0;
  }();
  static const int s256 = [] {
    const char* e = std::getenv("MPSV_JACOBI_SPLIT256");
    const int v = e ? std::atoi(e) : 2;
    return v == 3 ? 3 : 2;
  }();
  if (k > kJacobiOneWgCols) return s256;
  return k > 64 ? s128 : 0;
}

template <int NLOG, int GLOG, int RPT>
size_t split_lds() {
  using S = Split<NLOG, GLOG, RPT>;
  return (size_t)S::nodes * S::stride * sizeof(double);
}

template <int NLOG, int GLOG, int RPT>
size_t split_ws() {
  using S = Split<NLOG, GLOG, RPT>;
  // xg, xn, val; then xi and flags as ints
  return (size_t)S::slots * S::col + S::slots + 2 * S::wgs + (S::slots + S::wgs + 1) / 2 + 1;
}

template <int NLOG, int GLOG, int RPT>
void launch_split(hipStream_t s, const double* Xr, int k, long ldx, int cap,
                  double tol, int max_sweeps, double* Vt, double* sigbuf,
                  int* perm, double* info, double* ws) {
  using S = Split<NLOG, GLOG, RPT>;
  static std::once_flag once;
  std::call_once(once, [] {
    MPSV_HIP(hipFuncSetAttribute((const void*)jacobi_multi_kernel<NLOG, GLOG, RPT>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)kJacobiMaxLds));
  });
  // The workgroups of one decomposition wait for each other, so one launch
  // must never need more workgroups than the device holds at once: lock-step
  // instances are launched in groups that fit (one workgroup per compute
  // unit at this kernel's LDS, times the occupancy the runtime reports).
  static const int capacity = [] {
    int dev = 0, cus = 0, per = 0;
    MPSV_HIP(hipGetDevice(&dev));
    MPSV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    MPSV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per, (const void*)jacobi_multi_kernel<NLOG, GLOG, RPT>, S::threads,
        split_lds<NLOG, GLOG, RPT>()));
    return std::max(1, cus * std::max(1, per));
  }();
  MPSV_CHECK(S::wgs <= capacity, kEdevice,
             "split Jacobi: the device cannot hold the workgroups of one decomposition");
  const Lanes all = lanes();
  const int group = std::max(1, capacity / S::wgs);
  for (int i0 = 0; i0 < all.n; i0 += group) {
    LanesScope ls(Lanes{std::min(group, all.n - i0), all.first + (long)i0 * all.stride,
                        all.stride, all.tall_apply});
    MultiWs w;
    w.xg = ws;
    w.xn = w.xg + (size_t)S::slots * S::col;
    w.val = w.xn + S::slots;
    w.xi = (int*)(w.val + 2 * S::wgs);
    w.flags = w.xi + S::slots;
    fill_int(s, w.flags, S::wgs, 0);
    jacobi_multi_kernel<NLOG, GLOG, RPT><<<dim3(S::wgs, 1, inst_count()), dim3(S::threads),
                                           split_lds<NLOG, GLOG, RPT>(), s>>>(
        Xr, k, ldx, max_sweeps, cap, tol, Vt, sigbuf, perm, info, w, inst_off());
    MPSV_LAUNCHED();
  }
}

}  // namespace

int jacobi_split(int k) { return split_of(k); }

size_t jacobi_lds_bytes(int k) {
  switch (split_of(k)) {
    case 1: return split_lds<6, 1, 8>();
    case 2: return k > kJacobiOneWgCols ? split_lds<7, 2, 16>() : split_lds<6, 2, 8>();
    case 3: return split_lds<7, 3, 16>();
    default: break;
  }
  const Shape s = shape_of(k);
  const size_t xch = (size_t)2 * s.nodes * s.nl * s.rpt;
  const size_t cols = (size_t)k * (size_t)(k | 1);
  return (xch > cols ? xch : cols) * sizeof(double);
}

size_t jacobi_ws_doubles(int k) {
  switch (split_of(k)) {
    case 1: return split_ws<6, 1, 8>();
    case 2: return k > kJacobiOneWgCols ? split_ws<7, 2, 16>() : split_ws<6, 2, 8>();
    case 3: return split_ws<7, 3, 16>();
    default: return 0;
  }
}

void jacobi_svd(hipStream_t s, const double* Xr, int k, long ldx, int cap,
                double tol, int max_sweeps, double* Vt, double* sigbuf,
                int* perm, double* info, double* ws) {
  static std::once_flag once;
  std::call_once(once, [] {
    const void* fns[] = {(const void*)jacobi_hc_kernel<2, 16>,
                         (const void*)jacobi_hc_kernel<4, 16>,
                         (const void*)jacobi_hc_kernel<8, 16>,
                         (const void*)jacobi_hc_kernel<8, 8>,
                         (const void*)jacobi_hc_kernel<16, 8>,
                         (const void*)jacobi_hc_kernel<16, 4>,
                         (const void*)jacobi_hc_kernel<32, 4>};
    for (const void* f : fns)
      MPSV_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)kJacobiMaxLds));
  });
  MPSV_CHECK(k >= 1 && k <= kJacobiMaxCols, kEinval,
             "Jacobi SVD: matrix does not fit on chip");
  const size_t lds = jacobi_lds_bytes(k);
  MPSV_CHECK(lds <= kJacobiMaxLds, kEinval, "Jacobi SVD: LDS too small");
  const int split = split_of(k);
  if (split > 0) {
    MPSV_CHECK(ws != nullptr, kEinval, "Jacobi SVD: workspace missing");
    if (split == 1)
      launch_split<6, 1, 8>(s, Xr, k, ldx, cap, tol, max_sweeps, Vt, sigbuf, perm, info, ws);
    else if (split == 2 && k <= kJacobiOneWgCols)
      launch_split<6, 2, 8>(s, Xr, k, ldx, cap, tol, max_sweeps, Vt, sigbuf, perm, info, ws);
    else if (split == 2)
      launch_split<7, 2, 16>(s, Xr, k, ldx, cap, tol, max_sweeps, Vt, sigbuf, perm, info, ws);
    else
      launch_split<7, 3, 16>(s, Xr, k, ldx, cap, tol, max_sweeps, Vt, sigbuf, perm, info, ws);
    return;
  }
  const Shape sh = shape_of(k);
  const dim3 block(sh.nl * sh.nodes);
  MPSV_CHECK(sh.nl * sh.rpt >= k && (int)block.x <= 64 * sh.nl && block.x % 64 == 0,
             kEinval, "Jacobi SVD: bad layout");
  if (sh.nl == 16 && sh.rpt == 2)
    jacobi_hc_kernel<2, 16><<<dim3(1, 1, inst_count()), block, lds, s>>>(
        Xr, k, ldx, sh.d, max_sweeps, cap, tol, Vt, sigbuf, perm, info, inst_off());
  else if (sh.nl == 16 && sh.rpt == 4)
    jacobi_hc_kernel<4, 16><<<dim3(1, 1, inst_count()), block, lds, s>>>(
        Xr, k, ldx, sh.d, max_sweeps, cap, tol, Vt, sigbuf, perm, info, inst_off());
  else if (sh.nl == 16)
    jacobi_hc_kernel<8, 16><<<dim3(1, 1, inst_count()), block, lds, s>>>(
        Xr, k, ldx, sh.d, max_sweeps, cap, tol, Vt, sigbuf, perm, info, inst_off());
  else if (sh.nl == 8 && sh.rpt == 8)
    jacobi_hc_kernel<8, 8><<<dim3(1, 1, inst_count()), block, lds, s>>>(
        Xr, k, ldx, sh.d, max_sweeps, cap, tol, Vt, sigbuf, perm, info, inst_off());
  else if (sh.nl == 8)
    jacobi_hc_kernel<16, 8><<<dim3(1, 1, inst_count()), block, lds, s>>>(
        Xr, k, ldx, sh.d, max_sweeps, cap, tol, Vt, sigbuf, perm, info, inst_off());
  else if (sh.rpt == 16)
    jacobi_hc_kernel<16, 4><<<dim3(1, 1, inst_count()), block, lds, s>>>(
        Xr, k, ldx, sh.d, max_sweeps, cap, tol, Vt, sigbuf, perm, info, inst_off());
  else
    jacobi_hc_kernel<32, 4><<<dim3(1, 1, inst_count()), block, lds, s>>>(
        Xr, k, ldx, sh.d, max_sweeps, cap, tol, Vt, sigbuf, perm, info, inst_off());
  MPSV_LAUNCHED();
}

}  // namespace mpsv
