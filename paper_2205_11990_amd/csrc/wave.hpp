// Cross-lane sums of FP64 values inside one 64-lane wavefront (gfx950).
//
// Within a row of 16 lanes the data move with DPP; between rows with the
// gfx950 permlane swaps, which exchange whole 16- or 32-lane halves of two
// registers.  A swap of two different registers both reduces and packs: the
// sum of its two outputs holds the first value, reduced over lanes l and
// l^32, in lanes 0-31 and the second value in lanes 32-63.  Reducing N
// values therefore costs about N/2 + N/4 swaps plus N/4 row sums instead of
// N full reductions.
#pragma once
#include <hip/hip_runtime.h>

namespace mpsv {
namespace wave {

// Row-local DPP move of a double.  The patterns used here read valid lanes
// everywhere, so no "old" value is needed (and none is initialised).
template <int CTRL>
__device__ inline double dpp(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Sum over each aligned group of 4 lanes; every lane of the group gets it.
__device__ inline double sum4(double v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  return v;
}

// Sum over each aligned group of 8 lanes; every lane of the group gets it.
__device__ inline double sum8(double v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror: lane i <-> 7-i within 8
  return v;
}

// Sum over each aligned row of 16 lanes; every lane of the row gets it.
__device__ inline double sum16(double v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror: lane i <-> 7-i within 8
  v += dpp<0x140>(v);  // row_mirror: lane i <-> 15-i within 16
  return v;
}

// lanes 0-31: a(l) + a(l+32);  lanes 32-63: b(l-32) + b(l)
__device__ inline double swap32_sum(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

// rows (16 lanes) 0,1: a(row 0) + a(row 1) and b(row 0) + b(row 1);
// rows 2,3: a(row 2) + a(row 3) and b(row 2) + b(row 3)
__device__ inline double swap16_sum(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

__device__ inline double read_lane(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Sum over all 64 lanes; every lane gets it (a wave-uniform value).
__device__ inline double sum64(double v) {
  v = swap32_sum(v, v);
  v = swap16_sum(v, v);
  return read_lane(sum16(v), 0);
}

// p[i] <- sum over the 64 lanes of p[i], wave-uniform, for N in {1,2,4,8}.
template <int N>
__device__ inline void sums(double (&p)[N]) {
  if constexpr (N == 1) {
    p[0] = sum64(p[0]);
  } else if constexpr (N == 2) {
    double s = swap32_sum(p[0], p[1]);  // rows 0,1: p0; rows 2,3: p1
    s = sum16(swap16_sum(s, s));
    p[0] = read_lane(s, 0);
    p[1] = read_lane(s, 32);
  } else {
    static_assert(N % 4 == 0, "N must be 1, 2 or a multiple of 4");
    double t[N / 4];
#pragma unroll
    for (int i = 0; i < N / 4; ++i) {
      const double s0 = swap32_sum(p[4 * i], p[4 * i + 1]);
      const double s1 = swap32_sum(p[4 * i + 2], p[4 * i + 3]);
      // rows: p[4i], p[4i+2], p[4i+1], p[4i+3]
      t[i] = sum16(swap16_sum(s0, s1));
    }
#pragma unroll
    for (int i = 0; i < N / 4; ++i) {
      p[4 * i] = read_lane(t[i], 0);
      p[4 * i + 2] = read_lane(t[i], 16);
      p[4 * i + 1] = read_lane(t[i], 32);
      p[4 * i + 3] = read_lane(t[i], 48);
    }
  }
}

// Workgroup barrier that orders LDS traffic only: waits for this wave's
// LDS operations (lgkmcnt 0) but not for its global stores, then
// s_barrier.  Loops whose global stores
// are read only by later kernels use it so that every step does not wait
// for the store round trip to memory.
__device__ inline void lds_barrier() {
  // the memory clobber keeps the compiler from moving memory accesses
  // across the barrier
  __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

}  // namespace wave
}  // namespace mpsv
