// FP64 strided batched GEMM on MFMA (see gemm.hip).
#pragma once
#include "arena.hpp"
#include "common.hpp"

namespace mpsv {

// C[b] = alpha * A[b] * B[b] + beta * C[b]; A is M x K, B is K x N.
// beta == 0 never reads C.  Stream-ordered, no synchronisation.  prec 0:
// FP64; 1: products of FP32-rounded operands, 2: of BF16-rounded operands,
// both accumulated in FP32 on the matrix cores (results stored in FP64).
// ws: workspace for split-K partial products (allocated and released
// inside the call); without one K is never split.  Every lock-step
// instance of the calling thread's lanes is covered.
void gemm(hipStream_t s, int M, int N, int K, double alpha, CMatView A,
          CMatView B, double beta, MatView C, int batch = 1, int prec = 0,
          Arena* ws = nullptr);

// C[b] = beta * C[b] (beta == 0 writes zeros without reading).
void scale_matrix(hipStream_t s, int M, int N, double beta, MatView C,
                  int batch = 1);

}  // namespace mpsv
