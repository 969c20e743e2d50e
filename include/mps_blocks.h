/*
 * mps_blocks.h -- the building blocks of the MPS time step, exposed so that
 * each part of the step can be checked on its own against a CPU reference.
 * Same conventions as mps_vlasov.h (device/host pointers, stream ordering,
 * status codes, mps_last_error()).  All matrices are row-major FP64.
 */
#ifndef MPS_BLOCKS_H
#define MPS_BLOCKS_H

#include "mps_vlasov.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C = alpha A B + beta C on the matrix cores; A: M x K (lda), B: K x N
 * (ldb), C: M x N (ldc); device pointers. */
mps_status mpsb_gemm(int32_t M, int32_t N, int32_t K, double alpha,
                     const double* A, int64_t lda, const double* B,
                     int64_t ldb, double beta, double* C, int64_t ldc,
                     hipStream_t stream);

/* mpsb_gemm with the precision of the MPO x MPS contractions: MPS_PREC_FP64,
 * MPS_PREC_FP32_CONTRACT or MPS_PREC_BF16_CONTRACT (operands rounded to FP32,
 * or to BF16 through FP32, FP32 accumulation on the matrix cores, result
 * stored in FP64).  MPS_EINVAL for other values. */
mps_status mpsb_gemm_prec(int32_t M, int32_t N, int32_t K, double alpha,
                          const double* A, int64_t lda, const double* B,
                          int64_t ldb, double beta, double* C, int64_t ldc,
                          int32_t precision, hipStream_t stream);

/* Strided batched GEMM: C[b] = alpha A[b] B[b] + beta C[b] for b < batch,
 * element (i, j) of operand X[b] at X + b*xbs + i*xrs + j*xcs (device,
 * strides in elements; A is M x K, B is K x N, C is M x N).  The contraction
 * kernel of the MPO x MPS products (SI, "Matrix-vector multiplication");
 * precision as in mpsb_gemm_prec.  Synchronises the stream. */
mps_status mpsb_gemm_strided(int32_t M, int32_t N, int32_t K, double alpha,
                             const double* A, int64_t ars, int64_t acs, int64_t abs_,
                             const double* B, int64_t brs, int64_t bcs, int64_t bbs,
                             double beta, double* C, int64_t crs, int64_t ccs,
                             int64_t cbs, int32_t batch, int32_t precision,
                             hipStream_t stream);

/* Householder QR of A (m x n, device, overwritten): on return the upper
 * trapezoid of A holds R (min(m,n) x n); if Q is not NULL it receives the
 * thin factor Q (m x min(m,n), device).  Used by the QR left sweep (SI,
 * "Canonicalization and Compression"). */
mps_status mpsb_qr(int32_t m, int32_t n, double* A, double* Q,
                   hipStream_t stream);

/* mpsb_qr with the reflector-application mode of a problem, tall_apply as
 * in mps_problem.tall_apply (0 or 1, else MPS_EINVAL).  With 1 a block of
 * more than 512 rows is factored in groups of four 16-column panels: each
 * panel updates only the rest of its group, and the group's 64 reflectors
 * reach the trailing columns (and later products with Q) as one compact-WY
 * block.  The same factorisation as mpsb_qr up to rounding (SI,
 * "Canonicalization and Compression"). */
mps_status mpsb_qr_tall(int32_t m, int32_t n, double* A, double* Q,
                        int32_t tall_apply, hipStream_t stream);

/* Truncated SVD of X (m x c, device, overwritten) with the rank rule of the
 * compression sweep: D = min(cap, smallest D' with relative discarded weight
 * <= tol), cap <= 0 meaning no cap (eq. 5).  Outputs (device): Vt (D x c),
 * US (m x D, columns u_i sigma_i), sig (min(m,c) singular values,
 * descending, may be NULL); host: *D, *discarded.  Vt and US must hold
 * min(m, c, cap) rows / columns. */
mps_status mpsb_svd_truncate(int32_t m, int32_t c, double* X, int32_t cap,
                             double tol, double* Vt, double* US, double* sig,
                             int32_t* D, double* discarded, hipStream_t stream);

/* mpsb_svd_truncate without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same arguments, outputs and kernels, with
 * every workspace taken from a fixed device array of 32 MiB per GPU, held
 * from the first call on a device until the process ends.  Shapes: m <= 2048,
 * c <= 2048 and min(m, c) <= 256, else MPS_EINVAL (a shape that still
 * exceeds the array fails with MPS_ENOMEM).  All calls on one GPU share the
 * array and would race if they overlapped; the library serialises them
 * (a call holds the array until its stream has completed).  The array
 * keeps the last call's contents: nothing in it needs to start at zero
 * (what must be zero is cleared by the call's own kernels). */
mps_status mpsb_svd_truncate_noalloc(int32_t m, int32_t c, double* X, int32_t cap,
                                     double tol, double* Vt, double* US, double* sig,
                                     int32_t* D, double* discarded,
                                     hipStream_t stream);

/* Compress an MPS (SI, "Canonicalization and Compression"): QR sweep left
 * to right then truncated SVD sweep right to left.  bonds_in / bonds_out:
 * host int32[n+1]; cores: packed device arrays (see mps_get_cores);
 * cores_out holds `capacity` doubles; discarded: host double[n-1] or NULL.
 * If the MPO arguments are given (mpo_bonds host int32[n+1], mpo device
 * packed W[bl][o][i][br]), the MPO is applied first (SI, "Matrix-vector
 * multiplication") and the product is compressed without being formed. */
mps_status mpsb_compress(int32_t n, const int32_t* mpo_bonds,
                         const double* mpo, const int32_t* bonds_in,
                         const double* cores_in, int32_t cap, double tol,
                         int32_t* bonds_out, double* cores_out,
                         int64_t capacity, double* discarded,
                         hipStream_t stream);

/* Captured step graphs of a state.  When every truncation has a fixed rank
 * (tol = 0) and dt is fixed, the shapes of a step do not change between
 * steps: after one ordinary step from a given state layout, the next step
 * records all launches of the step (both lanes) into a HIP graph and later
 * steps replay it, without the host work of issuing each launch; the
 * results are the same launches with the same arguments.  enable: 1 on,
 * 0 off, < 0 leaves it unchanged.  captures / replays: host
 * int64 counters or NULL.  Off by default and while kernel timing
 * (mpsb_profile) is on; MPSV_STEP_GRAPH=0 in the environment turns it off
 * for the process.  The recording is made on the state's own stream by the
 * calling thread alone (both lanes), ordered after prior work on `stream`
 * of mps_step; instances of a batch or plasma species refuse it. */
mps_status mpsb_step_graph(mps_state* h, int32_t enable, int64_t* captures,
                           int64_t* replays);

/* mpsb_step_graph for a lock-step batch (mps_batch_*): the recording holds
 * the launches of a step of every instance (each launch covers them all)
 * and is replayed by later mps_batch_step calls while the layout of the
 * instances' states is unchanged; the same conditions (tol = 0, fixed dt,
 * timing off) and the same results, bit for bit, as the batch's ordinary
 * steps.  MPS_EINVAL for a NULL batch. */
mps_status mpsb_batch_step_graph(mps_batch* b, int32_t enable, int64_t* captures,
                                 int64_t* replays);

/* Centre-first compression (SI, "Modified Compression Scheme") of an MPS
 * cut at the bond between sites centre-1 and centre (1 <= centre <= n-1):
 * the cut is truncated first from the mixed canonical form around it, then
 * sites 0..centre-1 are compressed by a truncated SVD sweep right to left
 * and sites centre..n-1 by one left to right, each bond to (cap, tol), and
 * S^-1 of the cut is folded into the left bond of site `centre`.
 * Arguments as for mpsb_compress (no MPO); discarded[j] is the relative
 * discarded weight at bond j | j+1. */
mps_status mpsb_compress_centre(int32_t n, int32_t centre,
                                const int32_t* bonds_in, const double* cores_in,
                                int32_t cap, double tol, int32_t* bonds_out,
                                double* cores_out, int64_t capacity,
                                double* discarded, hipStream_t stream);

/* Sum of MPS terms sum_t coef[t] * g_t, compressed (SI, "Addition").
 * bonds: host int32[nterms*(n+1)]; cores: host array of nterms device
 * pointers to packed cores. */
mps_status mpsb_add_compress(int32_t n, int32_t nterms, const double* coef,
                             const int32_t* bonds, const double* const* cores,
                             int32_t cap, double tol, int32_t* bonds_out,
                             double* cores_out, int64_t capacity,
                             hipStream_t stream);

/* Field of the current state: the charge density n(x) as an Lx-site MPS
 * and E = -G n compressed to (df_max, tol), both reconstructed on the
 * grid: device double[Nx] each (n_out / E_out may be NULL). */
mps_status mpsb_density_field(mps_state* h, double* n_out, double* E_out,
                              hipStream_t stream);

/* Operator MPOs exactly as the library builds them, for the tests:
 * which = 0: periodic central d/dx (bond 3), 1: zero-gradient central d/dv
 * (bond 5), 2: G = Dx L^+ (bond 5), 3: diag(v) (bond 2), 4: periodic
 * second-order backward d/dx and 5: forward d/dx (bond 3, SI Derivatives),
 * 6: diag(max(v, 0)) and 7: diag(min(v, 0)) (v times H(v) and 1 - H(v), SI
 * Upwind time evolution; bond <= 4).  L sites, spacing h (for which = 3, 6,
 * 7: v_j = h0 + j h).  bonds: host int32[L+1]; W: host
 * array of capacity doubles (packed W[bl][o][i][br]) or NULL to query
 * *count. */
mps_status mpsb_operator(int32_t which, int32_t L, double h0, double h,
                         int32_t* bonds, double* W, int64_t* count);

/* Device memory of one state, per arena in the order operators, committed
 * state, step intermediates, right-hand-side intermediates, compression
 * workspace, and the right-hand-side and compression arenas of the side
 * lane: reserved[7] gets the bytes each holds, peak[7] the largest extent
 * each has had in use.  Host outputs. */
mps_status mpsb_arena_bytes(const mps_state* h, size_t* reserved, size_t* peak);

/* Linear-algebra counters since load: QR and SVD calls, Jacobi sweeps. */
mps_status mpsb_stats(int64_t* qr_calls, int64_t* svd_calls,
                      int64_t* jacobi_sweeps);

/* Cap on Jacobi sweeps (default 60); a tiny cap forces MPS_ENUMERIC. */
mps_status mpsb_set_jacobi_max_sweeps(int32_t n);

/* Per-kernel-class timing with HIP events on the launching stream (off by
 * default).  enable != 0 clears and starts recording; classes: 0 GEMM,
 * 1 Householder QR factorisation, 2 Jacobi SVD, 3 other, 4 application of
 * Householder reflectors, 5 the same as compact-WY blocks (tall_apply = 1;
 * its byte count is the algorithmic traffic: Y read twice and written
 * once, the reflectors read twice).  mpsb_profile_read synchronises the
 * device and returns, for one class, the number of launches, the summed
 * event time (ms) and the summed nominal FLOPs and bytes (host outputs). */
mps_status mpsb_profile(int32_t enable);
mps_status mpsb_profile_read(int32_t cls, int64_t* launches, double* ms,
                             double* flops, double* bytes);
/* The part of a class's FLOPs recorded by launches inside a truncated SVD
 * (its QRs, reflector applications and GEMM); the SVD's own record (class
 * 2) counts the nominal 6 m n^2 + 20 n^3 of the whole decomposition, so a
 * total over classes subtracts this part.  Synchronises the device. */
mps_status mpsb_profile_nested_flops(int32_t cls, double* flops);

/* ---- Launch-shape table (used by every call above and by mps_step).
 *
 * For two launches the library has several kernel variants that give
 * bit-identical results and differ only in how the work is spread over
 * workgroups and waves: the output tile of the FP64 GEMM (knob 1: value 0
 * = 64 x 64, 1 = 128 x 128, 2 = 128 x 64; used when K is not split) and the
 * kernel of a
 * Householder reflector application (knob 2: value 1, 2 or 4 columns per
 * wave streaming the reflectors into registers; 9 or 10 for 1 or 2 columns
 * per wave with the reflectors shared by a workgroup through LDS, from 257
 * rows; 17 or 18 for the same with the block of columns also staged
 * through LDS, read and written row by row).
 * A table maps a key of six integers {knob, a, b, c, d, instance class}
 * to a value; a launch whose exact key is in the table (and whose value is
 * valid for it) takes that variant, any other the built-in rule.  Keys:
 *   knob 1: a = M, b = N, c = K, d = 4 * batch + 2 * (A row-major) +
 *           (B row-major)
 *   knob 2: a = rows (per row chunk), b = reflectors, c = columns,
 *           d = 2 * chunks + (1 for Q^T, 0 for Q)
 * instance class: 0 for one instance, 1 for 2..7 lock-step instances, 2
 * for 8..31, 3 for 32 or more.  The table is loaded on first use from the
 * file named by MPSV_TUNING, else tuning_gfx950.txt next to the library
 * (MPSV_TUNING=none: start empty).  The text format is one entry per line,
 * "knob a b c d class value", '#' starting a comment line.  The table is
 * written by paper_2205_11990_amd/tune.py, which times the variants in
 * real steps.  All calls are host-only except mpsb_tune_records, which
 * synchronises the device.  Changing the table while steps run on other
 * threads is allowed; those launches take the old or the new value. */
mps_status mpsb_tune_clear(void);
/* value < 0 erases the key; MPS_EINVAL for an unknown knob, a negative key
 * integer or a value above 31. */
mps_status mpsb_tune_set(const int32_t* key6, int32_t value);
/* *found = 1 and *value = the entry, or *found = 0. */
mps_status mpsb_tune_get(const int32_t* key6, int32_t* value, int32_t* found);
mps_status mpsb_tune_size(int64_t* n);
/* Replaces the table with the file's entries (MPS_EINVAL on unreadable or
 * malformed text, the table unchanged). */
mps_status mpsb_tune_load(const char* path);
mps_status mpsb_tune_save(const char* path);
/* on != 0 clears earlier records and starts recording: every launch with a
 * key is noted and timed with HIP events on its stream.  Recording costs
 * two events per such launch. */
mps_status mpsb_tune_record(int32_t on);
/* Synchronises the device and returns up to cap records (keys: 6 int32
 * each; value used last; allowed values as a bit set; launches; summed
 * event time in ms); *n = the number of records (which may exceed cap).
 * Host buffers. */
mps_status mpsb_tune_records(int32_t* keys, int32_t* values, uint32_t* allowed,
                             int64_t* launches, double* ms, int64_t cap,
                             int64_t* n);

#ifdef __cplusplus
}
#endif

#endif /* MPS_BLOCKS_H */
