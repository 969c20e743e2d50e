/*
 * mps_vlasov.h -- C-ABI of the MI355X (gfx950) MPS time stepper for the
 * 1D1V Vlasov-Poisson equations (Ye & Loureiro, "A quantum-inspired method
 * for solving the Vlasov-Poisson equations", arXiv:2205.11990).
 *
 * The distribution function f(x, v, t) lives on a uniform grid of
 * Nx = 2^Lx by Nv = 2^Lv points and is stored as a matrix product state
 * (quantized tensor train) with one binary site per bit (Method Overview,
 * "MPS Representation of Classical Data", eq. 4):
 *   x_i = x_min + i dx, dx = (x_max - x_min) / Nx, periodic (half-open);
 *   v_j = v_min + j dv, dv = (v_max - v_min) / (Nv - 1), closed, with
 *   zero-gradient boundaries (Methods, "Numerical Experiments").
 * One call of mps_step advances f by classic RK4 (SI, "Compressed time
 * evolution algorithm") of the collisionless Vlasov equation for one
 * species with charge-to-mass ratio qm and a neutralising background
 * (Problem Statement, eqs. 1-3): df/dt = -v df/dx - qm E df/dv,
 * E = -d phi/dx, Laplacian(phi) = n - <n>, n = int f dv.
 * Derivatives are the second-order central MPOs of the SI ("Derivatives"),
 * products with E and v are diagonal MPOs (SI, "Dot Product"), the field is
 * an MPO of the inverse Laplacian (SI, "Inverse Laplacian"), integrals are
 * left Riemann sums (SI, "Integration").  After every operation the MPS is
 * recompressed by a QR left-canonicalisation sweep followed by a truncated
 * SVD right-to-left sweep (SI, "Canonicalization and Compression"), keeping
 * at every bond at most chi values and discarding a relative weight of at
 * most tol (eq. 5).
 *
 * Conventions for every entry point:
 *  - Pointers documented as "device" are HIP device pointers owned by the
 *    caller (e.g. torch tensors); they are only accessed during the call.
 *    "host" pointers are ordinary CPU memory.
 *  - Work is enqueued on `stream` (0 = the null stream).  Calls return after
 *    the work is complete unless stated otherwise (the truncation ranks are
 *    read back during a step, so mps_step is synchronous with `stream`).
 *  - Errors are reported as mps_status; no C++ exception crosses the ABI.
 *    mps_last_error() returns a thread-local description of the last
 *    failure.  On any error the state is unchanged.
 *  - Handles are not thread-safe: one handle, one thread at a time.
 *  - FP64 throughout, except the optional FP32 contraction mode.
 */
#ifndef MPS_VLASOV_H
#define MPS_VLASOV_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MPS_OK = 0,
  MPS_EINVAL = -1,   /* invalid argument / problem                     */
  MPS_ENOMEM = -2,   /* device allocation failed                       */
  MPS_ENUMERIC = -3, /* non-finite state or a factorisation failed     */
  MPS_EDEVICE = -4   /* a HIP runtime call failed                      */
} mps_status;

typedef enum {
  MPS_ORDER_SEQ = 0,          /* S1 */
  MPS_ORDER_INTERLEAVED = 1,  /* IF */
  MPS_ORDER_S2 = 2,
  MPS_ORDER_S3 = 3,
  MPS_ORDER_IG = 4            /* IG: IF with x_k v_k fused into one site */
} mps_order;

/* Arithmetic of the MPO x MPS contractions (SI, "Matrix-vector
 * multiplication"): FP64, or operands rounded to FP32 (mode 1) or to BF16
 * (mode 2: to FP32, then to the nearest BF16, ties to even) with FP32
 * accumulation on the matrix cores (results kept in FP64).  The QR and SVD
 * sweeps, the Poisson field and the moments are FP64 in every mode.
 * Reduced precision leaves rounding noise in every contracted term, near
 * 1e-7 (FP32) or 4e-3 (BF16) of its largest singular value: with a
 * tolerance below that, compression points without a chi cap keep the
 * noise and their bonds grow towards full rank, so such runs use a
 * tolerance above the noise or cap every point (level 5). */
typedef enum {
  MPS_PREC_FP64 = 0,
  MPS_PREC_FP32_CONTRACT = 1,
  MPS_PREC_BF16_CONTRACT = 2
} mps_precision;

/* x advection (SI, "Upwind time evolution"): the periodic second-order
 * central difference, or upwind: the second-order backward difference where
 * v > 0 and the forward one where v < 0 (SI, "First Derivative, Forward /
 * Backward, Periodic Boundary Conditions"), i.e. T1 = -(Db (x) diag(v H(v))
 * + Df (x) diag(v (1 - H(v)))).  The paper's sentence is followed where its
 * displayed formula pairs forward with H(v). */
typedef enum { MPS_X_CENTRAL = 0, MPS_X_UPWIND = 1 } mps_x_scheme;

/* Compression of the full chain at every compression point (SI,
 * "Canonicalization and Compression" and "Modified Compression Scheme"):
 * MPS_COMPRESS_SWEEP is a QR sweep left to right, then a truncated SVD sweep
 * right to left.  MPS_COMPRESS_CENTRE_FIRST (sequential ordering only)
 * first truncates the x|v bond, f = sum_r s_r g_r(x) h_r(v), from the
 * mixed canonical form around it, then compresses the x half G = [s_r g_r]
 * right to left and the v half H = [s_r h_r] left to right, and joins them
 * through S^-1 (folded into the first v site; a value at or below 1e-200 of
 * the largest, an exact zero of a rank-deficient cut, gets 0).  The result
 * is not in canonical form.  The field and the entanglement diagnostic
 * keep the sweep.  The centre-first scheme also holds the untruncated right
 * half in its workspace (mps_workspace_bound adds an allowance for it). */
typedef enum {
  MPS_COMPRESS_SWEEP = 0,
  MPS_COMPRESS_CENTRE_FIRST = 1
} mps_compression;

/* Problem statement.  Site orderings (Fig. 3): MPS_ORDER_SEQ is x bits
 * coarse->fine then v bits coarse->fine (S1); MPS_ORDER_S2 is x bits
 * fine->coarse then v bits coarse->fine; MPS_ORDER_S3 is x bits
 * coarse->fine then v bits fine->coarse; MPS_ORDER_INTERLEAVED is
 * x1, v1, x2, v2, ... (IF; needs Lx == Lv); MPS_ORDER_IG fuses each pair
 * (x_k, v_k) into one site of dimension 4 (IG).  An IG state is held as the
 * IF chain of binary sites in which the bond inside each pair is never
 * truncated (a dimension-4 site is exactly its two binary sites contracted),
 * so truncation acts on the bonds between pairs only; bond_dims and the
 * exported cores are those of the binary sites, and the memory model treats
 * it as IF.  Centre-first compression needs S1, S2 or S3.  The ordering only changes how
 * the grid maps to the chain: mps_to_dense, the moments and the field are
 * on the grid in every ordering, and mps_get_cores / mps_set_cores use
 * chain order.  Compression level (SI,
 * compression levels C1..C5): the final state (P1), the stage states (P2),
 * the sum of the k's (P3), each k (P4) and each term of a k (P5) are all
 * truncated with `tol`; level l additionally caps P1..Pl at chi_max. */
/* Adaptive time step (Methods, Time Evolution Procedure, eq. CFL), for one
 * collisionless species: when cfl > 0 every step takes
 * dt = cfl / (|v|_max / dx + |q/m| |E|_max / dv), |E|_max on the grid of the
 * state at the start of the step (the paper uses cfl = 0.9; with the upwind
 * scheme RK4 needs cfl < 0.696, its negative-real-axis limit over the
 * stencil's extreme eigenvalue -4 v / dx).  dt is then not used; the
 * elapsed time is reported by mps_info. */
typedef struct mps_problem {
  int32_t Lx, Lv;           /* bits per dimension, each in [2, 14]        */
  int32_t order;            /* mps_order                                   */
  double x_min, x_max;      /* periodic interval, x_max > x_min            */
  double v_min, v_max;      /* closed interval, v_max > v_min              */
  double qm;                /* charge / mass of the species (-1: electrons)*/
  double dt;                /* fixed RK4 step, > 0 (unless cfl > 0)        */
  int32_t chi_max;          /* bond cap (paper D), >= 1                    */
  int32_t level;            /* compression level 1..5 (1 = C1)             */
  int32_t df_max;           /* cap on the field bond D_F, 0 = uncapped     */
  double tol;               /* relative discarded weight per bond, >= 0    */
  int32_t precision;        /* mps_precision                               */
  int32_t x_scheme;         /* mps_x_scheme                                */
  double cfl;               /* > 0: adaptive dt (see below), 0: fixed dt   */
  int32_t compression;      /* mps_compression                             */
  double nu;                /* Dougherty collision rate, >= 0 (0: none)    */
  double nu_v0, nu_vth;     /* drift and thermal speed of coll_model 1     */
  int32_t coll_model;       /* 0: v0, vth from the moments of f; 1: fixed  */
  int32_t tall_apply;       /* mps_tall_apply, 0: one reflector at a time  */
} mps_problem;

/* How the QR sweeps apply their Householder reflectors to tall blocks (more
 * than 512 rows, panels of up to 16 reflectors, at least 32 columns; SI,
 * Canonicalization and Compression: the QR of each site).  Both are exact
 * applications of the same orthogonal factor; their results differ at the
 * rounding level, and a state's results depend on this choice, never on
 * how many lock-step instances share its launches.
 *   MPS_TALL_APPLY_REFLECTORS: one reflector at a time, each column in the
 *     registers of one wave (shortest chain: fastest for one state);
 *   MPS_TALL_APPLY_WY: blocks of 16-column panels are factored in groups
 *     of four, each panel updating only the rest of its group, and a
 *     group's 64 reflectors reach the trailing columns, and later products
 *     with Q, as one compact-WY block on the matrix cores (the block
 *     streamed twice per group); the remaining applications of up to 16
 *     reflectors to at least 32 columns take a compact-WY block of their
 *     own (fastest for large lock-step batches, where the launches fill
 *     the device). */
typedef enum mps_tall_apply {
  MPS_TALL_APPLY_REFLECTORS = 0,
  MPS_TALL_APPLY_WY = 1
} mps_tall_apply;

/* Collisions (Methods, "Collision Operator"): with nu > 0 the Vlasov
 * right-hand side gains the Dougherty operator
 * nu d/dv[(v - v0) f + vth^2 df/dv], both derivatives the zero-gradient
 * central difference.  coll_model 0 (the paper's operator): v0 and vth are
 * the species' average and thermal velocity at each x, the moments of the
 * stage's state, v0 = <v, f>_v / n, vth^2 = <v^2, f>_v / n - v0^2 with
 * n = <1, f>_v (0 where n = 0); the three contractions are formed as x-MPS,
 * evaluated on the x grid, divided there and brought back to x-MPS by
 * iterated SVD (relative cut 1e-14 when tol > 0, exact when tol = 0), then
 * compressed like the field (df_max, tol).  C f is then three terms of each
 * k, nu Dv diag(v) f, -nu (diag(v0) (x) Dv) f and nu (diag(vth^2) (x) Dv Dv) f,
 * each compressed like the other terms (P5).  It conserves density,
 * momentum and energy at every x.  coll_model 1: v0 = nu_v0 and vth = nu_vth
 * fixed (a linear operator, nu Dv (diag(v - nu_v0) + nu_vth^2 Dv), one term).
 * With cfl > 0 the step adds nu |v|_max / dv + 2 nu nu_vth^2 / dv^2 to the
 * CFL sum (eq. CFL) in both models. */

typedef struct mps_state mps_state; /* opaque; owns all device memory */

/* Create a state from f0(x_i, v_j) = sum_{r<rank} ax[r*Nx + i] * bv[r*Nv + j]
 * (device FP64 arrays).  Each 1-D profile is converted by iterated SVD
 * (eq. 4), the terms are combined per ordering, summed and compressed to
 * (chi_max, tol).  Returns MPS_EINVAL for invalid problems or non-finite
 * profiles. */
mps_status mps_init(const mps_problem* p, int32_t rank, const double* ax,
                    const double* bv, hipStream_t stream, mps_state** out);

/* Advance by nsteps RK4 steps.  Each step commits only if the new state is
 * finite and every factorisation converged; otherwise MPS_ENUMERIC is
 * returned and the state is the last good one. */
mps_status mps_step(mps_state* h, int32_t nsteps, hipStream_t stream);

/* Moments of the current state.  n_out, E_out: device double[Nx] or NULL
 * (density n = int f dv and field E).  scalars: host double[4] or NULL =
 * {mass, momentum, kinetic energy, field energy} = dx dv sum f,
 * dx dv sum v f, dx dv sum v^2 f / 2, dx sum E^2 / 2. */
mps_status mps_moments(mps_state* h, double* n_out, double* E_out,
                       double* scalars, hipStream_t stream);

/* Reconstruct f on the grid: device double[Nx*Nv], f_out[i*Nv + j]. */
mps_status mps_to_dense(mps_state* h, double* f_out, hipStream_t stream);

/* Entanglement entropy (Results, State Compressibility): for each of the
 * n-1 bonds, -sum_i t_i log2 t_i with t_i the squared Schmidt values of the
 * current state across that bond normalised to sum 1 (0 for a product
 * cut).  The Schmidt values come from an untruncated canonicalisation (QR
 * sweep, then SVD sweep) of a copy; the state is unchanged.  ee: host
 * double[n-1]; synchronises the stream. */
mps_status mps_entanglement(mps_state* h, double* ee, hipStream_t stream);

/* Release the state and all its device memory.  NULL is accepted. */
mps_status mps_free(mps_state* h);

/* Query.  Any output may be NULL.  n_sites: host int32; bond_dims: host
 * int32[n+1] (bond_dims[0] = bond_dims[n] = 1); discarded: host
 * double[n-1], relative discarded weight per bond of the last final
 * compression; t: host double (simulated time); steps: host int64. */
mps_status mps_info(const mps_state* h, int32_t* n_sites, int32_t* bond_dims,
                    double* discarded, double* t, int64_t* steps);

/* Export / import the state.  Cores are packed in site order, core j of
 * shape bond[j] x 2 x bond[j+1] row-major.  mps_get_cores with cores ==
 * NULL only reports bond_dims (host int32[n+1]) and *count (host int64,
 * total doubles).  cores: device.  mps_set_cores replaces the state (used
 * for checkpoint / resume and to start the oracle and the GPU from the same
 * MPS). */
mps_status mps_get_cores(const mps_state* h, int32_t* bond_dims,
                         int64_t* count, double* cores, hipStream_t stream);
mps_status mps_set_cores(mps_state* h, const int32_t* bond_dims,
                         const double* cores, hipStream_t stream);

/* f <- compress(f + alpha g, chi_max, tol) for an MPS g given as packed
 * device cores with host bond_dims[n+1] (SI, "Addition"). */
mps_status mps_add_scaled(mps_state* h, double alpha, const int32_t* bond_dims,
                          const double* cores, hipStream_t stream);

/* Device bytes a state of problem p may hold (for admission control of
 * several states sharing one GPU's memory), host output.  A size model per
 * arena, from the chi-capped state, the widest contraction of the field
 * term and the interleaved initial state at full rank, with coefficients
 * that envelope measured peaks (grids 2^6..2^13, chi 16..128, both
 * orderings), plus chunk rounding and a fixed allowance; the collision
 * terms, the IG ordering, the centre-first scheme and the compact-WY mode's
 * panel groups are included.  It assumes every compression point stays
 * within chi_max (level 5, or lower levels whose tolerance keeps the bonds
 * there).  A plasma of several species holds one such state per species.
 * A lock-step batch rounds its arena chunks for all instances at once and
 * may exceed the sum of its instances' bounds by a little (512 against 508
 * MiB per instance for 256 instances at 2^10 x 2^10, chi = 64); allow a
 * few percent more.  EINVAL for every problem that mps_init rejects on its
 * parameters (the same checks). */
mps_status mps_workspace_bound(const mps_problem* p, size_t* bytes);

/* Device bytes the state h holds right now (all of its arenas: operators,
 * committed state, step and compression workspace), host output.  The
 * arenas keep their high-water mark between steps. */
mps_status mps_device_bytes(const mps_state* h, size_t* bytes);

/* Advance several independent states (parameter sweeps, uneven sizes) by
 * nsteps each.  Every instance runs on a stream of its own, driven by its
 * own host thread (at most 16 at a time), so the factorisations of
 * different instances occupy different compute units at once; the result
 * of each instance is the same as stepping it alone.  The work is ordered
 * after prior work on `stream`, and later work on `stream` waits for all
 * instances.  A handle may appear only once (MPS_EINVAL otherwise).  On a
 * failure the failing instance keeps the state of its last completed step,
 * the others complete theirs, and the first failure (lowest index) is
 * returned, its message naming the instance. */
mps_status mps_step_batched(mps_state* const* hs, int32_t count, int32_t nsteps,
                            hipStream_t stream);

/* Lock-step batch: count instances of one problem shape advanced together,
 * every kernel launch of a step covering all of them (the method's cost is a
 * long chain of small factorisations, SI "Canonicalization and Compression";
 * one instance occupies a few compute units, a batch spreads the same chain
 * over one workgroup per instance).  The instances share Lx, Lv, order,
 * chi_max, level, df_max, precision, x_scheme, compression, qm and dt, have
 * tol = 0 and cfl = 0 (fixed ranks: every compression keeps min(chi, k)
 * values, so their shapes never differ) and are all collisional or all
 * collisionless; intervals, collision constants and data may differ.  Each
 * instance's result equals that of a stand-alone state stepped from the
 * same cores, bit for bit.
 * mps_batch_init: problems, ranks: host arrays of count (1..1024); ax[i],
 * bv[i]: device profiles of instance i as for mps_init.  Every instance's
 * initial state must come out with the same bond dimensions (MPS_EINVAL
 * otherwise).  Device memory: the workspace of one instance times count
 * (each arena chunk is allocated once for all instances). */
typedef struct mps_batch mps_batch;
mps_status mps_batch_init(int32_t count, const mps_problem* problems,
                          const int32_t* ranks, const double* const* ax,
                          const double* const* bv, hipStream_t stream,
                          mps_batch** out);
/* Replace every instance's state: bond_dims host (n + 1 entries, unit
 * ends), cores[i] device, packed as mps_set_cores, one array per instance. */
mps_status mps_batch_set_cores(mps_batch* b, const int32_t* bond_dims,
                               const double* const* cores, hipStream_t stream);
/* f_i <- compress(f_i + alpha[i] g_i) for every instance (alpha host,
 * count values; g_i device cores of one set of bonds). */
mps_status mps_batch_add_scaled(mps_batch* b, const double* alpha,
                                const int32_t* bond_dims,
                                const double* const* cores, hipStream_t stream);
/* nsteps RK4 steps of every instance, committed for all of them or for
 * none (a failure names its instance). */
mps_status mps_batch_step(mps_batch* b, int32_t nsteps, hipStream_t stream);
/* Instance i as a state handle owned by the batch (NULL if out of range):
 * mps_to_dense, mps_get_cores, mps_info, mps_moments, mps_entanglement and
 * mps_device_bytes (the whole batch) apply; mps_step, mps_set_cores,
 * mps_add_scaled and mps_free refuse it. */
mps_state* mps_batch_instance(mps_batch* b, int32_t i);
/* Release the batch and its instance handles.  NULL is accepted. */
mps_status mps_batch_free(mps_batch* b);

/* Several species sharing x and E (Methods: the two-species Landau and
 * Buneman set-ups).  Each species is an mps_problem of its own (its v grid,
 * q/m, collisions, compression settings); all share Lx, x_min, x_max and a
 * fixed dt (cfl = 0).  Poisson becomes Laplacian(phi) = -sum_s q_s n_s with
 * charges[s] = q_s (normalised units; the pseudo-inverse drops the mean,
 * i.e. a neutralising background), E = -G rho compressed with species 0's
 * df_max and tol.  One RK4 step advances every species, each stage's E from
 * all of them; the new states are committed for all species or for none.
 * mps_plasma_init: species, charges, ranks: host arrays of n_species (1..8);
 * ax[s], bv[s]: device profiles of species s as for mps_init.  A single
 * species of charge -1 is the one-species case of mps_step. */
typedef struct mps_plasma mps_plasma;
mps_status mps_plasma_init(int32_t n_species, const mps_problem* species,
                           const double* charges, const int32_t* ranks,
                           const double* const* ax, const double* const* bv,
                           hipStream_t stream, mps_plasma** out);
mps_status mps_plasma_step(mps_plasma* pl, int32_t nsteps, hipStream_t stream);
/* Species s as a state handle owned by the plasma (NULL if out of range):
 * mps_to_dense, mps_get_cores / mps_set_cores, mps_info, mps_entanglement and
 * mps_moments (density and scalars; its field there is of that species alone)
 * apply; mps_step and mps_free refuse it. */
mps_state* mps_plasma_species(mps_plasma* pl, int32_t s);
/* The shared field: E_out device double[Nx] or NULL; field_energy host
 * double or NULL = dx sum E^2 / 2.  Synchronises the stream. */
mps_status mps_plasma_field(mps_plasma* pl, double* E_out, double* field_energy,
                            hipStream_t stream);
/* Release the plasma and its species.  NULL is accepted. */
mps_status mps_plasma_free(mps_plasma* pl);

/* Thread-local text of the last error ("" if none). */
const char* mps_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MPS_VLASOV_H */
