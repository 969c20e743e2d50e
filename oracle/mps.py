"""CPU MPS reference in FP64 (oracle O2): the method itself, step by step.

An MPS is a list of cores ``A[j]`` with shape (left bond, 2, right bond);
site 0 is the most significant (coarsest) bit.  An MPO is a list of tensors
``W[j]`` with shape (left bond, out bit o, in bit i, right bond).

Sections of the paper followed here:
* Method overview, "MPS Representation of Classical Data": vector -> MPS by
  iterated SVD (eq. 4); per-bond error eps_j (eq. 5); full-rank bonds
  r_j = d^min(j, KL-j).
* SI "Matrix-vector multiplication": C(o) = sum_i B(o, i) A(i), bond product.
* SI "Addition": block-diagonal cores, bond sum.
* SI "Derivatives": the printed MPOs for the periodic central first
  derivative, the non-periodic backbone plus boundary matrices, and the
  periodic second derivative.
* SI "Derivatives", forward and backward periodic first derivatives: the
  printed forward MPO is garbled (its c3 is never defined), so both are
  rebuilt from their stencils (the coefficients the paper prints) through
  the dense matrix and TT-SVD, the SI's matrix -> MPO route.
* SI "Upwind time evolution": backward difference where v > 0, forward
  where v < 0 (the paper's sentence; its displayed formula pairs the labels
  the other way round), i.e. T1 = -(Db (x) diag(max(v,0)) +
  Df (x) diag(min(v,0))), the velocity split being H(v) times v.
* SI "Dot Product": MPS -> diagonal MPO, M(o, i) = M(i) delta_{io}.
* SI "Inverse Laplacian": dense inverse converted into an MPO.
* SI "Integration": dx [1, 1]^{(x) L}.
* SI "Canonicalization and Compression": QR sweep then truncated SVD sweep.
* SI "Modified Compression Scheme": centre-first compression of a sequential
  ordering (x|v bond first, then each half), optional per problem.
* SI "Compressed time evolution algorithm": RK4 and compression levels C1-C5.
* Results, "State Compressibility" (eq. 6 context) and Fig. 3 orderings:
  sequential S1, S2 (x fine->coarse, v coarse->fine), S3 (x coarse->fine,
  v fine->coarse), interleaved IF and grouped IG (sites of dimension 4
  holding x_k and v_k).

Readings where the paper is silent or garbled:
* The printed M_left of the zero-gradient derivative puts its only entry at
  (o, i) = (N/2-1, N-1); the mirror image of the printed M_right is used
  instead, P0^{(x)(L-1)} (x) [[0, -c1], [0, 0]], so rows 0 and N-1 vanish.
* eps_j sums the discarded values i = D+1 .. r_j (keep the D largest).
* Sweep order: QR left-to-right, then truncated SVD right-to-left; the
  norm ends in the first core.
* Rank rule: D = min(chi, min{D' >= 1 : sum_{i>D'} s~_i^2 <= tol^2}) with
  s~ = s / ||s||; tol = 0 keeps min(chi, len(s)), also for an all-zero
  block (eq. 5 discards nothing by weight then; with tol > 0 a zero block
  keeps one value).
* Compression points: P1 final state, P2 each stage state, P3 the sum of
  the k's, P4 each k, P5 each term of a k.  Every point truncates with tol;
  level C_l caps P1..P_l at chi (C1: only the final state is capped).
* The field MPS is compressed with tol and an optional cap D_F.
* Collisions: the Dougherty operator nu Dv (diag(v - v0) + vth^2 Dv) with
  Dv the zero-gradient central difference (Methods, Collision Operator).
  v0 and vth are the species' average and thermal velocity: the local
  moments of the state at each x, n = <1, g>_v, v0 = <v, g>_v / n,
  vth^2 = <v^2, g>_v / n - v0^2 (0 where n = 0), taken from the x-MPS of
  the three contractions on the grid of x, each brought back to an x-MPS
  (iterated SVD with relative cut 1e-14 when tol > 0, exact when tol = 0)
  and compressed like the field (cap D_F, tol).  Since v0 and vth do not
  depend on v, C g = nu Dv diag(v) g - nu (diag(v0) (x) Dv) g +
  nu (diag(vth^2) (x) Dv Dv) g: three terms of a k, each compressed at P5.
  The alternative model coll_model = 1 keeps v0 and vth fixed parameters
  of the species, one term nu Dv (diag(v - v0) + vth^2 Dv) g.
* Several species: rho = sum_s (-q_s) n_s is formed exactly (direct sum)
  and E = compress(-G rho) uses the first species' D_F and tol.
* Centre-first compression: the SVD is of the centre site (first v site)
  at its left bond, the x|v cut; U S joins the last x site and S V^T becomes
  the centre site (the printed step that merges S V^T into the next site
  would drop a site); the centre cut obeys the same rank rule (chi, tol) as
  every other bond; the x half is swept right to left and the v half left
  to right; S^-1 goes into the centre site's left bond, with 0 for a value
  at or below 1e-200 of the largest.  The full-chain compressions P1-P5
  (and the initial state) use it; the field keeps the plain sweep.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__``.
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

Mps = List[np.ndarray]
Mpo = List[np.ndarray]

# ---------------------------------------------------------------- basics

I2 = np.eye(2)
SP = np.array([[0.0, 0.0], [1.0, 0.0]])   # S+ : (o, i) = (1, 0)
SM = np.array([[0.0, 1.0], [0.0, 0.0]])   # S- : (o, i) = (0, 1)
Z2 = np.zeros((2, 2))
P0 = np.array([[1.0, 0.0], [0.0, 0.0]])
P1 = np.array([[0.0, 0.0], [0.0, 1.0]])


def rank_rule(s: np.ndarray, chi: Optional[int], tol: float) -> int:
    """Number of singular values kept (eq. 5 with the i = D+1 reading)."""
    k = len(s)
    cap = k if chi is None else min(chi, k)
    if tol <= 0.0:
        # nothing is discarded by weight: the cap alone sets D, whatever
        # the values (an all-zero block included)
        return max(1, cap)
    norm2 = float(np.sum(s * s))
    if k == 0 or norm2 == 0.0:
        return 1
    t = (s * s) / norm2
    # tail[D] = sum_{i >= D} t_i (0-based), summed from the smallest value
    tail = np.cumsum(t[::-1])[::-1]
    tail = np.append(tail, 0.0)
    D = k
    for Dp in range(1, k + 1):
        if tail[Dp] <= tol * tol:
            D = Dp
            break
    return max(1, min(D, cap))


def tt_svd(vec: np.ndarray, dims: Sequence[int], tol: float = 0.0,
           chi: Optional[int] = None) -> Mps:
    """Vector -> MPS by iterated SVD from the left (eq. 4, Fig. 1a):
    reshape (r_{j-1} d_j) x rest, SVD, keep U as core j, carry S V^T."""
    cores = []
    r = 1
    M = np.asarray(vec, dtype=np.float64).reshape(1, -1)
    for j, d in enumerate(dims[:-1]):
        M = M.reshape(r * d, -1)
        U, S, Vt = np.linalg.svd(M, full_matrices=False)
        D = rank_rule(S, chi, tol)
        cores.append(U[:, :D].reshape(r, d, D))
        M = S[:D, None] * Vt[:D]
        r = D
    cores.append(M.reshape(r, dims[-1], 1))
    return cores


def to_vector(mps: Mps) -> np.ndarray:
    """Contract all bonds: the represented vector, site 0 most significant."""
    v = mps[0].reshape(mps[0].shape[1], -1)
    for A in mps[1:]:
        v = (v @ A.reshape(A.shape[0], -1)).reshape(-1, A.shape[2])
    return v.reshape(-1)


def bond_dims(mps: Mps) -> List[int]:
    return [A.shape[2] for A in mps[:-1]]


def scale(mps: Mps, c: float) -> Mps:
    out = [A.copy() for A in mps]
    out[0] = out[0] * c
    return out


# ------------------------------------------------- MPO x MPS, sum, diag

def apply(W: Mpo, A: Mps) -> Mps:
    """SI, Matrix-vector multiplication: C^{(n)}_{(a,b),(a',b')}(o) =
    sum_i B_{b,b'}(o, i) A_{a,a'}(i); fused bond gamma = (alpha, beta)."""
    out = []
    for Wj, Aj in zip(W, A):
        C = np.einsum("bois,aic->abocs", Wj, Aj)
        a, b, o, c, s = C.shape
        out.append(C.reshape(a * b, o, c * s))
    return out


def add(terms: Sequence[Tuple[float, Mps]]) -> Mps:
    """SI, Addition: block-diagonal cores, bond = sum of bonds.  The scalar
    of each term is folded into its first core."""
    n = len(terms[0][1])
    out = []
    for j in range(n):
        blocks = [(c if j == 0 else 1.0) * m[j] for c, m in terms]
        if n == 1:
            out.append(sum(blocks))
            continue
        if j == 0:
            out.append(np.concatenate(blocks, axis=2))
        elif j == n - 1:
            out.append(np.concatenate(blocks, axis=0))
        else:
            L = sum(b.shape[0] for b in blocks)
            R = sum(b.shape[2] for b in blocks)
            C = np.zeros((L, blocks[0].shape[1], R))
            l0 = r0 = 0
            for b in blocks:
                C[l0:l0 + b.shape[0], :, r0:r0 + b.shape[2]] = b
                l0 += b.shape[0]
                r0 += b.shape[2]
            out.append(C)
    return out


def diag_mpo(mps: Mps) -> Mpo:
    """SI, Dot Product: M_{l,r}(o, i) = M_{l,r}(i) delta_{io}."""
    out = []
    for A in mps:
        a, d, b = A.shape
        W = np.zeros((a, d, d, b))
        for s in range(d):
            W[:, s, s, :] = A[:, s, :]
        out.append(W)
    return out


def inner(A: Mps, B: Mps) -> float:
    """<A, B> = sum over all indices of A * B (transfer-matrix contraction)."""
    E = np.ones((1, 1))
    for a, b in zip(A, B):
        E = np.einsum("xy,xsp,ysq->pq", E, a, b)
    return float(E[0, 0])


# ------------------------------------------------------ compression

def compress(mps: Mps, chi: Optional[int], tol: float,
             return_discarded: bool = False):
    """SI, Canonicalization and Compression.

    (i) QR sweep left to right: A_j as (a*2) x b = Q R, A_j <- Q,
        A_{j+1} <- R A_{j+1}.
    (ii) truncated SVD sweep right to left: A_j as a x (2*b) = U S V^T, keep D
        by the rank rule, A_j <- V^T_D, A_{j-1} <- A_{j-1} U_D S_D.
    Returns the compressed MPS (and the relative discarded weight per bond,
    eps_j of eq. 5, if asked)."""
    A = [c.copy() for c in mps]
    n = len(A)
    for j in range(n - 1):
        a, d, b = A[j].shape
        Q, R = np.linalg.qr(A[j].reshape(a * d, b))
        A[j] = Q.reshape(a, d, Q.shape[1])
        A[j + 1] = np.tensordot(R, A[j + 1], axes=(1, 0))
    disc = [0.0] * (n - 1)
    for j in range(n - 1, 0, -1):
        a, d, b = A[j].shape
        U, S, Vt = np.linalg.svd(A[j].reshape(a, d * b), full_matrices=False)
        D = rank_rule(S, chi, tol)
        nrm2 = float(np.sum(S * S))
        disc[j - 1] = math.sqrt(float(np.sum(S[D:] ** 2)) / nrm2) if nrm2 > 0 else 0.0
        A[j] = Vt[:D].reshape(D, d, b)
        A[j - 1] = np.tensordot(A[j - 1], U[:, :D] * S[:D], axes=(2, 0))
    return (A, disc) if return_discarded else A


def centre_pinv(S: np.ndarray) -> np.ndarray:
    """1 / s for the kept centre values; a value at or below 1e-200 of the
    largest (in practice an exact zero of a rank-deficient cut) carries no
    weight in either half and gets 0 instead of an overflow."""
    out = np.zeros_like(S)
    keep = S > S[0] * 1e-200 if len(S) and S[0] > 0 else np.zeros(len(S), bool)
    out[keep] = 1.0 / S[keep]
    return out


def compress_centre(mps: Mps, c: int, chi: Optional[int], tol: float,
                    return_discarded: bool = False):
    """SI, Modified Compression Scheme, for a sequential ordering whose two
    dimensions meet at the bond between sites c-1 and c.

    1. Mixed canonical form: sites 0..c-1 left canonical (QR sweep from the
       left), sites c+1..n-1 right canonical (QR of the transposed cores,
       sweeping from the right); site c holds the whole norm.
    2. Site c as (left bond) x (2 * right bond) = U S V^T, D kept by the rank
       rule.  These are the Schmidt values of the x|v cut: f = sum_r s_r
       g_r(x) h_r(v).
    3.-5. A_{c-1} <- A_{c-1} U S and A_c <- S V^T, with S^-1 between them,
       so the left half holds G = [s_r g_r] and the right half H = [s_r h_r].
    6. Truncated SVD sweep right to left over sites c-1 .. 1 (bonds inside x).
    7. Truncated SVD sweep left to right over sites c .. n-2 (bonds inside v).
    8. S^-1 absorbed into the left bond of site c.
    The result represents G' S^-1 H'; it is not in canonical form."""
    A = [x.copy() for x in mps]
    n = len(A)
    if not 1 <= c <= n - 1:
        raise ValueError("centre must lie in [1, n-1]")
    for j in range(c):
        a, d, b = A[j].shape
        Q, R = np.linalg.qr(A[j].reshape(a * d, b))
        A[j] = Q.reshape(a, d, Q.shape[1])
        A[j + 1] = np.tensordot(R, A[j + 1], axes=(1, 0))
    for j in range(n - 1, c, -1):
        a, d, b = A[j].shape
        Q, R = np.linalg.qr(A[j].reshape(a, d * b).T)
        A[j] = Q.T.reshape(Q.shape[1], d, b)
        A[j - 1] = np.tensordot(A[j - 1], R.T, axes=(2, 0))
    disc = [0.0] * (n - 1)

    def trunc(M):
        U, S, Vt = np.linalg.svd(M, full_matrices=False)
        D = rank_rule(S, chi, tol)
        nrm2 = float(np.sum(S * S))
        e = math.sqrt(float(np.sum(S[D:] ** 2)) / nrm2) if nrm2 > 0 else 0.0
        return U[:, :D], S[:D], Vt[:D], e

    a, d, b = A[c].shape
    U, S, Vt, disc[c - 1] = trunc(A[c].reshape(a, d * b))
    A[c - 1] = np.tensordot(A[c - 1], U * S, axes=(2, 0))
    A[c] = (S[:, None] * Vt).reshape(len(S), d, b)
    for j in range(c - 1, 0, -1):
        a, d, b = A[j].shape
        Uj, Sj, Vj, disc[j - 1] = trunc(A[j].reshape(a, d * b))
        A[j] = Vj.reshape(len(Sj), d, b)
        A[j - 1] = np.tensordot(A[j - 1], Uj * Sj, axes=(2, 0))
    for j in range(c, n - 1):
        a, d, b = A[j].shape
        Uj, Sj, Vj, disc[j] = trunc(A[j].reshape(a * d, b))
        A[j] = Uj.reshape(a, d, len(Sj))
        A[j + 1] = np.tensordot(Sj[:, None] * Vj, A[j + 1], axes=(1, 0))
    A[c] = centre_pinv(S)[:, None, None] * A[c]
    return (A, disc) if return_discarded else A


def left_canonicalize(mps: Mps) -> Mps:
    """Only the QR sweep of `compress` (left canonical form, SI)."""
    A = [c.copy() for c in mps]
    for j in range(len(A) - 1):
        a, d, b = A[j].shape
        Q, R = np.linalg.qr(A[j].reshape(a * d, b))
        A[j] = Q.reshape(a, d, Q.shape[1])
        A[j + 1] = np.tensordot(R, A[j + 1], axes=(1, 0))
    return A


def entanglement_entropy(mps: Mps) -> List[float]:
    """Eq. 6 at every bond, from the untruncated sweep's singular values."""
    A = left_canonicalize(mps)
    n = len(A)
    out = [0.0] * (n - 1)
    for j in range(n - 1, 0, -1):
        a, d, b = A[j].shape
        U, S, Vt = np.linalg.svd(A[j].reshape(a, d * b), full_matrices=False)
        t = S * S / np.sum(S * S)
        t = t[t > 0]
        out[j - 1] = float(-np.sum(t * np.log2(t)))
        A[j] = Vt.reshape(-1, d, b)
        A[j - 1] = np.tensordot(A[j - 1], U * S, axes=(2, 0))
    return out


# ------------------------------------------------------ operator MPOs

def _chain(first, bulk, last, L: int) -> Mpo:
    """Turn the printed operator-valued row/matrix/column form into MPO
    tensors W[bl, o, i, br] (site 0 = first factor)."""
    def tens(rows):
        rows = [[np.asarray(x, dtype=np.float64) for x in r] for r in rows]
        bl, br = len(rows), len(rows[0])
        W = np.zeros((bl, 2, 2, br))
        for a in range(bl):
            for b in range(br):
                W[a, :, :, b] = rows[a][b]
        return W
    if L < 2:
        raise ValueError("operator MPOs need at least two sites")
    return [tens([first])] + [tens(bulk) for _ in range(L - 2)] + \
        [tens([[x] for x in last])]


def mpo_d1_periodic(L: int, h: float) -> Mpo:
    """SI, First Derivative, Centered, Periodic: bond 3, c1 = 1/2, 1/h."""
    c1 = 0.5
    first = [I2, SP + SM, SP + SM]
    bulk = [[I2, SM, SP], [Z2, SP, Z2], [Z2, Z2, SM]]
    last = [c1 * (SM - SP), c1 * SP, -c1 * SM]
    W = _chain(first, bulk, last, L)
    W[0] = W[0] / h
    return W


def mpo_d1_zero_gradient(L: int, h: float) -> Mpo:
    """SI, First Derivative, Centered, Zero Gradient: the non-periodic
    backbone (bond 3) plus M_left and M_right (bond 1 each) as an MPO sum
    (bond 5).  M_left is the mirror of the printed M_right (see header)."""
    c1 = 0.5
    first = [I2, SM, SP]
    bulk = [[I2, SM, SP], [Z2, SP, Z2], [Z2, Z2, SM]]
    last = [c1 * (SM - SP), c1 * SP, -c1 * SM]
    back = _chain(first, bulk, last, L)
    right = [P1.reshape(1, 2, 2, 1) for _ in range(L - 1)] + \
        [np.array([[0.0, 0.0], [c1, 0.0]]).reshape(1, 2, 2, 1)]
    left = [P0.reshape(1, 2, 2, 1) for _ in range(L - 1)] + \
        [np.array([[0.0, -c1], [0.0, 0.0]]).reshape(1, 2, 2, 1)]
    W = mpo_sum([back, left, right])
    W[0] = W[0] / h
    return W


def mpo_d2_periodic(L: int, h: float) -> Mpo:
    """SI, Second Derivative, Centered, Periodic: bond 3, c0 = -2, c1 = 1."""
    c0, c1 = -2.0, 1.0
    first = [I2, SP + SM, SP + SM]
    bulk = [[I2, SP, SM], [Z2, SM, Z2], [Z2, Z2, SP]]
    last = [c0 * I2 + c1 * (SM + SP), c1 * SM, c1 * SP]
    W = _chain(first, bulk, last, L)
    W[0] = W[0] / (h * h)
    return W


def mpo_sum(mpos: Sequence[Mpo]) -> Mpo:
    """Direct sum of MPOs (SI, Addition, applied to operator-valued cores)."""
    n = len(mpos[0])
    out = []
    for j in range(n):
        blocks = [m[j] for m in mpos]
        if j == 0:
            out.append(np.concatenate(blocks, axis=3))
        elif j == n - 1:
            out.append(np.concatenate(blocks, axis=0))
        else:
            L = sum(b.shape[0] for b in blocks)
            R = sum(b.shape[3] for b in blocks)
            C = np.zeros((L, blocks[0].shape[1], blocks[0].shape[2], R))
            l0 = r0 = 0
            for b in blocks:
                C[l0:l0 + b.shape[0], :, :, r0:r0 + b.shape[3]] = b
                l0 += b.shape[0]
                r0 += b.shape[3]
            out.append(C)
    return out


def mpo_from_matrix(M: np.ndarray, L: int, tol: float = 1e-14) -> Mpo:
    """Dense N x N operator -> MPO with the bits of (o, i) paired per site
    (SI, Inverse Laplacian: build the matrix, then convert it)."""
    T = M.reshape([2] * (2 * L))
    perm = [k for j in range(L) for k in (j, L + j)]
    vec = T.transpose(perm).reshape(-1)
    cores = tt_svd(vec, [4] * L, tol=tol)
    return [c.reshape(c.shape[0], 2, 2, c.shape[2]) for c in cores]


def mpo_stencil_periodic(L: int, h: float, coeffs: dict) -> Mpo:
    """Circulant stencil (Af)_o = sum_d coeffs[d] f_{(o+d) mod N} / h as an
    MPO: the dense matrix converted by TT-SVD (SI, "Inverse Laplacian"
    route; small L only)."""
    N = 1 << L
    M = np.zeros((N, N))
    for d, c in coeffs.items():
        for o in range(N):
            M[o, (o + d) % N] += c / h
    return mpo_from_matrix(M, L)


# second-order one-sided periodic first derivatives (SI, Derivatives:
# forward c0 = -3/2, c1 = 2, c2 = -1/2 on f_i, f_{i+1}, f_{i+2}; backward
# c0 = 3/2, c1 = -2, c2 = 1/2 on f_i, f_{i-1}, f_{i-2})
D1_FORWARD = {0: -1.5, 1: 2.0, 2: -0.5}
D1_BACKWARD = {0: 1.5, -1: -2.0, -2: 0.5}


def mpo_d1_forward(L: int, h: float) -> Mpo:
    return mpo_stencil_periodic(L, h, D1_FORWARD)


def mpo_d1_backward(L: int, h: float) -> Mpo:
    return mpo_stencil_periodic(L, h, D1_BACKWARD)


def mpo_product(A: Mpo, B: Mpo) -> Mpo:
    """The operator product A B as an MPO: C(o, i) = sum_m A(o, m) B(m, i)
    site by site, bonds multiplied (A-major)."""
    out = []
    for Wa, Wb in zip(A, B):
        T = np.einsum("aomb,cmid->acoibd", Wa, Wb)
        a, c, o, i, b, d = T.shape
        out.append(T.reshape(a * c, o, i, b * d))
    return out


def mpo_to_matrix_d(W: Mpo, d: int) -> np.ndarray:
    """Dense matrix of an MPO whose sites have dimension d (tests)."""
    L = len(W)
    T = W[0]
    for Wj in W[1:]:
        T = np.tensordot(T, Wj, axes=(T.ndim - 1, 0))
    T = T.reshape([d] * (2 * L))
    perm = [2 * j for j in range(L)] + [2 * j + 1 for j in range(L)]
    N = d ** L
    return T.transpose(perm).reshape(N, N)


def mpo_to_matrix(W: Mpo) -> np.ndarray:
    """Contract an MPO to its dense N x N matrix (brute force, tests)."""
    L = len(W)
    T = W[0]
    for Wj in W[1:]:
        T = np.tensordot(T, Wj, axes=(T.ndim - 1, 0))
    T = T.reshape([2] * (2 * L))  # axes o1 i1 o2 i2 ...
    perm = [2 * j for j in range(L)] + [2 * j + 1 for j in range(L)]
    N = 2 ** L
    return T.transpose(perm).reshape(N, N)


def poisson_mpo(L: int, dx: float, tol: float = 1e-14) -> Mpo:
    """G = Dx L^+ as an MPO, E = -G n (Problem Statement eqs. 2-3, SI
    "Inverse Laplacian").

    The paper builds the dense inverse and converts it; for the periodic
    central difference and the pseudo-inverse of the periodic 3-point
    Laplacian that dense matrix has the closed form (discrete Green's
    function, derived by diagonalising both circulants)
        G[o, i] = dx * ( sign(o - i) / 2 - (o - i) / N ),  sign(0) = 0,
    i.e. the sawtooth dx (1/2 - m/N) of m = (o - i) mod N with G(0) = 0.
    Written element-wise over the paired bits (o_k, i_k), MSB first, it is
    the sum of a comparison automaton (bond 3: equal / greater / less so
    far) and a linear function of the bits (bond 2); the direct sum
    (bond 5) is compressed with `tol` (exact rank 3).  The tests pin this
    against pinv of the dense Laplacian built from the printed MPOs."""
    if L < 2:
        raise ValueError("operator MPOs need at least two sites")
    N = 2 ** L
    EQ, GT, LT = 0, 1, 2

    def step(s, o, i):
        if s != EQ:
            return s
        return EQ if o == i else (GT if o > i else LT)

    val = [0.0, 0.5 * dx, -0.5 * dx]
    sign = []
    for k in range(L):
        if k == 0:
            W = np.zeros((1, 2, 2, 3))
            for o in range(2):
                for i in range(2):
                    W[0, o, i, step(EQ, o, i)] = 1.0
        elif k < L - 1:
            W = np.zeros((3, 2, 2, 3))
            for s in range(3):
                for o in range(2):
                    for i in range(2):
                        W[s, o, i, step(s, o, i)] = 1.0
        else:
            W = np.zeros((3, 2, 2, 1))
            for s in range(3):
                for o in range(2):
                    for i in range(2):
                        W[s, o, i, 0] = val[step(s, o, i)]
        sign.append(W)
    lin = []
    for k in range(L):
        c = -dx * 2.0 ** (-1 - k)
        d = np.array([[0.0, -1.0], [1.0, 0.0]]) * c   # c (o - i)
        one = np.ones((2, 2))
        if k == 0:
            W = np.stack([one, d], axis=-1)[None]
        elif k < L - 1:
            W = np.zeros((2, 2, 2, 2))
            W[0, :, :, 0] = one
            W[0, :, :, 1] = d
            W[1, :, :, 1] = one
        else:
            W = np.stack([d, one], axis=0)[..., None]
        lin.append(W)
    G = mpo_sum([sign, lin])
    as_mps = [w.reshape(w.shape[0], 4, w.shape[3]) for w in G]
    as_mps = compress(as_mps, None, tol)
    return [c.reshape(c.shape[0], 2, 2, c.shape[2]) for c in as_mps]


def vector_mps(vec: np.ndarray, tol: float = 1e-14) -> Mps:
    L = int(round(math.log2(vec.size)))
    return tt_svd(vec, [2] * L, tol=tol)


# ------------------------------------------------------ orderings

def site_map(Lx: int, Lv: int, order: int) -> List[Tuple[str, int]]:
    """Fig. 3 orderings, as (dimension, bit k) per site, k = 0 the coarsest
    bit: 0 = S1 (x coarse->fine, then v coarse->fine), 1 = IF (x1, v1, x2,
    v2, ...), 2 = S2 (x fine->coarse, then v coarse->fine), 3 = S3 (x
    coarse->fine, then v fine->coarse), 4 = IG (IF with each pair x_k v_k
    fused into one site of dimension 4; this map lists its bits, which is
    also the order of the IG vector's base-4 digits)."""
    xs = [("x", k) for k in range(Lx)]
    vs = [("v", k) for k in range(Lv)]
    if order == 0:
        return xs + vs
    if order == 2:
        return xs[::-1] + vs
    if order == 3:
        return xs + vs[::-1]
    if order in (1, 4):
        if Lx != Lv:
            raise ValueError("interleaved ordering needs Lx == Lv")
        out = []
        for k in range(Lx):
            out += [("x", k), ("v", k)]
        return out
    raise ValueError("unknown ordering")


def site_dims(Lx: int, Lv: int, order: int) -> List[int]:
    """Physical dimension of each site: 4 for the fused IG sites, else 2."""
    return [4] * Lx if order == 4 else [2] * (Lx + Lv)


def fuse_pairs(cores: List[np.ndarray]) -> List[np.ndarray]:
    """Contract sites 2k and 2k+1 into one site of dimension 4 (fused index
    2 a + b, the first site's bit major): MPS cores (l, 2, r), MPO cores
    (l, o, i, r) with o and i fused alike."""
    out = []
    for a, b in zip(cores[0::2], cores[1::2]):
        if a.ndim == 3:
            T = np.einsum("lsm,mtr->lstr", a, b)
            out.append(T.reshape(a.shape[0], 4, b.shape[2]))
        else:
            T = np.einsum("loim,mpjr->lopijr", a, b)
            out.append(T.reshape(a.shape[0], 4, 4, b.shape[3]))
    return out


def reversed_dims(order: int) -> Tuple[bool, bool]:
    """Whether the x / v sites run from fine to coarse (S2 / S3).  A
    dimension visited fine to coarse uses its one-dimensional cores in
    reverse order with their two bonds swapped."""
    return order == 2, order == 3


def reverse_chain(cores: List[np.ndarray]) -> List[np.ndarray]:
    """The same tensor with the sites in reverse order: MPS cores (l, 2, r)
    -> (r, 2, l), MPO cores (l, o, i, r) -> (r, o, i, l)."""
    return [np.swapaxes(A, 0, A.ndim - 1) for A in cores[::-1]]


def dense_to_sites(F: np.ndarray, Lx: int, Lv: int, order: int) -> np.ndarray:
    """F[i, j] -> vector indexed by the site bits in chain order."""
    T = F.reshape([2] * (Lx + Lv))
    perm = [k if d == "x" else Lx + k for d, k in site_map(Lx, Lv, order)]
    return T.transpose(perm).reshape(-1)


def sites_to_dense(vec: np.ndarray, Lx: int, Lv: int, order: int) -> np.ndarray:
    perm = [k if d == "x" else Lx + k for d, k in site_map(Lx, Lv, order)]
    T = vec.reshape([2] * (Lx + Lv))
    inv = np.argsort(perm)
    return T.transpose(inv).reshape(2 ** Lx, 2 ** Lv)


def chain_mpo(Wx: Optional[Mpo], Wv: Optional[Mpo], Lx: int, Lv: int,
              order: int) -> Mpo:
    if order == 4:
        return fuse_pairs(chain_mpo(Wx, Wv, Lx, Lv, 1))
    return _chain_mpo_binary(Wx, Wv, Lx, Lv, order)


def _chain_mpo_binary(Wx: Optional[Mpo], Wv: Optional[Mpo], Lx: int, Lv: int,
                      order: int) -> Mpo:
    """Full-chain MPO of (x-operator) (x) (v-operator).  On a site of the
    other dimension an operator acts as delta_{bl,br} I_2, so in the
    interleaved order the bonds multiply (fused index x-major)."""
    Wx = Wx if Wx is not None else [np.eye(2).reshape(1, 2, 2, 1)] * Lx
    Wv = Wv if Wv is not None else [np.eye(2).reshape(1, 2, 2, 1)] * Lv
    rx, rv = reversed_dims(order)
    if rx:
        Wx = reverse_chain(Wx)[::-1]   # core k, bonds swapped
    if rv:
        Wv = reverse_chain(Wv)[::-1]
    bx = 1   # current x bond (right bond of the last x site seen)
    bv = 1
    out = []
    for d, k in site_map(Lx, Lv, order):
        if d == "x":
            W = Wx[k]
            T = np.einsum("aoib,cd->acoibd", W, np.eye(bv))
            a, c, o, i, b, dd = T.shape
            out.append(T.reshape(a * c, o, i, b * dd))
            bx = W.shape[3]
        else:
            W = Wv[k]
            T = np.einsum("cd,aoib->caoidb", np.eye(bx), W)
            c, a, o, i, d_, b = T.shape
            out.append(T.reshape(c * a, o, i, d_ * b))
            bv = W.shape[3]
    return out


def chain_product_mps(ux: Optional[Mps], uv: Optional[Mps], Lx: int, Lv: int,
                      order: int) -> Mps:
    if order == 4:
        return fuse_pairs(chain_product_mps(ux, uv, Lx, Lv, 1))
    return _chain_product_binary(ux, uv, Lx, Lv, order)


def _chain_product_binary(ux: Optional[Mps], uv: Optional[Mps], Lx: int, Lv: int,
                          order: int) -> Mps:
    """Full-chain MPS of a product function u(x) w(v) (same embedding)."""
    ux = ux if ux is not None else [np.ones((1, 2, 1))] * Lx
    uv = uv if uv is not None else [np.ones((1, 2, 1))] * Lv
    rx, rv = reversed_dims(order)
    if rx:
        ux = reverse_chain(ux)[::-1]
    if rv:
        uv = reverse_chain(uv)[::-1]
    bx = bv = 1
    out = []
    for d, k in site_map(Lx, Lv, order):
        if d == "x":
            A = ux[k]
            T = np.einsum("asb,cd->acsbd", A, np.eye(bv))
            a, c, s, b, e = T.shape
            out.append(T.reshape(a * c, s, b * e))
            bx = A.shape[2]
        else:
            A = uv[k]
            T = np.einsum("cd,asb->casdb", np.eye(bx), A)
            c, a, s, e, b = T.shape
            out.append(T.reshape(c * a, s, e * b))
            bv = A.shape[2]
    return out


# ------------------------------------------------------ physics on MPS

def density_mps(f: Mps, Lx: int, Lv: int, order: int, dv: float) -> Mps:
    """n(x) = <Iv, f>_v with Iv = dv [1,1]^{(x) Lv} (SI, Integration): each
    v-core summed over its bit; the resulting bond matrix is absorbed into
    the neighbouring x core.  Returns an Lx-site MPS in the natural bit
    order (coarsest first) whatever the ordering of f."""
    if order == 4:
        # each fused site (x_k, v_k): sum over its v bit
        xs = [A.reshape(A.shape[0], 2, 2, A.shape[2]).sum(axis=2) for A in f]
        xs[0] = xs[0] * dv
        return xs
    xs: Mps = []
    pending = None
    for (d, k), A in zip(site_map(Lx, Lv, order), f):
        if d == "v":
            M = A.sum(axis=1)
            if xs:
                xs[-1] = np.tensordot(xs[-1], M, axes=(2, 0))
            else:
                pending = M if pending is None else pending @ M
        else:
            C = A if pending is None else np.tensordot(pending, A, axes=(1, 0))
            pending = None
            xs.append(C)
    if reversed_dims(order)[0]:
        xs = reverse_chain(xs)
    xs[0] = xs[0] * dv
    return xs


class Operators:
    """The fixed operators of one problem (built once, SI Derivatives /
    Dot Product / Inverse Laplacian / Integration)."""

    def __init__(self, p):
        self.p = p
        self.Dx = mpo_d1_periodic(p.Lx, p.dx)
        self.Dv = mpo_d1_zero_gradient(p.Lv, p.dv)
        self.V = diag_mpo(vector_mps(p.v()))
        self.G = poisson_mpo(p.Lx, p.dx)
        if getattr(p, "x_scheme", 0) == 1:
            # upwind: T1 = -(Db (x) diag(v H(v)) + Df (x) diag(v (1 - H(v))))
            v = p.v()
            Wp = diag_mpo(vector_mps(np.maximum(v, 0.0)))
            Wn = diag_mpo(vector_mps(np.minimum(v, 0.0)))
            self.T1 = mpo_sum([chain_mpo(mpo_d1_backward(p.Lx, p.dx), Wp, p.Lx, p.Lv, p.order),
                               chain_mpo(mpo_d1_forward(p.Lx, p.dx), Wn, p.Lx, p.Lv, p.order)])
        else:
            # T1 = -(Dx (x) V) f
            self.T1 = chain_mpo(self.Dx, self.V, p.Lx, p.Lv, p.order)
        self.T1[0] = -self.T1[0]
        # Dougherty collisions (Methods, Collision Operator)
        self.T3 = None
        self.moments = False
        if getattr(p, "nu", 0.0) != 0.0:
            if getattr(p, "coll_model", 0) == 1:
                # fixed drift and thermal speed: nu Dv (diag(v - v0) + vth^2 Dv)
                inner = mpo_sum([diag_mpo(vector_mps(p.v() - p.nu_v0)),
                                 [W * (p.nu_vth ** 2 if j == 0 else 1.0)
                                  for j, W in enumerate(self.Dv)]])
                Cv = mpo_product(self.Dv, inner)
                Cv[0] = Cv[0] * p.nu
                self.T3 = chain_mpo(None, Cv, p.Lx, p.Lv, p.order)
            else:
                # moments of the state: nu Dv diag(v) is fixed; the terms with
                # v0(x) and vth^2(x) are built per stage (rhs_mps)
                self.moments = True
                Cv = mpo_product(self.Dv, diag_mpo(vector_mps(p.v())))
                Cv[0] = Cv[0] * p.nu
                self.T3 = chain_mpo(None, Cv, p.Lx, p.Lv, p.order)
                self.DvDv = mpo_product(self.Dv, self.Dv)
                self.Vw = chain_mpo(None, diag_mpo(vector_mps(p.v())), p.Lx, p.Lv, p.order)
                self.V2w = chain_mpo(None, diag_mpo(vector_mps(p.v() ** 2)), p.Lx, p.Lv,
                                     p.order)


def field_mps(g: Mps, ops: Operators) -> Mps:
    """E = compress(-G n, D_F, tol)."""
    p = ops.p
    n = density_mps(g, p.Lx, p.Lv, p.order, p.dv)
    En = scale(apply(ops.G, n), -1.0)
    return compress(En, p.df_max if p.df_max > 0 else None, p.tol)


def compress_state(m: Mps, chi: Optional[int], p) -> Mps:
    """Compression of a full-chain MPS at one of the points P1-P5: the sweep
    of SI "Canonicalization and Compression", or, when p.compression == 1
    (sequential orderings), the centre-first scheme of SI "Modified
    Compression Scheme" with its centre at the x|v bond."""
    if getattr(p, "compression", 0) == 1:
        if p.order not in (0, 2, 3):
            raise ValueError("centre-first compression needs a sequential ordering")
        return compress_centre(m, p.Lx, chi, p.tol)
    return compress(m, chi, p.tol)


def caps(p, point: int) -> Optional[int]:
    """Level C_l caps compression points P1..P_l at chi."""
    return p.chi_max if p.level >= point else None


def x_field_mps(u: np.ndarray, p) -> Mps:
    """A function of x on the grid (natural bit order) as an x-MPS: iterated
    SVD (eq. 4, relative cut 1e-14 when tol > 0, exact when tol = 0), then
    compressed like the field E (cap D_F, tol)."""
    m = tt_svd(u, [2] * p.Lx, tol=1e-14 if p.tol > 0 else 0.0)
    return compress(m, p.df_max if p.df_max > 0 else None, p.tol)


def collision_moment_fields(g: Mps, ops: Operators):
    """x-MPS of the local drift v0(x) and of vth^2(x) of g (the Dougherty
    operator's average and thermal velocity): the contractions n, <v, g>_v
    and <v^2, g>_v as x-MPS, evaluated on the grid of x, divided there."""
    p = ops.p
    n = to_vector(density_mps(g, p.Lx, p.Lv, p.order, p.dv))
    P = to_vector(density_mps(apply(ops.Vw, g), p.Lx, p.Lv, p.order, p.dv))
    W = to_vector(density_mps(apply(ops.V2w, g), p.Lx, p.Lv, p.order, p.dv))
    ok = n != 0.0
    v0 = np.zeros_like(n)
    v0[ok] = P[ok] / n[ok]
    T = np.zeros_like(n)
    T[ok] = W[ok] / n[ok] - v0[ok] ** 2
    return x_field_mps(v0, p), x_field_mps(T, p)


def rhs_mps(g: Mps, ops: Operators, E: Optional[Mps] = None) -> Mps:
    """k = R(g): T1 = -(Dx (x) V) g, T2 = -(q/m)(diag(E) (x) Dv) g and, with
    collisions, C g (one term with fixed v0 and vth; three with the moments
    of g: nu Dv diag(v) g, -nu (diag(v0) (x) Dv) g, nu (diag(vth^2) (x)
    Dv Dv) g), each compressed (P5), then their sum compressed (P4).  E from
    g alone (one electron species) unless given."""
    p = ops.p
    if E is None:
        E = field_mps(g, ops)
    WE = diag_mpo(E)
    WE[0] = WE[0] * (-p.qm)
    W2 = chain_mpo(WE, ops.Dv, p.Lx, p.Lv, p.order)
    terms = [compress_state(apply(ops.T1, g), caps(p, 5), p),
             compress_state(apply(W2, g), caps(p, 5), p)]
    if ops.T3 is not None:
        terms.append(compress_state(apply(ops.T3, g), caps(p, 5), p))
    if ops.moments:
        v0, T = collision_moment_fields(g, ops)
        Wu = diag_mpo(v0)
        Wu[0] = Wu[0] * (-p.nu)
        WT = diag_mpo(T)
        WT[0] = WT[0] * p.nu
        terms.append(compress_state(apply(chain_mpo(Wu, ops.Dv, p.Lx, p.Lv, p.order), g),
                                    caps(p, 5), p))
        terms.append(compress_state(apply(chain_mpo(WT, ops.DvDv, p.Lx, p.Lv, p.order), g),
                                    caps(p, 5), p))
    return compress_state(add([(1.0, T) for T in terms]), caps(p, 4), p)


def field_species_mps(gs: Sequence[Mps], opss: Sequence[Operators],
                      charges: Sequence[float]) -> Mps:
    """E of several species: rho = sum_s (-q_s) n_s as a direct sum (exact),
    then E = compress(-G rho, D_F, tol) with the first species' settings."""
    ns = [density_mps(g, o.p.Lx, o.p.Lv, o.p.order, o.p.dv) for g, o in zip(gs, opss)]
    rho = add([(-q, n) for q, n in zip(charges, ns)])
    p = opss[0].p
    En = scale(apply(opss[0].G, rho), -1.0)
    return compress(En, p.df_max if p.df_max > 0 else None, p.tol)


def rk4_step_species(fs: Sequence[Mps], opss: Sequence[Operators],
                     charges: Sequence[float], dt: float) -> List[Mps]:
    """RK4 of all species together (compression points per species as in
    rk4_step), the field of each stage from all of them."""
    def R(gs):
        E = field_species_mps(gs, opss, charges)
        return [rhs_mps(g, o, E) for g, o in zip(gs, opss)]

    def stage(ks, c):
        return [compress_state(add([(1.0, f), (c, k)]), caps(o.p, 2), o.p)
                for f, k, o in zip(fs, ks, opss)]
    k1 = R(fs)
    k2 = R(stage(k1, 0.5 * dt))
    k3 = R(stage(k2, 0.5 * dt))
    k4 = R(stage(k3, dt))
    out = []
    for f, a, b, c, d, o in zip(fs, k1, k2, k3, k4, opss):
        S = compress_state(add([(1.0, a), (2.0, b), (2.0, c), (1.0, d)]), caps(o.p, 3), o.p)
        out.append(compress_state(add([(1.0, f), (dt / 6.0, S)]), o.p.chi_max, o.p))
    return out


def cfl_dt(f: Mps, ops: Operators) -> float:
    """Adaptive step (Methods, eq. CFL, one collisionless species): cfl *
    (|v|_max / dx + |q/m| |E|_max / dv)^-1, |E|_max of the field of f."""
    p = ops.p
    vmax = max(abs(p.v_min), abs(p.v_max))
    emax = float(np.abs(field_dense(f, ops)).max())
    inv = vmax / p.dx + abs(p.qm) * emax / p.dv
    nu = getattr(p, "nu", 0.0)
    if nu != 0.0:
        # the collision terms of eq. CFL
        inv += nu * vmax / p.dv + 2.0 * nu * p.nu_vth ** 2 / p.dv ** 2
    return p.cfl / inv


def rk4_step(f: Mps, ops: Operators) -> Mps:
    """SI, Compressed time evolution: RK4 with compression points P1-P5; the
    fixed dt, or the adaptive CFL step when p.cfl > 0."""
    p = ops.p
    h = cfl_dt(f, ops) if getattr(p, "cfl", 0.0) > 0.0 else p.dt
    k1 = rhs_mps(f, ops)
    f2 = compress_state(add([(1.0, f), (0.5 * h, k1)]), caps(p, 2), p)
    k2 = rhs_mps(f2, ops)
    f3 = compress_state(add([(1.0, f), (0.5 * h, k2)]), caps(p, 2), p)
    k3 = rhs_mps(f3, ops)
    f4 = compress_state(add([(1.0, f), (h, k3)]), caps(p, 2), p)
    k4 = rhs_mps(f4, ops)
    S = compress_state(add([(1.0, k1), (2.0, k2), (2.0, k3), (1.0, k4)]),
                       caps(p, 3), p)
    return compress_state(add([(1.0, f), (h / 6.0, S)]), p.chi_max, p)


def init_mps(p, ax: np.ndarray, bv: np.ndarray) -> Mps:
    """f0 on the grid -> MPS by iterated SVD in chain order (eq. 4), then
    compressed to (chi, tol)."""
    F = np.einsum("ri,rj->ij", ax, bv)
    vec = dense_to_sites(F, p.Lx, p.Lv, p.order)
    m = tt_svd(vec, site_dims(p.Lx, p.Lv, p.order), tol=p.tol, chi=None)
    return compress_state(m, p.chi_max, p)


def to_dense(f: Mps, p) -> np.ndarray:
    return sites_to_dense(to_vector(f), p.Lx, p.Lv, p.order)


def field_dense(f: Mps, ops: Operators) -> np.ndarray:
    return to_vector(field_mps(f, ops))


def moments(f: Mps, ops: Operators) -> dict:
    """Mass, momentum, kinetic energy as full contractions with the product
    MPS 1(x) w(v) (w = 1, v, v^2/2) times dx dv; field energy from E."""
    p = ops.p
    v = p.v()
    out = {}
    for name, w in (("mass", np.ones_like(v)), ("momentum", v),
                    ("kinetic", 0.5 * v * v)):
        g = chain_product_mps(None, vector_mps(w), p.Lx, p.Lv, p.order)
        out[name] = p.dx * p.dv * inner(g, f)
    E = field_dense(f, ops)
    out["field_energy"] = 0.5 * p.dx * float(np.sum(E * E))
    return out
