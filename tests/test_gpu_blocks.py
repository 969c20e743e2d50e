"""GPU parity of the building blocks against NumPy/LAPACK and the CPU MPS
oracle, through the C-ABI (include/mps_blocks.h)."""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import mps as omps

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2205_11990_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (7, 5, 3), (64, 64, 16), (65, 130, 33),
                                   (300, 17, 129), (16, 1000, 2)])
def test_gemm_matches_numpy(B, M, N, K):
    _say("gemm %d %d %d" % (M, N, K))
    rng = np.random.default_rng(M * 1000 + N * 10 + K)
    A = rng.standard_normal((M, K))
    Bm = rng.standard_normal((K, N))
    C0 = rng.standard_normal((M, N))
    import torch
    C = torch.from_numpy(C0.copy()).cuda()
    out = B.gemm(A, Bm, alpha=0.7, beta=-1.3, C=C).cpu().numpy()
    ref = 0.7 * A @ Bm - 1.3 * C0
    assert np.abs(out - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()) * np.sqrt(K)


@pytest.mark.parametrize("M,N,K,batch,at,bt", [
    (4096, 2048, 64, 1, False, False), (4100, 2050, 37, 1, False, False),
    (4096, 2048, 128, 1, True, False), (2049, 4097, 48, 1, False, True),
    (2048, 2048, 33, 1, True, True), (2048, 1024, 128, 4, False, False),
    (20480, 256, 128, 1, False, False), (1000, 999, 17, 3, True, True)])
def test_gemm_strided_matches_numpy(B, M, N, K, batch, at, bt):
    """Strided batched GEMM with either operand transposed (read through its
    strides), ragged sizes and several batch entries; shapes with enough
    128 x 128 tiles take the large-tile kernel."""
    import torch
    _say("gemm strided %d %d %d batch %d at=%d bt=%d" % (M, N, K, batch, at, bt))
    rng = np.random.default_rng(M + N + K + batch)
    A = rng.standard_normal((batch, M, K))
    Bm = rng.standard_normal((batch, K, N))
    C0 = rng.standard_normal((batch, M, N))
    # stored transposed when asked: the kernel reads element (i, k) of A at
    # i*ars + k*acs
    Ad = torch.from_numpy(np.ascontiguousarray(A.transpose(0, 2, 1) if at else A)).cuda()
    Bd = torch.from_numpy(np.ascontiguousarray(Bm.transpose(0, 2, 1) if bt else Bm)).cuda()
    Cd = torch.from_numpy(C0.copy()).cuda()
    a_str = (1, M, M * K) if at else (K, 1, M * K)
    b_str = (1, K, K * N) if bt else (N, 1, K * N)
    out = B.gemm_strided(M, N, K, 0.7, Ad, a_str, Bd, b_str, -1.3, Cd, (N, 1, M * N),
                         batch=batch).cpu().numpy()
    ref = 0.7 * np.einsum("bik,bkj->bij", A, Bm) - 1.3 * C0
    assert np.abs(out - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()) * np.sqrt(K)


@pytest.mark.parametrize("M,N,K,batch,bt,beta", [
    (12, 64, 12, 384, False, 0.0), (40, 512, 40, 64, False, -1.3), (40, 64, 40, 512, True, 0.5),
    (33, 100, 7, 50, False, 2.0), (16, 1030, 48, 1, False, 0.0), (48, 64, 1, 40, True, -1.0),
    (1, 2000, 5, 3, False, 0.25)])
def test_gemm_small_shared_factor_matches_numpy(B, M, N, K, batch, bt, beta):
    """A small factor (at most 48 x 48) shared by every batch entry (A's
    batch stride 0) times many columns, as the MPO applications multiply:
    the streaming kernel, against numpy, with B read transposed through its
    strides and beta applied to C."""
    import torch
    _say("gemm small shared %d %d %d batch %d bt=%d" % (M, N, K, batch, bt))
    rng = np.random.default_rng(M * 7 + N + K + batch)
    A = rng.standard_normal((M, K))
    Bm = rng.standard_normal((batch, K, N))
    C0 = rng.standard_normal((batch, M, N))
    Ad = torch.from_numpy(A.copy()).cuda()
    Bd = torch.from_numpy(np.ascontiguousarray(Bm.transpose(0, 2, 1) if bt else Bm)).cuda()
    Cd = torch.from_numpy(C0.copy()).cuda()
    b_str = (1, K, K * N) if bt else (N, 1, K * N)
    out = B.gemm_strided(M, N, K, 0.7, Ad, (K, 1, 0), Bd, b_str, beta, Cd, (N, 1, M * N),
                         batch=batch).cpu().numpy()
    ref = 0.7 * np.einsum("ik,bkj->bij", A, Bm) + beta * C0
    assert np.abs(out - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()) * np.sqrt(K)


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (7, 5, 3), (64, 64, 16), (65, 130, 33),
                                   (300, 17, 129), (16, 1000, 2)])
def test_gemm_fp32_contract_matches_fp32_rounded_product(B, M, N, K):
    """Precision mode 1: the product of the FP32-rounded operands,
    accumulated in FP32 (checked against the exact product of the rounded
    operands at FP32 accumulation accuracy)."""
    _say("gemm fp32 %d %d %d" % (M, N, K))
    rng = np.random.default_rng(M * 1000 + N * 10 + K + 1)
    A = rng.standard_normal((M, K))
    Bm = rng.standard_normal((K, N))
    out = B.gemm(A, Bm, alpha=0.5, precision=1).cpu().numpy()
    Ar = A.astype(np.float32).astype(np.float64)
    Br = Bm.astype(np.float32).astype(np.float64)
    ref = 0.5 * Ar @ Br
    scale = 0.5 * (np.abs(Ar) @ np.abs(Br))
    assert np.all(np.abs(out - ref) <= 4 * K * 6e-8 * scale + 1e-30)


def _bf16(x):
    """Round to FP32, then to the nearest BF16 (ties to even), as float64."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (7, 5, 3), (64, 64, 16), (65, 130, 33),
                                   (200, 96, 700), (3, 300, 2000)])
def test_gemm_bf16_contract_matches_bf16_rounded_product(B, M, N, K):
    """Precision mode 2: the product of the BF16-rounded operands (exact in
    FP32), accumulated in FP32."""
    _say("gemm bf16 %d %d %d" % (M, N, K))
    rng = np.random.default_rng(M * 1000 + N * 10 + K + 2)
    A = rng.standard_normal((M, K))
    Bm = rng.standard_normal((K, N))
    out = B.gemm(A, Bm, alpha=0.5, precision=2).cpu().numpy()
    Ar, Br = _bf16(A), _bf16(Bm)
    assert np.all(np.abs(Ar - A) <= 2.0 ** -8 * np.abs(A))
    ref = 0.5 * Ar @ Br
    scale = 0.5 * (np.abs(Ar) @ np.abs(Br))
    assert np.all(np.abs(out - ref) <= 4 * K * 6e-8 * scale + 1e-30)


@pytest.mark.parametrize("m,n", [(1, 1), (5, 3), (3, 5), (40, 40), (130, 70), (257, 33),
                                 (600, 200), (2048, 8), (64, 300), (128, 128), (256, 128),
                                 (512, 64), (1024, 128), (1000, 100), (200, 129), (700, 700),
                                 (65, 17), (2048, 40), (1500, 300), (2048, 512),
                                 # taller than 2048 rows: TSQR panels
                                 (4000, 64), (2049, 700), (5120, 256), (8200, 48),
                                 (3000, 3000)])
def test_qr_is_orthogonal_factorisation(B, m, n):
    _say("qr %d x %d" % (m, n))
    A = wl.random_matrix(m, n, seed=m + 7 * n, decay=3.0)
    R, Q = B.qr(A)
    R = R.cpu().numpy()
    Q = Q.cpu().numpy()
    k = min(m, n)
    assert np.abs(Q.T @ Q - np.eye(k)).max() < 1e-13 * max(1, np.sqrt(m))
    assert np.abs(Q @ R - A).max() < 1e-13 * np.abs(A).max() * max(1, np.sqrt(m))
    assert np.allclose(np.tril(R, -1), 0)
    Rref = np.linalg.qr(A, mode="r")
    assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(Rref[:k])), rtol=1e-10, atol=1e-13)


@pytest.mark.parametrize("m,n", [(63, 21), (128, 127), (250, 101), (500, 77), (1000, 45)])
def test_qr_with_zero_and_repeated_columns(B, m, n):
    """Exactly rank-deficient columns give reflectors with tau = 0 (the
    identity) in the middle of the factor; the numbers of reflectors are
    not multiples of the application's block of four.  Q stays orthogonal
    and QR = A."""
    _say("qr rank-deficient columns %d x %d" % (m, n))
    A = wl.random_matrix(m, n, seed=5 * m + n, decay=2.0)
    A[:, 3] = 0.0
    A[:, 4] = 0.0
    A[:, 10] = A[:, 9]
    A[:, n - 1] = 0.0
    R, Q = B.qr(A)
    R = R.cpu().numpy()
    Q = Q.cpu().numpy()
    k = min(m, n)
    assert np.abs(Q.T @ Q - np.eye(k)).max() < 1e-13 * max(1, np.sqrt(m))
    assert np.abs(Q @ R - A).max() < 1e-13 * np.abs(A).max() * max(1, np.sqrt(m))
    assert np.allclose(np.tril(R, -1), 0)


@pytest.mark.parametrize("m,n,rankdef", [(600, 100, False), (1024, 512, False), (2048, 512, False),
                                          (1100, 300, True), (700, 64, False), (2048, 40, True),
                                          (530, 530, False), (1500, 70, False), (513, 33, True)])
def test_qr_panel_groups_of_the_compact_wy_mode(B, m, n, rankdef):
    """Blocks over 512 rows in the compact-WY mode are factored in groups of
    four 16-column panels whose 64 reflectors reach the trailing columns and
    the products with Q as one block (last groups of fewer panels and a
    last panel of fewer columns included): the same factorisation as the
    one-reflector mode up to rounding, Q orthogonal and QR = A."""
    _say("qr panel groups %d x %d" % (m, n))
    A = wl.random_matrix(m, n, seed=3 * m + n, decay=3.0)
    if rankdef:
        A[:, 5] = 0.0
        A[:, 20] = A[:, 19]
    R1, Q1 = B.qr(A, tall_apply=1)
    R0, Q0 = B.qr(A, tall_apply=0)
    R1, Q1, R0, Q0 = (x.cpu().numpy() for x in (R1, Q1, R0, Q0))
    k = min(m, n)
    scale = np.abs(A).max()
    assert np.abs(Q1.T @ Q1 - np.eye(k)).max() < 1e-13 * np.sqrt(m)
    assert np.abs(Q1 @ R1 - A).max() < 1e-13 * scale * np.sqrt(m)
    assert np.allclose(np.tril(R1, -1), 0)
    # the same reflectors (LAPACK signs) in both modes: R and Q agree to
    # rounding while the columns are independent (a duplicated column's
    # reflector is built from rounding noise, so rows from it on differ)
    lead = 20 if rankdef else k
    assert np.abs(R1[:lead] - R0[:lead]).max() < 1e-11 * scale * np.sqrt(m)
    assert np.abs(Q1[:, :lead] - Q0[:, :lead]).max() < 1e-10


@pytest.mark.parametrize("m,c,cap,tol,decay", [
    (2, 2, 0, 0.0, 0), (10, 4, 0, 0.0, 0), (4, 10, 0, 0.0, 0), (64, 64, 0, 0.0, 6),
    (96, 96, 40, 0.0, 8), (128, 128, 64, 0.0, 8), (500, 128, 64, 0.0, 12),
    (300, 60, 0, 1e-10, 14), (33, 90, 0, 1e-6, 10), (1024, 16, 8, 0.0, 2),
    (2000, 128, 64, 0.0, 10), (60, 1500, 0, 1e-8, 6),
    # 129..256 columns: the two-workgroup Jacobi kernel
    (129, 129, 0, 0.0, 6), (256, 256, 128, 0.0, 10), (1024, 256, 128, 0.0, 12),
    (200, 256, 0, 1e-10, 14), (256, 600, 100, 0.0, 8), (3000, 160, 0, 1e-12, 16),
    # more than 256 columns in the smaller dimension: the global-memory Jacobi
    (300, 300, 0, 0.0, 8), (600, 300, 150, 0.0, 10), (300, 700, 0, 1e-10, 12),
    (512, 512, 0, 1e-10, 12), (1000, 1000, 300, 0.0, 10)])
def test_svd_truncate_matches_lapack_and_rank_rule(B, m, c, cap, tol, decay):
    _say("svd %d x %d cap %d tol %g" % (m, c, cap, tol))
    X = wl.random_matrix(m, c, seed=3 * m + c, decay=decay)
    Vt, US, sig, disc = B.svd_truncate(X, cap=cap, tol=tol)
    Vt, US, sig = Vt.cpu().numpy(), US.cpu().numpy(), sig.cpu().numpy()
    s = np.linalg.svd(X, compute_uv=False)
    assert np.abs(sig - s).max() <= 1e-13 * s[0] * np.sqrt(max(m, c))
    D = omps.rank_rule(s, cap if cap > 0 else None, tol)
    assert Vt.shape[0] == D
    assert np.abs(Vt @ Vt.T - np.eye(D)).max() < 1e-12
    # truncated reconstruction equals the best rank-D approximation
    U, S, W = np.linalg.svd(X, full_matrices=False)
    best = (U[:, :D] * S[:D]) @ W[:D]
    assert np.abs(US @ Vt - best).max() <= 1e-12 * s[0] * np.sqrt(max(m, c))
    ref_disc = np.sqrt(np.sum(s[D:] ** 2) / np.sum(s ** 2))
    assert abs(disc - ref_disc) <= 1e-12 + 1e-8 * ref_disc


@pytest.mark.parametrize("m,c,r", [(128, 128, 5), (256, 128, 1), (64, 128, 3), (100, 40, 0),
                                   (96, 128, 60), (512, 128, 17), (256, 256, 7),
                                   (300, 200, 0), (256, 256, 150), (512, 192, 1)])
def test_svd_truncate_rank_deficient(B, m, c, r):
    """Numerically rank-deficient blocks (as in the TT-SVD of a separable
    profile): the kept rows of Vt are orthonormal or exactly zero and the
    product US Vt reproduces X."""
    _say("svd rank-deficient %d x %d rank %d" % (m, c, r))
    rng = np.random.default_rng(m + c + r)
    X = rng.standard_normal((m, r)) @ rng.standard_normal((r, c)) if r else np.zeros((m, c))
    Vt, US, sig, disc = B.svd_truncate(X, cap=0, tol=0.0)
    Vt, US, sig = Vt.cpu().numpy(), US.cpu().numpy(), sig.cpu().numpy()
    scale = max(np.abs(X).max(), 1e-300)
    assert np.abs(US @ Vt - X).max() <= 1e-13 * scale * np.sqrt(max(m, c))
    nz = np.abs(Vt).max(axis=1) > 0
    assert nz.sum() >= r
    if nz.any():
        G = Vt[nz] @ Vt[nz].T
        assert np.abs(G - np.eye(G.shape[0])).max() < 1e-12
    if r:
        s = np.linalg.svd(X, compute_uv=False)
        assert np.abs(sig[:r] - s[:r]).max() <= 1e-13 * s[0] * np.sqrt(max(m, c))


def _random_mps(n, chi, seed, decay=0.0):
    cores = wl.random_mps_cores(n, chi, seed=seed)
    if decay:
        # graded bonds so that truncation is non-degenerate
        for j, c in enumerate(cores[:-1]):
            r = c.shape[2]
            c *= (10.0 ** (-decay * np.arange(r) / max(r, 1)))[None, None, :]
    return cores


@pytest.mark.parametrize("n,chi,cap,tol", [(6, 8, 0, 0.0), (10, 16, 8, 0.0), (12, 32, 0, 1e-10),
                                           (9, 12, 5, 0.0), (16, 24, 10, 1e-8)])
def test_compress_matches_oracle(B, n, chi, cap, tol):
    _say("compress n=%d chi=%d cap=%d tol=%g" % (n, chi, cap, tol))
    cores = _random_mps(n, chi, seed=n + chi, decay=3.0)
    out, disc = B.compress(cores, cap=cap, tol=tol)
    ref, rdisc = omps.compress(cores, cap if cap > 0 else None, tol, return_discarded=True)
    assert omps.bond_dims(out) == omps.bond_dims(ref)
    v, r = omps.to_vector(out), omps.to_vector(ref)
    assert np.abs(v - r).max() <= 1e-10 * np.abs(r).max()
    assert np.allclose(disc, rdisc, atol=1e-12, rtol=1e-6)


@pytest.mark.parametrize("n,centre,chi,cap,tol", [(8, 4, 8, 0, 0.0), (8, 4, 8, 3, 0.0),
                                                  (9, 5, 12, 6, 0.0), (10, 5, 16, 0, 1e-3),
                                                  (7, 2, 6, 4, 1e-6), (7, 6, 6, 3, 0.0),
                                                  (12, 6, 32, 16, 0.0),
                                                  (16, 8, 160, 128, 0.0)])
def test_compress_centre_matches_oracle(B, n, centre, chi, cap, tol):
    """Centre-first compression (SI, Modified Compression Scheme) through
    the C-ABI against the oracle: the same represented vector, bonds and
    per-bond discarded weights; the last case cuts 128-wide factorisations
    on both sides of the centre."""
    _say("compress_centre n=%d centre=%d chi=%d cap=%d tol=%g" % (n, centre, chi, cap, tol))
    cores = _random_mps(n, chi, seed=3 * n + centre + chi, decay=3.0)
    out, disc = B.compress_centre(cores, centre, cap=cap, tol=tol)
    ref, rdisc = omps.compress_centre(cores, centre, cap if cap > 0 else None, tol,
                                      return_discarded=True)
    assert omps.bond_dims(out) == omps.bond_dims(ref)
    v, r = omps.to_vector(out), omps.to_vector(ref)
    assert np.abs(v - r).max() <= 1e-10 * np.abs(r).max()
    assert np.allclose(disc, rdisc, atol=1e-12, rtol=1e-6)
    if cap == 0 and tol == 0.0:
        w = omps.to_vector(cores)
        assert np.abs(v - w).max() <= 1e-12 * np.abs(w).max()


@pytest.mark.parametrize("n,chi,cap", [(6, 4, 0), (10, 8, 12), (12, 16, 0)])
def test_apply_compress_matches_oracle(B, n, chi, cap):
    _say("apply+compress n=%d chi=%d cap=%d" % (n, chi, cap))
    cores = _random_mps(n, chi, seed=2 * n + chi, decay=2.0)
    W = omps.mpo_d1_periodic(n, 0.3)
    W = omps.mpo_sum([W, omps.diag_mpo(omps.vector_mps(np.linspace(-1, 2, 2 ** n)))])
    out, _ = B.compress(cores, cap=cap, tol=0.0, mpo=W)
    ref = omps.compress(omps.apply(W, cores), cap if cap > 0 else None, 0.0)
    v, r = omps.to_vector(out), omps.to_vector(ref)
    assert np.abs(v - r).max() <= 1e-10 * np.abs(r).max()
    if cap == 0:
        dense = omps.mpo_to_matrix(W) @ omps.to_vector(cores)
        assert np.abs(v - dense).max() <= 1e-10 * np.abs(dense).max()


def test_add_compress_matches_oracle(B):
    _say("add+compress")
    a = _random_mps(10, 8, seed=1, decay=2.0)
    b = _random_mps(10, 6, seed=2, decay=2.0)
    c = _random_mps(10, 4, seed=3, decay=2.0)
    terms = [(1.0, a), (-0.25, b), (2.0, c)]
    out = B.add_compress(terms, cap=0, tol=0.0)
    ref = omps.add(terms)
    v, r = omps.to_vector(out), omps.to_vector(ref)
    assert np.abs(v - r).max() <= 1e-11 * np.abs(r).max()
    out5 = B.add_compress(terms, cap=5, tol=0.0)
    ref5 = omps.compress(ref, 5, 0.0)
    assert np.abs(omps.to_vector(out5) - omps.to_vector(ref5)).max() <= 1e-10 * np.abs(r).max()
