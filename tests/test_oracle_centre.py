"""Pins of the centre-first compression (SI, "Modified Compression Scheme")
of the CPU MPS reference: exact reconstruction when nothing is truncated,
Eckart-Young at the x|v cut when only that cut is truncated, and agreement
with a brute-force version of the same scheme written on the dense matrix
(one SVD per cut of the current tensor, each an orthogonal projection),
which shares no code with the MPS sweeps.  A dropped S^-1 is caught."""
import numpy as np
import pytest

import workloads as wl
from oracle import dense
from oracle import mps


def _random_state(Lx, Lv, decay=0.6, seed=0):
    """Dense F (Nx x Nv) with a decaying x|v spectrum and random structure
    inside each dimension, and its untruncated MPS (x bits, then v bits)."""
    rng = np.random.default_rng(seed)
    Nx, Nv = 1 << Lx, 1 << Lv
    k = min(Nx, Nv)
    u, _ = np.linalg.qr(rng.standard_normal((Nx, k)))
    w, _ = np.linalg.qr(rng.standard_normal((Nv, k)))
    s = decay ** np.arange(k) * (1.0 + 0.1 * rng.random(k))
    F = (u * s) @ w.T
    vec = mps.dense_to_sites(F, Lx, Lv, wl.ORDER_SEQ)
    return F, mps.tt_svd(vec, [2] * (Lx + Lv), tol=0.0)


def _keep(s, chi, tol):
    """Number of values kept at one cut (eq. 5 with the i = D+1 reading):
    the fewest whose discarded relative tail is <= tol^2, at most chi."""
    t = s * s / np.sum(s * s)
    D = len(s)
    if tol > 0:
        for d in range(len(s), 0, -1):
            if np.sum(t[d:]) <= tol * tol:
                D = d
    return max(1, min(D, chi if chi else len(s)))


def _project(M, chi, tol):
    u, s, vt = np.linalg.svd(M, full_matrices=False)
    d = _keep(s, chi, tol)
    return (u[:, :d] * s[:d]) @ vt[:d]


def _brute_centre(F, Lx, Lv, chi, tol):
    """The scheme on the dense matrix: truncate the x|v cut (F = U S V^T),
    then every cut inside x of G = U S from the finest x bit down, then
    every cut inside v of H = S V^T from the coarsest v bit up; f' =
    G' S^-1 H'."""
    Nx, Nv = F.shape
    u, s, vt = np.linalg.svd(F, full_matrices=False)
    D = _keep(s, chi, tol)
    G = u[:, :D] * s[:D]
    H = s[:D, None] * vt[:D]
    for j in range(Lx - 1, 0, -1):          # cut after x bit j-1
        G = _project(G.reshape(1 << j, -1), chi, tol).reshape(Nx, D)
    for j in range(1, Lv):                  # cut after v bit j-1
        H = _project(H.reshape(D << j, -1), chi, tol).reshape(D, Nv)
    return G @ np.diag(1.0 / s[:D]) @ H


def _dense(m, Lx, Lv):
    return mps.sites_to_dense(mps.to_vector(m), Lx, Lv, wl.ORDER_SEQ)


@pytest.mark.parametrize("Lx,Lv", [(3, 3), (4, 3), (2, 5)])
def test_untruncated_reconstructs_the_tensor(Lx, Lv):
    F, m = _random_state(Lx, Lv, decay=0.8, seed=Lx + 7 * Lv)
    out, disc = mps.compress_centre(m, Lx, None, 0.0, return_discarded=True)
    assert np.abs(_dense(out, Lx, Lv) - F).max() < 1e-13 * np.abs(F).max()
    assert max(disc) < 1e-14


def test_only_the_centre_cut_truncated_is_eckart_young():
    # Lx = Lv = 3 and chi = 4: every cut inside x or v has rank <= 4, so the
    # x|v cut (rank 8) is the only one truncated -> the best rank-4 matrix.
    F, m = _random_state(3, 3, decay=0.7, seed=3)
    out, disc = mps.compress_centre(m, 3, 4, 0.0, return_discarded=True)
    u, s, vt = np.linalg.svd(F)
    best = (u[:, :4] * s[:4]) @ vt[:4]
    assert np.abs(_dense(out, 3, 3) - best).max() < 1e-12 * np.abs(F).max()
    want = np.sqrt(np.sum(s[4:] ** 2) / np.sum(s ** 2))
    assert abs(disc[2] - want) < 1e-12
    assert max(mps.bond_dims(out)) <= 4


@pytest.mark.parametrize("Lx,Lv,chi,tol", [(4, 4, 3, 0.0), (4, 3, 5, 0.0),
                                           (4, 4, None, 0.05),
                                           (5, 3, 4, 0.02)])
def test_matches_the_dense_brute_force(Lx, Lv, chi, tol):
    F, m = _random_state(Lx, Lv, decay=0.55, seed=11 * Lx + Lv)
    out = mps.compress_centre(m, Lx, chi, tol)
    want = _brute_centre(F, Lx, Lv, chi, tol)
    assert np.abs(_dense(out, Lx, Lv) - want).max() < 1e-11 * np.abs(F).max()
    if chi:
        assert max(mps.bond_dims(out)) <= chi


def test_differs_from_the_plain_sweep_and_keeps_the_centre_values():
    # the scheme is a different truncation: with the same caps it keeps the
    # best rank-D x|v cut, the sweep truncates the cut after the v bonds
    F, m = _random_state(4, 4, decay=0.55, seed=5)
    a = _dense(mps.compress_centre(m, 4, 3, 0.0), 4, 4)
    b = _dense(mps.compress(m, 3, 0.0), 4, 4)
    assert np.abs(a - b).max() > 1e-6 * np.abs(F).max()


def test_dropped_inverse_is_caught(monkeypatch):
    F, m = _random_state(3, 3, decay=0.8, seed=2)
    monkeypatch.setattr(mps, "centre_pinv", lambda S: np.ones_like(S))
    out = mps.compress_centre(m, 3, None, 0.0)
    assert np.abs(_dense(out, 3, 3) - F).max() > 1e-3 * np.abs(F).max()


def test_rank_deficient_cut_gets_zero_inverse():
    # a product state with tol = 0: the centre keeps zero values, whose
    # inverse must be 0 and not inf
    rng = np.random.default_rng(4)
    F = np.outer(rng.random(8), rng.random(16))
    vec = mps.dense_to_sites(F, 3, 4, wl.ORDER_SEQ)
    m = mps.tt_svd(vec, [2] * 7, tol=0.0)
    m = mps.add([(0.5, m), (0.5, m)])        # bonds doubled, rank still 1
    out = mps.compress_centre(m, 3, None, 0.0)
    G = _dense(out, 3, 4)
    assert np.all(np.isfinite(G))
    assert np.abs(G - F).max() < 1e-13 * np.abs(F).max()


def test_untruncated_step_with_centre_first_equals_dense():
    w = wl.landau_small(L=4, tol=0.0)
    p = w.problem
    p.chi_max = None
    p.compression = 1
    ops = mps.Operators(p)
    F = dense.initial(w.ax, w.bv)
    f = mps.init_mps(p, w.ax, w.bv)
    for k in range(2):
        f = mps.rk4_step(f, ops)
        F = dense.rk4_step(F, p)
        err = np.abs(mps.to_dense(f, p) - F).max() / np.abs(F).max()
        assert err < 1e-12 * (k + 1), (k, err)


def test_truncated_step_with_centre_first_tracks_dense_and_caps_bonds():
    w = wl.landau_small(L=5, chi=8, tol=1e-10, level=5)
    p = w.problem
    p.compression = 1
    ops = mps.Operators(p)
    F = dense.initial(w.ax, w.bv)
    f = mps.init_mps(p, w.ax, w.bv)
    for _ in range(3):
        f = mps.rk4_step(f, ops)
        F = dense.rk4_step(F, p)
    assert max(mps.bond_dims(f)) <= 8
    assert np.abs(mps.to_dense(f, p) - F).max() < 1e-3 * np.abs(F).max()
