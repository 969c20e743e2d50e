"""Pins of the CPU MPS reference (O2): brute-force MPO decoding, exact
agreement with the dense oracle when nothing is truncated, Eckart-Young at a
single cut, canonical-form isometries, the paper's stated ranks, and
planted mistakes that these pins must catch."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import dense
from oracle import mps


def _stencil_periodic(N):
    D = np.zeros((N, N))
    for o in range(N):
        D[o, (o + 1) % N] += 0.5
        D[o, (o - 1) % N] -= 0.5
    return D


def _stencil_zero_gradient(N):
    D = np.zeros((N, N))
    for o in range(1, N - 1):
        D[o, o + 1] += 0.5
        D[o, o - 1] -= 0.5
    return D


def _stencil_second(N):
    D = np.zeros((N, N))
    for o in range(N):
        D[o, o] -= 2
        D[o, (o + 1) % N] += 1
        D[o, (o - 1) % N] += 1
    return D


@pytest.mark.parametrize("L", [2, 3, 4, 6, 7])
def test_printed_mpos_decode_to_stencils(L):
    N = 2 ** L
    h = 0.7
    assert np.abs(mps.mpo_to_matrix(mps.mpo_d1_periodic(L, h)) - _stencil_periodic(N) / h).max() < 1e-14
    assert np.abs(mps.mpo_to_matrix(mps.mpo_d1_zero_gradient(L, h)) - _stencil_zero_gradient(N) / h).max() < 1e-14
    assert np.abs(mps.mpo_to_matrix(mps.mpo_d2_periodic(L, h)) - _stencil_second(N) / h ** 2).max() < 1e-13


def test_mpo_bond_dimensions_as_printed():
    assert [w.shape[3] for w in mps.mpo_d1_periodic(6, 1.0)[:-1]] == [3] * 5
    assert [w.shape[3] for w in mps.mpo_d2_periodic(6, 1.0)[:-1]] == [3] * 5
    assert [w.shape[3] for w in mps.mpo_d1_zero_gradient(6, 1.0)[:-1]] == [5] * 5


def test_inverse_laplacian_mpo_rank_about_five():
    # SI "Inverse Laplacian": bond about 5 when keeping singular values to 1e-10
    for L in (6, 8):
        Lap = mps.mpo_to_matrix(mps.mpo_d2_periodic(L, 0.3))
        W = mps.mpo_from_matrix(np.linalg.pinv(Lap), L, tol=1e-10)
        assert max(w.shape[3] for w in W[:-1]) <= 5
        G = mps.poisson_mpo(L, 0.3)
        assert max(w.shape[3] for w in G[:-1]) <= 5


def test_poisson_mpo_equals_dense_field():
    for L in (4, 6):
        w = wl.landau_small(L=L)
        p = w.problem
        G = mps.poisson_mpo(L, p.dx)
        rng = np.random.default_rng(L)
        n = 1 + 0.1 * rng.random(p.Nx)
        E_mpo = -mps.mpo_to_matrix(G) @ n
        assert np.abs(E_mpo - dense.poisson_field_dense(n, p.dx)).max() < 1e-12


def test_tt_svd_round_trip_and_full_rank_bonds():
    rng = np.random.default_rng(0)
    for n in (5, 8, 10):
        vec = rng.standard_normal(2 ** n)
        m = mps.tt_svd(vec, [2] * n)
        assert mps.bond_dims(m) == [2 ** min(j, n - j) for j in range(1, n)]
        assert np.abs(mps.to_vector(m) - vec).max() < 1e-12


def test_eckart_young_single_cut_and_discarded_weight():
    rng = np.random.default_rng(1)
    n = 8
    vec = rng.standard_normal(2 ** n) * 10.0 ** (-np.arange(2 ** n) / 64.0)
    m = mps.tt_svd(vec, [2] * n)
    # chi = 8 truncates only the middle bond (16 -> 8)
    c, disc = mps.compress(m, 8, 0.0, return_discarded=True)
    s = np.linalg.svd(vec.reshape(16, 16), compute_uv=False)
    err = np.linalg.norm(mps.to_vector(c) - vec)
    best = math.sqrt(np.sum(s[8:] ** 2))
    assert abs(err - best) <= 1e-12 * np.linalg.norm(vec)
    assert abs(disc[3] - best / np.linalg.norm(vec)) < 1e-12
    assert all(d < 1e-14 for j, d in enumerate(disc) if j != 3)


def test_sweep_error_within_tt_bound():
    rng = np.random.default_rng(2)
    n = 10
    vec = rng.standard_normal(2 ** n)
    m = mps.tt_svd(vec, [2] * n)
    c, disc = mps.compress(m, 6, 0.0, return_discarded=True)
    err = np.linalg.norm(mps.to_vector(c) - vec) / np.linalg.norm(vec)
    assert err <= math.sqrt(sum(d * d for d in disc)) * (1 + 1e-10)
    assert max(mps.bond_dims(c)) == 6


def test_canonical_isometries():
    rng = np.random.default_rng(4)
    m = [rng.standard_normal(c.shape) for c in wl.random_mps_cores(9, 8, seed=5)]
    L = mps.left_canonicalize(m)
    for A in L[:-1]:
        a, d, b = A.shape
        Q = A.reshape(a * d, b)
        assert np.abs(Q.T @ Q - np.eye(b)).max() < 1e-13
    C = mps.compress(m, 5, 0.0)
    for A in C[1:]:
        a, d, b = A.shape
        R = A.reshape(a, d * b)
        assert np.abs(R @ R.T - np.eye(a)).max() < 1e-13


def test_rank_rule_cases():
    s = np.array([1.0, 1e-3, 1e-6, 1e-12])
    assert mps.rank_rule(s, None, 0.0) == 4
    assert mps.rank_rule(s, 2, 0.0) == 2
    assert mps.rank_rule(s, None, 1e-10) == 3     # 1e-12 discarded
    assert mps.rank_rule(s, None, 1e-5) == 2
    assert mps.rank_rule(s, None, 2e-3) == 1
    assert mps.rank_rule(np.zeros(3), None, 1e-10) == 1
    # tol = 0 discards nothing by weight: the cap alone, even for zeros
    assert mps.rank_rule(np.zeros(3), None, 0.0) == 3
    assert mps.rank_rule(np.zeros(3), 2, 0.0) == 2


@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_density_and_moments_equal_dense_riemann_sums(order):
    w = wl.landau_small(L=4, chi=64, tol=0.0)
    p = w.problem
    p.order = order
    F = dense.initial(w.ax, w.bv) + 0.01 * np.random.default_rng(7).random((p.Nx, p.Nv))
    f = mps.tt_svd(mps.dense_to_sites(F, p.Lx, p.Lv, order), [2] * p.n_sites)
    n = mps.to_vector(mps.density_mps(f, p.Lx, p.Lv, order, p.dv))
    assert np.abs(n - dense.density(F, p.dv)).max() < 1e-13
    ops = mps.Operators(p)
    m = mps.moments(f, ops)
    d = dense.diagnostics(F, p)
    for k in m:
        assert abs(m[k] - d[k]) <= 1e-12 * max(1.0, abs(d[k])), k


@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_untruncated_step_equals_dense(order):
    w = wl.landau_small(L=4, tol=0.0)
    p = w.problem
    p.order = order
    p.chi_max = None
    ops = mps.Operators(p)
    F = dense.initial(w.ax, w.bv)
    f = mps.init_mps(p, w.ax, w.bv)
    assert np.abs(mps.to_dense(f, p) - F).max() < 1e-14
    for k in range(3):
        f = mps.rk4_step(f, ops)
        F = dense.rk4_step(F, p)
        err = np.abs(mps.to_dense(f, p) - F).max() / np.abs(F).max()
        assert err < 1e-12 * (k + 1), (k, err)
    E = mps.field_dense(f, ops)
    Ed = dense.field(F, p)
    assert np.abs(E - Ed).max() <= 1e-11 * np.abs(Ed).max()


def test_two_stream_interleaved_untruncated_and_orderings_agree():
    w = wl.two_stream(L=3, chi=0, tol=0.0, dt_cfg=0.1)
    p = w.problem
    p.chi_max = None
    F = dense.initial(w.ax, w.bv)
    outs = []
    for order in (0, 1):
        p.order = order
        ops = mps.Operators(p)
        f = mps.init_mps(p, w.ax, w.bv)
        for _ in range(2):
            f = mps.rk4_step(f, ops)
        outs.append(mps.to_dense(f, p))
    for _ in range(2):
        F = dense.rk4_step(F, p)
    assert np.abs(outs[0] - F).max() < 1e-12 * np.abs(F).max()
    assert np.abs(outs[1] - F).max() < 1e-12 * np.abs(F).max()


def test_tol_1e10_landau_tracks_dense():
    w = wl.landau_small(L=5, chi=16, tol=1e-10)
    p = w.problem
    ops = mps.Operators(p)
    F = dense.initial(w.ax, w.bv)
    f = mps.init_mps(p, w.ax, w.bv)
    for _ in range(20):
        f = mps.rk4_step(f, ops)
        F = dense.rk4_step(F, p)
    assert np.abs(mps.to_dense(f, p) - F).max() < 1e-8 * np.abs(F).max()
    Wm = mps.moments(f, ops)["field_energy"]
    Wd = dense.diagnostics(F, p)["field_energy"]
    assert abs(Wm - Wd) < 1e-6 * Wd


def test_truncated_caps_bond_dimension_and_respects_tolerance():
    w = wl.landau_small(L=5, chi=4, tol=1e-10, level=5)
    p = w.problem
    ops = mps.Operators(p)
    f = mps.init_mps(p, w.ax, w.bv)
    f = mps.rk4_step(f, ops)
    assert max(mps.bond_dims(f)) <= 4


@pytest.mark.parametrize("mutation", ["garbled_m_left", "transposed_apply",
                                      "keep_smallest", "no_scalar_fold"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    if mutation == "garbled_m_left":
        # the printed M_left (first factor [[0,-c1],[0,0]], then [[0,0],[0,1]])
        L = 4
        c1 = 0.5
        left = [np.array([[0.0, -c1], [0.0, 0.0]]).reshape(1, 2, 2, 1)] + \
            [mps.P1.reshape(1, 2, 2, 1)] * (L - 1)
        back = mps.mpo_d1_zero_gradient(L, 1.0)
        M = mps.mpo_to_matrix(back) - 0.0
        bad = M + mps.mpo_to_matrix(left) - mps.mpo_to_matrix(
            [mps.P0.reshape(1, 2, 2, 1)] * (L - 1) +
            [np.array([[0.0, -c1], [0.0, 0.0]]).reshape(1, 2, 2, 1)])
        assert np.abs(bad - _stencil_zero_gradient(2 ** L)).max() > 0.1
    elif mutation == "transposed_apply":
        def bad_apply(W, A):
            return mps.apply.__wrapped__([w.transpose(0, 2, 1, 3) for w in W], A)
        orig = mps.apply
        bad_apply.__wrapped__ = orig
        monkeypatch.setattr(mps, "apply", bad_apply)
        w = wl.landau_small(L=3, tol=0.0)
        p = w.problem
        p.chi_max = None
        ops = mps.Operators(p)
        F = dense.initial(w.ax, w.bv)
        f = mps.rk4_step(mps.init_mps(p, w.ax, w.bv), ops)
        assert np.abs(mps.to_dense(f, p) - dense.rk4_step(F, p)).max() > 1e-9
    elif mutation == "keep_smallest":
        orig = np.linalg.svd

        def rev_svd(M, full_matrices=True, compute_uv=True):
            if not compute_uv:
                return orig(M, full_matrices=full_matrices, compute_uv=False)
            U, S, Vt = orig(M, full_matrices=full_matrices)
            return U[:, ::-1], S[::-1], Vt[::-1]
        rng = np.random.default_rng(1)
        vec = rng.standard_normal(256) * 10.0 ** (-np.arange(256) / 64.0)
        m = mps.tt_svd(vec, [2] * 8)
        monkeypatch.setattr(np.linalg, "svd", rev_svd)
        c = mps.compress(m, 8, 0.0)
        monkeypatch.setattr(np.linalg, "svd", orig)
        s = orig(vec.reshape(16, 16), compute_uv=False)
        err = np.linalg.norm(mps.to_vector(c) - vec)
        assert abs(err - math.sqrt(np.sum(s[8:] ** 2))) > 1e-6
    else:
        def bad_add(terms):
            return orig_add([(1.0, m) for c, m in terms])
        orig_add = mps.add
        monkeypatch.setattr(mps, "add", bad_add)
        w = wl.landau_small(L=3, tol=0.0)
        p = w.problem
        p.chi_max = None
        ops = mps.Operators(p)
        F = dense.initial(w.ax, w.bv)
        f = mps.rk4_step(mps.init_mps(p, w.ax, w.bv), ops)
        assert np.abs(mps.to_dense(f, p) - dense.rk4_step(F, p)).max() > 1e-9


@pytest.mark.slow
def test_mps_landau_damping_rate_at_chi16():
    """64 x 64 grid, sequential order, chi = 16, tol = 1e-10: the compressed
    MPS run still damps at the kinetic rate (gamma = -0.1534)."""
    from tests import _dispersion as disp
    w0 = disp.root(0.5, [(1.0, 0.0)], 1.4 - 0.15j)
    w = wl.landau_small(L=6, chi=16, tol=1e-10)
    p = w.problem
    ops = mps.Operators(p)
    f = mps.init_mps(p, w.ax, w.bv)
    t, W = [0.0], [mps.moments(f, ops)["field_energy"]]
    for s in range(600):
        f = mps.rk4_step(f, ops)
        t.append((s + 1) * p.dt)
        W.append(mps.moments(f, ops)["field_energy"])
    gamma, tp = disp.fit_rate(t, W, 0.0, 30.0, peaks=True)
    assert len(tp) >= 10
    assert abs(gamma - w0.imag) < 0.01, gamma
    assert max(mps.bond_dims(f)) <= 16


def test_printed_constants_fixture():
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "paper_constants.json")))
    L = 5
    W = mps.mpo_d1_periodic(L, 1.0)
    # last-site column [c1(S- - S+); c1 S+; -c1 S-] carries c1 in (o,i)=(0,1)
    assert W[-1][0, 0, 1, 0] == g["d1_periodic_central_c1"]["value"]
    W2 = mps.mpo_d2_periodic(L, 1.0)
    assert W2[-1][0, 0, 0, 0] == g["d2_periodic_c0"]["value"]
    assert W2[-1][0, 0, 1, 0] == g["d2_periodic_c1"]["value"]
    assert W[1].shape[0] == W[1].shape[3] == g["derivative_mpo_bond"]["value"]
    assert wl.landau_small().problem.tol == g["no_compression_threshold"]["value"]
