"""Pins of the sequential orderings S2 and S3 (Results, "State
Compressibility", Fig. 3: x fine->coarse then v coarse->fine, and x
coarse->fine then v fine->coarse) in the CPU MPS reference, against index
maps written out bit by bit: the site map, operators and product states
embedded in the chain, the density, an untruncated step with a grid of
unequal sides, and the x|v cut's entanglement, which no ordering of the
bits inside a dimension can change."""
import numpy as np
import pytest

import workloads as wl
from oracle import dense
from oracle import mps


def _chain_index(i, j, Lx, Lv, order):
    """Position in the chain vector of grid point (i, j), built bit by bit
    (site 0 is the most significant digit of the position)."""
    xb = [(i >> (Lx - 1 - k)) & 1 for k in range(Lx)]   # coarse -> fine
    vb = [(j >> (Lv - 1 - k)) & 1 for k in range(Lv)]
    if order == 2:
        xb = xb[::-1]
    if order == 3:
        vb = vb[::-1]
    idx = 0
    for b in xb + vb:
        idx = 2 * idx + b
    return idx


def _perm(Lx, Lv, order):
    P = np.zeros((1 << (Lx + Lv), 1 << (Lx + Lv)))
    for i in range(1 << Lx):
        for j in range(1 << Lv):
            P[_chain_index(i, j, Lx, Lv, order), i * (1 << Lv) + j] = 1.0
    return P


@pytest.mark.parametrize("order", [2, 3])
@pytest.mark.parametrize("Lx,Lv", [(3, 2), (2, 4)])
def test_site_map_matches_the_bit_by_bit_index(order, Lx, Lv):
    rng = np.random.default_rng(Lx * 10 + Lv + order)
    F = rng.standard_normal((1 << Lx, 1 << Lv))
    vec = mps.dense_to_sites(F, Lx, Lv, order)
    for i in range(1 << Lx):
        for j in range(1 << Lv):
            assert vec[_chain_index(i, j, Lx, Lv, order)] == F[i, j]
    assert np.array_equal(mps.sites_to_dense(vec, Lx, Lv, order), F)


@pytest.mark.parametrize("order", [0, 2, 3])
def test_chain_mpo_is_the_permuted_kronecker_product(order):
    Lx, Lv = 3, 2
    Wx = mps.mpo_sum([mps.mpo_d1_periodic(Lx, 0.7),
                      mps.diag_mpo(mps.vector_mps(np.arange(8.0) ** 2 - 3.0))])
    Wv = mps.mpo_d1_zero_gradient(Lv, 0.3)
    M = mps.mpo_to_matrix(mps.chain_mpo(Wx, Wv, Lx, Lv, order))
    K = np.kron(mps.mpo_to_matrix(Wx), mps.mpo_to_matrix(Wv))
    P = _perm(Lx, Lv, order)
    assert np.abs(M - P @ K @ P.T).max() < 1e-12


@pytest.mark.parametrize("order", [2, 3])
def test_product_state_and_density_in_natural_order(order):
    Lx, Lv = 3, 4
    rng = np.random.default_rng(order)
    u, w = rng.standard_normal(8), rng.standard_normal(16)
    g = mps.chain_product_mps(mps.vector_mps(u), mps.vector_mps(w), Lx, Lv, order)
    assert np.abs(mps.to_vector(g) - _perm(Lx, Lv, order) @ np.kron(u, w)).max() < 1e-12
    F = rng.standard_normal((8, 16))
    f = mps.tt_svd(mps.dense_to_sites(F, Lx, Lv, order), [2] * 7)
    n = mps.to_vector(mps.density_mps(f, Lx, Lv, order, 0.25))
    assert np.abs(n - 0.25 * F.sum(axis=1)).max() < 1e-12


@pytest.mark.parametrize("order", [2, 3])
def test_untruncated_step_on_an_unequal_grid_equals_dense(order):
    w = wl.landau_small(L=4, Lv=3, tol=0.0)
    p = w.problem
    p.order = order
    p.chi_max = None
    ops = mps.Operators(p)
    F = dense.initial(w.ax, w.bv)
    f = mps.init_mps(p, w.ax, w.bv)
    for k in range(2):
        f = mps.rk4_step(f, ops)
        F = dense.rk4_step(F, p)
        err = np.abs(mps.to_dense(f, p) - F).max() / np.abs(F).max()
        assert err < 1e-12 * (k + 1), (k, err)


@pytest.mark.parametrize("order", [2, 3])
def test_centre_first_untruncated_step_equals_dense(order):
    w = wl.landau_small(L=4, tol=0.0)
    p = w.problem
    p.order = order
    p.chi_max = None
    p.compression = 1
    ops = mps.Operators(p)
    F = dense.initial(w.ax, w.bv)
    f = mps.init_mps(p, w.ax, w.bv)
    f = mps.rk4_step(f, ops)
    F = dense.rk4_step(F, p)
    assert np.abs(mps.to_dense(f, p) - F).max() < 1e-12 * np.abs(F).max()


def test_xv_cut_entropy_is_the_same_in_s1_s2_s3():
    rng = np.random.default_rng(9)
    Lx, Lv = 4, 3
    F = rng.standard_normal((16, 3)) @ rng.standard_normal((3, 8))
    F += 1e-2 * rng.standard_normal((16, 8))
    ees = []
    for order in (0, 2, 3):
        f = mps.tt_svd(mps.dense_to_sites(F, Lx, Lv, order), [2] * 7)
        ees.append(mps.entanglement_entropy(f)[Lx - 1])
    s = np.linalg.svd(F, compute_uv=False)
    t = s ** 2 / np.sum(s ** 2)
    want = float(-np.sum(t * np.log2(t)))
    assert np.allclose(ees, want, atol=1e-12)
    # the cuts inside x differ: S2 reads x from its finest bit
    f1 = mps.tt_svd(mps.dense_to_sites(F, Lx, Lv, 0), [2] * 7)
    f2 = mps.tt_svd(mps.dense_to_sites(F, Lx, Lv, 2), [2] * 7)
    assert abs(mps.entanglement_entropy(f1)[0] - mps.entanglement_entropy(f2)[0]) > 1e-6


def test_missing_bond_swap_is_caught(monkeypatch):
    # a reversed dimension whose cores keep their bond order is wrong
    monkeypatch.setattr(mps, "reverse_chain", lambda cores: list(cores[::-1]))
    Lx, Lv = 3, 2
    Wx = mps.mpo_d1_periodic(Lx, 0.7)
    Wv = mps.mpo_d1_zero_gradient(Lv, 0.3)
    try:
        M = mps.mpo_to_matrix(mps.chain_mpo(Wx, Wv, Lx, Lv, 2))
    except ValueError:
        return
    K = np.kron(mps.mpo_to_matrix(Wx), mps.mpo_to_matrix(Wv))
    P = _perm(Lx, Lv, 2)
    assert np.abs(M - P @ K @ P.T).max() > 1e-3
