"""Pins of the grouped interleaved ordering IG (Results, "State
Compressibility", Fig. 3: x_k and v_k of equal resolution in one site of
dimension 4) in the CPU MPS reference: the fused chain represents the same
vector and operators as IF, an untruncated step equals the dense step, and
truncation cuts only between pairs -- checked against a dense brute force
that projects the vector at every pair cut in turn."""
import numpy as np
import pytest

import workloads as wl
from oracle import dense
from oracle import mps


def test_ig_sites_have_dimension_four_and_represent_the_same_vector():
    rng = np.random.default_rng(1)
    F = rng.standard_normal((8, 8))
    vec = mps.dense_to_sites(F, 3, 3, 4)
    assert np.array_equal(vec, mps.dense_to_sites(F, 3, 3, 1))
    m = mps.tt_svd(vec, mps.site_dims(3, 3, 4))
    assert [A.shape[1] for A in m] == [4, 4, 4]
    assert np.abs(mps.sites_to_dense(mps.to_vector(m), 3, 3, 4) - F).max() < 1e-13


def test_ig_operator_chain_is_the_if_chain_contracted():
    Wx = mps.mpo_d1_periodic(3, 0.5)
    Wv = mps.mpo_d1_zero_gradient(3, 0.25)
    M4 = mps.mpo_to_matrix_d(mps.chain_mpo(Wx, Wv, 3, 3, 4), 4)
    M2 = mps.mpo_to_matrix(mps.chain_mpo(Wx, Wv, 3, 3, 1))
    assert np.abs(M4 - M2).max() < 1e-13


def test_untruncated_ig_step_equals_dense():
    w = wl.landau_small(L=4, tol=0.0)
    p = w.problem
    p.order, p.chi_max = 4, None
    ops = mps.Operators(p)
    F = dense.initial(w.ax, w.bv)
    f = mps.init_mps(p, w.ax, w.bv)
    assert all(A.shape[1] == 4 for A in f)
    for k in range(2):
        f = mps.rk4_step(f, ops)
        F = dense.rk4_step(F, p)
        assert np.abs(mps.to_dense(f, p) - F).max() < 1e-12 * (k + 1) * np.abs(F).max()
    assert np.abs(mps.field_dense(f, ops) - dense.field(F, p)).max() < 1e-11


def _keep(s, chi):
    return max(1, min(chi, len(s)))


@pytest.mark.parametrize("L,chi", [(3, 3), (4, 5)])
def test_ig_truncation_is_the_pair_cut_brute_force(L, chi):
    rng = np.random.default_rng(L + chi)
    n = 2 * L
    m = mps.tt_svd(rng.standard_normal(1 << n) * np.exp(-0.3 * np.arange(1 << n) / 8.0),
                   [4] * L)
    out = mps.compress(m, chi, 0.0)
    # brute force: right to left over the pair cuts (4^j | 4^(L-j)), each
    # an orthogonal projection of the current vector on its top chi values
    cur = mps.to_vector(m)
    for j in range(L - 1, 0, -1):
        M = cur.reshape(4 ** j, -1)
        u, s, vt = np.linalg.svd(M, full_matrices=False)
        d = _keep(s, chi)
        cur = ((u[:, :d] * s[:d]) @ vt[:d]).reshape(-1)
    assert np.abs(mps.to_vector(out) - cur).max() < 1e-12 * np.abs(cur).max()
    assert max(mps.bond_dims(out)) <= chi
