"""The start states the parity tests hand to both sides (tests/_start.py):
the oracle's product-state initialisation equals its dense iterated-SVD
initialisation, and splitting a fused IG site into binary sites represents
the same tensor."""
import numpy as np

import workloads as wl
from oracle import dense as odense
from oracle import mps as omps
from tests import _start as S


def test_product_start_equals_dense_initialisation():
    for order in (0, 1, 2, 3):
        w = wl.landau_small(L=4, chi=16, tol=1e-10)
        w.problem.order = order
        p = w.problem
        a = omps.to_dense(S.oracle_start(w), p)
        b = omps.to_dense(omps.init_mps(p, w.ax, w.bv), p)
        ref = odense.initial(w.ax, w.bv)
        assert np.abs(a - ref).max() <= 1e-13 * np.abs(ref).max()
        assert np.abs(a - b).max() <= 1e-13 * np.abs(ref).max()


def test_perturbed_start_caps_bonds_and_adds_the_perturbation():
    w = wl.two_stream(L=4, chi=6, tol=0.0, level=5, df_max=4, dt_cfg=0.05)
    p = w.problem
    f = S.oracle_start(w, pert_chi=6, amp=1e-3)
    assert max(omps.bond_dims(f)) <= 6
    g = S.oracle_start(w)
    assert np.abs(omps.to_vector(f) - omps.to_vector(g)).max() > 1e-6


def test_binary_split_of_ig_sites_is_exact():
    w = wl.two_stream(L=4, chi=8, tol=0.0, level=5, df_max=4, dt_cfg=0.05, order=4)
    p = w.problem
    f = S.oracle_start(w, pert_chi=8, amp=1e-3)
    b = S.binary_cores(f, p)
    assert len(b) == p.n_sites and all(c.shape[1] == 2 for c in b)
    v1 = omps.to_vector(omps.fuse_pairs(b))
    v2 = omps.to_vector(f)
    assert np.abs(v1 - v2).max() <= 1e-13 * np.abs(v2).max()
