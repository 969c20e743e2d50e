"""Pins of the entanglement-entropy diagnostic (Results, "State
Compressibility": S = -sum_i s~_i^2 log2 s~_i^2 over the normalised
singular values of a bond) against states with known Schmidt values."""
import math

import numpy as np

import workloads as wl
from oracle import mps


def _schmidt_state(Lx, Lv, s, seed=1):
    """f(x, v) = sum_r s_r u_r(x) w_r(v) with orthonormal u, w, as an
    untruncated MPS in the sequential order (x bits, then v bits)."""
    rng = np.random.default_rng(seed)
    u, _ = np.linalg.qr(rng.standard_normal((1 << Lx, len(s))))
    w, _ = np.linalg.qr(rng.standard_normal((1 << Lv, len(s))))
    F = (u * np.asarray(s)) @ w.T
    vec = mps.dense_to_sites(F, Lx, Lv, wl.ORDER_SEQ)
    return mps.tt_svd(vec, [2] * (Lx + Lv), tol=0.0)


def test_entropy_of_a_known_schmidt_spectrum():
    s = np.array([3.0, 1.0, 0.5])
    t = s ** 2 / np.sum(s ** 2)
    want = float(-np.sum(t * np.log2(t)))
    ee = mps.entanglement_entropy(_schmidt_state(4, 3, s))
    assert abs(ee[4 - 1] - want) < 1e-12


def test_equal_weights_give_log2_of_the_rank():
    ee = mps.entanglement_entropy(_schmidt_state(3, 4, [1.0, 1.0, 1.0, 1.0]))
    assert abs(ee[3 - 1] - 2.0) < 1e-12


def test_product_cut_has_zero_entropy():
    ee = mps.entanglement_entropy(_schmidt_state(4, 4, [2.0]))
    assert abs(ee[4 - 1]) < 1e-12
    assert all(e >= -1e-12 for e in ee)
