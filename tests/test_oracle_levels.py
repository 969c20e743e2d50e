"""Pins of the compression-level schedule of the MPS oracle (SI, "Compressed
time evolution algorithm", levels C1-C5).

The SI lists, level by level, which intermediates of an RK4 step are cut to
the bond dimension D:
  C1  only the new state f_{n+1};
  C2  additionally the intermediate states f_n + c dt k;
  C3  additionally the sum k1 + 2 k2 + 2 k3 + k4;
  C4  additionally each derivative k;
  C5  additionally each term added up inside a derivative.
Every other intermediate is compressed by tolerance only; with tol = 0 it is
not truncated at all.

The pins below restate that list as a table and evaluate the whole scheme
on the dense grid, with no MPS at all: the derivatives are the dense
finite-difference operators (oracle O1) and "cut to D" is the truncation of
the full vector, from the last cut to the first, each cut replaced by its
best rank-D approximation of the current vector (the result of the QR +
truncated-SVD sweep, whose left part is orthonormal when a cut is
treated).  The MPS oracle must agree with it at every level, each level
must differ from the one before it (so every extra point really is cut),
and a schedule shifted by one point must fail.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import dense
from oracle import mps

# The SI's list, written out: the intermediates each level cuts to D.
CUT_AT_LEVEL = {
    1: {"new_state"},
    2: {"new_state", "stage_state"},
    3: {"new_state", "stage_state", "sum_of_k"},
    4: {"new_state", "stage_state", "sum_of_k", "k"},
    5: {"new_state", "stage_state", "sum_of_k", "k", "term"},
}


def _chain_vector(F, Lx, Lv, order):
    """The grid function as a vector in chain order: S1 = all x bits then
    all v bits (index i * Nv + j), IF = x1 v1 x2 v2 ... (MSB first)."""
    if order == wl.ORDER_SEQ:
        return F.reshape(-1).copy()
    assert order == wl.ORDER_INTERLEAVED and Lx == Lv
    T = F.reshape((2,) * (Lx + Lv))
    axes = [a for k in range(Lx) for a in (k, Lx + k)]
    return T.transpose(axes).reshape(-1).copy()


def _grid(vec, Lx, Lv, order):
    if order == wl.ORDER_SEQ:
        return vec.reshape(1 << Lx, 1 << Lv)
    L = Lx
    T = vec.reshape((2,) * (2 * L))
    # chain axis 2k is x bit k, 2k+1 is v bit k
    inv = [2 * k for k in range(L)] + [2 * k + 1 for k in range(L)]
    return T.transpose(inv).reshape(1 << Lx, 1 << Lv)


def _cut_dense(F, p, D):
    """Best rank-D approximation at every cut of the chain, from the last
    cut to the first, each of the current (already cut) vector."""
    n = p.Lx + p.Lv
    v = _chain_vector(F, p.Lx, p.Lv, p.order)
    for j in range(n - 1, 0, -1):
        M = v.reshape(1 << j, -1)
        U, S, Vt = np.linalg.svd(M, full_matrices=False)
        k = min(D, len(S))
        v = ((U[:, :k] * S[:k]) @ Vt[:k]).reshape(-1)
    return _grid(v, p.Lx, p.Lv, p.order)


def _dense_scheme_step(F, p, level):
    """One RK4 step of the dense scheme with the level's cuts (tol = 0,
    uncapped field)."""
    cut = CUT_AT_LEVEL[level]

    def C(X, what):
        return _cut_dense(X, p, p.chi_max) if what in cut else X

    def R(G):
        E = dense.field(G, p)
        t1 = C(-dense.advection(G, p), "term")
        t2 = C(-p.qm * E[:, None] * dense.ddv(G, p.dv), "term")
        return C(t1 + t2, "k")

    h = p.dt
    k1 = R(F)
    k2 = R(C(F + 0.5 * h * k1, "stage_state"))
    k3 = R(C(F + 0.5 * h * k2, "stage_state"))
    k4 = R(C(F + h * k3, "stage_state"))
    S = C(k1 + 2.0 * k2 + 2.0 * k3 + k4, "sum_of_k")
    return C(F + (h / 6.0) * S, "new_state")


def _problem(order, chi, level, L=3):
    w = wl.two_stream(L=L, chi=chi, tol=0.0, level=level, df_max=0, order=order,
                      dt_cfg=0.05)
    p = w.problem
    rng = np.random.default_rng(11 + order)
    # generic spectra at every cut: the profile plus a seeded full-rank part
    F = dense.initial(w.ax, w.bv)
    F = F + 0.05 * np.abs(F).max() * rng.standard_normal(F.shape)
    return p, F


def _mps_step(F, p):
    f = mps.tt_svd(_chain_vector(F, p.Lx, p.Lv, p.order), [2] * (p.Lx + p.Lv))
    g = mps.rk4_step(f, mps.Operators(p))
    return _grid(mps.to_vector(g), p.Lx, p.Lv, p.order), g


@pytest.mark.parametrize("order", [wl.ORDER_SEQ, wl.ORDER_INTERLEAVED])
@pytest.mark.parametrize("level", [1, 2, 3, 4, 5])
def test_level_schedule_equals_dense_scheme(order, level):
    p, F = _problem(order, chi=3, level=level)
    ref = _dense_scheme_step(F, p, level)
    got, g = _mps_step(F, p)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-9 * scale
    assert max(mps.bond_dims(g)) <= 3


@pytest.mark.parametrize("order", [wl.ORDER_SEQ, wl.ORDER_INTERLEAVED])
def test_each_level_cuts_more_than_the_one_before(order):
    """Each extra point of the list changes the result: a level that cut
    nothing new would equal the previous one."""
    outs = []
    for level in range(1, 6):
        p, F = _problem(order, chi=3, level=level)
        outs.append(_dense_scheme_step(F, p, level))
    for a, b in zip(outs, outs[1:]):
        assert np.abs(a - b).max() > 1e-6 * np.abs(a).max()


@pytest.mark.parametrize("level", [1, 2, 3, 4, 5])
def test_untruncated_step_equals_dense_at_every_level(level):
    """Caps at or above the full rank: every level is the plain dense step."""
    for order in (wl.ORDER_SEQ, wl.ORDER_INTERLEAVED):
        p, F = _problem(order, chi=64, level=level)
        got, _ = _mps_step(F, p)
        ref = dense.rk4_step(F, p)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("shift", [-1, +1])
def test_shifted_schedule_is_caught(monkeypatch, shift):
    """A schedule that caps one point more or one point fewer than the
    level says (an off-by-one in the point numbering) breaks the pin."""
    monkeypatch.setattr(
        mps, "caps",
        lambda p, point: p.chi_max if p.level + shift >= point else None)
    caught = 0
    for level in range(1, 6):
        p, F = _problem(wl.ORDER_SEQ, chi=3, level=level)
        ref = _dense_scheme_step(F, p, level)
        got, _ = _mps_step(F, p)
        if np.abs(got - ref).max() > 1e-6 * np.abs(ref).max():
            caught += 1
    assert caught >= 3


def test_term_left_uncut_at_level_five_is_caught(monkeypatch):
    """A C5 step that forgets to cut one of the terms of a derivative."""
    real = mps.compress_state
    calls = {"n": 0}

    def forgetful(m, chi, p):
        calls["n"] += 1
        # the second compression of each derivative is its T2 term
        if calls["n"] % 4 == 2:
            return real(m, None, p)
        return real(m, chi, p)

    monkeypatch.setattr(mps, "compress_state", forgetful)
    p, F = _problem(wl.ORDER_SEQ, chi=3, level=5)
    ref = _dense_scheme_step(F, p, 5)
    got, _ = _mps_step(F, p)
    assert np.abs(got - ref).max() > 1e-6 * np.abs(ref).max()
