"""Pins of the upwind x-advection in the oracles (SI, "Upwind time
evolution" and "First Derivative, Forward / Backward, Periodic Boundary
Conditions") against facts other than the oracle itself: the coefficients
the paper prints, the Fourier symbols and truncation error of the
one-sided stencils, the closed-form RK4 amplification of a single mode,
and the untruncated MPS step against the dense step.  Planted mistakes
(downwind choice, a first-order stencil) must break a pin."""
import json
import math
import os

import numpy as np
import pytest

import workloads as wl
from oracle import dense
from oracle import mps

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _symbol(c, theta, forward):
    """Eigenvalue (times h) of the stencil sum_m c_m f_{i +- m} on mode
    e^{i theta j}."""
    s = 1.0 if forward else -1.0
    return sum(cm * np.exp(1j * s * m * theta) for m, cm in enumerate(c))


@pytest.mark.parametrize("L", [3, 4, 6])
@pytest.mark.parametrize("forward", [True, False])
def test_one_sided_mpos_have_the_printed_stencil(L, forward):
    """The oracle's MPO, decoded to its matrix, acts on every Fourier mode
    with the symbol of the printed coefficients; its bonds stay <= 3."""
    h = 0.37
    c = GOLD["d1_forward_periodic_c" if forward else "d1_backward_periodic_c"]["value"]
    W = mps.mpo_d1_forward(L, h) if forward else mps.mpo_d1_backward(L, h)
    assert max(w.shape[3] for w in W) <= 3
    M = mps.mpo_to_matrix(W)
    N = 1 << L
    j = np.arange(N)
    for q in range(N):
        th = 2 * math.pi * q / N
        e = np.exp(1j * th * j)
        lam = _symbol(c, th, forward) / h
        assert np.abs(M @ e - lam * e).max() < 1e-12 * max(1.0, abs(lam))


@pytest.mark.parametrize("forward", [True, False])
def test_one_sided_stencils_are_second_order(forward):
    """D f = f' - (h^2/3) f''' + O(h^3) for both one-sided stencils (Taylor
    expansion), checked on sin(kx) at two resolutions."""
    Lbox = 2 * math.pi
    k = 3.0
    ratios = []
    for N in (512, 1024):
        h = Lbox / N
        x = h * np.arange(N)
        F = np.sin(k * x)[:, None]
        D = (dense.ddx_forward if forward else dense.ddx_backward)(F, h)[:, 0]
        err = D - k * np.cos(k * x)
        lead = (h * h / 3.0) * k ** 3 * np.cos(k * x)
        ratios.append(np.abs(err - lead).max() / np.abs(lead).max())
    # the remainder is O(h^3): relative to the h^2 term it halves with h
    assert ratios[0] < 0.05 and ratios[1] < ratios[0] / 1.8


def _advection_problem(L=5, Lv=4, dt=0.02):
    # q/m = 0 decouples the field: the step is pure x advection
    p = wl.Problem(Lx=L, Lv=Lv, order=wl.ORDER_SEQ, x_min=0.0, x_max=2 * math.pi,
                   v_min=-3.0, v_max=3.0, qm=0.0, dt=dt, chi_max=64, level=1,
                   tol=0.0, x_scheme=1)
    return p


def test_upwind_single_mode_matches_rk4_amplification():
    """With the field decoupled (q/m = 0), f0 = cos(k x) g(v) advects each
    velocity slice as one Fourier mode: after one RK4 step its complex
    amplitude is R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 with
    z = -v dt sym(theta)/h, sym the backward symbol where v > 0 and the
    forward one where v < 0, and |R| < 1 (the upwind choice damps)."""
    p = _advection_problem()
    v = p.v()
    q = 3
    th = 2 * math.pi * q / p.Nx
    g = np.exp(-v ** 2)
    F = np.cos(th * np.arange(p.Nx))[:, None] * g[None, :]
    G = dense.rk4_step(F, p)
    cb = GOLD["d1_backward_periodic_c"]["value"]
    cf = GOLD["d1_forward_periodic_c"]["value"]
    for jv, vj in enumerate(v):
        sym = _symbol(cb, th, False) if vj > 0 else _symbol(cf, th, True)
        z = -vj * p.dt * sym / p.dx
        R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
        expect = g[jv] * np.real(R * np.exp(1j * th * np.arange(p.Nx)))
        assert np.abs(G[:, jv] - expect).max() < 1e-13
        assert abs(R) < 1.0


@pytest.mark.parametrize("order", [0, 1])
def test_untruncated_upwind_mps_step_equals_dense_step(order):
    """No truncation (tol = 0, no caps): the MPS RK4 step with the upwind
    T1 equals the dense step (SI: the MPS is exact at full rank)."""
    w = wl.landau_small(L=4, chi=10 ** 6, tol=0.0)
    p = w.problem
    p.order = order
    p.x_scheme = 1
    F = dense.initial(np.atleast_2d(w.ax), np.atleast_2d(w.bv))
    f = mps.init_mps(p, np.atleast_2d(w.ax), np.atleast_2d(w.bv))
    ops = mps.Operators(p)
    for _ in range(2):
        F = dense.rk4_step(F, p)
        f = mps.rk4_step(f, ops)
    assert np.abs(mps.to_dense(f, p) - F).max() < 1e-12 * np.abs(F).max()


def test_velocity_split_ranks():
    """v H(v) and v (1 - H(v)) on a grid symmetric about 0 (H is the top-bit
    projector there) keep the bond of v itself, 2; the paper quotes bond 2
    for the Heaviside MPO."""
    v = wl.landau_small(L=6).problem.v()
    assert GOLD["heaviside_mpo_bond"]["value"] == 2
    for u in (np.maximum(v, 0.0), np.minimum(v, 0.0)):
        assert max(mps.bond_dims(mps.vector_mps(u))) <= 2
    Hv = mps.vector_mps((v > 0).astype(float))
    assert max(mps.bond_dims(Hv)) <= 2


@pytest.mark.parametrize("mutation", ["downwind", "first_order"])
def test_planted_upwind_mistakes_are_caught(monkeypatch, mutation):
    """Taking the forward difference where v > 0 (the displayed formula's
    pairing) makes the single mode grow; a first-order backward stencil
    breaks the second-order pin."""
    if mutation == "downwind":
        orig_f, orig_b = dense.ddx_forward, dense.ddx_backward
        monkeypatch.setattr(dense, "ddx_backward", orig_f)
        monkeypatch.setattr(dense, "ddx_forward", orig_b)
        with pytest.raises(AssertionError):
            test_upwind_single_mode_matches_rk4_amplification()
    else:
        monkeypatch.setattr(dense, "ddx_backward",
                            lambda F, dx: (F - np.roll(F, 1, axis=0)) / dx)
        with pytest.raises(AssertionError):
            test_one_sided_stencils_are_second_order(False)
