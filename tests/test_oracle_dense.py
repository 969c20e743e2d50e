"""Pins of the dense-grid oracle (O1) against facts other than itself:
closed forms, textbook plasma physics, invariants and convergence order."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import dense
from tests import _dispersion as disp


def _run_field_energy(p, F, steps, dt):
    t, W = [0.0], [dense.diagnostics(F, p)["field_energy"]]
    for s in range(steps):
        F = dense.rk4_step(F, p, dt)
        t.append((s + 1) * dt)
        W.append(dense.diagnostics(F, p)["field_energy"])
    return F, np.array(t), np.array(W)


def test_poisson_closed_form_single_mode():
    # n = 1 + a cos(k x): L phi = a cos(kx) -> phi = a cos / lam,
    # E = -Dx phi = -a (dx/2) cot(k dx/2) sin(k x)   (hand derivation)
    for N, q in ((64, 1), (64, 5), (256, 3), (32, 15)):
        Lbox = 4 * math.pi
        dx = Lbox / N
        x = dx * np.arange(N)
        k = 2 * math.pi * q / Lbox
        a = 0.01
        E = dense.poisson_field(1.0 + a * np.cos(k * x), dx)
        ref = -a * (dx / 2) / math.tan(k * dx / 2) * np.sin(k * x)
        assert np.abs(E - ref).max() <= 1e-15 * max(1.0, np.abs(ref).max()) * 50


def test_poisson_fft_equals_dense_pseudo_inverse():
    rng = np.random.default_rng(3)
    for N in (8, 16, 64):
        n = rng.random(N) + 1.0
        dx = 0.37
        assert np.allclose(dense.poisson_field(n, dx),
                           dense.poisson_field_dense(n, dx), atol=1e-14 * N * N, rtol=0)


def test_poisson_continuum_limit():
    # E -> -(a/k) sin(kx) as dx -> 0 (Gauss law, neutralising background)
    N = 4096
    Lbox = 4 * math.pi
    x = Lbox / N * np.arange(N)
    E = dense.poisson_field(1 + 0.01 * np.cos(0.5 * x), Lbox / N)
    assert np.abs(E + 0.02 * np.sin(0.5 * x)).max() < 1e-7


def test_initial_field_energy_landau_64():
    w = wl.landau_small()
    p = w.problem
    F = dense.initial(w.ax, w.bv)
    WE = dense.diagnostics(F, p)["field_energy"]
    # closed form: E_i = -a (dx/2) cot(k dx/2) sin(k x_i) times the Riemann
    # sum of the Maxwellian (n = (1 + a cos) * dv * sum_j M(v_j))
    nfac = p.dv * w.bv[0].sum()
    amp = 0.01 * nfac * (p.dx / 2) / math.tan(0.5 * p.dx / 2)
    ref = 0.5 * p.dx * np.sum((amp * np.sin(0.5 * p.x())) ** 2)
    assert abs(WE - ref) <= 1e-12 * ref
    assert abs(WE - 1.2546189e-3) < 1e-9


def test_derivatives_exact_on_low_order_polynomials_and_modes():
    p = wl.landau_small().problem
    v = p.v()
    x = p.x()
    F = np.ones((p.Nx, 1)) * (v ** 2)[None, :]
    D = dense.ddv(F, p.dv)
    assert np.allclose(D[:, 1:-1], 2 * v[None, 1:-1], atol=1e-12)
    assert np.all(D[:, 0] == 0) and np.all(D[:, -1] == 0)
    k = 0.5
    G = np.sin(k * x)[:, None] * np.ones((1, p.Nv))
    Dx = dense.ddx(G, p.dx)
    ref = np.sin(k * p.dx) / p.dx * np.cos(k * x)
    assert np.allclose(Dx[:, 0], ref, atol=1e-13)


def test_landau_damping_rate_matches_dispersion_root():
    w0 = disp.root(0.5, [(1.0, 0.0)], 1.4 - 0.15j)
    assert abs(w0.real - 1.415662) < 1e-5 and abs(w0.imag + 0.153359) < 1e-5
    w = wl.landau_small(L=6, Lv=7)
    p = w.problem
    F = dense.initial(w.ax, w.bv)
    _, t, W = _run_field_energy(p, F, 600, 0.05)
    gamma, tp = disp.fit_rate(t, W, 0.0, 30.0, peaks=True)
    assert len(tp) >= 10
    assert abs(gamma - w0.imag) < 0.006, gamma
    # frequency from the spacing of the field-energy maxima (period pi/omega)
    omega = math.pi / np.mean(np.diff(tp))
    assert abs(omega - w0.real) < 0.03, omega


def test_two_stream_growth_rate_matches_dispersion_root():
    w0 = disp.root(0.2, [(0.5, 2.4), (0.5, -2.4)], 0.2j)
    assert abs(w0.real) < 1e-8 and abs(w0.imag - 0.225844) < 1e-5
    w = wl.two_stream(L=5, chi=0, dt_cfg=0.1, order=wl.ORDER_SEQ)
    p = w.problem
    p.Lv = 8
    ax, bv = wl.two_stream_profiles(p, 0.2, 1e-3)
    F = dense.initial(ax, bv)
    # early times are dominated by beating of the oscillating beam modes;
    # the growing mode dominates before saturation (t ~ 35)
    _, t, W = _run_field_energy(p, F, 300, 0.1)
    gamma, _ = disp.fit_rate(t, W, 20.0, 30.0, peaks=False)
    assert abs(gamma - w0.imag) < 0.01, gamma


def test_mass_conserved_up_to_v_boundary_flux():
    w = wl.landau_small()
    p = w.problem
    F = dense.initial(w.ax, w.bv)
    M0 = dense.diagnostics(F, p)["mass"]
    for _ in range(100):
        F = dense.rk4_step(F, p)
    M1 = dense.diagnostics(F, p)["mass"]
    assert abs(M1 - M0) / M0 < 1e-10


def test_rk4_fourth_order_in_time():
    w = wl.landau_small(L=5)
    p = w.problem
    F0 = dense.initial(w.ax, w.bv)
    T = 0.8
    sols = []
    for m in (4, 8, 16):
        F = F0.copy()
        for _ in range(m):
            F = dense.rk4_step(F, p, T / m)
        sols.append(F)
    r = np.abs(sols[0] - sols[1]).max() / np.abs(sols[1] - sols[2]).max()
    assert 13.0 < r < 19.0, r


@pytest.mark.parametrize("mutation", ["field_sign", "no_v_boundary", "dv_endpoints"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    """A plausible mistake planted in the oracle must break one of the pins."""
    if mutation == "field_sign":
        orig = dense.poisson_field
        monkeypatch.setattr(dense, "poisson_field", lambda n, dx: -orig(n, dx))
        w0 = disp.root(0.5, [(1.0, 0.0)], 1.4 - 0.15j)
        w = wl.landau_small(L=6)
        F = dense.initial(w.ax, w.bv)
        _, t, W = _run_field_energy(w.problem, F, 300, 0.05)
        try:
            gamma, tp = disp.fit_rate(t, W, 0.0, 15.0, peaks=True)
            caught = len(tp) < 5 or abs(gamma - w0.imag) > 0.006
        except Exception:
            caught = True
        assert caught
    elif mutation == "no_v_boundary":
        def bad(F, dv):
            out = np.zeros_like(F)
            out[:, 1:-1] = (F[:, 2:] - F[:, :-2]) / (2 * dv)
            out[:, 0] = F[:, 1] / (2 * dv)
            out[:, -1] = -F[:, -2] / (2 * dv)
            return out
        monkeypatch.setattr(dense, "ddv", bad)
        p = wl.landau_small().problem
        F = np.ones((p.Nx, 1)) * (p.v() ** 2)[None, :]
        D = dense.ddv(F, p.dv)
        assert not (np.all(D[:, 0] == 0) and np.all(D[:, -1] == 0))
    else:
        w = wl.landau_small()
        p = w.problem
        F = dense.initial(w.ax, w.bv)
        bad_dv = (p.v_max - p.v_min) / p.Nv
        nfac = bad_dv * w.bv[0].sum()
        amp = 0.01 * nfac * (p.dx / 2) / math.tan(0.5 * p.dx / 2)
        ref = 0.5 * p.dx * np.sum((amp * np.sin(0.5 * p.x())) ** 2)
        assert abs(dense.diagnostics(F, p)["field_energy"] - ref) > 1e-12 * ref
