"""Pins of the adaptive time step (Methods, "Time Evolution Procedure",
eq. CFL: a fraction of dt_max = (sum_s |v_s|_max/dx + |q_s||E|_max/(m_s dv_s)
+ collision terms)^-1, here one collisionless electron species) against a
closed form: on the Landau initial state the field is the single mode of
the Poisson pin, so |E|_max and the step are known by hand."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import dense
from oracle import mps


def _landau(cfl=0.9, L=6):
    w = wl.landau_small(L=L, chi=10 ** 6, tol=0.0)
    w.problem.cfl = cfl
    return w


def test_cfl_step_on_the_landau_state_matches_the_closed_form():
    w = _landau()
    p = w.problem
    F = dense.initial(np.atleast_2d(w.ax), np.atleast_2d(w.bv))
    # n = nbar (1 + a cos(k x)); E = -a nbar (dx/2) cot(k dx/2) sin(k x)
    nbar = p.dv * float(np.atleast_2d(w.bv)[0].sum())
    k, a = 0.5, 0.01
    emax = a * nbar * (p.dx / 2) / math.tan(k * p.dx / 2) * np.abs(np.sin(k * p.x())).max()
    vmax = max(abs(p.v_min), abs(p.v_max))
    want = 0.9 / (vmax / p.dx + abs(p.qm) * emax / p.dv)
    assert abs(dense.cfl_dt(F, p) - want) <= 1e-12 * want


def test_mps_and_dense_choose_the_same_step():
    w = _landau(L=4)
    p = w.problem
    F = dense.initial(np.atleast_2d(w.ax), np.atleast_2d(w.bv))
    f = mps.init_mps(p, np.atleast_2d(w.ax), np.atleast_2d(w.bv))
    ops = mps.Operators(p)
    for _ in range(3):
        assert abs(mps.cfl_dt(f, ops) - dense.cfl_dt(F, p)) <= 1e-12 * dense.cfl_dt(F, p)
        F = dense.rk4_step(F, p)
        f = mps.rk4_step(f, ops)
    assert np.abs(mps.to_dense(f, p) - F).max() <= 1e-12 * np.abs(F).max()


def _run(scheme, cfl, steps=200):
    w = _landau(cfl=cfl, L=5)
    p = w.problem
    p.x_scheme = scheme
    F = dense.initial(np.atleast_2d(w.ax), np.atleast_2d(w.bv))
    m0 = dense.diagnostics(F, p)["mass"]
    fmax = np.abs(F).max()
    for _ in range(steps):
        F = dense.rk4_step(F, p)
    return np.abs(F).max() / fmax, abs(dense.diagnostics(F, p)["mass"] - m0) / m0


def _rk4(z):
    return 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24


def test_adaptive_central_run_at_the_papers_fraction_is_stable():
    """0.9 of the CFL limit keeps v dt/dx <= 0.9, inside RK4's stability
    region on the imaginary axis (2 sqrt 2) where the central stencil's
    spectrum lies: 200 steps stay bounded and conserve mass."""
    growth, dm = _run(0, 0.9)
    assert growth < 1.01 and dm < 1e-10


def test_upwind_stability_limit_of_rk4():
    """The second-order upwind stencil's spectrum reaches -4 v / dx (the
    mode theta = pi), and RK4 is stable on the negative real axis only up
    to 2.785: the Courant number must stay below 0.696.  At 0.65 the run is
    stable; at the paper's 0.9 the amplification |R(-3.6)| = 3.1 > 1 and
    the run grows (a reading: the paper's fraction is kept for the central
    scheme only)."""
    assert abs(_rk4(-4 * 0.65)) < 1.0 < abs(_rk4(-4 * 0.9))
    growth, dm = _run(1, 0.65)
    assert growth < 1.01 and dm < 1e-10
    growth, _ = _run(1, 0.9)
    assert growth > 1.01
