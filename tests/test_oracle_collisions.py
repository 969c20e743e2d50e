"""Pins of the Dougherty collision operator with the species' own moments
(Methods, Collision Operator: v0 the average velocity, vth the thermal
velocity of the species, here at each x).

Facts used (textbook properties of this operator, not from the paper):
* a local Maxwellian n(x) exp(-(v - u(x))^2 / 2T(x)) / sqrt(2 pi T(x)) is
  its equilibrium when v0 = u and vth^2 = T are the Maxwellian's own
  moments: the discrete operator vanishes on it up to O(dv^2);
* it conserves the density, momentum and energy at every x.  With the
  central difference the discrete sums do so exactly: summing by parts,
  sum_j v_j (Dv G)_j = -sum_j G_j and sum_j v_j^2 (Dv G)_j = -2 sum_j v_j G_j
  up to boundary rows, and the moments v0 = P / n, vth^2 = W / n - v0^2 make
  sum (v - v0) f = 0 and sum v [(v - v0) f + vth^2 Dv f] = 0, so the moments
  1, v, v^2 of C[f] vanish to rounding for any f confined inside the v
  interval.
A drift or temperature taken from the wrong moments (averaged over x, or
vth^2 without the -v0^2) breaks the equilibrium pin."""
import numpy as np
import pytest

import workloads as wl
from oracle import dense
from oracle import mps


def _problem(Lx, Lv, nu=0.8):
    return wl.Problem(Lx=Lx, Lv=Lv, order=0, x_min=0.0, x_max=2 * np.pi, v_min=-10.0,
                      v_max=10.0, nu=nu, tol=0.0)


def _local_maxwellian(p):
    x, v = p.x(), p.v()
    n = 1.0 + 0.3 * np.cos(x)
    u = 0.8 * np.sin(x)
    T = 1.0 + 0.4 * np.cos(2 * x)
    return (n[:, None] / np.sqrt(2 * np.pi * T[:, None])
            * np.exp(-(v[None, :] - u[:, None]) ** 2 / (2 * T[:, None])))


def _two_beams(p):
    """Two beams whose weights vary differently with x: the local drift and
    temperature vary with x."""
    x, v = p.x(), p.v()
    a = 1.0 + 0.2 * np.cos(x)
    b = 0.6 * (1.0 - 0.3 * np.sin(x))
    return (a[:, None] * np.exp(-(v[None, :] - 2.0) ** 2 / 1.2)
            + b[:, None] * np.exp(-(v[None, :] + 1.5) ** 2 / 0.8))


def test_local_maxwellian_is_the_equilibrium_at_second_order():
    errs = []
    for Lv in (8, 9, 10):
        p = _problem(5, Lv)
        F = _local_maxwellian(p)
        C = dense.collision(F, p)
        errs.append(np.abs(C).max() / (p.nu * np.abs(F).max()))
    assert errs[-1] < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_density_momentum_energy_are_conserved_exactly():
    out = []
    for Lv in (6, 8, 10):
        p = _problem(4, Lv)
        F = _two_beams(p)
        C = dense.collision(F, p)
        v = p.v()
        scale = p.nu * p.dv * np.abs(F).sum(axis=1).max() * 10.0
        m0 = np.abs(p.dv * C.sum(axis=1)).max() / scale
        m1 = np.abs(p.dv * (C * v).sum(axis=1)).max() / scale
        m2 = np.abs(p.dv * (C * v * v).sum(axis=1)).max() / scale
        out.append((m0, m1, m2))
        # the drift and temperature really vary with x (the operator is not
        # a single Maxwellian's linearisation)
        v0, T = dense.collision_moments(F, p)
        assert np.ptp(v0) > 1e-2 and np.ptp(T) > 1e-2
    for o in out:
        assert max(o) < 1e-13, o


def test_wrong_temperature_breaks_energy_conservation(monkeypatch):
    real = dense.collision_moments
    p = _problem(4, 9)
    F = _two_beams(p)
    monkeypatch.setattr(dense, "collision_moments",
                        lambda F, p: (real(F, p)[0], real(F, p)[1] + real(F, p)[0] ** 2))
    C = dense.collision(F, p)
    e = np.abs(p.dv * (C * p.v() ** 2).sum(axis=1)).max()
    assert e > 1e-3 * p.nu * p.dv * np.abs(F).sum(axis=1).max()


@pytest.mark.parametrize("mistake", ["x_average", "no_drift_in_vth"])
def test_wrong_moments_break_the_equilibrium(monkeypatch, mistake):
    real = dense.collision_moments

    def planted(F, p):
        v0, T = real(F, p)
        if mistake == "x_average":
            return np.full_like(v0, v0.mean()), np.full_like(T, T.mean())
        return v0, T + v0 ** 2

    p = _problem(5, 10)
    F = _local_maxwellian(p)
    good = np.abs(dense.collision(F, p)).max()
    monkeypatch.setattr(dense, "collision_moments", planted)
    bad = np.abs(dense.collision(F, p)).max()
    assert bad > 100 * good


@pytest.mark.parametrize("order", [0, 1, 2])
def test_mps_moment_fields_equal_the_dense_moments(order):
    p = _problem(5, 5)
    p.order = order
    F = _two_beams(p)
    g = mps.tt_svd(mps.dense_to_sites(F, p.Lx, p.Lv, order), [2] * (p.Lx + p.Lv))
    v0m, Tm = mps.collision_moment_fields(g, mps.Operators(p))
    v0, T = dense.collision_moments(F, p)
    assert np.abs(mps.to_vector(v0m) - v0).max() < 1e-12 * np.abs(v0).max()
    assert np.abs(mps.to_vector(Tm) - T).max() < 1e-12 * np.abs(T).max()


@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_untruncated_mps_step_with_moment_collisions_equals_dense(order):
    w = wl.two_stream(L=4, chi=0, tol=0.0, level=1, dt_cfg=0.05, order=order)
    p = w.problem
    p.chi_max = None
    p.nu = 0.3
    F = dense.initial(w.ax, w.bv)
    f = mps.init_mps(p, w.ax, w.bv)
    ops = mps.Operators(p)
    for k in range(2):
        f = mps.rk4_step(f, ops)
        F = dense.rk4_step(F, p)
        assert np.abs(mps.to_dense(f, p) - F).max() < 1e-12 * (k + 1) * np.abs(F).max()
