"""Pins of the collision operator and of several species in the CPU
oracles (Methods: Collision Operator; the two-species set-ups; Buneman
instability).

Collisions with fixed v0 and vth (coll_model 1), nu d/dv[(v - v0) f + vth^2
df/dv], are an Ornstein-Uhlenbeck (Fokker-Planck) operator: M(v) He_n((v - v0)/vth), M the
Maxwellian, is an eigenfunction with eigenvalue -n nu (textbook; not from
the paper).  Two species: identical species of opposite charge leave no
field; ions at rest with a uniform density reproduce the one-species run on
a neutralising background; the Buneman growth rate of the dense run matches
the root of the two-species kinetic dispersion relation."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import dense
from oracle import mps
from tests._dispersion import root_species


def _coll_problem(Lv, nu=1.0, v0=0.5, vth=1.3):
    # the fixed-parameter model: an Ornstein-Uhlenbeck operator
    return wl.Problem(Lx=2, Lv=Lv, order=0, x_min=0.0, x_max=1.0, v_min=-12.0,
                      v_max=12.0, nu=nu, nu_v0=v0, nu_vth=vth, coll_model=1)


def _hermite_mode(p, n):
    w = (p.v() - p.nu_v0) / p.nu_vth
    He = {0: np.ones_like(w), 1: w, 2: w * w - 1.0, 3: w ** 3 - 3.0 * w}[n]
    return np.tile(np.exp(-0.5 * w * w) * He, (p.Nx, 1))


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_collision_hermite_modes_decay_at_rate_n_nu(n):
    errs = []
    for Lv in (8, 9):
        p = _coll_problem(Lv, nu=0.7)
        F = _hermite_mode(p, n)
        CF = dense.collision(F, p)
        errs.append(np.abs(CF + n * p.nu * F).max() / np.abs(F).max())
    assert errs[1] < 1e-2
    assert 3.8 < errs[0] / errs[1] < 4.2        # second order in dv


def test_collision_conserves_mass_of_a_confined_distribution():
    p = _coll_problem(9)
    F = _hermite_mode(p, 0) * (1.0 + 0.3 * _hermite_mode(p, 1))
    CF = dense.collision(F, p)
    assert abs(CF.sum()) * p.dv < 1e-12 * np.abs(F).sum() * p.dv


def _stencil_zero_gradient(N, h):
    D = np.zeros((N, N))
    for o in range(1, N - 1):
        D[o, o + 1] += 0.5 / h
        D[o, o - 1] -= 0.5 / h
    return D


def test_collision_mpo_is_the_dense_operator():
    p = _coll_problem(4, nu=0.9)
    ops = mps.Operators(p)
    M = mps.mpo_to_matrix(ops.T3)
    D = _stencil_zero_gradient(p.Nv, p.dv)
    Cv = p.nu * D @ (np.diag(p.v() - p.nu_v0) + p.nu_vth ** 2 * D)
    assert np.abs(M - np.kron(np.eye(p.Nx), Cv)).max() < 1e-11 * np.abs(Cv).max()


@pytest.mark.parametrize("order", [0, 1])
def test_untruncated_step_with_collisions_equals_dense(order):
    w = wl.landau_small(L=4, tol=0.0)
    p = w.problem
    p.order, p.chi_max = order, None
    p.nu, p.nu_v0, p.nu_vth = 0.3, 0.2, 1.1
    ops = mps.Operators(p)
    F = dense.initial(w.ax, w.bv)
    f = mps.init_mps(p, w.ax, w.bv)
    for k in range(2):
        f = mps.rk4_step(f, ops)
        F = dense.rk4_step(F, p)
        assert np.abs(mps.to_dense(f, p) - F).max() < 1e-12 * (k + 1) * np.abs(F).max()


def test_opposite_charges_of_identical_species_leave_no_field():
    w = wl.landau_small(L=5)
    p = w.problem
    F = dense.initial(w.ax, w.bv)
    E = dense.field_species([F, F], [p, p], [-1.0, 1.0])
    assert np.abs(E).max() == 0.0
    # a sign mistake in the charge sum would double the field instead
    E1 = dense.field_species([F, F], [p, p], [-1.0, -1.0])
    assert np.abs(E1 - 2.0 * dense.field(F, p)).max() < 1e-14


def test_uniform_ions_at_rest_reproduce_the_neutralising_background():
    w = wl.landau_small(L=5)
    pe = w.problem
    pi_ = wl.Problem(Lx=pe.Lx, Lv=4, order=0, x_min=pe.x_min, x_max=pe.x_max,
                     v_min=-1.0, v_max=1.0, qm=0.0, dt=pe.dt)
    Fe = dense.initial(w.ax, w.bv)
    Fi = np.tile(np.exp(-np.linspace(-1, 1, 16) ** 2), (pe.Nx, 1))
    out = dense.rk4_step_species([Fe, Fi], [pe, pi_], [-1.0, 1.0], pe.dt)
    assert np.abs(out[0] - dense.rk4_step(Fe, pe)).max() < 1e-13 * np.abs(Fe).max()
    assert np.abs(out[1] - Fi).max() < 1e-13 * np.abs(Fi).max()   # qm = 0, v-advection only


def test_untruncated_two_species_mps_step_equals_dense():
    ws, q = wl.buneman(L=3, Lv=4, chi=1 << 10, tol=0.0, level=1)
    ps = [w.problem for w in ws]
    for p in ps:
        p.chi_max = None
        p.nu, p.nu_vth = 0.05, p.nu_vth
    opss = [mps.Operators(p) for p in ps]
    Fs = [dense.initial(w.ax, w.bv) for w in ws]
    fs = [mps.init_mps(p, w.ax, w.bv) for p, w in zip(ps, ws)]
    for _ in range(2):
        fs = mps.rk4_step_species(fs, opss, q, ps[0].dt)
        Fs = dense.rk4_step_species(Fs, ps, q, ps[0].dt)
    for f, F, p in zip(fs, Fs, ps):
        assert np.abs(mps.to_dense(f, p) - F).max() < 1e-11 * np.abs(F).max()
    E = mps.to_vector(mps.field_species_mps(fs, opss, q))
    Ed = dense.field_species(Fs, ps, q)
    assert np.abs(E - Ed).max() < 1e-10 * np.abs(Ed).max()


def test_buneman_growth_rate_matches_the_kinetic_dispersion_root():
    ws, q = wl.buneman(L=5, Lv=9)
    ps = [w.problem for w in ws]
    k = 0.1
    mr = 1.0 / ps[1].qm
    gamma = root_species(k, [(1.0, 1.0, 1.0 / k), (1.0 / mr, math.sqrt(1.0 / mr), 0.0)],
                         0.136 + 0.235j).imag
    assert abs(gamma - 0.19850) < 1e-4
    Fs = [dense.initial(w.ax, w.bv) for w in ws]
    t, T, A = 0.0, [], []
    for n in range(int(36.0 / ps[0].dt)):
        if n % 10 == 0:
            T.append(t)
            A.append(abs(np.fft.fft(dense.field_species(Fs, ps, q))[1]))
        Fs = dense.rk4_step_species(Fs, ps, q, ps[0].dt)
        t += ps[0].dt
    T, A = np.array(T), np.array(A)
    sel = (T >= 15.0) & (T <= 35.0)
    rate = np.polyfit(T[sel], np.log(A[sel]), 1)[0]
    assert abs(rate - gamma) < 0.05 * gamma, (rate, gamma)


def test_cfl_step_adds_the_collision_terms():
    w = wl.landau_small(L=4)
    p = w.problem
    p.cfl = 0.9
    F = dense.initial(w.ax, w.bv)
    dt0 = dense.cfl_dt(F, p)
    p.nu, p.nu_vth = 0.5, 1.0
    dt1 = dense.cfl_dt(F, p)
    vmax = max(abs(p.v_min), abs(p.v_max))
    extra = p.nu * vmax / p.dv + 2.0 * p.nu / p.dv ** 2
    assert abs(1.0 / dt1 - (1.0 / dt0 + extra / p.cfl)) < 1e-12 / dt1
    f = mps.init_mps(p, w.ax, w.bv)
    assert abs(mps.cfl_dt(f, mps.Operators(p)) - dt1) < 1e-12 * dt1
