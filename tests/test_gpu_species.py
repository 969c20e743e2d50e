"""GPU parity of collisions and of several species (Methods: Collision
Operator; the two-species set-ups) through the C-ABI, against the dense and
MPS oracles."""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import dense as odense
from oracle import mps as omps
from tests import _start as S

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2205_11990_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("order,model", [(0, 0), (1, 0), (2, 0), (3, 0), (0, 1), (1, 1)])
def test_untruncated_collisional_steps_equal_dense_oracle(B, order, model):
    """Dougherty collisions, untruncated: model 0 takes the drift and thermal
    speed from the moments of each stage's state (per x), model 1 keeps the
    given constants; the MPS steps equal the dense steps."""
    _say("untruncated collisions order=%d model=%d" % (order, model))
    w = wl.landau_small(L=4, tol=0.0)
    p = w.problem
    p.order, p.chi_max, p.level = order, 1 << 20, 1
    p.nu, p.nu_v0, p.nu_vth, p.coll_model = 0.3, 0.2, 1.1, model
    st = B.MpsState(p, w.ax, w.bv)
    F = odense.initial(w.ax, w.bv)
    for k in range(3):
        st.step(1)
        F = odense.rk4_step(F, p)
        G = st.to_dense().cpu().numpy()
        assert np.abs(G - F).max() <= 1e-12 * (k + 2) * np.abs(F).max(), k
    st.free()


@pytest.mark.parametrize("order,model,tol", [(0, 0, 0.0), (1, 0, 0.0), (0, 0, 1e-10),
                                             (0, 1, 0.0)])
def test_truncated_collisional_steps_match_mps_oracle(B, order, model, tol):
    """Collisions with every point capped (C5, chi = 8, the moment fields
    capped at D_F = 4 like E), or the paper's C1/tol schedule: f and E within
    1e-8 of the MPS oracle after two steps, same bonds."""
    _say("truncated collisions two-stream L=5 order=%d model=%d tol=%g" % (order, model, tol))
    w = wl.two_stream(L=5, chi=8, tol=tol, level=5 if tol == 0 else 1, df_max=4,
                      dt_cfg=0.05, order=order)
    p = w.problem
    p.nu, p.nu_v0, p.nu_vth, p.coll_model = 0.2, 0.0, 1.0, model
    f = S.oracle_start(w, pert_chi=8, amp=1e-3)
    st = S.gpu_state(B, w, f)
    ops = omps.Operators(p)
    for _ in range(2):
        st.step(1)
        f = omps.rk4_step(f, ops)
    G = st.to_dense().cpu().numpy()
    R = omps.to_dense(f, p)
    _, E = st.density_field()
    Eref = omps.field_dense(f, ops)
    assert np.abs(G - R).max() <= 1e-8 * np.abs(R).max()
    assert np.abs(E.cpu().numpy() - Eref).max() <= 1e-8 * np.abs(Eref).max()
    assert st.info()["bonds"][1:-1] == omps.bond_dims(f)
    st.free()


def test_one_species_plasma_equals_the_single_species_step(B):
    _say("plasma of one electron species == mps_step")
    w = wl.landau_small(L=5, chi=16, tol=1e-10)
    p = w.problem
    pl = B.Plasma([p], [-1.0], [(w.ax, w.bv)])
    st = B.MpsState(p, w.ax, w.bv)
    pl.step(3)
    st.step(3)
    a = pl.species(0).get_cores_host()
    b = st.get_cores_host()
    assert [x.shape for x in a] == [x.shape for x in b]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    E, W = pl.field()
    _, E1 = st.density_field()
    assert np.array_equal(E.cpu().numpy(), E1.cpu().numpy())
    st.free()
    pl.free()


def test_untruncated_buneman_plasma_equals_dense_oracle(B):
    _say("untruncated buneman plasma Lx=3 Lv=4")
    ws, q = wl.buneman(L=3, Lv=4, chi=1 << 20, tol=0.0, level=1)
    ps = [w.problem for w in ws]
    for p in ps:
        p.nu = 0.05
    pl = B.Plasma(ps, q, [(w.ax, w.bv) for w in ws])
    Fs = [odense.initial(w.ax, w.bv) for w in ws]
    for _ in range(3):
        pl.step(1)
        Fs = odense.rk4_step_species(Fs, ps, q, ps[0].dt)
    for s, (F, p) in enumerate(zip(Fs, ps)):
        G = pl.species(s).to_dense().cpu().numpy()
        assert np.abs(G - F).max() <= 1e-11 * np.abs(F).max(), s
    E, W = pl.field()
    Ed = odense.field_species(Fs, ps, q)
    assert np.abs(E.cpu().numpy() - Ed).max() <= 1e-10 * np.abs(Ed).max()
    assert abs(W - 0.5 * ps[0].dx * np.sum(Ed ** 2)) <= 1e-10 * W
    pl.free()


@pytest.mark.parametrize("order,comp,nu", [(0, 0, 0.0), (1, 0, 0.0), (2, 1, 0.02), (4, 0, 0.02)])
def test_truncated_buneman_plasma_matches_mps_oracle(B, order, comp, nu):
    """Electrons and ions, every point capped (C5, chi = 8, D_F = 4), the
    electrons perturbed to full bonds: both species and the shared field
    within 1e-8 of the MPS oracle after 2 steps from the same states (the
    oracle's, handed to the GPU; S1,
    IF, S2 with centre-first compression and collisions, IG with
    collisions)."""
    _say("truncated buneman plasma L=5 chi8 order=%d compression=%d nu=%g" % (order, comp, nu))
    ws, q = wl.buneman(L=5, chi=8, tol=0.0, level=5, df_max=4, order=order, nu=nu)
    ps = [w.problem for w in ws]
    for p in ps:
        p.compression = comp
    pl = B.Plasma(ps, q, [(w.ax, w.bv) for w in ws])
    fs = [S.oracle_start(ws[0], pert_chi=8, amp=1e-4), S.oracle_start(ws[1])]
    for s, (f, p) in enumerate(zip(fs, ps)):
        pl.species(s).set_cores(S.binary_cores(f, p))
    opss = [omps.Operators(p) for p in ps]
    for _ in range(2):
        pl.step(1)
        fs = omps.rk4_step_species(fs, opss, q, ps[0].dt)
    for s, (f, p) in enumerate(zip(fs, ps)):
        st = pl.species(s)
        G = st.to_dense().cpu().numpy()
        R = omps.to_dense(f, p)
        assert np.abs(G - R).max() <= 1e-8 * np.abs(R).max(), s
        b = st.info()["bonds"]
        assert (b[2:p.n_sites:2] if order == 4 else b[1:-1]) == omps.bond_dims(f), s
    E, _ = pl.field()
    Eref = omps.to_vector(omps.field_species_mps(fs, opss, q))
    assert np.abs(E.cpu().numpy() - Eref).max() <= 1e-8 * np.abs(Eref).max()
    pl.free()


@pytest.mark.parametrize("nu", [0.0, 0.05])
def test_two_species_landau_real_mass_ratio(B, nu):
    """The paper's nonlinear Landau set-up with mobile ions at the real mass
    ratio m_i/m_e = 1836 (ion thermal speed 1/sqrt(1836), A = 0.5,
    k = 0.75), with and without collisions: untruncated steps equal the
    dense steps of both species, and capped steps (C5, chi = 8, D_F = 4)
    match the MPS oracle within 1e-8."""
    _say("two-species Landau m_i/m_e = 1836 nu=%g" % nu)
    ws, q = wl.landau_two_species(L=3, Lv=4, chi=1 << 20, tol=0.0, level=1, nu=nu)
    ps = [w.problem for w in ws]
    pl = B.Plasma(ps, q, [(w.ax, w.bv) for w in ws])
    Fs = [odense.initial(w.ax, w.bv) for w in ws]
    for _ in range(2):
        pl.step(1)
        Fs = odense.rk4_step_species(Fs, ps, q, ps[0].dt)
    for s_, F in enumerate(Fs):
        G = pl.species(s_).to_dense().cpu().numpy()
        assert np.abs(G - F).max() <= 1e-11 * np.abs(F).max(), s_
    pl.free()
    ws, q = wl.landau_two_species(L=5, chi=8, tol=0.0, level=5, df_max=4, nu=nu)
    ps = [w.problem for w in ws]
    pl = B.Plasma(ps, q, [(w.ax, w.bv) for w in ws])
    fs = [S.oracle_start(ws[0], pert_chi=8, amp=1e-4), S.oracle_start(ws[1])]
    for s_, (f, p) in enumerate(zip(fs, ps)):
        pl.species(s_).set_cores(S.binary_cores(f, p))
    opss = [omps.Operators(p) for p in ps]
    for _ in range(2):
        pl.step(1)
        fs = omps.rk4_step_species(fs, opss, q, ps[0].dt)
    for s_, (f, p) in enumerate(zip(fs, ps)):
        G = pl.species(s_).to_dense().cpu().numpy()
        R = omps.to_dense(f, p)
        assert np.abs(G - R).max() <= 1e-8 * np.abs(R).max(), s_
    E, _ = pl.field()
    Eref = omps.to_vector(omps.field_species_mps(fs, opss, q))
    assert np.abs(E.cpu().numpy() - Eref).max() <= 1e-8 * np.abs(Eref).max()
    pl.free()


def test_plasma_species_cannot_be_stepped_or_freed_alone(B):
    _say("plasma species handles are owned by the plasma")
    ws, q = wl.buneman(L=3, Lv=4, chi=8)
    pl = B.Plasma([w.problem for w in ws], q, [(w.ax, w.bv) for w in ws])
    st = pl.species(1)
    with pytest.raises(B.MpsError):
        st.step(1)
    assert B.lib().mps_free(st.handle) != 0
    with pytest.raises(B.MpsError):
        B.step_batched([st], 1)
    pl.free()


def test_plasma_failure_leaves_every_species_unchanged(B):
    """A forced non-convergence in a plasma step fails it for all species:
    none of them is committed."""
    _say("plasma failure is all or none")
    ws, q = wl.buneman(L=5, chi=8, tol=0.0, level=5, df_max=4)
    pl = B.Plasma([w.problem for w in ws], q, [(w.ax, w.bv) for w in ws])
    pl.species(0).add_scaled(1e-4, wl.random_mps_cores(ws[0].problem.n_sites, 8, seed=3))
    before = [pl.species(s).get_cores_host() for s in range(2)]
    B.set_jacobi_max_sweeps(1)
    try:
        with pytest.raises(B.MpsError) as e:
            pl.step(1)
        assert e.value.status == B.MPS_ENUMERIC
    finally:
        B.set_jacobi_max_sweeps(60)
    for s in range(2):
        after = pl.species(s).get_cores_host()
        assert all(np.array_equal(x, y) for x, y in zip(before[s], after)), s
        assert pl.species(s).info()["steps"] == 0
    pl.step(1)
    assert all(pl.species(s).info()["steps"] == 1 for s in range(2))
    pl.free()


def test_gpu_landau_damping_rate(B):
    """Physics end to end on the GPU: 64 x 64 Landau, chi = 16, tol = 1e-10,
    600 steps (t = 30): the field energy decays at twice the kinetic damping
    rate (gamma = -0.1534, the root of the dispersion relation)."""
    _say("GPU Landau damping rate, 600 steps")
    from tests import _dispersion as disp
    w0 = disp.root(0.5, [(1.0, 0.0)], 1.4 - 0.15j)
    w = wl.landau_small(L=6, chi=16, tol=1e-10)
    p = w.problem
    st = B.MpsState(p, w.ax, w.bv)
    t, W = [0.0], [st.moments()[2]["field_energy"]]
    for s in range(600):
        st.step(1)
        t.append((s + 1) * p.dt)
        W.append(st.moments()[2]["field_energy"])
        if s % 100 == 99:
            _say("  step %d" % (s + 1))
    gamma, tp = disp.fit_rate(t, W, 0.0, 30.0, peaks=True)
    assert len(tp) >= 10
    assert abs(gamma - w0.imag) < 0.01, gamma
    st.free()


def test_gpu_buneman_growth_rate(B):
    """Physics end to end with two species on the GPU: Buneman at 32 x 512
    per species, chi = 32, tol = 1e-10; the k = 0.1 field mode grows at the
    root of the two-species kinetic dispersion relation (0.1985) within 5 %."""
    _say("GPU Buneman growth rate")
    import math
    from tests import _dispersion as disp
    ws, q = wl.buneman(L=5, Lv=9, chi=32, tol=1e-10, level=1)
    ps = [w.problem for w in ws]
    mr = 1.0 / ps[1].qm
    gamma = disp.root_species(0.1, [(1.0, 1.0, 10.0), (1.0 / mr, math.sqrt(1.0 / mr), 0.0)],
                              0.136 + 0.235j).imag
    pl = B.Plasma(ps, q, [(w.ax, w.bv) for w in ws])
    T, A = [], []
    n_steps = int(36.0 / ps[0].dt)
    for n in range(n_steps):
        if n % 10 == 0:
            E, _ = pl.field()
            T.append(n * ps[0].dt)
            A.append(abs(np.fft.fft(E.cpu().numpy())[1]))
        pl.step(1)
        if n % 200 == 199:
            _say("  step %d of %d" % (n + 1, n_steps))
    T, A = np.array(T), np.array(A)
    sel = (T >= 15.0) & (T <= 35.0)
    rate = np.polyfit(T[sel], np.log(A[sel]), 1)[0]
    assert abs(rate - gamma) < 0.05 * gamma, (rate, gamma)
    pl.free()
