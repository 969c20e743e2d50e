"""GPU tests of lock-step batches (mps_batch_*): several instances of one
problem shape stepped by launches that cover all of them.  Each instance
must equal a stand-alone state stepped from the same cores bit for bit, and
the CPU MPS oracle within the truncated-parity bound."""
import math
import sys

import numpy as np
import pytest

import workloads as wl
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


def _sweep(count, L=5, chi=8, order=1, level=5):
    """Two-stream instances of one shape: wave numbers k = 0.2 .. 0.35 (x
    intervals) and amplitudes alpha, one common dt (the smallest stable
    one)."""
    ws = []
    for i in range(count):
        k = 0.2 + 0.05 * i
        w = wl.two_stream(L=L, chi=chi, tol=0.0, level=level, df_max=4, dt_cfg=0.05,
                          order=order)
        p = w.problem
        p.x_max = 2.0 * math.pi / k
        ax, bv = wl.two_stream_profiles(p, k, 1e-3 * (1 + i))
        ws.append(wl.Workload("sweep_%d" % i, p, ax, bv, 10))
    dt = min(wl.stable_dt(w.problem, 0.05) for w in ws)
    for w in ws:
        w.problem.dt = dt
    return ws


@pytest.mark.parametrize("order,comp", [(1, 0), (0, 0), (0, 1)])
def test_batch_equals_solo_bit_for_bit(B, order, comp):
    """Four instances (different k and alpha, perturbed to full bonds) in
    one batch against the same four as stand-alone states from the same
    cores: after two steps every instance's cores and dense values are
    identical."""
    _say("batch == solo order=%d compression=%d" % (order, comp))
    ws = _sweep(4, order=order)
    for w in ws:
        w.problem.compression = comp
    starts = [S.oracle_start(w, pert_chi=8, amp=1e-3, seed=10 + i) for i, w in enumerate(ws)]
    bt = B.Batch([w.problem for w in ws], [(w.ax, w.bv) for w in ws])
    bt.set_cores(starts)
    bt.step(2)
    for i, w in enumerate(ws):
        st = S.gpu_state(B, w, starts[i])
        st.step(2)
        a, b = bt.instance(i).get_cores_host(), st.get_cores_host()
        assert [x.shape for x in a] == [x.shape for x in b], i
        for x, y in zip(a, b):
            assert np.array_equal(x, y), i
        assert np.array_equal(bt.instance(i).to_dense().cpu().numpy(),
                              st.to_dense().cpu().numpy()), i
        st.free()
    bt.free()


def test_wy_reflectors_batch_equals_solo_and_oracle(B):
    """Compact-WY reflector application on tall blocks (tall_apply = 1;
    two-stream 2^9, chi = 16, D_F = 4: the field term's blocks reach 640
    rows): three instances in one batch equal the same three stand-alone
    states with the same mode bit for bit after two steps; each is within
    1e-8 of the oracle and differs from the one-reflector mode only at the
    rounding level."""
    _say("batch == solo, compact-WY reflectors")
    ws = _sweep(3, L=9, chi=16)
    for w in ws:
        w.problem.tall_apply = 1
    starts = [S.oracle_start(w, pert_chi=16, amp=1e-3, seed=70 + i) for i, w in enumerate(ws)]
    bt = B.Batch([w.problem for w in ws], [(w.ax, w.bv) for w in ws])
    bt.set_cores(starts)
    bt.step(2)
    for i, w in enumerate(ws):
        st = S.gpu_state(B, w, starts[i])
        st.step(2)
        a, b = bt.instance(i).get_cores_host(), st.get_cores_host()
        assert [x.shape for x in a] == [x.shape for x in b], i
        for x, y in zip(a, b):
            assert np.array_equal(x, y), i
        G = st.to_dense().cpu().numpy()
        st.free()
        ops = omps.Operators(w.problem)
        R = omps.to_dense(omps.rk4_step(omps.rk4_step(starts[i], ops), ops), w.problem)
        assert np.abs(G - R).max() <= 1e-8 * np.abs(R).max(), i
        w.problem.tall_apply = 0
        st0 = S.gpu_state(B, w, starts[i])
        st0.step(2)
        G0 = st0.to_dense().cpu().numpy()
        st0.free()
        w.problem.tall_apply = 1
        # the two modes are different arithmetic of the same factor
        assert not np.array_equal(G, G0), i
        assert np.abs(G - G0).max() <= 1e-11 * np.abs(G0).max(), i
    bt.free()


def test_forty_instances_equal_solo_in_the_compact_wy_mode(B):
    """Forty lock-step instances (the launch-shape table's class of 32 or
    more; two-stream 2^9, chi = 16, compact-WY mode with panel groups on its
    640-row blocks) after two steps: instances 0, 17 and 39 equal the same
    problems stepped alone, bit for bit."""
    _say("batch of 40 == solo, compact-WY")
    ws = []
    for i in range(40):
        w = wl.two_stream(L=9, chi=16, tol=0.0, level=5, df_max=4, dt_cfg=0.05)
        w.problem.tall_apply = 1
        ax, bv = wl.two_stream_profiles(w.problem, 0.2, 1e-3 * (1 + 0.05 * i))
        ws.append(wl.Workload("forty_%d" % i, w.problem, ax, bv, 2))
    bt = B.Batch([w.problem for w in ws], [(w.ax, w.bv) for w in ws])
    p = ws[0].problem
    perts = [wl.random_mps_cores(p.n_sites, 16, seed=400 + i) for i in range(40)]
    amps = [1e-3] * 40
    bt.add_scaled(amps, perts)
    starts = [bt.instance(i).get_cores_host() for i in (0, 17, 39)]
    bt.step(2)
    for j, i in enumerate((0, 17, 39)):
        st = S.gpu_state(B, ws[i], starts[j])
        st.step(2)
        a, b = bt.instance(i).get_cores_host(), st.get_cores_host()
        assert [x.shape for x in a] == [x.shape for x in b], i
        for x, y in zip(a, b):
            assert np.array_equal(x, y), i
        st.free()
    bt.free()


@pytest.mark.parametrize("L,chi,tall", [(6, 16, 0), (9, 16, 1)])
def test_batch_step_graph_replays_equal_eager_steps(B, L, chi, tall):
    """A lock-step batch (three instances) stepped from a captured graph: after
    each of five steps, with moments read in between, every instance's
    cores equal those of the same batch stepped launch by launch, bit for
    bit (the one-reflector mode, and the compact-WY mode with panel groups
    of 640-row blocks).  The first step runs eagerly, the second captures,
    the rest replay."""
    _say("batch step graph L=%d chi=%d tall_apply=%d" % (L, chi, tall))
    ws = _sweep(3, L=L, chi=chi)
    for w in ws:
        w.problem.tall_apply = tall
    starts = [S.oracle_start(w, pert_chi=chi, amp=1e-3, seed=90 + i) for i, w in enumerate(ws)]
    a = B.Batch([w.problem for w in ws], [(w.ax, w.bv) for w in ws])
    b = B.Batch([w.problem for w in ws], [(w.ax, w.bv) for w in ws])
    a.set_cores(starts)
    b.set_cores(starts)
    a.step_graph(True)
    for k in range(5):
        a.step(1)
        b.step(1)
        for i in range(3):
            ca, cb = a.instance(i).get_cores_host(), b.instance(i).get_cores_host()
            assert [x.shape for x in ca] == [x.shape for x in cb], (k, i)
            for x, y in zip(ca, cb):
                assert np.array_equal(x, y), (k, i)
        a.instance(k % 3).moments()
    assert a.step_graph() == (1, 4)
    assert b.step_graph() == (0, 0)
    a.free()
    b.free()


def test_batch_matches_mps_oracle(B):
    """Three instances, C5, chi = 8: each instance's f and E within 1e-8 of
    the CPU MPS oracle after two steps from the same state, same bonds."""
    _say("batch vs oracle")
    ws = _sweep(3)
    starts = [S.oracle_start(w, pert_chi=8, amp=1e-3, seed=20 + i) for i, w in enumerate(ws)]
    bt = B.Batch([w.problem for w in ws], [(w.ax, w.bv) for w in ws])
    bt.set_cores(starts)
    bt.step(2)
    for i, w in enumerate(ws):
        ops = omps.Operators(w.problem)
        f = omps.rk4_step(omps.rk4_step(starts[i], ops), ops)
        st = bt.instance(i)
        G = st.to_dense().cpu().numpy()
        R = omps.to_dense(f, w.problem)
        assert np.abs(G - R).max() <= 1e-8 * np.abs(R).max(), i
        _, E, _ = st.moments()
        Eref = omps.field_dense(f, ops)
        assert np.abs(E.cpu().numpy() - Eref).max() <= 1e-8 * np.abs(Eref).max(), i
        assert st.info()["bonds"][1:-1] == omps.bond_dims(f), i
        assert st.info()["steps"] == 2
    bt.free()


def test_batch_initial_states_and_perturbation(B):
    """Batch initialisation from each instance's profiles equals the
    stand-alone initialisation bit for bit; the batched perturbation
    (alpha_i g_i added and compressed) matches the stand-alone one to
    rounding."""
    _say("batch init + add_scaled")
    ws = _sweep(3, L=6, chi=16)
    bt = B.Batch([w.problem for w in ws], [(w.ax, w.bv) for w in ws])
    solos = [B.MpsState(w.problem, w.ax, w.bv) for w in ws]
    for i, st in enumerate(solos):
        assert np.array_equal(bt.instance(i).to_dense().cpu().numpy(),
                              st.to_dense().cpu().numpy()), i
    perts = [wl.random_mps_cores(ws[0].problem.n_sites, 16, seed=30 + i) for i in range(3)]
    alphas = [1e-3 * (i + 1) for i in range(3)]
    bt.add_scaled(alphas, perts)
    for i, st in enumerate(solos):
        st.add_scaled(alphas[i], perts[i])
        a = bt.instance(i).to_dense().cpu().numpy()
        b = st.to_dense().cpu().numpy()
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max(), i
        assert bt.instance(i).info()["bonds"] == st.info()["bonds"]
        st.free()
    bt.free()


def test_batch_parameter_checks(B):
    _say("batch parameter checks")
    ws = _sweep(2)
    w2 = wl.two_stream(L=4, chi=8, tol=0.0, level=5, df_max=4, dt_cfg=0.05)
    with pytest.raises(B.MpsError) as e:
        B.Batch([ws[0].problem, w2.problem], [(ws[0].ax, ws[0].bv), (w2.ax, w2.bv)])
    assert e.value.status == B.MPS_EINVAL
    ws[1].problem.tol = 1e-10
    with pytest.raises(B.MpsError) as e:
        B.Batch([w.problem for w in ws], [(w.ax, w.bv) for w in ws])
    assert e.value.status == B.MPS_EINVAL
    ws[1].problem.tol = 0.0
    ws[1].problem.tall_apply = 1
    with pytest.raises(B.MpsError) as e:
        B.Batch([w.problem for w in ws], [(w.ax, w.bv) for w in ws])
    assert e.value.status == B.MPS_EINVAL
    ws[1].problem.tall_apply = 0
    ws[1].problem.dt *= 0.5
    with pytest.raises(B.MpsError) as e:
        B.Batch([w.problem for w in ws], [(w.ax, w.bv) for w in ws])
    assert e.value.status == B.MPS_EINVAL
    bt = B.Batch([ws[0].problem], [(ws[0].ax, ws[0].bv)])
    v = bt.instance(0)
    with pytest.raises(B.MpsError):
        v.step(1)
    with pytest.raises(B.MpsError):
        v.set_cores(v.get_cores_host())
    assert B.lib().mps_free(v.handle) != 0
    bt.free()


def test_batch_failure_is_all_or_none(B):
    """A forced non-convergence fails the batched step for every instance:
    none is committed, and the next step succeeds."""
    _say("batch failure")
    ws = _sweep(3)
    starts = [S.oracle_start(w, pert_chi=8, amp=1e-3, seed=40 + i) for i, w in enumerate(ws)]
    bt = B.Batch([w.problem for w in ws], [(w.ax, w.bv) for w in ws])
    bt.set_cores(starts)
    before = [bt.instance(i).get_cores_host() for i in range(3)]
    B.set_jacobi_max_sweeps(1)
    try:
        with pytest.raises(B.MpsError) as e:
            bt.step(1)
        assert e.value.status == B.MPS_ENUMERIC
        # the message names the first failing instance
        assert "instance 0: Jacobi SVD did not converge" in str(e.value)
    finally:
        B.set_jacobi_max_sweeps(60)
    for i in range(3):
        after = bt.instance(i).get_cores_host()
        assert all(np.array_equal(x, y) for x, y in zip(before[i], after)), i
    assert bt.instance(0).info()["steps"] == 0
    bt.step(1)
    assert bt.instance(2).info()["steps"] == 1
    bt.free()
