"""GPU checks of the launch-shape table: every variant a key allows gives
the same bits as the built-in choice (GEMM tiles, reflector columns per
wave, and whole steps of a state and of a lock-step batch under tables that
force every key to each of its values), and recording notes the keys the
launches use."""
import sys

import numpy as np
import pytest

import workloads as wl
from tests import _start as S

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2205_11990_amd import binding
    binding.lib()
    binding.tune_clear()
    yield binding
    binding.tune_record(False)
    binding.tune_clear()


def _recorded(B, fn, knob):
    B.tune_record(True)
    fn()
    recs = B.tune_records()
    B.tune_record(False)
    return [r for r in recs if r["key"][0] == knob]


@pytest.mark.parametrize("M,N,K,at,bt", [(300, 200, 70, False, False),
                                         (128, 128, 16, False, True),
                                         (513, 257, 129, True, False),
                                         (64, 1000, 33, True, True),
                                         (1000, 384, 240, False, False)])
def test_gemm_tiles_give_identical_bits(B, M, N, K, at, bt):
    import torch
    _say("gemm tiles %dx%dx%d at=%s bt=%s" % (M, N, K, at, bt))
    g = torch.Generator().manual_seed(M * 7 + N + K)
    A = torch.randn(K, M, generator=g, dtype=torch.float64).cuda() if at else \
        torch.randn(M, K, generator=g, dtype=torch.float64).cuda()
    Bm = torch.randn(N, K, generator=g, dtype=torch.float64).cuda() if bt else \
        torch.randn(K, N, generator=g, dtype=torch.float64).cuda()
    C0 = torch.randn(M, N, generator=g, dtype=torch.float64).cuda()
    a_str = (1, M, 0) if at else (K, 1, 0)
    b_str = (1, K, 0) if bt else (N, 1, 0)

    def run():
        C = C0.clone()
        B.gemm_strided(M, N, K, 0.75, A, a_str, Bm, b_str, 0.5, C, (N, 1, 0))
        torch.cuda.synchronize()
        return C.cpu().numpy()

    recs = _recorded(B, run, B.TUNE_GEMM_TILE)
    assert len(recs) == 1
    key = recs[0]["key"]
    assert key[1:4] == (M, N, K) and key[4] == 4 + 2 * (0 if at else 1) + (0 if bt else 1)
    assert key[5] == 0 and recs[0]["allowed"] == [0, 1, 2]
    base = run()
    for v in (0, 1, 2):
        B.tune_set(key, v)
        got = run()
        assert np.array_equal(got, base), v
    ref = 0.75 * (A.T if at else A).cpu().numpy() @ (Bm.T if bt else Bm).cpu().numpy() \
        + 0.5 * C0.cpu().numpy()
    assert np.abs(base - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("m,n", [(200, 64), (400, 128), (480, 96), (2000, 16), (3000, 40)])
def test_reflector_columns_give_identical_bits(B, m, n):
    """Shapes whose reflector applications take the tunable kernels (at
    most 512 rows, or more than 16 reflectors, or fewer than 32 columns;
    taller blocks with up to 16 reflectors take the compact-WY kernel,
    which has no variants)."""
    import torch
    _say("apply columns qr %dx%d" % (m, n))
    g = torch.Generator().manual_seed(m + n)
    A = torch.randn(m, n, generator=g, dtype=torch.float64).cuda()

    def run():
        R, Q = B.qr(A)
        torch.cuda.synchronize()
        return R.cpu().numpy(), Q.cpu().numpy()

    recs = _recorded(B, run, B.TUNE_APPLY_COLS)
    assert recs, "no reflector application recorded"
    R0, Q0 = run()
    rounds = max(len(r["allowed"]) for r in recs)
    assert rounds >= 2
    # the reflectors shared through LDS are among the variants from 257 rows
    if m > 256:
        assert any(9 in r["allowed"] for r in recs)
    for j in range(rounds):
        for r in recs:
            a = r["allowed"]
            B.tune_set(r["key"], a[j % len(a)])
        R, Q = run()
        assert np.array_equal(R, R0) and np.array_equal(Q, Q0), j
    assert np.abs(Q0.T @ Q0 - np.eye(n)).max() < 1e-12


def _force_round(B, recs, j):
    for r in recs:
        a = r["allowed"]
        B.tune_set(r["key"], a[j % len(a)])


def test_step_is_identical_under_every_table(B):
    """Two-stream 2^6 x 2^6, chi 16, C5, perturbed to full bonds: one step
    with the built-in rules, then one from the same cores with every key of
    the step forced to its first, second and third allowed value."""
    _say("step under forced tables")
    w = wl.two_stream(L=6, chi=16, tol=0.0, level=5, df_max=4, dt_cfg=0.05)
    f0 = S.oracle_start(w, pert_chi=16, amp=1e-3, seed=5)
    st = S.gpu_state(B, w, f0)
    B.tune_record(True)
    st.step(1)
    recs = B.tune_records()
    B.tune_record(False)
    assert {r["key"][0] for r in recs} == {1, 2}
    base = st.get_cores_host()
    st.free()
    for j in range(3):
        _force_round(B, recs, j)
        st = S.gpu_state(B, w, f0)
        st.step(1)
        got = st.get_cores_host()
        st.free()
        assert [x.shape for x in got] == [x.shape for x in base]
        assert all(np.array_equal(x, y) for x, y in zip(got, base)), j


def test_batch_step_is_identical_under_every_table(B):
    """Three lock-step instances (instance class 1): the same cores after
    one step under the built-in rules and under forced tables."""
    _say("batch step under forced tables")
    ws = []
    for i in range(3):
        w = wl.two_stream(L=5, chi=8, tol=0.0, level=5, df_max=4, dt_cfg=0.05)
        ax, bv = wl.two_stream_profiles(w.problem, 0.2, 1e-3 * (1 + i))
        ws.append(wl.Workload("b%d" % i, w.problem, ax, bv, 1))
    starts = [S.oracle_start(w, pert_chi=8, amp=1e-3, seed=60 + i) for i, w in enumerate(ws)]

    def run():
        bt = B.Batch([w.problem for w in ws], [(w.ax, w.bv) for w in ws])
        bt.set_cores(starts)
        bt.step(1)
        out = [bt.instance(i).get_cores_host() for i in range(3)]
        bt.free()
        return out

    B.tune_record(True)
    base = run()
    recs = B.tune_records()
    B.tune_record(False)
    assert any(r["key"][5] == 1 for r in recs)
    for j in range(3):
        _force_round(B, recs, j)
        got = run()
        for i in range(3):
            assert all(np.array_equal(x, y) for x, y in zip(got[i], base[i])), (j, i)
