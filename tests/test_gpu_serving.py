"""Serving loop (continuous batching of solve requests under an HBM budget):
every result is the same alone and in the mix, admission respects the
budget, oversized requests are rejected.  Requests are seeded Landau /
two-stream problems of different sizes."""
import sys

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2205_11990_amd import binding, serving
    binding.lib()
    return serving


def _requests(S, n=8, seed=11990):
    rng = np.random.default_rng(seed)
    arrivals = S.poisson_arrivals(n, rate=200.0, seed=seed)
    reqs = []
    for i in range(n):
        L = int(rng.integers(5, 7))
        chi = int(rng.choice([8, 16]))
        if i % 2 == 0:
            w = wl.landau_small(L=L, chi=chi, tol=1e-10)
            kind = "landau"
        else:
            w = wl.two_stream(L=L, chi=chi, tol=1e-10, level=1, order=0, dt_cfg=0.05)
            kind = "two-stream"
        reqs.append(S.Request(i, w.problem, w.ax, w.bv, steps=int(rng.integers(2, 5)),
                              arrival=float(arrivals[i]), kind=kind))
    return reqs


def test_serving_results_same_alone_and_in_the_mix(S):
    _say("serving mix")
    reqs = _requests(S)
    alone = [S.run_alone(r) for r in reqs]
    mixed = S.Server(budget_bytes=64 << 30, slots=4).run(reqs)
    for a, m in zip(alone, mixed):
        assert a.error is None and m.error is None, (a.error, m.error)
        assert m.bonds == a.bonds
        assert m.scalars == a.scalars  # bitwise: same calls, same arithmetic
    summ = S.summary(mixed)
    assert summ["served"] == len(reqs)
    assert 0 < summ["p50_latency_s"] <= summ["p99_latency_s"]
    # every request waited for its arrival
    assert all(r.admitted >= r.arrival - 1e-3 for r in mixed)


def test_serving_many_overlapping_requests(S):
    """48 small requests through 16 slots: more streams are created than
    torch's stream pool holds (32 per device), so later requests reuse the
    streams of earlier ones, some of them still running.  Every result is
    still the one it has alone (the library keeps no state per stream)."""
    _say("serving 48 requests")
    reqs = _requests(S, n=48, seed=4)
    alone = [S.run_alone(r) for r in reqs]
    mixed = S.Server(budget_bytes=64 << 30, slots=16).run(reqs, realtime=False)
    for a, m in zip(alone, mixed):
        assert a.error is None and m.error is None, (a.error, m.error)
        assert m.bonds == a.bonds
        assert m.scalars == a.scalars
    # the slots really overlapped
    ev = sorted([(r.admitted, 1) for r in mixed] + [(r.finished, -1) for r in mixed])
    live = peak = 0
    for _, d in ev:
        live += d
        peak = max(peak, live)
    assert peak >= 8


def test_serving_budget_limits_concurrency(S):
    _say("serving budget")
    from paper_2205_11990_amd import binding
    reqs = _requests(S, n=5, seed=7)
    budget = max(binding.workspace_bound(r.problem) for r in reqs) + 1
    res = S.Server(budget_bytes=budget, slots=8).run(reqs, realtime=False)
    assert all(r.error is None for r in res)
    # no two requests whose bounds together exceed the budget overlapped
    for a in res:
        for b in res:
            if a.rid < b.rid and a.bound + b.bound > budget:
                assert a.finished <= b.admitted + 1e-3 or b.finished <= a.admitted + 1e-3


def test_serving_rejects_request_above_budget(S):
    _say("serving reject")
    reqs = _requests(S, n=2, seed=3)
    res = S.Server(budget_bytes=1 << 20, slots=2).run(reqs, realtime=False)
    assert all(r.error is not None and "budget" in r.error for r in res)


@pytest.mark.parametrize("case", ["landau_6_chi16", "two_stream_8_chi32_C5",
                                  "two_stream_10_chi64_C5", "sweep_11_chi64",
                                  "two_stream_10_chi64_fp32", "two_stream_12_chi64_df4_C5",
                                  "collisions_10_chi64_C5", "collisions_fixed_9_chi32_seq",
                                  "centre_first_10_chi64", "ig_8_chi32",
                                  "two_stream_14_chi128_df4_C5", "two_stream_10_chi64_C5_wy"])
def test_device_bytes_within_workspace_bound(S, case):
    """The admission bound covers what a state holds after steps from a
    state with every bond at chi_max (random perturbation, no tolerance
    truncation); the arenas keep their high-water mark."""
    _say("device bytes " + case)
    from paper_2205_11990_amd import binding
    if case == "landau_6_chi16":
        w = wl.landau_small(L=6, chi=16, tol=0.0)
    elif case == "two_stream_8_chi32_C5":
        w = wl.two_stream(L=8, chi=32, tol=0.0, level=5)
    elif case == "two_stream_12_chi64_df4_C5":
        w = wl.two_stream(L=12, chi=64, tol=0.0, level=5, df_max=4)
    elif case == "collisions_10_chi64_C5":
        w = wl.two_stream(L=10, chi=64, tol=0.0, level=5, df_max=4)
        w.problem.nu = 0.05
    elif case == "collisions_fixed_9_chi32_seq":
        w = wl.two_stream(L=9, chi=32, tol=0.0, level=5, df_max=4, order=0)
        w.problem.nu, w.problem.coll_model = 0.05, 1
    elif case == "centre_first_10_chi64":
        w = wl.two_stream(L=10, chi=64, tol=0.0, level=5, df_max=4, order=0)
        w.problem.compression = 1
    elif case == "ig_8_chi32":
        w = wl.two_stream(L=8, chi=32, tol=0.0, level=5, df_max=4, order=4)
    elif case == "two_stream_14_chi128_df4_C5":
        w = wl.two_stream(L=14, chi=128, tol=0.0, level=5, df_max=4)
    elif case == "two_stream_10_chi64_C5_wy":
        # compact-WY mode: the panel groups keep a T beside their reflectors
        w = wl.two_stream(L=10, chi=64, tol=0.0, level=5, df_max=4)
        w.problem.tall_apply = 1
    elif case.startswith("two_stream_10"):
        w = wl.two_stream(L=10, chi=64, tol=0.0, level=5)
        if case.endswith("fp32"):
            w.problem.precision = 1
    else:
        # a sweep instance with every compression point capped (level 1
        # with tol = 0 would leave the intermediate bonds uncapped)
        w = [x for x in wl.landau_sweep(64) if x.problem.Lx == 11 and x.problem.chi_max == 64][0]
        w.problem.tol = 0.0
        w.problem.level = 5
    p = w.problem
    st = binding.MpsState(p, w.ax, w.bv)
    try:
        pert = wl.random_mps_cores(p.n_sites, p.chi_max, seed=5)
        st.add_scaled(1e-6 * float(np.linalg.norm(w.ax) * np.linalg.norm(w.bv)), pert)
        st.step(2)
        used = st.device_bytes()
        bound = binding.workspace_bound(p)
        print("bonds %s held %d bytes, bound %d" % (max(st.info()["bonds"]), used, bound),
              flush=True)
        cut = st.info()["bonds"][2:p.n_sites:2] if p.order == 4 else st.info()["bonds"]
        assert max(cut) == p.chi_max
        assert 0 < used <= bound
    finally:
        st.free()


def test_serving_mix_with_bond_cap_128_requests(S):
    """Requests at bond cap 128 (their SVDs of 129..256 columns run on four
    workgroups that meet through global memory) served beside small ones:
    every result bitwise the same as alone, bonds reaching 128."""
    _say("serving mix with chi 128")
    reqs = []
    for i in range(6):
        if i % 3 == 0:
            w = wl.two_stream(L=8, chi=128, tol=0.0, level=5, df_max=4)
            kind = "two-stream chi128"
        else:
            w = wl.landau_small(L=6, chi=16, tol=1e-10)
            kind = "landau"
        reqs.append(S.Request(i, w.problem, w.ax, w.bv, steps=4, arrival=0.01 * i, kind=kind))
    alone = [S.run_alone(r) for r in reqs]
    mixed = S.Server(budget_bytes=64 << 30, slots=6).run(reqs)
    for a, m in zip(alone, mixed):
        assert a.error is None and m.error is None, (a.error, m.error)
        assert m.bonds == a.bonds and m.scalars == a.scalars
    assert max(mixed[0].bonds) == 128
