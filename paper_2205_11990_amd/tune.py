"""Offline tuner of the launch-shape table (tuning_gfx950.txt).

Two launches of the library have kernel variants that compute the same bits
and differ only in how the work is spread over the device: the output tile
of the FP64 GEMM (64 x 64, 128 x 128 or 128 x 64) and, for a Householder reflector
application, the columns each wave carries (1, 2 or 4) and whether the
reflectors are streamed into each wave's registers or shared by the waves of
a workgroup through LDS (values 9 and 10: 1 or 2 columns per wave; 17 and 18:
the same with the workgroup's block of columns staged through LDS too, read
and written row by row).  Which is fastest
depends on the exact shape and on how many lock-step instances a launch
covers, so the library looks each launch up in a table keyed by both (see
mps_blocks.h, mpsb_tune_*); this script writes that table.

For each workload it steps the state once with recording on to learn the
keys its launches use, then runs rounds of steps in which every key takes
its j-th allowed value (keys are distinct launches, so one step measures all
of them at once), each launch timed with HIP events on its own stream.  A
key's value is the one with the least summed launch time, kept only when it
beats the built-in rule by more than --min-gain and by at least 10 us per
step; otherwise the key gets no entry.  Last, the whole step is timed with
and without the entries found (alternately, best of two each); they go into
the table only when the whole step is faster with them (--min-step-gain).

Usage (on the GPU):
  python -m paper_2205_11990_amd.tune [--workloads two_stream_1024,...]
                                      [--reps 3] [--out PATH]
Workloads: two_stream_1024 (2^10 x 2^10, chi 64, fixed rank), batchN
(N lock-step instances of it, e.g. batch256), two_stream_4096 (2^12 x 2^12,
chi 128), landau_sweep (the 64-instance Landau sweep in its lock-step
groups).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

import workloads as wl  # noqa: E402

from paper_2205_11990_amd import binding as B  # noqa: E402

DEFAULT_OUT = os.path.join(_HERE, "tuning_gfx950.txt")


def _two_stream(L, chi, amp_scale=1.0, seed=2205):
    w = wl.two_stream(L=L, chi=chi, tol=0.0, level=5, df_max=4, dt_cfg=0.02)
    st = B.MpsState(w.problem, w.ax, w.bv)
    cores = wl.random_mps_cores(w.problem.n_sites, chi, seed=seed)
    st.add_scaled(1e-6 * amp_scale * float(np.linalg.norm(w.ax) * np.linalg.norm(w.bv)), cores)
    return st


def _batch(n):
    ws = []
    for i in range(n):
        w = wl.two_stream(L=10, chi=64, tol=0.0, level=5, df_max=4, dt_cfg=0.02)
        w.problem.tall_apply = 1  # the throughput choice for large batches
        ax, bv = wl.two_stream_profiles(w.problem, 0.2, 1e-3 * (1 + 0.1 * i))
        ws.append(wl.Workload("two_stream_%d" % i, w.problem, ax, bv, 10))
    bt = B.Batch([w.problem for w in ws], [(w.ax, w.bv) for w in ws])
    p = ws[0].problem
    perts = [wl.random_mps_cores(p.n_sites, p.chi_max, seed=2205 + i) for i in range(n)]
    amps = [1e-6 * float(np.linalg.norm(w.ax) * np.linalg.norm(w.bv)) for w in ws]
    bt.add_scaled(amps, perts)
    return bt


def _landau_groups(count=64):
    ws = wl.landau_sweep(count)
    for w in ws:
        w.problem.tol, w.problem.level = 0.0, 5
        w.problem.tall_apply = 1
    groups = {}
    for w in ws:
        groups.setdefault((w.problem.Lx, w.problem.chi_max), []).append(w)
    out = []
    for g in groups.values():
        dt = min(w.problem.dt for w in g)
        for w in g:
            w.problem.dt = dt
        out.append(B.Batch([w.problem for w in g], [(w.ax, w.bv) for w in g]))
    return out


def _runners(name):
    """(label, step callable, free callable) for each state of a workload."""
    if name == "two_stream_1024":
        st = _two_stream(10, 64)
        return [("two-stream 2^10 chi 64", st.step, st.free)]
    if name == "two_stream_4096":
        st = _two_stream(12, 128)
        return [("two-stream 2^12 chi 128", st.step, st.free)]
    if name.startswith("batch"):
        n = int(name[5:])
        bt = _batch(n)
        return [("%d x two-stream 2^10 chi 64" % n, bt.step, bt.free)]
    if name == "landau_sweep":
        return [("landau sweep group %d (%d instances)" % (i, b.count), b.step, b.free)
                for i, b in enumerate(_landau_groups())]
    raise ValueError("unknown workload " + name)


def _sync():
    import torch
    torch.cuda.synchronize()


def _measure(step, reps):
    """{key: summed launch ms per step} over reps steps, and the records."""
    tot = {}
    B.tune_record(True)
    for _ in range(reps):
        step(1)
    _sync()
    recs = B.tune_records()
    B.tune_record(False)
    for r in recs:
        tot[r["key"]] = r["ms"] / reps
    return tot, recs


def tune_state(label, step, reps, min_gain, log):
    step(1)  # warm-up: allocations, first-touch
    _sync()
    base, recs = _measure(step, 1)
    keys = {r["key"]: r for r in recs}
    # the built-in value of every key: its recorded value with no entry
    for k in keys:
        B.tune_set(k, -1)
    base, recs = _measure(step, reps)
    default = {r["key"]: r["value"] for r in recs}
    allowed = {r["key"]: r["allowed"] for r in recs}
    trials = {k: {default[k]: base.get(k, 0.0)} for k in default}
    rounds = max(len(a) for a in allowed.values()) if allowed else 0
    for j in range(rounds):
        tried = False
        for k, a in allowed.items():
            alt = [v for v in a if v != default[k]]
            if j < len(alt):
                B.tune_set(k, alt[j])
                tried = True
            else:
                B.tune_set(k, -1)
        if not tried:
            continue
        t, _ = _measure(step, reps)
        for k, a in allowed.items():
            alt = [v for v in a if v != default[k]]
            if j < len(alt) and k in t:
                trials[k][alt[j]] = t[k]
    chosen = {}
    for k, tr in trials.items():
        best = min(tr, key=tr.get)
        d = tr[default[k]]
        # an entry must save a fraction of the key's time and at least
        # 10 us per step (below that the event timings are noise)
        if best != default[k] and tr[best] < (1.0 - min_gain) * d and d - tr[best] >= 0.01:
            chosen[k] = best
    for k in default:
        B.tune_set(k, chosen.get(k, -1))
    gain_ms = sum(trials[k][default[k]] - trials[k][v] for k, v in chosen.items())
    total_ms = sum(base.values())
    log.append({"state": label, "keys": len(default), "entries": len(chosen),
                "tuned_launch_ms_saved_per_step": round(gain_ms, 3),
                "tunable_launch_ms_per_step": round(total_ms, 3)})
    print(json.dumps(log[-1]), flush=True)
    return chosen, default


def _wall(step, n):
    _sync()
    t0 = time.perf_counter()
    step(n)
    _sync()
    return (time.perf_counter() - t0) / n


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", default="two_stream_1024,batch256,two_stream_4096,landau_sweep")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--min-gain", type=float, default=0.03)
    ap.add_argument("--wall-steps", type=int, default=3)
    ap.add_argument("--min-step-gain", type=float, default=0.01,
                    help="a workload's entries are kept only when its whole step gets this much faster")
    ap.add_argument("--out", default=DEFAULT_OUT)
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the tuner times kernels on a GPU"
    B.tune_clear()
    log, walls, table = [], [], {}
    for name in args.workloads.split(","):
        for label, step, free in _runners(name):
            chosen, default = tune_state(label, step, args.reps, args.min_gain, log)
            # whole-step wall time: built-in rules against the table found,
            # measured alternately, the best of two each; the entries are
            # kept only when the whole step is faster with them
            t_def, t_tun = [], []
            for _ in range(2):
                for k in default:
                    B.tune_set(k, -1)
                t_def.append(_wall(step, args.wall_steps))
                for k, v in chosen.items():
                    B.tune_set(k, v)
                t_tun.append(_wall(step, args.wall_steps))
            t_def, t_tun = min(t_def), min(t_tun)
            kept = t_tun < (1.0 - args.min_step_gain) * t_def
            if kept:
                table.update(chosen)
            for k in default:
                B.tune_set(k, -1)
            walls.append({"state": label, "ms_per_step_builtin": round(1e3 * t_def, 2),
                          "ms_per_step_tuned": round(1e3 * t_tun, 2), "kept": kept})
            print(json.dumps(walls[-1]), flush=True)
            free()
            _sync()
            torch.cuda.empty_cache()
    B.tune_clear()
    for k, v in table.items():
        B.tune_set(k, v)
    tmp = args.out + ".tmp"
    B.tune_save(tmp)
    body = open(tmp).read()
    os.remove(tmp)
    with open(args.out, "w") as f:
        f.write("# Launch-shape table of libmpsvlasov for gfx950, written by\n")
        f.write("# paper_2205_11990_amd/tune.py (--workloads %s --reps %d --min-gain %g).\n"
                % (args.workloads, args.reps, args.min_gain))
        f.write("# knob 1: FP64 GEMM tile (0: 64x64, 1: 128x128, 2: 128x64), key M N K 4*batch+layout;\n")
        f.write("# knob 2: reflector application (1, 2, 4 columns per wave; 9, 10: LDS-shared with 1, 2;\n")
        f.write("#         17, 18: LDS-shared with the columns staged),\n")
        f.write("#         key rows reflectors columns 2*chunks+trans;\n")
        f.write("# class: lock-step instances (0: 1, 1: 2-7, 2: 8-31, 3: 32+).\n")
        for w in walls:
            f.write("# %s: %.2f ms/step with the built-in rules, %.2f with its entries (%s)\n"
                    % (w["state"], w["ms_per_step_builtin"], w["ms_per_step_tuned"],
                       "kept" if w["kept"] else "not kept: under the step-gain threshold"))
        f.write(body)
    print(json.dumps({"entries": len(table), "out": args.out, "walls": walls}), flush=True)


if __name__ == "__main__":
    main()
