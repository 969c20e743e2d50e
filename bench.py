"""Benchmark of the MPS Vlasov-Poisson RK4 step on one MI355X.

Workload (the metric's configuration): two-stream instability on a
2^10 x 2^10 grid (x in [0, 10 pi) periodic, v in [-8, 8]), interleaved site
order (20 sites), bond cap chi = 64, FP64.  A step is one full RK4 step of
the MPS method: per stage the charge density and Poisson field, the two
MPO x MPS terms, their sum and the stage state, each recompressed by a QR
left sweep and a truncated SVD right sweep; then the sum of the k's and the
final state.

Two modes:
  fixed   (default, the reported `value`): every compression point capped at
          chi (level C5), tol = 0, field bond D_F = 4, initial state
          f0 + 1e-6 |f0| R with R a seeded random MPS of bond 64, so every
          bond runs at the full chi = 64 shape.
  physics: tol = 1e-10, level C1, from f0 (bonds follow the physics).

Beside the metric line, three measurements of the same JSON object
(skipped with --no-extras):
  mixed    the same workload with the MPO x MPS contractions in FP32 and
           in BF16 on the matrix cores (FP32 accumulation; QR, SVD, Poisson
           and moments in FP64): steps/s and the one-step error of f, E and
           the field energy against an FP64 step from the same state.
  physics  the same grid in the paper's default compression (C1, tol 1e-10,
           from f0): steps/s, bonds, truncated SVDs (host round trips) per step.
  chi128   bond cap 128 on a 2^12 x 2^12 two-stream grid (fixed-chi mode):
           FP64 steps/s and the same mixed-precision comparison.
  batched_metric  the metric's workload as one lock-step batch of 256
           instances (--batch; mps_batch_*: every launch covers all of them):
           aggregate steps/s against the single instance, the rate of the
           dominant kernel class, and the aggregate rate at 64 and 128.
  batched  64 Landau instances of a parameter sweep (k, alpha, 2^8..2^11
           grids, chi in {16, 32, 48, 64}, fixed rank), one lock-step batch
           per (grid, chi) shape: aggregate steps/s against stepping them one
           after the other and against one stream per instance.
  The batched legs apply the reflectors of tall blocks as compact-WY blocks
  on the matrix cores (mps_problem.tall_apply = 1, the throughput choice);
  the single-instance metric applies them one at a time (the default).
  tuning   the launch-shape table in use (tune.py; its variants give the
           same bits, so it changes speed only) and its entry count.
  serving  seeded Poisson arrivals (mean 20 requests/s) of Landau and
           two-stream solve requests (grids 2^8..2^10, chi in {32, 64},
           FP32 contraction, tol 1e-6 with every compression capped at chi),
           admitted by device-memory bound against a budget: p50/p99
           latency and aggregate steps/s.

Usage: python bench.py [--steps K] [--warmup W] [--mode fixed|physics]
Prints one JSON line.  Runs on one GPU only (--gpus must be 1).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# The batched-sweep and serving legs keep many streams busy at once (two per
# lock-step batch or request); with four hardware queues per process (HIP's
# default) their kernels queue behind each other.  Sixteen queues, set here
# before the runtime starts, let them overlap: the 64-instance sweep runs at
# 8.4x its sequential rate against 5.9x with four.
os.environ["GPU_MAX_HW_QUEUES"] = "16"

import numpy as np  # noqa: E402

import workloads as wl  # noqa: E402

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (matrix and vector)
MI355X_CUS = 256
PEAK_HBM_GBS = 8000.0


def make_workload(mode: str):
    if mode == "fixed":
        w = wl.two_stream(L=10, chi=64, tol=0.0, level=5, df_max=4, dt_cfg=0.02)
    else:
        w = wl.two_stream(L=10, chi=64, tol=1e-10, level=1, df_max=0, dt_cfg=0.02)
    return w


def perturbation(w):
    p = w.problem
    cores = wl.random_mps_cores(p.n_sites, p.chi_max, seed=2205)
    amp = 1e-6 * float(np.linalg.norm(w.ax) * np.linalg.norm(w.bv))
    return amp, cores


def start_state(binding, w, mode):
    st = binding.MpsState(w.problem, w.ax, w.bv)
    if mode == "fixed":
        amp, cores = perturbation(w)
        st.add_scaled(amp, cores)
    return st


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [d.get("num_threads", 0) for d in threadpool_info() if d.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)


def oracle_start(w, mode):
    """The workload's start state built by the oracle (the profile's product
    MPS compressed to the problem's cap, plus the seeded perturbation in
    fixed mode): host cores, handed to the GPU by mps_set_cores."""
    from oracle import mps as omps
    p = w.problem
    f = omps.chain_product_mps(omps.vector_mps(w.ax[0]), omps.vector_mps(w.bv[0]),
                               p.Lx, p.Lv, p.order)
    f = omps.compress_state(f, p.chi_max, p)
    if mode == "fixed":
        amp, cores = perturbation(w)
        f = omps.compress_state(omps.add([(1.0, f), (amp, cores)]), p.chi_max, p)
    return f


def cpu_baseline(w, mode):
    """The CPU MPS oracle, as it stands, timed on a bounded sample: one RK4
    step of the same workload from its start state.  Also returns that start
    state and the oracle's step from it (f on the grid, E), which the
    precision leg compares the GPU's one-step results against."""
    from oracle import mps as omps
    f0 = oracle_start(w, mode)
    ops = omps.Operators(w.problem)
    t0 = time.perf_counter()
    f1 = omps.rk4_step(f0, ops)
    dt = time.perf_counter() - t0
    ref = {"f": omps.to_dense(f1, w.problem), "E": omps.field_dense(f1, ops),
           "field_energy": omps.moments(f1, ops)["field_energy"]}
    return ({"value": 1.0 / dt, "unit": "steps/s", "cores": _blas_threads(), "kind": "oracle",
             "sample": "1 RK4 step of the same workload from its start state "
                       "(%.1f s of CPU time)" % dt}, f0, ref)


# Peak of the unit each kernel class runs on (MI355X, dense FP64).
_CLASS_BOUND = {
    "gemm_f64": ("mfma", PEAK_FP64_TFLOPS),     # v_mfma_f64_16x16x4f64
    "qr_factor": ("alu", PEAK_FP64_TFLOPS),     # FP64 vector FMA
    "qr_apply": ("alu", PEAK_FP64_TFLOPS),      # FP64 vector FMA
    "qr_wy": ("hbm", PEAK_HBM_GBS),             # compact-WY streams of Y
    "jacobi_svd": ("alu", PEAK_FP64_TFLOPS),    # FP64 vector FMA
}


# rocprofv3 FETCH_SIZE / WRITE_SIZE summaries of the kernels (committed under
# profiles/), valid while the kernel sources they were taken on are unchanged
_TRAFFIC = {
    "jacobi_svd": ("profiles/jacobi_svd_hbm_traffic_two_stream_1024_chi64.txt",
                   ("paper_2205_11990_amd/csrc/jacobi.hip", "paper_2205_11990_amd/csrc/wave.hpp")),
}


def _rate(r, bound):
    """A class's rate: algorithmic bytes over summed launch time (GB/s) for
    an HBM-bound class, nominal FLOPs over it (TFLOP/s) otherwise."""
    if r["ms"] <= 0:
        return 0.0, "GB/s" if bound == "hbm" else "TFLOP/s"
    if bound == "hbm":
        return r["bytes"] / (r["ms"] * 1e-3) / 1e9, "GB/s"
    return r["flops"] / (r["ms"] * 1e-3) / 1e12, "TFLOP/s"


def _class_entry(v):
    e = {"launches": v["launches"], "ms": round(v["ms"], 3),
         "tflops": round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 4) if v["ms"] > 0 else None}
    if v["ms"] > 0 and v.get("bytes"):
        e["gbps"] = round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1)
    return e


def measured_traffic(cls):
    """HBM bytes per launch from the committed counter summary, or None when
    there is none or the kernel changed since the counters were taken."""
    import hashlib
    if cls not in _TRAFFIC:
        return None
    summary, sources = _TRAFFIC[cls]
    try:
        text = open(os.path.join(ROOT, summary)).read()
        h = hashlib.sha256()
        for f in sources:
            h.update(open(os.path.join(ROOT, f), "rb").read())
    except OSError:
        return None
    vals = dict(l.split(":", 1) for l in text.splitlines() if ":" in l and not l.startswith("#"))
    try:
        if vals["source_sha256"].split()[0] != h.hexdigest():
            return None
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError, IndexError):
        return None


def roofline(binding, st, cores_host, steps, jacobi_cols):
    """Re-run `steps` steps from the same state with every launch of the
    instrumented kernels bracketed by HIP events on the launching stream;
    report the class with the largest event time.  achieved = nominal FLOPs
    of its launches / summed launch time."""
    import torch
    st.set_cores(cores_host)
    torch.cuda.synchronize()
    binding.profile(True)
    st.step(steps)
    torch.cuda.synchronize()
    rec = binding.profile_read()
    binding.profile(False)
    dom = max(_CLASS_BOUND, key=lambda k: rec[k]["ms"])
    r = rec[dom]
    bound, peak = _CLASS_BOUND[dom]
    ach, unit = _rate(r, bound)
    classes = {k: _class_entry(v) for k, v in rec.items() if k in _CLASS_BOUND}
    # the whole step: nominal FLOPs of every instrumented launch per step
    # (GEMM 2mnk, GEQRF, reflector applications, SVD 6mn^2 + 20n^3), the
    # launches inside an SVD counted once, in its nominal work
    step_gflop = sum(v["flops"] - v["nested_flops"] for k, v in rec.items()
                     if k in _CLASS_BOUND) / steps / 1e9
    out = {"bound": bound, "achieved": ach, "peak": peak, "unit": unit,
           "frac": ach / peak, "traffic": measured_traffic(dom), "kernel": dom,
           "launches": r["launches"], "avg_launch_us": 1000.0 * r["ms"] / max(r["launches"], 1),
           "flops_per_launch": r["flops"] / max(r["launches"], 1),
           "classes": classes, "step_gflop": step_gflop}
    if dom == "jacobi_svd":
        # a Jacobi SVD of up to 128 columns runs as one workgroup (one CU),
        # of up to 256 as four: its rate against the peak of the CUs it holds
        wgs = 1 if jacobi_cols <= 128 else 4
        out["workgroups_per_launch"] = wgs
        out["frac_of_its_cus"] = ach / (peak * wgs / MI355X_CUS)
    return out


_PREC_NAMES = {1: "fp32 contraction (MFMA f32, FP32 accumulate)",
               2: "bf16 contraction (MFMA bf16, FP32 accumulate)"}


def _one_step(binding, problem, w, cores_host, precision):
    import copy
    p = copy.copy(problem)
    p.precision = precision
    st = binding.MpsState(p, w.ax, w.bv)
    st.set_cores(cores_host)
    st.step(1)
    f = st.to_dense().cpu().numpy()
    _, E, sc = st.moments()
    E = E.cpu().numpy()
    return st, p, f, E, sc


def mixed_precision(binding, w, cores_host, steps, fp64_steps_per_s=None, oracle=None):
    """Reduced-precision contraction modes on a workload: steps/s from the
    same state, and the error of one step against an FP64 step from it
    (QR/SVD/Poisson/moments FP64 in every mode).  With `oracle` (the CPU MPS
    oracle's step from the same state: f, E, field energy) every mode's
    one-step error against the oracle is reported as well."""
    import torch
    ref, _, f64, E64, sc64 = _one_step(binding, w.problem, w, cores_host, 0)
    out = {}
    if oracle is not None:
        out["reference"] = "CPU MPS oracle (FP64), one RK4 step from the same state"
        out["fp64"] = _errors(f64, E64, sc64, oracle)
    if fp64_steps_per_s is None:
        ref.set_cores(cores_host)
        ref.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ref.step(steps)
        torch.cuda.synchronize()
        fp64_steps_per_s = steps / (time.perf_counter() - t0)
    out["fp64_steps_per_s"] = fp64_steps_per_s
    ref.free()
    for prec in (1, 2):
        st, _, f, E, sc = _one_step(binding, w.problem, w, cores_host, prec)
        st.set_cores(cores_host)
        st.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st.free()
        out[{1: "fp32", 2: "bf16"}[prec]] = {
            "precision": _PREC_NAMES[prec] + "; QR/SVD/Poisson/moments FP64",
            "steps_per_s": steps / el, "steps": steps,
            "speedup_vs_fp64": (steps / el) / fp64_steps_per_s,
            "f_max_rel_err_one_step": float(np.abs(f - f64).max() / np.abs(f64).max()),
            "E_max_rel_err_one_step": float(np.abs(E - E64).max() / np.abs(E64).max()),
            "field_energy_rel_err_one_step": float(abs(sc["field_energy"] - sc64["field_energy"])
                                                   / abs(sc64["field_energy"]))}
        if oracle is not None:
            out[{1: "fp32", 2: "bf16"}[prec]]["vs_oracle"] = _errors(f, E, sc, oracle)
    return out


def _errors(f, E, sc, ref):
    return {"f_max_rel_err_one_step": float(np.abs(f - ref["f"]).max() / np.abs(ref["f"]).max()),
            "E_max_rel_err_one_step": float(np.abs(E - ref["E"]).max() / np.abs(ref["E"]).max()),
            "field_energy_rel_err_one_step": float(abs(sc["field_energy"] - ref["field_energy"])
                                                   / abs(ref["field_energy"]))}


def chi128_run(binding, steps, with_oracle=True):
    """The bond cap 128 workload: two-stream 2^12 x 2^12, interleaved,
    every point capped at 128, D_F = 4, tol = 0, seeded perturbation to
    bond 128, started from the oracle's state; FP64 steps/s and the
    reduced-precision modes against it and (with_oracle) against the CPU
    MPS oracle's step from the same state (about a minute of host time)."""
    import torch
    w = wl.two_stream(L=12, chi=128, tol=0.0, level=5, df_max=4, dt_cfg=0.02)
    f0 = oracle_start(w, "fixed")
    ref = None
    if with_oracle:
        from oracle import mps as omps
        ops = omps.Operators(w.problem)
        t0 = time.perf_counter()
        f1 = omps.rk4_step(f0, ops)
        t_or = time.perf_counter() - t0
        ref = {"f": omps.to_dense(f1, w.problem), "E": omps.field_dense(f1, ops),
               "field_energy": omps.moments(f1, ops)["field_energy"]}
    st = binding.MpsState(w.problem, w.ax, w.bv)
    st.set_cores(f0)
    st.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.step(steps)
    torch.cuda.synchronize()
    v = steps / (time.perf_counter() - t0)
    # the kernel classes of one more step (the contraction GEMMs' rate at
    # bond cap 128 among them), and the largest GEMM shapes of a step with
    # their own rates (launch times from the launch-shape records)
    rates = _class_rates(binding, lambda: st.step(1), 1)
    torch.cuda.synchronize()
    binding.tune_record(True)
    st.step(1)
    recs = binding.tune_records()
    binding.tune_record(False)
    gemms = []
    for r in recs:
        k = r["key"]
        if k[0] != binding.TUNE_GEMM_TILE or r["ms"] <= 0:
            continue
        fl = 2.0 * k[1] * k[2] * k[3] * (k[4] // 4) * r["launches"]
        gemms.append({"M": k[1], "N": k[2], "K": k[3], "batch": k[4] // 4,
                      "tile": {0: "64x64", 1: "128x128", 2: "128x64"}[r["value"]], "launches": r["launches"],
                      "ms": round(r["ms"], 3), "tflops": round(fl / (r["ms"] * 1e-3) / 1e12, 2),
                      "frac_fp64_peak": round(fl / (r["ms"] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 3)})
    gemms.sort(key=lambda g: -g["ms"])
    st.free()
    out = {"workload": "two-stream 2^12 x 2^12, interleaved (24 sites), chi=128, C5, tol=0, "
                       "D_F=4, seeded random-MPS perturbation (start state built by the oracle)",
           "dt": w.problem.dt, "classes": rates["classes"], "largest_gemms": gemms[:4]}
    if ref is not None:
        out["oracle_s_per_step"] = t_or
    out.update(mixed_precision(binding, w, f0, steps, fp64_steps_per_s=v, oracle=ref))
    return out


def physics_run(binding, steps):
    """The metric's grid in the paper's default compression (C1: only the
    final state capped at chi = 64, every point truncated at tol = 1e-10,
    uncapped field) from f0: steps/s, the bonds reached, and the truncated
    SVDs per step, each of which returns its rank to the host (one stream
    synchronisation each: later launches are sized by it)."""
    import torch
    w = make_workload("physics")
    st = start_state(binding, w, "physics")
    st.step(1)
    torch.cuda.synchronize()
    s0 = binding.stats()["svd_calls"]
    t0 = time.perf_counter()
    st.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    svds = (binding.stats()["svd_calls"] - s0) / steps
    bonds = st.info()["bonds"]
    st.free()
    return {"workload": "two-stream 2^10 x 2^10, interleaved, C1, tol=1e-10, chi=64 at P1, "
                        "D_F uncapped, from f0 (steps 2..%d)" % (steps + 1),
            "steps_per_s": steps / el, "ms_per_step": 1000.0 * el / steps,
            "truncated_svds_per_step": svds, "max_bond": int(max(bonds)), "bonds": bonds}


def orderings(binding, steps):
    """The fixed-chi workload in the sequential orderings S1, S2, S3 and the
    grouped interleaved IG (Fig. 3; the default is IF), and with centre-first
    compression (SI, Modified Compression Scheme):
    steps/s from a perturbed state, the x|v cut's entanglement entropy and
    the largest bond after the timed steps."""
    import torch
    out = {}
    for name, order, comp in (("S1", 0, 0), ("S2", 2, 0), ("S3", 3, 0), ("IG", 4, 0),
                              ("S1_centre_first", 0, 1), ("S2_centre_first", 2, 1)):
        w = make_workload("fixed")
        p = w.problem
        p.order, p.compression = order, comp
        st = start_state(binding, w, "fixed")
        st.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ee = st.entanglement()
        out[name] = {"steps_per_s": steps / el, "steps": steps,
                     "ee_xv_cut": float(ee[p.Lx - 1]) if order != 4 else None,
                     "max_bond": int(max(st.info()["bonds"]))}
        st.free()
    return out


def buneman_run(binding, steps):
    """Electrons and ions (Buneman instability, 2^9 x 2^9 per species, S1,
    every point capped at chi = 64, D_F = 4, tol = 0), collisionless and
    with Dougherty collisions (nu = 0.01): plasma steps/s of both species
    with the shared field, from states perturbed to full bonds, and the
    field energy after the timed steps."""
    import torch
    out = {}
    for name, nu in (("collisionless", 0.0), ("collisions_nu_0.01", 0.01)):
        ws, q = wl.buneman(L=9, chi=64, tol=0.0, level=5, df_max=4, nu=nu)
        ps = [w.problem for w in ws]
        pl = binding.Plasma(ps, q, [(w.ax, w.bv) for w in ws])
        for s_, (w, p) in enumerate(zip(ws, ps)):
            amp = 1e-6 * float(np.linalg.norm(w.ax) * np.linalg.norm(w.bv))
            pl.species(s_).add_scaled(amp, wl.random_mps_cores(p.n_sites, 64, seed=2205 + s_))
        pl.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pl.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        _, W = pl.field()
        out[name] = {"steps_per_s": steps / el, "steps": steps, "dt": ps[0].dt,
                     "field_energy": W,
                     "max_bond": [int(max(pl.species(i).info()["bonds"])) for i in range(2)]}
        pl.free()
    out["workload"] = ("Buneman: electrons drifting at 1/k = 10 (v in +-60) and ions at rest "
                       "(m_i/m_e = 25, v in +-50 vth_i), k = 0.1, A = 1e-3, 2^9 x 2^9 each, "
                       "S1, chi = 64, C5, D_F = 4, tol = 0, seeded perturbation to full bonds")
    return out


def _class_rates(binding, run, steps):
    """Per-class launch records of `steps` steps run by run() with HIP
    events on the launching streams: the dominant class's rate and all
    classes' (nominal FLOPs over summed launch time)."""
    import torch
    torch.cuda.synchronize()
    binding.profile(True)
    run()
    torch.cuda.synchronize()
    rec = binding.profile_read()
    binding.profile(False)
    dom = max(_CLASS_BOUND, key=lambda k: rec[k]["ms"])
    r = rec[dom]
    bound, peak = _CLASS_BOUND[dom]
    ach, unit = _rate(r, bound)
    classes = {k: _class_entry(v) for k, v in rec.items() if k in _CLASS_BOUND}
    return {"bound": bound, "achieved": ach, "peak": peak, "unit": unit,
            "frac": ach / peak, "kernel": dom, "launches": r["launches"],
            "avg_launch_us": 1000.0 * r["ms"] / max(r["launches"], 1),
            "classes": classes,
            "step_gflop": sum(v["flops"] - v["nested_flops"] for k, v in rec.items()
                              if k in _CLASS_BOUND) / steps / 1e9}


def metric_sweep(count, tall_apply=1):
    """`count` instances of the metric's workload (two-stream 2^10 x 2^10,
    interleaved, chi = 64, fixed-chi mode) with amplitudes
    alpha = 1e-3 (1 + i/10) and the seeded perturbation of seed 2205 + i;
    tall blocks apply their reflectors as compact-WY blocks on the matrix
    cores (tall_apply = 1, the throughput choice for large batches)."""
    ws = []
    for i in range(count):
        w = make_workload("fixed")
        w.problem.tall_apply = tall_apply
        ax, bv = wl.two_stream_profiles(w.problem, 0.2, 1e-3 * (1 + 0.1 * i))
        ws.append(wl.Workload("two_stream_%d" % i, w.problem, ax, bv, 10))
    return ws


def graph_run(binding, w, cores, steps, eager_steps_per_s):
    """The metric's workload with captured step graphs: the first step from
    the state runs eagerly, the second is recorded and replayed, the timed
    ones replay."""
    import torch
    st = binding.MpsState(w.problem, w.ax, w.bv)
    st.set_cores(cores)
    st.step_graph(True)
    st.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    caps, reps = st.step_graph()
    st.free()
    return {"steps_per_s": steps / el, "ms_per_step": 1000.0 * el / steps,
            "speedup_vs_eager": (steps / el) / eager_steps_per_s,
            "captures": caps, "replays": reps}


def _metric_batch(binding, count, tall_apply=1, precision=0):
    ws = metric_sweep(count, tall_apply)
    for w in ws:
        w.problem.precision = precision
    p = ws[0].problem
    bt = binding.Batch([w.problem for w in ws], [(w.ax, w.bv) for w in ws])
    perts = [wl.random_mps_cores(p.n_sites, p.chi_max, seed=2205 + i) for i in range(count)]
    amps = [1e-6 * float(np.linalg.norm(w.ax) * np.linalg.norm(w.bv)) for w in ws]
    bt.add_scaled(amps, perts)
    return bt


def _batch_rate(binding, bt, count, steps):
    import torch
    bt.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return count * steps / el, el / steps


def batched_metric(binding, count, steps, single_steps_per_s, smaller=(64, 128), extras=True):
    """The metric's workload as a lock-step batch of `count` instances: every
    kernel launch covers all of them.  Aggregate steps/s (count x steps over
    the timed window) against the single instance's, the rate of the
    dominant kernel class over the instances of its launches, and the
    aggregate rate of smaller batches (2 timed steps each)."""
    scaling = {}
    for n in smaller:
        if n >= count:
            continue
        bt = _metric_batch(binding, n)
        scaling[str(n)] = round(_batch_rate(binding, bt, n, 2)[0], 2)
        bt.free()
    bt = _metric_batch(binding, count)
    agg, sec = _batch_rate(binding, bt, count, steps)
    scaling[str(count)] = round(agg, 2)
    roof = _class_rates(binding, lambda: bt.step(1), 1)
    roof["workgroups_per_launch_jacobi"] = count
    import torch
    dev_bytes = bt.instance(0).device_bytes()
    if not extras:
        bt.free()
        return {"workload": "%d lock-step instances of two-stream 2^10 x 2^10, interleaved, "
                            "chi=64, C5, tol=0, D_F=4, compact-WY reflector application on tall "
                            "blocks" % count,
                "instances": count, "steps_each": steps, "ms_per_batched_step": 1000.0 * sec,
                "aggregate_steps_per_s": agg, "aggregate_steps_per_s_by_instances": scaling,
                "device_bytes": dev_bytes, "roofline": roof}
    # the same batched steps replayed from a captured graph (an ordinary
    # step from the layout, the capture, then the timed replays)
    bt.step_graph(True)
    bt.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.step(steps)
    torch.cuda.synchronize()
    gsec = (time.perf_counter() - t0) / steps
    caps, reps = bt.step_graph()
    graph = {"ms_per_batched_step": 1000.0 * gsec, "aggregate_steps_per_s": count / gsec,
             "speedup_vs_eager": sec / gsec, "captures": caps, "replays": reps}
    bt.free()
    torch.cuda.synchronize()
    # the batch with FP32 / BF16 contractions (QR, SVD, Poisson and moments
    # FP64; their one-step errors are those of the single state, leg `mixed`),
    # one batch on the device at a time
    mixed = {}
    for name, prec in (("fp32", 1), ("bf16", 2)):
        bm = _metric_batch(binding, count, precision=prec)
        a, _ = _batch_rate(binding, bm, count, 2)
        bm.free()
        mixed[name] = {"aggregate_steps_per_s": a, "speedup_vs_fp64": a / agg}
    out = {"workload": "%d lock-step instances of two-stream 2^10 x 2^10, interleaved, chi=64, "
                       "C5, tol=0, D_F=4 (amplitudes 1e-3 (1 + i/10), seeded perturbations), "
                       "compact-WY reflector application on tall blocks" % count,
           "instances": count, "steps_each": steps, "ms_per_batched_step": 1000.0 * sec,
           "aggregate_steps_per_s": agg,
           "speedup_vs_single_instance": agg / single_steps_per_s if single_steps_per_s else None,
           "aggregate_steps_per_s_by_instances": scaling,
           "device_bytes": dev_bytes, "roofline": roof, "graph": graph,
           "contraction_precision": mixed}
    return out


def batched_sweep(binding, count, steps):
    """The 64-instance Landau parameter sweep (k, alpha, grids 2^8..2^11,
    chi in {16, 32, 48, 64}, seeded) in fixed-rank mode (tol = 0, every
    point capped): instances of one (grid, chi) shape form a lock-step
    batch with one dt (the smallest stable one of its members); aggregate
    steps/s of the batches against the same instances stepped one after
    the other, and against one stream per instance (mps_step_batched).
    Every instance applies the reflectors of tall blocks as compact-WY
    blocks (tall_apply = 1) in all three runs."""
    import torch
    ws = wl.landau_sweep(count)
    for w in ws:
        w.problem.tol, w.problem.level = 0.0, 5
        w.problem.tall_apply = 1  # the throughput choice (also for the sequential runs)
    groups = {}
    for w in ws:
        groups.setdefault((w.problem.Lx, w.problem.chi_max), []).append(w)
    for g in groups.values():
        dt = min(w.problem.dt for w in g)
        for w in g:
            w.problem.dt = dt
    batches = [binding.Batch([w.problem for w in g], [(w.ax, w.bv) for w in g])
               for g in groups.values()]
    for b in batches:
        b.step(1)
    torch.cuda.synchronize()
    # the batches of different shapes side by side: one host thread and
    # stream each
    import threading
    streams = [torch.cuda.Stream() for _ in batches]

    def run(b, st):
        with torch.cuda.stream(st):
            b.step(steps)

    t0 = time.perf_counter()
    th = [threading.Thread(target=run, args=(b, st)) for b, st in zip(batches, streams)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    for b in batches:
        b.free()
    states = [binding.MpsState(x.problem, x.ax, x.bv) for x in ws]
    for st in states:
        st.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for st in states:
        st.step(steps)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    binding.step_batched(states, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    binding.step_batched(states, steps)
    torch.cuda.synchronize()
    tt = time.perf_counter() - t0
    for st in states:
        st.free()
    return {"instances": count, "steps_each": steps, "grids": "2^8..2^11",
            "chi": "16, 32, 48, 64", "mode": "fixed rank (C5, tol=0)",
            "lockstep_batches": len(groups),
            "aggregate_steps_per_s": count * steps / tb,
            "sequential_steps_per_s": count * steps / ts,
            "streams_steps_per_s": count * steps / tt,
            "speedup_vs_sequential": ts / tb, "speedup_vs_streams": tt / tb}


def serving_run(binding, n_req, steps, seed=11990):
    """A bounded subset of the serving workload: seeded Poisson arrivals at a
    mean 20 requests/s, half Landau (S1) and half two-stream (IF) solves,
    grids 2^L x 2^L with L ~ U{8..14}, bond caps chi ~ U{32, 64, 128}, FP32
    contraction, every compression capped (C5) with tol = 1e-6 and D_F = 4,
    dt per the stability rule; n_req requests of `steps` steps each (the
    full set is 600 requests of 300 steps).  Admission by the device-memory
    bound against a 128 GiB budget, 16 slots."""
    from paper_2205_11990_amd import serving
    rng = np.random.default_rng(seed)
    arrivals = serving.poisson_arrivals(n_req, rate=20.0, seed=seed)
    reqs = []
    for i in range(n_req):
        L = int(rng.integers(8, 15))
        chi = int(rng.choice([32, 64, 128]))
        # FP32 contractions leave rounding noise near 1e-7 of the largest
        # singular value: the truncation tolerance sits above it and every
        # compression point is capped at chi
        if rng.random() < 0.5:
            x = wl.landau_small(L=L, chi=chi, tol=1e-6, level=5)
            x.problem.dt = wl.stable_dt(x.problem, 0.05)
            kind = "landau"
        else:
            x = wl.two_stream(L=L, chi=chi, tol=1e-6, level=5)
            kind = "two-stream"
        x.problem.precision = 1
        x.problem.df_max = 4
        reqs.append(serving.Request(i, x.problem, x.ax, x.bv, steps, float(arrivals[i]),
                                    "%s 2^%d chi %d" % (kind, L, chi)))
    budget = 128 << 30

    def done(r):
        print("[bench] serving request %d (%s) %s latency %.3f s" % (
            r.rid, r.kind, "ok" if r.error is None else r.error, r.latency),
            file=sys.stderr, flush=True)

    res = serving.Server(budget_bytes=budget, slots=16).run(reqs, on_done=done)
    out = serving.summary(res)
    out.update({"subset": "%d of the 600 requests, %d of the 300 steps each" % (n_req, steps),
                "arrival_rate_per_s": 20.0, "steps_each": steps, "grids": "2^8..2^14",
                "chi": "32, 64, 128", "precision": "fp32 contraction",
                "compression": "every point capped at chi (C5), tol=1e-6, D_F=4",
                "hbm_budget_bytes": budget,
                "max_request_bound_bytes": int(max(r.bound for r in res)),
                "largest_request": max((r.kind for r in res),
                                       key=lambda k: (int(k.split("2^")[1].split()[0]),
                                                      int(k.split("chi ")[1])))})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="fixed", choices=["fixed", "physics"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=256,
                    help="instances of the lock-step batch of the metric's workload")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the mixed-precision, batched, serving and chi=128 measurements")
    ap.add_argument("--chi128-only", action="store_true",
                    help="only time FP64 steps of the chi=128 2^12 configuration (for profiling)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only time the lock-step batch of --batch instances of the metric's "
                         "workload (for profiling)")
    ap.add_argument("--serving-only", action="store_true",
                    help="only run the serving workload: --serving-requests of its seeded "
                         "arrivals, --serving-steps steps each")
    ap.add_argument("--serving-requests", type=int, default=40)
    ap.add_argument("--serving-steps", type=int, default=20)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = (256 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the MPS step of one instance is "
              "not split across devices (independent instances would be placed "
              "one per GPU); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2205_11990_amd import binding
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    binding.lib()

    if args.chi128_only:
        w = wl.two_stream(L=12, chi=128, tol=0.0, level=5, df_max=4, dt_cfg=0.02)
        st = start_state(binding, w, "fixed")
        st.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.step(args.steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(json.dumps({"workload": "two-stream 2^12 x 2^12, interleaved, chi=128, C5, tol=0, D_F=4",
                          "steps": args.steps, "steps_per_s": args.steps / el,
                          "ms_per_step": 1000.0 * el / args.steps}))
        return

    if args.batched_only:
        print(json.dumps(batched_metric(binding, args.batch, args.steps, None, smaller=(),
                                        extras=False)))
        return

    if args.serving_only:
        print(json.dumps(serving_run(binding, args.serving_requests, args.serving_steps)))
        return

    w = make_workload(args.mode)
    p = w.problem
    st = start_state(binding, w, args.mode)
    print("[bench] %s mode: %d sites, chi=%d, dt=%.6g, bonds=%s" % (
        args.mode, p.n_sites, p.chi_max, p.dt, st.info()["bonds"]), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    st.step(args.warmup)
    torch.cuda.synchronize()
    print("[bench] warmup %d steps %.2f s" % (args.warmup, time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    cores_host = st.get_cores_host()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.step(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    value = args.steps / el
    print("[bench] timed %d steps %.3f s -> %.3f steps/s" % (args.steps, el, value),
          file=sys.stderr, flush=True)
    info = st.info()

    roof = None
    cpu = None
    if not args.no_roofline:
        roof = roofline(binding, st, cores_host, min(args.steps, 3), 2 * p.chi_max)
        # whole-step algorithmic rate at the timed steps/s, against FP64 peak
        roof["step_tflops"] = roof["step_gflop"] * value / 1e3
        roof["step_frac"] = roof["step_tflops"] / PEAK_FP64_TFLOPS
        print("[bench] roofline %s" % json.dumps(roof), file=sys.stderr, flush=True)
    oracle_f0, oracle_ref = None, None
    if not args.no_cpu_baseline:
        cpu, oracle_f0, oracle_ref = cpu_baseline(w, args.mode)
        print("[bench] cpu baseline %s" % cpu, file=sys.stderr, flush=True)

    extras = {}
    if not args.no_extras:
        extras["graph"] = graph_run(binding, w, cores_host, min(args.steps, 5), value)
        print("[bench] graph %s" % json.dumps(extras["graph"]), file=sys.stderr, flush=True)
        # the multi-stream sweep first, in a process that has created few streams
        extras["batched"] = batched_sweep(binding, 64, 3)
        print("[bench] batched %s" % json.dumps(extras["batched"]), file=sys.stderr, flush=True)
        extras["batched_metric"] = batched_metric(binding, args.batch, 3, value)
        print("[bench] batched_metric %s" % json.dumps(extras["batched_metric"]),
              file=sys.stderr, flush=True)
        # the precision modes from the oracle's start state, each one-step
        # result against the oracle's step from it (and against FP64)
        extras["mixed"] = mixed_precision(binding, w,
                                          oracle_f0 if oracle_f0 is not None else cores_host,
                                          min(args.steps, 5), fp64_steps_per_s=value,
                                          oracle=oracle_ref)
        print("[bench] mixed %s" % json.dumps(extras["mixed"]), file=sys.stderr, flush=True)
        extras["physics"] = physics_run(binding, 5)
        print("[bench] physics %s" % json.dumps(extras["physics"]), file=sys.stderr, flush=True)
        extras["chi128"] = chi128_run(binding, 3, with_oracle=not args.no_cpu_baseline)
        print("[bench] chi128 %s" % json.dumps(extras["chi128"]), file=sys.stderr, flush=True)
        extras["buneman"] = buneman_run(binding, 3)
        print("[bench] buneman %s" % json.dumps(extras["buneman"]), file=sys.stderr, flush=True)
        extras["orderings"] = orderings(binding, 3)
        print("[bench] orderings %s" % json.dumps(extras["orderings"]), file=sys.stderr, flush=True)
        extras["serving"] = serving_run(binding, args.serving_requests, args.serving_steps)
        print("[bench] serving %s" % json.dumps(extras["serving"]), file=sys.stderr, flush=True)

    out = {
        "metric": "time steps/s at Nx=Nv=2^10, chi=64",
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "two-stream 2^10 x 2^10, interleaved, chi=64, %s" % (
            "every compression capped at chi (C5), tol=0, D_F=4, seeded random-MPS perturbation"
            if args.mode == "fixed" else "C1, tol=1e-10, from f0"),
                   "dt": p.dt, "sites": p.n_sites, "final_bonds": info["bonds"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        # launch-shape table in use (bit-identical variants; speed only)
        "tuning": {"table": "paper_2205_11990_amd/tuning_gfx950.txt"
                   if os.environ.get("MPSV_TUNING", "") in ("",) else os.environ["MPSV_TUNING"],
                   "entries": binding.tune_size()},
    }
    out.update(extras)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
