"""Continuous-batching serving of solve requests on one GPU.

A request asks for a number of RK4 steps of one problem (grid, bond cap,
precision) from given initial profiles.  Requests are admitted in arrival
order while the device-memory bound of the admitted set
(`mps_workspace_bound` of each request) stays within the HBM budget and an
execution slot is free.  Every admitted request is driven by its own host
thread on its own stream, with its MPS state resident in device memory
from the first step to the last, so requests that arrive while others run
join the work on the chip as soon as memory and a slot free up.  The
factorisations of one request occupy single compute units, which is what
lets several requests share the device.

Latency is completion time minus arrival time.  Each result is computed by
the same library calls as a request run alone, so it is the same alone and
in the mix.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from . import binding


@dataclass
class Request:
    rid: int
    problem: object          # workloads.Problem-like (see binding.make_problem)
    ax: np.ndarray           # f0(x, v) = sum_r ax[r] (x) bv[r]
    bv: np.ndarray
    steps: int
    arrival: float = 0.0     # seconds after the start of the run
    kind: str = ""


@dataclass
class Result:
    rid: int
    kind: str
    arrival: float
    admitted: float
    finished: float
    steps: int
    bound: int
    scalars: Dict[str, float] = field(default_factory=dict)
    bonds: List[int] = field(default_factory=list)
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def run_alone(req: Request) -> Result:
    """The request on its own (reference for the in-the-mix results)."""
    return Server(budget_bytes=1 << 62, slots=1).run([Request(
        req.rid, req.problem, req.ax, req.bv, req.steps, 0.0, req.kind)],
        realtime=False)[0]


class Server:
    def __init__(self, budget_bytes: int, slots: int = 16):
        self.budget = int(budget_bytes)
        self.slots = int(slots)

    def run(self, requests: Sequence[Request], realtime: bool = True,
            on_done: Optional[Callable[[Result], None]] = None) -> List[Result]:
        """Serve the requests; with realtime, a request is not admitted
        before its arrival time.  on_done is called with each result as it
        completes.  Returns the results in request order."""
        import torch
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        cv = threading.Condition()
        used = [0, 0]  # bytes, active requests
        results: Dict[int, Result] = {}
        t0 = time.perf_counter()
        dev = torch.cuda.current_device()

        def now() -> float:
            return time.perf_counter() - t0

        def worker(req: Request, bound: int, admitted: float) -> None:
            sc: Dict[str, float] = {}
            bonds: List[int] = []
            err = None
            try:
                torch.cuda.set_device(dev)
                s = torch.cuda.Stream()
                with torch.cuda.stream(s):
                    st = binding.MpsState(req.problem, req.ax, req.bv, stream=s)
                    try:
                        for _ in range(req.steps):
                            st.step(1, stream=s)
                        _, _, sc = st.moments(stream=s)
                        bonds = st.info()["bonds"]
                    finally:
                        st.free()
            except Exception as e:  # reported per request
                err = "%s: %s" % (type(e).__name__, e)
            fin = now()
            res = Result(req.rid, req.kind, req.arrival, admitted, fin, req.steps, bound,
                         sc, bonds, err)
            with cv:
                results[req.rid] = res
                used[0] -= bound
                used[1] -= 1
                cv.notify_all()
            if on_done is not None:
                on_done(res)

        threads = []
        for req in reqs:
            bound = binding.workspace_bound(req.problem)
            if bound > self.budget:
                results[req.rid] = Result(req.rid, req.kind, req.arrival, now(), now(),
                                          req.steps, bound,
                                          error="device-memory bound exceeds the budget")
                continue
            if realtime:
                wait = req.arrival - now()
                if wait > 0:
                    time.sleep(wait)
            with cv:
                while used[1] >= self.slots or used[0] + bound > self.budget:
                    cv.wait()
                used[0] += bound
                used[1] += 1
            th = threading.Thread(target=worker, args=(req, bound, now()), daemon=True)
            th.start()
            threads.append(th)
        for th in threads:
            th.join()
        return [results[r.rid] for r in sorted(requests, key=lambda r: r.rid)]


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process (exponential gaps, mean 1/rate)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def summary(results: Sequence[Result]) -> Dict[str, float]:
    ok = [r for r in results if r.error is None]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    span = (max(r.finished for r in ok) - min(r.arrival for r in ok)) if ok else 1.0
    return {"requests": len(results), "served": len(ok),
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "aggregate_steps_per_s": float(sum(r.steps for r in ok) / max(span, 1e-9))}
