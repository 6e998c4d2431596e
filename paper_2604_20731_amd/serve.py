"""Continuous-batching serving of reservoir scenarios on one MI355X.

Scenarios (reservoir simulations of a given grid, network width and wells)
arrive over time.  A scenario is admitted as soon as a slot is free and its
device workspace fits the HBM budget; it is then pretrained and advanced one
coupled step at a time.  Every admitted scenario owns a HIP stream and a
libcrv context whose state (fields, network, Adam moments) stays on the
device; each coupled step is one replay of that context's captured step
graph, so the steps of different scenarios overlap on the GPU.  A scenario
retires after its last step, freeing its slot and memory for the next
arrival.

Scenarios share no device state and every kernel reduces in a fixed order,
so a scenario's results are the same alone and in any mix.

Reported: scenarios/s (completed / span from first arrival to last
completion), p50/p99 latency of a coupled step (GPU time from the moment the
step reaches the head of its stream to its completion), queue waits, the
largest number of scenarios active at once, and the arrivals refused because
their workspace alone exceeds the HBM budget.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque
from typing import Dict, List, Optional

import numpy as np

from . import crv, inputs


def cfl_dt(p: np.ndarray, log_perm: np.ndarray, poro: np.ndarray, ne: int, n_exp: float = 2.0,
           mu_g: float = 0.1, cfl: float = 0.5) -> float:
    """Step length cfl * h * phi_min / (max lambda_g' * max |K grad_+ p|) from
    the pretrained network pressure (2D or 3D nodal arrays)."""
    k = np.exp(log_perm)
    cut = tuple(slice(0, ne) for _ in range(p.ndim))
    g = sum((np.diff(p, axis=a)[cut] * ne) ** 2 for a in range(p.ndim))
    kmax = float(np.max(k[cut] * np.sqrt(g)))
    return cfl * (1.0 / ne) * float(poro.min()) / ((n_exp / mu_g) * max(kmax, 1e-30))


def scenario_problem(arr: inputs.Arrival) -> inputs.Problem:
    """The reservoir of one arrival: its own GRF log-permeability (l = 0.05),
    porosity 0.2, 1-8 balanced wells, quadratic B-splines, 4 hidden layers."""
    ne = arr.n_elem
    wells = inputs.wells_balanced(arr.n_wells, arr.seed)
    return inputs.make_problem("b512", seed=arr.seed, n_elem=ne, width=arr.width, wells=wells)


@dataclasses.dataclass
class Job:
    arr: inputs.Arrival
    prob: inputs.Problem
    sc: crv.Scenario
    ws: int
    t_admit: float
    dt: float = 0.0
    phase: str = "pretrain"
    steps_done: int = 0
    ev_start: object = None
    ev_end: object = None
    latencies_ms: List[float] = dataclasses.field(default_factory=list)


class Server:
    def __init__(self, hbm_budget_bytes: int, max_active: int = 16, precision: str = "bf16x3f",
                 pretrain_iters: int = 200, steps: int = 20, device: str = "cuda:0",
                 keep_fields: bool = False):
        self.budget = int(hbm_budget_bytes)
        self.max_active = max_active
        self.precision = precision
        self.pretrain_iters = pretrain_iters
        self.steps = steps
        self.device = device
        self.keep_fields = keep_fields

    def precision_for(self, width: int) -> str:
        """The requested form where it exists (split bf16 stops at width 64;
        the mixed form covers 32, 64 and 128), plain bf16 otherwise."""
        if self.precision == "bf16x3" and width not in (32, 64):
            return "bf16"
        if self.precision == "bf16x3f" and width not in (32, 64, 128):
            return "bf16"
        return self.precision

    def run(self, arrivals: List[inputs.Arrival], time_scale: float = 1.0) -> Dict:
        import torch
        pending = deque(sorted(arrivals, key=lambda a: a.t))
        active: List[Job] = []
        results = {}
        refused = []
        used = 0
        most_active = 0
        peak_bytes = 0
        waits, lat = [], []
        t0 = time.perf_counter()
        first_arrival = pending[0].t if pending else 0.0
        last_done = 0.0
        while pending or active:
            now = (time.perf_counter() - t0) * time_scale
            # ---- admission: arrived, a slot free, workspace fits the budget
            while pending and pending[0].t <= now and len(active) < self.max_active:
                arr = pending[0]
                prob = scenario_problem(arr)
                cfg = crv.config(dim=2, n_elem=prob.n_elem, degree=prob.degree, width=prob.width,
                                 hidden=prob.hidden, precision=self.precision_for(prob.width))
                ws = crv.workspace_size(cfg)
                if ws > self.budget:
                    # can never fit: refuse it rather than wait for memory
                    # that no retirement frees
                    refused.append(pending.popleft().seed)
                    continue
                if used + ws > self.budget:
                    break
                pending.popleft()
                stream = torch.cuda.Stream(device=self.device)
                sc = crv.Scenario(cfg, prob.log_perm, prob.porosity, prob.wells, prob.theta0,
                                  device=self.device, stream=stream)
                used += ws
                job = Job(arr=arr, prob=prob, sc=sc, ws=ws, t_admit=now)
                waits.append(now - arr.t)
                sc.train_async(self.pretrain_iters)
                job.ev_end = torch.cuda.Event()
                job.ev_end.record(stream)
                active.append(job)
                most_active = max(most_active, len(active))
                peak_bytes = max(peak_bytes, used)
            # ---- progress: every job whose in-flight work finished moves on
            progressed = False
            for job in list(active):
                if not job.ev_end.query():
                    continue
                progressed = True
                if job.phase == "pretrain":
                    p, _, _ = job.sc.fields()
                    job.dt = cfl_dt(p, job.prob.log_perm, job.prob.porosity, job.prob.n_elem)
                    job.phase = "step"
                else:
                    ms = job.ev_start.elapsed_time(job.ev_end)
                    job.latencies_ms.append(ms)
                    lat.append(ms)
                    job.steps_done += 1
                if job.steps_done >= self.steps:
                    out = job.sc.fields() if self.keep_fields else None
                    job.sc.sync()
                    results[job.arr.seed] = {"fields": out, "latencies_ms": job.latencies_ms,
                                             "n_elem": job.prob.n_elem, "width": job.prob.width,
                                             "admit_s": job.t_admit, "arrival_s": job.arr.t}
                    job.sc.close()
                    used -= job.ws
                    active.remove(job)
                    last_done = (time.perf_counter() - t0) * time_scale
                    continue
                st = job.sc.stream
                job.ev_start = torch.cuda.Event(enable_timing=True)
                job.ev_end = torch.cuda.Event(enable_timing=True)
                job.ev_start.record(st)
                job.sc.step(job.dt)
                job.ev_end.record(st)
            if not progressed:
                time.sleep(0.0002)
        span = max(last_done - first_arrival, 1e-9)
        lat_a = np.array(lat) if lat else np.array([np.nan])
        # the same percentiles per scenario shape: what the tail is made of
        by_shape = {}
        for r in results.values():
            by_shape.setdefault(f"{r['n_elem']}^2 w{r['width']}", []).extend(r["latencies_ms"])
        shapes = {k: {"steps": len(v), "p50_step_ms": float(np.percentile(v, 50)),
                      "p99_step_ms": float(np.percentile(v, 99))}
                  for k, v in sorted(by_shape.items()) if v}
        return {
            "scenarios": len(results),
            "scenarios_per_s": len(results) / span,
            "coupled_steps_per_s": len(lat) / span,
            "p50_step_ms": float(np.percentile(lat_a, 50)),
            "p99_step_ms": float(np.percentile(lat_a, 99)),
            "mean_queue_wait_s": float(np.mean(waits)) if waits else 0.0,
            "max_queue_wait_s": float(np.max(waits)) if waits else 0.0,
            "span_s": span,
            "by_shape": shapes,
            "max_active_seen": most_active,
            "peak_workspace_bytes": peak_bytes,
            "refused": refused,
            "results": results,
        }
