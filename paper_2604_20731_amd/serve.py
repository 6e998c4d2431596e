"""Continuous-batching serving of reservoir scenarios on one MI355X.

Scenarios (reservoir simulations of a given grid, network width and wells)
arrive over time.  A scenario is admitted as soon as a slot is free and the
device memory it needs fits the HBM budget; it is then pretrained and advanced
one coupled step at a time, its state (fields, network, Adam moments) staying
on the device.  A scenario retires after its last step, freeing its slot for
the next arrival.

Two ways to run the steps:

* batched (default): scenarios of one shape (grid, width, network form) live
  in the slots of a pool, one device allocation of `pool_slots` workspaces at
  a fixed stride with one stream.  Every pass of the loop takes the scenarios
  of a pool that are ready for their next step, splits them into runs of
  consecutive slots and advances each run with one crv_step_batch: one
  captured graph in which every kernel of the coupled step runs once for the
  whole run.  The HBM budget counts pools; a pool is freed when it empties.
  A pool has at most `pool_slots` slots and at most as many as keep its
  batched step's network work (elements x width^2 per scenario) within
  `batch_cost_cap`: a round of a pool is one step of all its scenarios, so
  the cap bounds the step latency of the heavy shapes (the default admits
  two 512^2 width-128 scenarios per pool, and eight of every shape at most
  a quarter of that).  Every kernel reduces in an order that does not depend
  on the batch, so the results are bitwise those of the scenario alone.
* streams: every scenario has its own workspace and stream; each step is one
  replay of its own captured graph, and the steps of different scenarios
  overlap on the device.  Scenarios share no device state and every kernel
  reduces in a fixed order, so the results are bitwise those of the
  scenario alone.

Reported: scenarios/s (completed / span from first arrival to last
completion), coupled steps/s, p50/p99 latency of a coupled step (GPU time
from the moment the step reaches the head of its stream to its completion;
a batched step's latency is its batch's), the same per scenario shape,
queue waits, the largest number of scenarios active at once, the largest
batch, the peak device memory held, and the arrivals refused because their
memory alone exceeds the budget.
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
    pool: object = None
    slot: int = -1
    waiting: bool = False   # its last work finished; ready for the next step
    latencies_ms: List[float] = dataclasses.field(default_factory=list)


class Pool:
    """Slots of one scenario shape: `n` workspaces at one stride in one
    device allocation, one stream."""

    def __init__(self, cfg: crv.CrvConfig, n: int, device: str):
        import torch
        self.cfg = cfg
        self.stride = (crv.workspace_size(cfg) + 255) // 256 * 256
        self.n = n
        self.mem = torch.empty(self.stride * n + 256, dtype=torch.uint8, device=device)
        self.lead = (-self.mem.data_ptr()) % 256
        self.stream = torch.cuda.Stream(device=device)
        self.jobs: List[Optional[Job]] = [None] * n
        self.bytes = self.stride * n + 256

    def free_slot(self) -> int:
        for k, j in enumerate(self.jobs):
            if j is None:
                return k
        return -1

    def view(self, k: int):
        a = self.lead + k * self.stride
        return self.mem[a:a + self.stride]

    def empty(self) -> bool:
        return all(j is None for j in self.jobs)


class Server:
    def __init__(self, hbm_budget_bytes: int, max_active: int = 16, precision: str = "bf16x3f",
                 pretrain_iters: int = 200, steps: int = 20, device: str = "cuda:0",
                 keep_fields: bool = False, batch: bool = True, pool_slots: int = 8,
                 batch_cost_cap: float = 2.0 * 512 ** 2 * 128 ** 2):
        self.budget = int(hbm_budget_bytes)
        self.max_active = max_active
        self.precision = precision
        self.pretrain_iters = pretrain_iters
        self.steps = steps
        self.device = device
        self.keep_fields = keep_fields
        self.batch = batch
        self.pool_slots = pool_slots
        self.batch_cost_cap = batch_cost_cap

    def slots_for(self, prob: inputs.Problem) -> int:
        """Slots of a new pool for this shape: pool_slots, fewer where one
        scenario's network work (elements x width^2, in proportion to its
        nodes x width^2) would make a full round exceed batch_cost_cap (at
        least one)."""
        cost = float(prob.n_elem ** prob.dim) * prob.width ** 2
        return max(1, min(self.pool_slots, int(self.batch_cost_cap // cost)))

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
        pools: Dict[tuple, List[Pool]] = {}
        results = {}
        refused = []
        used = 0
        most_active = 0
        peak_bytes = 0
        biggest_batch = 0
        waits, lat = [], []
        t0 = time.perf_counter()
        first_arrival = pending[0].t if pending else 0.0
        last_done = 0.0

        def step_timed(stream, jobs, launch):
            """launch() enqueues the jobs' step on stream, bracketed by a
            pair of timing events that all of the jobs share."""
            ev_s = torch.cuda.Event(enable_timing=True)
            ev_e = torch.cuda.Event(enable_timing=True)
            ev_s.record(stream)
            launch()
            ev_e.record(stream)
            for j in jobs:
                j.ev_start, j.ev_end = ev_s, ev_e

        while pending or active:
            now = (time.perf_counter() - t0) * time_scale
            # ---- admission: arrived, a slot free, memory within the budget
            while pending and pending[0].t <= now and len(active) < self.max_active:
                arr = pending[0]
                prob = scenario_problem(arr)
                cfg = crv.config(dim=2, n_elem=prob.n_elem, degree=prob.degree, width=prob.width,
                                 hidden=prob.hidden, precision=self.precision_for(prob.width))
                ws = crv.workspace_size(cfg)
                key = (prob.n_elem, prob.width, cfg.precision)
                pool, slot, need, n_slots = None, -1, ws, 0
                if self.batch:
                    for pl in pools.get(key, []):
                        slot = pl.free_slot()
                        if slot >= 0:
                            pool, need = pl, 0
                            break
                    if pool is None:
                        # a new pool: as many slots as the budget allows, at most pool_slots
                        stride = (ws + 255) // 256 * 256
                        n_slots = min(self.slots_for(prob), (self.budget - 256) // stride)
                        need = stride * n_slots + 256
                if (self.batch and pool is None and n_slots < 1) or ws > self.budget:
                    # can never fit: refuse it rather than wait for memory
                    # that no retirement frees
                    refused.append(pending.popleft().seed)
                    continue
                if used + need > self.budget:
                    break
                pending.popleft()
                if self.batch:
                    if pool is None:
                        pool = Pool(cfg, n_slots, self.device)
                        pools.setdefault(key, []).append(pool)
                        slot = 0
                    stream = pool.stream
                    sc = crv.Scenario(cfg, prob.log_perm, prob.porosity, prob.wells, prob.theta0,
                                      device=self.device, stream=stream,
                                      workspace=pool.view(slot))
                else:
                    stream = torch.cuda.Stream(device=self.device)
                    sc = crv.Scenario(cfg, prob.log_perm, prob.porosity, prob.wells, prob.theta0,
                                      device=self.device, stream=stream)
                used += need
                # a pool's memory is returned when the pool empties, not per job
                job = Job(arr=arr, prob=prob, sc=sc, ws=0 if self.batch else ws, t_admit=now,
                          pool=pool, slot=slot)
                if pool is not None:
                    pool.jobs[slot] = job
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
                if job.waiting or not job.ev_end.query():
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
                    active.remove(job)
                    used -= job.ws
                    if job.pool is not None:
                        job.pool.jobs[job.slot] = None
                        if job.pool.empty():
                            used -= job.pool.bytes
                            pools[(job.prob.n_elem, job.prob.width,
                                   job.pool.cfg.precision)].remove(job.pool)
                    last_done = (time.perf_counter() - t0) * time_scale
                    continue
                job.waiting = True
            # ---- steps: a pool advances in rounds, once none of its scenarios
            # has work in flight, each run of consecutive slots as one batch;
            # on their own streams every waiting scenario steps at once
            if self.batch:
                for plist in pools.values():
                    for pl in plist:
                        jobs = [j for j in pl.jobs if j is not None]
                        if not jobs or not all(j.waiting for j in jobs):
                            continue
                        for j in jobs:
                            j.waiting = False
                        jobs.sort(key=lambda j: j.slot)
                        runs, cur = [], [jobs[0]]
                        for j in jobs[1:]:
                            if j.slot == cur[-1].slot + 1:
                                cur.append(j)
                            else:
                                runs.append(cur)
                                cur = [j]
                        runs.append(cur)
                        for run in runs:
                            step_timed(pl.stream, run,
                                       lambda r=run: crv.step_batch([j.sc for j in r],
                                                                    [j.dt for j in r]))
                            biggest_batch = max(biggest_batch, len(run))
            else:
                for job in active:
                    if job.waiting:
                        job.waiting = False
                        step_timed(job.sc.stream, [job], lambda j=job: j.sc.step(j.dt))
                        biggest_batch = max(biggest_batch, 1)
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
            "mode": "batched" if self.batch else "streams",
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
            "largest_batch": biggest_batch,
            "peak_workspace_bytes": peak_bytes,
            "refused": refused,
            "results": results,
        }
