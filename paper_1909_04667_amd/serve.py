"""Serving loop: continuous batching of force requests over many systems.

Systems (N-body particle sets of uneven size) stay resident on the GPU with
their trees; requests name a system, an active subset (the particles whose
time-step bins are due, Sec. 7.2 of the Arepo paper) and a precision.  The
loop:

* admission -- a request's system is built when first needed if its memory
  estimate (``tpm_bytes_needed``) fits the HBM budget, evicting idle systems
  least recently used; otherwise the request waits;
* builds (and the PM solve of periodic systems) run on a build stream while
  the walk stream serves the systems that are ready;
* batching -- every iteration stages at most one request stage per system
  and launches ONE batched persistent walk per precision for all of them
  (``tpm_batch_launch``); requests that arrive while a launch is on the GPU
  join the next one;
* stages -- isolated systems with the relative criterion and periodic
  systems take two passes as in the paper's first force computation
  (Sec. 3.1): geometric criterion (plus PM long range), then the relative
  criterion with |a| of the first pass; Plummer systems take the geometric
  pass only;
* completion times come from GPU events on the walk stream, so latency =
  GPU completion time - arrival time, both relative to the same start.

All force arithmetic runs in the library's kernels; this module only
schedules them.
"""
from __future__ import annotations

import math
import time
from collections import OrderedDict
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as B
from . import workloads as W


def system_params(spec: W.SystemSpec, precision: str):
    """Solver settings per kind, as the numbered workloads use them."""
    if spec.kind == "plummer":
        return B.make_params(precision=precision, eps=0.01, theta=0.5), ("bh",)
    if spec.kind == "hernquist":
        return B.make_params(precision=precision, eps=0.005, theta=0.5,
                             alpha=0.0025), ("bh", "rel")
    ng = int(round(spec.n ** (1.0 / 3.0)))
    pm = 16
    while pm < 2 * ng and pm < 512:
        pm *= 2
    return B.make_params(precision=precision, periodic=True, box_size=100.0, pm_grid=pm,
                         eps=100.0 / (50 * ng), theta=0.5, alpha=0.0025), ("bh", "rel")


@dataclass
class Resident:
    key: tuple
    ctx: B.Context
    tensors: tuple
    bytes: int
    ready: torch.cuda.Event
    periodic: bool
    stages: tuple
    busy: int = 0          # requests admitted and not finished
    last_used: float = 0.0


@dataclass
class Job:
    req: W.Request
    key: tuple
    idx: torch.Tensor
    stage: int = 0
    acc: torch.Tensor | None = None
    acc_pm: torch.Tensor | None = None
    anorm: torch.Tensor | None = None
    done_event: torch.cuda.Event | None = None
    done_ms: float = math.nan
    admitted: bool = False
    rejected: bool = False


@dataclass
class Stats:
    latencies_ms: list = field(default_factory=list)
    force_evals: int = 0
    batches: int = 0
    items_per_batch: list = field(default_factory=list)
    builds: int = 0
    evictions: int = 0
    wall_s: float = 0.0
    span_ms: float = 0.0
    rejected: int = 0

    def summary(self):
        lat = sorted(self.latencies_ms)

        def q(p):
            if not lat:
                return math.nan
            return lat[min(len(lat) - 1, max(0, int(math.ceil(p / 100 * len(lat))) - 1))]

        return {"requests": len(lat), "force_evals": self.force_evals,
                "throughput_evals_per_s": self.force_evals / (self.span_ms * 1e-3)
                if self.span_ms > 0 else math.nan,
                "p50_ms": q(50), "p99_ms": q(99), "max_ms": q(100),
                "batches": self.batches,
                "mean_stages_per_batch": float(np.mean(self.items_per_batch))
                if self.items_per_batch else 0.0,
                "builds": self.builds, "evictions": self.evictions, "rejected": self.rejected,
                "wall_s": self.wall_s}


class Server:
    def __init__(self, pool, budget_bytes: int, device="cuda:0", max_inflight: int = 2):
        self.pool = pool
        self.budget = int(budget_bytes)
        self.dev = torch.device(device)
        self.build_stream = torch.cuda.Stream(device=self.dev)
        self.walk_stream = torch.cuda.Stream(device=self.dev)
        self.batch = B.Batch(stream=self.walk_stream)
        self.resident: "OrderedDict[tuple, Resident]" = OrderedDict()
        self.used = 0
        self.max_inflight = max_inflight
        self.particles = {}

    # -- memory admission ----------------------------------------------------
    def _particles(self, sid):
        if sid not in self.particles:
            self.particles[sid] = W.system_particles(self.pool[sid])
        return self.particles[sid]

    def _evict_for(self, need, stats):
        for key in list(self.resident):
            if self.used + need <= self.budget:
                break
            r = self.resident[key]
            if r.busy == 0:
                r.ctx.close()
                self.used -= r.bytes
                del self.resident[key]
                stats.evictions += 1
        return self.used + need <= self.budget

    def _admit(self, job: Job, stats) -> bool:
        if job.key in self.resident:
            r = self.resident[job.key]
            r.busy += 1
            self.resident.move_to_end(job.key)
            return True
        spec = self.pool[job.req.sid]
        params, stages = system_params(spec, job.req.precision)
        need = B.bytes_needed(params, spec.n)
        if need > self.budget:
            job.rejected = True  # can never fit
            return False
        if not self._evict_for(need, stats):
            return False
        p = self._particles(job.req.sid)
        with torch.cuda.stream(self.build_stream):
            t = lambda a: torch.as_tensor(a, dtype=torch.float64).to(self.dev, non_blocking=False)
            x, y, z = t(p.x), t(p.y), t(p.z)
            ctx = B.Context(params, stream=self.build_stream)
            ctx.build_tree(x, y, z)
            if spec.kind == "periodic":  # solve the mesh once per build
                ctx.pm_long_range(torch.zeros(0, dtype=torch.int32, device=self.dev))
            ev = torch.cuda.Event()
            ev.record(self.build_stream)
        ctx.set_stream(self.walk_stream)  # per-request work runs on the walk stream
        r = Resident(job.key, ctx, (x, y, z), need, ev, spec.kind == "periodic", stages,
                     busy=1)
        self.resident[job.key] = r
        self.used += need
        stats.builds += 1
        return True

    # -- the loop ---------------------------------------------------------------
    def run(self, requests, time_scale: float = 1.0):
        """Serve ``requests`` (arrival times in seconds, scaled by time_scale)
        and return Stats.  Active subsets are drawn and uploaded beforehand."""
        stats = Stats()
        jobs = []
        for sid in sorted({rq.sid for rq in requests}):
            self._particles(sid)  # host-side generation stays out of the clock
        for rq in requests:
            n = self.pool[rq.sid].n
            idx = torch.as_tensor(W.request_active(rq, n), dtype=torch.int32, device=self.dev)
            jobs.append(Job(rq, (rq.sid, rq.precision), idx))
        torch.cuda.synchronize()
        pending = list(jobs)          # not yet arrived or not yet admitted
        ready = []                    # admitted, waiting for a stage launch
        inflight = []                 # (event, [jobs whose stage ends there])
        start = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        start.record(self.walk_stream)
        finished = 0
        while finished < len(jobs):
            now = (time.perf_counter() - t0) / time_scale
            # arrivals and admission, in arrival order
            still = []
            for j in pending:
                if j.req.t_arrival <= now and self._admit(j, stats):
                    j.admitted = True
                    ready.append(j)
                elif j.rejected:
                    finished += 1
                else:
                    still.append(j)
            pending = still
            # completed launches
            while inflight and inflight[0][0].query():
                ev, done_jobs = inflight.pop(0)
                for j in done_jobs:
                    r = self.resident[j.key]
                    r.busy -= 1
                    r.last_used = now
                    finished += 1
            # launch the next batch if the GPU queue has room
            if len(inflight) < self.max_inflight and ready:
                staged, rest, ends = set(), [], []
                for j in ready:
                    r = self.resident[j.key]
                    if j.key in staged or not r.ready.query():
                        rest.append(j)
                        continue
                    staged.add(j.key)
                    self.walk_stream.wait_event(r.ready)
                    self._stage(j, r)
                    if j.stage >= len(r.stages):
                        ends.append(j)
                    else:
                        rest.append(j)
                ready = rest
                if staged:
                    self.batch.launch()
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(self.walk_stream)
                    for j in ends:
                        j.done_event = ev
                    inflight.append((ev, ends))
                    stats.batches += 1
                    stats.items_per_batch.append(len(staged))
            elif not ready and not inflight:
                time.sleep(1e-4)
        torch.cuda.synchronize()
        stats.wall_s = time.perf_counter() - t0
        first = min((j.req.t_arrival for j in jobs if not j.rejected), default=0.0) * 1e3 * time_scale
        last = 0.0
        stats.rejected = sum(j.rejected for j in jobs)
        for j in jobs:
            if j.rejected:
                continue
            j.done_ms = start.elapsed_time(j.done_event)
            stats.latencies_ms.append(j.done_ms - j.req.t_arrival * 1e3 * time_scale)
            stats.force_evals += j.idx.numel()
            last = max(last, j.done_ms)
        stats.span_ms = last - first
        return stats, jobs

    def _stage(self, j: Job, r: Resident):
        """Stage the next pass of job j into the current batch."""
        opening = r.stages[j.stage]
        dt = r.ctx.dtype
        if j.stage == 0:
            if r.periodic:
                j.acc_pm, _ = r.ctx.pm_long_range(j.idx, want_pot=False)
            j.acc = self.batch.add(r.ctx, j.idx, "bh",
                                   acc=torch.empty((3, j.idx.numel()), dtype=dt,
                                                   device=self.dev))
        else:
            # |a| of the first pass (tree + PM) feeds the relative criterion
            with torch.cuda.stream(self.walk_stream):
                j.anorm = torch.zeros(r.ctx.n, dtype=torch.float64, device=self.dev)
            r.ctx.accel_norm(j.idx, j.acc, j.acc_pm, out=j.anorm)
            j.acc = self.batch.add(r.ctx, j.idx, opening, a_old_norm=j.anorm,
                                   acc=torch.empty((3, j.idx.numel()), dtype=dt,
                                                   device=self.dev))
        j.stage += 1

    def close(self):
        for r in self.resident.values():
            r.ctx.close()
        self.resident.clear()
        self.batch.close()


def total_force(job: Job):
    """Tree (+ PM) acceleration of a finished job, [3][n_act]."""
    return job.acc if job.acc_pm is None else job.acc + job.acc_pm
