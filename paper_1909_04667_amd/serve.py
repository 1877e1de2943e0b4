"""Serving loop: continuous batching of force requests over many systems.

Systems (N-body particle sets of uneven size) stay resident on the GPU with
their trees; requests name a system, an active subset (the particles whose
time-step bins are due, Sec. 7.2 of the Arepo paper) and a precision.  The
walks run inside the library's device-resident request loop: one persistent
kernel per precision (``ResidentServer``) that takes requests while it runs,
so a request that arrives while others are on the GPU joins the running
kernel and its work items interleave with theirs.  This module schedules:

* admission -- a request's system is built when first needed if its memory
  estimate (``tpm_bytes_needed``) fits the HBM budget, evicting idle systems
  least recently used; otherwise the request waits; a system that can never
  fit is rejected;
* one request, one submission -- isolated systems with the relative
  criterion and periodic systems take the paper's first force computation
  (Sec. 3.1) as one device-side request (``submit_step``: geometric pass,
  the mesh force for periodic boxes, |a| of their sum, relative pass);
  Plummer systems take the geometric pass only.  One request per system is
  in flight; others wait in the system's queue;
* latency = host time at which completion is observed - arrival time.

All force arithmetic runs in the library's kernels; this module only
schedules them.
"""
from __future__ import annotations

import math
import time
from collections import OrderedDict, deque
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
    stream: torch.cuda.Stream
    periodic: bool
    stages: tuple
    queue: deque = field(default_factory=deque)  # admitted jobs, FIFO
    active: "Job | None" = None                  # the job in flight
    last_used: float = 0.0


@dataclass
class Job:
    req: W.Request
    key: tuple
    idx: torch.Tensor
    state: str = "new"      # new, queued, walking, done, rejected
    ticket: int = 0
    acc: torch.Tensor | None = None
    acc_pm: torch.Tensor | None = None
    done_s: float = math.nan
    waited: bool = False

    @property
    def rejected(self):
        return self.state == "rejected"


@dataclass
class Stats:
    latencies_ms: list = field(default_factory=list)
    force_evals: int = 0
    builds: int = 0
    evictions: int = 0
    waits: int = 0
    rejected: int = 0
    wall_s: float = 0.0
    span_ms: float = 0.0
    kernel_launches: int = 0

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
                "builds": self.builds, "evictions": self.evictions,
                "waited_for_memory": self.waits, "rejected": self.rejected,
                "server_kernel_launches": self.kernel_launches, "wall_s": self.wall_s}


class Server:
    def __init__(self, pool, budget_bytes: int, device="cuda:0", idle_ms: float = 5.0):
        self.pool = pool
        self.budget = int(budget_bytes)
        self.dev = torch.device(device)
        self.loops = {p: B.ResidentServer(p, idle_ms) for p in ("fp32", "fp64")}
        self.resident: "OrderedDict[tuple, Resident]" = OrderedDict()
        self.used = 0
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
            if r.active is None and not r.queue:
                r.ctx.close()
                self.used -= r.bytes
                del self.resident[key]
                stats.evictions += 1
        return self.used + need <= self.budget

    def _admit(self, job: Job, stats) -> bool:
        """Queue the job on its resident system, building the system if it is
        not resident and memory allows; False if it has to wait."""
        if job.key in self.resident:
            r = self.resident[job.key]
            self.resident.move_to_end(job.key)
            r.queue.append(job)
            return True
        spec = self.pool[job.req.sid]
        params, stages = system_params(spec, job.req.precision)
        need = B.bytes_needed(params, spec.n)
        if need > self.budget:
            job.state = "rejected"  # can never fit
            return False
        if not self._evict_for(need, stats):
            if not job.waited:
                job.waited = True
                stats.waits += 1
            return False
        p = self._particles(job.req.sid)
        st = torch.cuda.Stream(device=self.dev)
        with torch.cuda.stream(st):
            t = lambda a: torch.as_tensor(a, dtype=torch.float64).to(self.dev)
            x, y, z = t(p.x), t(p.y), t(p.z)
            ctx = B.Context(params, stream=st)
            ctx.build_tree(x, y, z)
            if spec.kind == "periodic":  # solve the mesh once per build
                ctx.pm_long_range(torch.zeros(0, dtype=torch.int32, device=self.dev))
            ev = torch.cuda.Event()
            ev.record(st)
        r = Resident(job.key, ctx, (x, y, z), need, ev, st, spec.kind == "periodic", stages)
        r.queue.append(job)
        self.resident[job.key] = r
        self.used += need
        stats.builds += 1
        return True

    # -- requests -------------------------------------------------------------
    def _start(self, j: Job, r: Resident):
        """Submit the job to the running kernel of its precision."""
        loop = self.loops[j.req.precision]
        if len(r.stages) > 1:
            j.ticket, j.acc, j.acc_pm = loop.submit_step(r.ctx, j.idx)
        else:
            j.ticket, j.acc = loop.submit(r.ctx, j.idx, "bh")
        j.state = "walking"

    def _advance(self, j: Job, r: Resident, now: float) -> bool:
        """True when the job finished."""
        if self.loops[j.req.precision].poll(j.ticket):
            j.state = "done"
            j.done_s = now
            return True
        return False

    # -- the loop ---------------------------------------------------------------
    def run(self, requests, progress=None, stall_s: float = 60.0):
        """Serve ``requests`` (arrival times in seconds) and return (Stats,
        jobs).  Active subsets are drawn and uploaded beforehand.  progress, if
        given, is called with (finished, total) about every 5 s; a run in which
        nothing finishes for stall_s seconds while requests are in flight
        raises RuntimeError naming them."""
        stats = Stats()
        jobs = []
        for sid in sorted({rq.sid for rq in requests}):
            self._particles(sid)  # host-side generation stays out of the clock
        for rq in requests:
            n = self.pool[rq.sid].n
            idx = torch.as_tensor(W.request_active(rq, n), dtype=torch.int32, device=self.dev)
            jobs.append(Job(rq, (rq.sid, rq.precision), idx))
        launches0 = sum(lp.info()["launches"] for lp in self.loops.values())
        torch.cuda.synchronize()
        pending = deque(sorted(jobs, key=lambda j: j.req.t_arrival))
        waiting = []        # arrived, not admitted (memory)
        finished = 0
        t0 = time.perf_counter()
        last_done, last_report = 0.0, 0.0
        while finished < len(jobs):
            now = time.perf_counter() - t0
            if progress is not None and now - last_report > 5.0:
                progress(finished, len(jobs))
                last_report = now
            if now - last_done > stall_s:
                flying = [(r.key, r.active.ticket) for r in self.resident.values()
                          if r.active is not None]
                raise RuntimeError(f"no request finished for {stall_s} s; in flight: {flying}")
            before = finished
            # arrivals
            while pending and pending[0].req.t_arrival <= now:
                waiting.append(pending.popleft())
            # admission, in arrival order
            still = []
            for j in waiting:
                if self._admit(j, stats):
                    j.state = "queued"
                elif j.rejected:
                    finished += 1
                else:
                    still.append(j)
            waiting = still
            # per resident system: advance the job in flight, start the next
            busy = False
            for r in list(self.resident.values()):
                if r.active is not None:
                    busy = True
                    if self._advance(r.active, r, now):
                        finished += 1
                        r.active = None
                        r.last_used = now
                if r.active is None and r.queue and r.ready.query():
                    r.active = r.queue.popleft()
                    self._start(r.active, r)
                    busy = True
            if finished != before or (not busy and not waiting):
                last_done = now
            if not busy and not waiting:
                time.sleep(5e-5)
        torch.cuda.synchronize()
        stats.wall_s = time.perf_counter() - t0
        stats.rejected = sum(j.rejected for j in jobs)
        stats.kernel_launches = sum(lp.info()["launches"] for lp in self.loops.values()) - \
            launches0
        served = [j for j in jobs if not j.rejected]
        if served:
            first = min(j.req.t_arrival for j in served)
            last = max(j.done_s for j in served)
            stats.span_ms = (last - first) * 1e3
        for j in served:
            stats.latencies_ms.append((j.done_s - j.req.t_arrival) * 1e3)
            stats.force_evals += j.idx.numel()
        return stats, jobs

    def close(self):
        for lp in self.loops.values():
            lp.close()
        for r in self.resident.values():
            r.ctx.close()
        self.resident.clear()


def total_force(job: Job):
    """Tree (+ PM) acceleration of a finished job, [3][n_act]."""
    return job.acc if job.acc_pm is None else job.acc + job.acc_pm
