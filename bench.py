#!/usr/bin/env python3
"""Benchmark of the TreePM force step on one MI355X.

One step = the whole hot path on all particles of the workload, as the
Arepo paper computes a force the first time (Sec. 3.1: geometric criterion
first, then the relative criterion with |a| of that first pass):

    build_tree -> pm_long_range (deposit, FFT solve, difference, interpolate)
    -> compute_forces(BH) -> |a_tree + a_pm| -> compute_forces(relative)

Default (headline) workload: the clustered periodic box, the largest
single-GPU configuration: L = 100, 256^3 particles drawn from a lognormal
density field (sigma_ln = 2, Gaussian field with P(k) ~ k^-2), eps = L/12800,
TreePM with a 256^3 mesh, r_s = 1.25 cells, r_cut = 4.5 r_s, theta = 0.5,
alpha = 0.0025; inputs are resident in HBM.  The value is force evaluations
per second (N per step); FP32 is the headline, the FP64 path is measured
beside it.  The other workloads (Plummer 4096, Hernquist 2^20, the 128^3
Zel'dovich box, active time-bin subsets, isolated TreePM, individual
softening, time integration, serving) are reported as entries of the same
line.  Kernel classes are timed by the library's own events around their
launches; the roofline denominators are also measured in the same run; the
FP64 CPU oracle is timed on a bounded sample of the headline workload.

Prints ONE JSON line.
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

METRIC = "particle force evals/s + p50/p99 latency, FP32 vs FP64 at 99%-ile err<=1%"

# Algorithmic flops per interaction (FMA = 2): Newtonian monopole or pair:
# 3 sub + r^2 (1 mul + 2 fma) + rinv^2, m rinv^3 (3 mul) + 3 fma accumulate
# = 17 (+1 rsqrt); the short-range factor adds r, x = r / 2 r_s, exp(-x^2),
# erfc(x), the combination and the product: 19 (+ exp, rcp).
FLOPS_NEWTON = 17
FLOPS_TREEPM = 17 + 19
PEAK = {"fp32": 157.3, "fp64": 78.6}  # TFLOP/s, MI355X vector ALU


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=4, choices=[2, 3, 4])
    ap.add_argument("--precision", default="both", choices=["both", "fp32", "fp64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-scale", type=int, default=2,
                    help="the oracle runs the headline generator with ng / cpu-scale cells per "
                         "side (mesh likewise): a bounded sample of the workload")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the local-timestep and serving legs")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="finish with one plain device copy of MIB MiB (calibrates the "
                         "profiler's HBM byte counters)")
    return ap.parse_args()


def workload(cfg):
    from paper_1909_04667_amd import workloads as W
    c = W.CONFIGS[cfg]
    p = W.make_config(cfg)
    kw = dict(eps=c["eps"], theta=c["theta"], alpha=c.get("alpha", 0.0025))
    if c["periodic"]:
        kw.update(periodic=True, box_size=c["box"], pm_grid=c["pm_grid"], asmth=c["asmth"],
                  rcut=c["rcut"])
    return c, p, kw


def run_gpu(p, kw, prec, steps, warmup, eps=None):
    import torch
    from paper_1909_04667_amd import binding as B
    dev = torch.device("cuda:0")
    t = lambda a, dt=torch.float64: torch.as_tensor(a, dtype=dt, device=dev).contiguous()
    x, y, z = t(p.x), t(p.y), t(p.z)
    n = p.n
    idx = torch.arange(n, dtype=torch.int32, device=dev)
    ctx = B.Context(precision=prec, **kw)
    dt = ctx.dtype
    acc_pm = torch.empty((3, n), dtype=dt, device=dev)
    acc_bh = torch.empty((3, n), dtype=dt, device=dev)
    acc = torch.empty((3, n), dtype=dt, device=dev)
    anorm = torch.zeros(n, dtype=torch.float64, device=dev)
    nint_bh = torch.empty(n, dtype=torch.int32, device=dev)
    nint = torch.empty(n, dtype=torch.int32, device=dev)
    has_pm = kw.get("pm_grid", 0) > 0

    def step():
        ctx.build_tree(x, y, z, eps=eps)
        if has_pm:
            ctx.pm_long_range(idx, acc=acc_pm)
        ctx.compute_forces(idx, "bh", acc=acc_bh, n_interactions=nint_bh)
        ctx.accel_norm(idx, acc_bh, acc_pm if has_pm else None, out=anorm)
        ctx.compute_forces(idx, "rel", a_old_norm=anorm, acc=acc, n_interactions=nint)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.check()
    for k in ctx.TIMERS:
        ctx.timing_read(k)  # drop warm-up records
    ctx.timing(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for s in range(steps):
        step()
        ev[s + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.timing(False)
    per_step = [ev[s].elapsed_time(ev[s + 1]) for s in range(steps)]
    durations = {k: ctx.timing_durations(k) for k in ctx.TIMERS}
    timers = {k: (sum(v), len(v)) for k, v in durations.items()}
    ctx.check()
    inter_bh = int(nint_bh.to(torch.int64).sum())
    inter_rel = int(nint.to(torch.int64).sum())
    total = (acc + acc_pm) if has_pm else acc
    out = dict(prec=prec, ms_per_step=sum(per_step) / steps, per_step=per_step, wall=wall,
               timers=timers, durations=durations, inter_bh=inter_bh, inter_rel=inter_rel, n=n,
               acc=total.double().cpu(), entries=ctx.tree_info()[1])
    ctx.close()
    return out


def run_local_timestep(steps, prec="fp32", wl=None):
    """Clustered 256^3 box: one build (+ PM solve) reused by every active set;
    per set the PM interpolation and the relative-criterion walk with |a| of
    a full geometric pass (the previous step's accelerations)."""
    import numpy as np
    import torch
    from paper_1909_04667_amd import binding as B
    from paper_1909_04667_amd import workloads as W
    c, p, kw = wl if wl is not None else workload(4)
    sets, bins = W.time_bin_active_sets(p.meta["rho"])
    dev = torch.device("cuda:0")
    t = lambda a, dt=torch.float64: torch.as_tensor(a, dtype=dt, device=dev).contiguous()
    x, y, z = t(p.x), t(p.y), t(p.z)
    ctx = B.Context(precision=prec, **kw)
    ctx.timing(True)
    ctx.build_tree(x, y, z)
    all_idx = torch.arange(p.n, dtype=torch.int32, device=dev)
    apm, _ = ctx.pm_long_range(all_idx)
    a0, _ = ctx.compute_forces(all_idx, "bh")
    anorm = ctx.accel_norm(all_idx, a0, apm)
    torch.cuda.synchronize()
    for k in ctx.TIMERS:
        ctx.timing_read(k)
    # rebuild timing (the tree is rebuilt per step in the paper's scheme)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(steps):
        ctx.build_tree(x, y, z)
        ctx.pm_long_range(all_idx[:0])
    ev[1].record()
    torch.cuda.synchronize()
    build_ms = ctx.timing_read("build")[0] / steps
    solve_ms = ctx.timing_read("pm_solve")[0] / steps
    out = {"workload": c["name"], "n_particles": p.n, "build_ms": build_ms,
           "pm_solve_ms": solve_ms, "tree_entries": ctx.tree_info()[1], "sets": {}}
    for f, ids in sets.items():
        idx = t(ids, torch.int32)
        acc = torch.empty((3, idx.numel()), dtype=ctx.dtype, device=dev)
        accl = torch.empty_like(acc)
        for _ in range(2):
            ctx.pm_long_range(idx, acc=accl)
            ctx.compute_forces(idx, "rel", a_old_norm=anorm, acc=acc)
        for k in ctx.TIMERS:
            ctx.timing_read(k)  # drop the warm-up records
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(steps):
            ctx.pm_long_range(idx, acc=accl)
            ctx.compute_forces(idx, "rel", a_old_norm=anorm, acc=acc)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / steps
        walk_ms = ctx.timing_read("walk_rel")[0] / steps
        interp_ms = ctx.timing_read("pm_interp")[0] / steps
        out["sets"][str(f)] = {"n_active": int(idx.numel()), "forces_ms": ms, "walk_ms": walk_ms,
                               "pm_interp_ms": interp_ms,
                               "force_evals_per_s": idx.numel() / (ms * 1e-3),
                               "with_rebuild_evals_per_s":
                                   idx.numel() / ((ms + build_ms + solve_ms) * 1e-3)}
    ctx.check()
    ctx.close()
    return out


def run_isolated(steps, warmup, pm_grid=128):
    """TreePM for an isolated system (Sec. 3.3 zero-padded mesh): the
    Hernquist 2^20 sphere with a pm_grid mesh over its root cube, padded to
    (2 pm_grid)^3; the same step as the headline (build, PM, BH, |a|,
    relative), FP32 and FP64."""
    c, p, kw = workload(2)
    kw = dict(kw, pm_grid=pm_grid, asmth=1.25, rcut=4.5)
    out = {"workload": f"{c['name']}_isolated_pm{pm_grid}", "n_particles": p.n,
           "pm_grid": pm_grid, "padded_fft": 2 * pm_grid}
    for prec in ("fp32", "fp64"):
        r = run_gpu(p, kw, prec, steps, warmup)
        t = r["timers"]
        out[prec] = {"ms_per_step": r["ms_per_step"],
                     "force_evals_per_s": r["n"] / (r["ms_per_step"] * 1e-3),
                     "kernel_ms": {k: t[k][0] / max(t[k][1], 1) for k in
                                   ("walk", "walk_rel", "build", "pm_solve", "pm_interp")},
                     "interactions_per_particle_rel": r["inter_rel"] / r["n"]}
    return out


def run_mixed_softening(steps, warmup):
    """Individual softening lengths (Sec. 3.2) on the Hernquist 2^20 step
    (build, BH, |a|, relative walk): log-normal spread around eps, against
    the uniform-softening step on the same positions."""
    import numpy as np
    import torch
    c, p, kw = workload(2)
    eps_arr = kw["eps"] * np.exp(np.random.default_rng(21).normal(0.0, 0.7, p.n))
    out = {"workload": f"{c['name']}_individual_softening", "n_particles": p.n,
           "eps_spread": "log-normal, sigma 0.7 (natural log)"}
    for prec in ("fp32", "fp64"):
        r = run_gpu(p, kw, prec, steps, warmup,
                    eps=torch.as_tensor(eps_arr, dtype=torch.float64, device="cuda:0"))
        out[prec] = {"ms_per_step": r["ms_per_step"],
                     "force_evals_per_s": r["n"] / (r["ms_per_step"] * 1e-3),
                     "interactions_per_particle_rel": r["inter_rel"] / r["n"]}
    return out


def run_integrators():
    """Sec. 7.2-7.3, one longest step dt_max of the block-step leapfrog and of
    the split-Hamiltonian integration, FP32 walks, six bins:
    * a 2^18 Hernquist sphere (tree forces), C = 0.025;
    * a clustered periodic box (64^3 particles, lognormal density, TreePM with a
      128^3 mesh), where block steps rebuild the tree and solve the mesh at
      every sync point while the split solves the mesh twice per longest step
      and builds trees over the fast parts only; dt_max is set so that half
      of the particles ask for a shorter step than dt_max (C = 0.025)."""
    import numpy as np
    import torch
    from paper_1909_04667_amd import binding as B
    from paper_1909_04667_amd import integrate as GI
    from paper_1909_04667_amd import workloads as W
    dev = torch.device("cuda:0")
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)

    def one(name, cls, p, v, **kw):
        integ = cls((t(p.x), t(p.y), t(p.z)), (t(v[0]), t(v[1]), t(v[2])), **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = integ.run(1)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        occ = np.bincount(integ.bins.cpu().numpy(), minlength=kw["max_bin"] + 1).tolist()
        integ.ctx.close()
        return {"wall_ms": wall * 1e3, "force_evals": st["force_evals"],
                "force_evals_per_s": st["force_evals"] / wall, "final_bins": occ,
                **{k: v for k, v in st.items() if k != "force_evals"}}

    p = W.hernquist(1 << 18, 31)
    rng = np.random.default_rng(32)
    r = np.sqrt(p.x ** 2 + p.y ** 2 + p.z ** 2)
    vc = np.sqrt(r) / (1.0 + r)  # circular speed of a Hernquist sphere (G = M = a = 1)
    v = rng.normal(0.0, 1.0, (3, p.n)) * (vc / np.sqrt(3.0))
    out = {"hernquist_2p18_kdk": {"n_particles": p.n, "C": 0.025, "dt_max": 0.05,
                                  "max_bin": 6}}
    for name, cls in (("block_leapfrog", GI.BlockLeapfrog), ("hierarchical", GI.Hierarchical)):
        out["hernquist_2p18_kdk"][name] = one(name, cls, p, v, C=0.025, dt_max=0.05, max_bin=6,
                                              precision="fp32", eps=0.005)
    # clustered periodic box with the mesh
    box, ng = 100.0, 128
    p = W.lognormal_box(64, box, 33)
    eps = box / (50 * 64)
    kw = dict(precision="fp32", eps=eps, periodic=True, box_size=box, pm_grid=ng)
    ctx = B.Context(**kw)
    ctx.build_tree(t(p.x), t(p.y), t(p.z))
    idx = torch.arange(p.n, dtype=torch.int32, device=dev)
    a, _ = ctx.compute_forces(idx, "bh")
    apm, _ = ctx.pm_long_range(idx)
    an = (a.double() + apm.double()).norm(dim=0).cpu().numpy()
    ctx.close()
    C = 0.025
    dt_max = float(np.median(np.sqrt(2.0 * C * eps / an)))
    v = np.random.default_rng(34).normal(0.0, 1.0, (3, p.n)) * (0.02 * box / dt_max)
    wl = {"n_particles": p.n, "pm_grid": ng, "C": C, "dt_max": dt_max, "max_bin": 6}
    for name, cls in (("block_leapfrog", GI.BlockLeapfrog), ("hierarchical", GI.Hierarchical)):
        wl[name] = one(name, cls, p, v, C=C, dt_max=dt_max, max_bin=6, **kw)
    wl["hierarchical_wall_vs_block"] = wl["hierarchical"]["wall_ms"] / \
        wl["block_leapfrog"]["wall_ms"]
    out["lognormal_64c_pm128_kdk"] = wl
    return out


def run_serving(n_poisson=4000, n_burst=2000, n_systems=16, seed=5):
    """Continuous batching through the device-resident request loop over a
    pool of resident systems: capacity from a burst of n_burst requests all
    present at t = 0, then n_poisson Poisson arrivals at 0.5, 0.7 and 0.9 of
    that capacity; latency = completion observed on the host - arrival.  The
    burst's first 500 requests are also served one at a time through the
    single-system path (tpm_compute_forces) for comparison."""
    import torch
    from paper_1909_04667_amd import serve as S
    from paper_1909_04667_amd import workloads as W
    pool = W.system_pool(n_systems, seed=seed)
    burst = W.request_stream(n_burst, rate=0.0, n_systems=n_systems, seed=seed)
    srv = S.Server(pool, budget_bytes=64 << 30)
    srv.run(burst[:n_systems * 4])  # warm-up: builds every resident system
    log("serving: systems resident")
    prog = lambda k, n: log(f"serving: {k}/{n} finished")
    st, _ = srv.run(burst, progress=prog)
    cap = st.summary()
    log(f"serving: burst capacity {cap['throughput_evals_per_s']:.3e} evals/s")
    req_rate = cap["requests"] / (st.span_ms * 1e-3)
    out = {"systems": n_systems, "n_range": [min(s.n for s in pool), max(s.n for s in pool)],
           "burst_requests": n_burst, "poisson_requests_per_load": n_poisson,
           "precisions": "fp32+fp64 mix", "loop": "device-resident (tpm_server_*)",
           "capacity": {"force_evals_per_s": cap["throughput_evals_per_s"],
                        "requests_per_s": req_rate, "p50_ms": cap["p50_ms"],
                        "p99_ms": cap["p99_ms"],
                        "server_kernel_launches": cap["server_kernel_launches"]}}
    for load in (0.5, 0.7, 0.9):
        stream = W.request_stream(n_poisson, rate=load * req_rate, n_systems=n_systems,
                                  seed=seed + 100 + int(10 * load))
        st2, _ = srv.run(stream, progress=prog)
        s2 = st2.summary()
        log(f"serving: load {load} p50 {s2['p50_ms']:.2f} ms p99 {s2['p99_ms']:.2f} ms")
        out[f"poisson_{load}"] = {"force_evals_per_s": s2["throughput_evals_per_s"],
                                  "p50_ms": s2["p50_ms"], "p99_ms": s2["p99_ms"],
                                  "max_ms": s2["max_ms"], "rejected": s2["rejected"],
                                  "server_kernel_launches": s2["server_kernel_launches"]}
    # the same mix, one request at a time through the single-system path
    seq = burst[:500]
    jobs = []
    for rq in seq:
        n = pool[rq.sid].n
        idx = torch.as_tensor(W.request_active(rq, n), dtype=torch.int32, device="cuda:0")
        jobs.append((rq, idx))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evals = 0
    for rq, idx in jobs:
        r = srv.resident[(rq.sid, rq.precision)]
        ctx = r.ctx
        with torch.cuda.stream(r.stream):
            a, _ = ctx.compute_forces(idx, "bh")
            apm = ctx.pm_long_range(idx)[0] if r.periodic else None
            if len(r.stages) > 1:
                an = ctx.accel_norm(idx, a, apm)
                a, _ = ctx.compute_forces(idx, "rel", a_old_norm=an)
        r.stream.synchronize()
        evals += idx.numel()
    dt = time.perf_counter() - t0
    out["same_mix_one_at_a_time"] = {"requests": len(seq), "force_evals_per_s": evals / dt}
    out["capacity_vs_one_at_a_time"] = cap["throughput_evals_per_s"] / (evals / dt)
    srv.close()
    return out


def counted_traffic(workload, kernel):
    """HBM bytes per launch of the dominant walk kernel from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE, each scaled by a copy probe),
    or None when the summary is missing, covers another workload, or the
    kernel's sources changed after the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_walk32_rel_{workload}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    rec = None
    with open(path) as f:
        for line in f:
            if line.startswith("traffic: "):
                rec = json.loads(line[len("traffic: "):])
    if rec is None or rec.get("workload") != workload or rec.get("kernel") != kernel:
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec["bytes_per_launch"]


def pct(v, q):
    v = sorted(v)
    if not v:
        return float("nan")
    k = min(len(v) - 1, max(0, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[k]


def pass_bytes(n, E, ng, prec, periodic, masses=False):
    """Algorithmic HBM bytes of one build and one mesh solve, per pass: what
    each pass must read and write at least once (caches absorb the rest).
    n particles, E depth-first entries (E - n nodes), ng mesh cells per side
    (0: none), prec "fp32"/"fp64"."""
    nodes = E - n
    t = 4 if prec == "fp32" else 8
    b = {}
    # root cube (isolated: one read of the positions) and keys: positions (and
    # masses) in, key, index and the packed 32-byte position/mass record out
    b["keys"] = (0 if periodic else 24 * n) + (32 if masses else 24) * n + 12 * n + 32 * n
    # digit histograms (one read of the keys) + 8 passes of (key, index) in and out
    b["sort"] = 8 * n + 8 * 24 * n
    # index in, the packed records gathered, permutation, rank, curve-order
    # positions, masses and packed integer coordinates out
    b["gather"] = 4 * n + 32 * n + 4 * n + 4 * n + 24 * n + 8 * n + 8 * n
    # counts (keys in, depth and count out), scan of the counts (two reads, two
    # writes), emission (keys, depths, bases, positions, masses, integer
    # coordinates in; 64-byte records, first/count words, particle entries and
    # level lists out)
    b["topology"] = (13 * n + 16 * n + (8 + 1 + 4 + 24 + 8 + 8) * n + 72 * E + 4 * n
                     + 4 * nodes)
    # moments: every entry read once as a child, every node written with its
    # count
    b["moments"] = 64 * E + 4 * E + 68 * nodes
    if prec == "fp32":
        # FP32 records: the emission writes a particle's (32 B), the moments a
        # node's (its first particle's packed coordinates in, 32 B out)
        b["topology"] += 32 * n
        b["moments"] += (8 + 32) * nodes
    if ng:
        M = ng if periodic else 2 * ng
        m3 = M ** 3
        planes = 1 if prec == "fp32" else 2
        half = M * M * (M // 2 + 1) * 2 * t
        # clear and one write of every fixed-point cell, positions and masses in
        b["deposit"] = 2 * planes * 8 * m3 + 32 * n
        # five passes over the half spectrum; the first reads the fixed-point
        # mesh, the last writes the real potential
        b["fft"] = planes * 8 * m3 + half + 3 * 2 * half + half + m3 * t
    return b


def interp_bytes(n_act, ng, prec, periodic):
    """Mesh interpolation of n_act targets: slot and position in, the
    potential mesh once, results out and scattered to caller order."""
    t = 4 if prec == "fp32" else 8
    M = ng if periodic else 2 * ng
    return n_act * (4 + 24 + 4 * t) + M ** 3 * t + n_act * (12 + 4 * t + 4 * t)


def run_config1(steps, warmup):
    """Plummer sphere, N = 4096, eps = 0.01, geometric criterion theta = 0.5,
    all particles, one evaluation (build + walk) in FP64 and FP32; the tree's
    error against the direct sum (and after a relative pass, the paper's
    second force computation) from the GPU's FP64 forces."""
    import numpy as np
    import torch
    import oracle as O
    from paper_1909_04667_amd import binding as B
    from paper_1909_04667_amd import workloads as W
    p = W.plummer(4096, 1)
    dev = torch.device("cuda:0")
    t = lambda a, dt=torch.float64: torch.as_tensor(a, dtype=dt, device=dev).contiguous()
    x, y, z = t(p.x), t(p.y), t(p.z)
    idx = torch.arange(p.n, dtype=torch.int32, device=dev)
    out = {"workload": "plummer_4096", "n_particles": p.n, "eps": 0.01, "theta": 0.5,
           "step": "build + BH walk, all particles"}
    accs = {}
    for prec in ("fp64", "fp32"):
        ctx = B.Context(precision=prec, eps=0.01, theta=0.5)
        acc = torch.empty((3, p.n), dtype=ctx.dtype, device=dev)

        def step():
            ctx.build_tree(x, y, z)
            ctx.compute_forces(idx, "bh", acc=acc)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record()
        for s_ in range(steps):
            step()
            ev[s_ + 1].record()
        torch.cuda.synchronize()
        ctx.check()
        per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
        ms = sum(per) / steps
        out[prec] = {"ms_per_step": ms, "force_evals_per_s": p.n / (ms * 1e-3),
                     "latency_ms": {"p50": pct(per, 50), "p99": pct(per, 99)}}
        accs[prec] = acc.double().cpu().numpy()
        if prec == "fp64":
            an = ctx.accel_norm(idx, acc)
            ar, _ = ctx.compute_forces(idx, "rel", a_old_norm=an)
            accs["rel"] = ar.cpu().numpy()
        ctx.close()
    ad, _ = O.direct(p.x, p.y, p.z, None, O.make_params(eps=0.01))

    def err(a, ref):
        na = np.linalg.norm(ref, axis=0)
        return np.linalg.norm(a - ref, axis=0) / np.maximum(na, 1e-3 * np.sqrt(np.mean(na ** 2)))
    e64, erel, e32 = err(accs["fp64"], ad), err(accs["rel"], ad), err(accs["fp32"], accs["fp64"])
    out["error_vs_direct"] = {
        "bh_theta0.5_fp64": {"p50": float(np.percentile(e64, 50)),
                             "p99": float(np.percentile(e64, 99))},
        "after_relative_alpha0.0025_fp64": {"p50": float(np.percentile(erel, 50)),
                                            "p99": float(np.percentile(erel, 99))}}
    out["fp32_vs_fp64_err"] = {"p99": float(np.percentile(e32, 99)), "max": float(e32.max())}
    return out


def run_config2(steps, warmup, sample=1024):
    """Hernquist sphere, N = 2^20: the step (build, BH, |a|, relative) in FP64
    and FP32; FP32 against FP64 over all targets; the relative pass against
    the direct sum on sampled targets."""
    import numpy as np
    import oracle as O
    c, p, kw = workload(2)
    out = {"workload": c["name"], "n_particles": p.n, "eps": kw["eps"], "theta": kw["theta"],
           "alpha": kw["alpha"], "step": "build + BH walk + |a| + relative walk, all particles"}
    res = {}
    for prec in ("fp32", "fp64"):
        r = run_gpu(p, kw, prec, steps, warmup)
        res[prec] = r
        out[prec] = {"ms_per_step": r["ms_per_step"],
                     "force_evals_per_s": r["n"] / (r["ms_per_step"] * 1e-3),
                     "latency_ms": {"p50": pct(r["per_step"], 50),
                                    "p99": pct(r["per_step"], 99)},
                     "kernel_ms": kernel_ms(r),
                     "interactions_per_particle_rel": r["inter_rel"] / r["n"],
                     "interactions_per_s_rel":
                         r["inter_rel"] / (r["timers"]["walk_rel"][0] / r["timers"]["walk_rel"][1]
                                           * 1e-3)}
    a32, a64 = res["fp32"]["acc"].numpy(), res["fp64"]["acc"].numpy()
    na = np.linalg.norm(a64, axis=0)
    e = np.linalg.norm(a32 - a64, axis=0) / np.maximum(na, 1e-3 * np.sqrt(np.mean(na ** 2)))
    out["fp32_vs_fp64_err"] = {"p50": float(np.percentile(e, 50)),
                               "p99": float(np.percentile(e, 99)), "max": float(e.max())}
    out["fp32_speedup_vs_fp64"] = res["fp64"]["ms_per_step"] / res["fp32"]["ms_per_step"]
    samp = np.sort(np.random.default_rng(0).choice(p.n, sample, replace=False))
    ad, _ = O.direct(p.x, p.y, p.z, None, O.make_params(eps=kw["eps"]), targets=samp)
    nd = np.linalg.norm(ad, axis=0)
    er = np.linalg.norm(a64[:, samp] - ad, axis=0) / np.maximum(
        nd, 1e-3 * np.sqrt(np.mean(nd ** 2)))
    out["error_vs_direct_fp64"] = {"targets": int(sample), "p50": float(np.percentile(er, 50)),
                                   "p99": float(np.percentile(er, 99))}
    return out


def kernel_ms(r):
    """Mean milliseconds per step of every timed kernel class."""
    steps = len(r["per_step"])
    return {k: v[0] / steps for k, v in r["timers"].items() if v[1]}


def cpu_baseline(c, kw, scale):
    """The FP64 oracle on the host, on a bounded sample of the headline
    workload: the same generator and settings with ng / scale particles per
    side and a mesh of pm_grid / scale cells (r_s and r_cut in mesh cells
    unchanged), the whole step on every particle: single-threaded tree build
    and mesh solve, both walks on all threads.  The GPU's FP64 step on the
    same sample is compared with the oracle's (each side's relative pass uses
    its own |a| from its own first pass)."""
    import numpy as np
    import oracle as O
    from paper_1909_04667_amd import workloads as W
    ngp = c["ng"] // scale
    ngm = kw["pm_grid"] // scale
    p = (W.lognormal_box if c["kind"] == "lognormal" else W.zeldovich_box)(ngp, c["box"],
                                                                           c["seed"])
    box = kw["box_size"]
    eps = box / (50 * ngp)
    rs = kw["asmth"] * box / ngm
    t0 = time.perf_counter()
    T = O.Tree(p.x, p.y, p.z, periodic=True, box=box)
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    apm, _ = O.pm(p.x, p.y, p.z, None, box, ngm, 1.0, rs, want_pot=False)
    t_pm = time.perf_counter() - t0
    Pb = O.make_params(periodic=True, box=box, eps=eps, theta=kw["theta"], treepm=True, rs=rs,
                       rcut=kw["rcut"] * rs)
    t0 = time.perf_counter()
    a, _, _ = T.walk(Pb)
    t_bh = time.perf_counter() - t0
    an = np.linalg.norm(a + apm, axis=0)
    Pr = O.make_params(periodic=True, box=box, eps=eps, opening="rel", alpha=kw["alpha"],
                       treepm=True, rs=rs, rcut=kw["rcut"] * rs)
    t0 = time.perf_counter()
    ar, _, _ = T.walk(Pr, anorm=an)
    t_rel = time.perf_counter() - t0
    step = t_build + t_pm + t_bh + t_rel
    # the GPU's FP64 step on the same sample
    kws = dict(kw, eps=eps, pm_grid=ngm)
    g = run_gpu(p, kws, "fp64", 1, 1)
    ref = ar + apm
    nr = np.linalg.norm(ref, axis=0)
    e = np.linalg.norm(g["acc"].numpy() - ref, axis=0) / np.maximum(
        nr, 1e-3 * np.sqrt(np.mean(nr ** 2)))
    return {"value": p.n / step, "unit": "force evals/s", "cores": O.max_threads(),
            "kind": "oracle",
            "sample": (f"{c['name']} generator at {ngp}^3 particles with a {ngm}^3 mesh "
                       f"(1/{scale ** 3} of the particles; eps = L/(50 x {ngp}), r_s and r_cut "
                       f"in mesh cells as in the workload): the whole step on all {p.n} "
                       f"particles, tree build ({t_build:.1f} s) and mesh solve ({t_pm:.1f} s) "
                       f"single-threaded, BH + relative walks ({t_bh + t_rel:.1f} s) on "
                       f"{O.max_threads()} threads"),
            "seconds": {"build": t_build, "pm": t_pm, "walk_bh": t_bh, "walk_rel": t_rel,
                        "step": step},
            "gpu_fp64_vs_oracle_err": {"p50": float(np.percentile(e, 50)),
                                       "p99": float(np.percentile(e, 99)),
                                       "max": float(e.max()),
                                       "note": "each side's relative pass uses its own |a|"}}


def summary(r, periodic, masses=False):
    ms_rel, k_rel = r["timers"]["walk_rel"]
    ms_bh, k_bh = r["timers"]["walk"]
    steps = len(r["per_step"])
    km = kernel_ms(r)
    # the build's time outside its kernels: the one host synchronisation that
    # sizes the node arrays
    inner = sum(km.get(k, 0.0) for k in ("keys", "sort", "gather", "topology", "moments"))
    ng = r.get("pm_grid", 0)
    pb = pass_bytes(r["n"], r["entries"], ng, r["prec"], periodic, masses)
    if ng:
        pb["interp"] = interp_bytes(r["n"], ng, r["prec"], periodic)
    gbs = {}
    for k, nbytes in pb.items():
        tk = {"interp": "pm_interp"}.get(k, k)
        if km.get(tk):
            gbs[k] = {"ms": km[tk], "algorithmic_bytes": nbytes,
                      "GB_per_s": nbytes / (km[tk] * 1e-3) / 1e9,
                      "frac_of_8TBps": nbytes / (km[tk] * 1e-3) / 8e12}
    return {
        "value": r["n"] / (r["ms_per_step"] * 1e-3),
        "ms_per_step": r["ms_per_step"],
        "latency_ms": {"p50": pct(r["per_step"], 50), "p99": pct(r["per_step"], 99)},
        "kernel_ms": km,
        "build_gap_ms": km.get("build", 0.0) - inner,
        "kernel_ms_p50_p99": {
            name: [pct(r["durations"][k], 50), pct(r["durations"][k], 99)]
            for name, k in (("walk_rel", "walk_rel"), ("walk_bh", "walk"),
                            ("build", "build"), ("sort", "sort"),
                            ("pm_solve", "pm_solve"), ("pm_interp", "pm_interp"))
            if r["durations"][k]},
        "pass_GB_per_s": gbs,
        "walk_rel_ms_per_launch": ms_rel / max(k_rel, 1),
        "walk_bh_ms_per_launch": ms_bh / max(k_bh, 1),
        "interactions_per_step": {"bh": r["inter_bh"], "rel": r["inter_rel"]},
        "interactions_per_particle_rel": r["inter_rel"] / r["n"],
        "tree_entries": r["entries"],
    }


def measured_peaks():
    from paper_1909_04667_amd import binding as B
    return {"fp32_fma_unpacked_tflops": B.probe_fma("fp32"),
            "fp64_fma_tflops": B.probe_fma("fp64"),
            "copy_GB_per_s": B.probe_copy(1 << 30),
            "note": "dependent vector FMAs (FMA = 2 flops; FP32 without packed instructions, "
                    "as the library is built) and a 1 GiB streaming copy (read + write), "
                    "best of five launches"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "only one GPU is measured: the library runs the whole path "
                          "on a single device and has no multi-GPU code", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    peaks = measured_peaks()
    log(f"measured peaks {peaks}")
    c, p, kw = workload(args.config)
    log(f"workload {c['name']} N={p.n} ready")
    precs = ["fp32", "fp64"] if args.precision == "both" else [args.precision]
    periodic = bool(kw.get("periodic"))
    res = {}
    for pr in precs:
        res[pr] = run_gpu(p, kw, pr, args.steps, args.warmup)
        res[pr]["pm_grid"] = kw.get("pm_grid", 0)
        log(f"{pr}: {res[pr]['ms_per_step']:.3f} ms/step")
    fl = FLOPS_TREEPM if kw.get("pm_grid", 0) else FLOPS_NEWTON
    out_prec = {pr: summary(r, periodic) for pr, r in res.items()}
    h = out_prec[precs[0]]
    walk_ms = h["walk_rel_ms_per_launch"]
    achieved = res[precs[0]]["inter_rel"] * fl / (walk_ms * 1e-3) / 1e12
    per, tpm = ("true", "true") if periodic else ("false", "false")
    walk_kernel = (f"k_walk32<{per}, {tpm}, 1, false, false>" if precs[0] == "fp32"
                   else f"k_walk64{'i' if periodic else ''}<{per}, {tpm}, 1, false, false>")
    meas = peaks["fp32_fma_unpacked_tflops" if precs[0] == "fp32" else "fp64_fma_tflops"]
    line = {
        "metric": METRIC,
        "value": h["value"],
        "unit": "force evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64"}[precs[0]],
        "data": "synthetic",
        "config": {"workload": c["name"], "n_particles": p.n, "box": kw.get("box_size"),
                   "pm_grid": kw.get("pm_grid"), "eps": kw["eps"], "theta": kw["theta"],
                   "alpha": kw["alpha"], "asmth": kw.get("asmth"), "rcut": kw.get("rcut"),
                   "step": "build + PM + BH walk + |a| + relative walk, all particles",
                   "parallelism": "single GPU"},
        "latency_ms": h["latency_ms"],
        "per_precision": out_prec,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK[precs[0]],
                     "unit": "TFLOP/s", "frac": achieved / PEAK[precs[0]],
                     "traffic": counted_traffic(c["name"], walk_kernel),
                     "kernel": walk_kernel, "flops_per_interaction": fl,
                     "interactions_per_launch": res[precs[0]]["inter_rel"],
                     "launch_ms": walk_ms,
                     "measured_peak": meas, "frac_of_measured_peak": achieved / meas},
        "measured_peaks": peaks,
    }
    if len(precs) == 2:
        a32, a64 = res["fp32"]["acc"].numpy(), res["fp64"]["acc"].numpy()
        na = np.linalg.norm(a64, axis=0)
        e = np.linalg.norm(a32 - a64, axis=0) / np.maximum(na, 1e-3 * np.sqrt(np.mean(na ** 2)))
        line["fp32_vs_fp64_err"] = {"p50": float(np.percentile(e, 50)),
                                    "p99": float(np.percentile(e, 99)),
                                    "max": float(e.max())}
        line["fp32_speedup_vs_fp64"] = out_prec["fp64"]["ms_per_step"] / h["ms_per_step"]
    del res
    if not args.no_extra:
        line["configs"] = {}
        log("config 1: Plummer 4096")
        line["configs"]["1"] = run_config1(max(10, args.steps), args.warmup)
        log("config 2: Hernquist 2^20")
        line["configs"]["2"] = run_config2(max(3, args.steps // 2), 2)
        if args.config != 3:
            log("config 3: Zel'dovich 128^3, 256^3 mesh")
            c3, p3, kw3 = workload(3)
            r3 = {}
            for pr in ("fp32", "fp64"):
                r3[pr] = run_gpu(p3, kw3, pr, max(3, args.steps // 2), 2)
                r3[pr]["pm_grid"] = kw3["pm_grid"]
            e3 = {pr: summary(r, True) for pr, r in r3.items()}
            a32, a64 = r3["fp32"]["acc"].numpy(), r3["fp64"]["acc"].numpy()
            na = np.linalg.norm(a64, axis=0)
            e = np.linalg.norm(a32 - a64, axis=0) / np.maximum(na, 1e-3 * np.sqrt(np.mean(na ** 2)))
            line["configs"]["3"] = {
                "workload": c3["name"], "n_particles": p3.n,
                "step": "build + PM + BH walk + |a| + relative walk, all particles",
                "fp32": e3["fp32"], "fp64": e3["fp64"],
                "fp32_vs_fp64_err": {"p50": float(np.percentile(e, 50)),
                                     "p99": float(np.percentile(e, 99)), "max": float(e.max())},
                "fp32_speedup_vs_fp64": e3["fp64"]["ms_per_step"] / e3["fp32"]["ms_per_step"]}
            del r3, p3
        log("local time-stepping workload (256^3 clustered box)")
        line["local_timestep"] = run_local_timestep(
            max(3, args.steps // 2), wl=(c, p, kw) if args.config == 4 else None)
        log("isolated TreePM (Hernquist 2^20, zero-padded mesh)")
        line["isolated_treepm"] = run_isolated(max(3, args.steps // 2), 2)
        log("individual softening (Hernquist 2^20)")
        line["mixed_softening"] = run_mixed_softening(max(3, args.steps // 2), 2)
        log("time integration (block steps, hierarchical split)")
        line["integration"] = run_integrators()
        log("serving stream")
        line["serving"] = run_serving()
    if not args.no_cpu and periodic:
        log("timing the CPU oracle on a sample of the headline workload")
        line["cpu_baseline"] = cpu_baseline(c, kw, args.cpu_scale)
    print(json.dumps(line))
    if args.copy_probe:
        import torch
        n = args.copy_probe * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)  # reads and writes exactly copy_probe MiB each
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
