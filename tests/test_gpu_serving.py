"""Serving (continuous batching over many systems): each request's result is
the same alone and in a mix, and the server completes a Poisson stream."""
import numpy as np
import pytest

from paper_1909_04667_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _system(spec, precision):
    from paper_1909_04667_amd import binding as B
    from paper_1909_04667_amd import serve as S
    params, stages = S.system_params(spec, precision)
    p = W.system_particles(spec)
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=_dev())
    ctx = B.Context(params)
    xyz = (t(p.x), t(p.y), t(p.z))
    ctx.build_tree(*xyz)
    return ctx, xyz, p


def test_batch_alone_equals_mix_equals_single():
    from paper_1909_04667_amd import binding as B
    specs = [W.SystemSpec(0, "plummer", 3000, 1), W.SystemSpec(1, "hernquist", 20000, 2),
             W.SystemSpec(2, "periodic", 16 ** 3, 3), W.SystemSpec(3, "plummer", 70000, 4)]
    precs = ["fp64", "fp32", "fp64", "fp32"]
    systems = [_system(s, pr) for s, pr in zip(specs, precs)]
    rng = np.random.default_rng(0)
    idx = []
    for (ctx, _, p), f in zip(systems, (1.0, 0.3, 0.05, 0.5)):
        sub = rng.choice(p.n, max(1, int(f * p.n)), replace=False).astype(np.int32)
        idx.append(torch.as_tensor(sub, device=_dev()))
    # single-system path
    single = [ctx.compute_forces(ix, "bh")[0].cpu() for (ctx, _, _), ix in zip(systems, idx)]
    # each alone in a batch
    alone = []
    for (ctx, _, _), ix in zip(systems, idx):
        b = B.Batch()
        acc = b.add(ctx, ix, "bh")
        b.launch()
        torch.cuda.synchronize()
        alone.append(acc.cpu())
        b.close()
    # all together in one batch
    b = B.Batch()
    accs = [b.add(ctx, ix, "bh") for (ctx, _, _), ix in zip(systems, idx)]
    b.launch()
    torch.cuda.synchronize()
    for k in range(len(systems)):
        assert torch.equal(alone[k], accs[k].cpu()), k
        assert torch.equal(single[k], accs[k].cpu()), k
    # relative pass in a mix, fed the first pass's |a|
    an = [ctx.accel_norm(ix, a) for (ctx, _, _), ix, a in zip(systems, idx, accs)]
    b2 = B.Batch()
    rel = [b2.add(ctx, ix, "rel", a_old_norm=a) for (ctx, _, _), ix, a in zip(systems, idx, an)]
    b2.launch()
    torch.cuda.synchronize()
    for k, ((ctx, _, _), ix) in enumerate(zip(systems, idx)):
        ref, _ = ctx.compute_forces(ix, "rel", a_old_norm=an[k])
        assert torch.equal(ref.cpu(), rel[k].cpu()), k
    for ctx, _, _ in systems:
        ctx.check()


def test_batch_rejects_same_context_twice():
    from paper_1909_04667_amd import binding as B
    ctx, _, p = _system(W.SystemSpec(0, "plummer", 500, 1), "fp32")
    ix = torch.arange(10, dtype=torch.int32, device=_dev())
    b = B.Batch()
    b.add(ctx, ix, "bh")
    with pytest.raises(B.TreePMError):
        b.add(ctx, ix, "bh")
    b.launch()
    torch.cuda.synchronize()


def test_resident_alone_equals_mix_equals_single():
    """Requests for four systems of both precisions submitted together to
    the running kernels (and one at a time): bit-identical to the
    single-system path, BH and relative pass, with interaction counts."""
    from paper_1909_04667_amd import binding as B
    specs = [W.SystemSpec(0, "plummer", 3000, 1), W.SystemSpec(1, "hernquist", 20000, 2),
             W.SystemSpec(2, "periodic", 16 ** 3, 3), W.SystemSpec(3, "plummer", 70000, 4),
             W.SystemSpec(4, "hernquist", 5000, 5), W.SystemSpec(5, "periodic", 20 ** 3, 6)]
    precs = ["fp64", "fp32", "fp64", "fp32", "fp32", "fp32"]
    systems = [_system(s, pr) for s, pr in zip(specs, precs)]
    rng = np.random.default_rng(0)
    idx = []
    for (ctx, _, p), f in zip(systems, (1.0, 0.3, 0.05, 0.5, 0.002, 1.0)):
        sub = rng.choice(p.n, max(1, int(f * p.n)), replace=False).astype(np.int32)
        sub = np.concatenate([sub, sub[:2]])  # duplicates
        idx.append(torch.as_tensor(sub, device=_dev()))
    single, nsingle = [], []
    for (ctx, _, _), ix in zip(systems, idx):
        n = torch.empty(ix.numel(), dtype=torch.int32, device=_dev())
        a, _ = ctx.compute_forces(ix, "bh", n_interactions=n)
        single.append(a.cpu())
        nsingle.append(n.cpu())
    torch.cuda.synchronize()
    loops = {p: B.ResidentServer(p) for p in ("fp32", "fp64")}
    # one at a time
    for k, ((ctx, _, _), ix) in enumerate(zip(systems, idx)):
        lp = loops[precs[k]]
        n = torch.zeros(ix.numel(), dtype=torch.int32, device=_dev())
        t, acc = lp.submit(ctx, ix, "bh", n_interactions=n)
        lp.wait(t)
        assert torch.equal(acc.cpu(), single[k]), k
        assert torch.equal(n.cpu(), nsingle[k]), k
    # all together
    sub = []
    for k, ((ctx, _, _), ix) in enumerate(zip(systems, idx)):
        n = torch.zeros(ix.numel(), dtype=torch.int32, device=_dev())
        t, acc = loops[precs[k]].submit(ctx, ix, "bh", n_interactions=n)
        sub.append((t, acc, n))
    for k, (t, acc, n) in enumerate(sub):
        loops[precs[k]].wait(t)
        assert torch.equal(acc.cpu(), single[k]), k
        assert torch.equal(n.cpu(), nsingle[k]), k
    # relative pass in a mix, fed the first pass's |a|
    an = [ctx.accel_norm(ix, a.to(_dev())) for (ctx, _, _), ix, a in zip(systems, idx, single)]
    torch.cuda.synchronize()
    rel = [loops[precs[k]].submit(ctx, ix, "rel", a_old_norm=an[k])
           for k, ((ctx, _, _), ix) in enumerate(zip(systems, idx))]
    for k, ((ctx, _, _), ix) in enumerate(zip(systems, idx)):
        loops[precs[k]].wait(rel[k][0])
        ref, _ = ctx.compute_forces(ix, "rel", a_old_norm=an[k])
        assert torch.equal(ref.cpu(), rel[k][1].cpu()), k
    for ctx, _, _ in systems:
        ctx.check()
    for lp in loops.values():
        lp.close()


def test_resident_step_equals_single_system_sequence():
    """One step request (geometric pass, mesh force, |a|, relative pass) run
    inside the resident kernel equals the four single-system calls in
    sequence, bit for bit: periodic boxes and isolated systems with and
    without a mesh, both precisions, several at once."""
    from paper_1909_04667_amd import binding as B
    cases = [(W.zeldovich_box(16, 100.0, 31), dict(periodic=True, box_size=100.0, pm_grid=32,
                                                   eps=100.0 / 800), 1.0),
             (W.lognormal_box(16, 100.0, 32), dict(periodic=True, box_size=100.0, pm_grid=64,
                                                   eps=100.0 / 800), 0.3),
             (W.hernquist(1 << 14, 33), dict(eps=0.005), 0.5),
             (W.hernquist(1 << 13, 34), dict(eps=0.005, pm_grid=32), 1.0)]
    for prec in ("fp64", "fp32"):
        lp = B.ResidentServer(prec)
        subs, refs = [], []
        for p, kw, f in cases:
            ctx = B.Context(precision=prec, **kw)
            t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=_dev())
            ctx.build_tree(t(p.x), t(p.y), t(p.z))
            rng = np.random.default_rng(5)
            ids = rng.choice(p.n, max(1, int(f * p.n)), replace=False).astype(np.int32)
            ix = torch.as_tensor(ids, device=_dev())
            a, _ = ctx.compute_forces(ix, "bh")
            apm = ctx.pm_long_range(ix)[0] if kw.get("pm_grid") else None
            an = ctx.accel_norm(ix, a, apm)
            n_ref = torch.empty(ids.size, dtype=torch.int32, device=_dev())
            ar, _ = ctx.compute_forces(ix, "rel", a_old_norm=an, n_interactions=n_ref)
            refs.append((ar.cpu(), None if apm is None else apm.cpu(), n_ref.cpu()))
            torch.cuda.synchronize()
            n = torch.zeros(ids.size, dtype=torch.int32, device=_dev())
            subs.append((ctx, n) + lp.submit_step(ctx, ix, n_interactions=n))
        for (ctx, n, tk, acc, acc_pm), (ar, apm, n_ref) in zip(subs, refs):
            lp.wait(tk)
            ctx.check()
            assert torch.equal(acc.cpu(), ar), prec
            assert (apm is None) == (acc_pm is None)
            if apm is not None:
                assert torch.equal(acc_pm.cpu(), apm), prec
            assert torch.equal(n.cpu(), n_ref), prec
        lp.close()


def test_resident_requests_join_the_running_kernel():
    """A large request keeps the kernel busy; requests submitted meanwhile
    are taken up by the same launch, and a context rebuilt meanwhile is
    served correctly (the kernel is drained and launched again first)."""
    from paper_1909_04667_amd import binding as B
    big, _, pb = _system(W.SystemSpec(0, "hernquist", 1 << 19, 7), "fp32")
    small = [_system(W.SystemSpec(k, "plummer", 2000 + 500 * k, 8 + k), "fp32")
             for k in range(1, 5)]
    lp = B.ResidentServer("fp32", idle_ms=200.0)
    ib = torch.arange(pb.n, dtype=torch.int32, device=_dev())
    t0 = lp.info()["launches"]
    tb, ab = lp.submit(big, ib, "bh")
    subs = []
    for ctx, _, p in small:
        ix = torch.arange(p.n, dtype=torch.int32, device=_dev())
        subs.append((ctx, ix) + lp.submit(ctx, ix, "bh"))
    for ctx, ix, t, acc in subs:
        lp.wait(t)
        ref, _ = ctx.compute_forces(ix, "bh")
        assert torch.equal(acc.cpu(), ref.cpu())
    lp.wait(tb)
    assert lp.info()["launches"] - t0 == 1  # all joined the first launch
    ref, _ = big.compute_forces(ib, "bh")
    assert torch.equal(ab.cpu(), ref.cpu())
    # rebuild one small system on moved positions while the kernel runs
    ctx, xyz, p = small[0]
    moved = [v * 1.5 for v in xyz]
    ctx.build_tree(*moved)
    ix = torch.arange(p.n, dtype=torch.int32, device=_dev())
    t, acc = lp.submit(ctx, ix, "bh")
    lp.wait(t)
    ref, _ = ctx.compute_forces(ix, "bh")
    assert torch.equal(acc.cpu(), ref.cpu())
    lp.close()


def test_server_admission_budget_evicts_waits_rejects():
    """A memory budget that holds about two of the systems at a time: the
    stream is served with evictions and waiting, a system that can never fit
    is rejected, and every served result equals the single-system path."""
    from paper_1909_04667_amd import binding as B
    from paper_1909_04667_amd import serve as S
    pool = [W.SystemSpec(0, "plummer", 20000, 21), W.SystemSpec(1, "hernquist", 24000, 22),
            W.SystemSpec(2, "plummer", 16000, 23), W.SystemSpec(3, "hernquist", 1 << 20, 24)]
    need = [B.bytes_needed(S.system_params(sp, "fp32")[0], sp.n) for sp in pool]
    budget = int(max(need[:3]) * 2.2)
    assert need[3] > budget
    reqs = [W.Request(i, 0.0005 * i, i % 4 if i % 7 else 3, 0.3, "fp32", 100 + i)
            for i in range(40)]
    srv = S.Server(pool, budget_bytes=budget)
    stats, jobs = srv.run(reqs)
    s = stats.summary()
    n_rej = sum(1 for r in reqs if r.sid == 3)
    assert s["rejected"] == n_rej and s["requests"] == len(reqs) - n_rej
    assert s["evictions"] > 0 and s["waited_for_memory"] > 0
    assert srv.used <= budget
    for j in jobs:
        if j.rejected:
            continue
        ctx, _, _ = _system(pool[j.req.sid], "fp32")
        a, _ = ctx.compute_forces(j.idx, "bh")
        an = ctx.accel_norm(j.idx, a)
        if pool[j.req.sid].kind == "hernquist":
            a, _ = ctx.compute_forces(j.idx, "rel", a_old_norm=an)
        assert torch.equal(S.total_force(j).cpu(), a.cpu())
        ctx.close()
    srv.close()


def test_server_stream_small():
    from paper_1909_04667_amd import serve as S
    pool = W.system_pool(6, seed=11, log2n=(10, 15))
    reqs = W.request_stream(40, rate=2000.0, n_systems=6, seed=11)
    srv = S.Server(pool, budget_bytes=8 << 30)
    stats, jobs = srv.run(reqs)
    s = stats.summary()
    assert s["requests"] == 40
    assert np.isfinite(s["p99_ms"]) and s["p50_ms"] > 0
    # every served result equals a fresh single-system computation
    for j in jobs[:8]:
        spec = pool[j.req.sid]
        ctx, _, _ = _system(spec, j.req.precision)
        params, stages = S.system_params(spec, j.req.precision)
        a, _ = ctx.compute_forces(j.idx, "bh")
        if spec.kind == "periodic":
            apm, _ = ctx.pm_long_range(j.idx)
        else:
            apm = None
        if len(stages) > 1:
            an = ctx.accel_norm(j.idx, a, apm)
            a, _ = ctx.compute_forces(j.idx, "rel", a_old_norm=an)
        tot = a if apm is None else a + apm
        assert torch.equal(S.total_force(j).cpu(), tot.cpu())
    srv.close()
