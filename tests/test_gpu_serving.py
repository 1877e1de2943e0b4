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


def test_server_stream_small():
    from paper_1909_04667_amd import serve as S
    pool = W.system_pool(6, seed=11, log2n=(10, 15))
    reqs = W.request_stream(40, rate=2000.0, n_systems=6, seed=11)
    srv = S.Server(pool, budget_bytes=2 << 30)
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
