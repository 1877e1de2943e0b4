"""Device memory of a context (the memory manager of Sec. 9.4): the admission
estimate tpm_bytes_needed bounds what a context holds after every kind of
call, on the four numbered workloads at full size and on isolated-TreePM and
individual-softening contexts; a context working in one arena of that size
gives bit-identical results without further allocation, and an arena that is
too small fails with TPM_ENOMEM before any output is written."""
import functools

import numpy as np
import pytest

from paper_1909_04667_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a, dt=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt or torch.float64, device=_dev())


# workload -> (particles, context keywords, individual softening factor or None)
@functools.lru_cache(maxsize=2)
def _case(name):
    if name == "plummer_4096":          # workload 1
        return W.plummer(4096, 1), dict(eps=0.01), None
    if name == "hernquist_2p20":        # workload 2
        return W.hernquist(1 << 20, 2), dict(eps=0.005, alpha=0.0025), None
    if name == "zeldovich_128c_pm256":  # workload 3
        return W.zeldovich_box(128, 100.0, 3), dict(
            eps=100.0 / 6400, periodic=True, box_size=100.0, pm_grid=256), None
    if name == "lognormal_256c_pm256":  # workload 4
        return W.lognormal_box(256, 100.0, 4), dict(
            eps=100.0 / 12800, periodic=True, box_size=100.0, pm_grid=256), None
    if name == "isolated_treepm":
        return W.hernquist(1 << 18, 5), dict(eps=0.005, pm_grid=128), None
    if name == "mixed_softening":
        return W.hernquist(1 << 18, 6), dict(eps=0.005), 0.5
    raise KeyError(name)


def _exercise(ctx, p, mix):
    """Build, both tree passes with |a|, the mesh, and a resident-server step:
    every kind of buffer a context takes."""
    from paper_1909_04667_amd import binding as B
    eps = None
    if mix is not None:
        eps = _t(ctx.params.eps * np.exp(mix * np.random.default_rng(1).normal(size=p.n)))
    ctx.build_tree(_t(p.x), _t(p.y), _t(p.z), eps=eps)
    idx = _t(np.arange(p.n), torch.int32)
    a, _ = ctx.compute_forces(idx, "bh")
    apm = ctx.pm_long_range(idx)[0] if ctx.params.pm_grid > 0 else None
    an = ctx.accel_norm(idx, a, apm)
    arel, _ = ctx.compute_forces(idx, "rel", a_old_norm=an)
    srv = B.ResidentServer("fp32" if ctx.params.precision == 1 else "fp64")
    sub = idx[: max(1, p.n // 100)].contiguous()
    tk, acc_s, _ = srv.submit_step(ctx, sub)
    srv.wait(tk)
    srv.close()
    ctx.check()
    out = [arel.cpu().numpy(), acc_s.cpu().numpy()]
    if apm is not None:
        out.append(apm.cpu().numpy())
    return out


CASES = ["plummer_4096", "hernquist_2p20", "zeldovich_128c_pm256", "lognormal_256c_pm256",
         "isolated_treepm", "mixed_softening"]


@pytest.mark.slow
@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_bytes_held_within_bytes_needed(name, prec):
    from paper_1909_04667_amd import binding as B
    p, kw, mix = _case(name)
    ctx = B.Context(precision=prec, **kw)
    _exercise(ctx, p, mix)
    held, need = ctx.bytes_held(), B.bytes_needed(ctx.params, p.n)
    ctx.close()
    assert 0 < held <= need, (name, prec, held, need)


@pytest.mark.parametrize("name", ["plummer_4096", "isolated_treepm", "mixed_softening"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_arena_matches_lazy_allocation(name, prec):
    from paper_1909_04667_amd import binding as B
    p, kw, mix = _case(name)
    lazy = B.Context(precision=prec, **kw)
    ref = _exercise(lazy, p, mix)
    lazy.close()
    need = B.bytes_needed(B.make_params(precision=prec, **kw), p.n)
    ctx = B.Context(precision=prec, arena_bytes=need, **kw)
    got = _exercise(ctx, p, mix)
    for k, (a, b) in enumerate(zip(ref, got)):
        assert np.array_equal(a, b), (k, np.abs(a - b).max(), np.count_nonzero(a != b), a.size)
    assert ctx.bytes_held() == need
    # a smaller rebuild in the same arena reuses it
    q = W.plummer(1000, 9)
    ctx.build_tree(_t(q.x), _t(q.y), _t(q.z))
    a, _ = ctx.compute_forces(_t(np.arange(q.n), torch.int32), "bh")
    ctx.check()
    c2 = B.Context(precision=prec, **kw)
    c2.build_tree(_t(q.x), _t(q.y), _t(q.z))
    a2, _ = c2.compute_forces(_t(np.arange(q.n), torch.int32), "bh")
    assert torch.equal(a, a2)
    ctx.close()
    c2.close()


def test_arena_too_small_fails_before_writing():
    from paper_1909_04667_amd import binding as B
    p = W.zeldovich_box(32, 100.0, 7)
    kw = dict(eps=100.0 / 1600, periodic=True, box_size=100.0, pm_grid=128)
    # what the tree and its walks need, without the mesh
    tree_only = B.bytes_needed(B.make_params(eps=kw["eps"]), p.n)
    # far too small: the build fails before any kernel, and leaves no tree
    ctx = B.Context(arena_bytes=tree_only // 4, **kw)
    with pytest.raises(B.TreePMError) as ei:
        ctx.build_tree(_t(p.x), _t(p.y), _t(p.z))
    assert ei.value.code == B.TPM_ENOMEM
    idx = _t(np.arange(p.n), torch.int32)
    with pytest.raises(B.TreePMError) as ei:
        ctx.compute_forces(idx, "bh")
    assert ei.value.code == B.TPM_ESTATE
    ctx.close()
    # room for the tree and its walks but not for the mesh: the mesh call
    # fails and leaves its output as it was
    ctx = B.Context(arena_bytes=tree_only, **kw)
    ctx.build_tree(_t(p.x), _t(p.y), _t(p.z))
    a, _ = ctx.compute_forces(idx, "bh")
    ctx.check()
    sentinel = torch.full((3, p.n), 7.0, dtype=torch.float64, device=_dev())
    with pytest.raises(B.TreePMError) as ei:
        ctx.pm_long_range(idx, acc=sentinel)
    assert ei.value.code == B.TPM_ENOMEM
    torch.cuda.synchronize()
    assert bool((sentinel == 7.0).all())
    ctx.close()
