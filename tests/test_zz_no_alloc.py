"""The allocation-free forces entry point (tpm_compute_forces_noalloc) against
tpm_compute_forces: same kernels, so results, potentials and interaction
counts must be bit-identical; two calls in a row on one GPU, the second on a
smaller tree and a smaller active set, share the library's fixed array."""
import numpy as np
import pytest

from paper_1909_04667_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=_dev())


CALLS = {
    # (particles, context parameters, opening, active set)
    "hernquist_bh_all": (lambda: W.hernquist(1 << 16, 71), dict(eps=0.005), "bh", None),
    "plummer_rel_subset": (lambda: W.plummer(5000, 72), dict(eps=0.01), "rel", 1234),
    "box_rel_all": (lambda: W.zeldovich_box(32, 100.0, 73),
                    dict(eps=100.0 / 1600, periodic=True, box_size=100.0, pm_grid=64), "rel",
                    None),
    "iso_bh_subset": (lambda: W.hernquist(3000, 74), dict(eps=0.005, pm_grid=32), "bh", 700),
}


def _one_call(name, prec):
    from paper_1909_04667_amd import binding as B
    mk, kw, opening, n_sub = CALLS[name]
    p = mk()
    ctx = B.Context(precision=prec, want_potential=True, **kw)
    ctx.build_tree(_t(p.x), _t(p.y), _t(p.z))
    rng = np.random.default_rng(7)
    ids = np.arange(p.n) if n_sub is None else rng.choice(p.n, n_sub, replace=False)
    ids = np.concatenate([ids, ids[:5]])  # duplicates take the same result
    idx = _t(ids, torch.int32)
    an = None
    if opening == "rel":
        c0 = B.Context(precision="fp64", **kw)
        c0.build_tree(_t(p.x), _t(p.y), _t(p.z))
        all_idx = _t(np.arange(p.n), torch.int32)
        a0, _ = c0.compute_forces(all_idx, "bh")
        an = c0.accel_norm(all_idx, a0)
        c0.close()
    torch.cuda.synchronize()
    held = ctx.bytes_held()
    acc = torch.full((3, ids.size), -7.0, dtype=ctx.dtype, device=_dev())
    pot = torch.full((ids.size,), -7.0, dtype=ctx.dtype, device=_dev())
    nint = torch.zeros(ids.size, dtype=torch.int32, device=_dev())
    # the allocation-free call first, on a context whose force buffers were
    # never allocated: it must not allocate them either
    ctx.compute_forces_noalloc(idx, opening, a_old_norm=an, acc=acc, pot=pot,
                               n_interactions=nint)
    ctx.check()
    assert ctx.bytes_held() == held
    nref = torch.zeros(ids.size, dtype=torch.int32, device=_dev())
    ref, rpot = ctx.compute_forces(idx, opening, a_old_norm=an, n_interactions=nref)
    ctx.check()
    assert torch.equal(acc, ref), name
    assert torch.equal(pot, rpot), name
    assert torch.equal(nint, nref), name
    ctx.close()
    return p.n, ids.size


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("first,second", [("hernquist_bh_all", "plummer_rel_subset"),
                                          ("box_rel_all", "iso_bh_subset")])
def test_noalloc_matches_compute_forces(first, second, prec):
    n1, a1 = _one_call(first, prec)
    n2, a2 = _one_call(second, prec)
    assert n2 < n1 and a2 < a1


def test_noalloc_rejects_trees_beyond_its_array():
    from paper_1909_04667_amd import binding as B
    nmax = B.noalloc_max_n()
    assert nmax == 1 << 20
    rng = np.random.default_rng(75)
    x, y, z = rng.uniform(-1.0, 1.0, (3, nmax + 1))
    ctx = B.Context(eps=0.01)
    ctx.build_tree(_t(x), _t(y), _t(z))
    idx = _t(np.arange(64), torch.int32)
    acc = torch.full((3, 64), -7.0, dtype=torch.float64, device=_dev())
    with pytest.raises(B.TreePMError) as ei:
        ctx.compute_forces_noalloc(idx, "bh", acc=acc)
    assert ei.value.code == B.TPM_EINVAL
    torch.cuda.synchronize()
    assert torch.all(acc == -7.0)  # nothing was written
    ctx.close()
