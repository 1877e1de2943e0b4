"""GPU parity of the relative opening criterion (Sec. 3.1) on the cases that
decide it exactly (see tests/test_oracle_relative.py): the hand-computed
threshold of a constructed node, and the invariance of every opening
decision under a change of units (G x 4, masses x 2)."""
import numpy as np
import pytest

import oracle as O
from paper_1909_04667_amd import workloads as W
from tests.test_oracle_relative import expected_forces, threshold_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=_dev())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_relative_threshold_exact_gpu(prec):
    from paper_1909_04667_amd import binding as B
    c = threshold_case()
    ctx = B.Context(eps=1e-3, G=c["G"], alpha=c["alpha"], precision=prec)
    ctx.build_tree(_t(c["x"]), _t(c["y"]), _t(c["z"]), _t(c["m"]))
    mono, pair = expected_forces(c)
    # FP32 takes the decision in float: stay clear of its rounding
    d = 1e-9 if prec == "fp64" else 1e-4
    tol = 1e-14 if prec == "fp64" else 1e-6
    idx = _t(np.array([0]), torch.int32)
    for f, n_expect, ref in ((1.0 + d, 1, mono), (1.0 - d, 2, pair),
                             (4.0 * (1.0 + d), 1, mono), (0.25, 2, pair)):
        an = _t(np.array([c["a_star"] * f, 0.0, 0.0]))
        nint = torch.empty(1, dtype=torch.int32, device=_dev())
        acc, _ = ctx.compute_forces(idx, "rel", a_old_norm=an, n_interactions=nint)
        ctx.check()
        assert int(nint.item()) == n_expect, (prec, f, int(nint.item()))
        a = acc.double().cpu().numpy()[:, 0]
        assert np.abs(a - ref).max() <= tol * np.linalg.norm(ref), (prec, f)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("treepm", [False, True])
def test_relative_unit_scaling_invariance_gpu(prec, treepm):
    """G x 4 and m x 2: the GPU's forces and |a| scale by exactly 8 and its
    interaction counts are unchanged; in FP64 they equal the oracle's."""
    from paper_1909_04667_amd import binding as B
    if treepm:
        p = W.lognormal_box(24, 100.0, 63)
        kw = dict(periodic=True, box_size=100.0, pm_grid=32, eps=100.0 / 1200)
    else:
        p = W.hernquist(1 << 12, 62)
        kw = dict(eps=0.005)
    n = p.n
    idx = _t(np.arange(n), torch.int32)
    out = []
    for G, mfac in ((1.0, 1.0), (4.0, 2.0)):
        m = np.full(n, mfac / n)
        ctx = B.Context(G=G, precision=prec, **kw)
        ctx.build_tree(_t(p.x), _t(p.y), _t(p.z), _t(m))
        a, _ = ctx.compute_forces(idx, "bh")
        an = ctx.accel_norm(idx, a)
        nint = torch.empty(n, dtype=torch.int32, device=_dev())
        ar, _ = ctx.compute_forces(idx, "rel", a_old_norm=an, n_interactions=nint)
        ctx.check()
        out.append((a.cpu(), an.cpu(), ar.cpu(), nint.cpu()))
        ctx.close()
    (a1, an1, ar1, n1), (a8, an8, ar8, n8) = out
    assert torch.equal(a8, 8 * a1)
    assert torch.equal(an8, 8 * an1)
    assert torch.equal(n8, n1)
    assert torch.equal(ar8, 8 * ar1)
    if prec == "fp64":
        rs = 1.25 * 100.0 / 32
        okw = (dict(periodic=True, box=100.0, eps=kw["eps"], treepm=True, rs=rs, rcut=4.5 * rs)
               if treepm else dict(eps=kw["eps"]))
        T = O.Tree(p.x, p.y, p.z, mass=np.full(n, 2.0 / n),
                   **(dict(periodic=True, box=100.0) if treepm else {}))
        ao, _, _ = T.walk(O.make_params(G=4.0, theta=0.5, **okw))
        ano = np.linalg.norm(ao, axis=0)
        aro, _, nro = T.walk(O.make_params(G=4.0, opening="rel", alpha=0.0025, **okw),
                             anorm=ano)
        e = np.linalg.norm(ar8.numpy() - aro, axis=0) / np.maximum(
            np.linalg.norm(aro, axis=0), 1e-3 * np.sqrt(np.mean(np.sum(aro ** 2, axis=0))))
        # both sides take their own |a| from their own first pass; the two
        # agree to rounding, so the decisions may differ only at exact ties
        assert np.array_equal(n8.numpy().astype(np.int64), nro)
        assert e.max() <= 1e-10, e.max()
