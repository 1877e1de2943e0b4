"""Pins for individual softening lengths in the oracle (Sec. 3.2): a pair
interacts with the larger of its two softenings; a node carries the largest
softening of its particles and is opened when that exceeds the target's and
the target lies within it of the node's centre of mass; otherwise the node
interacts with the larger of the target's and its own.

* Equal individual softenings reproduce the uniform-softening walk exactly.
* With every node opened the tree equals the direct pair sum with the
  symmetrised softening; that sum conserves momentum.
* A constructed three-particle case isolates the node rule: the node would be
  accepted by the geometric criterion, the rule opens it (two interactions,
  the exact pair sum); with a larger target softening or a node beyond its
  softening it is accepted (one interaction).
* The geometric and relative criteria keep their usual accuracy.
"""
import numpy as np
import pytest

from paper_1909_04667_amd import workloads as W


def _eps(n, seed):
    return 0.01 * np.exp(np.random.default_rng(seed).normal(0.0, 0.7, n))


@pytest.mark.parametrize("opening", ["bh", "rel"])
def test_equal_individual_softening_is_uniform(orc, opening):
    p = W.plummer(3000, 3)
    eps = np.full(p.n, 0.013)
    T0 = orc.Tree(p.x, p.y, p.z)
    T1 = orc.Tree(p.x, p.y, p.z, eps=eps)
    an = None
    if opening == "rel":
        a, _, _ = T0.walk(orc.make_params(eps=0.013))
        an = np.linalg.norm(a, axis=0)
    P = orc.make_params(eps=0.013, opening=opening, want_pot=True)
    a0, p0, n0 = T0.walk(P, anorm=an)
    a1, p1, n1 = T1.walk(P, anorm=an)
    assert np.array_equal(a0, a1) and np.array_equal(p0, p1) and np.array_equal(n0, n1)
    d0, q0 = orc.direct(p.x, p.y, p.z, None, P)
    d1, q1 = orc.direct(p.x, p.y, p.z, None, P, eps=eps)
    assert np.array_equal(d0, d1) and np.array_equal(q0, q1)


@pytest.mark.parametrize("treepm", [False, True])
def test_open_all_equals_direct_mixed(orc, treepm):
    p = W.plummer(2000, 4)
    eps = _eps(p.n, 5)
    kw = dict(treepm=True, rs=0.3, rcut=1.35) if treepm else {}
    P = orc.make_params(eps=0.01, theta=0.0, want_pot=True, **kw)
    T = orc.Tree(p.x, p.y, p.z, eps=eps)
    a, pot, _ = T.walk(P)
    d, q = orc.direct(p.x, p.y, p.z, None, P, eps=eps)
    na = np.linalg.norm(d, axis=0)
    floor = 1e-3 * np.sqrt(np.mean(na ** 2))  # targets with no pair inside the cutoff
    assert (np.linalg.norm(a - d, axis=0) / np.maximum(na, floor)).max() <= 1e-12
    assert np.abs(pot - q).max() <= 1e-12 * np.abs(q).max()


def test_mixed_direct_conserves_momentum(orc):
    p = W.plummer(1500, 6)
    eps = _eps(p.n, 7)
    m = np.random.default_rng(8).uniform(0.5, 1.5, p.n) / p.n
    d, _ = orc.direct(p.x, p.y, p.z, m, orc.make_params(eps=0.01), eps=eps)
    tot = np.abs((d * m).sum(axis=1)).max()
    assert tot <= 1e-13 * float(np.sum(m * np.linalg.norm(d, axis=0)))


def _three(orc, eps_t, eps_ab):
    # target at the origin, a pair 0.5 away along x; the pair's smallest
    # common node has side 1/16, its ancestors 1/8, 1/4 (BH accepts from 1/4)
    x = np.array([0.0, 0.5, 0.5])
    y = np.array([0.0, 0.02, -0.02])
    z = np.zeros(3)
    eps = np.array([eps_t, eps_ab, eps_ab])
    T = orc.Tree(x, y, z, eps=eps)
    P = orc.make_params(eps=0.01, theta=0.5)
    a, _, nint = T.walk(P, targets=[0])
    d, _ = orc.direct(x, y, z, None, P, targets=[0], eps=eps)
    return a[:, 0], d[:, 0], int(nint[0])


def test_softening_node_rule(orc):
    # node softening 2.8 * 0.25 = 0.7 above the target's and beyond d = 0.5:
    # opened, so the result is the exact pair sum
    a, d, k = _three(orc, 0.001, 0.25)
    assert k == 2
    assert np.abs(a - d).max() <= 1e-14 * np.abs(d).max()
    # the target's softening is the larger one: the node is used
    a, d, k = _three(orc, 0.3, 0.25)
    assert k == 1 and np.abs(a - d).max() > 1e-6 * np.abs(d).max()
    # the node's softening (0.42) is below the distance: the node is used
    a, d, k = _three(orc, 0.001, 0.15)
    assert k == 1


@pytest.mark.parametrize("opening", ["bh", "rel"])
def test_mixed_softening_accuracy(orc, opening):
    """Against the direct sum, individual softenings cost the walk no
    accuracy: its p99 error stays within 25 % of the uniform-softening
    walk's on the same positions (and within 2 %)."""
    p = W.plummer(4096, 9)
    eps = _eps(p.n, 10)
    errs = []
    for e_arr in (None, eps):
        T = orc.Tree(p.x, p.y, p.z, eps=e_arr)
        ref, _ = orc.direct(p.x, p.y, p.z, None, orc.make_params(eps=0.01), eps=e_arr)
        an = np.linalg.norm(ref, axis=0)
        a, _, _ = T.walk(orc.make_params(eps=0.01, opening=opening), anorm=an)
        e = np.linalg.norm(a - ref, axis=0) / np.maximum(an, 1e-3 * np.sqrt(np.mean(an ** 2)))
        errs.append(np.percentile(e, 99))
    assert errs[1] <= 1.25 * errs[0] and errs[1] <= 0.02, errs
