"""Pins for the oracle's insertion-built octree and monopole moments (Sec. 3.1).

The tree the paper describes (sequential insertion, a leaf splits when it
receives a second particle) is unique for a given point set, so it must not
depend on the insertion order, and its internal nodes must be exactly the
cells that hold at least two particles; both are checked by brute force.
"""
import numpy as np
import pytest

from paper_1909_04667_amd import workloads as W


def _brute_nodes(q, maxlev=21):
    """All (level, cell) pairs holding >= 2 particles, with their counts."""
    n = q.shape[1]
    out = {}
    for lev in range(0, maxlev + 1):
        sh = 21 - lev
        cells = {}
        for i in range(n):
            c = (int(q[0, i]) >> sh, int(q[1, i]) >> sh, int(q[2, i]) >> sh)
            cells[c] = cells.get(c, 0) + 1
        for c, k in cells.items():
            if k >= 2:
                out[(lev, c)] = k
    return out


def _clustered(n, seed):
    rng = np.random.default_rng(seed)
    x, y, z = rng.normal(0, 1.0, (3, n))
    # a few exact duplicates and near-duplicates exercise the depth limit
    x[5], y[5], z[5] = x[4], y[4], z[4]
    x[9], y[9], z[9] = x[4], y[4], z[4]
    x[7], y[7], z[7] = x[6] + 1e-13, y[6], z[6]
    return x, y, z


@pytest.mark.parametrize("seed", [0, 1])
def test_topology_brute_force(orc, seed):
    x, y, z = _clustered(400, seed)
    T = orc.Tree(x, y, z)
    ex = T.export()
    p, q, key = T.positions()
    brute = _brute_nodes(q)
    nodes = ex["level"] >= 0
    assert nodes.sum() == len(brute)
    perm = orc.sort(key)
    for e in np.flatnonzero(nodes):
        lev = int(ex["level"][e])
        i = perm[ex["first"][e]]
        sh = 21 - lev
        c = (int(q[0, i]) >> sh, int(q[1, i]) >> sh, int(q[2, i]) >> sh)
        assert brute[(lev, c)] == ex["count"][e]
    # the duplicated particles sit in one depth-21 node, in index order
    e21 = np.flatnonzero(ex["level"] == 21)
    assert e21.size >= 1
    grp = ex["pidx"][e21[0] + 1: ex["skip"][e21[0]]]
    assert list(grp) == sorted(grp)


def test_dfs_particle_order_is_key_order(orc):
    x, y, z = _clustered(3000, 2)
    T = orc.Tree(x, y, z)
    ex = T.export()
    _, _, key = T.positions()
    dfs = ex["pidx"][ex["level"] < 0]
    assert np.array_equal(dfs, orc.sort(key))
    # first/count/skip are consistent with the depth-first layout
    E = T.E
    for e in range(E):
        s = ex["skip"][e]
        assert e < s <= E
        npart = (ex["level"][e:s] < 0).sum()
        assert npart == ex["count"][e]
        assert (ex["level"][:e] < 0).sum() == ex["first"][e]
    # children follow the curve: first keys strictly increase among siblings
    for e in np.flatnonzero(ex["level"] >= 0):
        k = e + 1
        prev = -1
        while k < ex["skip"][e]:
            fk = int(key[dfs[ex["first"][k]]])
            assert fk >= prev
            prev = fk
            k = ex["skip"][k]


def test_insertion_order_independent(orc):
    x, y, z = _clustered(2000, 3)
    T1 = orc.Tree(x, y, z)
    order = np.random.default_rng(9).permutation(2000)
    T2 = orc.Tree(x, y, z, insert_order=order)
    e1, e2 = T1.export(), T2.export()
    for k in ("level", "first", "count", "skip", "pidx", "mass", "com", "cen"):
        assert np.array_equal(e1[k], e2[k]), k


def test_moments(orc):
    p = W.plummer(4096, 11)
    T = orc.Tree(p.x, p.y, p.z)
    ex = T.export()
    pos, _, _ = T.positions()
    perm = np.flatnonzero  # noqa: F841
    dfs = ex["pidx"][ex["level"] < 0]
    m = 1.0 / 4096
    for e in np.flatnonzero(ex["level"] >= 0):
        f, c = ex["first"][e], ex["count"][e]
        mem = dfs[f:f + c]
        # equal masses 2^-12: node mass = count * m exactly
        assert ex["mass"][e] == c * m
        com = pos[:, mem].mean(axis=1)
        scale = np.abs(pos[:, mem]).max() + 1e-300
        assert np.all(np.abs(ex["com"][:, e] - com) <= 1e-14 * scale)
    # centres are the geometric centres of the cubes: all members inside
    L0 = T.frame[3]
    for e in np.flatnonzero(ex["level"] >= 0)[:500]:
        L = L0 * 2.0 ** -ex["level"][e]
        f, c = ex["first"][e], ex["count"][e]
        mem = dfs[f:f + c]
        d = np.abs(pos[:, mem] - ex["cen"][:, e:e + 1])
        assert np.all(d <= 0.5 * L * (1 + 1e-12))


def test_unequal_masses(orc):
    rng = np.random.default_rng(12)
    x, y, z = rng.uniform(-1, 1, (3, 500))
    mass = rng.uniform(0.5, 2.0, 500)
    T = orc.Tree(x, y, z, mass=mass)
    ex = T.export()
    dfs = ex["pidx"][ex["level"] < 0]
    pos, _, _ = T.positions()
    e = 0
    assert ex["level"][0] == 0
    assert abs(ex["mass"][e] - mass.sum()) < 1e-13 * mass.sum()
    com = (pos * mass).sum(axis=1) / mass.sum()
    assert np.allclose(ex["com"][:, 0], com, rtol=0, atol=1e-14)
    assert np.array_equal(np.sort(dfs), np.arange(500))


def test_single_and_pair(orc):
    T = orc.Tree([0.5], [0.5], [0.5])
    ex = T.export()
    assert T.E == 1 and ex["level"][0] == -1
    T = orc.Tree([0.0, 1.0], [0.0, 0.0], [0.0, 0.0])
    ex = T.export()
    assert list(ex["level"]) == [0, -1, -1]
    assert list(ex["skip"]) == [3, 2, 3]
