"""Pins for the oracle's Peano-Hilbert keys, root cube and sort.

The paper orders domain pieces along the Peano-Hilbert curve (Sec. 8) but does
not print the curve; the oracle uses Skilling's transpose algorithm.  The pins
are the properties that make a key a Hilbert key and make its prefixes octree
cells: bijection, unit steps between consecutive keys, and nesting of every
aligned octant block into one contiguous key range (exhaustive for b <= 6).
"""
import numpy as np
import pytest


def _all_cells(b):
    n = 1 << b
    g = np.arange(n, dtype=np.uint32)
    q0, q1, q2 = np.meshgrid(g, g, g, indexing="ij")
    return q0.ravel(), q1.ravel(), q2.ravel()


@pytest.mark.parametrize("b", [1, 2, 3, 4, 5, 6])
def test_key_bijection_adjacency_nesting(orc, b):
    q0, q1, q2 = _all_cells(b)
    key = orc.ph_keys(b, q0, q1, q2)
    n3 = 8 ** b
    # bijection onto [0, 8^b)
    assert key.max() < n3
    assert np.unique(key).size == n3
    # consecutive keys are face neighbours (unit L1 step)
    order = np.argsort(key)
    c = np.stack([q0, q1, q2]).astype(np.int64)[:, order]
    step = np.abs(np.diff(c, axis=1)).sum(axis=0)
    assert np.all(step == 1)
    # every aligned block of side 2^(b-l) is one contiguous, aligned key range
    for lev in range(1, b + 1):
        sh = b - lev
        blk = (q0 >> sh).astype(np.int64) * (1 << (2 * lev)) + \
              (q1 >> sh).astype(np.int64) * (1 << lev) + (q2 >> sh).astype(np.int64)
        pref = key >> np.uint64(3 * sh)
        # the prefix is a function of the block and distinct across blocks
        df = np.zeros(8 ** lev, np.int64) - 1
        for bl, pr in zip(blk, pref):
            if df[bl] < 0:
                df[bl] = pr
            assert df[bl] == pr
        assert np.unique(df).size == 8 ** lev


def test_key_b21_prefix_is_cell(orc):
    """At 21 bits: two points share the level-l prefix iff they share the cell."""
    rng = np.random.default_rng(7)
    n = 20000
    q = rng.integers(0, 1 << 21, (3, n), dtype=np.uint32)
    # make many pairs share cells at assorted levels
    lev = rng.integers(0, 22, n)
    partner = q.copy()
    for i in range(n):
        sh = 21 - lev[i]
        mask = np.uint32((1 << sh) - 1)
        noise = rng.integers(0, 1 << 21, 3, dtype=np.uint32) & mask
        partner[:, i] = (q[:, i] & ~mask) | noise
    k1 = orc.ph_keys(21, *q)
    k2 = orc.ph_keys(21, *partner)
    assert k1.max() < (1 << 63) and k2.max() < (1 << 63)
    for i in range(0, n, 7):
        for l in (lev[i], min(21, lev[i] + 1)):
            sh = 21 - l
            same_cell = np.all((q[:, i] >> sh) == (partner[:, i] >> sh))
            same_pref = (int(k1[i]) >> (3 * sh)) == (int(k2[i]) >> (3 * sh))
            assert same_cell == same_pref


def test_frame_nonperiodic(orc):
    rng = np.random.default_rng(3)
    x, y, z = rng.normal(0, 3.0, (3, 5000))
    fr = orc.frame(x, y, z)
    L = fr[3]
    ext = max(np.ptp(x), np.ptp(y), np.ptp(z))
    # power of two, just enclosing the extent
    m, e = np.frexp(L)
    assert m == 0.5
    assert L >= ext * (1 + 2.0 ** -20) and L / 2 < ext * (1 + 2.0 ** -20)
    assert np.allclose(fr[:3], [x.min(), y.min(), z.min()], rtol=0, atol=0)
    p, q, key = orc.positions(x, y, z, False, fr)
    assert q.max() <= (1 << 21) - 1
    assert np.array_equal(p[0], x)
    # integer coordinate reproduces floor((x - x0) * 2^21 / L)
    assert np.array_equal(q[0], np.floor((x - fr[0]) * (2.0 ** 21 / L)).astype(np.uint32))


def test_frame_shift_and_periodic(orc):
    rng = np.random.default_rng(4)
    x, y, z = rng.uniform(0, 100.0, (3, 3000))
    fr = orc.frame(x, y, z, True, 100.0, (0.25, 0.5, 0.0))
    assert np.allclose(fr, [-25.0, -50.0, 0.0, 100.0])
    p, q, key = orc.positions(x, y, z, True, fr)
    # tree-frame positions lie in [x0, x0 + L) and differ from x by 0 or -L
    for a, c in enumerate((x, y, z)):
        assert np.all(p[a] >= fr[a]) and np.all(p[a] < fr[a] + 100.0)
        d = c - p[a]
        assert np.all((d == 0.0) | (np.abs(d - 100.0) < 1e-12))
    # non-periodic random placement keeps every particle inside the root
    fr2 = orc.frame(x, y, z, False, 0.0, (0.9, 0.1, 0.5))
    for a, c in enumerate((x, y, z)):
        assert c.min() >= fr2[a] and c.max() < fr2[a] + fr2[3]


def test_sort_matches_lexsort(orc):
    rng = np.random.default_rng(5)
    key = rng.integers(0, 50, 4000).astype(np.uint64)  # many ties
    perm = orc.sort(key)
    ref = np.lexsort((np.arange(key.size), key))
    assert np.array_equal(perm, ref)
