"""Pins for the oracle's time integration (Sec. 7.1-7.3).

* Kick-drift-kick leapfrog: a Kepler orbit keeps its energy with a bounded,
  non-growing error (symplectic, second order) and the integration retraces
  itself exactly when the velocities are reversed.
* Power-of-two time bins: every kick falls on its step's grid, a particle
  lengthens its step only at a synchronised time, several bins are used.
* Hierarchical split (Sec. 7.3): with pairwise forces it conserves momentum
  to round-off even with local steps, which the block-step scheme does not;
  with a single bin it is the plain leapfrog, bit for bit.  With a
  long-range part (kicked on the longest step) it still conserves momentum
  when both parts are pairwise, and with a single bin it equals the leapfrog
  on the summed force up to rounding (the kicks commute).
"""
import math

import numpy as np
import pytest

from oracle import integrate as I
from paper_1909_04667_amd import workloads as W


def _direct_force(orc, mass, eps):
    P = orc.make_params(eps=eps)

    def force(x, targets):
        a, _ = orc.direct(x[0], x[1], x[2], mass, P, targets=targets)
        return a
    return force


def _direct_force_sub(orc, mass, eps):
    """Forces among a subset: the other particles get zero mass."""
    P = orc.make_params(eps=eps)

    def force_sub(x, members):
        m = np.zeros_like(mass)
        m[members] = mass[members]
        a, _ = orc.direct(x[0], x[1], x[2], m, P, targets=members)
        return a
    return force_sub


def _energy(orc, x, v, mass, eps):
    P = orc.make_params(eps=eps, want_pot=True)
    _, pot = orc.direct(x[0], x[1], x[2], mass, P)
    return 0.5 * float(np.sum(mass * (v * v).sum(axis=0))) + 0.5 * float(np.sum(mass * pot))


def _kepler():
    x = np.array([[-0.5, 0.5], [0.0, 0.0], [0.0, 0.0]])
    v = np.array([[0.0, 0.0], [-0.35, 0.35], [0.0, 0.0]])  # eccentric bound orbit
    return x, v, np.array([0.5, 0.5])


def test_leapfrog_kepler_energy_bounded(orc):
    x, v, m = _kepler()
    eps = 1e-5
    force = _direct_force(orc, m, eps)
    E0 = _energy(orc, x, v, m, eps)
    a_major = 1.0 / (2.0 - 0.7 ** 2)  # G M = 1, separation 1, relative speed 0.7
    period = 2.0 * math.pi * a_major ** 1.5
    dt = period / 400
    errs = []
    for _ in range(20 * 10):  # 20 orbits, ten samples per orbit (all phases)
        x, v, _ = I.leapfrog_bins(x, v, force, eps=eps, C=1e9, dt_max=dt, max_bin=0,
                                  n_max_steps=40)
        errs.append(abs(_energy(orc, x, v, m, eps) / E0 - 1.0))
    first, last = max(errs[:30]), max(errs[-30:])
    assert max(errs) <= 2e-3, max(errs)
    assert first > 1e-6  # the sampling sees the O(dt^2) oscillation
    assert last <= 1.5 * first, (first, last)  # bounded: no secular growth


def test_leapfrog_time_reversible(orc):
    p = W.plummer(96, 3)
    x0 = np.stack([p.x, p.y, p.z])
    v0 = 0.3 * np.random.default_rng(4).normal(size=x0.shape)
    m = np.full(p.n, 1.0 / p.n)
    force = _direct_force(orc, m, 0.05)
    x1, v1, _ = I.leapfrog_bins(x0, v0, force, eps=0.05, C=1e9, dt_max=0.01, max_bin=0,
                                n_max_steps=25)
    x2, v2, _ = I.leapfrog_bins(x1, -v1, force, eps=0.05, C=1e9, dt_max=0.01, max_bin=0,
                                n_max_steps=25)
    assert np.abs(x2 - x0).max() <= 1e-12 * np.abs(x0).max()
    assert np.abs(-v2 - v0).max() <= 1e-11 * np.abs(v0).max()


def test_time_bins_follow_the_hierarchy(orc):
    p = W.plummer(400, 5)
    x0 = np.stack([p.x, p.y, p.z])
    v0 = 0.5 * np.random.default_rng(6).normal(size=x0.shape)
    m = np.full(p.n, 1.0 / p.n)
    force = _direct_force(orc, m, 0.02)
    ev = []
    N = 5
    I.leapfrog_bins(x0, v0, force, eps=0.02, C=0.02, dt_max=0.08, max_bin=N,
                    n_max_steps=2, record=ev)
    assert len({e[3] for e in ev}) >= 3  # several bins in use
    for t, i, old, new in ev:
        assert t % (1 << (N - old)) == 0  # the kick closes a step of the old bin
        if new < old:  # a longer step starts only on its own grid
            assert t % (1 << (N - new)) == 0


def test_hierarchical_conserves_momentum(orc):
    p = W.plummer(200, 7)
    x0 = np.stack([p.x, p.y, p.z])
    v0 = 0.4 * np.random.default_rng(8).normal(size=x0.shape)
    m = np.random.default_rng(9).uniform(0.5, 1.5, p.n) / p.n
    mom = lambda v: (v * m).sum(axis=1)
    scale = float(np.sum(m * np.linalg.norm(v0, axis=0)))
    kw = dict(eps=0.02, C=0.02, dt_max=0.04, max_bin=3, n_max_steps=2)
    _, vh, st = I.hierarchical(x0, v0, _direct_force_sub(orc, m, 0.02), **kw)
    assert st["levels"] >= 3
    dh = np.abs(mom(vh) - mom(v0)).max() / scale
    _, vb, _ = I.leapfrog_bins(x0, v0, _direct_force(orc, m, 0.02), **kw)
    db = np.abs(mom(vb) - mom(v0)).max() / scale
    assert dh <= 1e-14, dh
    assert db >= 100 * max(dh, 1e-17), (db, dh)  # block steps break it


def test_hierarchical_single_bin_is_leapfrog(orc):
    p = W.plummer(120, 10)
    x0 = np.stack([p.x, p.y, p.z])
    v0 = 0.3 * np.random.default_rng(11).normal(size=x0.shape)
    m = np.full(p.n, 1.0 / p.n)
    kw = dict(eps=0.03, C=1e9, dt_max=0.02, max_bin=3, n_max_steps=3)
    xh, vh, _ = I.hierarchical(x0, v0, _direct_force_sub(orc, m, 0.03), **kw)
    xb, vb, _ = I.leapfrog_bins(x0, v0, _direct_force(orc, m, 0.03), **kw)
    assert np.array_equal(xh, xb) and np.array_equal(vh, vb)


def _long_force(orc, mass):
    """A smooth pairwise stand-in for the mesh force: the direct sum with a
    wide softening (pairwise, so it conserves momentum)."""
    P = orc.make_params(eps=0.5)

    def force_long(x):
        a, _ = orc.direct(x[0], x[1], x[2], mass, P)
        return a
    return force_long


def test_hierarchical_long_range_conserves_momentum(orc):
    p = W.plummer(160, 12)
    x0 = np.stack([p.x, p.y, p.z])
    v0 = 0.4 * np.random.default_rng(13).normal(size=x0.shape)
    m = np.random.default_rng(14).uniform(0.5, 1.5, p.n) / p.n
    mom = lambda v: (v * m).sum(axis=1)
    scale = float(np.sum(m * np.linalg.norm(v0, axis=0)))
    kw = dict(eps=0.02, C=0.02, dt_max=0.04, max_bin=3, n_max_steps=2)
    _, vh, st = I.hierarchical(x0, v0, _direct_force_sub(orc, m, 0.02),
                               force_long=_long_force(orc, m), **kw)
    assert st["levels"] >= 3
    assert np.abs(mom(vh) - mom(v0)).max() / scale <= 1e-14


def test_hierarchical_long_range_single_bin_is_leapfrog(orc):
    p = W.plummer(120, 15)
    x0 = np.stack([p.x, p.y, p.z])
    v0 = 0.3 * np.random.default_rng(16).normal(size=x0.shape)
    m = np.full(p.n, 1.0 / p.n)
    kw = dict(eps=0.03, C=1e9, dt_max=0.02, max_bin=3, n_max_steps=3)
    short, long_ = _direct_force_sub(orc, m, 0.03), _long_force(orc, m)
    xh, vh, _ = I.hierarchical(x0, v0, short, force_long=long_, **kw)
    full = lambda x, t: short(x, np.arange(p.n))[:, t] + long_(x)[:, t]
    xb, vb, _ = I.leapfrog_bins(x0, v0, full, **kw)
    dv = np.abs(v0 - vb).max()  # the velocity change the forces made
    assert np.abs(xh - xb).max() <= 1e-13 * np.abs(x0).max()
    assert np.abs(vh - vb).max() <= 1e-11 * dv, (np.abs(vh - vb).max(), dv)


@pytest.mark.parametrize("mut,pin", [(1, "test_time_bins_follow_the_hierarchy"),
                                     (2, "test_hierarchical_conserves_momentum"),
                                     (3, "test_hierarchical_long_range_single_bin_is_leapfrog")])
def test_integrator_mutation_is_caught(orc, mut, pin):
    saved = I.MUTATION
    I.MUTATION = mut
    try:
        with pytest.raises(AssertionError):
            globals()[pin](orc)
    finally:
        I.MUTATION = saved
