"""Pins for the oracle's particle mesh without periodicity (Sec. 3.3: zero
padding and a different Green's function) and for TreePM on isolated systems.

* Without the deconvolution the mesh solve is an open (non-circular)
  convolution of the deposited masses with the sampled long-range kernel
  -G erf(r / 2 r_s) / r: checked against a brute-force real-space sum, with
  the difference stencil and the interpolation recomputed here.
* Far from a point mass the long-range force is Newtonian; at any
  separation the short-range pair force plus the mesh force is Newtonian
  (the split of Sec. 3.4).
* The mesh force conserves momentum.
* With every node opened, tree (short range) plus mesh follows the direct
  Newtonian sum of a Plummer sphere.
"""
import math

import numpy as np
import pytest
from scipy.special import erf

from paper_1909_04667_amd import workloads as W


def _kernel(r, G, rs):
    out = np.empty_like(r)
    z = r == 0.0
    out[z] = -G / (math.sqrt(math.pi) * rs)
    out[~z] = -G * erf(r[~z] / (2.0 * rs)) / r[~z]
    return out


def test_isolated_solve_is_open_convolution(orc):
    rng = np.random.default_rng(3)
    n, ng, G, asmth = 6, 16, 1.3, 1.25
    x, y, z = rng.uniform(-1.0, 1.0, (3, n))
    m = rng.uniform(0.5, 2.0, n)
    fr = orc.frame(x, y, z)
    h, rs = orc.isolated_scale(fr[3], ng, asmth)
    acc, pot = orc.pm_isolated(x, y, z, m, fr, ng, G, asmth, deconv=False)
    lo = fr[:3] - 2.0 * h
    pos = np.stack([x, y, z])
    f = (pos - lo[:, None]) / h
    i0 = np.floor(f).astype(int)
    w = f - i0
    # deposited cell masses
    cells = {}
    for p in range(n):
        for s in range(8):
            up = [(s >> (2 - a)) & 1 for a in range(3)]
            wt = np.prod([w[a, p] if up[a] else 1.0 - w[a, p] for a in range(3)])
            t = tuple(i0[a, p] + up[a] for a in range(3))
            cells[t] = cells.get(t, 0.0) + m[p] * wt
    cidx = np.array(list(cells.keys()), dtype=float)
    cm = np.array(list(cells.values()))

    def phi_at(t):  # open convolution at mesh point t
        d = np.linalg.norm(cidx - np.asarray(t, float), axis=1) * h
        return float(np.sum(cm * _kernel(d, G, rs)))

    for p in range(n):
        F, P = np.zeros(3), 0.0
        for s in range(8):
            up = [(s >> (2 - a)) & 1 for a in range(3)]
            wt = np.prod([w[a, p] if up[a] else 1.0 - w[a, p] for a in range(3)])
            t = np.array([i0[a, p] + up[a] for a in range(3)])
            for a in range(3):
                v = {}
                for st in (-2, -1, 1, 2):
                    u = t.copy()
                    u[a] += st
                    v[st] = phi_at(u)
                grad = ((2.0 / 3.0) * (v[1] - v[-1]) - (1.0 / 12.0) * (v[2] - v[-2])) / h
                F[a] += wt * -grad
            P += wt * phi_at(t)
        scale = np.abs(acc).max()
        assert np.abs(acc[:, p] - F).max() <= 1e-12 * scale, (p, acc[:, p], F)
        assert abs(pot[p] - P) <= 1e-12 * abs(P)


def _pair(orc, d, direction, ng=64, asmth=1.25, rcut=4.5):
    """Unit mass at the origin (inside a fixed root cube set by two far
    massless markers) and a massless test particle at offset d."""
    e = np.asarray(direction, float)
    e /= np.linalg.norm(e)
    x = np.array([0.0, d * e[0], -5.0, 5.0])
    y = np.array([0.0, d * e[1], -5.0, 5.0])
    z = np.array([0.0, d * e[2], -5.0, 5.0])
    m = np.array([1.0, 0.0, 0.0, 0.0])
    fr = orc.frame(x, y, z)
    h, rs = orc.isolated_scale(fr[3], ng, asmth)
    apm, _ = orc.pm_isolated(x, y, z, m, fr, ng, 1.0, asmth, targets=[1], want_pot=False)
    P = orc.make_params(eps=1e-4, treepm=True, rs=rs, rcut=rcut * rs)
    ash, _ = orc.direct(x, y, z, m, P, targets=[1])
    return apm[:, 0], ash[:, 0], rs, e


@pytest.mark.parametrize("dist_rs", [6.0, 9.0, 14.0])
def test_isolated_far_field_is_newtonian(orc, dist_rs):
    rng = np.random.default_rng(int(dist_rs))
    for _ in range(3):
        dirn = rng.normal(size=3)
        _, _, rs, _ = _pair(orc, 1.0, dirn)
        d = dist_rs * rs
        apm, ash, rs, e = _pair(orc, d, dirn)
        newton = -e / (d * d)
        assert np.linalg.norm(ash) < 1e-6 * np.linalg.norm(newton)  # beyond the cutoff
        assert np.linalg.norm(apm - newton) <= 0.01 * np.linalg.norm(newton)


@pytest.mark.parametrize("dist_rs", [0.3, 1.0, 2.0, 3.5])
def test_isolated_split_sums_to_newton(orc, dist_rs):
    rng = np.random.default_rng(7)
    dirn = rng.normal(size=3)
    _, _, rs, _ = _pair(orc, 1.0, dirn)
    d = dist_rs * rs
    apm, ash, _, e = _pair(orc, d, dirn)
    newton = -e / (d * d)
    assert np.linalg.norm(apm + ash - newton) <= 0.03 * np.linalg.norm(newton)


def test_isolated_momentum(orc):
    p = W.plummer(3000, 5)
    m = np.random.default_rng(6).uniform(0.5, 1.5, p.n) / p.n
    fr = orc.frame(p.x, p.y, p.z)
    acc, _ = orc.pm_isolated(p.x, p.y, p.z, m, fr, 32, 1.0, 1.25, want_pot=False)
    tot = np.abs((acc * m).sum(axis=1)).max()
    assert tot <= 1e-12 * float(np.sum(m * np.linalg.norm(acc, axis=0)))


def test_isolated_treepm_open_all_follows_direct(orc):
    p = W.plummer(2000, 9)
    eps, ng, asmth, rcut = 0.01, 32, 1.25, 4.5
    fr = orc.frame(p.x, p.y, p.z)
    h, rs = orc.isolated_scale(fr[3], ng, asmth)
    T = orc.Tree(p.x, p.y, p.z)
    P = orc.make_params(eps=eps, theta=0.0, treepm=True, rs=rs, rcut=rcut * rs)
    a_tree, _, _ = T.walk(P)
    apm, _ = orc.pm_isolated(p.x, p.y, p.z, None, fr, ng, 1.0, asmth, want_pot=False)
    ref, _ = orc.direct(p.x, p.y, p.z, None, orc.make_params(eps=eps))
    na = np.linalg.norm(ref, axis=0)
    e = np.linalg.norm(a_tree + apm - ref, axis=0) / np.maximum(na, 1e-3 * np.sqrt(np.mean(na ** 2)))
    assert np.percentile(e, 50) <= 0.005, np.percentile(e, [50, 99])
    assert np.percentile(e, 99) <= 0.02, np.percentile(e, [50, 99])
