"""Pins for the interaction kernels: spline softening (Sec. 3.2) and the
TreePM short-range factor (Sec. 3.4).

The paper states the softening's properties, not its formula: zero-lag
potential -G m / eps and a Newtonian force from 2.8 eps on.  These tests derive
the force and potential by quadrature of the cubic-spline mass density and
check the oracle against them and against those two stated facts; the split
factor is checked against the derivative of the erfc potential and against the
Fourier transform of the Gaussian-filtered Green's function.
"""
import json
import math
import os

import numpy as np
from scipy import integrate, special

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _kernel_density(u):
    """Normalised cubic spline density, support h = 1 (integrates to 1)."""
    if u < 0.5:
        return 8.0 / math.pi * (1 - 6 * u * u + 6 * u ** 3)
    if u < 1.0:
        return 8.0 / math.pi * 2 * (1 - u) ** 3
    return 0.0


def _mass_inside(u):
    f = lambda s: 4 * math.pi * s * s * _kernel_density(s)
    m = integrate.quad(f, 0, min(u, 0.5), epsabs=1e-16, epsrel=1e-13)[0]
    if u > 0.5:
        m += integrate.quad(f, 0.5, min(u, 1.0), epsabs=1e-16, epsrel=1e-13)[0]
    return m


def _pair_force(orc, r, eps, **kw):
    """Acceleration of particle 0 from particle 1 (mass 1/2) at distance r."""
    x = np.array([0.0, r])
    y = np.zeros(2)
    z = np.zeros(2)
    P = orc.make_params(eps=eps, want_pot=True, theta=0.0, **kw)
    T = orc.Tree(x, y, z)
    a, pot, _ = T.walk(P)
    return a[0, 0], pot[0]


def test_spline_against_quadrature(orc):
    eps = 0.1
    h = 2.8 * eps
    m = 0.5
    for u in [0.05, 0.2, 0.37, 0.49, 0.5, 0.51, 0.7, 0.93, 0.999, 1.0, 1.3, 2.0]:
        r = u * h
        a, pot = _pair_force(orc, r, eps)
        M = _mass_inside(min(u, 1.0))
        a_ref = m * M / (u * u) / (h * h)  # G M(<r)/r^2 in units of h
        assert abs(a - a_ref) <= 1e-12 * abs(a_ref), (u, a, a_ref)
        # potential: -G m [ M(<r)/r + int_r^inf 4 pi s rho ds ]
        outer = integrate.quad(lambda s: 4 * math.pi * s * _kernel_density(s), min(u, 1), 1,
                               epsabs=1e-15, epsrel=1e-14)[0]
        phi_ref = -m * (M / u + outer) / h
        assert abs(pot - phi_ref) <= 1e-12 * abs(phi_ref), (u, pot, phi_ref)


def test_stated_softening_facts(orc):
    """Sec. 3.2: zero-lag potential -G m / eps; Newtonian at 2.8 eps."""
    with open(os.path.join(GOLD, "softening.json")) as f:
        g = json.load(f)
    eps = 0.05
    m = 0.5
    # coincident distinct pair: zero force, potential -G m / eps
    T = orc.Tree(np.array([0.3, 0.3]), np.zeros(2), np.zeros(2))
    a, pot, _ = T.walk(orc.make_params(eps=eps, want_pot=True, theta=0.0))
    assert a[0, 0] == 0.0
    assert abs(pot[0] / (-m / eps) - g["zero_lag_potential_in_units_of_minus_Gm_over_eps"]) < 1e-14
    r = g["newtonian_from_r_over_eps"] * eps
    for rr in [r, r * 1.0001, r * 3]:
        a, pot = _pair_force(orc, rr, eps)
        assert abs(a - m / rr ** 2) <= 1e-14 * m / rr ** 2
        assert abs(pot + m / rr) <= 1e-14 * m / rr
    a, _ = _pair_force(orc, r * 0.9, eps)
    assert a < m / (r * 0.9) ** 2 * (1 - 1e-6)  # softened inside 2.8 eps


def test_short_range_factor_identity(orc):
    """f_s = -r^2 d/dr[erfc(r/2rs)/r]; f_s + f_l = 1; f_s(4.5 rs) value."""
    with open(os.path.join(GOLD, "split.json")) as f:
        g = json.load(f)
    rs = 0.7
    eps = 1e-4  # softening irrelevant at these distances
    for r in [0.2, 0.7, 1.4, 2.0, 3.15]:
        a, pot = _pair_force(orc, r, eps, treepm=True, rs=rs, rcut=100.0)
        newton = 0.5 / r ** 2
        fs = a / newton
        dr = 1e-5 * r
        phi = lambda s: special.erfc(s / (2 * rs)) / s
        deriv = (phi(r + dr) - phi(r - dr)) / (2 * dr)
        assert abs(fs - (-r * r * deriv)) < 1e-8
        assert abs(pot / (-0.5 / r) - special.erfc(r / (2 * rs))) < 1e-14
    a, _ = _pair_force(orc, 4.5 * rs, eps, treepm=True, rs=rs, rcut=100.0)
    fs = a / (0.5 / (4.5 * rs) ** 2)
    assert abs(fs - g["fs_at_4.5rs"]) < 5e-7
    # cutoff: a pair at r >= r_cut does not interact
    a, _ = _pair_force(orc, 2.0, eps, treepm=True, rs=rs, rcut=2.0)
    assert a == 0.0


def test_long_range_green_function():
    """-4 pi G m exp(-k^2 rs^2)/k^2 transforms to -G m erf(r/2rs)/r."""
    rs = 0.4
    for r in [0.1, 0.5, 1.0, 2.5]:
        f = lambda k: math.sin(k * r) * math.exp(-(k * rs) ** 2) / k
        val = integrate.quad(f, 0, 60 / rs, limit=400, epsabs=1e-14)[0]
        phi = -(2.0 / (math.pi * r)) * val  # (1/(2 pi^2 r)) int k sin(kr) Phi_k dk
        assert abs(phi - (-special.erf(r / (2 * rs)) / r)) < 1e-10


def test_two_body_closed_form(orc):
    """N = 2: exact Newtonian pair through the tree and the direct sum."""
    x = np.array([0.1, 1.1])
    y = np.array([0.2, -0.3])
    z = np.array([0.0, 0.4])
    P = orc.make_params(eps=1e-3, theta=0.5)
    T = orc.Tree(x, y, z)
    a, _, nint = T.walk(P)
    ad, _ = orc.direct(x, y, z, None, P)
    d = np.array([x[1] - x[0], y[1] - y[0], z[1] - z[0]])
    r = np.linalg.norm(d)
    ref = 0.5 * d / r ** 3
    assert np.allclose(a[:, 0], ref, rtol=1e-15, atol=0)
    assert np.allclose(a[:, 1], -ref, rtol=1e-15, atol=0)
    assert np.allclose(ad, a, rtol=1e-14, atol=0)
    assert list(nint) == [1, 1]
