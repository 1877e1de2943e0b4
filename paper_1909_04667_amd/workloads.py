"""Seeded synthetic inputs shaped like the gravity workloads of the Arepo paper.

This module only draws particle positions, masses, active sets and request
streams.  It holds none of the force method's arithmetic (no keys, no tree, no
softening, no mesh solve); both the FP64 CPU oracle and the HIP library are fed
from here so that they see identical inputs.

Every generator uses ``numpy.random.Generator(PCG64(seed))``.

Units: G = 1, total mass M = 1, equal particle masses m = 1/N (the paper's
gravity parameters, Table 1, do not fix units; a = 1, i.e. a static space).

Workloads (the paper's own initial conditions are not public, these stand in):

* ``plummer``   truncated Plummer sphere (isolated galaxy-like, Section 3.1/3.2)
* ``hernquist`` truncated Hernquist halo (isolated, cuspy)
* ``zeldovich_box`` periodic box, grid + Zel'dovich displacement of a Gaussian
  field with P(k) ~ k^-2 (cosmological box, Section 3.4 TreePM)
* ``lognormal_box`` periodic clustered box, lognormal density with
  sigma_ln(rho) = 2 (local time-stepping workload, Section 7.2/7.3)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _isotropic(rng: np.random.Generator, r: np.ndarray):
    cth = rng.uniform(-1.0, 1.0, r.size)
    phi = rng.uniform(0.0, 2.0 * math.pi, r.size)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    return r * sth * np.cos(phi), r * sth * np.sin(phi), r * cth


def plummer_mass_fraction(r_trunc: float, b: float = 1.0) -> float:
    """Untruncated Plummer enclosed-mass fraction M(<r_t)/M."""
    return r_trunc ** 3 / (r_trunc ** 2 + b ** 2) ** 1.5


def hernquist_mass_fraction(r_trunc: float, a: float = 1.0) -> float:
    """Untruncated Hernquist enclosed-mass fraction M(<r_t)/M."""
    return r_trunc ** 2 / (r_trunc + a) ** 2


@dataclass
class Particles:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    mass: np.ndarray | None = None          # None => equal masses 1/N
    periodic: bool = False
    box: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.size)

    def masses(self) -> np.ndarray:
        if self.mass is not None:
            return self.mass
        return np.full(self.n, 1.0 / self.n)


def plummer(n: int, seed: int = 1, b: float = 1.0, r_trunc: float = 20.0,
            velocities: bool = False) -> Particles:
    """Plummer sphere, total (truncated) mass 1, radii by inverse CDF.

    r = b / sqrt(X^(-2/3) - 1) with X ~ U(0, f_t), f_t = M(<r_t)/M.
    Velocities (optional, unused by the force path) by the Aarseth-Henon-
    Wielen rejection sampling of the isotropic distribution function.
    """
    rng = _rng(seed)
    ft = plummer_mass_fraction(r_trunc, b)
    X = rng.uniform(0.0, ft, n)
    with np.errstate(divide="ignore"):
        r = b / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    x, y, z = _isotropic(rng, r)
    meta = {"kind": "plummer", "b": b, "r_trunc": r_trunc, "f_t": ft, "seed": seed}
    p = Particles(x, y, z, None, False, 0.0, meta)
    if velocities:
        q = np.empty(n)
        filled = np.zeros(n, bool)
        while not filled.all():
            k = (~filled).sum()
            qq = rng.uniform(0.0, 1.0, k)
            gg = rng.uniform(0.0, 0.1, k)
            ok = gg < qq * qq * (1.0 - qq * qq) ** 3.5
            idx = np.flatnonzero(~filled)[ok]
            q[idx] = qq[ok]
            filled[idx] = True
        # escape speed of the (untruncated) model, scaled to the truncated mass
        vesc = np.sqrt(2.0 / ft) * (r * r + b * b) ** -0.25
        p.meta["v"] = _isotropic(rng, q * vesc)
    return p


def hernquist(n: int, seed: int = 2, a: float = 1.0, r_trunc: float = 100.0) -> Particles:
    """Hernquist halo, total (truncated) mass 1.

    M(<r)/M = r^2/(r+a)^2, so r = a sqrt(X) / (1 - sqrt(X)), X ~ U(0, f_t).
    """
    rng = _rng(seed)
    ft = hernquist_mass_fraction(r_trunc * a, a)
    X = rng.uniform(0.0, ft, n)
    s = np.sqrt(X)
    r = a * s / (1.0 - s)
    x, y, z = _isotropic(rng, r)
    meta = {"kind": "hernquist", "a": a, "r_trunc": r_trunc, "f_t": ft, "seed": seed}
    return Particles(x, y, z, None, False, 0.0, meta)


def uniform_cube(n: int, seed: int, side: float = 1.0) -> Particles:
    rng = _rng(seed)
    x, y, z = rng.uniform(0.0, side, (3, n))
    return Particles(x, y, z, None, False, 0.0, {"kind": "uniform", "seed": seed})


def _gaussian_field(rng: np.random.Generator, ng: int, slope: float = -2.0):
    """Real Gaussian random field on ng^3 with power spectrum ~ k^slope.

    White noise is drawn in real space and coloured in Fourier space, which
    makes the modes Hermitian by construction.  k = 0 and the Nyquist planes
    are removed.  Returns (delta_k on the rfft grid, kx, ky, kz integer grids).
    """
    white = rng.standard_normal((ng, ng, ng))
    wk = np.fft.rfftn(white)
    n1 = np.fft.fftfreq(ng, 1.0 / ng)
    n3 = np.fft.rfftfreq(ng, 1.0 / ng)
    nx = n1[:, None, None]
    ny = n1[None, :, None]
    nz = n3[None, None, :]
    k2 = nx * nx + ny * ny + nz * nz
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (slope / 4.0), 0.0)
    half = ng // 2
    nyq = (np.abs(nx) == half) | (np.abs(ny) == half) | (np.abs(nz) == half)
    amp = np.where(nyq, 0.0, amp)
    return wk * amp, nx, ny, nz, k2


def zeldovich_box(ng: int = 128, box: float = 100.0, seed: int = 3,
                  rms_cells: float = 0.1) -> Particles:
    """Grid of ng^3 particles displaced by the Zel'dovich field psi.

    delta_k Gaussian with P(k) ~ k^-2, psi_k = i k delta_k / k^2 (so that
    div psi = -delta), normalised so that the 3-D rms |psi| equals
    ``rms_cells`` mesh cells.  Positions are wrapped into [0, box).
    """
    rng = _rng(seed)
    dk, nx, ny, nz, k2 = _gaussian_field(rng, ng)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = np.where(k2 > 0, 1.0 / k2, 0.0)
    psi = [np.fft.irfftn(1j * kk * dk * inv, s=(ng, ng, ng), axes=(0, 1, 2)) for kk in (nx, ny, nz)]
    rms = math.sqrt(sum(float(np.mean(c * c)) for c in psi))
    cell = box / ng
    scale = rms_cells * cell / rms
    g = (np.arange(ng) + 0.5) * cell
    qx, qy, qz = np.meshgrid(g, g, g, indexing="ij")
    pos = []
    for q, c in zip((qx, qy, qz), psi):
        v = (q + scale * c).reshape(-1)
        v = np.mod(v, box)
        v[v >= box] = 0.0
        pos.append(v)
    meta = {"kind": "zeldovich", "ng": ng, "box": box, "seed": seed, "rms_cells": rms_cells}
    return Particles(pos[0], pos[1], pos[2], None, True, box, meta)


def lognormal_box(ng: int = 256, box: float = 100.0, seed: int = 4,
                  sigma_ln: float = 2.0, n: int | None = None) -> Particles:
    """Clustered periodic box: N cell draws from rho ~ exp(g - sigma^2/2).

    g is a Gaussian field on ng^3 with P(k) ~ k^-2 scaled to std sigma_ln.
    Each particle picks a cell from the categorical distribution ~ rho (by
    inverse CDF on sorted uniforms) and a uniform position inside it.  The
    cell's density is kept in ``meta['rho']`` (per particle), which sets the
    particle's dynamical time and hence its time-step bin.
    """
    rng = _rng(seed)
    n = ng ** 3 if n is None else n
    dk, *_ = _gaussian_field(rng, ng)
    gfield = np.fft.irfftn(dk, s=(ng, ng, ng), axes=(0, 1, 2))
    gfield *= sigma_ln / gfield.std()
    rho = np.exp(gfield - 0.5 * sigma_ln ** 2).reshape(-1)
    del gfield, dk
    cdf = np.cumsum(rho)
    cdf /= cdf[-1]
    u = rng.uniform(0.0, 1.0, n)
    cell = np.searchsorted(cdf, u, side="right")
    np.minimum(cell, ng ** 3 - 1, out=cell)
    del cdf, u
    h = box / ng
    ix, rem = np.divmod(cell, ng * ng)
    iy, iz = np.divmod(rem, ng)
    off = rng.uniform(0.0, 1.0, (3, n))
    pos = []
    for i, o in zip((ix, iy, iz), off):
        v = (i + o) * h
        v[v >= box] -= box
        pos.append(v)
    meta = {"kind": "lognormal", "ng": ng, "box": box, "seed": seed,
            "sigma_ln": sigma_ln, "rho": rho[cell]}
    return Particles(pos[0], pos[1], pos[2], None, True, box, meta)


def time_bin_active_sets(rho: np.ndarray, fractions=(0.001, 0.01, 0.1, 1.0)):
    """Nested active sets from power-of-two time-step bins.

    A particle's time step scales with its local dynamical time,
    dt ~ (G rho)^(-1/2); bins are dt_max / 2^bin.  The set active at a
    synchronisation point of bin b is every particle in bins >= b, i.e. the
    densest particles.  To hit the requested fractions exactly, particles are
    ranked by density (ties by index) and the top f*N are taken, which yields
    nested sets.  Returns ({f: sorted int32 index array}, bins array).
    """
    n = rho.size
    order = np.lexsort((np.arange(n), -rho))
    tdyn = 1.0 / np.sqrt(rho)
    bins = np.floor(np.log2(tdyn.max() / tdyn)).astype(np.int32)
    sets = {}
    for f in fractions:
        k = max(1, int(round(f * n)))
        sets[f] = np.sort(order[:k]).astype(np.int32)
    return sets, bins


def random_active(n: int, frac: float, seed: int) -> np.ndarray:
    rng = _rng(seed)
    k = max(1, int(round(frac * n)))
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int32)


CONFIGS = {
    1: dict(name="plummer_4096", kind="plummer", n=4096, eps=0.01, opening="bh",
            theta=0.5, periodic=False, seed=1),
    2: dict(name="hernquist_2p20", kind="hernquist", n=1 << 20, eps=0.005,
            opening="bh_then_rel", theta=0.5, alpha=0.0025, periodic=False, seed=2),
    3: dict(name="zeldovich_128c_pm256", kind="zeldovich", ng=128, box=100.0,
            eps=100.0 / (50 * 128), pm_grid=256, asmth=1.25, rcut=4.5,
            opening="bh_then_rel", theta=0.5, alpha=0.0025, periodic=True, seed=3),
    4: dict(name="lognormal_256c_pm256", kind="lognormal", ng=256, box=100.0,
            eps=100.0 / (50 * 256), pm_grid=256, asmth=1.25, rcut=4.5,
            opening="bh_then_rel", theta=0.5, alpha=0.0025, periodic=True, seed=4),
}


def make_config(cfg: int, scale: int = 1) -> Particles:
    """Particles of a numbered workload; ``scale`` > 1 shrinks N (tests)."""
    c = CONFIGS[cfg]
    if c["kind"] == "plummer":
        return plummer(max(2, c["n"] // scale), c["seed"])
    if c["kind"] == "hernquist":
        return hernquist(max(2, c["n"] // scale), c["seed"])
    if c["kind"] == "zeldovich":
        return zeldovich_box(max(4, c["ng"] // scale), c["box"], c["seed"])
    if c["kind"] == "lognormal":
        return lognormal_box(max(4, c["ng"] // scale), c["box"], c["seed"])
    raise ValueError(cfg)


# --------------------------------------------------------------------------
# Serving request stream (Poisson arrivals over mixed systems)
# --------------------------------------------------------------------------

@dataclass
class SystemSpec:
    sid: int
    kind: str          # plummer | hernquist | periodic
    n: int
    seed: int


@dataclass
class Request:
    rid: int
    t_arrival: float   # seconds after the start of the stream
    sid: int           # index into the system pool
    f_active: float
    precision: str     # fp32 | fp64
    seed: int          # draws the active subset


def system_pool(n_systems: int, seed: int = 5, log2n=(10, 21)):
    """Systems of uneven size: kind uniform over {plummer, hernquist,
    periodic}, N = 2^U(log2n) rounded (periodic: the nearest cube)."""
    rng = _rng(seed)
    kinds = rng.choice(["plummer", "hernquist", "periodic"], n_systems)
    ns = np.rint(2.0 ** rng.uniform(*log2n, n_systems)).astype(np.int64)
    seeds = rng.integers(0, 2 ** 31, n_systems)
    out = []
    for i in range(n_systems):
        n = int(ns[i])
        if kinds[i] == "periodic":
            n = max(8, int(round(n ** (1.0 / 3.0)))) ** 3
        out.append(SystemSpec(i, str(kinds[i]), n, int(seeds[i])))
    return out


def request_stream(n_requests: int, rate: float, n_systems: int, seed: int = 5,
                   log10f=(-3.0, 0.0)):
    """Poisson arrivals at ``rate`` per second over a pool of systems; each
    request picks a system, an active fraction 10^U(log10f) (the share of
    particles in the time-step bins due at that moment) and a precision."""
    rng = _rng(seed + 1)
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests)) if rate > 0 else np.zeros(n_requests)
    sids = rng.integers(0, n_systems, n_requests)
    fs = 10.0 ** rng.uniform(*log10f, n_requests)
    prec = rng.choice(["fp32", "fp64"], n_requests)
    seeds = rng.integers(0, 2 ** 31, n_requests)
    return [Request(i, float(t[i]), int(sids[i]), float(fs[i]), str(prec[i]), int(seeds[i]))
            for i in range(n_requests)]


def system_particles(spec: SystemSpec) -> Particles:
    if spec.kind == "plummer":
        return plummer(spec.n, spec.seed)
    if spec.kind == "hernquist":
        return hernquist(spec.n, spec.seed)
    ng = int(round(spec.n ** (1.0 / 3.0)))
    return zeldovich_box(ng, 100.0, spec.seed)


def request_active(req: Request, n: int) -> np.ndarray:
    """The request's active set: a seeded random subset of size f_active N."""
    return random_active(n, req.f_active, req.seed)
