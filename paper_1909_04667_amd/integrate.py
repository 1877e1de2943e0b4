"""Time integration on the GPU (Sec. 7.1-7.3 of the Arepo paper).

``BlockLeapfrog`` is the kick-drift-kick leapfrog with the power-of-two time
bins of Sec. 7.2: every active particle interacts with the full mass
distribution (the tree is rebuilt from all particles at every sync point).
``Hierarchical`` is the split-Hamiltonian variant of Sec. 7.3: over a step of
level b the particles of bins >= b split into slow (bin b) and fast (bins >
b) parts; mutual kicks, the slow part's own leapfrog and two fast steps of
level b + 1, with trees built over the parts only.  With a mesh the split
applies to the short-range tree force and the mesh force kicks everyone on
the longest step (solved from all particles at its start and end).

Random placement (Sec. 3.1): with ``shift_seed`` every tree construction
takes a new root placement (non-periodic) or box shift (periodic), drawn
from a seeded generator here and passed to the library, so that tree force
errors decorrelate from step to step.

Every kick, drift, time-bin assignment, selection and gather runs in the
library's kernels (``tpm_kick``, ``tpm_drift``, ``tpm_time_bins``,
``tpm_select_bins``, ``tpm_gather``); this module only decides what runs when.
State lives on the device as FP64 arrays in the caller's particle order.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import binding as B


def _i32(n, dev):
    return torch.arange(n, dtype=torch.int32, device=dev)


class _Base:
    def __init__(self, pos, vel, mass=None, softening=None, *, C, dt_max, max_bin,
                 params=None, shift_seed=None, **ctx_kw):
        """pos, vel: (x, y, z) device FP64 tensors; mass: FP64 or None (1/n);
        softening: individual softening lengths or None (the context's eps);
        C, dt_max, max_bin: time-step parameter, longest step, deepest bin;
        shift_seed: None (the context's fixed placement) or the seed of the
        placements drawn before every build (three uniform numbers in [0, 1)
        per build, numpy's default generator); the context is made from
        ``params`` or the remaining keywords."""
        x, y, z = pos
        self.dev = x.device
        self.n = x.numel()
        self.x, self.y, self.z = (t.clone().contiguous() for t in (x, y, z))
        self.vx, self.vy, self.vz = (t.clone().contiguous() for t in vel)
        self.mass = None if mass is None else mass.contiguous()
        self.eps = None if softening is None else softening.contiguous()
        self.C, self.dt_max, self.max_bin = float(C), float(dt_max), int(max_bin)
        if not 0 <= self.max_bin <= 40:
            raise ValueError("max_bin must lie in [0, 40]")
        self.ctx = B.Context(params, **ctx_kw)
        P = self.ctx.params
        self.prec = P.precision
        self.eps0 = P.eps
        self.box = P.box_size if P.periodic else 0.0
        self.has_pm = P.pm_grid > 0
        self.bins = torch.zeros(self.n, dtype=torch.int32, device=self.dev)
        self.hist = torch.zeros(self.max_bin + 1, dtype=torch.int32, device=self.dev)
        self.force_evals = 0
        self.builds = 0
        self._shifts = None if shift_seed is None else np.random.default_rng(shift_seed)

    def _build(self, x, y, z, mass=None, eps=None):
        """One tree construction, with a new placement when shifts are on."""
        if self._shifts is not None:
            self.ctx.set_shift(self._shifts.random(3))
        self.ctx.build_tree(x, y, z, mass, eps=eps)
        self.builds += 1

    def momentum(self):
        """Total momentum sum m v (FP64, on the host)."""
        m = self.mass if self.mass is not None else \
            torch.full((self.n,), 1.0 / self.n, dtype=torch.float64, device=self.dev)
        return np.array([float((m * t).sum()) for t in (self.vx, self.vy, self.vz)])

    # -- kernel calls through the C ABI -------------------------------------------
    def _kick(self, idx, acc, acc_b=None, b_sign=1, dt=0.0, by_bins=False):
        L = B.lib()
        self.ctx._rc(L.tpm_kick(self.ctx.h, self.n, idx.numel(), B._ptr(idx), self.prec,
                                B._ptr(acc), B._ptr(acc_b), int(b_sign),
                                B._ptr(self.bins) if by_bins else None, self.dt_max,
                                float(dt), B._ptr(self.vx), B._ptr(self.vy), B._ptr(self.vz)))

    def _drift(self, idx, dt):
        L = B.lib()
        m = self.n if idx is None else idx.numel()
        self.ctx._rc(L.tpm_drift(self.ctx.h, self.n, m, B._ptr(idx), B._ptr(self.x),
                                 B._ptr(self.y), B._ptr(self.z), B._ptr(self.vx),
                                 B._ptr(self.vy), B._ptr(self.vz), float(dt), self.box))

    def _time_bins(self, idx, acc, acc_b, t):
        self.hist.zero_()
        self.ctx._rc(B.lib().tpm_time_bins(
            self.ctx.h, self.n, idx.numel(), B._ptr(idx), self.prec, B._ptr(acc),
            B._ptr(acc_b), B._ptr(self.eps), self.eps0, self.C, self.dt_max, self.max_bin,
            int(t), B._ptr(self.bins), B._ptr(self.hist)))
        return self.hist.cpu().numpy().astype(np.int64)

    def _select(self, lst, mode, t=0, level=0, local=False):
        m = self.n if lst is None else lst.numel()
        out = torch.empty(max(m, 1), dtype=torch.int32, device=self.dev)
        n_out = ctypes.c_int64(0)
        self.ctx._rc(B.lib().tpm_select_bins(self.ctx.h, m, B._ptr(lst), B._ptr(self.bins),
                                             int(mode), int(t), int(level), self.max_bin,
                                             int(local), B._ptr(out), ctypes.byref(n_out)))
        return out[: n_out.value]


class BlockLeapfrog(_Base):
    """Leapfrog with power-of-two time bins (Sec. 7.2, 7.3): the same event
    sequence as the reference integrator (initial half kick; per sync point
    drift of everyone, force on the active ones, closing half kick, new bin,
    opening half kick)."""

    def _force(self, idx):
        self._build(self.x, self.y, self.z, self.mass, eps=self.eps)
        a, _ = self.ctx.compute_forces(idx, "bh", want_pot=False)
        apm = self.ctx.pm_long_range(idx, want_pot=False)[0] if self.has_pm else None
        self.force_evals += idx.numel()
        return a, apm

    def run(self, n_max_steps):
        N = self.max_bin
        T = 1 << N
        dt_tick = self.dt_max / T
        everyone = _i32(self.n, self.dev)
        a, apm = self._force(everyone)
        occ = self._time_bins(everyone, a, apm, 0)
        self._kick(everyone, a, apm, 1, by_bins=True)
        t, t_end = 0, int(n_max_steps) * T
        steps = 0
        while t < t_end:
            b_max = int(np.nonzero(occ)[0].max())
            s_min = 1 << (N - b_max)
            t_next = (t // s_min + 1) * s_min
            self._drift(None, (t_next - t) * dt_tick)
            t = t_next
            act = self._select(None, 0, t=t)
            a, apm = self._force(act)
            self._kick(act, a, apm, 1, by_bins=True)  # close the old step
            steps += 1
            if t == t_end:
                break
            # every particle of a bin whose step divides t is active
            for b in range(N + 1):
                if t % (1 << (N - b)) == 0:
                    occ[b] = 0
            occ += self._time_bins(act, a, apm, t)
            self._kick(act, a, apm, 1, by_bins=True)  # open the new step
        self.ctx.check()
        return {"sync_points": steps, "force_evals": self.force_evals, "builds": self.builds}


class Hierarchical(_Base):
    """Split-Hamiltonian integration (Sec. 7.3; Pelupessy et al. 2012), with
    the mesh force (if the context has a mesh) on the longest step."""

    def __init__(self, *a, **kw):
        super().__init__(*a, **kw)
        if self.mass is None:  # a tree over a part must keep the system's masses
            self.mass = torch.full((self.n,), 1.0 / self.n, dtype=torch.float64,
                                   device=self.dev)
        z = lambda: torch.empty(self.n, dtype=torch.float64, device=self.dev)
        self.sx, self.sy, self.sz = z(), z(), z()
        self.sm = z() if self.mass is not None else None
        self.se = z() if self.eps is not None else None
        self.levels = 0

    def _gather(self, idx, src, dst):
        self.ctx._rc(B.lib().tpm_gather(self.ctx.h, self.n, idx.numel(), B._ptr(idx),
                                        B._ptr(src), B._ptr(dst)))

    def _build_sub(self, members):
        m = members.numel()
        for s, d in ((self.x, self.sx), (self.y, self.sy), (self.z, self.sz)):
            self._gather(members, s, d)
        if self.sm is not None:
            self._gather(members, self.mass, self.sm)
        if self.se is not None:
            self._gather(members, self.eps, self.se)
        sl = lambda t: None if t is None else t[:m]
        self._build(self.sx[:m], self.sy[:m], self.sz[:m], sl(self.sm), eps=sl(self.se))

    def _forces(self, members, targets_local=None):
        """Forces among ``members`` at the members listed (by position) in
        targets_local, or at all of them."""
        self._build_sub(members)
        t = _i32(members.numel(), self.dev) if targets_local is None else targets_local
        a, _ = self.ctx.compute_forces(t, "bh", want_pot=False)
        self.force_evals += t.numel()
        return a

    def _kdk(self, P, dt):
        a = self._forces(P)
        self._kick(P, a, dt=0.5 * dt)
        self._drift(P, dt)
        a = self._forces(P)
        self._kick(P, a, dt=0.5 * dt)

    def _cross(self, P, S_loc, S, F_loc, F, h):
        self._build_sub(P)
        aPS, _ = self.ctx.compute_forces(S_loc, "bh", want_pot=False)
        aPF, _ = self.ctx.compute_forces(F_loc, "bh", want_pot=False)
        aS = self._forces(S)
        aF = self._forces(F)
        self.force_evals += P.numel()
        self._kick(S, aPS, aS, -1, dt=h)
        self._kick(F, aPF, aF, -1, dt=h)

    def _level(self, P, b, dt):
        self.levels = max(self.levels, b + 1)
        S_loc = self._select(P, 1, level=b, local=True)
        F_loc = self._select(P, 2, level=b, local=True)
        if F_loc.numel() == 0:
            self._kdk(P, dt)
            return
        F = self._select(P, 2, level=b)
        if S_loc.numel() == 0:
            self._level(F, b + 1, 0.5 * dt)
            self._level(F, b + 1, 0.5 * dt)
            return
        S = self._select(P, 1, level=b)
        self._cross(P, S_loc, S, F_loc, F, 0.5 * dt)
        self._kdk(S, dt)
        self._level(F, b + 1, 0.5 * dt)
        self._level(F, b + 1, 0.5 * dt)
        self._cross(P, S_loc, S, F_loc, F, 0.5 * dt)

    def _long(self, everyone):
        """Mesh force of all particles from all of them (the last build must
        be over everyone: the mesh is solved from the particles of the last
        build)."""
        a, _ = self.ctx.pm_long_range(everyone, want_pot=False)
        self.force_evals += self.n
        return a

    def run(self, n_max_steps):
        everyone = _i32(self.n, self.dev)
        for _ in range(int(n_max_steps)):
            a = self._forces(everyone)
            if not self.has_pm:
                self._time_bins(everyone, a, None, 0)
                self._level(everyone, 0, self.dt_max)
                continue
            a_long = self._long(everyone)
            self._time_bins(everyone, a, a_long, 0)
            self._kick(everyone, a_long, dt=0.5 * self.dt_max)
            self._level(everyone, 0, self.dt_max)
            self._build_sub(everyone)
            self._kick(everyone, self._long(everyone), dt=0.5 * self.dt_max)
        self.ctx.check()
        return {"levels": self.levels, "force_evals": self.force_evals, "builds": self.builds}
