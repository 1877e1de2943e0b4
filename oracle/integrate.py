"""Time integration in the oracle (test infrastructure only; plain NumPy over
the oracle's force routines, shares nothing with the HIP path).

* ``leapfrog_bins``: the second-order kick-drift-kick leapfrog (Sec. 7.3)
  with the power-of-two time-step hierarchy of Sec. 7.2.  The interval
  ``dt_max`` is cut into 2^max_bin ticks; bin b steps by dt_max / 2^b.  A
  particle takes the bin of the largest step not above its criterion
  sqrt(2 C eps / |a|) (Sec. 7.1); it may always move to a shorter step and
  to a longer one only when the current time is a multiple of that step
  (otherwise it takes the longest synchronised step not shorter than the
  one it asks for).  Every active particle interacts with the full mass
  distribution.  At a bin boundary the closing half-kick of the old step
  and the opening half-kick of the new one are applied in turn.
* ``hierarchical``: the split Hamiltonian of Sec. 7.3 (after Pelupessy et
  al. 2012): over a step dt of level b, the particles P with bins >= b split
  into slow S (bin b) and fast F (bins > b);
      K_SF(dt/2)  KDK of H_S over dt  [F: two steps of level b + 1]  K_SF(dt/2)
  where K_SF kicks S and F with their mutual forces only and H_S = T_S + V_SS.
  Bins are assigned at the start of every dt_max step from the full force and
  kept over that step.  The mutual forces are the difference of the forces of
  P and of the part itself, so every level needs forces among P, S and F only.
  With a mesh (TreePM, Sec. 3.3) the split applies to the short-range
  Hamiltonian: each dt_max step is K_long(dt/2) [the split integration of
  T + V_short] K_long(dt/2), the long-range kicks taking the mesh force of
  all particles from all of them at the step's start and end (the mesh part
  moves on the longest step), and the bins come from |a_short + a_long|.

Arithmetic: a kick is v + a * dt per component with dt = 0.5 * dt_max *
2^-b, a drift is x + v * dt with dt = ticks * dt_max / 2^max_bin (products
rounded before the sums), periodic positions folded back by one box length.
"""
from __future__ import annotations

import math

import numpy as np

# test hook: a nonzero value plants one deliberate mistake (see the tests)
MUTATION = 0


def norm3(a):
    """|a| as sqrt(ax ax + ay ay + az az), in that order."""
    a = np.asarray(a, np.float64)
    return np.sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2])


def bin_of(anorm, eps, C, dt_max, max_bin):
    """Bin of the largest step dt_max / 2^b not above sqrt(2 C eps / |a|)."""
    anorm = np.asarray(anorm, np.float64)
    eps = np.broadcast_to(np.asarray(eps, np.float64), anorm.shape)
    out = np.empty(anorm.shape, np.int64)
    for i, (a, e) in enumerate(zip(anorm, eps)):
        if a <= 0.0:
            out[i] = 0
            continue
        dt = math.sqrt(2.0 * C * e / a)
        b = 0
        while b < max_bin and dt_max * 2.0 ** -b > dt:
            b += 1
        out[i] = b
    return out


def synchronised(b_new, b_old, t_ticks, max_bin):
    """Sec. 7.2: a shorter step is always allowed; a longer one only if the
    current tick is a multiple of its length (else the longest such step not
    shorter than the one asked for)."""
    b = int(b_new)
    if b >= b_old or MUTATION == 1:  # mutation 1: no synchronisation check
        return b
    while b < b_old and t_ticks % (1 << (max_bin - b)) != 0:
        b += 1
    return b


def kick(v, idx, a, dt):
    """v[:, idx] += a * dt (product rounded, then the sum)."""
    for c in range(3):
        v[c, idx] = v[c, idx] + a[c] * dt


def drift(x, v, dt, box=0.0):
    """x += v * dt (product rounded, then the sum); periodic positions are
    folded back by one box length."""
    for c in range(3):
        x[c] = x[c] + v[c] * dt
        if box > 0.0:
            x[c] = np.where(x[c] >= box, x[c] - box, np.where(x[c] < 0.0, x[c] + box, x[c]))


def leapfrog_bins(x, v, force, *, eps, C, dt_max, max_bin, n_max_steps, box=0.0,
                  record=None):
    """Advance positions x [3, n] and velocities v [3, n] (copies) over
    n_max_steps intervals dt_max.  force(x, targets) -> acc [3, len(targets)]
    from the full mass distribution.  Returns x, v (synchronised at the end)
    and per-step statistics; ``record`` (a list) receives per-kick events
    (tick, particle, old bin, new bin) for the tests."""
    x = np.array(x, np.float64)
    v = np.array(v, np.float64)
    n = x.shape[1]
    T = 1 << max_bin
    dt_tick = dt_max / T
    everyone = np.arange(n)
    acc = force(x, everyone)
    bins = bin_of(norm3(acc), eps, C, dt_max, max_bin)
    kick(v, everyone, acc, 0.5 * dt_max * np.exp2(-bins.astype(float)))
    ti = np.zeros(n, np.int64)  # tick of each particle's last kick
    t = 0
    t_end = n_max_steps * T
    nforce = n
    while t < t_end:
        step = np.left_shift(1, max_bin - bins)
        t_next = int((ti + step).min())
        drift(x, v, (t_next - t) * dt_tick, box)
        t = t_next
        act = np.nonzero(ti + step == t)[0]
        a = force(x, act)
        nforce += act.size
        old = bins[act]
        kick(v, act, a, 0.5 * dt_max * np.exp2(-old.astype(float)))  # close
        ti[act] = t
        if t == t_end:
            break
        want = bin_of(norm3(a), eps if np.ndim(eps) == 0 else
                      np.asarray(eps)[act], C, dt_max, max_bin)
        new = np.array([synchronised(w, o, t, max_bin) for w, o in zip(want, old)], np.int64)
        if record is not None:
            for i, o, b in zip(act, old, new):
                record.append((t, int(i), int(o), int(b)))
        bins[act] = new
        kick(v, act, a, 0.5 * dt_max * np.exp2(-new.astype(float)))  # open
    return x, v, {"force_evals": nforce, "final_bins": bins}


def hierarchical(x, v, force_sub, *, eps, C, dt_max, max_bin, n_max_steps, box=0.0,
                 force_long=None):
    """The split-Hamiltonian integration (Sec. 7.3).  force_sub(x, members)
    -> acc [3, len(members)] of the members from the members only (a tree or
    sum over that subset; the short-range force when there is a mesh).
    force_long(x) -> acc [3, n], the mesh force of all particles, or None.
    Returns x, v and statistics."""
    x = np.array(x, np.float64)
    v = np.array(v, np.float64)
    n = x.shape[1]
    stats = {"force_evals": 0, "levels": 0}

    def forces(members):
        stats["force_evals"] += members.size
        return force_sub(x, members)

    def kdk(P, dt):
        a = forces(P)
        kick(v, P, a, 0.5 * dt)
        xs = x[:, P]
        drift(xs, v[:, P], dt, box)
        x[:, P] = xs
        a = forces(P)
        kick(v, P, a, 0.5 * dt)

    def cross_kick(P, S, F, dt):
        aP = forces(P)
        pos = {int(i): k for k, i in enumerate(P)}
        aS = forces(S)
        aF = forces(F)
        kS = np.array([pos[int(i)] for i in S])
        kF = np.array([pos[int(i)] for i in F])
        if MUTATION != 2:  # mutation 2: the slow side misses its mutual kick
            kick(v, S, aP[:, kS] - aS, dt)
        kick(v, F, aP[:, kF] - aF, dt)

    def level(P, b, bins, dt):
        stats["levels"] = max(stats["levels"], b + 1)
        S = P[bins[P] <= b]
        F = P[bins[P] > b]
        if F.size == 0:
            kdk(P, dt)
            return
        if S.size == 0:
            level(F, b + 1, bins, 0.5 * dt)
            level(F, b + 1, bins, 0.5 * dt)
            return
        cross_kick(P, S, F, 0.5 * dt)
        kdk(S, dt)
        level(F, b + 1, bins, 0.5 * dt)
        level(F, b + 1, bins, 0.5 * dt)
        cross_kick(P, S, F, 0.5 * dt)

    everyone = np.arange(n)
    for _ in range(n_max_steps):
        a = forces(everyone)
        if force_long is None:
            bins = bin_of(norm3(a), eps, C, dt_max, max_bin)
        else:
            a_long = force_long(x)
            bins = bin_of(norm3(a + a_long), eps, C, dt_max, max_bin)
            if MUTATION != 3:  # mutation 3: the opening long-range kick is lost
                kick(v, everyone, a_long, 0.5 * dt_max)
        level(everyone, 0, bins, dt_max)
        if force_long is not None:
            kick(v, everyone, force_long(x), 0.5 * dt_max)
    return x, v, stats
