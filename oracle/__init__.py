"""FP64 CPU oracle for the TreePM gravity hot path (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  The product library never loads it, and it
shares no code with the HIP path.  The C source (``oracle.c``) is built by
``build()`` into ``liboracle.so`` next to it.

Parity notes: every function here is pinned by ``tests/test_oracle_*.py``
against the paper's statements, closed forms, exhaustive small cases or brute
force; the TreePM total force near the split scale has no printed reference in
the paper and is reported rather than gated (parity unpinned beyond the Ewald
comparison).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared"]


def build(out: str = _LIB, mutation: int = 0) -> str:
    """Compile the oracle (``mutation`` > 0 plants a test mistake)."""
    cmd = ["gcc", *CFLAGS, f"-DORC_MUTATION={mutation}", _SRC, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


class OrcParams(C.Structure):
    _fields_ = [("periodic", C.c_int), ("opening", C.c_int), ("treepm", C.c_int),
                ("want_pot", C.c_int), ("box", C.c_double), ("G", C.c_double),
                ("eps", C.c_double), ("theta", C.c_double), ("alpha", C.c_double),
                ("rs", C.c_double), ("rcut", C.c_double)]


def make_params(*, periodic=False, opening="bh", treepm=False, want_pot=False, box=0.0,
                G=1.0, eps=0.01, theta=0.5, alpha=0.0025, rs=0.0, rcut=0.0) -> OrcParams:
    op = {"bh": 0, "rel": 1}[opening]
    return OrcParams(int(periodic), op, int(treepm), int(want_pot), float(box), float(G),
                     float(eps), float(theta), float(alpha), float(rs), float(rcut))


_P = C.POINTER
_d = _P(C.c_double)
_i64 = _P(C.c_int64)
_u32 = _P(C.c_uint32)
_u64 = _P(C.c_uint64)
_i32 = _P(C.c_int32)


def _ptr(a, t):
    if a is None:
        return C.cast(None, t)
    return a.ctypes.data_as(t)


class Lib:
    def __init__(self, path: str = _LIB):
        if not os.path.exists(path):
            build(path)
        L = C.CDLL(path)
        self.L = L
        L.orc_ph_key.restype = C.c_uint64
        L.orc_ph_key.argtypes = [C.c_int, C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_ph_keys_b.argtypes = [C.c_int, C.c_int64, _u32, _u32, _u32, _u64]
        L.orc_frame.argtypes = [C.c_int64, _d, _d, _d, C.c_int, C.c_double, _d, _d]
        L.orc_positions.argtypes = [C.c_int64, _d, _d, _d, C.c_int, _d, _d, _u32, _u64]
        L.orc_sort.argtypes = [C.c_int64, _u64, _i64]
        L.orc_tree_build.restype = C.c_void_p
        L.orc_tree_build.argtypes = [C.c_int64, _d, _d, _d, _d, C.c_int, C.c_double, _d,
                                     _i64]
        L.orc_tree_entries.restype = C.c_int64
        L.orc_tree_entries.argtypes = [C.c_void_p]
        L.orc_tree_frame.argtypes = [C.c_void_p, _d]
        L.orc_tree_export.argtypes = [C.c_void_p, _i32, _i64, _i64, _i64, _i64, _d, _d, _d]
        L.orc_tree_positions.argtypes = [C.c_void_p, _d, _u32, _u64]
        L.orc_tree_free.argtypes = [C.c_void_p]
        L.orc_tree_walk.argtypes = [C.c_void_p, _P(OrcParams), C.c_int64, _i64, _d, _d, _d,
                                    _i64]
        L.orc_direct.argtypes = [C.c_int64, _d, _d, _d, _d, _d, _P(OrcParams), C.c_int64,
                                 _i64, _d, _d]
        L.orc_tree_set_softening.argtypes = [C.c_void_p, _d]
        L.orc_fft3.argtypes = [C.c_int, _d, _d, C.c_int]
        L.orc_pm_mesh.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, _d, _d, _d,
                                  _d, _d]
        L.orc_cic_deposit.argtypes = [C.c_int64, _d, _d, _d, _d, C.c_double, C.c_int, _d]
        L.orc_pm.argtypes = [C.c_int64, _d, _d, _d, _d, C.c_double, C.c_int, C.c_double,
                             C.c_double, C.c_int64, _i64, _d, _d]
        L.orc_pm_isolated.argtypes = [C.c_int64, _d, _d, _d, _d, _d, C.c_int, C.c_double,
                                      C.c_double, C.c_int, C.c_int64, _i64, _d, _d]
        L.orc_ewald.argtypes = [C.c_int64, _d, _d, _d, _d, C.c_double, C.c_double,
                                C.c_double, C.c_double, C.c_int64, _i64, _d]
        L.orc_max_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]


_lib: Lib | None = None


def lib() -> Lib:
    global _lib
    if _lib is None:
        _lib = Lib()
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _targets(n, targets):
    if targets is None:
        return np.arange(n, dtype=np.int64)
    return np.ascontiguousarray(targets, dtype=np.int64)


def max_threads() -> int:
    return lib().L.orc_max_threads()


def set_threads(k: int) -> None:
    lib().L.orc_set_threads(int(k))


# ---- keys ---------------------------------------------------------------

def ph_keys(b: int, q0, q1, q2) -> np.ndarray:
    q0, q1, q2 = (np.ascontiguousarray(v, dtype=np.uint32) for v in (q0, q1, q2))
    out = np.empty(q0.size, np.uint64)
    lib().L.orc_ph_keys_b(b, q0.size, _ptr(q0, _u32), _ptr(q1, _u32), _ptr(q2, _u32),
                          _ptr(out, _u64))
    return out


def frame(x, y, z, periodic=False, box=0.0, shift=(0.0, 0.0, 0.0)) -> np.ndarray:
    x, y, z = _f64(x), _f64(y), _f64(z)
    sh = _f64(shift)
    fr = np.empty(4)
    lib().L.orc_frame(x.size, _ptr(x, _d), _ptr(y, _d), _ptr(z, _d), int(periodic),
                      float(box), _ptr(sh, _d), _ptr(fr, _d))
    return fr


def positions(x, y, z, periodic, fr):
    """Tree-frame positions p [3, n], integer coordinates q [3, n] and keys."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.size
    fr = _f64(fr)
    p = np.empty(3 * n)
    q = np.empty(3 * n, np.uint32)
    key = np.empty(n, np.uint64)
    lib().L.orc_positions(n, _ptr(x, _d), _ptr(y, _d), _ptr(z, _d), int(periodic),
                          _ptr(fr, _d), _ptr(p, _d), _ptr(q, _u32), _ptr(key, _u64))
    return p.reshape(3, n), q.reshape(3, n), key


def sort(key) -> np.ndarray:
    key = np.ascontiguousarray(key, dtype=np.uint64)
    perm = np.empty(key.size, np.int64)
    lib().L.orc_sort(key.size, _ptr(key, _u64), _ptr(perm, _i64))
    return perm


# ---- tree ---------------------------------------------------------------

class Tree:
    """Insertion-built octree with its canonical depth-first entry list."""

    def __init__(self, x, y, z, mass=None, periodic=False, box=0.0,
                 shift=(0.0, 0.0, 0.0), insert_order=None, eps=None):
        self.x, self.y, self.z = _f64(x), _f64(y), _f64(z)
        self.n = self.x.size
        self.mass = None if mass is None else _f64(mass)
        self.periodic = bool(periodic)
        self.box = float(box)
        sh = _f64(shift)
        io = None if insert_order is None else np.ascontiguousarray(insert_order, np.int64)
        L = lib().L
        self.h = L.orc_tree_build(self.n, _ptr(self.x, _d), _ptr(self.y, _d),
                                  _ptr(self.z, _d), _ptr(self.mass, _d), int(periodic),
                                  float(box), _ptr(sh, _d), _ptr(io, _i64))
        self.E = L.orc_tree_entries(self.h)
        self.frame = np.empty(4)
        L.orc_tree_frame(self.h, _ptr(self.frame, _d))
        if eps is not None:  # individual softening lengths (Sec. 3.2)
            self.eps = _f64(eps)
            L.orc_tree_set_softening(self.h, _ptr(self.eps, _d))

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.L.orc_tree_free(h)
            self.h = None

    def export(self) -> dict:
        E = self.E
        out = dict(level=np.empty(E, np.int32), first=np.empty(E, np.int64),
                   count=np.empty(E, np.int64), skip=np.empty(E, np.int64),
                   pidx=np.empty(E, np.int64), mass=np.empty(E),
                   com=np.empty(3 * E), cen=np.empty(3 * E))
        lib().L.orc_tree_export(self.h, _ptr(out["level"], _i32), _ptr(out["first"], _i64),
                                _ptr(out["count"], _i64), _ptr(out["skip"], _i64),
                                _ptr(out["pidx"], _i64), _ptr(out["mass"], _d),
                                _ptr(out["com"], _d), _ptr(out["cen"], _d))
        out["com"] = out["com"].reshape(3, E)
        out["cen"] = out["cen"].reshape(3, E)
        return out

    def positions(self):
        n = self.n
        p = np.empty(3 * n)
        q = np.empty(3 * n, np.uint32)
        key = np.empty(n, np.uint64)
        lib().L.orc_tree_positions(self.h, _ptr(p, _d), _ptr(q, _u32), _ptr(key, _u64))
        return p.reshape(3, n), q.reshape(3, n), key

    def walk(self, params: OrcParams, targets=None, anorm=None):
        t = _targets(self.n, targets)
        nt = t.size
        acc = np.empty(3 * nt)
        pot = np.empty(nt) if params.want_pot else None
        nint = np.empty(nt, np.int64)
        an = None if anorm is None else _f64(anorm)
        if params.opening == 1 and an is None:
            raise ValueError("relative criterion needs |a_old|")
        lib().L.orc_tree_walk(self.h, C.byref(params), nt, _ptr(t, _i64), _ptr(an, _d),
                              _ptr(acc, _d), _ptr(pot, _d), _ptr(nint, _i64))
        return acc.reshape(3, nt), pot, nint


# ---- exact references ---------------------------------------------------

def direct(x, y, z, mass, params: OrcParams, targets=None, eps=None):
    """Direct pair sum; ``eps`` gives individual softening lengths (a pair
    uses the larger), else params.eps for all."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    m = None if mass is None else _f64(mass)
    e = None if eps is None else _f64(eps)
    t = _targets(x.size, targets)
    acc = np.empty(3 * t.size)
    pot = np.empty(t.size)
    lib().L.orc_direct(x.size, _ptr(x, _d), _ptr(y, _d), _ptr(z, _d), _ptr(m, _d),
                       _ptr(e, _d), C.byref(params), t.size, _ptr(t, _i64), _ptr(acc, _d),
                       _ptr(pot, _d))
    return acc.reshape(3, t.size), pot


def ewald(x, y, z, mass, box, G, eps, sigma, targets):
    x, y, z = _f64(x), _f64(y), _f64(z)
    m = None if mass is None else _f64(mass)
    t = _targets(x.size, targets)
    acc = np.empty(3 * t.size)
    lib().L.orc_ewald(x.size, _ptr(x, _d), _ptr(y, _d), _ptr(z, _d), _ptr(m, _d),
                      float(box), float(G), float(eps), float(sigma), t.size,
                      _ptr(t, _i64), _ptr(acc, _d))
    return acc.reshape(3, t.size)


# ---- particle mesh ------------------------------------------------------

def fft3(re, im, sign):
    n = re.shape[0]
    re = np.ascontiguousarray(re, np.float64).copy()
    im = np.ascontiguousarray(im, np.float64).copy()
    lib().L.orc_fft3(n, _ptr(re, _d), _ptr(im, _d), int(sign))
    return re, im


def cic_deposit(x, y, z, mass, box, ng):
    x, y, z = _f64(x), _f64(y), _f64(z)
    m = None if mass is None else _f64(mass)
    rho = np.empty(ng ** 3)
    lib().L.orc_cic_deposit(x.size, _ptr(x, _d), _ptr(y, _d), _ptr(z, _d), _ptr(m, _d),
                            float(box), ng, _ptr(rho, _d))
    return rho.reshape(ng, ng, ng)


def pm_mesh(rho, box, G, rs):
    ng = rho.shape[0]
    rho = np.ascontiguousarray(rho, np.float64)
    phi, fx, fy, fz = (np.empty(ng ** 3) for _ in range(4))
    lib().L.orc_pm_mesh(ng, float(box), float(G), float(rs), _ptr(rho, _d), _ptr(phi, _d),
                        _ptr(fx, _d), _ptr(fy, _d), _ptr(fz, _d))
    return tuple(a.reshape(ng, ng, ng) for a in (phi, fx, fy, fz))


def pm(x, y, z, mass, box, ng, G, rs, targets=None, want_pot=True):
    x, y, z = _f64(x), _f64(y), _f64(z)
    m = None if mass is None else _f64(mass)
    t = _targets(x.size, targets)
    acc = np.empty(3 * t.size)
    pot = np.empty(t.size) if want_pot else None
    lib().L.orc_pm(x.size, _ptr(x, _d), _ptr(y, _d), _ptr(z, _d), _ptr(m, _d), float(box),
                   int(ng), float(G), float(rs), t.size, _ptr(t, _i64), _ptr(acc, _d),
                   _ptr(pot, _d))
    return acc.reshape(3, t.size), pot


def isolated_scale(L_root, ng, asmth):
    """Mesh spacing and split scale of the isolated mesh: h = L / (ng - 4),
    r_s = asmth h."""
    h = float(L_root) / (int(ng) - 4)
    return h, float(asmth) * h


def pm_isolated(x, y, z, mass, frame4, ng, G, asmth, targets=None, want_pot=True,
                deconv=True):
    """Long-range force without periodicity (zero-padded (2 ng)^3 mesh over
    the root cube ``frame4`` = (x0, y0, z0, L)); acc [3][nt], pot [nt]."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    m = None if mass is None else _f64(mass)
    fr = _f64(frame4)
    t = _targets(x.size, targets)
    acc = np.empty(3 * t.size)
    pot = np.empty(t.size) if want_pot else None
    lib().L.orc_pm_isolated(x.size, _ptr(x, _d), _ptr(y, _d), _ptr(z, _d), _ptr(m, _d),
                            _ptr(fr, _d), int(ng), float(G), float(asmth), int(bool(deconv)),
                            t.size, _ptr(t, _i64), _ptr(acc, _d), _ptr(pot, _d))
    return acc.reshape(3, t.size), pot
