"""Thin ctypes binding of ``libtreepm.so`` (argument marshalling only).

Every step of the force computation runs in the library's HIP kernels; this
module only turns torch tensors into device pointers and the current torch
stream into the library's stream.  If the library is missing the binding
raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtreepm.so")

TPM_OK, TPM_EINVAL, TPM_ENOMEM, TPM_EDEVICE, TPM_ESTATE, TPM_EINDEX = 0, -1, -2, -3, -4, -5
OPEN = {"bh": 0, "rel": 1}
PRECISION = {"fp64": 0, "fp32": 1}


class TpmParams(C.Structure):
    _fields_ = [("periodic", C.c_int32), ("precision", C.c_int32),
                ("want_potential", C.c_int32), ("pm_grid", C.c_int32),
                ("box_size", C.c_double), ("G", C.c_double), ("eps", C.c_double),
                ("theta", C.c_double), ("alpha", C.c_double), ("asmth", C.c_double),
                ("rcut", C.c_double), ("shift", C.c_double * 3)]


class TreePMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"treepm error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with paper_1909_04667_amd.build.build() "
                "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        P = C.POINTER
        L.tpm_create.argtypes = [P(TpmParams), vp, P(vp)]
        L.tpm_create_arena.argtypes = [P(TpmParams), vp, i64, P(vp)]
        L.tpm_destroy.argtypes = [vp]
        L.tpm_last_error.argtypes = [vp]
        L.tpm_last_error.restype = C.c_char_p
        L.tpm_set_stream.argtypes = [vp, vp]
        L.tpm_bytes_needed.argtypes = [P(TpmParams), i64]
        L.tpm_bytes_needed.restype = i64
        L.tpm_bytes_held.argtypes = [vp]
        L.tpm_bytes_held.restype = i64
        L.tpm_build_tree.argtypes = [vp, i64, vp, vp, vp, vp]
        L.tpm_build_tree_eps.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.tpm_compute_forces.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp]
        L.tpm_pm_long_range.argtypes = [vp, i64, vp, vp, vp]
        L.tpm_set_shift.argtypes = [vp, P(d)]
        L.tpm_compute_forces_noalloc.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp]
        L.tpm_noalloc_max_n.restype = i64
        L.tpm_check.argtypes = [vp]
        L.tpm_tree_info.argtypes = [vp, P(i64), P(i64), P(d)]
        L.tpm_export_tree.argtypes = [vp] + [vp] * 10
        L.tpm_accel_norm.argtypes = [vp, i64, vp, vp, vp, vp]
        L.tpm_export_mesh.argtypes = [vp, vp, vp]
        L.tpm_probe_fma.argtypes = [i32, vp, vp, P(d)]
        L.tpm_probe_copy.argtypes = [vp, vp, i64, vp, P(d)]
        L.tpm_timing_enable.argtypes = [vp, C.c_int]
        L.tpm_timing_read.argtypes = [vp, C.c_int, P(d), P(i64)]
        L.tpm_timing_durations.argtypes = [vp, C.c_int, P(d), i64, P(i64)]
        L.tpm_server_create.argtypes = [i32, d, P(vp)]
        L.tpm_server_destroy.argtypes = [vp]
        L.tpm_server_last_error.argtypes = [vp]
        L.tpm_server_last_error.restype = C.c_char_p
        L.tpm_server_submit.argtypes = [vp, vp, i32, i64, vp, vp, vp, vp, P(C.c_uint64)]
        L.tpm_server_submit_step.argtypes = [vp, vp, i64, vp, vp, vp, vp, P(C.c_uint64)]
        L.tpm_server_poll.argtypes = [vp, C.c_uint64]
        L.tpm_server_wait.argtypes = [vp, C.c_uint64]
        L.tpm_server_info.argtypes = [vp, P(i64), P(i64)]
        L.tpm_batch_create.argtypes = [vp, P(vp)]
        L.tpm_batch_destroy.argtypes = [vp]
        L.tpm_batch_last_error.argtypes = [vp]
        L.tpm_batch_last_error.restype = C.c_char_p
        L.tpm_batch_add.argtypes = [vp, vp, i32, i64, vp, vp, vp, vp]
        L.tpm_batch_launch.argtypes = [vp]
        L.tpm_kick.argtypes = [vp, i64, i64, vp, i32, vp, vp, i32, vp, d, d, vp, vp, vp]
        L.tpm_drift.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, d, d]
        L.tpm_time_bins.argtypes = [vp, i64, i64, vp, i32, vp, vp, vp, d, d, d, i32, i64, vp,
                                    vp]
        L.tpm_select_bins.argtypes = [vp, i64, vp, vp, i32, i64, i32, i32, i32, vp, P(i64)]
        L.tpm_gather.argtypes = [vp, i64, i64, vp, vp, vp]
        _lib = L
    return _lib


def make_params(*, periodic=False, precision="fp64", want_potential=False, pm_grid=0,
                box_size=0.0, G=1.0, eps=0.01, theta=0.5, alpha=0.0025, asmth=1.25,
                rcut=4.5, shift=(0.0, 0.0, 0.0)) -> TpmParams:
    p = TpmParams()
    p.periodic = int(periodic)
    p.precision = PRECISION[precision]
    p.want_potential = int(want_potential)
    p.pm_grid = int(pm_grid)
    p.box_size = float(box_size)
    p.G = float(G)
    p.eps = float(eps)
    p.theta = float(theta)
    p.alpha = float(alpha)
    p.asmth = float(asmth)
    p.rcut = float(rcut)
    for a in range(3):
        p.shift[a] = float(shift[a])
    return p


def probe_fma(precision: str, stream=None) -> float:
    """Measured dependent-FMA rate of the device in TFLOP/s."""
    sink = torch.zeros(2, dtype=torch.float64, device="cuda")
    out = C.c_double()
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = lib().tpm_probe_fma(PRECISION[precision], _ptr(sink), _stream_handle(st), C.byref(out))
    if rc != TPM_OK:
        raise TreePMError(rc, "tpm_probe_fma failed")
    return float(out.value)


def probe_copy(nbytes: int = 1 << 30, stream=None) -> float:
    """Measured streaming-copy bandwidth (read + write) in GB/s."""
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = C.c_double()
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = lib().tpm_probe_copy(_ptr(src), _ptr(dst), 4 * n, _stream_handle(st), C.byref(out))
    if rc != TPM_OK:
        raise TreePMError(rc, "tpm_probe_copy failed")
    return float(out.value)


def noalloc_max_n() -> int:
    return int(lib().tpm_noalloc_max_n())


def bytes_needed(params: TpmParams, n: int) -> int:
    return int(lib().tpm_bytes_needed(C.byref(params), int(n)))


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensors must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class Context:
    """One tree (and PM mesh) on one device, bound to a stream."""

    def __init__(self, params: TpmParams | None = None, stream=None, arena_bytes=None, **kw):
        """arena_bytes: None (buffers allocated as needed) or the size of the
        one device arena the context works in (tpm_create_arena)."""
        self.params = params if params is not None else make_params(**kw)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.dtype = torch.float32 if self.params.precision == 1 else torch.float64
        h = C.c_void_p()
        if arena_bytes is None:
            rc = lib().tpm_create(C.byref(self.params), _stream_handle(self.stream),
                                  C.byref(h))
        else:
            rc = lib().tpm_create_arena(C.byref(self.params), _stream_handle(self.stream),
                                        int(arena_bytes), C.byref(h))
        if rc != TPM_OK:
            raise TreePMError(rc, "tpm_create rejected the parameters or the arena")
        self.h = h
        self.n = 0
        self._keep = ()

    def _rc(self, rc):
        if rc != TPM_OK:
            raise TreePMError(rc, lib().tpm_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().tpm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self.stream = stream
        self._rc(lib().tpm_set_stream(self.h, _stream_handle(stream)))

    # -- the three operations of the hot path ---------------------------------
    def set_shift(self, shift):
        """Root placement for the builds that follow (three numbers in [0, 1),
        drawn by the caller)."""
        arr = (C.c_double * 3)(*[float(v) for v in shift])
        self._rc(lib().tpm_set_shift(self.h, arr))

    def build_tree(self, x, y, z, mass=None, eps=None):
        """eps: optional individual softening lengths (float64, build order)."""
        extra = tuple(t for t in (mass, eps) if t is not None)
        for t in (x, y, z) + extra:
            if t.dtype != torch.float64:
                raise ValueError("positions, masses and softenings must be float64")
        n = x.numel()
        self._keep = (x, y, z, mass, eps)  # inputs stay alive while the stream uses them
        self._rc(lib().tpm_build_tree_eps(self.h, n, _ptr(x), _ptr(y), _ptr(z), _ptr(mass),
                                          _ptr(eps)))
        self.n = n

    def compute_forces(self, active_idx, opening="bh", a_old_norm=None, acc=None, pot=None,
                       n_interactions=None, want_pot=None):
        if active_idx.dtype != torch.int32:
            raise ValueError("active_idx must be int32")
        na = active_idx.numel()
        dev = active_idx.device
        if acc is None:
            acc = torch.empty((3, na), dtype=self.dtype, device=dev)
        if pot is None and (want_pot or (want_pot is None and self.params.want_potential)):
            pot = torch.empty(na, dtype=self.dtype, device=dev)
        if a_old_norm is not None and a_old_norm.dtype != torch.float64:
            raise ValueError("a_old_norm must be float64")
        self._rc(lib().tpm_compute_forces(self.h, OPEN[opening], na, _ptr(active_idx),
                                          _ptr(a_old_norm), _ptr(acc), _ptr(pot),
                                          _ptr(n_interactions)))
        return acc, pot

    def compute_forces_noalloc(self, active_idx, opening="bh", a_old_norm=None, acc=None,
                               pot=None, n_interactions=None):
        """compute_forces through the allocation-free entry point; the caller
        passes every output (acc [3][n_act] of the context's dtype, pot and
        n_interactions optional)."""
        if active_idx.dtype != torch.int32:
            raise ValueError("active_idx must be int32")
        if a_old_norm is not None and a_old_norm.dtype != torch.float64:
            raise ValueError("a_old_norm must be float64")
        self._rc(lib().tpm_compute_forces_noalloc(self.h, OPEN[opening], active_idx.numel(),
                                                  _ptr(active_idx), _ptr(a_old_norm),
                                                  _ptr(acc), _ptr(pot), _ptr(n_interactions)))
        return acc, pot

    def pm_long_range(self, active_idx, acc=None, pot=None, want_pot=None):
        if active_idx.dtype != torch.int32:
            raise ValueError("active_idx must be int32")
        na = active_idx.numel()
        if acc is None:
            acc = torch.empty((3, na), dtype=self.dtype, device=active_idx.device)
        if pot is None and (want_pot or (want_pot is None and self.params.want_potential)):
            pot = torch.empty(na, dtype=self.dtype, device=active_idx.device)
        self._rc(lib().tpm_pm_long_range(self.h, na, _ptr(active_idx), _ptr(acc), _ptr(pot)))
        return acc, pot

    def accel_norm(self, active_idx, acc_a, acc_b=None, out=None):
        """|acc_a + acc_b| into a float64 array in build order (for 'rel')."""
        if out is None:
            out = torch.zeros(self.n, dtype=torch.float64, device=active_idx.device)
        self._rc(lib().tpm_accel_norm(self.h, active_idx.numel(), _ptr(active_idx),
                                      _ptr(acc_a), _ptr(acc_b), _ptr(out)))
        return out

    # -- measurement -----------------------------------------------------------
    TIMERS = {"walk": 0, "build": 1, "pm_solve": 2, "pm_interp": 3, "sort": 4, "walk_rel": 5,
              "keys": 6, "gather": 7, "topology": 8, "moments": 9, "deposit": 10, "fft": 11}

    def timing(self, on: bool = True):
        self._rc(lib().tpm_timing_enable(self.h, int(on)))

    def timing_read(self, kind: str):
        ms = C.c_double()
        k = C.c_int64()
        self._rc(lib().tpm_timing_read(self.h, self.TIMERS[kind], C.byref(ms), C.byref(k)))
        return float(ms.value), int(k.value)

    def timing_durations(self, kind: str, cap: int = 1 << 16):
        """Milliseconds of each timed launch of one class (launch order)."""
        buf = (C.c_double * cap)()
        k = C.c_int64()
        self._rc(lib().tpm_timing_durations(self.h, self.TIMERS[kind], buf, cap, C.byref(k)))
        return [buf[i] for i in range(min(int(k.value), cap))]

    # -- checks and verification --------------------------------------------
    def check(self):
        rc = lib().tpm_check(self.h)
        if rc != TPM_OK:
            raise TreePMError(rc, lib().tpm_last_error(self.h).decode())

    def bytes_held(self) -> int:
        return int(lib().tpm_bytes_held(self.h))

    def tree_info(self):
        n = C.c_int64()
        E = C.c_int64()
        fr = (C.c_double * 4)()
        self._rc(lib().tpm_tree_info(self.h, C.byref(n), C.byref(E), fr))
        return int(n.value), int(E.value), list(fr)

    def export_tree(self):
        import numpy as np
        n, E, fr = self.tree_info()
        out = dict(level=np.empty(E, np.int32), first=np.empty(E, np.int64),
                   count=np.empty(E, np.int64), skip=np.empty(E, np.int64),
                   pidx=np.empty(E, np.int64), mass=np.empty(E), com=np.empty(3 * E),
                   cen=np.empty(3 * E), key=np.empty(n, np.uint64), perm=np.empty(n, np.int64))
        args = [C.c_void_p(out[k].ctypes.data) for k in
                ("level", "first", "count", "skip", "pidx", "mass", "com", "cen", "key", "perm")]
        self._rc(lib().tpm_export_tree(self.h, *args))
        out["com"] = out["com"].reshape(3, E)
        out["cen"] = out["cen"].reshape(3, E)
        out["frame"] = np.array(fr)
        return out

    def export_mesh(self):
        """Deposited density (mass per cell when isolated) and potential of
        the last PM solve, as host arrays of shape (M, M, M)."""
        import numpy as np
        M = self.params.pm_grid * (1 if self.params.periodic else 2)
        rho = np.empty(M ** 3)
        phi = np.empty(M ** 3)
        self._rc(lib().tpm_export_mesh(self.h, C.c_void_p(rho.ctypes.data),
                                       C.c_void_p(phi.ctypes.data)))
        return rho.reshape(M, M, M), phi.reshape(M, M, M)


class ResidentServer:
    """The device-resident request loop of one precision: a persistent kernel
    that takes tree-force requests while it runs (tpm_server_*)."""

    def __init__(self, precision="fp32", idle_ms=5.0):
        h = C.c_void_p()
        rc = lib().tpm_server_create(PRECISION[precision], float(idle_ms), C.byref(h))
        if rc != TPM_OK:
            raise TreePMError(rc, "tpm_server_create failed")
        self.h = h
        self.precision = precision
        self._keep = {}

    def _rc(self, rc):
        if rc < 0:
            raise TreePMError(rc, lib().tpm_server_last_error(self.h).decode())
        return rc

    def submit(self, ctx: Context, active_idx, opening="bh", a_old_norm=None, acc=None,
               n_interactions=None):
        """Returns (ticket, acc); acc is valid once poll(ticket) is true."""
        na = active_idx.numel()
        if acc is None:
            acc = torch.empty((3, na), dtype=ctx.dtype, device=active_idx.device)
        t = C.c_uint64()
        rc = lib().tpm_server_submit(self.h, ctx.h, OPEN[opening], na, _ptr(active_idx),
                                     _ptr(a_old_norm), _ptr(acc), _ptr(n_interactions),
                                     C.byref(t))
        if rc != TPM_OK:
            msg = lib().tpm_server_last_error(self.h).decode() or lib().tpm_last_error(
                ctx.h).decode()
            raise TreePMError(rc, msg)
        self._keep[t.value] = (active_idx, a_old_norm, acc, n_interactions)
        return t.value, acc

    def submit_step(self, ctx: Context, active_idx, acc=None, acc_pm=None, n_interactions=None):
        """The first force computation (BH, mesh, |a|, relative) as one request.
        Returns (ticket, acc, acc_pm); acc_pm is None without a mesh."""
        na = active_idx.numel()
        dev = active_idx.device
        if acc is None:
            acc = torch.empty((3, na), dtype=ctx.dtype, device=dev)
        if acc_pm is None and ctx.params.pm_grid > 0:
            acc_pm = torch.empty((3, na), dtype=ctx.dtype, device=dev)
        t = C.c_uint64()
        rc = lib().tpm_server_submit_step(self.h, ctx.h, na, _ptr(active_idx), _ptr(acc),
                                          _ptr(acc_pm), _ptr(n_interactions), C.byref(t))
        if rc != TPM_OK:
            msg = lib().tpm_server_last_error(self.h).decode() or lib().tpm_last_error(
                ctx.h).decode()
            raise TreePMError(rc, msg)
        self._keep[t.value] = (active_idx, acc, acc_pm, n_interactions)
        return t.value, acc, acc_pm

    def poll(self, ticket) -> bool:
        done = self._rc(lib().tpm_server_poll(self.h, ticket)) == 1
        if done:
            self._keep.pop(ticket, None)
        return done

    def wait(self, ticket, timeout_s=120.0):
        """Polls until the request finished; raises after timeout_s."""
        import time
        t_end = time.perf_counter() + timeout_s
        while not self.poll(ticket):
            if time.perf_counter() > t_end:
                raise TreePMError(TPM_ESTATE, f"request {ticket} not finished in {timeout_s} s")
            time.sleep(0)

    def info(self):
        a, b = C.c_int64(), C.c_int64()
        self._rc(lib().tpm_server_info(self.h, C.byref(a), C.byref(b)))
        return {"launches": int(a.value), "in_flight": int(b.value)}

    def close(self):
        if getattr(self, "h", None):
            lib().tpm_server_destroy(self.h)
            self.h = None
            self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Continuous batching of tree-force requests over many contexts."""

    def __init__(self, stream=None):
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        rc = lib().tpm_batch_create(_stream_handle(self.stream), C.byref(h))
        if rc != TPM_OK:
            raise TreePMError(rc, "tpm_batch_create failed")
        self.h = h
        self._keep = []

    def _rc(self, rc):
        if rc != TPM_OK:
            raise TreePMError(rc, lib().tpm_batch_last_error(self.h).decode())

    def add(self, ctx: Context, active_idx, opening="bh", a_old_norm=None, acc=None,
            n_interactions=None):
        na = active_idx.numel()
        if acc is None:
            acc = torch.empty((3, na), dtype=ctx.dtype, device=active_idx.device)
        self._rc(lib().tpm_batch_add(self.h, ctx.h, OPEN[opening], na, _ptr(active_idx),
                                     _ptr(a_old_norm), _ptr(acc), _ptr(n_interactions)))
        self._keep.append((active_idx, a_old_norm, acc, n_interactions))
        return acc

    def launch(self):
        self._rc(lib().tpm_batch_launch(self.h))
        self._keep = []

    def close(self):
        if getattr(self, "h", None):
            lib().tpm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
