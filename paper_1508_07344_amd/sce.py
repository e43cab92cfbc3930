"""ctypes binding of ``include/sce.h``: same names as the C ABI, argument
marshalling only.

Host arrays are numpy float64; device arrays are torch tensors on the GPU
(passed with ``on_device=1``).  Status codes other than SCE_OK raise
``SceError`` carrying the library's message.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsce.so")
_HEADER = os.path.join(os.path.dirname(_HERE), "include", "sce.h")

SCE_OK, SCE_EINVAL, SCE_ENOMEM, SCE_EDEVICE, SCE_ESTATE, SCE_ENOTSUP, SCE_EUNSTABLE = 0, -1, -2, -3, -4, -5, -6
PREC = {"fp64": 0, "fp32": 1, "split_f16": 2}
SCHEME = {"kdk": 0, "dkd": 1}
SHAPE = {"delta": 0, "gaussian": 1, "tent": 2}
FIELD = {"delta": 0, "tent": 1}

_lib = None


def library_path() -> str:
    return _LIB_PATH


class _Diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("time", ctypes.c_double), ("kinetic", ctypes.c_double),
                ("field", ctypes.c_double), ("field_self", ctypes.c_double),
                ("interaction", ctypes.c_double), ("total", ctypes.c_double),
                ("momentum", ctypes.c_double * 3), ("momentum_abs_sum", ctypes.c_double),
                ("rho_abs_max", ctypes.c_double)]


class _ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("precision", ctypes.c_int32),
                ("max_active", ctypes.c_int32), ("no_graph", ctypes.c_int32),
                ("hip_stream", ctypes.c_void_p)]


class _Request(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double), ("a", ctypes.c_double), ("eps0", ctypes.c_double),
                ("dt", ctypes.c_double), ("n_max", ctypes.c_int32), ("shape_kind", ctypes.c_int32),
                ("N", ctypes.c_int64), ("n_steps", ctypes.c_int64),
                ("x", ctypes.c_void_p), ("v", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("m", ctypes.c_void_p), ("dim", ctypes.c_int32)]


class _ServerReport(ctypes.Structure):
    _fields_ = [("ticks", ctypes.c_int64), ("request_steps", ctypes.c_int64),
                ("requests_done", ctypes.c_int64), ("active", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("busy_s", ctypes.c_double), ("pairs", ctypes.c_double),
                ("p50_step_s", ctypes.c_double), ("p99_step_s", ctypes.c_double),
                ("max_step_s", ctypes.c_double), ("p50_wait_s", ctypes.c_double),
                ("p99_wait_s", ctypes.c_double), ("hbm_used_bytes", ctypes.c_double),
                ("hbm_peak_bytes", ctypes.c_double), ("gpu_p50_step_s", ctypes.c_double),
                ("gpu_p99_step_s", ctypes.c_double)]


@dataclasses.dataclass
class Diag:
    step: int
    time: float
    kinetic: float
    field: float
    field_self: float
    interaction: float
    total: float
    momentum: np.ndarray
    momentum_abs_sum: float
    rho_abs_max: float


class SceError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"sce status {status}: {msg}")
        self.status = status


def exported_symbols() -> list:
    """Function names declared in include/sce.h."""
    txt = open(_HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(sce_[a-z_0-9]+)\s*\(", txt, re.M)))


def load_library():
    """Load libsce.so.  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built; run paper_1508_07344_amd.build.build()")
    lib = ctypes.CDLL(_LIB_PATH)
    P, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "sce_create": ([f64, i32, i32, f64, ctypes.POINTER(P)], i32),
        "sce_create_2d": ([f64, i32, i32, f64, ctypes.POINTER(P)], i32),
        "sce_dimension": ([P, ctypes.POINTER(i32)], i32),
        "sce_create_tent": ([f64, i32, i32, ctypes.POINTER(P)], i32),
        "sce_field_shape": ([P, ctypes.POINTER(i32)], i32),
        "sce_set_options": ([P, f64, i32, i32, P], i32),
        "sce_set_particles": ([P, i64, P, P, P, P, i32], i32),
        "sce_get_particles": ([P, P, P, i32], i32),
        "sce_mode_count": ([P, ctypes.POINTER(i64)], i32),
        "sce_modes": ([P, P], i32),
        "sce_deposit": ([P, P, i32], i32),
        "sce_psi": ([P, P, i32], i32),
        "sce_force": ([P, P, i32], i32),
        "sce_force_noalloc": ([P, P, i32], i32),
        "sce_step": ([P, f64, i64], i32),
        "sce_set_step_graph": ([P, i32], i32),
        "sce_set_small_step": ([P, i64], i32),
        "sce_diagnostics": ([P, ctypes.POINTER(_Diag), P], i32),
        "sce_get_state": ([P, P, ctypes.POINTER(ctypes.c_size_t)], i32),
        "sce_set_state": ([P, P, ctypes.c_size_t], i32),
        "sce_sync": ([P], i32),
        "sce_timing_enable": ([P, i32], i32),
        "sce_timing_read": ([P, ctypes.POINTER(f64), ctypes.POINTER(i64), ctypes.POINTER(f64),
                             ctypes.POINTER(i64)], i32),
        "sce_destroy": ([P], None),
        "sce_status_string": ([i32], ctypes.c_char_p),
        "sce_last_error": ([P], ctypes.c_char_p),
        "sce_server_create": ([ctypes.POINTER(_ServerOpts), ctypes.POINTER(P)], i32),
        "sce_server_submit": ([P, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_uint64)], i32),
        "sce_server_tick": ([P, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "sce_server_poll": ([P, P, i32, ctypes.POINTER(i32)], i32),
        "sce_server_result": ([P, ctypes.c_uint64, P, P, P, ctypes.POINTER(_Diag),
                               ctypes.POINTER(_Diag)], i32),
        "sce_server_stats": ([P, ctypes.POINTER(_ServerReport)], i32),
        "sce_server_last_error": ([P], ctypes.c_char_p),
        "sce_server_destroy": ([P], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _host(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _torch_sync_if_device(*arrays):
    """Device tensors are produced and consumed on torch's stream; the library
    works on its own stream, so order the two around each device-pointer call."""
    if any(not isinstance(a, np.ndarray) and a is not None for a in arrays):
        import torch
        torch.cuda.current_stream().synchronize()


def _ptr(a):
    """(pointer, on_device) for a numpy array or a torch tensor."""
    if isinstance(a, np.ndarray):
        if not a.flags.c_contiguous or a.dtype != np.float64:
            raise ValueError("host arrays must be C-contiguous float64")
        return _host(a), 0
    import torch
    if isinstance(a, torch.Tensor):
        if a.dtype != torch.float64 or not a.is_contiguous():
            raise ValueError("tensors must be contiguous float64")
        return ctypes.c_void_p(a.data_ptr()), 1 if a.is_cuda else 0
    raise TypeError(type(a))


class Context:
    """One simulation context (``sce_ctx``); ``dim`` = 2 makes a two-dimensional
    one (``sce_create_2d``), whose particle vectors are [2, N]; ``field`` =
    "tent" makes a tent-field context (``sce_create_tent``: point particles,
    ``shape`` and ``width`` must be "delta" and 0)."""

    def __init__(self, L: float, n_max: int, shape: str = "gaussian", width: float = 0.0,
                 dim: int = 3, field: str = "delta"):
        self._lib = load_library()
        h = ctypes.c_void_p()
        if dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        if field == "tent":
            if shape != "delta" or width != 0.0:
                raise ValueError("tent-field contexts take point particles (shape 'delta', width 0)")
            st = self._lib.sce_create_tent(float(L), int(n_max), int(dim), ctypes.byref(h))
        elif field == "delta":
            create = self._lib.sce_create_2d if dim == 2 else self._lib.sce_create
            st = create(float(L), int(n_max), SHAPE[shape], float(width), ctypes.byref(h))
        else:
            raise ValueError("field must be 'delta' or 'tent'")
        if st != SCE_OK:
            raise SceError(st, "sce_create: " + self._lib.sce_status_string(st).decode())
        self._h = h
        self.L, self.n_max, self.N, self.dim, self.field = float(L), int(n_max), 0, int(dim), field

    def _chk(self, st: int, what: str):
        if st != SCE_OK:
            msg = self._lib.sce_last_error(self._h).decode()
            raise SceError(st, f"{what}: {msg}")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sce_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------ C ABI mirrors
    def sce_set_options(self, eps0: float = 1.0, precision: str = "fp64", scheme: str = "kdk",
                        stream=None):
        s = ctypes.c_void_p(int(stream)) if stream else None
        self._chk(self._lib.sce_set_options(self._h, float(eps0), PREC[precision], SCHEME[scheme], s),
                  "sce_set_options")

    def sce_dimension(self) -> int:
        d = ctypes.c_int32()
        self._chk(self._lib.sce_dimension(self._h, ctypes.byref(d)), "sce_dimension")
        return int(d.value)

    def sce_field_shape(self) -> str:
        f = ctypes.c_int32()
        self._chk(self._lib.sce_field_shape(self._h, ctypes.byref(f)), "sce_field_shape")
        return {v: k for k, v in FIELD.items()}[int(f.value)]

    def sce_set_particles(self, x, v, q, m):
        """x, v: [dim, N]; q, m: [N]; numpy (host) or torch CUDA tensors (device)."""
        N = int(q.shape[0])
        px, dx = _ptr(x)
        pv, dv = _ptr(v)
        pq, dq = _ptr(q)
        pm, dm = _ptr(m)
        if len({dx, dv, dq, dm}) != 1:
            raise ValueError("all particle arrays must be on the same side (host or device)")
        _torch_sync_if_device(x, v, q, m)
        self._chk(self._lib.sce_set_particles(self._h, N, px, pv, pq, pm, dx), "sce_set_particles")
        if dx:
            self.sce_sync()
        self.N = N

    def sce_get_particles(self, x=None, v=None):
        if x is None and v is None:
            x = np.zeros((self.dim, self.N))
            v = np.zeros((self.dim, self.N))
        px, dx = _ptr(x) if x is not None else (None, 0)
        pv, dv = _ptr(v) if v is not None else (None, dx)
        _torch_sync_if_device(x, v)
        self._chk(self._lib.sce_get_particles(self._h, px, pv, dx if x is not None else dv),
                  "sce_get_particles")
        self.sce_sync()
        return x, v

    def sce_mode_count(self) -> int:
        n = ctypes.c_int64()
        self._chk(self._lib.sce_mode_count(self._h, ctypes.byref(n)), "sce_mode_count")
        return int(n.value)

    def sce_modes(self) -> np.ndarray:
        out = np.zeros((self.sce_mode_count(), self.dim), dtype=np.int32)
        self._chk(self._lib.sce_modes(self._h, _host(out)), "sce_modes")
        return out

    def sce_deposit(self, out=None):
        """Returns complex128 rho [|H|] (host) unless ``out`` (a device float64
        tensor of 2|H|) is given."""
        if out is None:
            buf = np.zeros(2 * self.sce_mode_count())
            self._chk(self._lib.sce_deposit(self._h, _host(buf), 0), "sce_deposit")
            return buf[0::2] + 1j * buf[1::2]
        p, d = _ptr(out)
        _torch_sync_if_device(out)
        self._chk(self._lib.sce_deposit(self._h, p, d), "sce_deposit")
        self.sce_sync()
        return out

    def sce_psi(self):
        buf = np.zeros(2 * self.sce_mode_count())
        self._chk(self._lib.sce_psi(self._h, _host(buf), 0), "sce_psi")
        return buf[0::2] + 1j * buf[1::2]

    def sce_force(self, out=None):
        """Returns F [dim, N] float64 (host) unless ``out`` is given."""
        if out is None:
            buf = np.zeros((self.dim, self.N))
            self._chk(self._lib.sce_force(self._h, _host(buf), 0), "sce_force")
            return buf
        p, d = _ptr(out)
        _torch_sync_if_device(out)
        self._chk(self._lib.sce_force(self._h, p, d), "sce_force")
        self.sce_sync()
        return out

    def sce_force_noalloc(self, out=None):
        """``sce_force`` with the pass's scratch in the library's static
        per-GPU array (no device allocation)."""
        if out is None:
            buf = np.zeros((self.dim, self.N))
            self._chk(self._lib.sce_force_noalloc(self._h, _host(buf), 0), "sce_force_noalloc")
            return buf
        p, d = _ptr(out)
        _torch_sync_if_device(out)
        self._chk(self._lib.sce_force_noalloc(self._h, p, d), "sce_force_noalloc")
        self.sce_sync()
        return out

    def sce_force_device_only(self):
        self._chk(self._lib.sce_force(self._h, None, 1), "sce_force")

    def sce_step(self, dt: float, n_steps: int = 1):
        self._chk(self._lib.sce_step(self._h, float(dt), int(n_steps)), "sce_step")

    def sce_set_step_graph(self, steps_per_graph: int):
        self._chk(self._lib.sce_set_step_graph(self._h, int(steps_per_graph)), "sce_set_step_graph")

    def sce_set_small_step(self, max_pairs: int):
        self._chk(self._lib.sce_set_small_step(self._h, int(max_pairs)), "sce_set_small_step")

    def sce_diagnostics(self, rho_abs: bool = False, allow_unstable: bool = False):
        d = _Diag()
        ra = np.zeros(self.sce_mode_count()) if rho_abs else None
        st = self._lib.sce_diagnostics(self._h, ctypes.byref(d), _host(ra) if ra is not None else None)
        if not (allow_unstable and st == SCE_EUNSTABLE):
            self._chk(st, "sce_diagnostics")
        out = Diag(d.step, d.time, d.kinetic, d.field, d.field_self, d.interaction, d.total,
                   np.array(list(d.momentum)), d.momentum_abs_sum, d.rho_abs_max)
        return (out, ra, st) if rho_abs else (out, st)

    def sce_get_state(self) -> bytes:
        n = ctypes.c_size_t(0)
        self._chk(self._lib.sce_get_state(self._h, None, ctypes.byref(n)), "sce_get_state")
        buf = ctypes.create_string_buffer(n.value)
        self._chk(self._lib.sce_get_state(self._h, buf, ctypes.byref(n)), "sce_get_state")
        return buf.raw

    def sce_set_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._chk(self._lib.sce_set_state(self._h, buf, len(blob)), "sce_set_state")
        self.N = int(np.frombuffer(blob[8:16], dtype=np.int64)[0])  # header: magic, N, ...

    def sce_sync(self):
        self._chk(self._lib.sce_sync(self._h), "sce_sync")

    def sce_timing_enable(self, enable: bool = True):
        self._chk(self._lib.sce_timing_enable(self._h, 1 if enable else 0), "sce_timing_enable")

    def sce_timing_read(self):
        a, b = ctypes.c_double(), ctypes.c_double()
        na, nb = ctypes.c_int64(), ctypes.c_int64()
        self._chk(self._lib.sce_timing_read(self._h, ctypes.byref(a), ctypes.byref(na), ctypes.byref(b),
                                            ctypes.byref(nb)), "sce_timing_read")
        return {"deposit_ms": a.value, "deposit_launches": na.value,
                "force_ms": b.value, "force_launches": nb.value}

    # ------------------------------------------------------------ conveniences
    @classmethod
    def from_particles(cls, p, precision: str = "fp64", scheme: str = "kdk", device: bool = False):
        """Context for a ``workloads.Particles`` record, particles already set."""
        c = cls(p.L, p.n_max, p.shape, p.a, dim=getattr(p, "dim", 3), field=getattr(p, "field", "delta"))
        c.sce_set_options(p.eps0, precision, scheme)
        if device:
            import torch
            t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
            c.sce_set_particles(t(p.positions()), t(p.velocities()), t(p.q), t(p.m))
            c.sce_sync()
        else:
            c.sce_set_particles(p.positions(), p.velocities(), np.ascontiguousarray(p.q),
                                np.ascontiguousarray(p.m))
        return c


def _diag(d: _Diag) -> Diag:
    return Diag(d.step, d.time, d.kinetic, d.field, d.field_self, d.interaction, d.total,
                np.array(list(d.momentum)), d.momentum_abs_sum, d.rho_abs_max)


class Server:
    """Batched server of independent simulations (``sce_server``)."""

    def __init__(self, hbm_budget_bytes: int = 0, precision: str = "fp32", max_active: int = 0,
                 graph: bool = True):
        lib = load_library()
        self._lib = lib
        o = _ServerOpts(hbm_budget_bytes, PREC[precision], max_active, 0 if graph else 1, None)
        h = ctypes.c_void_p()
        st = lib.sce_server_create(ctypes.byref(o), ctypes.byref(h))
        if st != SCE_OK:
            raise SceError(st, lib.sce_status_string(st).decode())
        self._h = h
        self._sizes = {}

    def _chk(self, st: int, what: str):
        if st != SCE_OK:
            msg = self._lib.sce_server_last_error(self._h).decode()
            raise SceError(st, f"{what}: {msg}")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sce_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def sce_server_submit(self, p, n_steps: int | None = None) -> int:
        """Queue a ``workloads.Particles`` record (its dt, n_steps unless given)."""
        x = np.ascontiguousarray(p.positions(), dtype=np.float64)
        v = np.ascontiguousarray(p.velocities(), dtype=np.float64)
        q = np.ascontiguousarray(p.q, dtype=np.float64)
        m = np.ascontiguousarray(p.m, dtype=np.float64)
        steps = p.n_steps if n_steps is None else n_steps
        dim = getattr(p, "dim", 3)
        r = _Request(p.L, p.a, p.eps0, p.dt, p.n_max, SHAPE[p.shape], p.N, steps,
                     _host(x), _host(v), _host(q), _host(m), dim)
        rid = ctypes.c_uint64()
        self._chk(self._lib.sce_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)), "submit")
        self._sizes[rid.value] = (p.N, dim)
        return rid.value

    def sce_server_tick(self):
        a, q = ctypes.c_int32(), ctypes.c_int32()
        self._chk(self._lib.sce_server_tick(self._h, ctypes.byref(a), ctypes.byref(q)), "tick")
        return a.value, q.value

    def sce_server_poll(self, max_ids: int = 4096) -> list:
        ids = (ctypes.c_uint64 * max(max_ids, 1))()
        n = ctypes.c_int32()
        self._chk(self._lib.sce_server_poll(self._h, ids, max_ids, ctypes.byref(n)), "poll")
        return [ids[i] for i in range(n.value)]

    def sce_server_result(self, rid: int):
        """(x, v, F, first Diag, last Diag) of a finished request."""
        if rid not in self._sizes:
            raise SceError(SCE_EINVAL, f"result: unknown or already fetched request {rid}")
        N, dim = self._sizes[rid]
        x, v, F = (np.empty((dim, N)) for _ in range(3))
        d0, d1 = _Diag(), _Diag()
        self._chk(self._lib.sce_server_result(self._h, rid, _host(x), _host(v), _host(F),
                                              ctypes.byref(d0), ctypes.byref(d1)), "result")
        del self._sizes[rid]
        return x, v, F, _diag(d0), _diag(d1)

    def sce_server_stats(self) -> dict:
        r = _ServerReport()
        self._chk(self._lib.sce_server_stats(self._h, ctypes.byref(r)), "stats")
        return {name: getattr(r, name) for name, _ in r._fields_}
