"""CPU comparison baseline with the paper's own mode-sum optimisations
(Section 8): the half space of modes only, and D = 3 exponentials per particle
whose integer powers give every mode's phase (``cpu_paper.c``).

NOT A CHECKER.  The oracle (this package's ``__init__``, ``sce_oracle.c``) is
the definition the HIP library is checked against.  This module is timed by
the benchmark's CPU-baseline leg beside the oracle, as the faster of the two
CPU programs, and ``tests/test_cpu_paper.py`` pins it against the oracle.
Like the oracle, only the tests and the benchmark load it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cpu_paper.c")
_LIB = os.path.join(_HERE, "libsce_cpu_paper.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile with gcc: -O3, AVX2 and FMA (x86-64-v3 hosts), OpenMP."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-std=gnu11", "-mavx2", "-mfma", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
            lib.sce_cpu_paper_deposit.argtypes = [i64, P, P, P, P, f64, i32, P, P]
            lib.sce_cpu_paper_deposit.restype = i32
            lib.sce_cpu_paper_force.argtypes = [i64, P, P, P, P, f64, i32, P, P]
            lib.sce_cpu_paper_force.restype = i32
            lib.sce_cpu_paper_threads.argtypes = []
            lib.sce_cpu_paper_threads.restype = i32
            lib.sce_cpu_paper_set_threads.argtypes = [i32]
            lib.sce_cpu_paper_set_threads.restype = None
            _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _coords(pos):
    pos = np.asarray(pos, dtype=np.float64)
    return [np.ascontiguousarray(pos[d]) for d in range(3)]


def threads() -> int:
    """OpenMP threads the loops use (OMP_NUM_THREADS, else every core)."""
    return int(_load().sce_cpu_paper_threads())


def set_threads(n: int) -> None:
    """OpenMP threads for the loops (the deposit's rounding depends on it)."""
    _load().sce_cpu_paper_set_threads(int(n))


def deposit(pos, q, L: float, n_max: int, S: np.ndarray) -> np.ndarray:
    """rho_n = S_n sum_j q_j exp(-i k_n . x_j) over the three-dimensional half
    space in canonical order; ``S`` holds the shape factor of each of those
    modes.  Returns complex128 [|H|]."""
    lib = _load()
    x, y, z = _coords(pos)
    q = np.ascontiguousarray(q, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    out = np.zeros(2 * len(S))
    if lib.sce_cpu_paper_deposit(len(q), _p(x), _p(y), _p(z), _p(q), float(L), int(n_max), _p(S), _p(out)):
        raise MemoryError("cpu_paper.deposit: work buffers")
    return out[0::2] + 1j * out[1::2]


def force(pos, q, L: float, n_max: int, psi_c: np.ndarray) -> np.ndarray:
    """F_j = 2 q_j sum_{n in H} k_n Im(psi_n exp(i k_n . x_j)), [3, N]."""
    lib = _load()
    x, y, z = _coords(pos)
    q = np.ascontiguousarray(q, dtype=np.float64)
    ps = np.empty(2 * len(psi_c))
    ps[0::2], ps[1::2] = np.real(psi_c), np.imag(psi_c)
    F = np.zeros(3 * len(q))
    if lib.sce_cpu_paper_force(len(q), _p(x), _p(y), _p(z), _p(q), float(L), int(n_max), _p(ps), _p(F)):
        raise MemoryError("cpu_paper.force: work buffers")
    return F.reshape(3, len(q))
