"""FP64 CPU oracle for the spectral canonical electrostatic method
(Webb, "A Spectral Canonical Electrostatic Algorithm", arXiv:1508.07344).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The HIP library and
its Python binding never import it, and it never imports them; the two share
only the seeded inputs of ``workloads``.

The mode sums live in ``sce_oracle.c`` (plain double loops, one cos/sin per
particle-mode pair).  This module adds the time steps, written as the paper's
update sequences:

* ``step_dkd`` -- the velocity form of the discrete Euler-Lagrange equations
  (Section 4): drift h/2, deposit + Poisson solve at the half step, kick h,
  drift h/2.
* ``step_kdk`` -- the kick-drift-kick arrangement of the same leapfrog: half
  kick, drift h, deposit + solve + force at the new positions, half kick.  The
  force at the end of a step is reused at the start of the next.

Positions are wrapped into [0, L) after every drift (periodic box, Section 8):
wrap(x) = x - L floor(x / L), and a result equal to L becomes 0.

Two dimensions: the paper's own test problems (Sections 6 and 7) are
two-dimensional, with line charges in the periodic square [0, L)^2 of area
A = L^2.  Every function below takes 2-component arrays as well: positions and
velocities [2, N], modes [n, 2] (``half_modes(n_max, dim=2)``), and the solve
and energies divide by A instead of V.  The 2-D sums are their own plain loops
in ``sce_oracle.c``.

Energies (Section 3's discrete Lagrangian, delta field shape):
kinetic K = 1/2 sum m |v|^2, field W (see ``field_energy``), total E = K + W,
interaction sum_j q_j Phi_j (= 2 W), and the constant self-energy of the
retained modes W_self = (sum q^2 / (eps0 V)) sum_H S^2 / |k|^2.

``cpu_paper`` is not part of the oracle: it is a faster CPU program (the
paper's per-axis powers, Section 8) that the benchmark times beside it, pinned
against the oracle by ``tests/test_cpu_paper.py``.

Parity: all functions here are pinned by ``tests/test_oracle_pins.py`` (FFT
special case, Ewald alpha-independence, rock-salt Madelung constant, gradient,
adjointness, conservation laws, reversibility, h^2 energy error, cold-plasma
dispersion), the two-dimensional ones also by ``tests/test_oracle_pins_2d.py``,
and ``self_energy`` by ``tests/test_oracle_pins_self.py`` (a lone particle's
field energy; the grid mean of a pair's).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sce_oracle.c")
_LIB = os.path.join(_HERE, "libsce_oracle.so")
_lock = threading.Lock()
_lib = None

SHAPES = {"delta": 0, "gaussian": 1, "tent": 2}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, strict IEEE: no fast-math),
    and the CPU comparison baseline of ``cpu_paper`` beside it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    from . import cpu_paper
    cpu_paper.build(force)
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
            lib.sce_oracle_half_modes.argtypes = [i32, P]
            lib.sce_oracle_half_modes.restype = i64
            lib.sce_oracle_cube_modes.argtypes = [i32, P]
            lib.sce_oracle_cube_modes.restype = i64
            lib.sce_oracle_shape.argtypes = [i32, f64, f64, f64, f64]
            lib.sce_oracle_shape.restype = f64
            lib.sce_oracle_deposit.argtypes = [i64, P, P, P, P, f64, i64, P, i32, f64, P]
            lib.sce_oracle_deposit.restype = None
            lib.sce_oracle_psi.argtypes = [i64, P, P, f64, f64, i32, f64, P]
            lib.sce_oracle_psi.restype = None
            lib.sce_oracle_force.argtypes = [i64, P, P, P, P, f64, i64, P, P, P]
            lib.sce_oracle_force.restype = None
            lib.sce_oracle_potential.argtypes = [i64, P, P, P, f64, i64, P, P, P]
            lib.sce_oracle_potential.restype = None
            lib.sce_oracle_field_energy.argtypes = [i64, P, P, f64, f64]
            lib.sce_oracle_field_energy.restype = f64
            lib.sce_oracle_shape_2d.argtypes = [i32, f64, f64, f64]
            lib.sce_oracle_shape_2d.restype = f64
            lib.sce_oracle_half_modes_2d.argtypes = [i32, P]
            lib.sce_oracle_half_modes_2d.restype = i64
            lib.sce_oracle_square_modes.argtypes = [i32, P]
            lib.sce_oracle_square_modes.restype = i64
            lib.sce_oracle_deposit_2d.argtypes = [i64, P, P, P, f64, i64, P, i32, f64, P]
            lib.sce_oracle_deposit_2d.restype = None
            lib.sce_oracle_psi_2d.argtypes = [i64, P, P, f64, f64, i32, f64, P]
            lib.sce_oracle_psi_2d.restype = None
            lib.sce_oracle_force_2d.argtypes = [i64, P, P, P, f64, i64, P, P, P]
            lib.sce_oracle_force_2d.restype = None
            lib.sce_oracle_potential_2d.argtypes = [i64, P, P, f64, i64, P, P, P]
            lib.sce_oracle_potential_2d.restype = None
            lib.sce_oracle_field_energy_2d.argtypes = [i64, P, P, f64, f64]
            lib.sce_oracle_field_energy_2d.restype = f64
            lib.sce_oracle_threads.argtypes = []
            lib.sce_oracle_threads.restype = i32
            lib.sce_oracle_set_threads.argtypes = [i32]
            lib.sce_oracle_set_threads.restype = None
            _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(_load().sce_oracle_threads())


def set_threads(n: int) -> None:
    """Threads for the oracle's OpenMP loops (results do not depend on it)."""
    _load().sce_oracle_set_threads(int(n))


def half_modes(n_max: int, dim: int = 3) -> np.ndarray:
    """Half-space modes in canonical order, int32 array [|H|, dim] (dim 3: H;
    dim 2: the half plane H2)."""
    lib = _load()
    fn = lib.sce_oracle_half_modes if dim == 3 else lib.sce_oracle_half_modes_2d
    n = fn(int(n_max), None)
    out = np.zeros((n, dim), dtype=np.int32)
    fn(int(n_max), _p(out))
    return out


def cube_modes(n_max: int, dim: int = 3) -> np.ndarray:
    """Every mode with max|n_i| <= n_max except n = 0, int32 [M^dim - 1, dim]."""
    lib = _load()
    fn = lib.sce_oracle_cube_modes if dim == 3 else lib.sce_oracle_square_modes
    n = fn(int(n_max), None)
    out = np.zeros((n, dim), dtype=np.int32)
    fn(int(n_max), _p(out))
    return out


def shape(kind: str, a: float, k: np.ndarray) -> np.ndarray:
    """S(k) for an array of wave vectors k [..., 3] or [..., 2]."""
    lib = _load()
    k = np.asarray(k, dtype=np.float64)
    if k.shape[-1] == 2:
        k = k.reshape(-1, 2)
        return np.array([lib.sce_oracle_shape_2d(SHAPES[kind], a, *kk) for kk in k])
    k = k.reshape(-1, 3)
    return np.array([lib.sce_oracle_shape(SHAPES[kind], a, *kk) for kk in k])


def wave_vectors(modes: np.ndarray, L: float) -> np.ndarray:
    """k = 2 pi n / L, float64 [n_modes, dim]."""
    return (2.0 * np.pi / L) * modes.astype(np.float64)


def wrap(x: np.ndarray, L: float) -> np.ndarray:
    """Periodic wrap into [0, L): x - L floor(x / L); a result equal to L becomes 0."""
    w = x - L * np.floor(x / L)
    return np.where(w >= L, 0.0, w)


def deposit(pos, q, L: float, modes: np.ndarray, kind: str = "gaussian", a: float = 0.0) -> np.ndarray:
    """rho_n = S(k_n) sum_j q_j exp(-i k_n . x_j) for each row of ``modes``.
    ``pos`` is [3, N] (or [2, N] with 2-component modes).  Returns complex128 [n_modes]."""
    lib = _load()
    pos = _f64(pos)
    q = _f64(q)
    modes = np.ascontiguousarray(modes, dtype=np.int32)
    rho = np.zeros(2 * len(modes))
    if modes.shape[1] == 2:
        x, y = (np.ascontiguousarray(pos[d]) for d in range(2))
        lib.sce_oracle_deposit_2d(len(q), _p(x), _p(y), _p(q), float(L), len(modes), _p(modes),
                                  SHAPES[kind], float(a), _p(rho))
        return rho[0::2] + 1j * rho[1::2]
    x, y, z = (np.ascontiguousarray(pos[d]) for d in range(3))
    lib.sce_oracle_deposit(len(q), _p(x), _p(y), _p(z), _p(q), float(L), len(modes), _p(modes),
                           SHAPES[kind], float(a), _p(rho))
    return rho[0::2] + 1j * rho[1::2]


def psi(rho: np.ndarray, L: float, modes: np.ndarray, eps0: float = 1.0,
        kind: str = "gaussian", a: float = 0.0) -> np.ndarray:
    """psi_n = S(k_n) rho_n / (eps0 |k_n|^2 V) (V = L^3; A = L^2 in two dimensions)."""
    lib = _load()
    modes = np.ascontiguousarray(modes, dtype=np.int32)
    r = np.empty(2 * len(modes))
    r[0::2], r[1::2] = rho.real, rho.imag
    out = np.zeros_like(r)
    fn = lib.sce_oracle_psi_2d if modes.shape[1] == 2 else lib.sce_oracle_psi
    fn(len(modes), _p(modes), _p(r), float(L), float(eps0), SHAPES[kind], float(a), _p(out))
    return out[0::2] + 1j * out[1::2]


def force_from_psi(pos, q, L: float, modes: np.ndarray, psi_c: np.ndarray) -> np.ndarray:
    """F_j = 2 q_j sum_{n in H} k_n Im(psi_n exp(i k_n . x_j)), returns [dim, N]."""
    lib = _load()
    pos = _f64(pos)
    q = _f64(q)
    modes = np.ascontiguousarray(modes, dtype=np.int32)
    ps = np.empty(2 * len(modes))
    ps[0::2], ps[1::2] = psi_c.real, psi_c.imag
    if modes.shape[1] == 2:
        x, y = (np.ascontiguousarray(pos[d]) for d in range(2))
        F = np.zeros(2 * len(q))
        lib.sce_oracle_force_2d(len(q), _p(x), _p(y), _p(q), float(L), len(modes), _p(modes),
                                _p(ps), _p(F))
        return F.reshape(2, len(q))
    x, y, z = (np.ascontiguousarray(pos[d]) for d in range(3))
    F = np.zeros(3 * len(q))
    lib.sce_oracle_force(len(q), _p(x), _p(y), _p(z), _p(q), float(L), len(modes), _p(modes),
                         _p(ps), _p(F))
    return F.reshape(3, len(q))


def potential_from_psi(pos, L: float, modes: np.ndarray, psi_c: np.ndarray) -> np.ndarray:
    """Phi_j = 2 sum_{n in H} Re(psi_n exp(i k_n . x_j))."""
    lib = _load()
    pos = _f64(pos)
    modes = np.ascontiguousarray(modes, dtype=np.int32)
    ps = np.empty(2 * len(modes))
    ps[0::2], ps[1::2] = psi_c.real, psi_c.imag
    out = np.zeros(pos.shape[1])
    if modes.shape[1] == 2:
        x, y = (np.ascontiguousarray(pos[d]) for d in range(2))
        lib.sce_oracle_potential_2d(pos.shape[1], _p(x), _p(y), float(L), len(modes), _p(modes),
                                    _p(ps), _p(out))
        return out
    x, y, z = (np.ascontiguousarray(pos[d]) for d in range(3))
    lib.sce_oracle_potential(pos.shape[1], _p(x), _p(y), _p(z), float(L), len(modes), _p(modes),
                             _p(ps), _p(out))
    return out


def field_energy(rho: np.ndarray, L: float, modes: np.ndarray, eps0: float = 1.0) -> float:
    """W = (1/(eps0 V)) sum_{n in H} |rho_n|^2 / |k_n|^2 (half-space sum; A in 2-D)."""
    lib = _load()
    modes = np.ascontiguousarray(modes, dtype=np.int32)
    r = np.empty(2 * len(modes))
    r[0::2], r[1::2] = rho.real, rho.imag
    fn = lib.sce_oracle_field_energy_2d if modes.shape[1] == 2 else lib.sce_oracle_field_energy
    return float(fn(len(modes), _p(modes), _p(r), float(L), float(eps0)))


def self_energy(q, L: float, modes: np.ndarray, eps0: float = 1.0, kind: str = "gaussian",
                a: float = 0.0) -> float:
    """Constant self-energy of the retained modes: (sum q^2/(eps0 V)) sum_H S^2/|k|^2
    (V = L^dim)."""
    k = wave_vectors(modes, L)
    s = shape(kind, a, k)
    vol = L ** modes.shape[1]
    return float(np.sum(np.asarray(q) ** 2) / (eps0 * vol) * np.sum(s * s / np.sum(k * k, axis=1)))


@dataclasses.dataclass
class Fields:
    rho: np.ndarray      # complex [|H|]
    psi: np.ndarray      # complex [|H|]
    F: np.ndarray        # [dim, N]
    W: float


def fields(pos, q, L: float, n_max: int, kind: str = "gaussian", a: float = 0.0,
           eps0: float = 1.0, modes: np.ndarray | None = None) -> Fields:
    """Deposit, solve and force at positions ``pos`` [dim, N] (one pass of the hot path)."""
    if modes is None:
        modes = half_modes(n_max, dim=np.asarray(pos).shape[0])
    rho = deposit(pos, q, L, modes, kind, a)
    ps = psi(rho, L, modes, eps0, kind, a)
    F = force_from_psi(pos, q, L, modes, ps)
    return Fields(rho, ps, F, field_energy(rho, L, modes, eps0))


@dataclasses.dataclass
class State:
    """Particle state advanced by the oracle's time steps."""
    pos: np.ndarray   # [dim, N]
    vel: np.ndarray   # [dim, N]
    q: np.ndarray
    m: np.ndarray
    L: float
    n_max: int
    kind: str = "gaussian"
    a: float = 0.0
    eps0: float = 1.0
    F: np.ndarray | None = None       # force at pos (kick-drift-kick reuses it)
    W: float | None = None            # field energy at pos
    rho: np.ndarray | None = None     # rho at pos
    step: int = 0
    modes: np.ndarray | None = None

    @classmethod
    def from_particles(cls, p) -> "State":
        return cls(pos=p.positions(), vel=p.velocities(), q=p.q.copy(), m=p.m.copy(), L=p.L,
                   n_max=p.n_max, kind=p.shape, a=p.a, eps0=p.eps0)

    def _modes(self):
        if self.modes is None:
            self.modes = half_modes(self.n_max, dim=self.pos.shape[0])
        return self.modes

    def refresh(self):
        f = fields(self.pos, self.q, self.L, self.n_max, self.kind, self.a, self.eps0, self._modes())
        self.F, self.W, self.rho = f.F, f.W, f.rho
        return f


def step_kdk(s: State, h: float, n_steps: int = 1) -> State:
    """Kick-drift-kick leapfrog: v += (h/2) F/m; x = wrap(x + h v); F = F(x);
    v += (h/2) F/m.  The force of the previous step's end is reused."""
    if s.F is None:
        s.refresh()
    for _ in range(n_steps):
        s.vel = s.vel + (0.5 * h) * s.F / s.m
        s.pos = wrap(s.pos + h * s.vel, s.L)
        s.refresh()
        s.vel = s.vel + (0.5 * h) * s.F / s.m
        s.step += 1
    return s


def step_dkd(s: State, h: float, n_steps: int = 1) -> State:
    """Drift-kick-drift (the paper's velocity form, Section 4):
    x = wrap(x + (h/2) v); F = F(x) at the half step; v += h F/m; x = wrap(x + (h/2) v).
    After the step, F/W/rho refer to the half-step positions, not to ``pos``."""
    for _ in range(n_steps):
        s.pos = wrap(s.pos + (0.5 * h) * s.vel, s.L)
        s.refresh()
        s.vel = s.vel + h * s.F / s.m
        s.pos = wrap(s.pos + (0.5 * h) * s.vel, s.L)
        s.step += 1
    s.F = None
    s.W = None
    s.rho = None
    return s


def kinetic(s: State) -> float:
    return float(0.5 * np.sum(s.m * np.sum(s.vel * s.vel, axis=0)))


def momentum(s: State) -> np.ndarray:
    return np.sum(s.m * s.vel, axis=1)


def energy(s: State) -> dict:
    """Energies at the state's current positions and velocities.  Recomputes the
    fields when they are not current (after a drift-kick-drift step)."""
    if s.W is None:
        s.refresh()
    K = kinetic(s)
    return {"kinetic": K, "field": s.W, "total": K + s.W,
            "momentum": momentum(s), "momentum_abs_sum": float(np.sum(s.m * np.linalg.norm(s.vel, axis=0)))}
