"""Seeded synthetic particle sets for the spectral electrostatic hot path.

This module is shared by the FP64 oracle (``oracle/``) and the HIP path
(``paper_1508_07344_amd``).  It builds inputs only: positions, velocities,
charges and masses.  It contains none of the method's arithmetic (no phases,
no mode sums, no field solve, no time stepping), so the two sides that are
compared against each other share nothing but their inputs.

Every generator returns a ``Particles`` record with float64 structure-of-arrays
fields ``x, y, z, vx, vy, vz, q, m`` (each shape ``[N]``) plus the run
parameters of the workload it stands for.

Workload recipes (the paper's own runs are 2D and only partly specified, so
these are 3D periodic-box stand-ins with the paper's ingredients: point-like
Gaussian macroparticles, discrete Fourier modes, a periodic box, a neutral or
background-neutralised plasma):

* ``two_body``      -- two opposite unit charges, 3D analogue of the two-body
                       (Kepler-like) test of the paper's Section 6.
* ``random_plasma`` -- neutral random plasma, uniform positions, alternating
                       +/- charges, Maxwellian velocities (Section 7 stand-in).
* ``cold_lattice``  -- cold electron plasma on a jittered uniform lattice with a
                       sinusoidal density perturbation along x; the uniform
                       neutralising background is the excluded n = 0 mode.
                       Used for the cold-plasma dispersion relation of
                       Section 5.
* ``two_species``   -- neutral ion/electron plasma with mass ratio 100.
* ``serving_requests`` -- a stream of independent small simulations with
                       log-uniform particle counts and step counts.

Two-dimensional records (``dim = 2``; positions and velocities [2, N], the
z fields are zero and unused) follow the paper's own test settings:

* ``kepler_2d``     -- an electron and a "double positron" (twice the mass,
                       twice the opposite charge) in a periodic square with
                       tent shapes and some net linear momentum (Section 6).
* ``thermal_2d``    -- 16 macroparticles with about 80 half-plane modes
                       (n_max = 6: 84), the size of the paper's thermal-plasma
                       run (Section 7), with its stated ratios L = 4 lambda_D and
                       width 0.1 lambda_D; its time step and its table's
                       physical values are not self-consistent and are not taken.
* ``random_plasma_2d``, ``cold_lattice_2d``, ``random_particles_2d`` -- the 2-D
                       counterparts of the 3-D generators.

Tent-field records (``field = "tent"``: finite-width field shapes on all of
R^D, point particles, no periodic box):

* ``tent_plasma``   -- a neutral plasma of point charges, uniform in the
                       central cube [-L/4, L/4]^D where the basis envelope is
                       largest, alternating +/-1, Maxwellian velocities, in 2-D
                       or 3-D.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ROOT_SEED = 20150828  # arXiv submission date of the paper, used as a fixed root seed

# index of each named workload in the root seed's spawned children
_STREAM = {"two_body": 0, "random_plasma": 1, "cold_lattice": 2,
           "two_species": 3, "serving": 4, "misc": 5, "two_d": 6, "tent": 7}


def _rng(name: str, salt: int = 0) -> np.random.Generator:
    children = np.random.SeedSequence(ROOT_SEED).spawn(len(_STREAM))
    ss = children[_STREAM[name]]
    if salt:
        ss = np.random.SeedSequence([ROOT_SEED, _STREAM[name], int(salt)])
    return np.random.Generator(np.random.PCG64(ss))


@dataclasses.dataclass
class Particles:
    """Particle state plus the run parameters of one workload."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    q: np.ndarray
    m: np.ndarray
    L: float = 1.0
    n_max: int = 8
    shape: str = "gaussian"   # "gaussian" | "delta" | "tent"
    a: float = 0.05           # Gaussian width, or tent half-width
    eps0: float = 1.0
    dt: float = 1e-3
    n_steps: int = 1
    name: str = ""
    dim: int = 3              # 2: line charges in the periodic square, z unused
    field: str = "delta"      # "tent": finite-width field shapes, open domain, point particles

    @property
    def N(self) -> int:
        return int(self.x.shape[0])

    def positions(self) -> np.ndarray:
        """[dim, N] float64 copy of the positions."""
        if self.dim == 2:
            return np.stack([self.x, self.y]).copy()
        return np.stack([self.x, self.y, self.z]).copy()

    def velocities(self) -> np.ndarray:
        if self.dim == 2:
            return np.stack([self.vx, self.vy]).copy()
        return np.stack([self.vx, self.vy, self.vz]).copy()

    def copy(self) -> "Particles":
        return dataclasses.replace(self, **{f: getattr(self, f).copy() for f in
                                            ("x", "y", "z", "vx", "vy", "vz", "q", "m")})

    def subset(self, idx) -> "Particles":
        return dataclasses.replace(self, **{f: np.ascontiguousarray(getattr(self, f)[idx]) for f in
                                            ("x", "y", "z", "vx", "vy", "vz", "q", "m")})

    def with_(self, **kw) -> "Particles":
        return dataclasses.replace(self, **kw)


def _make(x, y, z, vx, vy, vz, q, m, **kw) -> Particles:
    f = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return Particles(f(x), f(y), f(z), f(vx), f(vy), f(vz), f(q), f(m), **kw)


def two_body(dt: float = 1e-3, n_steps: int = 2000, n_max: int = 8, a: float = 0.05) -> Particles:
    """+1 charge at (0.3, 0.5, 0.5) moving +y, -1 charge at (0.7, 0.5, 0.5) moving -y,
    unit masses, transverse speed 0.05 each, unit box, eps0 = 1."""
    return _make([0.3, 0.7], [0.5, 0.5], [0.5, 0.5],
                 [0.0, 0.0], [0.05, -0.05], [0.0, 0.0],
                 [1.0, -1.0], [1.0, 1.0],
                 L=1.0, n_max=n_max, shape="gaussian", a=a, eps0=1.0,
                 dt=dt, n_steps=n_steps, name="two_body")


def random_plasma(N: int = 65536, n_max: int = 16, a: float = 0.02, sigma_v: float = 0.01,
                  dt: float = 1e-3, n_steps: int = 100, L: float = 1.0, salt: int = 0,
                  shape: str = "gaussian", eps0: float = 1.0) -> Particles:
    """Neutral random plasma: uniform positions in [0, L)^3, charges +1 (even index)
    and -1 (odd index), unit masses, Maxwellian velocities with std sigma_v per
    Cartesian component."""
    g = _rng("random_plasma", salt)
    pos = g.random((3, N)) * L
    vel = g.normal(0.0, sigma_v, (3, N))
    q = np.where(np.arange(N) % 2 == 0, 1.0, -1.0)
    m = np.ones(N)
    return _make(pos[0], pos[1], pos[2], vel[0], vel[1], vel[2], q, m,
                 L=L, n_max=n_max, shape=shape, a=a, eps0=eps0, dt=dt, n_steps=n_steps,
                 name=f"random_plasma_N{N}_n{n_max}")


def cold_lattice(nx: int = 128, ny: int = 128, nz: int = 64, n_max: int = 32, a: float = 0.01,
                 amplitude: float = 0.01, jitter: float = 1e-3, dt: float = 5e-4,
                 n_steps: int = 50, L: float = 1.0, salt: int = 0, mode: int = 1) -> Particles:
    """Cold electron plasma (q = -1, m = 1, v = 0) on an nx*ny*nz lattice of
    cell-centred sites, each coordinate jittered uniformly in [-jitter, jitter]*L,
    then displaced along x by xi(x0) = -(A/k1) sin(k1 x0), k1 = 2 pi mode / L,
    which realises the density n0 (1 + A cos(k1 x)) to first order in A."""
    g = _rng("cold_lattice", salt)
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    x0 = (i.ravel() + 0.5) / nx * L
    y0 = (j.ravel() + 0.5) / ny * L
    z0 = (k.ravel() + 0.5) / nz * L
    N = x0.size
    jit = g.uniform(-jitter, jitter, (3, N)) * L
    x0 = x0 + jit[0]
    y0 = y0 + jit[1]
    z0 = z0 + jit[2]
    k1 = 2.0 * math.pi * mode / L
    x = x0 - (amplitude / k1) * np.sin(k1 * x0)
    wrap = lambda u: u - L * np.floor(u / L)
    zeros = np.zeros(N)
    return _make(wrap(x), wrap(y0), wrap(z0), zeros, zeros, zeros,
                 -np.ones(N), np.ones(N), L=L, n_max=n_max, shape="gaussian", a=a, eps0=1.0,
                 dt=dt, n_steps=n_steps, name=f"cold_lattice_{nx}x{ny}x{nz}_n{n_max}")


def two_species(N: int = 262144, n_max: int = 16, a: float = 0.02, sigma_v: float = 0.02,
                m_ion: float = 100.0, dt: float = 1e-3, n_steps: int = 100000,
                L: float = 1.0, salt: int = 0) -> Particles:
    """Neutral two-species plasma: even index = ion (q=+1, m=m_ion), odd index =
    electron (q=-1, m=1), uniform positions, Maxwellian velocities with std
    sigma_v per component for both species."""
    g = _rng("two_species", salt)
    pos = g.random((3, N)) * L
    vel = g.normal(0.0, sigma_v, (3, N))
    even = np.arange(N) % 2 == 0
    q = np.where(even, 1.0, -1.0)
    m = np.where(even, m_ion, 1.0)
    return _make(pos[0], pos[1], pos[2], vel[0], vel[1], vel[2], q, m,
                 L=L, n_max=n_max, shape="gaussian", a=a, eps0=1.0, dt=dt, n_steps=n_steps,
                 name=f"two_species_N{N}_n{n_max}")


def random_particles(N: int, L: float = 1.0, salt: int = 0, charge: str = "alternating",
                     sigma_v: float = 0.01) -> Particles:
    """Small generic particle set for parity and property tests: uniform positions,
    charges alternating +/-1 ("alternating"), uniform in [-1, 1] ("uniform"), or
    all +1 ("positive"); masses uniform in [0.5, 2]."""
    g = _rng("misc", salt + 1)
    pos = g.random((3, N)) * L
    vel = g.normal(0.0, sigma_v, (3, N))
    if charge == "alternating":
        q = np.where(np.arange(N) % 2 == 0, 1.0, -1.0)
    elif charge == "uniform":
        q = g.uniform(-1.0, 1.0, N)
    elif charge == "positive":
        q = np.ones(N)
    else:
        raise ValueError(charge)
    m = g.uniform(0.5, 2.0, N)
    return _make(pos[0], pos[1], pos[2], vel[0], vel[1], vel[2], q, m, L=L,
                 name=f"random_{charge}_N{N}")


@dataclasses.dataclass
class Request:
    """One independent simulation of the serving workload."""
    id: int
    arrival_s: float
    particles: Particles


def serving_requests(n_requests: int = 4096, rate_per_s: float = 100.0,
                     n_max_choices=(4, 8, 16), N_range=(2, 8192), steps_range=(100, 10000),
                     sigma_v: float = 0.01, a: float = 0.05, dt: float = 1e-3,
                     salt: int = 0) -> list:
    """Independent requests with Poisson arrivals at ``rate_per_s``: N log-uniform
    in N_range rounded up to even (neutral +/-1 pairs), n_max uniform over
    n_max_choices, step count log-uniform in steps_range, uniform positions in the
    unit box, Maxwellian velocities with std sigma_v."""
    g = _rng("serving", salt)
    out = []
    t = 0.0
    for rid in range(n_requests):
        t += g.exponential(1.0 / rate_per_s)
        N = int(round(math.exp(g.uniform(math.log(N_range[0]), math.log(N_range[1])))))
        N = max(2, N + (N % 2))
        n_max = int(n_max_choices[int(g.integers(len(n_max_choices)))])
        steps = int(round(math.exp(g.uniform(math.log(steps_range[0]), math.log(steps_range[1])))))
        pos = g.random((3, N))
        vel = g.normal(0.0, sigma_v, (3, N))
        q = np.where(np.arange(N) % 2 == 0, 1.0, -1.0)
        p = _make(pos[0], pos[1], pos[2], vel[0], vel[1], vel[2], q, np.ones(N),
                  L=1.0, n_max=n_max, shape="gaussian", a=a, eps0=1.0, dt=dt,
                  n_steps=steps, name=f"request{rid}")
        out.append(Request(rid, t, p))
    return out


def rock_salt(L: float = 1.0) -> Particles:
    """Eight ions of a rock-salt (NaCl) conventional cubic cell filling the periodic
    box: +1 on the fcc sites (0,0,0), (0,h,h), (h,0,h), (h,h,0) and -1 on
    (h,0,0), (0,h,0), (0,0,h), (h,h,h) with h = L/2; nearest-neighbour distance L/2."""
    h = 0.5 * L
    pos = np.array([[0, 0, 0], [0, h, h], [h, 0, h], [h, h, 0],
                    [h, 0, 0], [0, h, 0], [0, 0, h], [h, h, h]], dtype=np.float64)
    q = np.array([1, 1, 1, 1, -1, -1, -1, -1], dtype=np.float64)
    z = np.zeros(8)
    return _make(pos[:, 0], pos[:, 1], pos[:, 2], z, z, z, q, np.ones(8), L=L,
                 name="rock_salt")


def grid_particles(G: int, L: float = 1.0, salt: int = 0) -> Particles:
    """One particle on every site of a G^3 grid (x = L*i/G), random charges in
    [-1, 1]; the index order is C order over (i, j, k)."""
    g = _rng("misc", 1000 + salt)
    i, j, k = np.meshgrid(np.arange(G), np.arange(G), np.arange(G), indexing="ij")
    q = g.uniform(-1.0, 1.0, G ** 3)
    z = np.zeros(G ** 3)
    return _make(i.ravel() * L / G, j.ravel() * L / G, k.ravel() * L / G, z, z, z, q,
                 np.ones(G ** 3), L=L, name=f"grid{G}")


# ---------------------------------------------------------------- two dimensions
def _make2(x, y, vx, vy, q, m, **kw) -> Particles:
    z = np.zeros(len(x))
    return _make(x, y, z, vx, vy, z, q, m, dim=2, **kw)


def kepler_2d(dt: float = 5e-3, n_steps: int = 2000, n_max: int = 16, a: float = 0.05,
              L: float = 1.0) -> Particles:
    """Line charges: an electron (q = -1, m = 1) at (0.4, 0.5) and a double
    positron (q = +2, m = 2) at (0.6, 0.5), tent shapes of half-width a, eps0 = 1.
    Velocities: a near-circular relative orbit for the line-charge attraction
    |F| = |q1 q2| / (2 pi eps0 r) at r = 0.2 (relative speed 0.69, split by the
    masses), plus a common drift (0.05, 0.02), so the total momentum is not zero."""
    r, q1q2, mu = 0.2, 2.0, 2.0 / 3.0
    vrel = math.sqrt(q1q2 / (2.0 * math.pi) / mu)
    v1 = vrel * 2.0 / 3.0     # m2 / (m1 + m2)
    v2 = -vrel * 1.0 / 3.0    # m1 / (m1 + m2)
    dx, dy = 0.05, 0.02
    return _make2([0.5 - r / 2, 0.5 + r / 2], [0.5, 0.5], [dx, dx], [v1 + dy, v2 + dy],
                  [-1.0, 2.0], [1.0, 2.0], L=L, n_max=n_max, shape="tent", a=a, eps0=1.0,
                  dt=dt, n_steps=n_steps, name="kepler_2d")


def thermal_2d(N: int = 16, n_max: int = 6, L: float = 1.0, n_steps: int = 1000,
               salt: int = 0) -> Particles:
    """Neutral thermal plasma of N line charges (alternating +/-1, unit masses,
    eps0 = 1), uniform positions, Maxwellian velocities, with the ratios the
    paper states for its thermal run (Section 7): box L = 4 Debye lengths and
    particle width 0.1 Debye length.  With omega_p^2 = N / L^2: lambda_D = L/4,
    sigma_v = omega_p lambda_D per component, Gaussian a = 0.1 lambda_D.  The
    paper's step, a fifth of a plasma period, lets a thermal particle cross
    the shortest retained wavelength twice per step (k_max sigma_v h = 12); the
    step here keeps k_max sigma_v h = 0.1."""
    wp = math.sqrt(N) / L
    lam = L / 4.0
    sigma_v, a = wp * lam, 0.1 * lam
    dt = 0.1 / (2.0 * math.pi * n_max / L * sigma_v)
    g = _rng("two_d", 100 + salt)
    pos = g.random((2, N)) * L
    vel = g.normal(0.0, sigma_v, (2, N))
    q = np.where(np.arange(N) % 2 == 0, 1.0, -1.0)
    return _make2(pos[0], pos[1], vel[0], vel[1], q, np.ones(N), L=L, n_max=n_max,
                  shape="gaussian", a=a, eps0=1.0, dt=dt, n_steps=n_steps,
                  name=f"thermal_2d_N{N}_n{n_max}")


def random_plasma_2d(N: int = 65536, n_max: int = 32, a: float = 0.01, sigma_v: float = 0.01,
                     dt: float = 1e-3, n_steps: int = 100, L: float = 1.0, salt: int = 0,
                     shape: str = "gaussian", eps0: float = 1.0) -> Particles:
    """Neutral random plasma in the square: uniform positions, charges +1 (even
    index) and -1 (odd index), unit masses, Maxwellian velocities."""
    g = _rng("two_d", salt)
    pos = g.random((2, N)) * L
    vel = g.normal(0.0, sigma_v, (2, N))
    q = np.where(np.arange(N) % 2 == 0, 1.0, -1.0)
    return _make2(pos[0], pos[1], vel[0], vel[1], q, np.ones(N), L=L, n_max=n_max,
                  shape=shape, a=a, eps0=eps0, dt=dt, n_steps=n_steps,
                  name=f"random_plasma_2d_N{N}_n{n_max}")


def cold_lattice_2d(nx: int = 64, ny: int = 64, n_max: int = 8, a: float = 0.02,
                    amplitude: float = 0.01, jitter: float = 1e-3, dt: float = 5e-3,
                    n_steps: int = 100, L: float = 1.0, salt: int = 0, mode: int = 1) -> Particles:
    """Cold electron plasma (q = -1, m = 1, v = 0) on an nx*ny lattice of
    cell-centred sites in the square, each coordinate jittered uniformly in
    [-jitter, jitter]*L, then displaced along x by -(A/k1) sin(k1 x0),
    k1 = 2 pi mode / L (density n0 (1 + A cos(k1 x)) to first order in A)."""
    g = _rng("two_d", 200 + salt)
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    x0 = (i.ravel() + 0.5) / nx * L
    y0 = (j.ravel() + 0.5) / ny * L
    N = x0.size
    jit = g.uniform(-jitter, jitter, (2, N)) * L
    x0 = x0 + jit[0]
    y0 = y0 + jit[1]
    k1 = 2.0 * math.pi * mode / L
    x = x0 - (amplitude / k1) * np.sin(k1 * x0)
    wrap = lambda u: u - L * np.floor(u / L)
    zeros = np.zeros(N)
    return _make2(wrap(x), wrap(y0), zeros, zeros, -np.ones(N), np.ones(N), L=L, n_max=n_max,
                  shape="gaussian", a=a, eps0=1.0, dt=dt, n_steps=n_steps,
                  name=f"cold_lattice_2d_{nx}x{ny}_n{n_max}")


def random_particles_2d(N: int, L: float = 1.0, salt: int = 0, charge: str = "alternating",
                        sigma_v: float = 0.01) -> Particles:
    """Small 2-D particle set for parity and property tests (charges as in
    ``random_particles``; masses uniform in [0.5, 2])."""
    g = _rng("two_d", 300 + salt)
    pos = g.random((2, N)) * L
    vel = g.normal(0.0, sigma_v, (2, N))
    if charge == "alternating":
        q = np.where(np.arange(N) % 2 == 0, 1.0, -1.0)
    elif charge == "uniform":
        q = g.uniform(-1.0, 1.0, N)
    elif charge == "positive":
        q = np.ones(N)
    else:
        raise ValueError(charge)
    m = g.uniform(0.5, 2.0, N)
    return _make2(pos[0], pos[1], vel[0], vel[1], q, m, L=L, name=f"random2d_{charge}_N{N}")


def grid_particles_2d(G: int, L: float = 1.0, salt: int = 0) -> Particles:
    """One line charge on every site of a G^2 grid (x = L*i/G), random charges in
    [-1, 1]; C order over (i, j)."""
    g = _rng("two_d", 400 + salt)
    i, j = np.meshgrid(np.arange(G), np.arange(G), indexing="ij")
    q = g.uniform(-1.0, 1.0, G * G)
    z = np.zeros(G * G)
    return _make2(i.ravel() * L / G, j.ravel() * L / G, z, z, q, np.ones(G * G), L=L,
                  name=f"grid2d_{G}")


def tent_plasma(N: int = 4096, n_max: int = 8, dim: int = 3, L: float = 1.0, half: float = 0.25,
                sigma_v: float = 0.01, dt: float | None = None, n_steps: int = 100,
                salt: int = 0) -> Particles:
    """Neutral plasma of N point charges for the tent-field variant: positions
    uniform in [-half L, half L]^dim (the envelope of the basis functions peaks
    at the origin and vanishes at |x_d| = L), charges alternating +1 / -1, unit
    masses, Maxwellian velocities of spread sigma_v, eps0 = 1.  The default step
    is dt = 0.1 / omega_p, omega_p^2 = N / (2 half L)^dim (unit q, m, eps0)."""
    if dt is None:
        dt = 0.1 / math.sqrt(N / (2.0 * half * L) ** dim)
    g = _rng("tent", salt)
    pos = g.uniform(-half * L, half * L, size=(3, N))
    vel = g.normal(0.0, sigma_v, size=(3, N))
    q = np.where(np.arange(N) % 2 == 0, 1.0, -1.0)
    m = np.ones(N)
    if dim == 2:
        return _make2(pos[0], pos[1], vel[0], vel[1], q, m, L=L, n_max=n_max, shape="delta", a=0.0,
                      eps0=1.0, dt=dt, n_steps=n_steps, name=f"tent_plasma_2d_{N}_n{n_max}",
                      field="tent")
    return _make(pos[0], pos[1], pos[2], vel[0], vel[1], vel[2], q, m, L=L, n_max=n_max,
                 shape="delta", a=0.0, eps0=1.0, dt=dt, n_steps=n_steps,
                 name=f"tent_plasma_{N}_n{n_max}", field="tent")
