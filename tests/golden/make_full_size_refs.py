"""Write the FP64 oracle's values for the full-size parity tests.

Calls only ``oracle`` and ``workloads``: every stored number is the plain
double-loop oracle's, on the seeded synthetic inputs the tests regenerate.
The tests only read these files; they never write them.

Each case stores the oracle's rho on a sample of modes (always including
(1, 0, 0)) and its force on a sample of particles, computed from the oracle's
own full deposit (the force of any particle needs every mode's psi, which
needs every particle).  Run from the repository root:

    python tests/golden/make_full_size_refs.py [case ...]

Cases (about an hour on 8 cores in total, most of it the first two):

* ``cold_lattice_1M_n32``  2^20-particle jittered lattice, n_max = 32, the
                           Gaussian a = 0.01 (the timed workload), step 0.
* ``random_plasma_65536_n16_kdk`` 65,536-particle neutral plasma, n_max = 16,
                           a = 0.02, dt = 1e-3: the oracle's own kick-drift-kick
                           run, with the positions and the fields stored at
                           steps 50 and 100 (the GPU is fed the oracle's
                           positions there, so both sides see identical states).
* ``two_species_262144_n16`` 262,144-particle ion/electron plasma, n_max = 16.
* ``random_plasma_262144_n17`` 262,144 particles, n_max = 17.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

N_SAMPLE_PARTICLES = 4096
N_SAMPLE_MODES = 4096


def _sample(n: int, k: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, min(k, n), replace=False))


def _mode_sample(modes: np.ndarray, seed: int) -> np.ndarray:
    k1 = int(np.nonzero((modes == [1, 0, 0]).all(axis=1))[0][0])
    return np.unique(np.concatenate([[k1], _sample(len(modes), N_SAMPLE_MODES, seed)]))


def _fields_sampled(p, pos, seed: int) -> dict:
    """Full oracle deposit and solve at ``pos``; rho on sampled modes, F and
    Phi on sampled particles, W."""
    modes = oracle.half_modes(p.n_max)
    t = time.time()
    rho = oracle.deposit(pos, p.q, p.L, modes, p.shape, p.a)
    ps = oracle.psi(rho, p.L, modes, p.eps0, p.shape, p.a)
    pj = _sample(p.N, N_SAMPLE_PARTICLES, seed + 1)
    F = oracle.force_from_psi(pos[:, pj], p.q[pj], p.L, modes, ps)
    phi = oracle.potential_from_psi(pos[:, pj], p.L, modes, ps)
    mi = _mode_sample(modes, seed)
    print(f"  fields of {p.N} x {len(modes)} in {time.time() - t:.1f} s", flush=True)
    return {"mode_idx": mi, "rho": rho[mi], "rho_abs_max": np.max(np.abs(rho)),
            "particle_idx": pj, "F": F, "phi": phi,
            "W": oracle.field_energy(rho, p.L, modes, p.eps0)}


def _save(name: str, **arrays):
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, **arrays)
    print(f"  wrote {path} ({os.path.getsize(path) / 1e6:.2f} MB)", flush=True)


def cold_lattice_1M_n32():
    p = workloads.cold_lattice()
    _save("cold_lattice_1M_n32", **_fields_sampled(p, p.positions(), 101))


def two_species_262144_n16():
    p = workloads.two_species()
    _save("two_species_262144_n16", **_fields_sampled(p, p.positions(), 201))


def random_plasma_262144_n17():
    p = workloads.random_plasma(N=262144, n_max=17, a=0.02, salt=17)
    _save("random_plasma_262144_n17", **_fields_sampled(p, p.positions(), 301))


def random_plasma_65536_n16_kdk():
    p = workloads.random_plasma()
    s = oracle.State.from_particles(p)
    out = {}
    done = 0
    for stop in (50, 100):
        t = time.time()
        oracle.step_kdk(s, p.dt, stop - done)
        done = stop
        print(f"  oracle KDK to step {stop} in {time.time() - t:.1f} s", flush=True)
        f = _fields_sampled(p, s.pos, 400 + stop)
        e = oracle.energy(s)
        out.update({f"x{stop}": s.pos.copy(),
                    f"kinetic{stop}": e["kinetic"], f"momentum{stop}": e["momentum"]})
        out.update({f"{k}{stop}": v for k, v in f.items()})
    _save("random_plasma_65536_n16_kdk", **out)


CASES = {f.__name__: f for f in (two_species_262144_n16, random_plasma_262144_n17,
                                  cold_lattice_1M_n32, random_plasma_65536_n16_kdk)}

if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    print(f"oracle threads: {oracle.threads()}", flush=True)
    for name in names:
        print(name, flush=True)
        CASES[name]()
