"""Full-size parity of the HIP path against the FP64 oracle, in the launch
configurations that the large workloads run.

The oracle's values at these sizes (a full deposit over every particle and
mode, then the force on sampled particles) take minutes on the host, so they
are stored under ``tests/golden/`` by ``tests/golden/make_full_size_refs.py``,
a script that calls only the oracle on the seeded inputs regenerated here.

Cases:
* 262,144 particles: above 261,888 the one-particle-per-lane VALU force runs
  (its n_z register chunk is 16 in FP64 and 32 in FP32 at n_max = 17); the
  ion/electron plasma at n_max = 16 is the long-run workload itself.
* the 2^20-particle lattice at n_max = 32: rho on 4,097 sampled modes and F on
  4,096 sampled particles, every precision.
* the 65,536-particle plasma at the oracle's own steps 50 and 100: both sides
  take the oracle's positions there, so the fields are compared at identical
  states; the GPU's own FP64 trajectory is compared with the oracle's too.
* two dimensions above the small-count kernels, where the force visits only
  the n_x = 0 line of rows.

Bars: FP64 1e-12, FP32 and split FP16 1e-5 (normwise, as in the other parity
tests).
"""
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "split_f16": 1e-5}
PRECS = ["fp64", "fp32", "split_f16"]
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1508_07344_amd as sce
    sce.load_library()
    return sce


def _golden(name):
    path = os.path.join(GOLDEN, name + ".npz")
    if not os.path.exists(path):
        pytest.fail(f"{path} missing: run tests/golden/make_full_size_refs.py {name}")
    return np.load(path)


def e_rel(a, ref):
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))


def e_F(F, ref):
    return float(np.max(np.linalg.norm(F - ref, axis=0)) / np.max(np.linalg.norm(ref, axis=0)))


def _check(sce, p, pos, ref, prec, label):
    """Deposit and force at ``pos`` through the C ABI; rho on the stored modes,
    F and Phi on the stored particles, W and max|rho| against the oracle's."""
    with sce.Context(p.L, p.n_max, p.shape, p.a) as c:
        c.sce_set_options(p.eps0, prec, "kdk")
        c.sce_set_particles(np.ascontiguousarray(pos), np.zeros_like(pos), p.q, p.m)
        rho = c.sce_deposit()
        F = c.sce_force()
        d, st = c.sce_diagnostics()
    pj = ref["particle_idx"]
    er = e_rel(rho[ref["mode_idx"]], ref["rho"])
    ef = e_F(F[:, pj], ref["F"])
    ew = abs(d.field - float(ref["W"])) / abs(float(ref["W"]))
    em = abs(d.rho_abs_max - float(ref["rho_abs_max"])) / float(ref["rho_abs_max"])
    print(f"{label} {prec}: e_rho={er:.3e} e_F={ef:.3e} e_W={ew:.3e} e_max|rho|={em:.3e}", flush=True)
    assert er <= TOL[prec] and ef <= TOL[prec] and ew <= TOL[prec] and em <= TOL[prec]
    return rho, F


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", ["two_species_262144_n16", "random_plasma_262144_n17"])
def test_262144_particles_match_oracle(case, prec):
    sce = _gpu()
    p = workloads.two_species() if case.startswith("two_species") else \
        workloads.random_plasma(N=262144, n_max=17, a=0.02, salt=17)
    _check(sce, p, p.positions(), _golden(case), prec, case)


@pytest.mark.parametrize("prec", PRECS)
def test_cold_lattice_1M_n32_matches_oracle(prec):
    """The timed workload: 1,048,576 particles x 137,312 modes."""
    sce = _gpu()
    p = workloads.cold_lattice()
    _check(sce, p, p.positions(), _golden("cold_lattice_1M_n32"), prec, "cold_lattice_1M_n32")


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("step", [50, 100])
def test_random_plasma_at_oracle_steps(prec, step):
    """Fields at the oracle's own kick-drift-kick states of the 65,536-particle
    plasma (steps 50 and 100 of dt = 1e-3)."""
    sce = _gpu()
    p = workloads.random_plasma()
    g = _golden("random_plasma_65536_n16_kdk")
    ref = {k: g[f"{k}{step}"] for k in ("mode_idx", "rho", "particle_idx", "F", "W", "rho_abs_max")}
    _check(sce, p, g[f"x{step}"], ref, prec, f"random_plasma step {step}")


def test_random_plasma_gpu_trajectory_against_oracle_states():
    """The GPU's own FP64 run of the whole 100-step workload from the same
    start, against the oracle's states at steps 50 and 100, with kinetic energy
    and momentum.  Over these 100 steps (25 inverse plasma frequencies) the
    two trajectories stay within a few 1e-15 L of each other; the bounds leave
    three orders of magnitude for roundoff growth."""
    sce = _gpu()
    p = workloads.random_plasma()
    g = _golden("random_plasma_65536_n16_kdk")
    with sce.Context.from_particles(p) as c:
        for step in (50, 100):
            c.sce_step(p.dt, 50)
            x, v = c.sce_get_particles()
            d, st = c.sce_diagnostics()
            dx = np.max(np.abs((x - g[f"x{step}"] + 0.5 * p.L) % p.L - 0.5 * p.L))
            dK = abs(d.kinetic - float(g[f"kinetic{step}"])) / float(g[f"kinetic{step}"])
            dP = np.max(np.abs(d.momentum - g[f"momentum{step}"])) / d.momentum_abs_sum
            print(f"step {step}: max|dx| = {dx:.3e} L, dK/K = {dK:.3e}, dP = {dP:.3e}", flush=True)
            assert dx < 1e-11 * p.L and dK < 1e-12 and dP <= 1e-12


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("N,n_max,a,n_sample", [(20000, 8, 0.04, 0), (262144, 32, 0.01, 4096)])
def test_2d_force_above_the_small_count_kernels(N, n_max, a, n_sample, prec):
    """Two dimensions: the force kernels visit only the n_x = 0 line of rows
    (20,000 particles at n_max = 8: one line group; 262,144 particles: one
    particle per lane at any n_max).  rho on every mode, F on every particle
    or on a sample, against the oracle's 2-D loops."""
    sce = _gpu()
    p = workloads.random_plasma_2d(N=N, n_max=n_max, a=a, salt=N)
    modes = oracle.half_modes(n_max, dim=2)
    rho_ref = oracle.deposit(p.positions(), p.q, p.L, modes, p.shape, p.a)
    psi_ref = oracle.psi(rho_ref, p.L, modes, p.eps0, p.shape, p.a)
    pj = np.arange(N) if not n_sample else np.sort(np.random.default_rng(N).choice(N, n_sample, replace=False))
    F_ref = oracle.force_from_psi(p.positions()[:, pj], p.q[pj], p.L, modes, psi_ref)
    with sce.Context.from_particles(p, precision=prec) as c:
        rho = c.sce_deposit()
        F = c.sce_force()
    er, ef = e_rel(rho, rho_ref), e_F(F[:, pj], F_ref)
    print(f"2d N={N} n_max={n_max} {prec}: e_rho={er:.3e} e_F={ef:.3e}", flush=True)
    assert er <= TOL[prec] and ef <= TOL[prec]
