"""GPU parity of two-dimensional contexts (``sce_create_2d``: line charges in a
periodic square, the setting of the paper's Sections 6 and 7) against the FP64
oracle's own 2-D sums, through the C ABI, in every precision.

Error measures and tolerances as in the 3-D parity tests: normwise
e_rho = max|d rho| / max|rho_ref|, e_F = max_j |d F_j|_2 / max_j |F_ref,j|_2;
FP64 <= 1e-12, FP32 and split FP16 <= 1e-5.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "split_f16": 1e-5}
PRECS = ["fp64", "fp32", "split_f16"]


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1508_07344_amd as sce
    sce.load_library()
    return sce


def e_rho(r, ref):
    return float(np.max(np.abs(r - ref)) / np.max(np.abs(ref)))


def e_F(F, ref):
    return float(np.max(np.linalg.norm(F - ref, axis=0)) / np.max(np.linalg.norm(ref, axis=0)))


def _cases():
    r2 = workloads.random_particles_2d
    return [
        ("one", r2(1, L=1.0, charge="positive").with_(n_max=3, a=0.05)),
        ("kepler", workloads.kepler_2d()),
        ("thermal16", workloads.thermal_2d()),
        ("tent", r2(333, L=2.3, charge="uniform").with_(n_max=5, shape="tent", a=0.2)),
        ("delta", r2(1237, L=1.7, charge="alternating").with_(n_max=12, shape="delta", a=0.0)),
        ("eps0", r2(517, L=1.0, charge="uniform").with_(n_max=4, a=0.03, eps0=0.25)),
        ("plasma16", workloads.random_plasma_2d(N=3001, n_max=16, a=0.02)),
        ("plasma32", workloads.random_plasma_2d(N=4099, n_max=32, a=0.01)),
        ("n40", r2(700, L=1.0, charge="alternating").with_(n_max=40, a=0.01)),
        ("n64", r2(2570, L=1.3, charge="uniform").with_(n_max=64, a=0.005)),
    ]


@pytest.fixture(scope="module")
def references():
    _gpu()
    out = {}
    for name, p in _cases():
        out[name] = (p, oracle.fields(p.positions(), p.q, p.L, p.n_max, p.shape, p.a, p.eps0))
    return out


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", [c[0] for c in _cases()])
def test_2d_deposit_and_force_match_oracle(references, name, prec):
    sce = _gpu()
    p, ref = references[name]
    with sce.Context.from_particles(p, precision=prec) as c:
        assert c.sce_dimension() == 2
        assert np.array_equal(c.sce_modes(), oracle.half_modes(p.n_max, dim=2))
        rho = c.sce_deposit()
        psi = c.sce_psi()
        F = c.sce_force()
        d, st = c.sce_diagnostics()
    assert F.shape == (2, p.N)
    er, ep = e_rho(rho, ref.rho), e_rho(psi, ref.psi)
    ef = e_F(F, ref.F) if p.N > 1 else 0.0
    print(f"2d {name} {prec}: e_rho={er:.3e} e_psi={ep:.3e} e_F={ef:.3e}")
    assert er <= TOL[prec] and ep <= TOL[prec]
    if p.N > 1:
        assert ef <= TOL[prec]
    else:
        modes = oracle.half_modes(p.n_max, dim=2)
        k = oracle.wave_vectors(modes, p.L)
        S = oracle.shape(p.shape, p.a, k)
        scale = np.sum(2 * np.linalg.norm(k, axis=1) * S * S / np.sum(k * k, axis=1)) / (p.eps0 * p.L ** 2)
        assert np.max(np.abs(F)) < TOL[prec] * scale
    assert abs(d.field - ref.W) <= TOL[prec] * abs(ref.W)
    assert abs(d.interaction - 2 * ref.W) <= (1e-12 if prec == "fp64" else 1e-5) * abs(ref.W)
    assert d.momentum[2] == 0.0
    e = oracle.self_energy(p.q, p.L, oracle.half_modes(p.n_max, dim=2), p.eps0, p.shape, p.a)
    assert abs(d.field_self - e) <= 1e-12 * abs(e)


@pytest.mark.parametrize("prec", PRECS)
def test_2d_full_size_sampled(prec):
    """N = 65536 line charges, n_max = 32 (2,112 modes): every rho against the
    oracle, F on 2,048 sampled particles."""
    sce = _gpu()
    p = workloads.random_plasma_2d(N=65536, n_max=32, a=0.01)
    modes = oracle.half_modes(p.n_max, dim=2)
    pos = p.positions()
    rho_ref = oracle.deposit(pos, p.q, p.L, modes, p.shape, p.a)
    psi_ref = oracle.psi(rho_ref, p.L, modes, p.eps0, p.shape, p.a)
    idx = np.random.default_rng(3).choice(p.N, 2048, replace=False)
    F_ref = oracle.force_from_psi(pos[:, idx], p.q[idx], p.L, modes, psi_ref)
    with sce.Context.from_particles(p, precision=prec) as c:
        rho = c.sce_deposit()
        F = c.sce_force()
    er, ef = e_rho(rho, rho_ref), e_F(F[:, idx], F_ref)
    print(f"2d full {prec}: e_rho={er:.3e} e_F={ef:.3e}")
    assert er <= TOL[prec] and ef <= TOL[prec]


@pytest.mark.parametrize("scheme,steps", [("kdk", 2000), ("dkd", 300)])
def test_kepler_2d_trajectory_matches_oracle(scheme, steps):
    """The paper's 2-D two-body test: the GPU trajectory follows the oracle's,
    and the non-zero total momentum is conserved to roundoff."""
    sce = _gpu()
    p = workloads.kepler_2d()
    s = oracle.State.from_particles(p)
    P0 = oracle.momentum(s).copy()
    (oracle.step_kdk if scheme == "kdk" else oracle.step_dkd)(s, p.dt, steps)
    with sce.Context.from_particles(p, scheme=scheme) as c:
        c.sce_step(p.dt, steps)
        x, v = c.sce_get_particles()
        d, st = c.sce_diagnostics()
    assert x.shape == (2, 2)
    dx = np.max(np.abs((x - s.pos + 0.5) % 1.0 - 0.5))
    dv = np.max(np.abs(v - s.vel))
    print(f"kepler 2d {scheme} {steps} steps: dx={dx:.3e} dv={dv:.3e}")
    assert dx < 1e-9 and dv < 1e-9
    e = oracle.energy(s)
    assert abs(d.total - e["total"]) < 1e-10 * abs(e["total"])
    assert np.max(np.abs(d.momentum[:2] - P0)) <= 1e-12 * d.momentum_abs_sum


@pytest.mark.parametrize("prec", PRECS)
def test_2d_short_plasma_run_matches_oracle(prec):
    sce = _gpu()
    p = workloads.random_plasma_2d(N=512, n_max=8, a=0.05, sigma_v=0.05)
    s = oracle.State.from_particles(p)
    oracle.step_kdk(s, 1e-3, 20)
    with sce.Context.from_particles(p, precision=prec) as c:
        c.sce_step(1e-3, 20)
        x, v = c.sce_get_particles()
    dx = np.max(np.abs((x - s.pos + 0.5) % 1.0 - 0.5))
    tol = 1e-11 if prec == "fp64" else 1e-7
    print(f"2d plasma512 {prec} 20 steps: dx={dx:.3e}")
    assert dx < tol


def test_2d_momentum_resume_and_device_tensors():
    """Momentum conserved to roundoff over 20 FP64 steps; a checkpoint resumes
    bit for bit; device tensors in and out give the host results."""
    sce = _gpu()
    import torch
    p = workloads.random_plasma_2d(N=20000, n_max=16, a=0.02)
    with sce.Context.from_particles(p) as c:
        d0, _ = c.sce_diagnostics()
        c.sce_step(p.dt, 10)
        blob = c.sce_get_state()
        c.sce_step(p.dt, 10)
        d1, _ = c.sce_diagnostics()
        xa, va = c.sce_get_particles()
        Fa = c.sce_force()
    rel = np.max(np.abs(d1.momentum - d0.momentum)) / d1.momentum_abs_sum
    print(f"2d momentum error after 20 steps: {rel:.3e}")
    assert rel <= 1e-12
    with sce.Context(p.L, p.n_max, p.shape, p.a, dim=2) as c2:
        c2.sce_set_state(blob)
        c2.sce_step(p.dt, 10)
        xb, vb = c2.sce_get_particles()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    with sce.Context(p.L, p.n_max, p.shape, p.a, dim=3) as c3:
        with pytest.raises(sce.SceError):
            c3.sce_set_state(blob)
    with sce.Context.from_particles(p.with_(x=xa[0].copy(), y=xa[1].copy()), device=True) as cd:
        Fd = torch.zeros((2, p.N), dtype=torch.float64, device="cuda")
        cd.sce_force(Fd)
        xd = torch.zeros((2, p.N), dtype=torch.float64, device="cuda")
        cd.sce_get_particles(xd, None)
    assert np.array_equal(Fd.cpu().numpy(), Fa)
    assert np.array_equal(xd.cpu().numpy(), xa)


def _k1_index_2d(n):
    """Canonical index of mode (1, 0): after the n_x = 0 row (n modes) and
    n_y = -n..-1 of n_x = 1."""
    return n + n


@pytest.mark.parametrize("prec", ["fp64", "split_f16"])
def test_cold_plasma_frequency_2d(prec):
    """Cold 2-D plasma, 256 x 256 lattice: the (1, 0) mode oscillates at the
    paper's discrete frequency (2/h) asin(w_p h S(k1)/2), w_p^2 = N/(eps0 L^2)."""
    sce = _gpu()
    p = workloads.cold_lattice_2d(256, 256, n_max=16, a=0.01, dt=2e-3, n_steps=60)
    wp = math.sqrt(p.N / p.L ** 2)
    S1 = math.exp(-0.5 * (2 * math.pi * p.a / p.L) ** 2)
    w_ref = (2.0 / p.dt) * math.asin(wp * p.dt * S1 / 2.0)
    k1 = _k1_index_2d(p.n_max)
    assert tuple(oracle.half_modes(p.n_max, dim=2)[k1]) == (1, 0)
    series = []
    with sce.Context.from_particles(p, precision=prec) as c:
        for _ in range(p.n_steps):
            c.sce_step(p.dt, 1)
            series.append(c.sce_deposit()[k1].real)
    series = np.array(series)
    t = p.dt * np.arange(1, len(series) + 1)
    best = None
    for w in np.linspace(0.9 * w_ref, 1.1 * w_ref, 2001):
        A = np.stack([np.cos(w * t), np.sin(w * t), np.ones_like(t)], axis=1)
        coef, *_ = np.linalg.lstsq(A, series, rcond=None)
        r = np.sum((A @ coef - series) ** 2)
        if best is None or r < best[0]:
            best = (r, w)
    print(f"2d omega={best[1]:.3f} reference={w_ref:.3f} ({prec})")
    assert abs(best[1] / w_ref - 1) < 2e-3
