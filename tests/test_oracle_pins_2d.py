"""Pins of the FP64 oracle's two-dimensional sums (line charges in a periodic
square, the setting of the paper's own test problems, Sections 6 and 7)
against facts independent of the oracle's code: a library 2-D FFT, the 2-D
Ewald summation identity (exponential-integral real-space kernel), the
scaling law of the logarithmic interaction, quadrature of the particle
shapes, central-difference gradients, conservation laws, time reversibility,
second-order energy error and the cold-plasma discrete dispersion relation of
Section 5 with the areal density.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import workloads


# ---------------------------------------------------------------- mode set
@pytest.mark.parametrize("n_max", [1, 2, 5, 8])
def test_half_plane_partitions_square(orc, n_max):
    """|H2| = (M^2 - 1)/2, H2 and -H2 are disjoint, and H2 u -H2 u {0} is the square."""
    H = orc.half_modes(n_max, dim=2)
    M = 2 * n_max + 1
    assert H.shape == ((M * M - 1) // 2, 2)
    s = {tuple(v) for v in H.tolist()}
    neg = {(-a, -b) for a, b in s}
    assert len(s) == len(H) and not (s & neg)
    sq = {(a, b) for a in range(-n_max, n_max + 1) for b in range(-n_max, n_max + 1)}
    assert s | neg | {(0, 0)} == sq
    assert sorted(s) == [tuple(v) for v in H.tolist()]
    assert len(orc.cube_modes(n_max, dim=2)) == M * M - 1


def test_shape_transforms_2d_match_quadrature(orc):
    """S(k) of a 2-D Gaussian density and of a tensor tent, by quadrature."""
    a = 0.07
    g1 = lambda kd: integrate.quad(lambda x: math.exp(-x * x / (2 * a * a)) / math.sqrt(2 * math.pi * a * a)
                                   * math.cos(kd * x), -12 * a, 12 * a, limit=200)[0]
    t1 = lambda kd: integrate.quad(lambda x: (1.0 - abs(x) / a) / a * math.cos(kd * x), -a, a,
                                   points=[0.0], limit=200)[0]
    for k in ([3.0, 0.0], [10.0, -20.0], [40.0, 33.0]):
        assert abs(orc.shape("gaussian", a, np.array(k))[0] - g1(k[0]) * g1(k[1])) < 1e-12
        assert abs(orc.shape("tent", a, np.array(k))[0] - t1(k[0]) * t1(k[1])) < 1e-12
        assert orc.shape("delta", a, np.array(k))[0] == 1.0


# ---------------------------------------------------------------- deposit
@pytest.mark.parametrize("L", [1.0, 2.7])
def test_deposit_2d_on_grid_equals_fft(orc, L):
    """Line charges exactly on a G^2 grid: rho_n = FFT2(q)[n mod G] (delta shape)."""
    G, n_max = 8, 3
    p = workloads.grid_particles_2d(G, L=L)
    modes = orc.cube_modes(n_max, dim=2)
    rho = orc.deposit(p.positions(), p.q, L, modes, "delta")
    Q = np.fft.fft2(p.q.reshape(G, G))
    ref = Q[modes[:, 0] % G, modes[:, 1] % G]
    assert np.max(np.abs(rho - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_deposit_2d_symmetry_translation_single(orc):
    """rho_{-n} = conj(rho_n); a shift d multiplies rho_n by exp(-i k_n . d); a
    box-length shift of one particle changes nothing; one particle gives |rho_n| = |q| S."""
    L = 1.3
    p = workloads.random_particles_2d(40, L=L, charge="uniform")
    pos = p.positions()
    modes = orc.cube_modes(4, dim=2)
    rho = orc.deposit(pos, p.q, L, modes, "gaussian", 0.05)
    idx = {tuple(v): i for i, v in enumerate(modes.tolist())}
    neg = np.array([idx[(-a, -b)] for a, b in modes.tolist()])
    assert np.max(np.abs(rho[neg] - np.conj(rho))) <= 1e-14 * np.max(np.abs(rho))
    d = np.array([0.123, -0.377])
    k = orc.wave_vectors(modes, L)
    rho_d = orc.deposit(pos + d[:, None], p.q, L, modes, "gaussian", 0.05)
    assert np.max(np.abs(rho_d - rho * np.exp(-1j * k @ d))) <= 1e-13 * np.max(np.abs(rho))
    pos2 = pos.copy()
    pos2[0, 7] += L
    pos2[1, 3] -= L
    assert np.max(np.abs(orc.deposit(pos2, p.q, L, modes, "gaussian", 0.05) - rho)) <= 1e-13 * np.max(np.abs(rho))
    one = orc.deposit(np.array([[0.31], [0.77]]), [-1.5], 1.0, orc.half_modes(5, dim=2), "delta")
    assert np.max(np.abs(np.abs(one) - 1.5)) < 1e-13


# ---------------------------------------------------------------- 2-D Ewald
def _ewald_real_2d(pos, q, L, alpha, images=2):
    """Real-space and self parts of the 2-D Ewald energy (eps0 = 1) and the
    real-space forces: pairs and periodic images interact through
    E1(alpha^2 r^2) / (4 pi); each charge adds q^2 (-gamma - ln alpha^2) / (8 pi)."""
    N = pos.shape[1]
    E = 0.0
    F = np.zeros_like(pos)
    rng = range(-images, images + 1)
    shifts = np.array([[a, b] for a in rng for b in rng], dtype=float) * L
    for i in range(N):
        for j in range(N):
            r = pos[:, i][None, :] - pos[:, j][None, :] + shifts
            d = np.linalg.norm(r, axis=1)
            if i == j:
                keep = d > 0
                r, d = r[keep], d[keep]
            E += 0.5 * q[i] * q[j] * np.sum(special.exp1((alpha * d) ** 2)) / (4 * np.pi)
            g = 2.0 * np.exp(-(alpha * d) ** 2) / d ** 2
            F[:, i] += q[i] * q[j] * np.sum(g[:, None] * r, axis=0) / (4 * np.pi)
    E += np.sum(q ** 2) * (-np.euler_gamma - math.log(alpha * alpha)) / (8 * np.pi)
    return E, F


def _log_total_2d(orc, pos, q, L, a, n_max):
    f = orc.fields(pos, q, L, n_max, "gaussian", a, 1.0)
    Er, Fr = _ewald_real_2d(pos, q, L, 1.0 / (2.0 * a))
    return f.W + Er, f.F + Fr


@pytest.mark.parametrize("L", [1.0, 1.6])
def test_ewald_2d_alpha_independence_and_scaling(orc, L):
    """The 2-D Ewald split of the periodic logarithmic interaction is exact: the
    spectral field energy W (Gaussian shape of width a, S^2 = exp(-k^2/(4 alpha^2))
    with alpha = 1/(2a)) plus the real-space and self parts does not depend on a,
    nor does the force.  Scaling a neutral configuration and its box by lambda
    adds sum q^2 ln(lambda) / (4 pi eps0) (the Green's function of the periodic
    square is scale invariant; only the regularised self-interaction shifts).
    Pins the 1/A and eps0 factors, the factor 2 of the half-plane sum, the S^2
    placement and the sign of the force."""
    pos = L * np.array([[0.11, 0.52, 0.83, 0.40], [0.20, 0.75, 0.33, 0.91]])
    q = np.array([1.0, -2.0, 0.5, 0.5])
    E1, F1 = _log_total_2d(orc, pos, q, L, 0.06 * L, 40)
    E2, F2 = _log_total_2d(orc, pos, q, L, 0.09 * L, 28)
    assert abs(E1 - E2) < 1e-11 * max(1.0, abs(E1))
    assert np.max(np.abs(F1 - F2)) < 1e-10 * np.max(np.abs(F1))
    if L != 1.0:
        E_unit, _ = _log_total_2d(orc, pos / L, q, 1.0, 0.06, 40)
        assert abs(E1 - (E_unit + np.sum(q ** 2) * math.log(L) / (4 * np.pi))) < 1e-11


# ---------------------------------------------------------------- force
def test_2d_lone_particle_newton_attraction(orc):
    """No self-force; total force zero; two-body forces equal and opposite;
    opposite line charges attract, like charges repel."""
    L, n_max, a = 1.0, 10, 0.03
    modes = orc.half_modes(n_max, dim=2)
    k = orc.wave_vectors(modes, L)
    S = orc.shape("gaussian", a, k)
    scale = np.sum(2 * np.linalg.norm(k, axis=1) * S * S / np.sum(k * k, axis=1) / L ** 2)
    for pos in ([0.3, 0.2], [0.0, 0.0], [0.999999, 0.123456789]):
        f = orc.fields(np.array(pos)[:, None], [1.7], L, n_max, "gaussian", a)
        assert np.max(np.abs(f.F)) <= 1e-14 * 1.7 ** 2 * scale
    p = workloads.random_particles_2d(50, L=1.0, charge="uniform")
    f = orc.fields(p.positions(), p.q, 1.0, 6, "gaussian", 0.05)
    assert np.max(np.abs(f.F.sum(axis=1))) <= 1e-13 * np.sum(np.abs(f.F))
    pos = np.array([[0.45, 0.55], [0.5, 0.5]])
    for qq, sign in (([1.0, -1.0], +1), ([1.0, 1.0], -1)):
        F = orc.fields(pos, qq, 1.0, 12, "gaussian", 0.03).F
        assert np.max(np.abs(F[:, 0] + F[:, 1])) < 1e-14 * np.abs(F[0, 0])
        assert np.sign(F[0, 0]) == sign and abs(F[1, 0]) < 1e-14 * np.abs(F[0, 0])


def test_2d_force_is_minus_energy_gradient_and_adjoint(orc):
    """F_j = -dW/dx_j by central differences; sum_j q_j Phi_j = 2 W."""
    L, n_max, a = 1.5, 6, 0.06
    p = workloads.random_particles_2d(12, L=L, charge="uniform")
    pos = p.positions()
    modes = orc.half_modes(n_max, dim=2)
    f = orc.fields(pos, p.q, L, n_max, "tent", a, modes=modes)
    d = 1e-6 * L
    for j in (0, 5, 11):
        for c in range(2):
            pp, pm = pos.copy(), pos.copy()
            pp[c, j] += d
            pm[c, j] -= d
            Wp = orc.field_energy(orc.deposit(pp, p.q, L, modes, "tent", a), L, modes)
            Wm = orc.field_energy(orc.deposit(pm, p.q, L, modes, "tent", a), L, modes)
            assert abs(-(Wp - Wm) / (2 * d) - f.F[c, j]) < 1e-7 * np.max(np.abs(f.F))
    U = np.sum(p.q * orc.potential_from_psi(pos, L, modes, f.psi))
    assert abs(U - 2 * f.W) < 1e-13 * abs(U)


# ---------------------------------------------------------------- time step
def test_kepler_2d_energy_bounded_momentum_conserved(orc):
    """The paper's 2-D two-body test (Section 6): energy bounded with no secular
    trend over 2000 kick-drift-kick steps, and the non-zero total momentum
    conserved to roundoff."""
    p = workloads.kepler_2d()
    s = orc.State.from_particles(p)
    e0 = orc.energy(s)
    E0, P0 = e0["total"], e0["momentum"].copy()
    assert np.max(np.abs(P0)) > 0.05
    Es, Ps = [], []
    for _ in range(40):
        orc.step_kdk(s, p.dt, 50)
        e = orc.energy(s)
        Es.append(e["total"] - E0)
        Ps.append(np.max(np.abs(e["momentum"] - P0)) / e["momentum_abs_sum"])
    Es = np.array(Es)
    assert np.max(np.abs(Es)) < 1e-3 * abs(E0)
    slope = np.polyfit(np.arange(len(Es)), Es, 1)[0] * len(Es)
    assert abs(slope) < 0.5 * np.max(np.abs(Es))
    assert max(Ps) < 1e-13


@pytest.mark.parametrize("scheme", ["kdk", "dkd"])
def test_kepler_2d_time_reversibility(orc, scheme):
    p = workloads.kepler_2d()
    s = orc.State.from_particles(p)
    x0, v0 = s.pos.copy(), s.vel.copy()
    step = orc.step_kdk if scheme == "kdk" else orc.step_dkd
    step(s, p.dt, 300)
    s.vel = -s.vel
    step(s, p.dt, 300)
    assert np.max(np.abs(s.pos - x0)) < 1e-11
    assert np.max(np.abs(s.vel + v0)) < 1e-11


def test_kepler_2d_energy_error_scales_as_h_squared(orc):
    errs = []
    hs = [1.6e-2, 8e-3, 4e-3, 2e-3]
    for h in hs:
        p = workloads.kepler_2d(dt=h)
        s = orc.State.from_particles(p)
        E0 = orc.energy(s)["total"]
        dev = 0.0
        for _ in range(int(round(1.6 / h))):
            orc.step_kdk(s, h, 1)
            dev = max(dev, abs(orc.energy(s)["total"] - E0))
        errs.append(dev)
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert 1.85 < slope < 2.15, (slope, errs)


def _dispersion_2d(orc, h, n_steps, G=32, n_max=4, a=0.05, L=1.0, eps0=1.0, amp=0.01):
    p = workloads.cold_lattice_2d(G, G, n_max=n_max, a=a, amplitude=amp, jitter=0.0, dt=h, L=L)
    p = p.with_(eps0=eps0)
    s = orc.State.from_particles(p)
    k1 = np.array([[1, 0]], dtype=np.int32)
    series = []
    for _ in range(n_steps):
        orc.step_kdk(s, h, 1)
        series.append(orc.deposit(s.pos, s.q, s.L, k1, "gaussian", a)[0].real)
    return np.array(series)


@pytest.mark.parametrize("L,eps0", [(1.0, 1.0), (0.8, 0.5)])
def test_cold_plasma_dispersion_2d(orc, L, eps0):
    """Cold 2-D plasma: the k1 = (1, 0) density mode oscillates at
    omega = (2/h) asin(omega_p h S(k1) / 2) (Section 5), with
    omega_p^2 = n q^2 / (eps0 m) for the areal density n = N / L^2."""
    G, a = 32, 0.05 * L
    wp = math.sqrt(G * G / (eps0 * L * L))
    S1 = math.exp(-0.5 * (2 * math.pi * a / L) ** 2)
    h = 0.5 / wp
    series = _dispersion_2d(orc, h, 60, G=G, a=a, L=L, eps0=eps0)
    omega_ref = (2.0 / h) * math.asin(wp * h * S1 / 2.0)
    t = h * np.arange(1, len(series) + 1)
    best = None
    for w in np.linspace(0.8 * omega_ref, 1.2 * omega_ref, 4001):
        A = np.stack([np.cos(w * t), np.sin(w * t), np.ones_like(t)], axis=1)
        coef, *_ = np.linalg.lstsq(A, series, rcond=None)
        r = np.sum((A @ coef - series) ** 2)
        if best is None or r < best[0]:
            best = (r, w)
    assert abs(best[1] / omega_ref - 1.0) < 2e-3, (best[1], omega_ref, wp * S1)
    assert abs(best[1] / (wp * S1) - 1.0) > 5e-3


def test_omega_p_dt_instability_2d(orc):
    """Above omega_p h S(k1)/2 = 1 the 2-D cold-plasma mode grows; below, it stays bounded."""
    G, a = 32, 0.05
    wp = float(G)
    S1 = math.exp(-0.5 * (2 * math.pi * a) ** 2)
    hs = 2.0 / (wp * S1)
    grow = _dispersion_2d(orc, 1.15 * hs, 25, G=G, a=a)
    stay = _dispersion_2d(orc, 0.85 * hs, 25, G=G, a=a)
    assert np.max(np.abs(grow)) > 50 * abs(grow[0])
    assert np.max(np.abs(stay)) < 3 * np.max(np.abs(stay[:3]))
