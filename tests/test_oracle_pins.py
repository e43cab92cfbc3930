"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics
independent of the oracle's code: a library FFT, the Ewald summation identity,
the rock-salt Madelung constant, numerical quadrature of the particle shapes,
central-difference gradients, conservation laws and the cold-plasma discrete
dispersion relation derived in the paper's Section 5.

Each pin is chosen so that a plausible slip in the oracle (a dropped factor 2,
a wrong sign or power of S, a swapped axis, a wrong volume or eps0 factor, a
kick with the wrong weight) fails at least one of them.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import workloads


# ---------------------------------------------------------------- mode set
@pytest.mark.parametrize("n_max", [1, 2, 5, 8])
def test_half_space_partitions_cube(orc, n_max):
    """|H| = (M^3 - 1)/2, H and -H are disjoint, and H u -H u {0} is the cube."""
    H = orc.half_modes(n_max)
    M = 2 * n_max + 1
    assert len(H) == (M ** 3 - 1) // 2
    s = {tuple(v) for v in H.tolist()}
    neg = {(-a, -b, -c) for a, b, c in s}
    assert len(s) == len(H) and not (s & neg)
    cube = {(a, b, c) for a in range(-n_max, n_max + 1) for b in range(-n_max, n_max + 1)
            for c in range(-n_max, n_max + 1)}
    assert s | neg | {(0, 0, 0)} == cube
    # canonical order: lexicographic in (n_x, n_y, n_z) with n_x from 0
    assert sorted(s) == [tuple(v) for v in H.tolist()]


# ---------------------------------------------------------------- shapes
def test_shape_transforms_match_quadrature(orc):
    """S(k) is the Fourier transform of the real-space particle shape, computed here
    by numerical quadrature of a 3D Gaussian density and of a tensor tent."""
    a = 0.07
    for k in ([3.0, 0.0, 0.0], [10.0, -20.0, 5.0], [40.0, 33.0, -12.0]):
        g1 = lambda kd: integrate.quad(lambda x: math.exp(-x * x / (2 * a * a)) / math.sqrt(2 * math.pi * a * a)
                                       * math.cos(kd * x), -12 * a, 12 * a, limit=200)[0]
        t1 = lambda kd: integrate.quad(lambda x: (1.0 - abs(x) / a) / a * math.cos(kd * x), -a, a,
                                       points=[0.0], limit=200)[0]
        sg = np.prod([g1(kd) for kd in k])
        st = np.prod([t1(kd) for kd in k])
        assert abs(orc.shape("gaussian", a, np.array(k))[0] - sg) < 1e-12
        assert abs(orc.shape("tent", a, np.array(k))[0] - st) < 1e-12
        assert orc.shape("delta", a, np.array(k))[0] == 1.0


# ---------------------------------------------------------------- deposit
@pytest.mark.parametrize("L", [1.0, 2.7])
def test_deposit_on_grid_equals_fft(orc, L):
    """Particles exactly on a G^3 grid: rho_n = FFT(q)[n mod G] (delta shape)."""
    G, n_max = 8, 3
    p = workloads.grid_particles(G, L=L)
    modes = orc.cube_modes(n_max)
    rho = orc.deposit(p.positions(), p.q, L, modes, "delta")
    Q = np.fft.fftn(p.q.reshape(G, G, G))
    ref = Q[modes[:, 0] % G, modes[:, 1] % G, modes[:, 2] % G]
    assert np.max(np.abs(rho - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_deposit_conjugate_symmetry(orc):
    """rho_{-n} = conj(rho_n) over the full cube."""
    p = workloads.random_particles(40, L=1.3, charge="uniform")
    n_max = 4
    modes = orc.cube_modes(n_max)
    rho = orc.deposit(p.positions(), p.q, 1.3, modes, "gaussian", 0.05)
    idx = {tuple(v): i for i, v in enumerate(modes.tolist())}
    neg = np.array([idx[(-a, -b, -c)] for a, b, c in modes.tolist()])
    assert np.max(np.abs(rho[neg] - np.conj(rho))) <= 1e-14 * np.max(np.abs(rho))


def test_deposit_translation(orc):
    """Shifting every particle by d multiplies rho_n by exp(-i k_n . d); shifting
    one particle by a box length changes nothing."""
    L = 1.0
    p = workloads.random_particles(30, L=L, charge="uniform")
    modes = orc.half_modes(4)
    pos = p.positions()
    rho = orc.deposit(pos, p.q, L, modes, "gaussian", 0.04)
    d = np.array([0.123, -0.377, 0.051])
    rho_d = orc.deposit(pos + d[:, None], p.q, L, modes, "gaussian", 0.04)
    k = orc.wave_vectors(modes, L)
    assert np.max(np.abs(rho_d - rho * np.exp(-1j * k @ d))) <= 1e-13 * np.max(np.abs(rho))
    pos2 = pos.copy()
    pos2[1, 7] += L
    pos2[2, 3] -= L
    assert np.max(np.abs(orc.deposit(pos2, p.q, L, modes, "gaussian", 0.04) - rho)) <= 1e-13 * np.max(np.abs(rho))


def test_single_particle_deposit(orc):
    """One particle: |rho_n| = |q| S(k_n) for every mode."""
    modes = orc.half_modes(5)
    rho = orc.deposit(np.array([[0.31], [0.77], [0.05]]), [-1.5], 1.0, modes, "delta")
    assert np.max(np.abs(np.abs(rho) - 1.5)) < 1e-13


# ---------------------------------------------------------------- Ewald / Madelung
def _ewald_real_space(pos, q, L, alpha, images=2):
    """Real-space Ewald energy and forces (eps0 = 1): sum over pairs and periodic
    images of q_i q_j erfc(alpha r) / (4 pi r), minus the Gaussian self-energy
    alpha/sqrt(pi) * sum q^2 / (4 pi)."""
    N = pos.shape[1]
    E = 0.0
    F = np.zeros_like(pos)
    rng = range(-images, images + 1)
    shifts = np.array([[a, b, c] for a in rng for b in rng for c in rng], dtype=float) * L
    for i in range(N):
        for j in range(N):
            r = pos[:, i][None, :] - pos[:, j][None, :] + shifts
            d = np.linalg.norm(r, axis=1)
            if i == j:
                keep = d > 0
                r, d = r[keep], d[keep]
            e = special.erfc(alpha * d) / d
            E += 0.5 * q[i] * q[j] * np.sum(e) / (4 * np.pi)
            g = (e + 2 * alpha / np.sqrt(np.pi) * np.exp(-(alpha * d) ** 2)) / d ** 2
            F[:, i] += q[i] * q[j] * np.sum(g[:, None] * r, axis=0) / (4 * np.pi)
    E -= alpha / np.sqrt(np.pi) * np.sum(q ** 2) / (4 * np.pi)
    return E, F


def _coulomb_total(orc, pos, q, L, a, n_max):
    """Total periodic Coulomb energy and force = spectral part (Gaussian shape of
    width a, whose squared transform is the Ewald screening exp(-k^2/(4 alpha^2))
    with alpha = 1/(2a)) + real-space remainder."""
    f = orc.fields(pos, q, L, n_max, "gaussian", a, 1.0)
    Er, Fr = _ewald_real_space(pos, q, L, 1.0 / (2.0 * a))
    return f.W + Er, f.F + Fr


@pytest.mark.parametrize("L", [1.0, 1.6])
def test_ewald_alpha_independence(orc, L):
    """The Ewald split is exact: field energy W and force F of the spectral method
    plus the real-space erfc sums must not depend on the Gaussian width a.  Pins
    the 1/V and eps0 factors, the factor 2 of the half-space sum, the S^2 placement
    and the sign of the force."""
    pos = L * np.array([[0.11, 0.52, 0.83, 0.40], [0.20, 0.75, 0.33, 0.91], [0.64, 0.08, 0.47, 0.29]])
    q = np.array([1.0, -2.0, 0.5, 0.5])
    E1, F1 = _coulomb_total(orc, pos, q, L, 0.06 * L, 17)
    E2, F2 = _coulomb_total(orc, pos, q, L, 0.09 * L, 12)
    # and the absolute value scales as 1/L (Coulomb energy of a scaled configuration)
    if L != 1.0:
        E_unit, _ = _coulomb_total(orc, pos / L, q, 1.0, 0.06, 17)
        assert abs(E1 * L - E_unit) < 1e-11 * abs(E_unit)
    assert abs(E1 - E2) < 1e-11 * abs(E1)
    assert np.max(np.abs(F1 - F2)) < 1e-10 * np.max(np.abs(F1))


@pytest.mark.parametrize("L", [1.0, 2.5])
def test_rock_salt_madelung(orc, L):
    """Eight ions of a rock-salt cell in the periodic box: total Coulomb energy is
    -4 M q^2 / (4 pi eps0 r0) with nearest-neighbour distance r0 = L/2 and the
    rock-salt Madelung constant M = 1.747564594633182 (standard value)."""
    M = 1.747564594633182
    p = workloads.rock_salt(L)
    E, F = _coulomb_total(orc, p.positions(), p.q, L, 0.05 * L, 20)
    ref = -4.0 * M / (4.0 * np.pi * 0.5 * L)
    assert abs(E - ref) < 1e-12
    assert np.max(np.abs(F)) < 1e-11  # every ion sits at a centre of inversion symmetry


# ---------------------------------------------------------------- force
def test_lone_particle_has_no_self_force(orc):
    """A single particle feels no force from its own field (Section 4, delta field shape)."""
    L, n_max, a = 1.0, 6, 0.03
    modes = orc.half_modes(n_max)
    k = orc.wave_vectors(modes, L)
    S = orc.shape("gaussian", a, k)
    scale = np.sum(2 * np.linalg.norm(k, axis=1) * S * S / np.sum(k * k, axis=1) / L ** 3)
    for pos in ([0.3, 0.2, 0.9], [0.0, 0.0, 0.0], [0.999999, 0.5, 0.123456789]):
        f = orc.fields(np.array(pos)[:, None], [1.7], L, n_max, "gaussian", a)
        assert np.max(np.abs(f.F)) <= 1e-14 * 1.7 ** 2 * scale


def test_pair_forces_cancel_and_opposite_charges_attract(orc):
    """Newton's third law for the delta field shape (Section 4): total force zero,
    two-body forces equal and opposite; opposite charges attract, like repel."""
    p = workloads.random_particles(50, L=1.0, charge="uniform")
    f = orc.fields(p.positions(), p.q, 1.0, 4, "gaussian", 0.05)
    assert np.max(np.abs(f.F.sum(axis=1))) <= 1e-13 * np.sum(np.abs(f.F))
    pos = np.array([[0.45, 0.55], [0.5, 0.5], [0.5, 0.5]])
    for q, sign in (([1.0, -1.0], +1), ([1.0, 1.0], -1)):
        F = orc.fields(pos, q, 1.0, 8, "gaussian", 0.03).F
        assert np.max(np.abs(F[:, 0] + F[:, 1])) < 1e-14 * np.abs(F[0, 0])
        assert np.sign(F[0, 0]) == sign and abs(F[1, 0]) < 1e-14 * np.abs(F[0, 0])


def test_force_is_minus_energy_gradient(orc):
    """F_j = -dW/dx_j by central differences."""
    L, n_max, a = 1.5, 4, 0.06
    p = workloads.random_particles(12, L=L, charge="uniform")
    pos = p.positions()
    modes = orc.half_modes(n_max)
    F = orc.fields(pos, p.q, L, n_max, "gaussian", a, modes=modes).F
    d = 1e-6 * L
    for j in (0, 5, 11):
        for c in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[c, j] += d
            pm[c, j] -= d
            Wp = orc.field_energy(orc.deposit(pp, p.q, L, modes, "gaussian", a), L, modes)
            Wm = orc.field_energy(orc.deposit(pm, p.q, L, modes, "gaussian", a), L, modes)
            assert abs(-(Wp - Wm) / (2 * d) - F[c, j]) < 1e-7 * np.max(np.abs(F))


def test_potential_adjoint_to_deposit(orc):
    """sum_j q_j Phi_j = 2 W, and for any psi: sum_j q_j Phi_j(psi) = 2 Re sum_H psi conj(rho)
    with rho deposited without shape factor."""
    L, n_max = 1.0, 5
    p = workloads.random_particles(25, L=L, charge="uniform")
    pos = p.positions()
    modes = orc.half_modes(n_max)
    f = orc.fields(pos, p.q, L, n_max, "gaussian", 0.05, modes=modes)
    U = np.sum(p.q * orc.potential_from_psi(pos, L, modes, f.psi))
    assert abs(U - 2 * f.W) < 1e-13 * abs(U)
    rng = np.random.default_rng(7)
    c = rng.normal(size=len(modes)) + 1j * rng.normal(size=len(modes))
    lhs = np.sum(p.q * orc.potential_from_psi(pos, L, modes, c))
    rho = orc.deposit(pos, p.q, L, modes, "delta")
    assert abs(lhs - 2 * np.real(np.sum(c * np.conj(rho)))) < 1e-12 * np.sum(np.abs(c) * np.abs(rho))


# ---------------------------------------------------------------- time step
def test_two_body_energy_bounded_and_momentum_conserved(orc):
    """Two-body run (2000 kick-drift-kick steps): energy stays bounded with no
    secular trend (Section 6) and total momentum stays zero to roundoff."""
    p = workloads.two_body()
    s = orc.State.from_particles(p)
    E0 = orc.energy(s)["total"]
    Es, Ps = [], []
    for _ in range(40):
        orc.step_kdk(s, p.dt, 50)
        e = orc.energy(s)
        Es.append(e["total"] - E0)
        Ps.append(np.max(np.abs(e["momentum"])) / e["momentum_abs_sum"])
    Es = np.array(Es)
    assert np.max(np.abs(Es)) < 1e-4 * abs(E0)
    slope = np.polyfit(np.arange(len(Es)), Es, 1)[0] * len(Es)
    assert abs(slope) < 0.5 * np.max(np.abs(Es))
    assert max(Ps) < 1e-12


@pytest.mark.parametrize("scheme", ["kdk", "dkd"])
def test_time_reversibility(orc, scheme):
    """n steps, velocity reversal, n steps returns to the start (symmetric leapfrog)."""
    p = workloads.two_body()
    s = orc.State.from_particles(p)
    x0, v0 = s.pos.copy(), s.vel.copy()
    step = orc.step_kdk if scheme == "kdk" else orc.step_dkd
    step(s, p.dt, 500)
    s.vel = -s.vel
    step(s, p.dt, 500)
    assert np.max(np.abs(s.pos - x0)) < 1e-11
    assert np.max(np.abs(s.vel + v0)) < 1e-11


def test_energy_error_scales_as_h_squared(orc):
    """Second-order accuracy (Section 6): the maximum energy deviation over a fixed
    time falls as h^2."""
    errs = []
    hs = [4e-3, 2e-3, 1e-3, 5e-4]
    for h in hs:
        p = workloads.two_body(dt=h)
        s = orc.State.from_particles(p)
        E0 = orc.energy(s)["total"]
        dev = 0.0
        for _ in range(int(round(1.0 / h))):
            orc.step_kdk(s, h, 1)
            dev = max(dev, abs(orc.energy(s)["total"] - E0))
        errs.append(dev)
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert 1.85 < slope < 2.15, (slope, errs)


def _dispersion_run(orc, scheme, h, n_steps, a=0.05, G=16, n_max=4, amp=0.01, L=1.0, eps0=1.0):
    p = workloads.cold_lattice(G, G, G, n_max=n_max, a=a, amplitude=amp, jitter=0.0, dt=h, L=L)
    p = p.with_(eps0=eps0)
    s = orc.State.from_particles(p)
    k1 = np.array([[1, 0, 0]], dtype=np.int32)
    series = []
    step = orc.step_kdk if scheme == "kdk" else orc.step_dkd
    for _ in range(n_steps):
        step(s, h, 1)
        series.append(orc.deposit(s.pos, s.q, s.L, k1, "gaussian", a)[0].real)
    wp = math.sqrt(p.N * 1.0 / (eps0 * p.L ** 3))  # n q^2 / (eps0 m), q = -1, m = 1
    S1 = math.exp(-0.5 * (2 * math.pi * a / L) ** 2)
    return np.array(series), wp, S1


@pytest.mark.parametrize("scheme,L,eps0", [("kdk", 1.0, 1.0), ("dkd", 1.0, 1.0), ("kdk", 0.8, 0.5)])
def test_cold_plasma_dispersion(orc, scheme, L, eps0):
    """Cold plasma: the k1 = (1,0,0) density mode oscillates at
    omega = (2/h) asin(omega_p h S(k1) / 2), the paper's cold-plasma discrete
    dispersion relation (Section 5) with the shape-modified plasma frequency
    omega_p S(k1)."""
    G, a = 16, 0.05 * L
    wp = math.sqrt(G ** 3 / (eps0 * L ** 3))
    h = 0.5 / wp
    series, wp, S1 = _dispersion_run(orc, scheme, h, 60, a=a, G=G, L=L, eps0=eps0)
    omega_ref = (2.0 / h) * math.asin(wp * h * S1 / 2.0)
    t = h * np.arange(1, len(series) + 1)
    best = None
    for w in np.linspace(0.8 * omega_ref, 1.2 * omega_ref, 4001):
        A = np.stack([np.cos(w * t), np.sin(w * t), np.ones_like(t)], axis=1)
        coef, res, *_ = np.linalg.lstsq(A, series, rcond=None)
        r = np.sum((A @ coef - series) ** 2)
        if best is None or r < best[0]:
            best = (r, w)
    assert abs(best[1] / omega_ref - 1.0) < 2e-3, (best[1], omega_ref, wp * S1)
    # and it is not the continuum frequency omega_p S, nor omega_p
    assert abs(best[1] / (wp * S1) - 1.0) > 5e-3


def test_omega_p_dt_instability(orc):
    """Above the omega_p-dt limit omega_p h S(k1)/2 > 1 the cold-plasma mode grows
    exponentially (Section 5); just below it, it stays bounded."""
    G, a = 16, 0.05
    wp = math.sqrt(G ** 3)
    S1 = math.exp(-0.5 * (2 * math.pi * a) ** 2)
    hs = 2.0 / (wp * S1)
    grow, _, _ = _dispersion_run(orc, "kdk", 1.15 * hs, 25, a=a, G=G)
    stay, _, _ = _dispersion_run(orc, "kdk", 0.85 * hs, 25, a=a, G=G)
    assert np.max(np.abs(grow)) > 50 * abs(grow[0])
    assert np.max(np.abs(stay)) < 3 * np.max(np.abs(stay[:3]))
