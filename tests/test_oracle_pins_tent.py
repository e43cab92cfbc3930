"""Pins of the tent-field oracle (finite-width field shapes Psi, Sections 3
and 4 of the paper, point macroparticles) against facts independent of its
code: hand-integrated closed forms and adaptive quadrature of the tent Gram
integrals, a direct k-space quadrature of the k-squared matrix (no per-axis
factorisation), the defining integral of the particle-mode convolution, the
stationarity of the discrete Lagrangian in the field coefficients, the energy
identity, central-difference gradients, the narrow-tent limit (the periodic
delta-shape method, pinned on its own), symmetries, time reversibility and the
second-order energy error of the leapfrog.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import tent_field as tf

TWO_PI = 2.0 * math.pi


def _neutral(rng, dim, N, half=0.2):
    x = rng.uniform(-half, half, (dim, N))
    q = np.where(np.arange(N) % 2 == 0, 1.0, -1.0)
    return x, q


def _conj_symmetric(rng, n, dim):
    """Random vector over the full cube with v(-sigma) = conj(v(sigma))."""
    m = tf.modes(n, dim)
    v = rng.normal(size=len(m)) + 1j * rng.normal(size=len(m))
    neg = tf.mode_index(-m, n)
    v = 0.5 * (v + np.conj(v[neg]))
    return v


# ---------------------------------------------------------------- Gram integrals
def test_gram_closed_forms():
    """Integrated by hand: int T^2 = 2w/3, int T(u)T(u-w) = w/6, int u^2 T(u-c)^2 =
    (2/3) c^2 w + w^3/15, int u^2 T(u-c) T(u-c-w) = w c^2/6 + w^2 c/6 + w^3/20
    (w = dk: neighbouring tents overlap on one cell), zero beyond neighbours."""
    n, L = 5, 0.8
    dk = TWO_PI / L
    B, A = tf.gram_1d(n, dk)
    for a in range(-n, n + 1):
        c = a * dk
        i = a + n
        assert B[i, i] == pytest.approx(2 * dk / 3, rel=1e-13)
        assert A[i, i] == pytest.approx(2 / 3 * c * c * dk + dk ** 3 / 15, rel=1e-13)
        if a < n:
            assert B[i, i + 1] == pytest.approx(dk / 6, rel=1e-13)
            assert A[i, i + 1] == pytest.approx(dk * c * c / 6 + dk * dk * c / 6 + dk ** 3 / 20, rel=1e-12, abs=1e-12 * dk ** 3)
            assert A[i + 1, i] == A[i, i + 1]
        for b in range(a + 2, n + 1):
            assert B[i, b + n] == 0.0 and A[i, b + n] == 0.0


@pytest.mark.parametrize("wfrac", [1.0, 0.37])
def test_gram_against_adaptive_quadrature(wfrac):
    n, L = 3, 1.3
    dk = TWO_PI / L
    w = wfrac * dk
    B, A = tf.gram_1d(n, dk, w)
    T = lambda u, c: max(0.0, 1.0 - abs(u - c) / w)
    for a, b in [(0, 0), (-3, -3), (2, 3), (-1, 0), (1, -1), (3, 3)]:
        ca, cb = a * dk, b * dk
        lo, hi = min(ca, cb) - w, max(ca, cb) + w
        pts = sorted({ca - w, ca, ca + w, cb - w, cb, cb + w})
        b_ref = integrate.quad(lambda u: T(u, ca) * T(u, cb), lo, hi, points=pts, limit=200, epsabs=1e-14)[0]
        a_ref = integrate.quad(lambda u: u * u * T(u, ca) * T(u, cb), lo, hi, points=pts, limit=200, epsabs=1e-14)[0]
        assert B[a + n, b + n] == pytest.approx(b_ref, rel=1e-10, abs=1e-13)
        assert A[a + n, b + n] == pytest.approx(a_ref, rel=1e-10, abs=1e-12)


# ---------------------------------------------------------------- k-squared matrix
def _psi(k, centre, w):
    return np.prod(np.maximum(0.0, 1.0 - np.abs(k - centre[:, None]) / w), axis=0)


def _k_entry_direct(s, sp_, dk, w):
    """int |k|^2 Psi(k - k_s) Psi(-k - k_s') dk on the tensor grid of the kink
    cells of the overlap box, 3-point Gauss-Legendre per cell and axis (the
    integrand is a polynomial on each cell), without separating the axes."""
    dim = len(s)
    ks, kp = np.array(s) * dk, -np.array(sp_) * dk  # Psi(-k - k_s') = Psi(k + k_s')
    gx = 0.5 + 0.5 * np.array([-math.sqrt(0.6), 0.0, math.sqrt(0.6)])
    gw = 0.5 * np.array([5 / 9, 8 / 9, 5 / 9])
    axes_pts, axes_w = [], []
    for d in range(dim):
        lo, hi = max(ks[d], kp[d]) - w, min(ks[d], kp[d]) + w
        if hi <= lo:
            return 0.0
        knots = np.unique(np.clip(np.array([ks[d] - w, ks[d], ks[d] + w, kp[d] - w, kp[d], kp[d] + w]), lo, hi))
        p = (knots[:-1, None] + np.diff(knots)[:, None] * gx[None, :]).ravel()
        ww = (np.diff(knots)[:, None] * gw[None, :]).ravel()
        axes_pts.append(p)
        axes_w.append(ww)
    grids = np.meshgrid(*axes_pts, indexing="ij")
    wts = np.ones_like(grids[0])
    for d, g in enumerate(np.meshgrid(*axes_w, indexing="ij")):
        wts = wts * g
    k = np.stack([g.ravel() for g in grids])
    f = np.sum(k * k, axis=0) * _psi(k, ks, w) * _psi(k, kp, w)
    return float(np.sum(f * wts.ravel()))


@pytest.mark.parametrize("dim", [2, 3])
def test_k_matrix_entries_against_direct_quadrature(dim):
    n, L = 3, 1.0
    dk = TWO_PI / L
    K = tf.k_matrix(n, L, dim).toarray()
    rng = np.random.default_rng(3)
    pairs = [((0,) * dim, (0,) * dim), ((1,) + (0,) * (dim - 1), (-1,) + (0,) * (dim - 1))]
    for _ in range(12):
        s = rng.integers(-n, n + 1, dim)
        o = rng.integers(-1, 2, dim)
        sp_ = -(s + o)
        if np.all(np.abs(sp_) <= n):
            pairs.append((tuple(s), tuple(sp_)))
    pairs.append(((2,) * dim, (2,) * dim))  # -sigma' two steps away: no overlap
    for s, sp_ in pairs:
        ref = _k_entry_direct(s, sp_, dk, dk)
        got = K[tf.mode_index(np.array(s), n), tf.mode_index(np.array(sp_), n)]
        assert got == pytest.approx(ref, rel=1e-11, abs=1e-9 * dk ** (dim + 2)), (s, sp_)


@pytest.mark.parametrize("dim", [2, 3])
def test_k_matrix_symmetries_and_positivity(dim):
    n, L = 3, 0.9
    K = tf.k_matrix(n, L, dim)
    Kd = K.toarray()
    m = tf.modes(n, dim)
    neg = tf.mode_index(-m, n)
    tol = 1e-13 * np.max(np.abs(Kd))
    assert np.allclose(Kd, Kd.T, rtol=0, atol=tol)
    assert np.allclose(Kd[np.ix_(neg, neg)], Kd, rtol=0, atol=tol)
    assert np.max(np.count_nonzero(Kd, axis=1)) <= 3 ** dim
    rng = np.random.default_rng(4)
    for _ in range(5):
        v = _conj_symmetric(rng, n, dim)
        qf = v @ (K @ v)  # = int |k|^2 |sum v Psi|^2 dk > 0
        assert abs(qf.imag) <= 1e-12 * abs(qf.real) and qf.real > 0


# ---------------------------------------------------------------- basis functions
def test_basis_matches_defining_integral():
    """f_sigma(x) = (2 pi)^(-D/2) int Psi(k - k_sigma) e^{i k.x} dk, per axis by quadrature."""
    n, L = 4, 1.0
    dk = TWO_PI / L
    pts = np.array([[0.0, 0.13, -0.41, 0.9, 2.3], [0.0, -0.07, 0.33, -1.7, 0.05]])
    f = tf.basis(pts, n, L)
    m = tf.modes(n, 2)
    for idx in [0, 7, len(m) // 2, len(m) - 3]:
        s = m[idx]
        for j in range(pts.shape[1]):
            val = 1.0 + 0j
            for d in range(2):
                c, x = s[d] * dk, pts[d, j]
                T = lambda k: max(0.0, 1.0 - abs(k - c) / dk)
                re = integrate.quad(lambda k: T(k) * math.cos(k * x), c - dk, c + dk, points=[c], limit=200, epsabs=1e-14)[0]
                im = integrate.quad(lambda k: T(k) * math.sin(k * x), c - dk, c + dk, points=[c], limit=200, epsabs=1e-13)[0]
                val *= (re + 1j * im) / math.sqrt(TWO_PI)
            assert abs(f[idx, j] - val) <= 1e-11 * max(1.0, abs(val)), (s, j)


def test_deposit_on_listed_modes_matches_full_cube():
    rng = np.random.default_rng(13)
    x, q = _neutral(rng, 3, 50)
    n, L = 3, 1.0
    full = tf.deposit(x, q, n, L)
    m = tf.modes(n, 3)
    pick = rng.choice(len(m), 20, replace=False)
    part = tf.deposit_modes(x, q, L, m[pick], chunk=7)
    assert np.allclose(part, full[pick], rtol=1e-13, atol=1e-13 * np.max(np.abs(full)))


def test_envelope_gradient_central_difference():
    rng = np.random.default_rng(5)
    x = rng.uniform(-0.8, 0.8, (3, 7))
    E, dE = tf.envelope(x, 1.0)
    h = 1e-6
    for d in range(3):
        xp, xm = x.copy(), x.copy()
        xp[d] += h
        xm[d] -= h
        fd = (tf.envelope(xp, 1.0)[0] - tf.envelope(xm, 1.0)[0]) / (2 * h)
        assert np.allclose(dE[d], fd, rtol=1e-7, atol=1e-9)


# ---------------------------------------------------------------- field solve
@pytest.mark.parametrize("dim,n", [(2, 6), (3, 3)])
def test_solution_is_stationary_point_of_the_lagrangian(dim, n):
    """The field part of the discrete Lagrangian, -sum_j q_j phi(x_j) + (eps0/2)
    phi~^T K phi~, changes only at second order, by (eps0/2) d^T K d, when the
    solved phi~ is moved along any real-field direction d."""
    rng = np.random.default_rng(6)
    x, q = _neutral(rng, dim, 9)
    q[0] = 2.0  # net charge: the zero mode is excited too
    eps0, L = 0.7, 1.1
    r = tf.deposit(x, q, n, L)
    ph = tf.solve(r, n, L, dim, eps0)
    K = tf.k_matrix(n, L, dim)
    f = tf.basis(x, n, L)

    def lag(p):
        return float(np.real(-(q @ (f.T @ p)) + 0.5 * eps0 * (p @ (K @ p))))

    base = lag(ph)
    for _ in range(3):
        d = _conj_symmetric(rng, n, dim)
        d *= 1e-3 * np.linalg.norm(ph) / np.linalg.norm(d)
        second = 0.5 * eps0 * float(np.real(d @ (K @ d)))
        assert lag(ph + d) - base == pytest.approx(second, rel=1e-5)
        assert lag(ph - d) - base == pytest.approx(second, rel=1e-5)
    neg = tf.mode_index(-tf.modes(n, dim), n)
    assert np.allclose(ph[neg], np.conj(ph), rtol=0, atol=1e-12 * np.max(np.abs(ph)))


@pytest.mark.parametrize("dim,n", [(2, 5), (3, 3)])
def test_energy_identity(dim, n):
    """(1/2) sum_j q_j Phi_j = (eps0/2) phi~^T K phi~ at the solution."""
    rng = np.random.default_rng(7)
    x, q = _neutral(rng, dim, 8)
    f = tf.fields(x, q, n, 1.0, eps0=1.3)
    assert 0.5 * np.dot(q, f.Phi) == pytest.approx(f.W, rel=1e-11)
    assert f.W > 0


@pytest.mark.parametrize("dim,n", [(2, 5), (3, 3)])
def test_force_is_minus_gradient_of_field_energy(dim, n):
    """F_j = -dW/dx_j by central differences, the field solved again at each
    displaced configuration (the envelope-gradient term included)."""
    rng = np.random.default_rng(8)
    x, q = _neutral(rng, dim, 4, half=0.35)
    L = 1.0
    F = tf.fields(x, q, n, L).F
    h = 1e-6
    for j in range(4):
        for d in range(dim):
            xp, xm = x.copy(), x.copy()
            xp[d, j] += h
            xm[d, j] -= h
            g = (tf.fields(xp, q, n, L).W - tf.fields(xm, q, n, L).W) / (2 * h)
            assert -g == pytest.approx(F[d, j], rel=1e-6, abs=1e-7 * np.max(np.abs(F)))


@pytest.mark.parametrize("dim,n", [(2, 6), (3, 3)])
def test_narrow_tent_limit_is_the_periodic_method(dim, n):
    """Tents of half-width w << dk do not overlap; for a neutral system F and W
    tend to (3/2)^D (w/dk)^D times the periodic delta-shape values on the same
    cube of modes, with an O(w^2) deviation."""
    rng = np.random.default_rng(9)
    x, q = _neutral(rng, dim, 6)
    L = 1.0
    dk = TWO_PI / L
    ref = oracle.fields(np.mod(x, L), q, L, n, "delta", 0.0, 1.0)
    errs = []
    for wf in (1e-2, 1e-3):
        f = tf.fields(x, q, n, L, w=wf * dk)
        sc = 1.5 ** dim * wf ** dim
        eF = np.max(np.abs(f.F / sc - ref.F)) / np.max(np.abs(ref.F))
        eW = abs(f.W / sc - ref.W) / abs(ref.W)
        errs.append(max(eF, eW))
    assert errs[1] <= 1e-5
    assert errs[0] / errs[1] == pytest.approx(100.0, rel=0.05)  # second order in w


# ---------------------------------------------------------------- symmetries
def test_symmetries_and_self_force():
    L, n = 1.0, 4
    # a lone charge at the centre: no force; away from it: a force of its own
    # (translations are not a symmetry, so momentum is not conserved)
    for dim in (2, 3):
        f0 = tf.fields(np.zeros((dim, 1)), np.array([1.0]), n, L)
        assert np.max(np.abs(f0.F)) <= 1e-12
        x1 = np.zeros((dim, 1))
        x1[0] = 0.17
        f1 = tf.fields(x1, np.array([1.0]), n, L)
        assert abs(f1.F[0, 0]) > 1e-3 and np.max(np.abs(f1.F[1:])) <= 1e-12
    # mirror pair about the centre: equal and opposite forces
    x = np.array([[0.11, -0.11], [0.05, -0.05], [-0.2, 0.2]])
    f = tf.fields(x, np.array([1.0, 1.0]), n, L)
    assert np.allclose(f.F[:, 0], -f.F[:, 1], rtol=1e-12, atol=1e-13)
    # reality: the complex sums have no imaginary part (Section 4: the total
    # momentum change is real for even shapes and paired modes)
    rng = np.random.default_rng(10)
    xs, q = _neutral(rng, 3, 7)
    fr = tf.fields(xs, q, n, L)
    Fc = tf.force(xs, q, n, L, fr.phi_t, complex_out=True)
    Pc = tf.potential(xs, n, L, fr.phi_t, complex_out=True)
    assert np.max(np.abs(Fc.imag)) <= 1e-12 * np.max(np.abs(Fc.real))
    assert np.max(np.abs(Pc.imag)) <= 1e-12 * np.max(np.abs(Pc.real))


# ---------------------------------------------------------------- time steps
def _state(dim, n, seed):
    rng = np.random.default_rng(seed)
    x, q = _neutral(rng, dim, 4)
    v = rng.normal(scale=0.05, size=(dim, 4))
    return tf.State(x, v, q, np.full(4, 1.0), n, 1.0)


@pytest.mark.parametrize("stepper", ["kdk", "dkd"])
def test_steps_are_reversible(stepper):
    step = tf.step_kdk if stepper == "kdk" else tf.step_dkd
    s = _state(2, 4, 11)
    x0, v0 = s.x.copy(), s.v.copy()
    s = step(s, 2e-3, 20)
    s.v = -s.v
    s.F = None
    s = step(s, 2e-3, 20)
    assert np.allclose(s.x, x0, rtol=0, atol=1e-11)
    assert np.allclose(-s.v, v0, rtol=0, atol=1e-10)


@pytest.mark.parametrize("stepper", ["kdk", "dkd"])
def test_energy_error_is_second_order(stepper):
    step = tf.step_kdk if stepper == "kdk" else tf.step_dkd
    errs = []
    for h in (4e-3, 2e-3):
        s = _state(2, 4, 12)
        e0 = tf.energy(s)["total"]
        emax = 0.0
        for _ in range(int(round(0.16 / h))):
            s = step(s, h)
            emax = max(emax, abs(tf.energy(s)["total"] - e0))
        errs.append(emax)
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.15)
