"""FP64 CPU oracle for the finite-width field shapes of Webb, "A Spectral
Canonical Electrostatic Algorithm" (arXiv:1508.07344), Sections 3 and 4:
tent functions Psi in k-space, point macroparticles.

TEST INFRASTRUCTURE ONLY, under the same rule as the rest of ``oracle``: only
``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg may
import it; it imports nothing from the HIP library.

What is computed (Section 3, the potential expansion and the k-squared matrix;
Section 4, the discrete Euler-Lagrange equations):

* Modes sigma range over the full cube {-n..n}^D, sigma = 0 included, with
  k_sigma = dk sigma and dk = 2 pi / L.  Each mode is spread over k-space by
  Psi(k - k_sigma) = prod_d T(k_d - k_sigma,d), T(u) = max(0, 1 - |u| / dk):
  neighbouring tents overlap, and the field lives on all of R^D (no periodic
  box).
* Point particles, Lambda = delta, so Lambda~ = (2 pi)^(-D/2) and the
  particle-mode convolution f_sigma(x) = int dk Lambda~*(k) Psi(k - k_sigma)
  e^{i k.x} has the closed form f_sigma(x) = e^{i k_sigma.x} E(x) with the
  envelope E(x) = prod_d (2 pi)^(-1/2) dk sinc^2(dk x_d / 2),
  sinc(u) = sin(u) / u.  It is also the basis function of the potential,
  phi(x) = sum_sigma phi~_sigma f_sigma(x).
* K_{sigma sigma'} = int dk |k|^2 Psi(k - k_sigma) Psi(-k - k_sigma'), which
  separates per axis into the 1-D integrals of ``gram_1d``.
* Field equation (stationarity of the discrete Lagrangian in phi~, with the
  field term (eps0 / 2) int |grad phi|^2):
      eps0 sum_sigma' K_{sigma sigma'} phi~_sigma' = r_sigma,
      r_sigma = sum_j q_j f_sigma(x_j).
  In Gaussian units (eps0 = 1 / (4 pi)) the factor in front of the charge sum
  is 4 pi; the printed 8 pi does not follow from differentiating the
  quadratic field term and is read as a slip.
* Force F_j = -q_j sum_sigma phi~_sigma grad f_sigma(x_j), with
  grad f_sigma = e^{i k_sigma.x} (i k_sigma E + grad E); potential at a
  particle Phi_j = sum_sigma phi~_sigma f_sigma(x_j); field energy
  W = (eps0 / 2) phi~^T K phi~ = (1/2) sum_j q_j Phi_j.
* Steps: the same KDK and DKD leapfrogs as the periodic method, with no wrap.

The paper drops this variant because it breaks exact momentum conservation;
a lone particle away from the origin feels a force of its own.

Every function takes an optional tent half-width w in (0, dk] (default dk,
the paper's tents); narrow tents only serve a pin: as w -> 0 a neutral
system's F and W tend to those of the periodic delta-shape method on the same
cube of modes, times (3/2)^D (w / dk)^D.

Pins: ``tests/test_oracle_pins_tent.py`` (Gram integrals against adaptive
quadrature and closed forms, the K entries against a direct k-space
quadrature, f_sigma against its defining integral, stationarity of the
Lagrangian, the energy identity, F = -grad W, the narrow-tent limit,
symmetries, reversibility and the h^2 energy error of the steps).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

TWO_PI = 2.0 * np.pi


def modes(n: int, dim: int = 3) -> np.ndarray:
    """Full cube {-n..n}^dim, sigma = 0 included, last axis fastest: [M^dim, dim]."""
    axes = np.meshgrid(*([np.arange(-n, n + 1)] * dim), indexing="ij")
    return np.stack([a.ravel() for a in axes], axis=1).astype(np.int64)


def mode_index(sig: np.ndarray, n: int) -> np.ndarray:
    """Row of ``modes(n, dim)`` holding each sigma (sig [..., dim])."""
    sig = np.asarray(sig, dtype=np.int64)
    M = 2 * n + 1
    idx = np.zeros(sig.shape[:-1], dtype=np.int64)
    for d in range(sig.shape[-1]):
        idx = idx * M + (sig[..., d] + n)
    return idx


def tent(u, w: float):
    """T(u) = max(0, 1 - |u| / w): half-width w (the paper's tents: w = dk)."""
    return np.maximum(0.0, 1.0 - np.abs(u) / w)


def _width(L: float, w):
    dk = TWO_PI / L
    w = dk if w is None else float(w)
    if not (0.0 < w <= dk):
        raise ValueError("tent half-width must lie in (0, dk]")
    return dk, w


# 3-point Gauss-Legendre on [0, 1]: exact for polynomials of degree <= 5
_GL_X = 0.5 + 0.5 * np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])
_GL_W = 0.5 * np.array([5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0])


def gram_1d(n: int, dk: float, w: float | None = None):
    """B[a, b] = int T(u - a dk) T(u - b dk) du and A[a, b] = int u^2 T(u - a dk)
    T(u - b dk) du for a, b in -n..n (array index a + n), tents of half-width
    w (default dk).  Between consecutive kinks a dk + {-w, 0, w} each
    integrand is a polynomial of degree <= 4, so cellwise 3-point
    Gauss-Legendre sums are exact."""
    w = dk if w is None else w
    centres = np.arange(-n, n + 1) * dk
    knots = np.unique(np.concatenate([centres - w, centres, centres + w]))
    lo, width = knots[:-1], np.diff(knots)
    u = (lo[:, None] + width[:, None] * _GL_X[None, :]).ravel()
    wt = (width[:, None] * _GL_W[None, :]).ravel()
    T = tent(u[None, :] - centres[:, None], w)  # [M, points]
    B = (T * wt) @ T.T
    A = (T * (wt * u * u)) @ T.T
    return B, A


def k_matrix(n: int, L: float, dim: int = 3, w: float | None = None) -> sp.csr_matrix:
    """K_{sigma sigma'} over ``modes(n, dim)``.  Psi(-k - k_sigma') = Psi(k +
    k_sigma') (Psi is even), and |k|^2 = sum_d k_d^2, so each entry is
    sum_d A(sigma_d, -sigma'_d) prod_{e != d} B(sigma_e, -sigma'_e); it is
    non-zero only when -sigma' is within one step of sigma on every axis
    (w <= dk)."""
    dk, w = _width(L, w)
    B, A = gram_1d(n, dk, w)
    sig = modes(n, dim)
    rows, cols, vals = [], [], []
    offsets = modes(1, dim)  # -sigma' = sigma + o, o in {-1, 0, 1}^dim
    for o in offsets:
        t = sig + o[None, :]  # t = -sigma'
        ok = np.all(np.abs(t) <= n, axis=1)
        s, t = sig[ok], t[ok]
        ia, ib = s + n, t + n
        v = np.zeros(len(s))
        for d in range(dim):
            term = A[ia[:, d], ib[:, d]].copy()
            for e in range(dim):
                if e != d:
                    term *= B[ia[:, e], ib[:, e]]
            v += term
        rows.append(mode_index(s, n))
        cols.append(mode_index(-t, n))
        vals.append(v)
    Msz = (2 * n + 1) ** dim
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(Msz, Msz))


def envelope(pos, L: float, w: float | None = None):
    """E(x) = prod_d (2 pi)^(-1/2) w sinc^2(w x_d / 2) (w = dk by default)
    and its gradient: (E [N], dE [dim, N])."""
    x = np.atleast_2d(np.asarray(pos, dtype=np.float64))
    dk, w = _width(L, w)
    u = 0.5 * w * x
    # d/dx sinc^2(u) = 2 sinc(u) sinc'(u) du/dx, sinc'(u) = (cos u - sinc u) / u.
    # For |u| < 0.1 that difference cancels; there both come from the series
    # sinc(u) = sum_k (-u^2)^k / (2k+1)!, k <= 6.
    small = np.abs(u) < 0.1
    us = np.where(small, 1.0, u)
    s = np.where(small, 0.0, np.sin(us) / us)
    ds = np.where(small, 0.0, (np.cos(us) - np.sin(us) / us) / us)
    s_ser = np.zeros_like(u)
    ds_ser = np.zeros_like(u)
    for k in range(7):
        c = (-1.0) ** k / math.factorial(2 * k + 1)
        s_ser += c * u ** (2 * k)
        if k > 0:
            ds_ser += c * 2 * k * u ** (2 * k - 1)
    s = np.where(small, s_ser, s)
    ds = np.where(small, ds_ser, ds)
    e = w / np.sqrt(TWO_PI) * s * s
    de = w / np.sqrt(TWO_PI) * 2.0 * s * ds * 0.5 * w
    E = np.prod(e, axis=0)
    dE = np.empty_like(x)
    for d in range(x.shape[0]):
        others = np.prod(np.delete(e, d, axis=0), axis=0) if x.shape[0] > 1 else 1.0
        dE[d] = de[d] * others
    return E, dE


def basis(pos, n: int, L: float, w: float | None = None) -> np.ndarray:
    """f_sigma(x_j) = e^{i k_sigma.x_j} E(x_j): [M^dim, N] complex."""
    x = np.atleast_2d(np.asarray(pos, dtype=np.float64))
    k = modes(n, x.shape[0]) * (TWO_PI / L)
    E, _ = envelope(x, L, w)
    return np.exp(1j * (k @ x)) * E[None, :]


def deposit(pos, q, n: int, L: float, w: float | None = None, chunk: int = 2048) -> np.ndarray:
    """r_sigma = sum_j q_j f_sigma(x_j) over the full cube."""
    x = np.atleast_2d(np.asarray(pos, dtype=np.float64))
    q = np.asarray(q, dtype=np.float64)
    r = np.zeros((2 * n + 1) ** x.shape[0], dtype=np.complex128)
    for j0 in range(0, x.shape[1], chunk):
        r += basis(x[:, j0:j0 + chunk], n, L, w) @ q[j0:j0 + chunk]
    return r


def deposit_modes(pos, q, L: float, sig: np.ndarray, w: float | None = None,
                  chunk: int = 65536) -> np.ndarray:
    """r_sigma for the listed modes only (sig [K, dim]), same sum as ``deposit``."""
    x = np.atleast_2d(np.asarray(pos, dtype=np.float64))
    q = np.asarray(q, dtype=np.float64)
    k = np.asarray(sig, dtype=np.float64) * (TWO_PI / L)
    r = np.zeros(len(k), dtype=np.complex128)
    for j0 in range(0, x.shape[1], chunk):
        xs = x[:, j0:j0 + chunk]
        E, _ = envelope(xs, L, w)
        r += np.exp(1j * (k @ xs)) @ (q[j0:j0 + chunk] * E)
    return r


def solve(r: np.ndarray, n: int, L: float, dim: int = 3, eps0: float = 1.0,
          w: float | None = None) -> np.ndarray:
    """phi~ from eps0 K phi~ = r (sparse direct solve)."""
    K = (eps0 * k_matrix(n, L, dim, w)).tocsc().astype(np.complex128)
    return spla.spsolve(K, r)


def _sums(pos, n: int, L: float, phi_t: np.ndarray, chunk: int = 2048):
    """P_j = sum phi~ e^{ik.x}, G_j = sum phi~ (i k) e^{ik.x}, complex."""
    x = np.atleast_2d(np.asarray(pos, dtype=np.float64))
    k = modes(n, x.shape[0]) * (TWO_PI / L)
    P = np.zeros(x.shape[1], dtype=np.complex128)
    G = np.zeros(x.shape, dtype=np.complex128)
    for j0 in range(0, x.shape[1], chunk):
        e = np.exp(1j * (k @ x[:, j0:j0 + chunk])) * phi_t[:, None]
        P[j0:j0 + chunk] = e.sum(axis=0)
        G[:, j0:j0 + chunk] = (1j * k.T) @ e
    return P, G


def potential(pos, n: int, L: float, phi_t: np.ndarray, complex_out: bool = False,
              w: float | None = None):
    """Phi_j = sum_sigma phi~_sigma f_sigma(x_j) (real for a real field)."""
    E, _ = envelope(pos, L, w)
    P, _ = _sums(pos, n, L, phi_t)
    out = E * P
    return out if complex_out else out.real


def force(pos, q, n: int, L: float, phi_t: np.ndarray, complex_out: bool = False,
          w: float | None = None):
    """F_j = -q_j sum_sigma phi~_sigma e^{i k_sigma.x_j} (i k_sigma E + grad E)."""
    q = np.asarray(q, dtype=np.float64)
    E, dE = envelope(pos, L, w)
    P, G = _sums(pos, n, L, phi_t)
    F = -q[None, :] * (G * E[None, :] + dE * P[None, :])
    return F if complex_out else F.real


def field_energy(phi_t: np.ndarray, n: int, L: float, dim: int = 3, eps0: float = 1.0,
                 w: float | None = None) -> float:
    """W = (eps0 / 2) sum_{sigma sigma'} phi~_sigma K_{sigma sigma'} phi~_sigma'."""
    K = k_matrix(n, L, dim, w)
    return float(np.real(0.5 * eps0 * phi_t @ (K @ phi_t)))


@dataclasses.dataclass
class Fields:
    r: np.ndarray       # full cube, modes(n, dim) order
    phi_t: np.ndarray   # full cube
    F: np.ndarray       # [dim, N]
    Phi: np.ndarray     # [N]
    W: float


def fields(pos, q, n: int, L: float, eps0: float = 1.0, w: float | None = None) -> Fields:
    x = np.atleast_2d(np.asarray(pos, dtype=np.float64))
    dim = x.shape[0]
    r = deposit(x, q, n, L, w)
    ph = solve(r, n, L, dim, eps0, w)
    return Fields(r, ph, force(x, q, n, L, ph, w=w), potential(x, n, L, ph, w=w),
                  field_energy(ph, n, L, dim, eps0, w))


@dataclasses.dataclass
class State:
    x: np.ndarray
    v: np.ndarray
    q: np.ndarray
    m: np.ndarray
    n: int
    L: float
    eps0: float = 1.0
    F: np.ndarray | None = None

    def copy(self) -> "State":
        return State(self.x.copy(), self.v.copy(), self.q.copy(), self.m.copy(), self.n, self.L,
                     self.eps0, None if self.F is None else self.F.copy())


def _force(s: State) -> np.ndarray:
    return fields(s.x, s.q, s.n, s.L, s.eps0).F


def step_kdk(s: State, h: float, n_steps: int = 1) -> State:
    """Half kick, drift h, field solve + force at the new positions, half kick
    (the end-of-step force is reused); positions are not wrapped."""
    for _ in range(n_steps):
        if s.F is None:
            s.F = _force(s)
        s.v = s.v + 0.5 * h * s.F / s.m[None, :]
        s.x = s.x + h * s.v
        s.F = _force(s)
        s.v = s.v + 0.5 * h * s.F / s.m[None, :]
    return s


def step_dkd(s: State, h: float, n_steps: int = 1) -> State:
    """Section 4's velocity form: drift h/2, solve + kick h, drift h/2."""
    for _ in range(n_steps):
        s.x = s.x + 0.5 * h * s.v
        s.F = _force(s)
        s.v = s.v + h * s.F / s.m[None, :]
        s.x = s.x + 0.5 * h * s.v
        s.F = None
    return s


def energy(s: State) -> dict:
    f = fields(s.x, s.q, s.n, s.L, s.eps0)
    K = 0.5 * float(np.sum(s.m[None, :] * s.v * s.v))
    return {"kinetic": K, "field": f.W, "total": K + f.W,
            "momentum": np.sum(s.m[None, :] * s.v, axis=1)}
