"""Pins of the oracle's constant self-energy W_self = (sum q^2/(eps0 V)) sum_H S^2/|k|^2
(V = L^3, or the area L^2 in two dimensions), the part of the discrete
Lagrangian's field term that every particle carries on its own (Section 3).

Two facts fix it independently of its formula:
* a lone particle's field energy, deposited and summed by the oracle's own
  (separately pinned) deposit and field-energy loops, is exactly W_self;
* for two particles the pair part of W is a sum of cos(k.r) over the retained
  modes, which averages to zero over the displacements r of a G^D grid with
  G > 2 n_max, so the grid mean of W is W_self exactly.
A slip such as S instead of S^2, V instead of the area in 2-D, a missing eps0 or
the full cube instead of the half space fails both.  The eps0 factor of the
field energy itself is tied to the force's (pinned by the dispersion relation)
through F = -dW/dx at eps0 != 1.
"""
import numpy as np
import pytest

import workloads


def _pos(dim, L, u):
    return (L * np.asarray(u[:dim], dtype=float))[:, None]


@pytest.mark.parametrize("dim", [3, 2])
@pytest.mark.parametrize("kind,a", [("gaussian", 0.07), ("tent", 0.11), ("delta", 0.0)])
@pytest.mark.parametrize("L,eps0", [(1.0, 1.0), (1.7, 0.3)])
def test_self_energy_is_lone_particle_field_energy(orc, dim, kind, a, L, eps0):
    n_max = 5
    modes = orc.half_modes(n_max, dim=dim)
    for q, u in ((1.0, [0.3, 0.6, 0.9]), (-2.5, [0.0, 0.999, 0.41])):
        pos = _pos(dim, L, u)
        rho = orc.deposit(pos, [q], L, modes, kind, a * L)
        W = orc.field_energy(rho, L, modes, eps0)
        Ws = orc.self_energy([q], L, modes, eps0, kind, a * L)
        assert abs(W - Ws) <= 1e-13 * Ws


@pytest.mark.parametrize("dim", [3, 2])
def test_self_energy_is_grid_mean_of_pair_field_energy(orc, dim):
    n_max, G, L, eps0, a = 3, 8, 1.3, 0.6, 0.05
    modes = orc.half_modes(n_max, dim=dim)
    q = np.array([1.5, -0.7])
    x1 = L * np.array([0.123, 0.456, 0.789][:dim])
    axes = np.meshgrid(*[np.arange(G)] * dim, indexing="ij")
    shifts = np.stack([a_.ravel() for a_ in axes]) * (L / G)
    Ws = []
    for r in shifts.T:
        pos = np.stack([x1, (x1 + r) % L], axis=1)
        Ws.append(orc.field_energy(orc.deposit(pos, q, L, modes, "gaussian", a), L, modes, eps0))
    ref = orc.self_energy(q, L, modes, eps0, "gaussian", a)
    assert abs(np.mean(Ws) - ref) <= 1e-13 * ref
    # and the pair part is not identically zero, so the mean is a real test
    assert np.ptp(Ws) > 1e-3 * ref


@pytest.mark.parametrize("dim", [3, 2])
def test_field_energy_eps0_matches_force(orc, dim):
    """F = -dW/dx with eps0 = 0.3: the field energy carries the same 1/eps0 as
    the solve that the force uses."""
    L, n_max, a, eps0 = 1.2, 4, 0.06, 0.3
    mk = workloads.random_particles if dim == 3 else workloads.random_particles_2d
    p = mk(6, L=L, charge="uniform")
    pos = p.positions()
    modes = orc.half_modes(n_max, dim=dim)
    F = orc.fields(pos, p.q, L, n_max, "gaussian", a, eps0, modes=modes).F
    d = 1e-6 * L
    for j in (0, 4):
        for c in range(dim):
            pp, pm = pos.copy(), pos.copy()
            pp[c, j] += d
            pm[c, j] -= d
            Wp = orc.field_energy(orc.deposit(pp, p.q, L, modes, "gaussian", a), L, modes, eps0)
            Wm = orc.field_energy(orc.deposit(pm, p.q, L, modes, "gaussian", a), L, modes, eps0)
            assert abs(-(Wp - Wm) / (2 * d) - F[c, j]) < 1e-7 * np.max(np.abs(F))
