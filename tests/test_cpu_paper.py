"""The benchmark's faster CPU baseline (``oracle.cpu_paper``: the paper's
per-axis powers, Section 8) against the oracle's plain definition: deposit and
force on ragged particle counts (not multiples of its 8-particle blocks), unit
and non-unit boxes, delta and Gaussian shapes."""
import numpy as np
import pytest

import oracle
from oracle import cpu_paper


@pytest.mark.parametrize("N,n_max,L,kind,a", [
    (1, 3, 1.0, "delta", 0.0),
    (13, 4, 1.0, "gaussian", 0.05),
    (301, 8, 2.5, "gaussian", 0.1),
    (250, 16, 0.7, "delta", 0.0),
])
def test_matches_oracle(N, n_max, L, kind, a):
    rng = np.random.default_rng(N + 7 * n_max)
    pos = rng.random((3, N)) * L
    q = rng.choice([-1.0, 1.0], N) * (1.0 + rng.random(N))
    modes = oracle.half_modes(n_max)
    S = oracle.shape(kind, a, oracle.wave_vectors(modes, L))
    rho_o = oracle.deposit(pos, q, L, modes, kind, a)
    rho = cpu_paper.deposit(pos, q, L, n_max, S)
    assert rho.shape == rho_o.shape
    assert np.abs(rho - rho_o).max() <= 1e-12 * np.abs(rho_o).max()
    ps = oracle.psi(rho_o, L, modes, 1.0, kind, a)
    F_o = oracle.force_from_psi(pos, q, L, modes, ps)
    F = cpu_paper.force(pos, q, L, n_max, ps)
    assert F.shape == F_o.shape
    # a lone particle's force is zero up to rounding of its terms: scale by
    # them there (2 max|q| sum |k| |psi| bounds every |F_j|)
    terms = 2.0 * np.abs(q).max() * (np.linalg.norm(oracle.wave_vectors(modes, L), axis=1) * np.abs(ps)).sum()
    scale = max(np.linalg.norm(F_o, axis=0).max(), 1e-3 * terms)
    assert np.linalg.norm(F - F_o, axis=0).max() <= 1e-12 * scale
