"""Accuracy of the reduced-precision paths beyond the timed size: a cold
lattice of 4,194,304 particles (256 x 128 x 128 jittered sites, the recipe of
the 2^20 lattice), where the split-precision deposit runs the longest FP32 sum
it ever runs (8,192 particles per split) over four times as many splits.

Split FP16 and FP32 are compared with the FP64 GPU path on every mode and
particle (the FP64 path is itself held to 1e-12 of the oracle by the other
parity tests), and rho on sampled modes with the oracle directly.  The
normwise errors and their margin to the 1e-5 bar are printed.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1508_07344_amd as sce
    sce.load_library()
    return sce


def e_rel(a, ref):
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))


def e_F(F, ref):
    return float(np.max(np.linalg.norm(F - ref, axis=0)) / np.max(np.linalg.norm(ref, axis=0)))


@pytest.mark.parametrize("n_max,a", [(32, 0.01), (16, 0.02)])
def test_4M_lattice_reduced_precision_against_fp64(n_max, a):
    sce = _gpu()
    p = workloads.cold_lattice(nx=256, ny=128, nz=128, n_max=n_max, a=a)
    assert p.N == 1 << 22
    out = {}
    for prec in ("fp64", "fp32", "split_f16"):
        with sce.Context.from_particles(p, precision=prec) as c:
            out[prec] = (c.sce_deposit(), c.sce_force())
    modes = oracle.half_modes(n_max)
    rng = np.random.default_rng(22)
    k1 = int(np.nonzero((modes == [1, 0, 0]).all(axis=1))[0][0])
    mi = np.unique(np.concatenate([[k1], rng.choice(len(modes), 31, replace=False)]))
    ref = oracle.deposit(p.positions(), p.q, p.L, modes[mi], p.shape, p.a)
    e64 = e_rel(out["fp64"][0][mi], ref)
    print(f"4M lattice n_max={n_max} fp64: e_rho(sampled, oracle)={e64:.3e}", flush=True)
    assert e64 <= 1e-12
    for prec in ("fp32", "split_f16"):
        er = e_rel(out[prec][0], out["fp64"][0])
        ef = e_F(out[prec][1], out["fp64"][1])
        eo = e_rel(out[prec][0][mi], ref)
        print(f"4M lattice n_max={n_max} {prec} vs fp64: e_rho={er:.3e} e_F={ef:.3e} "
              f"(margin to 1e-5: {1e-5 / max(er, ef):.1f}x); e_rho(sampled, oracle)={eo:.3e}", flush=True)
        assert er <= 1e-5 and ef <= 1e-5 and eo <= 1e-5
