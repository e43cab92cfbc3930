"""The single-workgroup multi-step kernel for small systems (sce_set_small_step):
trajectories against the FP64 oracle's leapfrog for the paper's problem
sizes (the 3-D two-body problem at n_max = 8, the 2-D Kepler problem, the
16-particle 2-D thermal plasma), agreement with the multi-kernel step, the
eligibility limits, and its speed."""
import time

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


def _oracle_run(p, scheme, h, n):
    s = oracle.State.from_particles(p)
    step = oracle.step_kdk if scheme == "kdk" else oracle.step_dkd
    return step(s, h, n)


def _gpu_run(sce, p, scheme, h, n, max_pairs=1 << 16):
    with sce.Context.from_particles(p, precision="fp64", scheme=scheme) as c:
        c.sce_set_small_step(max_pairs)
        c.sce_step(h, n)
        x, v = c.sce_get_particles()
        d, _ = c.sce_diagnostics()
    return x, v, d


def _wrapped_err(a, b, L):
    d = np.abs(a - b)
    return np.minimum(d, L - d)


@pytest.mark.parametrize("scheme", ["kdk", "dkd"])
@pytest.mark.parametrize("case", ["two_body", "kepler_2d", "thermal_2d"])
def test_small_step_trajectory_matches_oracle(case, scheme):
    sce = _gpu()
    p = {"two_body": workloads.two_body(), "kepler_2d": workloads.kepler_2d(),
         "thermal_2d": workloads.thermal_2d()}[case]
    n = 100 if case == "thermal_2d" else 400
    ref = _oracle_run(p, scheme, p.dt, n)
    x, v, d = _gpu_run(sce, p, scheme, p.dt, n)
    ex = np.max(_wrapped_err(x, ref.pos, p.L)) / p.L
    ev = np.max(np.abs(v - ref.vel)) / np.max(np.abs(ref.vel))
    print(f"small-step {case} {scheme}: e_x={ex:.2e} e_v={ev:.2e}")
    assert ex <= 1e-11 and ev <= 1e-10
    assert d.step == n


@pytest.mark.parametrize("scheme", ["kdk", "dkd"])
@pytest.mark.parametrize("N,n_max,dim", [(1, 8, 3), (3, 8, 3), (37, 5, 3), (256, 3, 3), (100, 9, 2)])
def test_small_step_matches_multi_kernel_step(N, n_max, dim, scheme):
    """Same runs through the multi-kernel step (max_pairs = 0): rounding-level
    agreement, and the KDK end force reused by the next step either way."""
    sce = _gpu()
    if dim == 3:
        p = workloads.random_plasma(N=N, n_max=n_max, a=0.08, sigma_v=0.05, dt=2e-3, salt=N)
    else:
        p = workloads.random_plasma_2d(N=N, n_max=n_max, a=0.05, sigma_v=0.05, salt=N).with_(dt=2e-3)
    xa, va, da = _gpu_run(sce, p, scheme, p.dt, 60)
    xb, vb, db = _gpu_run(sce, p, scheme, p.dt, 60, max_pairs=0)
    ex = np.max(_wrapped_err(xa, xb, p.L)) / p.L
    ev = np.max(np.abs(va - vb)) / max(np.max(np.abs(vb)), 1e-300)
    print(f"small vs multi-kernel N={N} n={n_max} {dim}d {scheme}: e_x={ex:.2e} e_v={ev:.2e}")
    assert ex <= 1e-12 and ev <= 1e-10
    assert abs(da.total - db.total) <= 1e-11 * abs(db.total)


def test_small_step_continues_the_multi_kernel_state():
    """Steps split between the two paths (and a checkpoint in between) agree
    with one uninterrupted run."""
    sce = _gpu()
    p = workloads.random_plasma(N=24, n_max=6, a=0.08, sigma_v=0.05, dt=2e-3, salt=5)
    x0, v0, _ = _gpu_run(sce, p, "kdk", p.dt, 90)
    with sce.Context.from_particles(p, precision="fp64") as c:
        c.sce_set_small_step(0)
        c.sce_step(p.dt, 30)
        c.sce_set_small_step(1 << 16)
        c.sce_step(p.dt, 30)
        blob = c.sce_get_state()
    with sce.Context.from_particles(p, precision="fp64") as c:
        c.sce_set_state(blob)
        c.sce_step(p.dt, 30)
        x1, v1 = c.sce_get_particles()
    assert np.max(_wrapped_err(x0, x1, p.L)) <= 1e-12 * p.L
    assert np.max(np.abs(v0 - v1)) <= 1e-10 * np.max(np.abs(v0))


def test_small_step_limits_fall_back_to_the_multi_kernel_step():
    """Past the limits (N > 256, N (n_max + 1) > 1024, N |H| > max_pairs) or
    with timing on, the step runs as separate kernels, with the same results."""
    sce = _gpu()
    for p in (workloads.random_plasma(N=257, n_max=2, a=0.1, sigma_v=0.05, dt=2e-3, salt=1),
              workloads.random_plasma(N=120, n_max=9, a=0.1, sigma_v=0.05, dt=2e-3, salt=2)):
        xa, va, _ = _gpu_run(sce, p, "kdk", p.dt, 10)
        xb, vb, _ = _gpu_run(sce, p, "kdk", p.dt, 10, max_pairs=0)
        assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    p = workloads.two_body()
    with sce.Context.from_particles(p) as c:
        c.sce_timing_enable(True)
        c.sce_step(p.dt, 5)
        tm = c.sce_timing_read()
    assert tm["force_launches"] >= 5
    with sce.Context.from_particles(p) as c:
        with pytest.raises(sce.SceError):
            c.sce_set_small_step(-1)
        with pytest.raises(sce.SceError):
            c.sce_set_small_step((1 << 24) + 1)


def test_small_step_speed():
    """Microseconds per step of the paper's problems, one kernel per block of
    steps against the multi-kernel step (both reported); the fused form must
    be at least three times faster."""
    sce = _gpu()
    out = {}
    for case, p in (("two_body", workloads.two_body()), ("kepler_2d", workloads.kepler_2d()),
                    ("thermal_2d", workloads.thermal_2d())):
        for mp in (1 << 16, 0):
            with sce.Context.from_particles(p) as c:
                c.sce_set_small_step(mp)
                c.sce_step(p.dt, 100)
                c.sce_sync()
                t0 = time.perf_counter()
                c.sce_step(p.dt, 4000)
                c.sce_sync()
                out[(case, mp)] = 1e6 * (time.perf_counter() - t0) / 4000
    print("us per step (fused, multi-kernel):",
          {k[0]: (round(out[(k[0], 1 << 16)], 2), round(out[(k[0], 0)], 2)) for k in out if k[1] == 0})
    for case in ("two_body", "kepler_2d", "thermal_2d"):
        assert out[(case, 1 << 16)] * 3 < out[(case, 0)]
