"""Graph replay of multi-step runs (sce_step with sce_set_step_graph) against
direct launches: bit-identical states, over replays interleaved with the
program's own eager work (diagnostics, single steps, a dt change that forces a
new capture), for each precision and both leapfrog forms."""
import time

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1508_07344_amd as sce
    sce.load_library()
    return sce


def _run(sce, p, prec, scheme, graph):
    out = []
    with sce.Context.from_particles(p, precision=prec, scheme=scheme) as c:
        c.sce_set_small_step(0)  # the multi-kernel step, whose launches the graph replays
        c.sce_set_step_graph(graph)
        for n, dt in ((37, p.dt), (1, p.dt), (50, p.dt), (33, 0.5 * p.dt), (40, p.dt)):
            c.sce_step(dt, n)
            x, v = c.sce_get_particles()
            d, _ = c.sce_diagnostics()
            out.append((x, v, d.total, d.step))
    return out


@pytest.mark.parametrize("prec,scheme,case", [
    ("fp64", "kdk", "kepler2d"), ("fp64", "dkd", "kepler2d"), ("fp32", "kdk", "plasma3d"),
    ("split_f16", "kdk", "plasma3d"), ("split_f16", "dkd", "plasma2d")])
def test_graph_replay_matches_direct_launches(prec, scheme, case):
    sce = _gpu()
    p = {"kepler2d": workloads.kepler_2d(),
         "plasma3d": workloads.random_plasma(N=3000, n_max=8, a=0.05, sigma_v=0.05),
         "plasma2d": workloads.random_plasma_2d(N=3000, n_max=16, a=0.02, sigma_v=0.05)}[case]
    direct = _run(sce, p, prec, scheme, 0)
    for G in (8, 5):
        graph = _run(sce, p, prec, scheme, G)
        for (xa, va, ea, sa), (xb, vb, eb, sb) in zip(direct, graph):
            assert sa == sb
            assert np.array_equal(xa, xb) and np.array_equal(va, vb) and ea == eb


def test_graph_replay_timing_on_small_systems():
    """The paper's two-body problem: time per step with graph replay and with
    direct launches, reported only (wall-clock ratios on a shared machine are
    not asserted).  The states after the timed runs must be bit-identical."""
    sce = _gpu()
    p = workloads.kepler_2d()
    rates, states = {}, {}
    for G in (0, 8, 32):
        with sce.Context.from_particles(p) as c:
            c.sce_set_small_step(0)
            c.sce_set_step_graph(G)
            c.sce_step(p.dt, 200)
            c.sce_sync()
            t0 = time.perf_counter()
            c.sce_step(p.dt, 4000)
            c.sce_sync()
            rates[G] = 1e6 * (time.perf_counter() - t0) / 4000
            states[G] = c.sce_get_particles()
    print("us per step by steps per graph:", {k: round(v, 2) for k, v in rates.items()})
    for G in (8, 32):
        assert np.array_equal(states[G][0], states[0][0]) and np.array_equal(states[G][1], states[0][1])


def test_step_graph_argument_checks():
    sce = _gpu()
    p = workloads.kepler_2d()
    with sce.Context.from_particles(p) as c:
        for bad in (-1, 4097):
            with pytest.raises(sce.SceError):
                c.sce_set_step_graph(bad)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "split_f16"])
@pytest.mark.parametrize("case", ["plasma3d", "plasma2d", "tent3d"])
def test_multi_step_call_matches_single_steps(prec, case):
    """One sce_step call of n kick-drift-kick steps applies a step's closing
    half kick, the next step's opening half kick and its drift in one pass
    after the force (inside the split-precision force kernel); the states must
    be bit for bit those of n calls of one step each, graphs off (direct
    launches) and on."""
    sce = _gpu()
    p = {"plasma3d": workloads.random_plasma(N=20000, n_max=8, a=0.05, sigma_v=0.05),
         "plasma2d": workloads.random_plasma_2d(N=20000, n_max=12, a=0.03, sigma_v=0.05),
         "tent3d": workloads.tent_plasma(N=3000, n_max=6)}[case]
    states = {}
    for mode in ("single", "direct", "graph"):
        with sce.Context.from_particles(p, precision=prec, scheme="kdk") as c:
            c.sce_set_small_step(0)
            c.sce_set_step_graph(4 if mode == "graph" else 0)
            if mode == "single":
                for _ in range(11):
                    c.sce_step(p.dt, 1)
            else:
                c.sce_step(p.dt, 11)
            x, v = c.sce_get_particles()
            d, _ = c.sce_diagnostics()
            states[mode] = (x, v, d.total, d.step)
    xs, vs, es, ss = states["single"]
    for mode in ("direct", "graph"):
        x, v, e, s = states[mode]
        print(f"{case} {prec} {mode}: max|dx| {np.max(np.abs(x - xs)):.1e}", flush=True)
        assert s == ss == 11
        assert np.array_equal(x, xs) and np.array_equal(v, vs) and e == es
