"""GPU parity of the batched serving path (sce_server_*) against the FP64 oracle.

Every request of a batch is compared with the oracle's kick-drift-kick run of
the same request: positions, velocities and the force at the end, and the
diagnostics at the start and the end.  Requests are resident together, so the
batched kernels' per-request indexing (ragged N, several n_max, shapes, box
sizes, eps0) is exercised in the same launches.  Tolerances as for the single
simulation path: FP64 1e-12 normwise, FP32 1e-5.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1508_07344_amd as sce
    sce.load_library()
    return sce


def _requests():
    rp = workloads.random_particles
    return [
        ("one", rp(1, L=1.0, charge="positive").with_(n_max=3, a=0.05, dt=1e-3), 2),
        ("two_body", workloads.two_body(), 3),
        ("tent", rp(333, L=2.3, charge="uniform").with_(n_max=5, shape="tent", a=0.2, dt=2e-3), 3),
        ("delta", rp(1237, L=1.7, charge="alternating").with_(n_max=12, shape="delta", a=0.0, dt=1e-3), 1),
        ("eps0", rp(517, L=1.0, charge="uniform").with_(n_max=4, a=0.03, eps0=0.25, dt=1e-3), 2),
        ("n1", rp(64, L=0.9, charge="alternating").with_(n_max=1, a=0.1, dt=1e-3), 4),
        ("n8", workloads.random_plasma(N=1025, n_max=8, a=0.05, salt=3), 2),
        ("plasma16", workloads.random_plasma(N=3001, n_max=16, a=0.02), 2),
        ("steps0", workloads.random_plasma(N=700, n_max=16, a=0.02, salt=5), 0),
        # two-dimensional requests (line charges), resident in the same batches
        ("kepler2d", workloads.kepler_2d(), 5),
        ("thermal2d", workloads.thermal_2d(), 3),
        ("plasma2d", workloads.random_plasma_2d(N=1500, n_max=12, a=0.03, salt=4), 2),
    ]


def _oracle_run(p, steps):
    s = oracle.State.from_particles(p)
    s.refresh()
    e0 = oracle.energy(s)
    u0 = float(np.sum(s.q * oracle.potential_from_psi(s.pos, s.L, s._modes(),
                                                      oracle.psi(s.rho, s.L, s._modes(), s.eps0, s.kind, s.a))))
    oracle.step_kdk(s, p.dt, steps)
    return s, e0, u0


def _periodic_err(x, ref, L):
    d = np.mod(x - ref + 0.5 * L, L) - 0.5 * L
    return float(np.max(np.abs(d)) / L)


def _fscale(p, Fref):
    """Denominator of e_F: the largest reference force, or for a lone particle
    (no self-force) the scale of one mode sum, 2 q^2 sum_H |k| S^2 / (eps0 k^2 V)."""
    if p.N > 1:
        return float(np.max(np.linalg.norm(Fref, axis=0)))
    k = oracle.wave_vectors(oracle.half_modes(p.n_max), p.L)
    S = oracle.shape(p.shape, p.a, k)
    return float(np.sum(2 * p.q[0] ** 2 * np.linalg.norm(k, axis=1) * S * S / np.sum(k * k, axis=1))
                 / (p.eps0 * p.L ** 3))


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def ref_runs():
    return {name: (p, steps, _oracle_run(p, steps)) for name, p, steps in _requests()}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_requests_match_oracle(prec, ref_runs):
    sce = _gpu()
    tol = TOL[prec]
    with sce.Server(hbm_budget_bytes=1 << 30, precision=prec) as srv:
        ids = {srv.sce_server_submit(p, n_steps=steps): name for name, (p, steps, _) in ref_runs.items()}
        for _ in range(100):
            na, nq = srv.sce_server_tick()
            if na == 0 and nq == 0:
                break
        done = srv.sce_server_poll()
        assert sorted(done) == sorted(ids)
        for rid in done:
            name = ids[rid]
            p, steps, (s, e0, u0) = ref_runs[name]
            x, v, F, d0, d1 = srv.sce_server_result(rid)
            ef = float(np.max(np.linalg.norm(F - s.F, axis=0))) / _fscale(p, s.F)
            print(f"{prec} {name}: N={p.N} n={p.n_max} steps={steps} e_F={ef:.2e}", flush=True)
            assert ef <= tol, (name, ef)
            assert _periodic_err(x, s.pos, p.L) <= (1e-13 if prec == "fp64" else 1e-9), name
            assert _rel(v, s.vel) <= tol * 10, name
            assert d0.step == 0 and d1.step == steps
            assert abs(d0.kinetic - e0["kinetic"]) <= 1e-13 * max(e0["kinetic"], 1e-300) + 1e-300
            assert abs(d0.field - e0["field"]) <= tol * abs(e0["field"]), name
            assert abs(d0.interaction - u0) <= tol * abs(u0) + 1e-14, name
            e1 = oracle.energy(s)
            assert abs(d1.field - e1["field"]) <= tol * abs(e1["field"]), name
            assert abs(d1.kinetic - e1["kinetic"]) <= tol * max(e1["kinetic"], 1e-12), name
            assert abs(d1.total - (d1.kinetic + d1.field)) <= 1e-15 * abs(d1.total)
            assert x.shape == (p.dim, p.N) and F.shape == (p.dim, p.N)
            assert np.allclose(d1.momentum[:p.dim], e1["momentum"], rtol=0,
                               atol=tol * e1["momentum_abs_sum"] + 1e-15)
            assert p.dim == 3 or d1.momentum[2] == 0.0
        st = srv.sce_server_stats()
        assert st["requests_done"] == len(ids)
        assert st["request_steps"] == sum(steps + 1 for _, (_, steps, _) in ref_runs.items())
        assert 0 < st["p50_step_s"] <= st["p99_step_s"] <= st["max_step_s"]
        assert st["active"] == 0 and st["queued"] == 0 and st["hbm_used_bytes"] == 0


def test_results_do_not_depend_on_batching():
    """A request's result is bit-identical whether it runs alone, in a full
    batch, or queued behind a small device budget."""
    sce = _gpu()
    reqs = workloads.serving_requests(n_requests=24, N_range=(2, 2000), steps_range=(2, 12), salt=7)

    def run(budget, only=None):
        out = {}
        with sce.Server(hbm_budget_bytes=budget, precision="fp32") as srv:
            idmap = {}
            for r in reqs:
                if only is None or r.id == only:
                    idmap[srv.sce_server_submit(r.particles)] = r.id
            peak_active = 0
            for _ in range(10000):
                na, nq = srv.sce_server_tick()
                peak_active = max(peak_active, na)
                if na == 0 and nq == 0:
                    break
            for rid in srv.sce_server_poll():
                x, v, F, d0, d1 = srv.sce_server_result(rid)
                out[idmap[rid]] = (x, v, F, d1.total)
            st = srv.sce_server_stats()
        return out, peak_active, st

    full, peak_full, _ = run(1 << 30)
    small, peak_small, st_small = run(2 << 20)
    assert peak_full == len(reqs)
    assert peak_small < len(reqs)
    assert st_small["hbm_peak_bytes"] <= 2 << 20
    alone, _, _ = run(1 << 30, only=reqs[5].id)
    assert set(full) == set(small) == {r.id for r in reqs}
    for rid in full:
        for a, b in zip(full[rid], small[rid]):
            assert np.array_equal(a, b), rid
    for a, b in zip(full[reqs[5].id], alone[reqs[5].id]):
        assert np.array_equal(a, b)


def test_server_rejects_invalid_requests():
    sce = _gpu()
    p = workloads.random_plasma(N=100, n_max=8, a=0.05)
    with sce.Server(hbm_budget_bytes=1 << 20, precision="fp32") as srv:
        for bad in [p.with_(n_max=17), p.with_(n_max=0), p.with_(L=-1.0), p.with_(a=-0.1),
                    p.with_(eps0=0.0), p.with_(dt=float("nan")), p.with_(m=np.zeros(100)),
                    p.with_(dim=5)]:
            with pytest.raises(sce.SceError) as ei:
                srv.sce_server_submit(bad)
            assert ei.value.status == sce.SCE_EINVAL
        big = workloads.random_plasma(N=8192, n_max=16, a=0.05)
        with pytest.raises(sce.SceError) as ei:
            srv.sce_server_submit(big)
        assert "budget" in str(ei.value)
        with pytest.raises(sce.SceError):
            srv.sce_server_submit(p, n_steps=-1)
        rid = srv.sce_server_submit(p, n_steps=1)
        with pytest.raises(sce.SceError):
            srv.sce_server_result(rid)
        while srv.sce_server_tick() != (0, 0):
            pass
        srv.sce_server_result(rid)
        with pytest.raises(sce.SceError):
            srv.sce_server_result(rid)


def test_graph_replay_matches_direct_launches():
    """Each tick replays a HIP graph of its four launches (captured again when
    the resident set changes, with admissions and retirements between
    replays).  Every request's final state and diagnostics must be bit-identical
    to ticks launched directly."""
    sce = _gpu()
    reqs = workloads.serving_requests(n_requests=16, N_range=(2, 3000), steps_range=(3, 40), salt=11)

    def run(graph):
        out = {}
        with sce.Server(hbm_budget_bytes=4 << 20, precision="fp32", graph=graph) as srv:
            idmap = {srv.sce_server_submit(r.particles): r.id for r in reqs}
            ticks = 0
            while srv.sce_server_tick() != (0, 0):
                ticks += 1
            for rid in srv.sce_server_poll():
                x, v, F, d0, d1 = srv.sce_server_result(rid)
                out[idmap[rid]] = (x, v, F, d0.total, d1.total, d1.kinetic)
        return out, ticks

    g, tg = run(True)
    d, td = run(False)
    assert tg == td and tg > 20
    assert set(g) == set(d) == {r.id for r in reqs}
    for rid in g:
        for a, b in zip(g[rid], d[rid]):
            assert np.array_equal(a, b), rid
