"""Throughput benchmark of the spectral electrostatic hot path on one MI355X.

One step = one kick-drift-kick leapfrog step: half kick, drift, phase tables,
deposit (type-1 sum), cross-tile reduction + field solve, force (type-2 sum)
with the fused half kick.  Workload: cold electron plasma, 128 x 128 x 64
jittered lattice (N = 1,048,576) with a 1% density perturbation along x,
n_max = 32 (|H| = 137,312 half-space modes), Gaussian shape a = 0.01,
dt = 5e-4 (seeded synthetic input, see workloads.cold_lattice).

Metric: particle x mode pairs per second per step, N |H| pairs per step
(each pair is visited once by the deposit and once by the force).

Prints ONE JSON line.  Timing: W warmup steps, then K steps bracketed by
device synchronisation; the deposit- and force-kernel durations come from HIP
events recorded by the library on its own stream over the timed region.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("particle×mode pairs/s per step (FP64 vs split-precision); "
          "serve p50/p99 step latency")

# Published MI355X peaks (256 CUs, 2.4 GHz): vector FP64 and FP32 (the FP32
# figure counts packed-FP32 issue), dense FP16 matrix cores for the split path.
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "split_f16": 2500.0}
BOUND = {"fp64": "alu", "fp32": "alu", "split_f16": "mfma"}
DTYPE = {"fp64": "f64", "fp32": "f32", "split_f16": "f16"}
# Algorithmic flops per particle x mode pair, counted as complex multiply-adds
# of the separable sums: deposit 1 complex MAC (8), force 2 complex MACs (16).
FLOPS_PER_PAIR = {"deposit": 8, "force": 16}
# Matrix-core flops the split kernels issue per pair (three FP16 products per
# real product; the deposit's real-form sums serve +-k_y and +-n_z together).
MFMA_ISSUED_PER_PAIR = {"deposit": 12, "force": 24}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="split_f16", choices=["fp64", "fp32", "split_f16"])
    ap.add_argument("--also", default="fp64,fp32", help="comma list of extra precisions to time")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--n16", type=int, default=1,
                    help="also time the split step of the two n_max = 16 workloads (informational)")
    ap.add_argument("--cpu-sample", type=int, default=49152,
                    help="particles in the oracle's timed sample (all modes)")
    ap.add_argument("--cpu-paper-sample", type=int, default=262144,
                    help="particles in the timed sample of the CPU program with the paper's "
                         "per-axis powers (all modes; 0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=4096,
                    help="requests of the serving workload (0 = skip the serving run)")
    ap.add_argument("--serve-loads", default="0.5,0.7,0.9",
                    help="offered loads, as fractions of the measured saturated capacity")
    ap.add_argument("--serve-check", type=int, default=64,
                    help="requests sampled for the per-request force error against FP64")
    ap.add_argument("--peaks", type=int, default=1,
                    help="measure the matrix-core and vector throughput peaks (libsce_peak.so)")
    ap.add_argument("--study", default="", choices=["", "longrun", "dispersion", "h2", "twod", "tent", "medium"],
                    help="run one validation study instead of the throughput benchmark")
    ap.add_argument("--long-steps", type=int, default=100000,
                    help="steps of the long-run conservation study")
    ap.add_argument("--long-precisions", default="split_f16,fp32,fp64",
                    help="comma list of precisions of the long-run study")
    ap.add_argument("--tent-precisions", default="split_f16,fp32,fp64",
                    help="comma list of precisions of the tent-field study")
    ap.add_argument("--twod-steps", type=int, default=200000,
                    help="steps of each long run of the two-dimensional study")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="only run a plain device-to-device copy of this many MiB (five times), "
                         "the reference kernel for scaling the FETCH_SIZE/WRITE_SIZE counters")
    return ap.parse_args()


def time_path(sce, p, precision, steps, warmup):
    import torch
    c = sce.Context.from_particles(p, precision=precision, scheme="kdk")
    c.sce_step(p.dt, warmup)
    c.sce_sync()
    torch.cuda.synchronize()
    c.sce_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.sce_step(p.dt, steps)
    c.sce_sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = c.sce_timing_read()
    c.sce_timing_enable(False)
    d, st = c.sce_diagnostics()
    H = c.sce_mode_count()
    c.close()
    pairs = p.N * H
    wall = t1 - t0
    out = {
        "precision": precision,
        "pairs_per_s": pairs * steps / wall,
        "ms_per_step": 1e3 * wall / steps,
        "deposit_ms_avg": tm["deposit_ms"] / max(tm["deposit_launches"], 1),
        "force_ms_avg": tm["force_ms"] / max(tm["force_launches"], 1),
        "deposit_launches": tm["deposit_launches"],
        "force_launches": tm["force_launches"],
        "modes_half": H,
        "energy_total": d.total,
        "momentum_rel": float(max(abs(x) for x in d.momentum) / max(d.momentum_abs_sum, 1e-300)),
    }
    return out


def code_hash(path):
    """First 16 hex digits of the SHA-256 of a source file's code: the text
    with // comments removed and runs of white space collapsed, so that an
    edit of comments alone keeps the hash."""
    import hashlib
    import re
    txt = open(path, encoding="utf-8").read()
    txt = re.sub(r"//[^\n]*", "", txt)
    txt = " ".join(txt.split())
    return hashlib.sha256(txt.encode()).hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of a matrix-core kernel from the committed rocprofv3
    summary, or None if the kernel code changed since it was measured."""
    import re
    src = os.path.join(ROOT, "paper_1508_07344_amd", "csrc", "kernels_mfma.hip")
    summ = os.path.join(ROOT, "profiles", "traffic_cold_lattice_1M_n32.md")
    try:
        sha = code_hash(src)
        txt = open(summ).read()
    except OSError:
        return None
    m = re.search(r"traffic kernel=%s fetch_bytes=(\S+) write_bytes=(\S+) code_sha256_16=(\w+)" % kernel, txt)
    if not m or m.group(3) != sha:
        return None
    return float(m.group(1)) + float(m.group(2))


PEAK_PROBE = {"split_f16": "mfma_f16", "fp32": "fma_f32", "fp64": "fma_f64"}


def measure_peaks():
    """Sustained throughput of the three units the kernels are bound by, from
    the probes of libsce_peak.so (TFLOP/s): dense FP16 matrix core, FP32 FMA
    (no packed issue), FP64 FMA."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1508_07344_amd", "libsce_peak.so"))
    out = {}
    for name in ("mfma_f16", "fma_f32", "fma_f64"):
        fn = getattr(lib, "sce_peak_" + name)
        fn.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        fn.restype = ctypes.c_int
        tf, ms = ctypes.c_double(), ctypes.c_double()
        if fn(ctypes.byref(tf), ctypes.byref(ms)) != 0:
            raise RuntimeError("peak probe failed: " + name)
        out[name] = round(tf.value, 2)
    return out


def roofline(r, N, peaks=None):
    """Roofline of the dominant (longer) of the two particle x mode kernels.
    achieved = algorithmic flops per launch / average launch time, with the
    algorithmic count of complex multiply-adds: 8 flops per pair for the
    deposit, 16 for the force.  The split path's deposit time covers both of
    its launches (the chunk-image build and the matrix-core kernel).  With
    measured peaks, frac_measured is achieved over the probe's sustained rate
    of the same unit."""
    pairs = N * r["modes_half"]
    mf = r["precision"] == "split_f16"
    peak = PEAK_TFLOPS[r["precision"]]
    kern = {"deposit": ("k_deposit_mfma" if mf else "k_deposit", r["deposit_ms_avg"]),
            "force": ("k_force_mfma" if mf else "k_force", r["force_ms_avg"])}
    rates = {k: FLOPS_PER_PAIR[k] * pairs / (t * 1e-3) / 1e12 for k, (_, t) in kern.items()}
    dom = max(kern, key=lambda k: kern[k][1])
    other = "force" if dom == "deposit" else "deposit"
    traffic = measured_traffic(kern[dom][0]) if mf else None
    out = {"bound": BOUND[r["precision"]], "kernel": kern[dom][0],
           "achieved": round(rates[dom], 3), "peak": peak, "unit": "TFLOP/s",
           "frac": round(rates[dom] / peak, 4), "traffic": traffic,
           "other_kernel": {"kernel": kern[other][0], "achieved": round(rates[other], 3),
                            "frac": round(rates[other] / peak, 4)}}
    if mf:
        # matrix-core flops the split kernels issue: three products per real
        # product, and the real-form sums serve the +-k_y and +-n_z modes of
        # a row pair together (12 per pair in the deposit, 24 in the force)
        for k, o in ((dom, out), (other, out["other_kernel"])):
            o["issued"] = round(rates[k] * MFMA_ISSUED_PER_PAIR[k] / FLOPS_PER_PAIR[k], 3)
            o["issued_frac"] = round(o["issued"] / peak, 4)
    if peaks:
        pm = peaks[PEAK_PROBE[r["precision"]]]
        out["peak_measured"] = pm
        out["frac_measured"] = round(rates[dom] / pm, 4)
        out["other_kernel"]["frac_measured"] = round(rates[other] / pm, 4)
        if mf:
            out["issued_frac_measured"] = round(out["issued"] / pm, 4)
            out["other_kernel"]["issued_frac_measured"] = round(out["other_kernel"]["issued"] / pm, 4)
    return out


def _drive(srv, reqs, t_arrive, label=""):
    """Submit each request at its arrival time (seconds from now) and tick until
    every request has finished.  Returns wall seconds and the server's ids.
    Prints a progress line to stderr every 10 s of wall time."""
    order = sorted(range(len(reqs)), key=lambda i: t_arrive[i])
    ids = {}
    t0 = time.perf_counter()
    t_print = t0
    k = 0
    done = 0
    while True:
        now = time.perf_counter() - t0
        while k < len(order) and t_arrive[order[k]] <= now:
            i = order[k]
            ids[srv.sce_server_submit(reqs[i].particles)] = i
            k += 1
        na, nq = srv.sce_server_tick()
        if label and time.perf_counter() - t_print > 10.0:
            t_print = time.perf_counter()
            print(f"serving {label}: {t_print - t0:.0f} s, submitted {k}/{len(reqs)}, "
                  f"active {na}, queued {nq}", file=sys.stderr, flush=True)
        if na == 0 and nq == 0:
            if k == len(order):
                break
            time.sleep(max(0.0, min(1e-3, t_arrive[order[k]] - (time.perf_counter() - t0))))
    return time.perf_counter() - t0, ids


def _e_F(F, ref):
    import numpy as np
    return float(np.max(np.linalg.norm(F - ref, axis=0)) / max(np.max(np.linalg.norm(ref, axis=0)), 1e-300))


def serving(sce, n_requests, loads, n_check):
    """Serving workload: independent requests (N log-uniform in [2, 8192], n_max
    in {4, 8, 16}, steps log-uniform in [100, 10^4]) with Poisson arrivals at
    each offered load x the saturated capacity, which is measured first on the
    same mix.  Per load: throughput, per-step latency (wall time of the tick
    that carried it, and the device time of the tick's kernels alone),
    admission wait, per-request energy change and the force error of sampled
    requests at completion against an FP64 context at their final state.  Once:
    the force error at admission against the FP64 oracle (the sampled requests
    run for zero steps), and the request with the largest energy change run
    again in FP64."""
    import numpy as np
    import oracle
    import workloads

    def half(n):
        return ((2 * n + 1) ** 3 - 1) // 2

    # saturated capacity: 256 requests of the same mix (steps / 10) submitted at once
    cal = workloads.serving_requests(n_requests=256, steps_range=(10, 1000), salt=1)
    with sce.Server(hbm_budget_bytes=16 << 30, precision="fp32") as srv:
        _drive(srv, cal, [0.0] * len(cal), "capacity")
        st = srv.sce_server_stats()
    capacity = st["pairs"] / st["busy_s"]
    print(f"serving capacity {capacity:.3e} pairs/s", file=sys.stderr, flush=True)

    # unit-rate Poisson arrivals, rescaled per load (the draws do not depend on the rate)
    reqs = workloads.serving_requests(n_requests=n_requests, rate_per_s=1.0)
    work = np.array([r.particles.N * half(r.particles.n_max) * (r.particles.n_steps + 1) for r in reqs],
                    dtype=np.float64)
    check = set(range(0, n_requests, max(1, n_requests // n_check)))
    rows, worst = [], None
    for load in loads:
        rate = load * capacity / float(np.mean(work))
        t_arrive = [r.arrival_s / rate for r in reqs]
        with sce.Server(hbm_budget_bytes=16 << 30, precision="fp32") as srv:
            wall, ids = _drive(srv, reqs, t_arrive, f"load {load}")
            st = srv.sce_server_stats()
            done = srv.sce_server_poll(len(reqs) + 1)
            drift, errs = [], []
            for rid in done:
                x, v, F, d0, d1 = srv.sce_server_result(rid)
                i = ids[rid]
                drift.append(abs(d1.total - d0.total) / abs(d0.total))
                if worst is None or drift[-1] > worst[0]:
                    worst = (drift[-1], i, load)
                if i in check:
                    p = reqs[i].particles
                    with sce.Context(p.L, p.n_max, p.shape, p.a) as c:
                        c.sce_set_options(p.eps0, "fp64", "kdk")
                        c.sce_set_particles(np.ascontiguousarray(x), np.ascontiguousarray(v),
                                            np.ascontiguousarray(p.q), np.ascontiguousarray(p.m))
                        errs.append(_e_F(F, c.sce_force()))
        rows.append({
            "offered_load": load,
            "arrival_rate_per_s": rate,
            "wall_s": wall,
            "pairs_per_s": st["pairs"] / wall,
            "request_steps_per_s": st["request_steps"] / wall,
            "p50_step_ms": 1e3 * st["p50_step_s"],
            "p99_step_ms": 1e3 * st["p99_step_s"],
            "max_step_ms": 1e3 * st["max_step_s"],
            "gpu_p50_step_ms": 1e3 * st["gpu_p50_step_s"],
            "gpu_p99_step_ms": 1e3 * st["gpu_p99_step_s"],
            "p50_wait_ms": 1e3 * st["p50_wait_s"],
            "p99_wait_ms": 1e3 * st["p99_wait_s"],
            "requests": int(st["requests_done"]),
            "hbm_peak_bytes": st["hbm_peak_bytes"],
            "energy_drift_rel_p50": float(np.median(drift)),
            "energy_drift_rel_max": float(np.max(drift)),
            "e_F_completion_vs_fp64_max": float(np.max(errs)),
        })
        print(f"serving load {load} done: " + json.dumps(rows[-1]), file=sys.stderr, flush=True)

    # force error at admission: the sampled requests run zero steps (one pass
    # at their initial positions) through the server, against the oracle
    sub = [reqs[i] for i in sorted(check)]
    adm = []
    with sce.Server(hbm_budget_bytes=16 << 30, precision="fp32") as srv:
        rid_of = {srv.sce_server_submit(r.particles, n_steps=0): r for r in sub}
        while True:
            na, nq = srv.sce_server_tick()
            if na == 0 and nq == 0:
                break
        for rid in srv.sce_server_poll(len(sub) + 1):
            x, v, F, d0, d1 = srv.sce_server_result(rid)
            p = rid_of[rid].particles
            ref = oracle.fields(p.positions(), p.q, p.L, p.n_max, p.shape, p.a, p.eps0)
            if p.N > 1:
                adm.append(_e_F(F, ref.F))
    # the largest energy change, run again in FP64
    drift64 = None
    p = reqs[worst[1]].particles
    with sce.Server(hbm_budget_bytes=4 << 30, precision="fp64") as srv:
        rid = srv.sce_server_submit(p)
        while True:
            na, nq = srv.sce_server_tick()
            if na == 0 and nq == 0:
                break
        x, v, F, d0, d1 = srv.sce_server_result(rid)
        drift64 = abs(d1.total - d0.total) / abs(d0.total)
    return {
        "workload": f"{n_requests} requests, N log-uniform [2, 8192], n_max in {{4, 8, 16}}, "
                    "steps log-uniform [100, 1e4], Gaussian a = 0.05, dt = 1e-3, Poisson arrivals",
        "precision": "fp32",
        "capacity_pairs_per_s": capacity,
        "loads": rows,
        "e_F_admission_vs_oracle_max": float(np.max(adm)),
        "e_F_sampled_requests": len(check),
        "worst_energy_change": {"N": p.N, "n_max": p.n_max, "steps": p.n_steps, "load": worst[2],
                                "fp32": worst[0], "fp64": drift64},
    }


# ---------------------------------------------------------------- studies
def _mode_index(n, m):
    """Canonical index of mode (m, 0, 0): the n_x = 0 block (n + n M modes), the
    n_x = 1 .. m-1 blocks (M^2 each), then n_y = -n .. -1 rows of n_x = m, then n_z = 0."""
    M = 2 * n + 1
    return n + n * M + (m - 1) * M * M + n * M + n


def _fit_omega(series, t, w_guess):
    """Least-squares frequency of a + b cos(w t) + c sin(w t): a grid over
    [0.7, 1.3] w_guess, then a bounded scalar minimisation around the best point."""
    import numpy as np
    from scipy.optimize import minimize_scalar

    def resid(w):
        A = np.stack([np.cos(w * t), np.sin(w * t), np.ones_like(t)], axis=1)
        coef, *_ = np.linalg.lstsq(A, series, rcond=None)
        return float(np.sum((A @ coef - series) ** 2))

    ws = np.linspace(0.7 * w_guess, 1.3 * w_guess, 1201)
    i = int(np.argmin([resid(w) for w in ws]))
    lo, hi = ws[max(i - 1, 0)], ws[min(i + 1, len(ws) - 1)]
    return float(minimize_scalar(resid, bounds=(lo, hi), method="bounded",
                                 options={"xatol": 1e-9 * w_guess}).x)


def study_dispersion(sce):
    """Cold-plasma oscillation of mode (m, 0, 0) on the 2^20-particle lattice
    against the discrete dispersion relation (Section 5),
    w = (2/h) asin(w_p h S(k)/2), for several m and h, and the growth factor of
    the unstable regime w_p h S / 2 > 1, where |lambda| + 1/|lambda| = (w_p h S)^2 - 2."""
    import math
    import numpy as np
    import workloads
    rows = []
    for m, h, steps in [(1, 2.5e-4, 100), (1, 5e-4, 50), (1, 1e-3, 30), (1, 1.5e-3, 24),
                        (2, 5e-4, 50), (4, 5e-4, 50), (8, 5e-4, 50)]:
        p = workloads.cold_lattice(mode=m, dt=h, n_steps=steps)
        wp = math.sqrt(p.N / p.L ** 3)
        S = math.exp(-0.5 * (2 * math.pi * m * p.a / p.L) ** 2)
        w_ref = (2.0 / h) * math.asin(wp * h * S / 2.0)
        idx = _mode_index(p.n_max, m)
        series = []
        with sce.Context.from_particles(p, precision="fp32") as c:
            for _ in range(steps):
                c.sce_step(h, 1)
                series.append(c.sce_deposit()[idx].real)
        t = h * np.arange(1, steps + 1)
        w = _fit_omega(np.array(series), t, w_ref)
        rows.append({"m": m, "h": h, "steps": steps, "wp_h_S_over_2": wp * h * S / 2,
                     "omega": w, "omega_theory": w_ref, "rel_err": w / w_ref - 1,
                     "omega_continuum": wp * S})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    # unstable: h = 2.5e-3, w_p h S / 2 = 1.28; small amplitude keeps the mode linear
    h, m = 2.5e-3, 1
    p = workloads.cold_lattice(mode=m, dt=h, amplitude=1e-4, n_steps=5)
    wp = math.sqrt(p.N / p.L ** 3)
    S = math.exp(-0.5 * (2 * math.pi * m * p.a / p.L) ** 2)
    b = (wp * h * S) ** 2 - 2.0
    lam = (b + math.sqrt(b * b - 4.0)) / 2.0
    idx = _mode_index(p.n_max, m)
    amps = []
    with sce.Context.from_particles(p, precision="fp64") as c:
        amps.append(c.sce_deposit()[idx].real)
        for _ in range(4):
            c.sce_step(h, 1)
            amps.append(c.sce_deposit()[idx].real)
    ratios = [amps[i + 1] / amps[i] for i in range(1, len(amps) - 1)]
    return {"study": "dispersion",
            "workload": "cold lattice 128x128x64 (N = 1,048,576), n_max = 32, Gaussian a = 0.01, "
                        "perturbation A cos(2 pi m x / L), A = 0.01 (1e-4 for the unstable case)",
            "precision": "fp32 (unstable case fp64)", "stable": rows,
            "unstable": {"h": h, "wp_h_S_over_2": wp * h * S / 2, "lambda_theory": -lam,
                         "step_ratios": ratios}}


def study_h2(sce):
    """Two-body problem at fixed T = 1 with h = 4e-3 .. 2.5e-4 (FP64): the largest
    energy deviation scales as h^2 (Section 6) and the largest single-step
    change as h^3."""
    import numpy as np
    import workloads
    out = []
    for h in [4e-3, 2e-3, 1e-3, 5e-4, 2.5e-4]:
        p = workloads.two_body(dt=h)
        steps = int(round(1.0 / h))
        with sce.Context.from_particles(p, precision="fp64") as c:
            E0 = c.sce_diagnostics()[0].total
            dev, step_max, prev = 0.0, 0.0, E0
            for i in range(steps):
                c.sce_step(h, 1)
                E = c.sce_diagnostics()[0].total
                step_max = max(step_max, abs(E - prev))
                dev = max(dev, abs(E - E0))
                prev = E
        out.append({"h": h, "steps": steps, "max_dE": dev, "max_step_dE": step_max, "E0": E0})
    hs = np.log([r["h"] for r in out])
    slope = float(np.polyfit(hs, np.log([r["max_dE"] for r in out]), 1)[0])
    slope1 = float(np.polyfit(hs, np.log([r["max_step_dE"] for r in out]), 1)[0])
    return {"study": "h2", "workload": "two-body, L = 1, n_max = 8, Gaussian a = 0.05, T = 1, KDK, fp64",
            "rows": out, "slope_max_dE": slope, "slope_max_step_dE": slope1}


def study_longrun(sce, steps, every=1000, precisions=("split_f16", "fp32", "fp64")):
    """Two-species neutral plasma, N = 262,144, n_max = 16, h = 1e-3: relative
    energy drift per 1,000 steps (least-squares slope over the second half of the
    run, relative to |E0| and to the mean kinetic energy there) and the largest
    momentum error, for each precision."""
    import numpy as np
    import workloads
    p = workloads.two_species()
    res = {}
    for prec in precisions:
        with sce.Context.from_particles(p, precision=prec, scheme="kdk") as c:
            d = c.sce_diagnostics()[0]
            P0 = np.array(d.momentum)
            ts, Es, Ks, perr = [0], [d.total], [d.kinetic], [0.0]
            t0 = time.perf_counter()
            for i in range(steps // every):
                c.sce_step(p.dt, every)
                d = c.sce_diagnostics()[0]
                ts.append((i + 1) * every)
                Es.append(d.total)
                Ks.append(d.kinetic)
                perr.append(float(np.max(np.abs(np.array(d.momentum) - P0)) / d.momentum_abs_sum))
                print(f"{prec} step {ts[-1]} E={d.total:.10e} K={d.kinetic:.6e} perr={perr[-1]:.2e}",
                      file=sys.stderr, flush=True)
            wall = time.perf_counter() - t0
        ts, Es, Ks = np.array(ts), np.array(Es), np.array(Ks)
        half = ts >= ts[-1] / 2
        slope = float(np.polyfit(ts[half], Es[half], 1)[0]) * 1000.0
        res[prec] = {"steps": int(ts[-1]), "ms_per_step": 1e3 * wall / max(ts[-1], 1),
                     "E0": float(Es[0]), "K0": float(Ks[0]), "K_mean_second_half": float(np.mean(Ks[half])),
                     "drift_per_1000_rel_E0": slope / abs(Es[0]),
                     "drift_per_1000_rel_Kbar": slope / float(np.mean(Ks[half])),
                     "max_dE_rel_E0": float(np.max(np.abs(Es - Es[0])) / abs(Es[0])),
                     "momentum_err_max": float(np.max(perr))}
    return {"study": "longrun",
            "workload": "two-species neutral plasma N = 262,144 (m_ion = 100), n_max = 16, Gaussian a = 0.02, "
                        "sigma_v = 0.02, h = 1e-3, KDK", "results": res}


def _energy_series(c, h, steps, every):
    """Run ``steps`` steps of size h, sampling the diagnostics every ``every``
    steps: returns (steps, E, K, W, momentum error relative to sum m|v|)."""
    import numpy as np
    d = c.sce_diagnostics()[0]
    P0 = np.array(d.momentum)
    ts, Es, Ks, Ws, perr = [0], [d.total], [d.kinetic], [d.field], [0.0]
    for i in range(steps // every):
        c.sce_step(h, every)
        d = c.sce_diagnostics()[0]
        ts.append((i + 1) * every)
        Es.append(d.total)
        Ks.append(d.kinetic)
        Ws.append(d.field)
        perr.append(float(np.max(np.abs(np.array(d.momentum) - P0)) / d.momentum_abs_sum))
    return np.array(ts), np.array(Es), np.array(Ks), np.array(Ws), np.array(perr)


def study_twod(sce, steps):
    """The paper's own two-dimensional settings (FP64, KDK), line charges in
    the unit periodic square:
    * Kepler problem (Section 6): an electron and a double positron, tent
      shapes, delta field shape, net linear momentum; at about 10 steps per
      orbit (the paper's resolution) and at 100, energy sampled every 250
      steps: relative energy deviation after the first 5% of the run (the
      transient), the kinetic and field parts, the momentum error; and the
      largest energy deviation over two orbits against h (slope 2).
    * Thermal plasma (Section 7): 16 line charges, n_max = 6 (84 modes), the
      paper's ratios L = 4 lambda_D and width 0.1 lambda_D, k_max sigma_v h = 0.1:
      energy deviation and momentum error over the run."""
    import numpy as np
    import workloads
    out = {"study": "twod"}
    p0 = workloads.kepler_2d()
    T_orbit = 2.0 * math.pi * 0.2 / math.sqrt(2.0 / (2.0 * math.pi) / (2.0 / 3.0))
    kep = []
    for per_orbit in (10, 100):
        h = T_orbit / per_orbit
        with sce.Context.from_particles(p0.with_(dt=h), precision="fp64") as c:
            t0 = time.perf_counter()
            ts, Es, Ks, Ws, perr = _energy_series(c, h, steps, 250)
            wall = time.perf_counter() - t0
        late = ts >= 0.05 * ts[-1]
        kep.append({"steps_per_orbit": per_orbit, "h": h, "steps": int(ts[-1]),
                    "orbits": float(ts[-1] / per_orbit), "ms_per_step": 1e3 * wall / ts[-1],
                    "E0": float(Es[0]),
                    "max_dE_rel": float(np.max(np.abs(Es - Es[0])) / abs(Es[0])),
                    "max_dE_rel_after_transient": float(np.max(np.abs(Es[late] - np.mean(Es[late]))) / abs(Es[0])),
                    "drift_rel_per_1e5_steps": float(np.polyfit(ts[late], Es[late], 1)[0]) * 1e5 / abs(Es[0]),
                    "K_range": [float(Ks.min()), float(Ks.max())], "W_range": [float(Ws.min()), float(Ws.max())],
                    "momentum_err_max": float(np.max(perr))})
        print(f"kepler2d {per_orbit}/orbit done", file=sys.stderr, flush=True)
    out["kepler"] = kep
    rows = []
    for per_orbit in (20, 40, 80, 160, 320):
        h = T_orbit / per_orbit
        with sce.Context.from_particles(p0.with_(dt=h), precision="fp64") as c:
            E0 = c.sce_diagnostics()[0].total
            dev = 0.0
            for _ in range(2 * per_orbit):
                c.sce_step(h, 1)
                dev = max(dev, abs(c.sce_diagnostics()[0].total - E0))
        rows.append({"h": h, "max_dE": dev})
    slope = float(np.polyfit(np.log([r["h"] for r in rows]), np.log([r["max_dE"] for r in rows]), 1)[0])
    out["kepler_h2"] = {"rows": rows, "slope": slope}
    pt = workloads.thermal_2d()
    wp = math.sqrt(pt.N / pt.L ** 2)
    h = pt.dt
    with sce.Context.from_particles(pt, precision="fp64") as c:
        ts, Es, Ks, Ws, perr = _energy_series(c, h, steps, 250)
    out["thermal"] = {"N": pt.N, "n_max": pt.n_max, "modes": (pt.n_max * 2 + 1) ** 2 // 2,
                      "omega_p_h": wp * h, "L_over_lambda_D": 4.0, "steps": int(ts[-1]),
                      "plasma_periods": float(ts[-1] * h * wp / (2 * math.pi)),
                      "E0": float(Es[0]), "max_dE_rel": float(np.max(np.abs(Es - Es[0])) / abs(Es[0])),
                      "drift_rel_per_1e5_steps": float(np.polyfit(ts, Es, 1)[0]) * 1e5 / abs(Es[0]),
                      "momentum_err_max": float(np.max(perr))}
    out["workload"] = ("kepler_2d (q = -1, m = 1 and q = +2, m = 2, r = 0.2, tent a = 0.05, n_max = 16), "
                       "thermal_2d (16 line charges, L = 4 lambda_D, Gaussian a = 0.1 lambda_D, n_max = 6, "
                       "k_max sigma_v h = 0.1), unit square, FP64 KDK")
    return out


def n16_split_steps(sce):
    """Wall time per split step of the two n_max = 16 workloads (the
    65,536-particle random plasma, the 262,144-particle two-species plasma),
    reported beside the headline line for information: 200 and 100 KDK steps
    after 10 warmup steps, no timing events."""
    import torch
    import workloads
    out = {}
    for name, p, n in (("random_plasma_65536", workloads.random_plasma(), 200),
                       ("two_species_262144", workloads.two_species(), 100)):
        with sce.Context.from_particles(p, precision="split_f16", scheme="kdk") as c:
            c.sce_step(p.dt, 10)
            c.sce_sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c.sce_step(p.dt, n)
            c.sce_sync()
            torch.cuda.synchronize()
            out[name] = round(1e3 * (time.perf_counter() - t0) / n, 5)
    return out


def study_medium(sce, steps):
    """The two n_max = 16 workloads of the longer runs: the 65,536-particle
    random plasma and the 262,144-particle two-species plasma, KDK, in every
    precision.  Wall time per step over 10 * steps (split) or 2 * steps
    (FP32, FP64) steps after 10 warmup steps, without timing events; then the
    deposit and force times from the library's events over 20 more steps."""
    import torch
    import workloads
    rows = []
    for name, p in (("random_plasma_65536_n16", workloads.random_plasma()),
                    ("two_species_262144_n16", workloads.two_species())):
        for prec in ("split_f16", "fp32", "fp64"):
            n = 10 * steps if prec == "split_f16" else 2 * steps
            with sce.Context.from_particles(p, precision=prec, scheme="kdk") as c:
                c.sce_step(p.dt, 10)
                c.sce_sync()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                c.sce_step(p.dt, n)
                c.sce_sync()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                c.sce_timing_enable(True)
                c.sce_step(p.dt, 20)
                tm = c.sce_timing_read()
                c.sce_timing_enable(False)
                H = c.sce_mode_count()
            ms = 1e3 * (t1 - t0) / n
            rows.append({"workload": name, "precision": prec, "steps": n, "ms_per_step": round(ms, 5),
                         "pairs_per_s": p.N * H / (ms * 1e-3),
                         "deposit_ms_avg": round(tm["deposit_ms"] / max(tm["deposit_launches"], 1), 5),
                         "force_ms_avg": round(tm["force_ms"] / max(tm["force_launches"], 1), 5)})
            print(f"medium study {name} {prec}: {ms:.4f} ms/step", file=sys.stderr, flush=True)
    return {"study": "medium", "rows": rows,
            "workload": "random_plasma (N = 65,536, n_max = 16, a = 0.02) and two_species "
                        "(N = 262,144, n_max = 16, m_ion = 100), KDK"}


def study_tent(sce, steps, warmup, precisions):
    """Finite-width (tent) field shapes at the size of the headline workload:
    N = 1,048,576 point charges uniform in [-L/4, L/4]^3, n_max = 32 (the
    274,625-mode cube, origin included, 137,313 stored), KDK, dt = 1e-3.  Per
    precision: wall time per step and the deposit and force kernel times, next
    to the periodic delta-field step of the cold lattice at the same N and
    n_max; the difference is the tent solve, the envelope and the combine.
    Energy and momentum change over the run (FP64 diagnostics)."""
    import numpy as np
    import workloads
    pt = workloads.tent_plasma(N=1 << 20, n_max=32, dim=3)
    pd = workloads.cold_lattice()
    rows = []
    for prec in precisions:
        for field, p in (("tent", pt), ("delta", pd)):
            r = time_path(sce, p, prec, steps, warmup)
            rows.append({"field": field, "precision": prec,
                         "ms_per_step": round(r["ms_per_step"], 4),
                         "deposit_ms_avg": round(r["deposit_ms_avg"], 4),
                         "force_ms_avg": round(r["force_ms_avg"], 4),
                         "pairs_per_s": r["pairs_per_s"], "modes_stored": r["modes_half"]})
            print(f"tent study {field} {prec} done", file=sys.stderr, flush=True)
    cons = {}
    with sce.Context.from_particles(pt, precision="split_f16") as c:
        d0, _ = c.sce_diagnostics()
        c.sce_step(pt.dt, 200)
        d1, _ = c.sce_diagnostics()
    cons = {"steps": 200, "E0": d0.total, "dE_rel": abs(d1.total - d0.total) / abs(d0.total),
            "dP_rel": float(np.linalg.norm(d1.momentum - d0.momentum) / d0.momentum_abs_sum)}
    return {"study": "tent", "rows": rows, "split_f16_conservation": cons,
            "workload": "tent_plasma N=1048576 n_max=32 3-D in [-L/4, L/4]^3 (tent field, point particles) "
                        "vs cold_lattice_128x128x64_n32 (delta field, Gaussian a = 0.01)"}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_paper_baseline(p, sample):
    """The FP64 CPU program with the paper's own optimisations of the mode sums
    (Section 8: the half space, and D = 3 exponentials per particle whose
    integer powers give every phase), on every thread and on one: one deposit,
    solve and force pass of a sample of the particles against all modes."""
    import numpy as np
    import oracle
    from oracle import cpu_paper
    modes = oracle.half_modes(p.n_max)
    S = oracle.shape(p.shape, p.a, oracle.wave_vectors(modes, p.L))

    def one(n):
        idx = np.arange(0, p.N, max(1, p.N // n))[:n]
        sub = p.subset(idx)
        t0 = time.perf_counter()
        rho = cpu_paper.deposit(sub.positions(), sub.q, p.L, p.n_max, S)
        ps = oracle.psi(rho, p.L, modes, p.eps0, p.shape, p.a)
        cpu_paper.force(sub.positions(), sub.q, p.L, p.n_max, ps)
        t = time.perf_counter() - t0
        return len(idx) * len(modes) / t, len(idx), t

    threads = cpu_paper.threads()
    rate, n_all, t_all = one(sample)
    cpu_paper.set_threads(1)
    try:
        rate1, n_one, t_one = one(max(64, sample // max(threads, 1)))
    finally:
        cpu_paper.set_threads(threads)
    return {"value": rate, "unit": "pairs/s", "cores": threads,
            "kind": "paper-optimized CPU program (Section 8 per-axis powers, FP64, AVX2 + OpenMP)",
            "sample": f"{n_all} of {p.N} particles x all {len(modes)} half-space modes, "
                      f"one deposit + solve + force pass ({t_all:.1f} s)",
            "value_1core": rate1,
            "sample_1core": f"{n_one} particles x all modes ({t_one:.1f} s)"}


def cpu_baseline(p, sample, paper_sample=0):
    """The FP64 oracle on the host: one deposit and one force pass of a sample
    of the particles against all modes, on every thread it uses by default and
    on one thread (a smaller sample; the rate of a direct double loop does not
    depend on the sample size).  With paper_sample > 0, the faster CPU program
    with the paper's per-axis powers is timed too ("paper_optimized")."""
    import numpy as np
    import oracle
    modes = oracle.half_modes(p.n_max)

    def one(n):
        idx = np.arange(0, p.N, max(1, p.N // n))[:n]
        sub = p.subset(idx)
        t0 = time.perf_counter()
        rho = oracle.deposit(sub.positions(), sub.q, p.L, modes, p.shape, p.a)
        ps = oracle.psi(rho, p.L, modes, p.eps0, p.shape, p.a)
        oracle.force_from_psi(sub.positions(), sub.q, p.L, modes, ps)
        t = time.perf_counter() - t0
        return len(idx) * len(modes) / t, len(idx), t

    threads = oracle.threads()
    rate, n_all, t_all = one(sample)
    oracle.set_threads(1)
    try:
        rate1, n_one, t_one = one(max(64, sample // max(threads, 1)))
    finally:
        oracle.set_threads(threads)
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"value": rate, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_all} of {p.N} particles x all {len(modes)} half-space modes, "
                      f"one deposit + one force pass ({t_all:.1f} s)",
            "value_1core": rate1,
            "sample_1core": f"{n_one} particles x all modes, one deposit + one force pass ({t_one:.1f} s)",
            "nproc": os.cpu_count(), "affinity_cpus": affinity, "cpu_model": _cpu_model(),
            **({"paper_optimized": cpu_paper_baseline(p, paper_sample)} if paper_sample > 0 else {})}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU "
              "particle-sharded path is a design, not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads
    import paper_1508_07344_amd as sce

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if a.study:
        if a.study == "longrun":
            r = study_longrun(sce, a.long_steps, precisions=[x for x in a.long_precisions.split(",") if x])
        elif a.study == "dispersion":
            r = study_dispersion(sce)
        elif a.study == "twod":
            r = study_twod(sce, a.twod_steps)
        elif a.study == "tent":
            r = study_tent(sce, a.steps, a.warmup, [x for x in a.tent_precisions.split(",") if x])
        elif a.study == "medium":
            r = study_medium(sce, a.steps)
        else:
            r = study_h2(sce)
        print(json.dumps(r), flush=True)
        return
    if a.copy_calibration:
        n = a.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": 4 * n, "launches": 5}), flush=True)
        return
    p = workloads.cold_lattice()
    main_r = time_path(sce, p, a.precision, a.steps, a.warmup)
    print(f"timed {a.precision}: {main_r['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    variants = {}
    for prec in [x for x in a.also.split(",") if x and x != a.precision]:
        variants[prec] = time_path(sce, p, prec, a.steps, a.warmup)
        print(f"timed {prec}: {variants[prec]['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    peaks = measure_peaks() if a.peaks else None
    for prec in variants:
        variants[prec]["roofline"] = roofline(variants[prec], p.N, peaks)
    line = {
        "metric": METRIC,
        "value": main_r["pairs_per_s"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[a.precision],
        "data": "synthetic",
        "config": {"workload": "cold_lattice_128x128x64_n32", "N": p.N, "n_max": p.n_max,
                   "modes_half": main_r["modes_half"], "shape": "gaussian", "a": p.a,
                   "dt": p.dt, "scheme": "kdk", "precision": a.precision},
        "roofline": roofline(main_r, p.N, peaks),
        "detail": {k: v for k, v in main_r.items() if k not in ("precision",)},
        "variants": variants,
    }
    if peaks:
        line["peaks_measured_tflops"] = peaks
    if a.n16:
        line["n16_split_ms_per_step"] = n16_split_steps(sce)
    if a.serve_requests:
        line["serving"] = serving(sce, a.serve_requests,
                                  [float(x) for x in a.serve_loads.split(",") if x], a.serve_check)
    if a.cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p, a.cpu_sample, a.cpu_paper_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
