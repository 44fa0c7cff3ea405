#!/usr/bin/env python3
"""Throughput of nested slice sampling on one MI355X.

A step is one "replace the k lowest" iteration of the sampler over the whole
live population: bit-exact selection of the k lowest, evidence and
prior-volume update, covariance tuning, k constrained slice chains whose
every probe is a fused TaylorF2 + Whittle likelihood, refill and the
termination test.  The default workload is the 3-detector, 11-parameter,
4017-bin full-grid problem (n_live 1000, n_delete 500, 55 slice steps) in
double precision, on synthetic data.

Prints one JSON line: likelihood evaluations/s over K timed iterations (after
W warm-up iterations), seconds per complete run, the roofline of the
dominant kernel (the slice-chain kernel) and the oracle timed on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X vector units: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz
LANE_OPS = 256 * 4 * 16 * 2.4e9            # 39.3e12 lane-instructions/s
FP64_PEAK_TFLOPS = 2 * LANE_OPS / 1e12     # FMA: 78.6 TFLOP/s
FP32_PEAK_TFLOPS = 4 * LANE_OPS / 1e12     # packed FMA: 157.3 TFLOP/s
# single-precision sine/cosine on the transcendental unit: half rate on gfx950,
# 19.7 Tops/s (the rate probe, `bench.py --unit-rates`, measures 8.3 cycles per
# wave64 instruction, dependent or not, against 4.3 for a double FMA)
TRANS_PEAK_TOPS = LANE_OPS / 2 / 1e12
SINCOS_FLOPS = 44                # flops of the double-precision sincos in cycles
PHASE_FLOPS = 24                 # per (probe, bin): PN phase series, shared by the detectors
DET_FLOPS = 2 + SINCOS_FLOPS + 8 # per (probe, bin, detector): delay, sincos, complex accumulate
# relative binning per (probe, edge read): the phase (24) and per detector
# delay, sincos and the complex ratio (2 + sincos + 6); per (probe, active
# coarse bin, detector) the linear-model terms (27).  A probe reads the edges
# of its active bins, one more than the bins, so the bins are counted per edge
# as (edges - probes) / edges of it
RB_EDGE_DET = 2 + SINCOS_FLOPS + 6
RB_BIN_DET = 27
# the batched relative-binning kernel sums the same linear model per edge:
# per (probe, edge, detector) |r|^2, Re(conj(r_prev) r), Re(W r), the G and E
# terms and the accumulation (15) replace the per-bin terms
RB_EDGE_FORM_DET = 15

_GRID2 = "3-detector aligned-spin TaylorF2 (11 parameters), 4017 bins/detector (20-1024 Hz, df 0.25 Hz), network SNR 20"
WORKLOADS = {
    "tf2_3det": _GRID2 + ", full-grid Whittle, n_live 1000, n_delete 500, 55 slice steps, FP64",
    "tf2_1det": "1-detector TaylorF2 (4 parameters), full-grid Whittle, 473 bins (20-256 Hz, df 0.5 Hz), "
            "SNR 15, n_live 500, n_delete 250, 20 slice steps, FP64",
    "tf2_3det_rb": _GRID2 + ", relative binning (128 geometric bins), n_live 1000, n_delete 500, 55 slice steps, FP64",
    "tf2_3det_mixed": _GRID2 + ", full-grid Whittle, n_live 2000, n_delete 1000, 55 slice steps, mixed precision",
    "tf2_3det_rb_mixed": _GRID2 + ", relative binning (128 bins), n_live 2000, n_delete 1000, 55 slice steps, mixed precision",
    "tf2_3det_n2000": _GRID2 + ", full-grid Whittle, n_live 2000, n_delete 1000, 55 slice steps, FP64",
    "tf2_3det_rb_n2000": _GRID2 + ", relative binning (128 bins), n_live 2000, n_delete 1000, 55 slice steps, FP64",
    "tf2_3det_so": "3-detector aligned-spin TaylorF2 with the spin-orbit phase terms through 3.5PN (11 parameters), "
                   "4017 bins/detector (20-1024 Hz, df 0.25 Hz), network SNR 20, full-grid Whittle, n_live 1000, "
                   "n_delete 500, 55 slice steps, FP64",
    "tf2_3det_rb_walk": _GRID2 + ", relative binning (128 bins), n_live 1000, n_delete 500, random-walk chains "
                        "(differential-evolution proposals, 60 accepted per chain), FP64",
    "tf2_3det_rb_paper": _GRID2 + ", relative binning (128 bins), the paper's settings: n_live 3000, n_delete 1500, "
                         "110 slice steps (10 per dimension), phase, polarisation and right ascension wrapped, FP64",
    "scaling": "runtime of complete tf2_3det_rb runs against n_live at n_delete = n_live/2 and against n_delete "
               "at n_live 1000",
    "coverage": "seed-to-seed scatter of log Z against the sampler's error bar, at chains of 5, 10 and 20 steps per "
                "dimension, for tf2_3det and serving events 28 and 51, and at the paper's settings",
    "serving": "64 Poisson-arriving events, 4/8/16/32 s (4017-32129 bins per detector), 1-3 detectors, "
            "SNR U[8,40], Mc U[5,60], q U[0.125,1], 11 parameters, n_live U{500,1000,2000}, n_delete n_live/2, "
            "full-grid Whittle",
}


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def op_mix(w, bins_per_edge=None, edge_form=False):
    """Algorithmic work of one counted term (full grid: one active bin of one
    probe; relative binning: one edge read by one probe, with bins_per_edge
    active coarse bins per edge, by default nb/(nb+1)) as (double-precision
    flops, single-precision flops, single-precision transcendental ops).
    The mixed form keeps the phase, the delay and the cycle reduction in
    double (4 flops per detector) and takes sin and cos on the transcendental
    unit.  edge_form: the relative-binning linear model summed per edge (the
    batched kernel) instead of per bin (the chain kernel)."""
    from paper_2509_24949_amd import synth

    nd = w.n_det
    if w.likelihood == synth.LIKE_RB:
        bpe = w.rb_n_bins / (w.rb_n_bins + 1) if bins_per_edge is None else bins_per_edge
        bins = nd * (RB_EDGE_FORM_DET if edge_form else RB_BIN_DET * bpe)
        if w.precision == 1:
            return PHASE_FLOPS + 4 * nd, 6 * nd + bins, 2 * nd
        return PHASE_FLOPS + nd * RB_EDGE_DET + bins, 0.0, 0.0
    if w.precision == 1:
        return PHASE_FLOPS + 4 * nd, 8 * nd, 2 * nd
    return PHASE_FLOPS + nd * DET_FLOPS, 0.0, 0.0


def seconds_per_term(w, bins_per_edge=None, edge_form=False) -> float:
    """Shortest time the vector units need for one term of this workload."""
    f64, f32, tr = op_mix(w, bins_per_edge, edge_form)
    return (f64 / FP64_PEAK_TFLOPS + f32 / FP32_PEAK_TFLOPS + tr / TRANS_PEAK_TOPS) * 1e-12


def flops_per_term(w, bins_per_edge=None, edge_form=False) -> float:
    """Algorithmic operations per counted term (all kinds together)."""
    return sum(op_mix(w, bins_per_edge, edge_form))


def bins_per_edge(terms: int, probes: int) -> float:
    """Active coarse bins per edge read, from a batch's totals: each probe
    reads one edge more than it has active bins (a probe with no active bin
    reads none, so this errs low)."""
    return max(terms - probes, 0) / terms if terms > 0 else 0.0


def peak_tflops(w, bins_per_edge=None, edge_form=False) -> float:
    """Rate of the vector units on this workload's operation mix: its
    operations over the shortest time the units need for them (double FMA at
    78.6 TFLOP/s, packed single FMA at 157.3, transcendentals at 19.7 Tops/s).
    Equals the double-precision peak for the double-precision forms."""
    f64, f32, tr = op_mix(w, bins_per_edge, edge_form)
    t = f64 / FP64_PEAK_TFLOPS + f32 / FP32_PEAK_TFLOPS + tr / TRANS_PEAK_TOPS
    return (f64 + f32 + tr) / t


def cpu_baseline(name: str, seconds: float, threads: int):
    """The oracle as it stands, on the host cores: NS iterations of the same
    workload until about `seconds` of work; likelihood evaluations/s."""
    import oracle
    from paper_2509_24949_amd import synth

    w = synth.workload(name)
    re, im = oracle.make_data(w)
    prob = oracle.OracleProblem(w, re, im)
    run = oracle.Run(prob, oracle.opts_for(w, n_threads=threads, term_frac=0.0, max_iter=200))
    e0 = run.state()["n_evals"]
    t0 = time.perf_counter()
    iters = 0
    while time.perf_counter() - t0 < seconds and iters < 50:
        run.step(1)
        iters += 1
    dt = time.perf_counter() - t0
    ev = run.state()["n_evals"] - e0
    # one host thread on every 16th probe of the standalone batch
    u = synth.proposal_batch(w, 65536, seed=77)[::16]
    t1 = time.perf_counter()
    prob.loglike_batch(u, 1)
    dt1 = time.perf_counter() - t1
    return {"value": ev / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{iters} sampler iterations of the same workload from its initial population "
                      f"({ev} likelihood evaluations in {dt:.1f} s, OpenMP over chains)",
            "single_thread_batch": {"value": len(u) / dt1, "unit": "evals/s", "cores": 1,
                                    "sample": f"every 16th of the standalone batch's 65536 probes ({len(u)} probes "
                                              f"in {dt1:.2f} s)"},
            "host": host_info()}


def _pct(x, q):
    import numpy as np

    return float(np.percentile(np.asarray(x, dtype=float), q))


_SERVING_DATA = {}


def serving(args, precision_name=None) -> dict:
    """Serving benchmark: the events run one at a time (service times), then
    arrive as a Poisson process at twice the sequential service rate and are
    served by the packed scheduler.  Time-to-posterior runs from an event's
    arrival to its evidence (log Z with its spread) being ready on the host."""
    import numpy as np
    import torch

    from paper_2509_24949_amd import binding, synth

    n_ev = args.events
    precision_name = precision_name or args.precision
    precision = 1 if precision_name == "mixed" else 0
    events = [synth.serving_event(i) for i in range(n_ev)]
    for w in events:
        w.precision = precision
    if n_ev not in _SERVING_DATA:        # the data do not depend on the precision
        log(f"bench: serving: building data of {n_ev} events")
        specs = []
        for w in events:
            re, im = binding.make_data(w)
            specs.append(binding.ProblemSpec(w, re, im))
        _SERVING_DATA[n_ev] = specs
    specs = _SERVING_DATA[n_ev]
    opts = [binding.opts_for(w, max_iter=args.max_iter) for w in events]

    # warm-up: load every code object the two modes use
    for mode in ("seq", "srv"):
        w = synth.serving_event(0)
        w.precision = precision
        o = binding.opts_for(w, max_iter=2)
        if mode == "seq":
            r = binding.Run(specs[0], o)
            r.run(5)
            r.logZ(200)
            r.close()
        else:
            srv = binding.Server(max_runs=2)
            t = srv.submit(specs[0], o)
            while not srv.poll():
                srv.tick(1)
            srv.take(t).close()
            srv.close()
    torch.cuda.synchronize()

    # sequential: one event at a time, back to back
    service, seq_logz, seq_evals = [], [], 0
    seq_flops = 0.0
    t_all = time.perf_counter()
    for i, (spec, o) in enumerate(zip(specs, opts)):
        t0 = time.perf_counter()
        r = binding.Run(spec, o)
        r.run(args.max_iter)
        z = r.logZ(200)
        st = r.state()
        stats = r.stats()
        r.close()
        service.append(time.perf_counter() - t0)
        seq_logz.append((z["logZ"], z["sigma"]))
        seq_evals += st["n_evals"]
        seq_flops += stats["bin_terms"] * flops_per_term(events[i])
    seq_makespan = time.perf_counter() - t_all
    rate = args.load * n_ev / sum(service)
    arrivals = synth.serving_arrivals(n_ev) / rate
    # the same arrivals served first-in first-out by the sequential runs
    fin, seq_lat = 0.0, []
    for a, s in zip(arrivals, service):
        fin = max(fin, a) + s
        seq_lat.append(fin - a)
    seq_span = fin - arrivals[0]
    log(f"bench: sequential: {sum(service):.2f} s of service for {n_ev} events; arrival rate {rate:.2f}/s")

    # served: arrivals in real time, packed ticks in between
    stream = torch.cuda.Stream()
    srv = binding.Server(max_runs=args.max_runs, graph=args.graph, stream=stream.cuda_stream)
    t0 = time.perf_counter()
    nxt, tickets, lat, srv_logz = 0, {}, {}, {}
    srv_evals, srv_flops, srv_tmin, ticks = 0, 0.0, 0.0, 0
    while len(lat) < n_ev:
        now = time.perf_counter() - t0
        while nxt < n_ev and arrivals[nxt] <= now:
            tickets[srv.submit(specs[nxt], opts[nxt])] = nxt
            nxt += 1
        info = srv.info()
        if info["running"] == 0 and info["queued"] == 0:
            time.sleep(max(0.0, min(arrivals[nxt] - now, 0.05)) if nxt < n_ev else 0.0)
            continue
        srv.tick(args.tick_iters)
        ticks += 1
        for inf in srv.poll():
            i = tickets[inf["ticket"]]
            if inf["status"] != 0:
                raise RuntimeError(f"event {i} failed to start: status {inf['status']}")
            r = srv.take(inf["ticket"])
            z = r.logZ(200)
            st = r.state()
            stats = r.stats()
            r.close()
            lat[i] = time.perf_counter() - t0 - arrivals[i]
            srv_logz[i] = (z["logZ"], z["sigma"])
            srv_evals += st["n_evals"]
            srv_flops += stats["bin_terms"] * flops_per_term(events[i])
            srv_tmin += stats["bin_terms"] * seconds_per_term(events[i])
    span = time.perf_counter() - t0
    srv.close()
    # capacity: every event submitted at once
    srv = binding.Server(max_runs=args.max_runs, graph=args.graph, stream=stream.cuda_stream)
    t1 = time.perf_counter()
    tickets_all = {srv.submit(specs[i], opts[i]): i for i in range(n_ev)}
    sat_lat = {}
    while len(sat_lat) < n_ev:
        srv.tick(args.tick_iters)
        for inf in srv.poll():
            i = tickets_all[inf["ticket"]]
            if inf["status"] != 0:
                raise RuntimeError(f"event {i} failed to start: status {inf['status']}")
            r = srv.take(inf["ticket"])
            r.logZ(200)
            r.close()
            sat_lat[i] = time.perf_counter() - t1
    sat_span = time.perf_counter() - t1
    srv.close()
    lat_v = [lat[i] for i in range(n_ev)]
    dz = [abs(srv_logz[i][0] - seq_logz[i][0]) / max(1e-9, math.hypot(srv_logz[i][1], seq_logz[i][1]))
          for i in range(n_ev)]
    log(f"bench: served {n_ev} events in {span:.2f} s over {ticks} ticks; p50 {_pct(lat_v, 50):.2f} s, "
        f"p99 {_pct(lat_v, 99):.2f} s")
    peak = srv_flops / srv_tmin / 1e12       # the events' operation mix at the unit rates
    achieved = srv_flops / span / 1e12
    out = {
        "metric": "events/hour",
        "value": n_ev / span * 3600.0,
        "unit": "events/hour",
        "n_gpus": 1,
        "steps": n_ev,
        "warmup": 1,
        "ms_per_step": span / n_ev * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if precision else "f64",
        "data": "synthetic (seeded Gaussian noise plus injected TaylorF2 signals; no real detector data)",
        "config": {"workload": f"serving: {WORKLOADS['serving']}", "events": n_ev, "max_runs": args.max_runs,
                   "tick_iters": args.tick_iters, "graph": bool(args.graph), "load": args.load,
                   "precision": precision_name},
        "latency_p50_s": _pct(lat_v, 50),
        "latency_p99_s": _pct(lat_v, 99),
        "makespan_s": span,
        "evals_per_s": srv_evals / span,
        "sequential": {"events_per_hour": n_ev / seq_span * 3600.0, "latency_p50_s": _pct(seq_lat, 50),
                       "latency_p99_s": _pct(seq_lat, 99), "service_s": sum(service),
                       "back_to_back_events_per_hour": n_ev / seq_makespan * 3600.0,
                       "evals_per_s": seq_evals / sum(service),
                       "note": "measured service time of each event run alone; latencies are those service "
                               "times queued first-in first-out at the same arrival times"},
        "saturated": {"events_per_hour": n_ev / sat_span * 3600.0, "makespan_s": sat_span,
                      "latency_p50_s": _pct(list(sat_lat.values()), 50),
                      "latency_p99_s": _pct(list(sat_lat.values()), 99),
                      "note": "every event submitted at time zero: the server's capacity"},
        "logZ_served_vs_sequential": {"max_abs_over_sigma": max(dz), "median_abs_over_sigma": _pct(dz, 50),
                                      "within_2_sigma": bool(max(dz) <= 2.0),
                                      "events_beyond_2_sigma": int(sum(1 for v in dz if v > 2.0))},
        "roofline": {"bound": "alu", "kernel": "whole serving loop (algorithmic flops over the makespan)",
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": None},
    }
    return out


SCALING_N = (250, 500, 1000, 2000, 4000)       # n_live at n_delete = n_live / 2
SCALING_K = (1, 10, 100, 500, 999)              # n_delete at n_live = 1000


def scaling(args) -> dict:
    """Runtime of complete runs against the population and against the
    number deleted per iteration (the paper's runtime figure, Section 3), on
    the relative-binning workload: one complete run per point, from ns_init
    to the evidence, after a warm-up run; the oracle times the smallest
    population on the host threads."""
    import torch

    from paper_2509_24949_amd import binding, synth

    w = synth.workload("tf2_3det_rb")
    log("bench: scaling: building data (library-injected waveform)")
    re, im = binding.make_data(w)
    spec = binding.ProblemSpec(w, re, im)
    r = binding.Run(spec, binding.opts_for(w, n_live=250, n_delete=125, max_iter=3))
    r.run(3)
    r.close()
    points = []
    grid = [(n, n // 2) for n in SCALING_N] + [(1000, k) for k in SCALING_K if k != 500]
    for n, k in grid:
        max_iter = int(60 * n / k) + 200
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = binding.Run(spec, binding.opts_for(w, n_live=n, n_delete=k, max_iter=max_iter))
        # iterations are enqueued in chunks of about two e-folds of prior
        # volume, so that few run past termination
        chunk, done, it = max(4, (2 * n) // k), False, 0
        while not done and it < max_iter:
            done = r.step(min(chunk, max_iter - it))
            it += chunk
        z = r.logZ(200)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = r.state()
        r.close()
        points.append({"n_live": n, "n_delete": k, "s_per_run": dt, "iterations": st["iter"],
                       "evals": st["n_evals"], "evals_per_s": st["n_evals"] / dt, "logZ": z["logZ"],
                       "sigma_logZ": z["sigma"], "terminated": bool(done)})
        log(f"bench: scaling n_live {n} n_delete {k}: {dt:.3f} s, {st['iter']} iterations, "
            f"{st['n_evals'] / dt / 1e6:.0f} M evals/s, logZ {z['logZ']:.3f} +- {z['sigma']:.3f}")
    out = {"metric": "s/run", "value": next(p["s_per_run"] for p in points if p["n_live"] == 1000
                                              and p["n_delete"] == 500),
           "unit": "s", "n_gpus": 1, "steps": len(points), "warmup": 1, "higher_is_better": False,
           "scaling": "strong", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded Gaussian noise plus an injected TaylorF2 signal; no real detector data)",
           "config": {"workload": f"scaling: {WORKLOADS['scaling']}", "likelihood": "relative binning (128 bins)",
                      "n_steps": w.n_steps},
           "points": points}
    if not args.no_cpu_baseline:
        import oracle

        threads = min(16, os.cpu_count() or 1)
        n, k = SCALING_N[0], SCALING_N[0] // 2
        log(f"bench: scaling: the oracle's complete run at n_live {n} on {threads} host threads")
        ore, oim = oracle.make_data(w)
        prob = oracle.OracleProblem(w, ore, oim)
        t0 = time.perf_counter()
        ro = oracle.Run(prob, oracle.opts_for(w, n_threads=threads, n_live=n, n_delete=k, max_iter=400))
        ro.run(400)
        dt = time.perf_counter() - t0
        st = ro.state()
        out["cpu_baseline"] = {"value": dt, "unit": "s/run", "cores": threads, "kind": "oracle",
                               "sample": f"one complete run at n_live {n}, n_delete {k} ({st['iter']} iterations, "
                                         f"{st['n_evals']} likelihood evaluations, OpenMP over chains)"}
    return out


COVERAGE_STEPS = (5, 10, 20)     # slice steps per dimension
COVERAGE_SEEDS = 8


def coverage(args) -> dict:
    """Does the evidence error bar cover the run-to-run scatter?  For each
    workload and chain length, COVERAGE_SEEDS complete runs with different
    sampler seeds: the standard deviation of their log Z over the mean of
    their error bars (the spread of log Z over prior-volume replicas) should
    be about one when the chains are long enough to decorrelate."""
    import numpy as np
    import torch

    from paper_2509_24949_amd import binding, synth

    cases = [("tf2_3det", synth.workload("tf2_3det")), ("event/28", synth.serving_event(28)),
             ("event/51", synth.serving_event(51))]
    rows = []

    def runs(name, w, spec, n_steps):
        zs, sig, secs = [], [], []
        for s in range(COVERAGE_SEEDS):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = binding.Run(spec, binding.opts_for(w, seed=w.sampler_seed + 100 + s, n_steps=n_steps, max_iter=400))
            r.run(400)
            z = r.logZ(200)
            secs.append(time.perf_counter() - t0)
            r.close()
            zs.append(z["logZ"])
            sig.append(z["sigma"])
        sd, ms = float(np.std(zs, ddof=1)), float(np.mean(sig))
        row = {"workload": name, "n_live": w.n_live, "n_delete": w.n_delete, "steps_per_dim": n_steps // w.n_dim,
               "seeds": COVERAGE_SEEDS, "logZ_mean": float(np.mean(zs)), "logZ_std": sd, "sigma_mean": ms,
               "std_over_sigma": sd / ms, "s_per_run": float(np.median(secs)), "logZ": zs}
        log(f"bench: coverage {name} m = {n_steps // w.n_dim} d: log Z {row['logZ_mean']:.3f}, std {sd:.3f}, "
            f"sigma {ms:.3f}, ratio {sd / ms:.2f}, {row['s_per_run']:.3f} s/run")
        rows.append(row)

    for name, w in cases:
        re, im = binding.make_data(w)
        spec = binding.ProblemSpec(w, re, im)
        for k in COVERAGE_STEPS:
            runs(name, w, spec, k * w.n_dim)
    w = synth.workload("tf2_3det_rb_paper")
    re, im = binding.make_data(w)
    runs("tf2_3det_rb_paper", w, binding.ProblemSpec(w, re, im), w.n_steps)
    return {"metric": "std(log Z) / mean(sigma)", "unit": "ratio", "n_gpus": 1, "higher_is_better": False,
            "dtype": "f64", "data": "synthetic", "config": {"workload": f"coverage: {WORKLOADS['coverage']}"},
            "rows": rows}


# stored complete oracle runs (tests/golden/full_runs.json) with the same
# seeds as a workload, where the key differs from the workload's name
GOLDEN_RUN = {"tf2_3det_n2000": "tf2_3det_n2000_fp64"}
PAIRED_SEEDS = 32
# (workload, its probes' stored oracle values, stored oracle run to compare
# the complete run with): the configurations the error is reported for
ACCURACY_CONFIGS = (
    ("tf2_1det", "tf2_1det", "tf2_1det"),
    ("tf2_3det", "tf2_3det", "tf2_3det"),
    ("tf2_3det_rb", "tf2_3det_rb", "tf2_3det_rb"),
    ("tf2_3det_mixed", "tf2_3det", "tf2_3det_n2000_fp64"),
    ("tf2_3det_rb_mixed", "tf2_3det_rb", "tf2_3det_rb_n2000_fp64"),
)


def accuracy() -> dict:
    """Error against the double-precision oracle per configuration, from the
    oracle's stored values (tests/golden): the log-likelihood ratio on 512
    seeded probes (all, and the half around the injection), and the complete
    run's log Z against the stored oracle run of the same event and
    population in double precision (same seeds: identical runs in double
    precision; independent runs in the mixed form, so |d log Z| is also given
    in units of the two runs' combined sigma).  Each side injects the signal
    into the same seeded noise with its own waveform code.  Also the
    relative-binning likelihood against the full grid on 4096 probes around
    the injection and on equal-weight posterior draws, both on the GPU."""
    import numpy as np
    import torch

    from paper_2509_24949_amd import binding, synth

    gdir = os.path.join(ROOT, "tests", "golden")
    with open(os.path.join(gdir, "loglike_samples.json")) as fh:
        samples = json.load(fh)
    with open(os.path.join(gdir, "full_runs.json")) as fh:
        runs = json.load(fh)
    out = {}
    for name, lam_key, run_key in ACCURACY_CONFIGS:
        w = synth.workload(name)
        spec = binding.ProblemSpec(w, *binding.make_data(w))
        r = binding.Run(spec, binding.opts_for(w))
        n = samples["n_probes"]
        u = torch.from_numpy(synth.proposal_batch(w, n, seed=samples["seed"])).cuda()
        lam = torch.empty(n, dtype=torch.float64, device="cuda")
        r.loglike(u, lam)
        torch.cuda.synchronize()
        d = np.abs(lam.cpu().numpy() - np.asarray(samples[lam_key]))
        row = {"probes": n, "max_abs_dlogl": float(d.max()), "max_abs_dlogl_near_injection": float(d[: n // 2].max()),
               "median_abs_dlogl": float(np.median(d))}
        assert r.run(1000)
        z = r.logZ(200)
        if name == "tf2_3det":     # equal-weight posterior draws for the relative-binning comparison
            idx, _ = r.resample(4096)
            u_all = np.concatenate([r.dead()["u"], r.live()[0]])
            u_post = u_all[idx]
        r.close()
        g = runs.get(run_key)
        if g:
            dz = abs(z["logZ"] - g["logZ"])
            row.update({"logZ": z["logZ"], "sigma_logZ": z["sigma"], "logZ_oracle": g["logZ"], "oracle_run": run_key,
                        "abs_dlogZ": dz, "abs_dlogZ_over_sigma": dz / math.hypot(z["sigma"], g["sigma"])})
        if w.precision == 1:
            # one mixed run is one draw of a stochastic estimate whose seed-to-seed
            # scatter exceeds its prior-volume sigma; the evidence is compared over
            # paired seeds with the double-precision GPU runs, which reproduce the
            # oracle's runs of the same seeds
            diffs = []
            for sd in range(PAIRED_SEEDS):
                zz = []
                for prec in (1, 0):
                    rr = binding.Run(spec, binding.opts_for(w, seed=7100 + sd, precision=prec))
                    assert rr.run(1000)
                    zz.append(rr.logZ(200)["logZ"])
                    rr.close()
                diffs.append(zz[0] - zz[1])
            dd = np.asarray(diffs)
            row["paired_seeds_vs_double"] = {"seeds": PAIRED_SEEDS, "mean_dlogZ": float(dd.mean()),
                                             "stderr": float(dd.std(ddof=1) / math.sqrt(len(dd))),
                                             "seed_to_seed_sd": float(dd.std(ddof=1))}
        out[name] = row
    # relative binning against the full grid, both on the GPU: on 4096
    # equal-weight posterior draws of the complete tf2_3det run, and on 4096
    # probes scattered around the injection (0.02 of the cube)
    w_full, w_rb = synth.workload("tf2_3det"), synth.workload("tf2_3det_rb")
    re, im = binding.make_data(w_full)
    sets = {"posterior_draws": u_post, "near_injection": synth.proposal_batch(w_full, 4096, seed=99, frac_local=1.0)}
    runs_ = [binding.Run(binding.ProblemSpec(w, re, im), binding.opts_for(w)) for w in (w_full, w_rb)]
    for key, uu in sets.items():
        u = torch.from_numpy(np.ascontiguousarray(uu)).cuda()
        vals = []
        for r in runs_:
            lam = torch.empty(len(uu), dtype=torch.float64, device="cuda")
            r.loglike(u, lam)
            torch.cuda.synchronize()
            vals.append(lam.cpu().numpy())
        d = np.abs(vals[1] - vals[0])
        out[f"rb_vs_full_{key}"] = {"probes": len(uu), "max_abs_dlogl": float(d.max()),
                                    "median_abs_dlogl": float(np.median(d)),
                                    "logl_range": [float(vals[0].min()), float(vals[0].max())]}
    for r in runs_:
        r.close()
    return out


def unit_rates():
    """The vector-unit rate probe's JSON (None if it is not built)."""
    import subprocess

    exe = os.path.join(ROOT, "paper_2509_24949_amd", "unit_rates")
    if not os.path.exists(exe):
        return None
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    return json.loads(res.stdout) if res.returncode == 0 else None


def host_info() -> dict:
    """The host the CPU baseline ran on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = None
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def standalone_loglike(w, spec, n_probes: int = 65536, reps: int = 20) -> dict:
    """The fused waveform-plus-likelihood kernel alone on a batch of probes,
    half prior draws and half around the injection; HIP events on the
    stream the kernel runs on."""
    import torch

    from paper_2509_24949_amd import binding, synth

    r = binding.Run(spec, binding.opts_for(w, max_iter=2))
    u = torch.from_numpy(synth.proposal_batch(w, n_probes, seed=77)).cuda()
    out = torch.empty(n_probes, dtype=torch.float64, device="cuda")
    terms = torch.zeros(n_probes, dtype=torch.int32, device="cuda")
    r.loglike(u, out, terms)
    for _ in range(3):
        r.loglike(u, out)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        r.loglike(u, out)
    b.record()
    torch.cuda.synchronize()
    launch_s = a.elapsed_time(b) / reps * 1e-3
    n_terms = int(terms.sum().item())
    r.close()
    bpe = bins_per_edge(n_terms, n_probes)
    flops = n_terms * flops_per_term(w, bpe, edge_form=True)
    peak = peak_tflops(w, bpe, edge_form=True)
    achieved = flops / launch_s / 1e12
    return {"kernel": "k_rb_lane" if w.likelihood == 1 else "k_probe_setup2 + k_probe_bins", "probes": n_probes,
            "probe_mix": "half prior draws, half Gaussian (0.02) around the injection in the unit cube",
            "evals_per_s": n_probes / launch_s, "launch_ms": launch_s * 1e3, "terms_per_launch": n_terms,
            "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak}


def iteration_metrics(trace, K, k, spec, w, W):
    """Per-iteration metrics of the K timed iterations (their records from
    the device), and the walk's moves from a separate untimed run of the
    move-counting chain kernels over the same iterations (same seeds, so the
    same walk)."""
    import numpy as np

    from paper_2509_24949_amd import binding

    probes = trace["probes"][-K:].astype(float)
    steps = trace["steps"][-K:].astype(float)
    out = {"iterations": K,
           "evals_per_step": float(probes.sum() / steps.sum()),
           "chain_evals_mean": float(probes.mean() / k),
           "chain_evals_max_over_mean": float(np.mean(trace["probes_max"][-K:] / (probes / k))),
           "chain_evals_min_over_mean": float(np.mean(trace["probes_min"][-K:] / (probes / k)))}
    if w.kernel != 0:
        return out
    n_count = min(K, 3)
    r = binding.Run(spec, binding.opts_for(w, term_frac=0.0, max_iter=W + n_count + 1, count_moves=True))
    r.step(W + n_count)
    tr = r.trace()
    r.close()
    st = tr["steps"][W:].astype(float).sum()
    hist = tr["hist"][W:].sum(axis=0)
    out["moves"] = {"iterations": n_count, "expansions_per_step": float(tr["stepouts"][W:].sum() / st),
                    "rejected_shrinks_per_step": float(tr["shrinks"][W:].sum() / st),
                    "moved_fraction": float(tr["accepted"][W:].sum() / st),
                    "evals_per_step_hist": [int(v) for v in hist[:16]] + [int(hist[16:].sum())]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="tf2_3det", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-run", action="store_true", help="skip the complete-run timing")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving summary")
    ap.add_argument("--no-standalone", action="store_true", help="skip the standalone likelihood kernel")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the per-configuration error against the stored oracle values")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "slice_kernel_traffic.json"))
    ap.add_argument("--events", type=int, default=64, help="serving: number of events")
    ap.add_argument("--max-runs", type=int, default=32, help="serving: resident-run slots")
    ap.add_argument("--tick-iters", type=int, default=1, help="serving: iterations per tick")
    ap.add_argument("--no-graph", dest="graph", action="store_false",
                    help="serving: launch each tick's kernels directly instead of replaying a captured graph")
    ap.add_argument("--load", type=float, default=2.0, help="serving: arrival rate / sequential service rate")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "mixed"), help="serving: arithmetic")
    ap.add_argument("--max-iter", type=int, default=400, help="serving: iteration capacity per run")
    ap.add_argument("--unit-rates", action="store_true",
                    help="only run the vector-unit rate probe (cycles per instruction, core clock, chip FMA and "
                         "sine/cosine throughput) and print its JSON")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.unit_rates:
        rates = unit_rates()
        if rates is None:
            print("bench.py: the rate probe is not built or failed (python -m paper_2509_24949_amd.build)",
                  file=sys.stderr)
            sys.exit(1)
        print(json.dumps(rates), flush=True)
        return
    if args.copy_calibration:
        import torch

        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.copy_calibration, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the sampler and the server each run on a single GPU)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2509_24949_amd import binding, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    binding.lib()
    if args.workload == "serving":
        print(json.dumps(serving(args)), flush=True)
        return
    if args.workload == "scaling":
        print(json.dumps(scaling(args)), flush=True)
        return
    if args.workload == "coverage":
        print(json.dumps(coverage(args)), flush=True)
        return
    w = synth.workload(args.workload)
    log(f"bench: workload {args.workload}: building data (library-injected waveform)")
    re, im = binding.make_data(w)
    spec = binding.ProblemSpec(w, re, im)

    run_info = {}
    if not args.no_run:
        for attempt in range(2):          # the first complete run also loads the code objects
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = binding.Run(spec, binding.opts_for(w, max_iter=400))
            done = r.run(400)
            z = r.logZ(200)
            torch.cuda.synchronize()
            t_run = time.perf_counter() - t0
            st = r.state()
            r.close()
            log(f"bench: complete run {attempt}: {t_run:.3f} s, {st['iter']} iterations, "
                f"logZ {z['logZ']:.3f} +- {z['sigma']:.3f}, done={done}")
        run_info = {"s_per_run": t_run, "run_iterations": st["iter"], "run_evals": st["n_evals"],
                    "logZ": z["logZ"], "sigma_logZ": z["sigma"], "ess_kish": z["ess"]}
        golden = os.path.join(ROOT, "tests", "golden", "full_runs.json")
        if os.path.exists(golden):
            with open(golden) as fh:
                g = json.load(fh).get(GOLDEN_RUN.get(args.workload, args.workload))
            if g:   # the stored complete run of the double-precision oracle, same seeds
                run_info["accuracy_vs_oracle"] = {
                    "logZ_oracle": g["logZ"], "abs_delta_logZ": abs(z["logZ"] - g["logZ"]),
                    "iterations_oracle": g["iterations"], "evals_oracle": g["n_evals"]}

    K, W = args.steps, args.warmup
    r = binding.Run(spec, binding.opts_for(w, term_frac=0.0, max_iter=W + K + 2))
    r.step(W)
    r.profile(True)
    bins0 = r.stats()["bin_terms"]
    s0 = r.state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r.step(K)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = r.stats()
    s1 = r.state()
    evals = s1["n_evals"] - s0["n_evals"]
    bins_timed = stats["bin_terms"] - bins0
    log(f"bench: {K} timed iterations in {dt:.3f} s ({evals} evaluations); slice kernel "
        f"{stats['ms_slice'] / K:.3f} ms/iter, select {stats['ms_select'] / K:.3f}, prep {stats['ms_prep'] / K:.3f}, "
        f"term {stats['ms_term'] / K:.3f}")
    metrics = iteration_metrics(r.trace(), K, w.n_delete, spec, w, W)
    r.close()
    bpe = bins_per_edge(bins_timed, evals)
    flops_launch = bins_timed / K * flops_per_term(w, bpe)
    slice_s = stats["ms_slice"] / K * 1e-3
    achieved = flops_launch / slice_s / 1e12
    mixed = w.precision == 1
    peak = peak_tflops(w, bpe)
    traffic = None
    if os.path.exists(args.traffic):
        try:
            with open(args.traffic) as fh:
                tr = json.load(fh)
            if tr.get("workload") == args.workload and tr.get("source_sha") == _kernel_sha():
                traffic = tr.get("bytes_per_launch")
        except (OSError, ValueError):
            traffic = None
    out = {
        "metric": "logL evals/s",
        "value": evals / dt,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": dt / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic (seeded Gaussian noise plus an injected TaylorF2 signal; no real detector data)",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "n_live": w.n_live,
                   "n_delete": w.n_delete, "n_steps": w.n_steps, "n_bins": w.n_bins, "n_det": w.n_det,
                   "n_dim": w.n_dim, "likelihood": "relative binning" if w.likelihood == 1 else "full grid",
                   "precision": "mixed" if mixed else "fp64"},
        "roofline": {"bound": "alu", "kernel": "k_slice", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                     "flops_per_launch": flops_launch, "launch_ms": slice_s * 1e3,
                     "bin_terms_per_launch": bins_timed / K},
        "iteration_metrics": metrics,
        **run_info,
    }
    if not args.no_standalone:
        out["standalone_loglike"] = standalone_loglike(w, spec)
        log(f"bench: standalone likelihood: {out['standalone_loglike']['evals_per_s'] / 1e6:.0f} M evals/s, "
            f"{out['standalone_loglike']['frac'] * 100:.1f}% of peak")
    if not args.no_serving and args.workload == "tf2_3det":
        keys = ("value", "unit", "latency_p50_s", "latency_p99_s", "makespan_s", "evals_per_s", "sequential",
                "saturated", "logZ_served_vs_sequential", "roofline", "config")
        sv = serving(args, "fp64")
        out["serving"] = {k: sv[k] for k in keys}
        sv = serving(args, "mixed")
        out["serving_mixed"] = {k: sv[k] for k in keys}
    if not args.no_accuracy and args.workload == "tf2_3det":
        out["accuracy_vs_oracle_per_config"] = accuracy()
        out["unit_rates"] = unit_rates()
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        log(f"bench: timing the oracle on {threads} host threads for about {args.cpu_seconds:.0f} s")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds, threads)
    print(json.dumps(out), flush=True)


def _kernel_sha() -> str:
    """Hash of the kernel sources with line comments and blank lines removed,
    so that stored counter readings stay valid across comment-only edits."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in ("ns_device.h", "ns_kernels.h", "ns_internal.h"):
        with open(os.path.join(ROOT, "paper_2509_24949_amd", "csrc", f), encoding="utf-8") as fh:
            for line in fh:
                code = re.sub(r"//.*", "", line).strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
