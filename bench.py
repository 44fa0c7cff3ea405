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
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6          # MI355X vector FP64
FP32_PEAK_TFLOPS = 157.3         # MI355X vector FP32 (packed)
SINCOS_FLOPS = 44                # flops of the double-precision sincos in cycles
PHASE_FLOPS = 24                 # per (probe, bin): PN phase series, shared by the detectors
DET_FLOPS = 2 + SINCOS_FLOPS + 8 # per (probe, bin, detector): delay, sincos, complex accumulate
# mixed form per (probe, bin, detector): delay and reduction in double (4), two
# transcendental float ops (sin, cos), complex accumulate (8)
DET_FLOPS_MIXED = 4 + 2 + 8
# relative binning per (probe, edge): the phase (24) and per detector delay,
# sincos and the complex ratio (2 + sincos + 6); per (probe, coarse bin,
# detector) the linear-model terms (27), counted per edge as nb/(nb+1) of it
RB_EDGE_DET = 2 + SINCOS_FLOPS + 6
RB_EDGE_DET_MIXED = 4 + 2 + 6
RB_BIN_DET = 27

_GRID2 = "3-detector aligned-spin TaylorF2 (11 parameters), 4017 bins/detector (20-1024 Hz, df 0.25 Hz), network SNR 20"
WORKLOADS = {
    "cfg2": _GRID2 + ", full-grid Whittle, n_live 1000, n_delete 500, 55 slice steps, FP64",
    "cfg1": "1-detector TaylorF2 (4 parameters), full-grid Whittle, 473 bins (20-256 Hz, df 0.5 Hz), "
            "SNR 15, n_live 500, n_delete 250, 20 slice steps, FP64",
    "cfg3": _GRID2 + ", relative binning (128 geometric bins), n_live 1000, n_delete 500, 55 slice steps, FP64",
    "cfg4": _GRID2 + ", full-grid Whittle, n_live 2000, n_delete 1000, 55 slice steps, mixed precision",
    "cfg4rb": _GRID2 + ", relative binning (128 bins), n_live 2000, n_delete 1000, 55 slice steps, mixed precision",
}


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def flops_per_term(w) -> float:
    """Algorithmic flops per counted term (full grid: one active bin of one
    probe; relative binning: one edge of one probe)."""
    from paper_2509_24949_amd import synth

    mixed = w.precision == 1
    if w.likelihood == synth.LIKE_RB:
        nb = w.rb_n_bins
        edge = RB_EDGE_DET_MIXED if mixed else RB_EDGE_DET
        return PHASE_FLOPS + w.n_det * edge + w.n_det * RB_BIN_DET * nb / (nb + 1)
    return PHASE_FLOPS + w.n_det * (DET_FLOPS_MIXED if mixed else DET_FLOPS)


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
    return {"value": ev / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{iters} sampler iterations of the same workload from its initial population "
                      f"({ev} likelihood evaluations in {dt:.1f} s, OpenMP over chains)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg2", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-run", action="store_true", help="skip the complete-run timing")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "slice_kernel_traffic.json"))
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (reference for HBM byte counters)")
    args = ap.parse_args()
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
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build "
              "(the sampler runs on a single GPU)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2509_24949_amd import binding, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    binding.lib()
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
    r.close()
    flops_launch = bins_timed / K * flops_per_term(w)
    slice_s = stats["ms_slice"] / K * 1e-3
    achieved = flops_launch / slice_s / 1e12
    mixed = w.precision == 1
    peak = FP32_PEAK_TFLOPS if mixed else FP64_PEAK_TFLOPS
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
        **run_info,
    }
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        log(f"bench: timing the oracle on {threads} host threads for about {args.cpu_seconds:.0f} s")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds, threads)
    print(json.dumps(out), flush=True)


def _kernel_sha() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in ("ns_device.h", "ns_kernels.hip", "ns_internal.h"):
        with open(os.path.join(ROOT, "paper_2509_24949_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
