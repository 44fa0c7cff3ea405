"""Write tests/golden/full_runs.json: complete oracle runs of the one-detector,
full-grid, relative-binning, spin-orbit and large-population workloads and of
a few serving events.

Calls only the oracle (on its own injected data).  For each run it stores
the evidence summary and a digest of the dead-point sequence (slot and
iteration of every death) plus evenly spaced dead-point log-likelihoods, so
that a GPU run with the same seeds can be checked end to end without
re-running the oracle.

    python tests/golden/make_full_runs.py [n_threads] [--only=key1,key2]

--only recomputes the named entries and keeps the others as stored.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2509_24949_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_runs.json")
SERVING_SAMPLE = (26, 45, 57, 61)   # short serving events (few active bins)
# long serving events with many active bins, run at n_live 500 (k 250) to keep
# the oracle's time down: 32 s three-detector (k_lim 2650 bins, tables read
# through the caches), 16 s three-detector, 32 s one-detector at low chirp
# mass (k_lim about 11 600 bins)
SERVING_LONG = (32, 16, 39)
LONG_OPTS = {"n_live": 500, "n_delete": 250}


def digest(slot, it) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(slot, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(it, dtype=np.int32).tobytes())
    return h.hexdigest()


def full_run(w, n_threads: int, **kw) -> dict:
    re, im = oracle.make_data(w)
    prob = oracle.OracleProblem(w, re, im)
    t0 = time.perf_counter()
    run = oracle.Run(prob, oracle.opts_for(w, n_threads=n_threads, **kw))
    run.step(100000)
    st = run.state()
    z = run.logZ(200)
    d = run.dead()
    nd = len(d["slot"])
    idx = np.unique(np.linspace(0, nd - 1, 32).astype(int))
    return {
        "iterations": st["iter"], "n_dead": st["n_dead"], "n_evals": st["n_evals"],
        "logZ": z["logZ"], "sigma": z["sigma"], "sigma_h": z["sigma_h"], "ess": z["ess"], "H": st["H"],
        "dead_digest": digest(d["slot"], d["iter"]),
        "logl_index": idx.tolist(), "logl_at": [float(d["logl"][i]) for i in idx],
        "oracle_seconds": time.perf_counter() - t0, "oracle_threads": n_threads, "opts": dict(kw),
    }


def main():
    args = [a for a in sys.argv[1:] if not a.startswith("--only=")]
    only = [a.split("=", 1)[1].split(",") for a in sys.argv[1:] if a.startswith("--only=")]
    only = set(only[0]) if only else None
    n_threads = int(args[0]) if args else (os.cpu_count() or 1)
    out = {}
    if only is not None and os.path.exists(OUT):
        with open(OUT) as fh:
            out = json.load(fh)
    jobs = []
    for name in ("tf2_1det", "tf2_3det", "tf2_3det_rb", "tf2_3det_so"):
        jobs.append((name, lambda name=name: full_run(synth.workload(name), n_threads)))

    def large_population():
        # the large-population workload in double precision (the GPU's mixed
        # form is compared statistically against it)
        return full_run(synth.workload("tf2_3det_n2000"), n_threads)

    jobs.append(("tf2_3det_n2000_fp64", large_population))
    jobs.append(("tf2_3det_rb_n2000_fp64", lambda: full_run(synth.workload("tf2_3det_rb_n2000"), n_threads)))
    for i in SERVING_SAMPLE:
        jobs.append((f"event/{i}", lambda i=i: full_run(synth.serving_event(i), n_threads)))
    for i in SERVING_LONG:
        jobs.append((f"event/{i}", lambda i=i: full_run(synth.serving_event(i), n_threads, **LONG_OPTS)))
    for key, job in jobs:
        if only is not None and key not in only:
            continue
        out[key] = job()
        print(key, out[key]["iterations"], out[key]["logZ"], f"{out[key]['oracle_seconds']:.1f} s", flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
        fh.write("\n")


if __name__ == "__main__":
    main()
