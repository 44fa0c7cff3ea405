"""Write tests/golden/full_runs.json: complete oracle runs of the full-grid,
relative-binning and large-population workloads and of a few serving events.

Calls only the oracle (on its own injected data).  For each run it stores
the evidence summary and a digest of the dead-point sequence (slot and
iteration of every death) plus evenly spaced dead-point log-likelihoods, so
that a GPU run with the same seeds can be checked end to end without
re-running the oracle.

    python tests/golden/make_full_runs.py [n_threads]
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
        "oracle_seconds": time.perf_counter() - t0, "oracle_threads": n_threads,
    }


def main():
    n_threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    out = {}
    for name in ("tf2_3det", "tf2_3det_rb"):
        out[name] = full_run(synth.workload(name), n_threads)
        print(name, out[name]["iterations"], out[name]["logZ"], flush=True)
    # the large-population workload in double precision (the GPU's mixed form
    # is compared statistically against it)
    w = synth.workload("tf2_3det_mixed")
    w.precision = 0
    out["tf2_3det_n2000_fp64"] = full_run(w, n_threads)
    print("tf2_3det_n2000_fp64", out["tf2_3det_n2000_fp64"]["logZ"], flush=True)
    for i in SERVING_SAMPLE:
        key = f"event/{i}"
        out[key] = full_run(synth.serving_event(i), n_threads)
        print(key, out[key]["iterations"], out[key]["logZ"], flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
        fh.write("\n")


if __name__ == "__main__":
    main()
