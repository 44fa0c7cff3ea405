"""Write tests/golden/loglike_samples.json: the oracle's log-likelihood ratio
on a seeded probe batch of each double-precision workload.

Calls only the oracle (on its own injected data).  The probes are
synth.proposal_batch(w, N_PROBES, seed=SEED) (half prior draws, half around
the injection); the stored values let the benchmark report its likelihood
error against the oracle per workload without running the oracle.

    python tests/golden/make_loglike_samples.py [n_threads]
"""
from __future__ import annotations

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2509_24949_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "loglike_samples.json")
N_PROBES = 512
SEED = 4242
# the mixed-precision workloads share these workloads' events and probes
WORKLOADS = ("tf2_1det", "tf2_3det", "tf2_3det_rb", "tf2_3det_so")


def main():
    n_threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    out = {"n_probes": N_PROBES, "seed": SEED}
    for name in WORKLOADS:
        w = synth.workload(name)
        re, im = oracle.make_data(w)
        prob = oracle.OracleProblem(w, re, im)
        u = synth.proposal_batch(w, N_PROBES, seed=SEED)
        lam = prob.loglike_batch(u, n_threads)
        out[name] = [float(v) for v in lam]
        print(name, float(min(lam)), float(max(lam)), flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
        fh.write("\n")


if __name__ == "__main__":
    main()
