"""Derive the SNR-scaled injection distances of the synthetic workloads.

Calls only the oracle.  For each workload the injected waveform is computed
at 1 Mpc, its optimal network SNR rho_1 = sqrt(sum_det <h|h>) is taken, and
the distance that gives the target SNR is rho_1 / rho_target (the amplitude
is inversely proportional to distance).  The serving events get one
distance each.  Writes
``paper_2509_24949_amd/injections.json``.

    python -m oracle.derive_injections
"""
from __future__ import annotations

import json
import math
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402
from paper_2509_24949_amd import synth  # noqa: E402


def optimal_snr(w, theta, fixed_dist_mpc=None) -> float:
    prob = oracle.OracleProblem(w, fixed_dist_mpc=fixed_dist_mpc)
    rho2 = 0.0
    for det in range(w.n_det):
        hr, hi = prob.waveform(theta, det, cut=True)
        rho2 += prob.inner(det, hr, hi, hr, hi)
    return math.sqrt(rho2)


def derive() -> dict:
    out = {}
    w1 = synth.workload("tf2_1det", distance=1.0)
    rho1 = optimal_snr(w1, w1.theta_inj, fixed_dist_mpc=1.0)
    out["tf2_1det"] = {"distance_mpc": rho1 / w1.snr_target, "snr": w1.snr_target,
                   "note": "effective distance of the optimally oriented single-detector injection"}
    w2 = synth.workload("tf2_3det", distance=1.0)
    th = np.array(w2.theta_inj, dtype=np.float64)
    th[4] = 1.0
    rho1 = optimal_snr(w2, th)
    out["tf2_3det"] = {"distance_mpc": rho1 / w2.snr_target, "snr": w2.snr_target,
                   "note": "luminosity distance of the H1/L1/V1 injection"}
    dist, snr = [], []
    for i in range(synth.SERVING_EVENTS):
        w = synth.serving_event(i, distance=1.0)
        rho1 = optimal_snr(w, np.array(w.theta_inj, dtype=np.float64))
        dist.append(rho1 / w.snr_target)
        snr.append(w.snr_target)
    out["serving"] = {"distance_mpc": dist, "snr": snr,
                   "note": "luminosity distances of the serving events, in event order"}
    return out


if __name__ == "__main__":
    res = derive()
    with open(synth.INJECTIONS_JSON, "w") as fh:
        json.dump(res, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(json.dumps(res, indent=1))
