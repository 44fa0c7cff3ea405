"""Equal-weight posterior samples (ns_resample) against the oracle's
systematic resampling of the same complete run.

The running weight sums decide the picks; the two sides add the weights in
different orders (a sequential sum in the oracle, chunked sums scanned across
a workgroup on the GPU), so a pick may differ where a position falls within
rounding of a boundary.  Bars: almost every pick identical; every GPU pick
valid under the oracle's running sums to 1e-9 of the total; the parameters
of each pick equal the weighted sample it names.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2509_24949_amd import binding, synth

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()
    return torch


@pytest.mark.parametrize("name,n_out", [("tf2_1det", 5000), ("gauss", 777)])
def test_resample_matches_oracle(torch_cuda, name, n_out):
    if name == "gauss":
        w = synth.gauss_workload(4, 0.05)
        orc, spec = oracle.OracleProblem(w), binding.ProblemSpec(w)
    else:
        w = synth.workload(name)
        re, im = oracle.make_data(w)
        orc, spec = oracle.OracleProblem(w, re, im), binding.ProblemSpec(w, re, im)
    print(f"resample {name} n_out {n_out}", flush=True)
    ro = oracle.Run(orc, oracle.opts_for(w, n_threads=NTHREADS))
    ro.run()
    run = binding.Run(spec, binding.opts_for(w))
    run.run()
    assert run.state()["n_dead"] == ro.state()["n_dead"]
    io, tho = ro.resample(n_out)
    ig, thg = run.resample(n_out)
    th_all, _, lw = ro.samples()
    cum = np.cumsum(np.exp(lw))
    word = oracle.philox([0, 0, 0, 6 << 48], [w.sampler_seed, 0])[0]
    u0 = (word >> 11) * 2.0 ** -53
    pos = (np.arange(n_out) + u0) / n_out * cum[-1]
    tol = 1e-9 * cum[-1]
    lo = np.where(ig > 0, cum[np.maximum(ig - 1, 0)], 0.0)
    assert np.all(ig >= 0) and np.all(ig < len(cum))
    assert np.all(lo <= pos + tol) and np.all((cum[ig] > pos - tol) | (ig == len(cum) - 1))
    assert np.mean(ig == io) >= 0.999
    assert np.all(np.diff(ig) >= 0)
    # the parameters of a pick are those of the weighted sample it names
    g_th, _, _ = run.samples()
    assert np.array_equal(thg, g_th[ig])
    assert np.max(np.abs(tho - th_all[io])) == 0.0
    run.close()
