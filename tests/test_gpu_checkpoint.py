"""Checkpoint and resume, and the noise-model constant, through the C ABI.

Bars: a run restored from a checkpoint continues bit-identically to the
uninterrupted run (the random numbers are counter-based); the noise-model
log-likelihood equals the oracle's to 1e-12 relative.
"""
import numpy as np
import pytest

import oracle
from paper_2509_24949_amd import binding, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()
    return torch


def _record(run):
    d = run.dead()
    st = run.state()
    u, l = run.live()
    return dict(d, live_u=u, live_l=l, logZ=st["logZ"], H=st["H"], logX=st["logX"], n_evals=st["n_evals"],
                iterations=st["iter"], done=st["done"], final=run.logZ(200), trace=run.trace())


def _identical(a, b):
    for key in ("u", "logl", "logx", "logw", "iter", "slot", "live_u", "live_l"):
        np.testing.assert_array_equal(a[key], b[key], err_msg=key)
    for key in ("logZ", "H", "logX", "n_evals", "iterations", "done", "final"):
        assert a[key] == b[key], key
    # the per-iteration metrics, those before the checkpoint included
    assert len(a["trace"]["iter"]) == a["iterations"]
    for key in a["trace"]:
        np.testing.assert_array_equal(a["trace"][key], b["trace"][key], err_msg=key)


@pytest.mark.parametrize("name,first,then,count", [("tf2_1det", 5, 200, False), ("tf2_3det_rb", 2, 2, False),
                                                  ("tf2_3det_mixed", 1, 2, False), ("tf2_3det", 1, 2, True)])
def test_resume_is_bit_identical(torch_cuda, name, first, then, count):
    w = synth.workload(name)
    re, im = binding.make_data(w)
    spec = binding.ProblemSpec(w, re, im)
    opts = binding.opts_for(w, max_iter=first + then, count_moves=count)
    a = binding.Run(spec, opts)
    a.step(first)
    blob = a.save()
    a.step(then)
    ra = _record(a)
    a.close()
    b = binding.Run.load(blob, spec, opts)
    assert b.state()["iter"] == first
    b.step(then)
    _identical(ra, _record(b))
    # a checkpoint of the finished run restores the same evidence
    blob2 = b.save()
    c = binding.Run.load(blob2, spec, opts)
    _identical(ra, _record(c))
    b.close()
    c.close()


def test_truncated_checkpoint_is_rejected(torch_cuda):
    w = synth.workload("tf2_1det")
    spec = binding.ProblemSpec(w, *binding.make_data(w))
    opts = binding.opts_for(w)
    a = binding.Run(spec, opts)
    a.step(2)
    blob = a.save()
    a.close()
    with pytest.raises(binding.NSError) as e:
        binding.Run.load(blob[:-8], spec, opts)
    assert e.value.code == binding.NS_E_ARG


@pytest.mark.parametrize("name", ["tf2_1det", "tf2_3det"])
def test_noise_loglike_parity(torch_cuda, name):
    w = synth.workload(name)
    re, im = oracle.make_data(w)
    want = oracle.OracleProblem(w, re, im).noise_loglike()
    r = binding.Run(binding.ProblemSpec(w, re, im), binding.opts_for(w))
    got = r.noise_loglike()
    r.close()
    assert abs(got - want) <= 1e-12 * abs(want)


def test_nan_and_minus_inf_likelihoods_die_first(torch_cuda):
    """Failure injection through a checkpoint: two live points' log-likelihoods
    replaced by NaN and by -inf (the sampler orders NaN as -inf, ties going to
    the lower slot) die first in the next iteration, add nothing to the
    evidence, and the run still terminates with a finite evidence."""
    w = synth.gauss_workload(3, 0.05, mu=[0.4, 0.5, 0.6], n_live=200, n_delete=100)
    spec = binding.ProblemSpec(w)
    opts = binding.opts_for(w)
    a = binding.Run(spec, opts)
    a.step(2)
    st0 = a.state()
    _, lam = a.live()
    blob = bytearray(a.save())
    a.close()
    raw = np.ascontiguousarray(lam, dtype=np.float64).tobytes()
    pos = blob.find(raw)
    assert pos >= 0 and blob.find(raw, pos + 1) < 0      # the live log-likelihoods, stored once
    bad = lam.copy()
    bad[7] = np.nan
    bad[3] = -np.inf
    blob[pos:pos + len(raw)] = bad.tobytes()
    b = binding.Run.load(bytes(blob), spec, opts)
    b.step(1)
    d = b.dead()
    nd = st0["n_dead"]
    np.testing.assert_array_equal(d["slot"][nd:nd + 2], [3, 7])
    assert np.isneginf(d["logl"][nd]) and np.isnan(d["logl"][nd + 1])   # the record keeps the raw values
    assert np.all(np.isneginf(d["logw"][nd:nd + 2]))
    assert np.all(np.isfinite(d["logw"][nd + 2:nd + 100]))
    assert np.isfinite(b.state()["logZ"])
    assert b.run()
    z = b.logZ(200)
    assert np.isfinite(z["logZ"]) and np.isfinite(z["sigma"])
    assert np.all(np.isfinite(b.live()[1]))
    b.close()
