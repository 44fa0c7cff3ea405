"""Determinism as the race detector: the same run repeated on the GPU gives
bit-identical results (dead-point record, live points, evidence state and
per-iteration records) in every chain-kernel configuration and precision,
and the batched likelihood gives bit-identical values.  A missing barrier or
an order-dependent reduction shows up here as a difference between two
otherwise identical runs."""
import numpy as np
import pytest

from paper_2509_24949_amd import binding, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()
    return torch


def _run(spec, w, iters, **kw):
    r = binding.Run(spec, binding.opts_for(w, max_iter=iters + 1, term_frac=0.0, **kw))
    r.step(iters)
    d = r.dead()
    u, l = r.live()
    out = dict(d, live_u=u, live_l=l, state=r.state(), trace=r.trace())
    r.close()
    return out


def _same(a, b):
    for key in ("u", "logl", "logx", "logw", "iter", "slot", "live_u", "live_l"):
        np.testing.assert_array_equal(a[key], b[key], err_msg=key)
    assert a["state"] == b["state"]
    for key in a["trace"]:
        np.testing.assert_array_equal(a["trace"][key], b["trace"][key], err_msg=key)


@pytest.mark.parametrize("name,threads,stage,count", [
    ("tf2_3det", 256, "1", False), ("tf2_3det", 128, "1", False), ("tf2_3det", 64, "0", False),
    ("tf2_3det_rb", 256, "1", False), ("tf2_3det_mixed", 64, "1", False), ("tf2_3det_rb_mixed", 128, "1", False),
    ("tf2_3det", 64, "1", True), ("tf2_3det_rb_walk", 0, "1", False)])
def test_repeated_runs_are_bit_identical(torch_cuda, monkeypatch, name, threads, stage, count):
    if threads:
        monkeypatch.setenv("NS_SLICE_THREADS", str(threads))
    monkeypatch.setenv("NS_LDS_TABLES", stage)
    w = synth.workload(name)
    spec = binding.ProblemSpec(w, *binding.make_data(w))
    print(f"determinism {name} threads={threads} stage={stage} count={count}", flush=True)
    _same(_run(spec, w, 3, count_moves=count), _run(spec, w, 3, count_moves=count))


@pytest.mark.parametrize("name", ["tf2_3det", "tf2_3det_rb", "tf2_3det_mixed"])
def test_repeated_batches_are_bit_identical(torch_cuda, name):
    torch = torch_cuda
    w = synth.workload(name)
    spec = binding.ProblemSpec(w, *binding.make_data(w))
    r = binding.Run(spec, binding.opts_for(w))
    u = torch.tensor(synth.proposal_batch(w, 4099, seed=77), dtype=torch.float64, device="cuda")
    a = r.loglike(u).cpu().numpy()
    b = r.loglike(u).cpu().numpy()
    r.close()
    np.testing.assert_array_equal(a, b)
