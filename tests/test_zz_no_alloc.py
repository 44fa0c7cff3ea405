"""ns_loglike_noalloc (the batched likelihood without allocation, for callers
that cannot allocate) against ns_loglike: the same kernels, so the results
and term counts are identical, over two calls in a row (the second smaller),
for the full grid, relative binning and the mixed form; batches beyond the
per-device maximum are rejected before any launch."""
import ctypes as C

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


def _run(name):
    w = synth.workload(name)
    re, im = oracle.make_data(w)
    spec = binding.ProblemSpec(w, re, im)
    return w, binding.Run(spec, binding.opts_for(w))


@pytest.mark.parametrize("name", ["tf2_3det", "tf2_3det_rb", "tf2_3det_mixed", "tf2_1det"])
def test_noalloc_matches_loglike(torch_cuda, name):
    torch = torch_cuda
    w, run = _run(name)
    sizes = [binding.NS_LOGLIKE_NOALLOC_MAX, 1031]     # the maximum, then a smaller ragged batch
    for call, n in enumerate(sizes):
        print(f"noalloc {name} call {call} n {n}", flush=True)
        u = torch.from_numpy(synth.proposal_batch(w, n, seed=40 + call)).cuda()
        ref_t = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        ref = run.loglike(u, terms=ref_t)
        got_t = torch.full((n,), -9, dtype=torch.int32, device="cuda")
        got = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        run.loglike(u, out=got, terms=got_t, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (name, call)
        assert torch.equal(got_t, ref_t), (name, call)
    run.close()


def test_noalloc_rejects_oversized_batches(torch_cuda):
    torch = torch_cuda
    w, run = _run("tf2_3det")
    n = binding.NS_LOGLIKE_NOALLOC_MAX + 1
    u = torch.zeros((n, w.n_dim), dtype=torch.float64, device="cuda")
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    rc = binding.lib().ns_loglike_noalloc(run.h, C.c_void_p(u.data_ptr()), n, C.c_void_p(out.data_ptr()), None)
    assert rc == binding.NS_E_ARG
    assert b"NS_LOGLIKE_NOALLOC_MAX" in binding.lib().ns_last_error()
    assert torch.count_nonzero(out).item() == 0
    run.close()
