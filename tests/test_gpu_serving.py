"""Serving: many runs resident on one GPU, advanced by packed launches.

Bars: a served run follows the oracle in lockstep (identical dead-point
slots, log-likelihoods to 1e-9 of the cancellation scale); each run's record
is bit-identical alone and inside a mix of runs of other sizes, networks and
likelihood forms, with and without graph replay and with several iterations
per tick; admission respects the slot count and the memory budget.
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


def _spec(w):
    re, im = binding.make_data(w)
    return binding.ProblemSpec(w, re, im)


def _requests():
    """Runs of different sizes, networks and likelihood forms, each bounded
    to a few iterations (capacity) except the small complete one."""
    out = []
    w = synth.workload("tf2_1det")
    out.append(("tf2_1det", _spec(w), binding.opts_for(w)))
    out.append(("tf2_1det-b", out[0][1], binding.opts_for(w, seed=77, n_live=300, n_delete=100)))
    w = synth.workload("tf2_3det")
    out.append(("tf2_3det", _spec(w), binding.opts_for(w, max_iter=3)))
    w = synth.workload("tf2_3det_rb")
    out.append(("tf2_3det_rb", _spec(w), binding.opts_for(w, max_iter=3)))
    w = synth.workload("tf2_3det_mixed")
    out.append(("tf2_3det_mixed", _spec(w), binding.opts_for(w, max_iter=2)))
    w = synth.serving_event(1)                 # one detector, 4 s, n_live 2000
    out.append(("event1", _spec(w), binding.opts_for(w, max_iter=2)))
    return out


def _serve(reqs, max_runs, graph=False, n_iters=1, budget=0, stream=None, trace=None):
    srv = binding.Server(hbm_budget=budget, max_runs=max_runs, graph=graph, stream=stream)
    tickets = {srv.submit(spec, opts): name for name, spec, opts in reqs}
    results = {}
    for _ in range(100000):
        running, queued, finished = srv.tick(n_iters)
        if trace is not None:
            trace.append((running, queued, srv.info()["used"]))
        for info in srv.poll():
            assert info["status"] == 0, info
            run = srv.take(info["ticket"])
            results[tickets[info["ticket"]]] = (info, _record(run))
            run.close()
        if running == 0 and queued == 0 and len(results) == len(reqs):
            break
    srv.close()
    return results


def _record(run):
    d = run.dead()
    st = run.state()
    z = run.logZ(200)
    return dict(d, logZ=st["logZ"], H=st["H"], n_evals=st["n_evals"], iterations=st["iter"], final=z)


def _assert_identical(a, b, name):
    for key in ("u", "logl", "logx", "logw", "iter", "slot"):
        np.testing.assert_array_equal(a[key], b[key], err_msg=f"{name}: {key}")
    assert a["logZ"] == b["logZ"] and a["H"] == b["H"] and a["n_evals"] == b["n_evals"], name
    assert a["iterations"] == b["iterations"], name
    assert a["final"] == b["final"], name


def test_served_run_matches_oracle(torch_cuda):
    w = synth.workload("tf2_1det")
    re, im = oracle.make_data(w)
    orc = oracle.OracleProblem(w, re, im)
    spec = binding.ProblemSpec(w, re, im)
    res = _serve([("tf2_1det", spec, binding.opts_for(w))], max_runs=1)
    info, g = res["tf2_1det"]
    ro = oracle.Run(orc, oracle.opts_for(w, n_threads=NTHREADS))
    ro.step(1000)
    a = ro.dead()
    assert info["done"] == 1 and info["iterations"] == ro.state()["iter"]
    np.testing.assert_array_equal(g["slot"], a["slot"])
    np.testing.assert_array_equal(g["iter"], a["iter"])
    assert np.max(np.abs(g["logl"] - a["logl"]) / (np.abs(a["logl"]) + 1.0)) <= 1e-9
    assert np.max(np.abs(g["u"] - a["u"])) <= 1e-9
    so = ro.state()
    assert g["n_evals"] == so["n_evals"]
    assert abs(g["logZ"] - so["logZ"]) <= 1e-9 * (abs(so["logZ"]) + 1.0)


@pytest.mark.parametrize("name", ["tf2_3det", "tf2_3det_rb"])
def test_served_iterations_match_oracle(torch_cuda, name):
    w = synth.workload(name)
    re, im = oracle.make_data(w)
    orc = oracle.OracleProblem(w, re, im)
    spec = binding.ProblemSpec(w, re, im)
    res = _serve([(name, spec, binding.opts_for(w, max_iter=2))], max_runs=1)
    info, g = res[name]
    assert info["done"] == 2 and info["iterations"] == 2
    ro = oracle.Run(orc, oracle.opts_for(w, n_threads=NTHREADS, max_iter=2))
    ro.step(5)
    a = ro.dead()
    np.testing.assert_array_equal(g["slot"], a["slot"])
    assert np.max(np.abs(g["logl"] - a["logl"]) / (np.abs(a["logl"]) + 1.0)) <= 1e-9
    assert g["n_evals"] == ro.state()["n_evals"]


def test_result_same_alone_and_in_mix(torch_cuda):
    reqs = _requests()
    alone = {}
    for r in reqs:
        alone.update(_serve([r], max_runs=1))
    mixed = _serve(reqs, max_runs=len(reqs))
    for name, _, _ in reqs:
        _assert_identical(alone[name][1], mixed[name][1], name)
    # graph replay of the ticks, several iterations per tick, fewer slots
    stream = torch_cuda.cuda.Stream()
    with torch_cuda.cuda.stream(stream):
        replay = _serve(reqs, max_runs=4, graph=True, n_iters=3, stream=stream.cuda_stream)
    for name, _, _ in reqs:
        _assert_identical(alone[name][1], replay[name][1], name + " (graph)")


def test_admission_by_slots_and_memory(torch_cuda):
    w = synth.workload("tf2_1det")
    spec = _spec(w)
    reqs = [(f"r{i}", spec, binding.opts_for(w, seed=500 + i, max_iter=4)) for i in range(4)]
    alone = _serve(reqs[:1], max_runs=1)
    trace = []
    _serve(reqs, max_runs=2, trace=trace)
    assert max(t[0] for t in trace) == 2
    # a budget that holds one run at a time
    srv = binding.Server(max_runs=8)
    srv.submit(spec, reqs[0][2])
    srv.tick(1)
    one = srv.info()["used"]
    srv.close()
    assert one > 0
    trace = []
    res = _serve(reqs, max_runs=8, budget=int(one * 1.5), trace=trace)
    assert max(t[0] for t in trace) == 1
    assert max(t[2] for t in trace) <= int(one * 1.5)
    assert len(res) == 4
    _assert_identical(alone["r0"][1], res["r0"][1], "r0 under a memory cap")
    # a request larger than the whole budget is refused at submission
    srv = binding.Server(hbm_budget=one // 2, max_runs=2)
    with pytest.raises(binding.NSError) as e:
        srv.submit(spec, reqs[0][2])
    assert e.value.code == binding.NS_E_OOM
    srv.close()


def test_ticket_states(torch_cuda):
    w = synth.workload("tf2_1det")
    spec = _spec(w)
    srv = binding.Server(max_runs=1)
    t1 = srv.submit(spec, binding.opts_for(w, max_iter=2))
    t2 = srv.submit(spec, binding.opts_for(w, max_iter=2, seed=9))
    with pytest.raises(binding.NSError) as e:
        srv.take(t2)
    assert e.value.code == binding.NS_E_STATE          # queued
    running, queued, _ = srv.tick(1)
    assert (running, queued) == (1, 1)
    with pytest.raises(binding.NSError) as e:
        srv.take(t1)
    assert e.value.code == binding.NS_E_STATE          # running
    for _ in range(10):
        srv.tick(1)
    infos = srv.poll()
    assert [i["ticket"] for i in infos] == [t1, t2]
    assert all(i["done"] == 2 and i["iterations"] == 2 for i in infos)
    assert all(i["t_submit"] <= i["t_admit"] <= i["t_finish"] for i in infos)
    assert srv.poll() == []
    r = srv.take(t1)
    assert r.state()["iter"] == 2
    r.close()
    with pytest.raises(binding.NSError):
        srv.take(t1)
    srv.close()                                         # frees the untaken run
