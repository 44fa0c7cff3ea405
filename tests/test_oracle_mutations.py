"""Mutation check of the oracle's pins: copies of the oracle source with one
coefficient or factor changed by about one percent (or one structural slip)
are compiled on the CPU, and the pin that covers that part must reject each
copy.  Nothing here touches the HIP library."""
import ctypes as C
import math
import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import test_oracle_pins as pins
from paper_2509_24949_amd import synth

# (name, text in nsorc.c, replacement, the pin that must fail)
MUTATIONS = [
    ("psi2 constant", "3715.0 / 756.0", "1.01 * 3715.0 / 756.0", "phase"),
    ("psi3 spin-orbit", "4.0 * beta", "4.04 * beta", "phase"),
    ("psi4 constant", "15293365.0 / 508032.0", "1.01 * 15293365.0 / 508032.0", "phase"),
    ("psi4 spin-spin", "10.0 * sigma", "10.1 * sigma", "phase"),
    ("psi5 constant", "38645.0 / 756.0", "1.01 * 38645.0 / 756.0", "phase"),
    ("psi5 logarithm", "(1.0 + 3.0 * lv)", "(1.0 + 3.03 * lv)", "phase"),
    ("psi6 constant", "11583231236531.0 / 4694215680.0", "1.01 * 11583231236531.0 / 4694215680.0", "phase"),
    ("psi6 pi^2", "640.0 * PI * PI / 3.0", "1.01 * 640.0 * PI * PI / 3.0", "phase"),
    ("psi6 Euler gamma", "6848.0 * EULER_GAMMA / 21.0", "1.01 * 6848.0 * EULER_GAMMA / 21.0", "phase"),
    ("psi6 logarithm", "(6848.0 / 21.0) * log(4.0 * v)", "1.01 * (6848.0 / 21.0) * log(4.0 * v)", "phase"),
    ("psi6 eta", "(-15737765635.0 / 3048192.0 + 2255.0 * PI * PI / 12.0) * eta",
     "1.01 * (-15737765635.0 / 3048192.0 + 2255.0 * PI * PI / 12.0) * eta", "phase"),
    ("psi6 eta^2", "76055.0 * e2 / 1728.0", "1.01 * 76055.0 * e2 / 1728.0", "phase"),
    ("psi6 eta^3", "127825.0 * e3 / 1296.0", "1.01 * 127825.0 * e3 / 1296.0", "phase"),
    ("psi7 constant", "77096675.0 / 254016.0", "1.01 * 77096675.0 / 254016.0", "phase"),
    ("psi7 eta", "378515.0 * eta / 1512.0", "1.01 * 378515.0 * eta / 1512.0", "phase"),
    ("psi7 eta^2", "74045.0 * e2 / 756.0", "1.01 * 74045.0 * e2 / 756.0", "phase"),
    ("beta mass factor", "113.0 * m1 * m1", "114.13 * m1 * m1", "phase"),
    ("beta eta factor", "75.0 * s->eta) + c2", "75.75 * s->eta) + c2", "phase"),
    ("sigma factor", "79.0 / 8.0", "79.79 / 8.0", "phase"),
    ("plus inclination factor", "s->hp_fac = 0.5 * (1.0 + ci * ci);", "s->hp_fac = 0.505 * (1.0 + ci * ci);",
     "polarisation"),
    ("cross inclination factor", "s->hx_fac = ci;", "s->hx_fac = 1.01 * ci;", "polarisation"),
    ("cross part real", "double xr = s->hx_fac * bi, xi = -s->hx_fac * br;",
     "double xr = s->hx_fac * br, xi = s->hx_fac * bi;", "polarisation"),
    ("information", "*H = h - z;", "*H = h - 1.01 * z;", "posterior"),
    ("Kish ESS", "*ess = 1.0 / s2;", "*ess = 1.01 / s2;", "posterior"),
    ("resample positions", "((double)m + u0) / (double)n_out * acc",
     "((double)m + u0) / (double)n_out * acc * 0.99", "resample"),
    ("no wrap of periodic coordinates", "if (is_periodic(p, i)) y[i] -= floor(y[i]);",
     "if (is_periodic(p, i)) y[i] -= 0.0;", "wrap"),
    ("wrap to the centred interval", "if (is_periodic(p, i)) y[i] -= floor(y[i]);",
     "if (is_periodic(p, i)) y[i] -= floor(y[i] + 0.5);", "wrap"),
    ("2.5PN spin-orbit (chi_s)", "*g5 = (732985.0 / 2268.0 - 24260.0 * eta / 81.0",
     "*g5 = (1.01 * 732985.0 / 2268.0 - 24260.0 * eta / 81.0", "so_phase"),
    ("2.5PN spin-orbit (chi_a)", "+ (732985.0 / 2268.0 + 140.0 * eta / 9.0) * delta * ca;",
     "+ (732985.0 / 2268.0 + 1.01 * 140.0 * eta / 9.0) * delta * ca;", "so_phase"),
    ("3PN spin-orbit tail", "*so6 = PI * (2270.0 / 3.0 * delta * ca + (2270.0 / 3.0 - 520.0 * eta) * cs);",
     "*so6 = PI * (2270.0 / 3.0 * delta * ca + (2270.0 / 3.0 - 525.2 * eta) * cs);", "so_phase"),
    ("3.5PN spin-orbit (chi_s)", "*so7 = (-25150083775.0 / 3048192.0 + 10566655595.0 * eta / 762048.0",
     "*so7 = (-25150083775.0 / 3048192.0 + 1.01 * 10566655595.0 * eta / 762048.0", "so_phase"),
    ("3.5PN spin-orbit (chi_a)", "+ delta * (-25150083775.0 / 3048192.0 + 26804935.0 * eta / 6048.0",
     "+ delta * (-25150083775.0 / 3048192.0 + 1.01 * 26804935.0 * eta / 6048.0", "so_phase"),
    ("walk scale", "double g_de = 2.38 / sqrt(2.0 * d);", "double g_de = 2.4 / sqrt(2.0 * d);", "walk_step"),
    ("walk pair not distinct", "if (ib >= ia) ++ib;", "if (ib > ia) ++ib;", "walk_step"),
    ("walk stops at a count of acceptances", "for (int s = 0; s < n_prop; ++s) {",
     "for (int s = 0; s < n_prop && *n_acc < 4; ++s) {", "walk_invariance"),
    ("right expansions not counted", "hi += w;\n        ++mv->expansions;", "hi += w;", "moves"),
    ("accepted candidate counted as a shrink", "mv->moved = 1;\n",
     "mv->moved = 1;\n            ++mv->shrinks;\n", "moves"),
    ("histogram bin off by one", "+ (pe < ORC_PROBE_HIST - 1 ? pe : ORC_PROBE_HIST - 1)] += 1;",
     "+ (pe + 1 < ORC_PROBE_HIST - 1 ? pe + 1 : ORC_PROBE_HIST - 1)] += 1;", "trace"),
    ("remaining evidence offset", "rec->log_remaining = logz_live - r->logZ;",
     "rec->log_remaining = logz_live - r->logZ + 1e-9;", "trace"),
]


def _walk(L, p, o, pop, n_prop, x0, lstar, t, j):
    x = np.ascontiguousarray(x0, dtype=np.float64).copy()
    lx, ev = C.c_double(0.0), C.c_long()
    acc = L.orc_walk_from(p.ref, C.byref(o), pop.ctypes.data_as(oracle._dp), len(pop), n_prop,
                          x.ctypes.data_as(oracle._dp), C.byref(lx), lstar, t, j, C.byref(ev))
    return x, ev.value, acc


def _walk_step_bad(L):
    """The hand-computed single proposals of test_walk_step_by_hand."""
    d = 2
    w = synth.gauss_workload(d, 10.0)
    w.kernel, w.walk_accept, w.walk_max = 1, 1, 1
    o = oracle.opts_for(w)
    p = oracle.OracleProblem(w)
    pop = np.array([[0.1, 0.2], [0.7, 0.9], [0.4, 0.35], [0.55, 0.05]])
    x0 = np.array([0.5, 0.5])
    for j in range(12):
        words = oracle.philox([0, j, 0, 8 << 48], [w.sampler_seed, 0])
        u = [(x >> 11) * 2.0**-53 for x in words]
        a = int(math.floor(u[0] * 4))
        b = int(math.floor(u[1] * 3))
        b += b >= a
        g = (1.0 if u[2] < 0.5 else 2.38 / math.sqrt(2 * d)) * (0.9 + 0.2 * u[3])
        y = x0 + g * (pop[a] - pop[b])
        inside = bool(np.all((y >= 0) & (y <= 1)))
        x, _, _ = _walk(L, p, o, pop, 1, x0, -np.inf, 0, j)
        if np.max(np.abs(x - (y if inside else x0))) > 1e-15:
            return True
    return False


def _walk_invariance_bad(L):
    """The constrained-prior invariance of test_walk_chains_keep_the_constrained_prior."""
    from scipy import stats

    d, s, rho = 3, 0.1, 0.3
    w = synth.gauss_workload(d, s)
    w.kernel, w.walk_accept, w.walk_max = 1, 12, 400
    o = oracle.opts_for(w)
    p = oracle.OracleProblem(w)
    rng = np.random.default_rng(4)
    pop = rng.uniform(0.5 - rho, 0.5 + rho, (4000, d))
    pop = np.ascontiguousarray(pop[np.linalg.norm(pop - 0.5, axis=1) < rho][:500])
    c = 0.5 * d * math.log(2 * math.pi * s * s)
    lstar = -(rho**2) / (2 * s * s) - c
    starts = pop[rng.integers(0, len(pop), 1500)]
    pts = np.array([_walk(L, p, o, pop, 30, starts[j], lstar, 2, j)[0] for j in range(1500)])
    r = np.linalg.norm(pts - 0.5, axis=1)
    return stats.kstest((r / rho) ** d, "uniform").pvalue <= 1e-3


def _wrap_bad(L):
    """The hand-computed wrapped slice move (test_wrapped_slice_hand_computed),
    driven through the build L: the accepted point must lie in [0, 1] and
    equal the line point modulo 1, after a full step-out budget."""
    w = synth.gauss_workload(1, 0.1, mu=[0.5])
    w.slice_width = 0.15
    w.periodic = np.array([1], dtype=np.int32)
    p = oracle.OracleProblem(w)
    o = oracle.opts_for(w)
    x = np.array([0.95])
    d = np.array([1.0])
    us = np.array([0.3])
    lx, ev = C.c_double(0.0), C.c_long()
    L.orc_slice_update_fixed(p.ref, C.byref(o), x.ctypes.data_as(oracle._dp), C.byref(lx),
                             d.ctypes.data_as(oracle._dp), -1e300, 0.5, 0.5, us.ctypes.data_as(oracle._dp), 1,
                             C.byref(ev), None)
    return not (0.0 <= x[0] <= 1.0 and ev.value == 100 and abs(x[0] - 0.875) < 1e-9)


def _moves_bad(L):
    """The hand-counted slice moves of test_slice_hand_computed, driven
    through the build L."""
    w = synth.gauss_workload(1, 0.1, mu=[0.5])
    w.slice_width = 0.15
    p = oracle.OracleProblem(w)
    o = oracle.opts_for(w)
    c = 0.5 * math.log(2 * math.pi * 0.01)
    lstar = -0.04 / 0.02 - c
    cases = [([0.5], lstar, 0.5, [0.0, 0.9, 0.25], (2, 1, 1)), ([0.5], lstar, 0.0, [0.0], (1, 0, 1)),
             ([0.05], -1e300, 0.5, [0.01, 0.0, 0.5], (6, 2, 1))]
    for x0, ls, uj, us, want in cases:
        x = np.array(x0, dtype=np.float64)
        d = np.array([1.0])
        u = np.array(us, dtype=np.float64)
        lx, ev = C.c_double(-c), C.c_long()
        mv = np.zeros(3, dtype=np.int32)
        L.orc_slice_update_fixed(p.ref, C.byref(o), x.ctypes.data_as(oracle._dp), C.byref(lx),
                                 d.ctypes.data_as(oracle._dp), ls, 0.5, uj, u.ctypes.data_as(oracle._dp), len(u),
                                 C.byref(ev), mv.ctypes.data_as(oracle._ip))
        if tuple(int(v) for v in mv) != want:
            return True
    return False


def _trace_bad(L):
    """The per-iteration record's histogram sums and remaining-evidence
    term (test_iteration_metrics_closed_forms_and_invariants), driven through
    the build L."""
    n, k = 100, 50
    w = synth.gauss_workload(2, 0.05, n_live=n, n_delete=k)
    p = oracle.OracleProblem(w)
    o = oracle.opts_for(w, term_frac=0.0, max_iter=3)
    h = C.c_void_p()
    assert L.orc_init(C.byref(h), p.ref, C.byref(o)) == 0
    done = C.c_int()
    L.orc_step(h, 3, C.byref(done))
    recs = (oracle.IterRec * 3)()
    n_out = C.c_long()
    L.orc_trace(h, 3, recs, C.byref(n_out))
    u, lam = np.zeros((n, 2)), np.zeros(n)
    L.orc_live(h, u.ctypes.data_as(oracle._dp), lam.ctypes.data_as(oracle._dp))
    L.orc_free(h)
    tr = oracle.trace_dict(recs[: n_out.value])
    mx = lam.max()
    rem = tr["logX"][-1] + mx + math.log(np.mean(np.exp(lam - mx))) - tr["logZ"][-1]
    return (n_out.value != 3 or not np.array_equal(tr["hist"] @ np.arange(oracle.PROBE_HIST), tr["probes"])
            or abs(tr["log_remaining"][-1] - rem) >= 1e-12 * max(1.0, abs(rem)))


def _posterior_bad(L):
    """The constant-likelihood pins of H (zero) and the Kish ESS (closed form),
    driven through the build L."""
    w = synth.gauss_workload(3, 1e8, n_live=100, n_delete=50)
    p = oracle.OracleProblem(w)
    o = oracle.opts_for(w, max_iter=30, term_frac=0.0)
    h = C.c_void_p()
    assert L.orc_init(C.byref(h), p.ref, C.byref(o)) == 0
    done = C.c_int()
    L.orc_step(h, 30, C.byref(done))
    H, ess = C.c_double(), C.c_double()
    L.orc_information(h, C.byref(H), C.byref(ess))
    L.orc_free(h)
    want = pins._constant_likelihood_ess(100, 50, 30)
    return abs(H.value) >= 1e-9 or abs(ess.value - want) >= 1e-9 * want


def _resample_bad(L):
    """The systematic-resampling count property, driven through the build L."""
    w = synth.gauss_workload(2, 0.08, mu=[0.2, 0.5], n_live=200, n_delete=100)
    p = oracle.OracleProblem(w)
    o = oracle.opts_for(w, seed=5)
    h = C.c_void_p()
    assert L.orc_init(C.byref(h), p.ref, C.byref(o)) == 0
    done = C.c_int()
    L.orc_step(h, 1000, C.byref(done))
    nd, ne = C.c_long(), C.c_long()
    L.orc_state(h, None, None, None, None, C.byref(nd), C.byref(ne))
    tot = nd.value + 200
    lw = np.zeros(tot)
    n_out = C.c_long()
    L.orc_samples(h, tot, None, None, lw.ctypes.data_as(oracle._dp), C.byref(n_out))
    bad = False
    for n in (17, 1000):
        idx = np.zeros(n, dtype=np.int32)
        L.orc_resample(h, n, idx.ctypes.data_as(oracle._ip), None)
        cum = n * np.cumsum(np.exp(lw)) / np.exp(lw).sum()
        drawn = np.cumsum(np.bincount(idx, minlength=tot))
        bad = bad or bool(np.max(np.abs(drawn - cum)) >= 1.0 + 1e-9)
    L.orc_free(h)
    return bad


CHECKS = {
    "phase": lambda L: pins._eb_worst(L) >= 1.0,
    "polarisation": lambda L: pins._polarisation_worst(L) >= 1e-11,
    "posterior": _posterior_bad,
    "resample": _resample_bad,
    "wrap": _wrap_bad,
    "walk_step": _walk_step_bad,
    "so_phase": lambda L: pins._so_worst(L) >= 1.0,
    "walk_invariance": _walk_invariance_bad,
    "moves": _moves_bad,
    "trace": _trace_bad,
}


def _compile(src_text, path):
    c = path + ".c"
    with open(c, "w") as fh:
        fh.write(src_text)
    subprocess.run(["gcc", "-O1", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-I", os.path.dirname(oracle.SRC),
                    "-o", path, c, "-lm"], check=True)


@pytest.fixture(scope="module")
def mutants():
    src = open(oracle.SRC).read()
    tmp = tempfile.mkdtemp(prefix="orc_mut_")
    jobs = []
    for i, (name, old, new, _) in enumerate(MUTATIONS):
        assert src.count(old) == 1, name          # each mutation hits exactly one place
        jobs.append((src.replace(old, new), os.path.join(tmp, f"mut{i}.so")))
    with ThreadPoolExecutor(max_workers=8) as ex:
        list(ex.map(lambda j: _compile(*j), jobs))
    return [oracle.load(path) for _, path in jobs]


def test_unmutated_oracle_passes_every_check():
    L = oracle.lib()
    for kind, bad in CHECKS.items():
        assert not bad(L), kind


@pytest.mark.parametrize("i", range(len(MUTATIONS)), ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(mutants, i):
    name, _, _, kind = MUTATIONS[i]
    assert CHECKS[kind](mutants[i]), f"the {kind} pin misses a changed {name}"
