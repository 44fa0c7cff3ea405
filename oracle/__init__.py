"""Python access to the reference oracle (``nsorc.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The HIP library never imports this
package, and this package never imports the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liborc.so")
SRC = os.path.join(_HERE, "nsorc.c")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over chains only)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"],
                       check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Problem(C.Structure):
    _fields_ = [
        ("model", C.c_int), ("likelihood", C.c_int), ("n_dim", C.c_int),
        ("prior_kind", _ip), ("prior_lo", _dp), ("prior_hi", _dp),
        ("f_lo", C.c_double), ("df", C.c_double), ("n_bins", C.c_int), ("n_det", C.c_int),
        ("data_re", _dp), ("data_im", _dp), ("psd", _dp), ("det_geom", _dp),
        ("gmst", C.c_double), ("fixed_dist_mpc", C.c_double),
        ("rb_n_bins", C.c_int), ("rb_fiducial", _dp), ("gauss_mu", _dp), ("gauss_sigma", C.c_double),
        ("periodic", _ip),
    ]


class Opts(C.Structure):
    _fields_ = [
        ("n_live", C.c_int), ("n_delete", C.c_int), ("n_steps", C.c_int), ("slice_width", C.c_double),
        ("max_stepout", C.c_int), ("max_shrink", C.c_int), ("term_frac", C.c_double),
        ("seed", C.c_uint64), ("run_id", C.c_uint64), ("max_iter", C.c_int), ("n_threads", C.c_int),
        ("kernel", C.c_int), ("walk_accept", C.c_int), ("walk_max", C.c_int),
    ]


_lib = None


PROBE_HIST = 32


class IterRec(C.Structure):
    """orc_iter: one iteration's metrics."""
    _fields_ = [("iter", C.c_int), ("probes_min", C.c_int), ("probes_max", C.c_int), ("pad", C.c_int),
                ("lstar", C.c_double), ("logX", C.c_double), ("logZ", C.c_double), ("log_remaining", C.c_double),
                ("probes", C.c_longlong), ("steps", C.c_longlong), ("accepted", C.c_longlong),
                ("stepouts", C.c_longlong), ("shrinks", C.c_longlong), ("hist", C.c_int * PROBE_HIST)]


def load(path: str):
    """A CDLL of an oracle build at ``path`` with every signature set."""
    L = C.CDLL(path)
    L.orc_philox4x64.argtypes = [C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
    L.orc_prior_transform.argtypes = [C.c_void_p, _dp, _dp]
    L.orc_antenna.argtypes = [_dp, C.c_double, C.c_double, C.c_double, C.c_double, _dp, _dp, _dp]
    L.orc_waveform.argtypes = [C.c_void_p, _dp, C.c_int, C.c_int, _dp, _dp]
    L.orc_tf2_phase.argtypes = [C.c_double] * 7
    L.orc_tf2_phase.restype = C.c_double
    L.orc_tf2_phase_so.argtypes = [C.c_double] * 10
    L.orc_tf2_phase_so.restype = C.c_double
    L.orc_pn_params_so.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
    L.orc_inner.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp]
    L.orc_inner.restype = C.c_double
    L.orc_noise_loglike.argtypes = [C.c_void_p]
    L.orc_noise_loglike.restype = C.c_double
    L.orc_loglike_full.argtypes = [C.c_void_p, _dp]
    L.orc_loglike_full.restype = C.c_double
    L.orc_rb_build.argtypes = [C.c_void_p]
    L.orc_rb_build.restype = C.c_void_p
    L.orc_rb_free.argtypes = [C.c_void_p]
    L.orc_rb_edges.argtypes = [C.c_void_p, _ip]
    L.orc_loglike_rb.argtypes = [C.c_void_p, _dp]
    L.orc_loglike_rb.restype = C.c_double
    L.orc_loglike_gauss.argtypes = [C.c_void_p, _dp]
    L.orc_loglike_gauss.restype = C.c_double
    L.orc_loglike_batch.argtypes = [C.c_void_p, _dp, C.c_long, _dp, C.c_int]
    L.orc_select.argtypes = [C.c_int, _dp, C.c_int, _ip, _dp]
    L.orc_init.argtypes = [C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p]
    L.orc_step.argtypes = [C.c_void_p, C.c_int, _ip]
    L.orc_state.argtypes = [C.c_void_p, _dp, _dp, _dp, _ip, C.POINTER(C.c_long), C.POINTER(C.c_long)]
    L.orc_live.argtypes = [C.c_void_p, _dp, _dp]
    L.orc_dead.argtypes = [C.c_void_p, C.c_long, _dp, _dp, _dp, _dp, _ip, _ip, C.POINTER(C.c_long)]
    L.orc_logZ.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp]
    L.orc_samples.argtypes = [C.c_void_p, C.c_long, _dp, _dp, _dp, C.POINTER(C.c_long)]
    L.orc_information.argtypes = [C.c_void_p, _dp, _dp]
    L.orc_walk_from.argtypes = [C.c_void_p, C.c_void_p, _dp, C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_uint64,
                                C.c_uint64, C.POINTER(C.c_long)]
    L.orc_resample.argtypes = [C.c_void_p, C.c_long, _ip, _dp]
    L.orc_pn_params.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
    L.orc_free.argtypes = [C.c_void_p]
    L.orc_slice_update_fixed.argtypes = [C.c_void_p, C.c_void_p, _dp, _dp, _dp, C.c_double, C.c_double,
                                         C.c_double, _dp, C.c_int, C.POINTER(C.c_long), _ip]
    L.orc_trace.argtypes = [C.c_void_p, C.c_long, C.POINTER(IterRec), C.POINTER(C.c_long)]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=True)
        _lib = load(LIB_PATH)
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


class OracleProblem:
    """Holds the numpy arrays a ``Problem`` points to (keeps them alive)."""

    def __init__(self, w, data_re=None, data_im=None, fixed_dist_mpc=None, rb_fiducial=None, psd=None):
        self.w = w
        self.kind = np.ascontiguousarray(w.prior_kind, dtype=np.int32)
        self.lo = np.ascontiguousarray(w.prior_lo, dtype=np.float64)
        self.hi = np.ascontiguousarray(w.prior_hi, dtype=np.float64)
        nd, nb = max(w.n_det, 1), max(w.n_bins, 1)
        if psd is None:
            psd = w.psd() if w.n_bins else np.ones((nd, nb))
        self.psd = np.ascontiguousarray(psd, dtype=np.float64)
        self.geom = np.ascontiguousarray(w.det_geom() if w.n_det else np.zeros((1, 9)), dtype=np.float64)
        z = np.zeros((nd, nb))
        self.dre = np.ascontiguousarray(z if data_re is None else data_re, dtype=np.float64)
        self.dim = np.ascontiguousarray(z if data_im is None else data_im, dtype=np.float64)
        fid = w.theta_inj if rb_fiducial is None else rb_fiducial
        self.fid = np.ascontiguousarray(fid, dtype=np.float64)
        self.mu = np.ascontiguousarray(w.gauss_mu if len(w.gauss_mu) else np.zeros(w.n_dim), dtype=np.float64)
        per = getattr(w, "periodic", None)
        self.per = np.ascontiguousarray(per, dtype=np.int32) if per is not None and len(per) else None
        self.s = Problem(
            model=w.model, likelihood=w.likelihood, n_dim=w.n_dim,
            prior_kind=_i(self.kind), prior_lo=_d(self.lo), prior_hi=_d(self.hi),
            f_lo=w.f_lo, df=w.df, n_bins=w.n_bins, n_det=w.n_det,
            data_re=_d(self.dre), data_im=_d(self.dim), psd=_d(self.psd), det_geom=_d(self.geom),
            gmst=w.gmst, fixed_dist_mpc=(w.fixed_dist_mpc if fixed_dist_mpc is None else fixed_dist_mpc),
            rb_n_bins=w.rb_n_bins, rb_fiducial=_d(self.fid), gauss_mu=_d(self.mu), gauss_sigma=w.gauss_sigma,
            periodic=_i(self.per) if self.per is not None else None,
        )

    @property
    def ref(self):
        return C.byref(self.s)

    # -- physics helpers -------------------------------------------------
    def waveform(self, theta, det: int, cut: bool = True):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        hr = np.zeros(self.w.n_bins)
        hi = np.zeros(self.w.n_bins)
        rc = lib().orc_waveform(self.ref, _d(th), det, 1 if cut else 0, _d(hr), _d(hi))
        if rc:
            raise ValueError("orc_waveform failed")
        return hr, hi

    def noise_loglike(self) -> float:
        return lib().orc_noise_loglike(self.ref)

    def inner(self, det, a_re, a_im, b_re, b_im):
        a_re, a_im, b_re, b_im = (np.ascontiguousarray(x, dtype=np.float64) for x in (a_re, a_im, b_re, b_im))
        return lib().orc_inner(self.ref, det, _d(a_re), _d(a_im), _d(b_re), _d(b_im))

    def prior_transform(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        flat = u.reshape(-1, self.w.n_dim)
        th = np.zeros_like(flat)
        for i in range(flat.shape[0]):
            row, out = np.ascontiguousarray(flat[i]), np.zeros(self.w.n_dim)
            lib().orc_prior_transform(self.ref, _d(row), _d(out))
            th[i] = out
        return th.reshape(u.shape)

    def loglike_theta(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        return lib().orc_loglike_full(self.ref, _d(th))

    def pn_params(self, theta):
        """(eta, beta, sigma) of a physical parameter point."""
        th = np.ascontiguousarray(theta, dtype=np.float64)
        e, b, s = C.c_double(), C.c_double(), C.c_double()
        if lib().orc_pn_params(self.ref, _d(th), C.byref(e), C.byref(b), C.byref(s)):
            raise ValueError("orc_pn_params failed")
        return e.value, b.value, s.value

    def loglike_batch(self, u, n_threads: int = 1):
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, self.w.n_dim)
        out = np.zeros(u.shape[0])
        rc = lib().orc_loglike_batch(self.ref, _d(u), u.shape[0], _d(out), n_threads)
        if rc:
            raise ValueError("orc_loglike_batch failed")
        return out


class RB:
    """Relative-binning summary data built by the oracle at the fiducial point."""

    def __init__(self, prob: OracleProblem):
        self.prob = prob
        self.h = lib().orc_rb_build(prob.ref)
        if not self.h:
            raise ValueError("orc_rb_build failed")

    def edges(self):
        e = np.zeros(self.prob.w.rb_n_bins + 1, dtype=np.int32)
        lib().orc_rb_edges(self.h, _i(e))
        return e

    def loglike_theta(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        return lib().orc_loglike_rb(self.h, _d(th))

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_rb_free(self.h)
            self.h = None


def philox(ctr, key):
    c = (C.c_uint64 * 4)(*ctr)
    k = (C.c_uint64 * 2)(*key)
    o = (C.c_uint64 * 4)()
    lib().orc_philox4x64(c, k, o)
    return [int(x) for x in o]


def select(logl, k):
    logl = np.ascontiguousarray(logl, dtype=np.float64)
    dead = np.zeros(k, dtype=np.int32)
    ls = C.c_double()
    rc = lib().orc_select(len(logl), _d(logl), k, _i(dead), C.byref(ls))
    if rc:
        raise ValueError("orc_select failed")
    return dead, ls.value


def antenna(geom9, ra, dec, psi, gmst):
    g = np.ascontiguousarray(geom9, dtype=np.float64)
    fp, fc, dt = C.c_double(), C.c_double(), C.c_double()
    lib().orc_antenna(_d(g), ra, dec, psi, gmst, C.byref(fp), C.byref(fc), C.byref(dt))
    return fp.value, fc.value, dt.value


def opts_for(w, n_threads: int = 1, seed=None, run_id: int = 0, max_iter: int = 1000, term_frac=None,
             n_live=None, n_delete=None, n_steps=None, kernel=None, walk_accept=None, walk_max=None):
    return Opts(
        n_live=w.n_live if n_live is None else n_live, n_delete=w.n_delete if n_delete is None else n_delete,
        n_steps=w.n_steps if n_steps is None else n_steps, slice_width=w.slice_width,
        max_stepout=w.max_stepout, max_shrink=w.max_shrink,
        term_frac=w.term_frac if term_frac is None else term_frac,
        seed=w.sampler_seed if seed is None else seed, run_id=run_id, max_iter=max_iter, n_threads=n_threads,
        kernel=w.kernel if kernel is None else kernel,
        walk_accept=w.walk_accept if walk_accept is None else walk_accept,
        walk_max=w.walk_max if walk_max is None else walk_max,
    )


def make_data(w, fixed_dist_mpc=None):
    """Seeded noise plus the oracle's own injected waveform (ISCO-cut)."""
    re, im = w.noise()
    prob = OracleProblem(w, fixed_dist_mpc=fixed_dist_mpc)
    for det in range(w.n_det):
        hr, hi = prob.waveform(w.theta_inj, det, cut=True)
        re[det] += hr
        im[det] += hi
    return re, im


class Run:
    """A nested sampling run of the oracle."""

    def __init__(self, prob: OracleProblem, opts: Opts):
        self.prob = prob
        self.opts = opts
        h = C.c_void_p()
        rc = lib().orc_init(C.byref(h), prob.ref, C.byref(opts))
        if rc:
            raise ValueError(f"orc_init failed ({rc})")
        self.h = h

    def step(self, max_iters: int = 1) -> bool:
        done = C.c_int()
        lib().orc_step(self.h, max_iters, C.byref(done))
        return bool(done.value)

    def run(self, max_iters: int = 100000) -> bool:
        return self.step(max_iters)

    def state(self):
        lx, lz, H = C.c_double(), C.c_double(), C.c_double()
        it = C.c_int()
        nd, ne = C.c_long(), C.c_long()
        lib().orc_state(self.h, C.byref(lx), C.byref(lz), C.byref(H), C.byref(it), C.byref(nd), C.byref(ne))
        return dict(logX=lx.value, logZ=lz.value, H=H.value, iter=it.value, n_dead=nd.value, n_evals=ne.value)

    def live(self):
        n, d = self.opts.n_live, self.prob.w.n_dim
        u = np.zeros((n, d))
        l = np.zeros(n)
        lib().orc_live(self.h, _d(u), _d(l))
        return u, l

    def dead(self):
        nd = self.state()["n_dead"]
        d = self.prob.w.n_dim
        u = np.zeros((max(nd, 1), d))
        l, lx, lw = (np.zeros(max(nd, 1)) for _ in range(3))
        it = np.zeros(max(nd, 1), dtype=np.int32)
        sl = np.zeros(max(nd, 1), dtype=np.int32)
        n_out = C.c_long()
        lib().orc_dead(self.h, max(nd, 1), _d(u), _d(l), _d(lx), _d(lw), _i(it), _i(sl), C.byref(n_out))
        return dict(u=u[:nd], logl=l[:nd], logx=lx[:nd], logw=lw[:nd], iter=it[:nd], slot=sl[:nd])

    def logZ(self, n_sim: int = 200):
        z, ss, sh, ess = C.c_double(), C.c_double(), C.c_double(), C.c_double()
        lib().orc_logZ(self.h, n_sim, C.byref(z), C.byref(ss), C.byref(sh), C.byref(ess))
        return dict(logZ=z.value, sigma=ss.value, sigma_h=sh.value, ess=ess.value)

    def information(self):
        """Information H of the posterior against the prior and the Kish ESS."""
        h, e = C.c_double(), C.c_double()
        lib().orc_information(self.h, C.byref(h), C.byref(e))
        return h.value, e.value

    def samples(self):
        st = self.state()
        tot = st["n_dead"] + self.opts.n_live
        d = self.prob.w.n_dim
        th = np.zeros((tot, d))
        l = np.zeros(tot)
        lw = np.zeros(tot)
        n_out = C.c_long()
        lib().orc_samples(self.h, tot, _d(th), _d(l), _d(lw), C.byref(n_out))
        return th, l, lw

    def trace(self):
        """Per-iteration metrics of the iterations so far: a dict of arrays
        (one entry per iteration; hist has one row per iteration)."""
        n = self.state()["iter"]
        recs = (IterRec * max(n, 1))()
        n_out = C.c_long()
        if lib().orc_trace(self.h, max(n, 1), recs, C.byref(n_out)):
            raise ValueError("orc_trace failed")
        return trace_dict(recs[: n_out.value])

    def resample(self, n_out: int):
        """Equal-weight samples by systematic resampling: (indices into the
        samples() order, physical parameters)."""
        idx = np.zeros(n_out, dtype=np.int32)
        th = np.zeros((n_out, self.prob.w.n_dim))
        if lib().orc_resample(self.h, n_out, _i(idx), _d(th)):
            raise ValueError("orc_resample failed")
        return idx, th

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_free(self.h)
            self.h = None


def trace_dict(recs):
    """Columns of a sequence of per-iteration records."""
    names = [f[0] for f in IterRec._fields_ if f[0] not in ("pad", "hist")]
    out = {k: np.array([getattr(r, k) for r in recs]) for k in names}
    out["hist"] = np.array([list(r.hist) for r in recs], dtype=np.int64).reshape(len(recs), PROBE_HIST)
    return out


def walk_from(prob: OracleProblem, opts: Opts, pop, n_prop: int, x, lx, lstar, t: int = 0, j: int = 0):
    """One random-walk chain of n_prop proposals from x over the population
    pop (all survivors); returns (x, lambda, likelihood calls, accepted)."""
    pop = np.ascontiguousarray(pop, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).copy()
    lxc = C.c_double(lx)
    ev = C.c_long()
    acc = lib().orc_walk_from(prob.ref, C.byref(opts), _d(pop), len(pop), n_prop, _d(x), C.byref(lxc), lstar, t, j,
                              C.byref(ev))
    if acc < 0:
        raise ValueError("orc_walk_from failed")
    return x, lxc.value, ev.value, acc


def slice_update_fixed(prob: OracleProblem, opts: Opts, x, lx, direction, lstar, uw, uj, ushr, moves=False):
    """One slice update with given direction and uniforms: (x, lambda,
    likelihood calls), and with moves=True also (bracket expansions, rejected
    shrink candidates, 1 if the point moved)."""
    x = np.ascontiguousarray(x, dtype=np.float64).copy()
    d = np.ascontiguousarray(direction, dtype=np.float64)
    us = np.ascontiguousarray(ushr, dtype=np.float64)
    lxc = C.c_double(lx)
    ev = C.c_long()
    mv = np.zeros(3, dtype=np.int32)
    lib().orc_slice_update_fixed(prob.ref, C.byref(opts), _d(x), C.byref(lxc), _d(d), lstar, uw, uj, _d(us),
                                 len(us), C.byref(ev), _i(mv))
    if moves:
        return x, lxc.value, ev.value, tuple(int(v) for v in mv)
    return x, lxc.value, ev.value
