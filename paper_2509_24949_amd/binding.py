"""Thin Python binding of libns (include/ns.h): argument marshalling only.

Every computation runs in the HIP library.  PyTorch supplies device memory
and the stream.  Importing this module fails loudly when libns.so has not
been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import synth

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libns.so")

NS_OK, NS_E_ARG, NS_E_OOM, NS_E_HIP, NS_E_CAPACITY, NS_E_STATE = 0, -1, -2, -3, -4, -5
NS_FP64, NS_MIXED = 0, 1
NS_KERNEL_SLICE, NS_KERNEL_WALK = 0, 1
NS_LOGLIKE_NOALLOC_MAX = 16384

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_lp = C.POINTER(C.c_long)


class NSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libns error {code}: {msg}")
        self.code = code


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
        ("seed", C.c_uint64), ("run_id", C.c_uint64), ("max_iter", C.c_int), ("precision", C.c_int),
        ("kernel", C.c_int), ("walk_accept", C.c_int), ("walk_max", C.c_int), ("count_moves", C.c_int),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("iterations", C.c_long), ("ms_select", C.c_double), ("ms_prep", C.c_double),
        ("ms_slice", C.c_double), ("ms_term", C.c_double), ("evals", C.c_longlong),
        ("bin_terms", C.c_longlong), ("slice_threads", C.c_int), ("lds_tables", C.c_int),
    ]


PROBE_HIST = 32


class IterRec(C.Structure):
    """ns_iter_t: one iteration's metrics."""
    _fields_ = [
        ("iter", C.c_int), ("probes_min", C.c_int), ("probes_max", C.c_int), ("pad", C.c_int),
        ("lstar", C.c_double), ("logX", C.c_double), ("logZ", C.c_double), ("log_remaining", C.c_double),
        ("probes", C.c_longlong), ("steps", C.c_longlong), ("accepted", C.c_longlong),
        ("stepouts", C.c_longlong), ("shrinks", C.c_longlong), ("hist", C.c_int * PROBE_HIST),
    ]


# Every entry point of include/ns.h with its ctypes signature.
class TicketInfo(C.Structure):
    _fields_ = [
        ("ticket", C.c_longlong), ("status", C.c_int), ("done", C.c_int), ("iterations", C.c_int),
        ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_finish", C.c_double), ("bytes", C.c_size_t),
    ]


NS_SERVER_GRAPH = 1

SIGNATURES = {
    "ns_init": (C.c_int, [C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p, C.c_void_p]),
    "ns_step": (C.c_int, [C.c_void_p, C.c_int, _ip]),
    "ns_step_async": (C.c_int, [C.c_void_p, C.c_int]),
    "ns_logZ": (C.c_int, [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp]),
    "ns_samples": (C.c_int, [C.c_void_p, C.c_long, _dp, _dp, _dp, _lp]),
    "ns_resample": (C.c_int, [C.c_void_p, C.c_long, _ip, _dp]),
    "ns_state": (C.c_int, [C.c_void_p, _dp, _dp, _dp, _ip, _lp, _lp, _ip]),
    "ns_live": (C.c_int, [C.c_void_p, _dp, _dp]),
    "ns_dead": (C.c_int, [C.c_void_p, C.c_long, _dp, _dp, _dp, _dp, _ip, _ip, _lp]),
    "ns_loglike": (C.c_int, [C.c_void_p, C.c_void_p, C.c_long, C.c_void_p, C.c_void_p]),
    "ns_loglike_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_long, C.c_void_p, C.c_void_p]),
    "ns_waveform": (C.c_int, [C.c_void_p, _dp, C.c_int, C.c_int, _dp, _dp, C.c_void_p]),
    "ns_select": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ns_profile": (C.c_int, [C.c_void_p, C.c_int]),
    "ns_stats": (C.c_int, [C.c_void_p, C.POINTER(Stats)]),
    "ns_trace": (C.c_int, [C.c_void_p, C.c_long, C.POINTER(IterRec), _lp]),
    "ns_noise_loglike": (C.c_int, [C.c_void_p, _dp]),
    "ns_save": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t)]),
    "ns_load": (C.c_int, [C.POINTER(C.c_void_p), C.c_void_p, C.c_size_t, C.c_void_p]),
    "ns_free": (None, [C.c_void_p]),
    "ns_server_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_size_t, C.c_int, C.c_int, C.c_void_p]),
    "ns_server_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_longlong)]),
    "ns_server_tick": (C.c_int, [C.c_void_p, C.c_int, _ip, _ip, _ip]),
    "ns_server_poll": (C.c_int, [C.c_void_p, C.POINTER(TicketInfo), C.c_int, _ip]),
    "ns_server_take": (C.c_int, [C.c_void_p, C.c_longlong, C.POINTER(C.c_void_p)]),
    "ns_server_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t), _ip, _ip]),
    "ns_server_free": (None, [C.c_void_p]),
    "ns_last_error": (C.c_char_p, []),
}

_lib = None


def lib():
    """The loaded libns.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2509_24949_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != NS_OK:
        raise NSError(rc, lib().ns_last_error().decode())


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return C.c_void_p(0)


class ProblemSpec:
    """An ns_problem built from a workload and its data; owns the arrays."""

    def __init__(self, w: synth.Workload, data_re=None, data_im=None, rb_fiducial=None):
        self.w = w
        self.kind = np.ascontiguousarray(w.prior_kind, dtype=np.int32)
        self.lo = np.ascontiguousarray(w.prior_lo, dtype=np.float64)
        self.hi = np.ascontiguousarray(w.prior_hi, dtype=np.float64)
        nd, nb = max(w.n_det, 1), max(w.n_bins, 1)
        self.psd = np.ascontiguousarray(w.psd() if w.n_bins else np.ones((nd, nb)), dtype=np.float64)
        self.geom = np.ascontiguousarray(w.det_geom() if w.n_det else np.zeros((1, 9)), dtype=np.float64)
        z = np.zeros((nd, nb))
        self.dre = np.ascontiguousarray(z if data_re is None else data_re, dtype=np.float64)
        self.dim = np.ascontiguousarray(z if data_im is None else data_im, dtype=np.float64)
        self.fid = np.ascontiguousarray(w.theta_inj if rb_fiducial is None else rb_fiducial, dtype=np.float64)
        self.mu = np.ascontiguousarray(w.gauss_mu if len(w.gauss_mu) else np.zeros(w.n_dim), dtype=np.float64)
        self.per = np.ascontiguousarray(w.periodic, dtype=np.int32) if len(w.periodic) else None
        self.s = Problem(
            model=w.model, likelihood=w.likelihood, n_dim=w.n_dim,
            prior_kind=_i(self.kind), prior_lo=_d(self.lo), prior_hi=_d(self.hi),
            f_lo=w.f_lo, df=w.df, n_bins=w.n_bins, n_det=w.n_det,
            data_re=_d(self.dre), data_im=_d(self.dim), psd=_d(self.psd), det_geom=_d(self.geom),
            gmst=w.gmst, fixed_dist_mpc=w.fixed_dist_mpc, rb_n_bins=w.rb_n_bins, rb_fiducial=_d(self.fid),
            gauss_mu=_d(self.mu), gauss_sigma=w.gauss_sigma,
            periodic=_i(self.per) if self.per is not None else None,
        )

    @property
    def ref(self):
        return C.byref(self.s)


def opts_for(w: synth.Workload, seed=None, run_id: int = 0, max_iter: int = 1000, term_frac=None, n_live=None,
             n_delete=None, n_steps=None, precision=None, kernel=None, walk_accept=None, walk_max=None,
             count_moves: bool = False) -> Opts:
    return Opts(
        n_live=w.n_live if n_live is None else n_live, n_delete=w.n_delete if n_delete is None else n_delete,
        n_steps=w.n_steps if n_steps is None else n_steps, slice_width=w.slice_width,
        max_stepout=w.max_stepout, max_shrink=w.max_shrink,
        term_frac=w.term_frac if term_frac is None else term_frac,
        seed=w.sampler_seed if seed is None else seed, run_id=run_id, max_iter=max_iter,
        precision=w.precision if precision is None else precision,
        kernel=w.kernel if kernel is None else kernel,
        walk_accept=w.walk_accept if walk_accept is None else walk_accept,
        walk_max=w.walk_max if walk_max is None else walk_max,
        count_moves=1 if count_moves else 0,
    )


def waveform(spec: ProblemSpec, theta, det: int, cut: bool = True, stream=None):
    """ns_waveform: detector strain on the grid (host arrays)."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    hr = np.zeros(spec.w.n_bins)
    hi = np.zeros(spec.w.n_bins)
    _check(lib().ns_waveform(spec.ref, _d(th), det, 1 if cut else 0, _d(hr), _d(hi), _stream(stream)))
    return hr, hi


def make_data(w: synth.Workload, stream=None):
    """Seeded noise plus the library's own injected waveform (ISCO-cut)."""
    re, im = w.noise()
    spec = ProblemSpec(w)
    for det in range(w.n_det):
        hr, hi = waveform(spec, w.theta_inj, det, cut=True, stream=stream)
        re[det] += hr
        im[det] += hi
    return re, im


def select(logl, k: int, stream=None):
    """ns_select on a CUDA float64 tensor: (dead indices int32 tensor, L*)."""
    import torch
    assert logl.is_cuda and logl.dtype == torch.float64 and logl.is_contiguous()
    n = logl.numel()
    dead = torch.empty(k, dtype=torch.int32, device=logl.device)
    ls = torch.empty(1, dtype=torch.float64, device=logl.device)
    _check(lib().ns_select(C.c_void_p(logl.data_ptr()), n, k, C.c_void_p(dead.data_ptr()),
                           C.c_void_p(ls.data_ptr()), _stream(stream)))
    return dead, ls


class Run:
    """An ns_run: nested slice sampling state resident on the GPU."""

    def __init__(self, spec: ProblemSpec, opts: Opts, stream=None):
        self.spec = spec
        self.opts = opts
        h = C.c_void_p()
        _check(lib().ns_init(C.byref(h), spec.ref, C.byref(opts), _stream(stream)))
        self.h = h

    @classmethod
    def adopt(cls, h: C.c_void_p, spec: ProblemSpec, opts: Opts) -> "Run":
        """Wrap a run handed over by a server (ns_server_take)."""
        r = cls.__new__(cls)
        r.spec, r.opts, r.h = spec, opts, h
        return r

    def step(self, max_iters: int = 1) -> bool:
        done = C.c_int()
        _check(lib().ns_step(self.h, max_iters, C.byref(done)))
        return bool(done.value)

    def step_async(self, n_iters: int):
        _check(lib().ns_step_async(self.h, n_iters))

    def run(self, max_iters: int = 100000) -> bool:
        return self.step(max_iters)

    def state(self):
        lx, lz, H = C.c_double(), C.c_double(), C.c_double()
        it, done = C.c_int(), C.c_int()
        nd, ne = C.c_long(), C.c_long()
        _check(lib().ns_state(self.h, C.byref(lx), C.byref(lz), C.byref(H), C.byref(it), C.byref(nd), C.byref(ne),
                              C.byref(done)))
        return dict(logX=lx.value, logZ=lz.value, H=H.value, iter=it.value, n_dead=nd.value, n_evals=ne.value,
                    done=done.value)

    def live(self):
        n, d = self.opts.n_live, self.spec.w.n_dim
        u = np.zeros((n, d))
        l = np.zeros(n)
        _check(lib().ns_live(self.h, _d(u), _d(l)))
        return u, l

    def dead(self):
        nd = self.state()["n_dead"]
        d = self.spec.w.n_dim
        m = max(nd, 1)
        u = np.zeros((m, d))
        l, lx, lw = (np.zeros(m) for _ in range(3))
        it = np.zeros(m, dtype=np.int32)
        sl = np.zeros(m, dtype=np.int32)
        n_out = C.c_long()
        _check(lib().ns_dead(self.h, m, _d(u), _d(l), _d(lx), _d(lw), _i(it), _i(sl), C.byref(n_out)))
        return dict(u=u[:nd], logl=l[:nd], logx=lx[:nd], logw=lw[:nd], iter=it[:nd], slot=sl[:nd])

    def logZ(self, n_sim: int = 200):
        z, ss, sh, ess = C.c_double(), C.c_double(), C.c_double(), C.c_double()
        _check(lib().ns_logZ(self.h, n_sim, C.byref(z), C.byref(ss), C.byref(sh), C.byref(ess)))
        return dict(logZ=z.value, sigma=ss.value, sigma_h=sh.value, ess=ess.value)

    def samples(self):
        st = self.state()
        tot = st["n_dead"] + self.opts.n_live
        d = self.spec.w.n_dim
        th = np.zeros((tot, d))
        l = np.zeros(tot)
        lw = np.zeros(tot)
        n_out = C.c_long()
        _check(lib().ns_samples(self.h, tot, _d(th), _d(l), _d(lw), C.byref(n_out)))
        return th, l, lw

    def resample(self, n_out: int):
        """ns_resample: (indices into ns_samples' order [n_out], physical
        parameters [n_out, n_dim])."""
        idx = np.zeros(n_out, dtype=np.int32)
        th = np.zeros((n_out, self.spec.w.n_dim))
        _check(lib().ns_resample(self.h, n_out, _i(idx), _d(th)))
        return idx, th

    def loglike(self, u, out=None, terms=None, noalloc: bool = False):
        """ns_loglike on a CUDA float64 tensor [n, n_dim]; returns the tensor
        [n] of log-likelihoods (written into ``out`` when given).  ``terms``:
        an optional CUDA int32 tensor [n] that receives each probe's terms.
        ``noalloc`` calls ns_loglike_noalloc (the library's fixed per-device
        scratch, at most NS_LOGLIKE_NOALLOC_MAX probes) instead."""
        import torch
        assert u.is_cuda and u.dtype == torch.float64 and u.is_contiguous()
        n = u.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=u.device)
        assert out.is_cuda and out.dtype == torch.float64 and out.numel() >= n
        tp = None
        if terms is not None:
            assert terms.is_cuda and terms.dtype == torch.int32 and terms.numel() >= n
            tp = C.c_void_p(terms.data_ptr())
        fn = lib().ns_loglike_noalloc if noalloc else lib().ns_loglike
        _check(fn(self.h, C.c_void_p(u.data_ptr()), n, C.c_void_p(out.data_ptr()), tp))
        return out

    def noise_loglike(self) -> float:
        v = C.c_double()
        _check(lib().ns_noise_loglike(self.h, C.byref(v)))
        return v.value

    def save(self) -> bytes:
        """ns_save into a bytes object."""
        n = C.c_size_t()
        rc = lib().ns_save(self.h, None, 0, C.byref(n))
        if rc != NS_E_CAPACITY:
            _check(rc)
        buf = C.create_string_buffer(n.value)
        _check(lib().ns_save(self.h, buf, n.value, C.byref(n)))
        return buf.raw[:n.value]

    @classmethod
    def load(cls, blob: bytes, spec: ProblemSpec, opts: Opts, stream=None) -> "Run":
        """ns_load of a checkpoint (spec and opts describe the same run)."""
        h = C.c_void_p()
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().ns_load(C.byref(h), buf, len(blob), _stream(stream)))
        return cls.adopt(h, spec, opts)

    def profile(self, enable: bool = True):
        _check(lib().ns_profile(self.h, 1 if enable else 0))

    def trace(self) -> dict:
        """Per-iteration metrics of the iterations so far: a dict of arrays
        with one entry per iteration (hist: one row per iteration)."""
        n_out = C.c_long()
        _check(lib().ns_trace(self.h, 0, None, C.byref(n_out)))
        recs = (IterRec * max(n_out.value, 1))()
        _check(lib().ns_trace(self.h, max(n_out.value, 1), recs, C.byref(n_out)))
        recs = recs[: n_out.value]
        out = {name: np.array([getattr(r, name) for r in recs])
               for name, _ in IterRec._fields_ if name not in ("pad", "hist")}
        out["hist"] = np.array([list(r.hist) for r in recs], dtype=np.int64).reshape(len(recs), PROBE_HIST)
        return out

    def stats(self) -> dict:
        st = Stats()
        _check(lib().ns_stats(self.h, C.byref(st)))
        return {name: getattr(st, name) for name, _ in Stats._fields_}

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ns_free(self.h)
        self.h = None

    def __del__(self):
        self.close()


class Server:
    """An ns_server: queued requests, memory-based admission, packed ticks."""

    def __init__(self, hbm_budget: int = 0, max_runs: int = 8, graph: bool = False, stream=None):
        h = C.c_void_p()
        _check(lib().ns_server_create(C.byref(h), hbm_budget, max_runs, NS_SERVER_GRAPH if graph else 0,
                                      _stream(stream)))
        self.h = h
        self.requests = {}

    def submit(self, spec: ProblemSpec, opts: Opts) -> int:
        t = C.c_longlong()
        _check(lib().ns_server_submit(self.h, spec.ref, C.byref(opts), C.byref(t)))
        self.requests[t.value] = (spec, opts)
        return t.value

    def tick(self, n_iters: int = 1):
        """(resident, queued, finished-not-yet-polled) after the tick."""
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        _check(lib().ns_server_tick(self.h, n_iters, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def poll(self, cap: int = 256):
        buf = (TicketInfo * cap)()
        n = C.c_int()
        _check(lib().ns_server_poll(self.h, buf, cap, C.byref(n)))
        return [{name: getattr(buf[i], name) for name, _ in TicketInfo._fields_} for i in range(n.value)]

    def take(self, ticket: int) -> Run:
        h = C.c_void_p()
        _check(lib().ns_server_take(self.h, ticket, C.byref(h)))
        spec, opts = self.requests.pop(ticket)
        return Run.adopt(h, spec, opts)

    def info(self) -> dict:
        b, u = C.c_size_t(), C.c_size_t()
        r, q = C.c_int(), C.c_int()
        _check(lib().ns_server_info(self.h, C.byref(b), C.byref(u), C.byref(r), C.byref(q)))
        return dict(budget=b.value, used=u.value, running=r.value, queued=q.value)

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ns_server_free(self.h)
        self.h = None

    def __del__(self):
        self.close()
