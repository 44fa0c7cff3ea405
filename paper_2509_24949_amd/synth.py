"""Seeded synthetic inputs shared by the HIP path, the tests and the benchmark.

This module holds no arithmetic of the sampling method: it makes frequency
grids, the analytic noise power spectral density, seeded Gaussian noise,
approximate detector geometry, prior boxes and injection parameters.  The
injected signal itself is never computed here: the product path adds the
waveform its own library returns (``ns_waveform``), the oracle adds its own.

The workloads stand in for the paper's single real-data analysis (the
GW150914 H1/L1 strain of its Section 3), which is not reproduced here.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

import numpy as np

# Prior kinds (unit-cube transforms): uniform in the parameter, uniform in its
# cosine, uniform in its sine, uniform in volume (density proportional to x^2).
PRIOR_UNIFORM, PRIOR_COS, PRIOR_SIN, PRIOR_VOLUME = 0, 1, 2, 3

# Waveform models.  MODEL_TF2_4P: (Mc, eta, t_c, phi_c), one optimally oriented
# detector at a fixed distance.  MODEL_TF2_11P: aligned-spin network model with
# (Mc, q, chi1, chi2, d_L, theta_jn, psi, RA, Dec, t_c, phi_c); MODEL_TF2_11P_SO: the
# same with the spin-orbit phase terms through 3.5PN.
MODEL_TF2_4P, MODEL_TF2_11P, MODEL_TF2_11P_SO = 1, 2, 3

# Likelihood forms.
LIKE_FULL, LIKE_RB, LIKE_GAUSS = 0, 1, 2

PARAMS_4P = ("Mc", "eta", "t_c", "phi_c")
PARAMS_11P = ("Mc", "q", "chi1", "chi2", "d_L", "theta_jn", "psi", "ra", "dec", "t_c", "phi_c")

_HERE = os.path.dirname(os.path.abspath(__file__))
INJECTIONS_JSON = os.path.join(_HERE, "injections.json")


def psd_fit(f):
    """Analytic one-sided noise PSD of the workloads, in 1/Hz.

    S(f) = 1e-46 [x^-4.14 - 5 x^-2 + 111 (1 - x^2 + x^4/2) / (1 + x^2/2)],
    x = f / 215 Hz.
    """
    x = np.asarray(f, dtype=np.float64) / 215.0
    return 1e-46 * (x ** -4.14 - 5.0 * x ** -2 + 111.0 * (1.0 - x ** 2 + 0.5 * x ** 4) / (1.0 + 0.5 * x ** 2))


def grid(f_lo: float, df: float, n_bins: int) -> np.ndarray:
    """Inclusive frequency grid f_k = f_lo + k df, k < n_bins."""
    return f_lo + df * np.arange(n_bins, dtype=np.float64)


def noise(seed: int, psd: np.ndarray, df: float):
    """Seeded complex Gaussian noise: Re, Im ~ N(0, S_k / (4 df)) per bin.

    ``psd`` has shape [n_det, n_bins]; returns (re, im) of the same shape.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    sd = np.sqrt(psd / (4.0 * df))
    re = rng.standard_normal(psd.shape) * sd
    im = rng.standard_normal(psd.shape) * sd
    return re, im


# Approximate detector sites on a spherical Earth (radius 6371 km): geodetic
# latitude and longitude in degrees and the bearings (clockwise from local
# North) of the x and y arms.  Only the structure of a three-detector network
# matters to the workloads; the positions are not survey-grade.
_SITES = {
    "H1": (46.455, -119.408, 324.0, 234.0),
    "L1": (30.563, -90.774, 252.3, 162.3),
    "V1": (43.631, 10.504, 70.6, 340.6),
}
EARTH_RADIUS_M = 6.371e6


def detector_geometry(names) -> np.ndarray:
    """[n_det, 9] array: vertex (m, Earth-fixed), x-arm unit vector, y-arm unit vector."""
    out = np.zeros((len(names), 9))
    for i, nm in enumerate(names):
        lat, lon, bx, by = _SITES[nm]
        la, lo = math.radians(lat), math.radians(lon)
        up = np.array([math.cos(la) * math.cos(lo), math.cos(la) * math.sin(lo), math.sin(la)])
        east = np.array([-math.sin(lo), math.cos(lo), 0.0])
        north = np.array([-math.sin(la) * math.cos(lo), -math.sin(la) * math.sin(lo), math.cos(la)])
        ax = math.cos(math.radians(bx)) * north + math.sin(math.radians(bx)) * east
        ay = math.cos(math.radians(by)) * north + math.sin(math.radians(by)) * east
        out[i, 0:3] = EARTH_RADIUS_M * up
        out[i, 3:6] = ax
        out[i, 6:9] = ay
    return out


@dataclass
class Workload:
    """One synthetic analysis: grid, noise, detectors, prior box, injection, sampler settings."""

    name: str
    model: int
    likelihood: int
    f_lo: float
    df: float
    n_bins: int
    detectors: tuple
    prior_kind: np.ndarray
    prior_lo: np.ndarray
    prior_hi: np.ndarray
    theta_inj: np.ndarray
    noise_seed: int
    gmst: float = 0.0
    fixed_dist_mpc: float = 0.0
    snr_target: float = 0.0
    n_live: int = 500
    n_delete: int = 250
    n_steps: int = 20
    slice_width: float = 1.0
    max_stepout: int = 100
    max_shrink: int = 100
    term_frac: float = 1e-3
    precision: int = 0  # 0 = FP64, 1 = mixed (FP32 bulk, FP64 phase and evidence)
    rb_n_bins: int = 128
    sampler_seed: int = 1001
    gauss_mu: np.ndarray = field(default_factory=lambda: np.zeros(0))
    gauss_sigma: float = 0.0
    # per coordinate: 1 = the unit-cube coordinate wraps around (its prior is
    # uniform over one full period); empty = none
    periodic: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int32))
    # chain kernel: 0 slice sampling (the paper's), 1 random walk with
    # differential-evolution proposals (walk_accept accepted proposals per
    # chain, at most walk_max proposals)
    kernel: int = 0
    walk_accept: int = 60
    walk_max: int = 2000

    @property
    def n_dim(self) -> int:
        return len(self.prior_kind)

    @property
    def n_det(self) -> int:
        return len(self.detectors)

    def freqs(self) -> np.ndarray:
        return grid(self.f_lo, self.df, self.n_bins)

    def psd(self) -> np.ndarray:
        return np.tile(psd_fit(self.freqs()), (self.n_det, 1))

    def det_geom(self) -> np.ndarray:
        return detector_geometry(self.detectors)

    def noise(self):
        return noise(self.noise_seed, self.psd(), self.df)


def _load_injections():
    if not os.path.exists(INJECTIONS_JSON):
        return {}
    with open(INJECTIONS_JSON) as fh:
        return json.load(fh)


def _kinds(*k):
    return np.array(k, dtype=np.int32)


def workload(name: str, distance: float | None = None) -> Workload:
    """The named workload.

    ``tf2_1det``  one detector, 473 bins (20-256 Hz, df 0.5), 4 parameters, FP64, n 500 / k 250.
    ``tf2_3det``  H1/L1/V1, 4017 bins (20-1024 Hz, df 0.25), 11 parameters, FP64, n 1000 / k 500.
    ``tf2_3det_rb``  tf2_3det with the relative-binning likelihood (128 geometric bins).
    ``tf2_3det_mixed``  tf2_3det in the mixed-precision form with n 2000 / k 1000.
    ``tf2_3det_rb_mixed`` tf2_3det_rb in the mixed-precision form with n 2000 / k 1000.
    ``tf2_3det_n2000``, ``tf2_3det_rb_n2000``  the same two at n 2000 / k 1000 in
        double precision (same seeds as the mixed forms).
    ``tf2_3det_so`` tf2_3det with the spin-orbit phase terms through 3.5PN
        (waveform model 3).
    ``tf2_3det_rb_walk`` tf2_3det_rb with the random-walk chain kernel (60
        accepted proposals per chain, at most 2000 proposals).
    ``tf2_3det_rb_paper`` tf2_3det_rb at the paper's own settings (Section 2):
        n 3000 / k 1500, chains of 10 d = 110 steps, the coalescence phase,
        the polarisation angle and the right ascension wrapped in the unit cube.

    ``distance`` overrides the stored SNR-scaled injection distance (used only
    by the script that derives those distances).
    """
    inj = _load_injections()
    two_pi = 2.0 * math.pi
    if name == "tf2_1det":
        d_eff = distance if distance is not None else inj.get("tf2_1det", {}).get("distance_mpc", 0.0)
        return Workload(
            name=name, model=MODEL_TF2_4P, likelihood=LIKE_FULL, f_lo=20.0, df=0.5, n_bins=473,
            detectors=("H1",),
            prior_kind=_kinds(0, 0, 0, 0),
            prior_lo=np.array([20.0, 0.1, -0.1, 0.0]),
            prior_hi=np.array([40.0, 0.25, 0.1, two_pi]),
            theta_inj=np.array([24.0, 0.20, 0.0, 1.0]),
            noise_seed=101, fixed_dist_mpc=d_eff, snr_target=15.0,
            n_live=500, n_delete=250, n_steps=20, sampler_seed=1001,
        )
    if name in ("tf2_3det", "tf2_3det_rb", "tf2_3det_mixed", "tf2_3det_rb_mixed", "tf2_3det_rb_paper",
                "tf2_3det_rb_walk", "tf2_3det_so", "tf2_3det_n2000", "tf2_3det_rb_n2000"):
        d_inj = distance if distance is not None else inj.get("tf2_3det", {}).get("distance_mpc", 0.0)
        w = Workload(
            name=name, model=MODEL_TF2_11P, likelihood=LIKE_FULL, f_lo=20.0, df=0.25, n_bins=4017,
            detectors=("H1", "L1", "V1"),
            prior_kind=_kinds(0, 0, 0, 0, 3, 1, 0, 0, 2, 0, 0),
            prior_lo=np.array([20.0, 0.125, -0.8, -0.8, 0.25 * d_inj, 0.0, 0.0, 0.0, -0.5 * math.pi, -0.1, 0.0]),
            prior_hi=np.array([40.0, 1.0, 0.8, 0.8, 3.0 * d_inj, math.pi, math.pi, two_pi, 0.5 * math.pi, 0.1, two_pi]),
            theta_inj=np.array([25.0, 0.8, 0.3, -0.1, d_inj, 0.4, 0.6, 1.2, -0.3, 0.0, 2.0]),
            noise_seed=102, snr_target=20.0,
            n_live=1000, n_delete=500, n_steps=55, sampler_seed=2001,
        )
        if name == "tf2_3det_rb":
            w.likelihood = LIKE_RB
            w.sampler_seed = 3001
        if name in ("tf2_3det_mixed", "tf2_3det_rb_mixed", "tf2_3det_n2000", "tf2_3det_rb_n2000"):
            w.n_live, w.n_delete = 2000, 1000
            w.precision = 1 if name.endswith("mixed") else 0
            w.sampler_seed = 4001
            if name in ("tf2_3det_rb_mixed", "tf2_3det_rb_n2000"):
                w.likelihood = LIKE_RB
        if name == "tf2_3det_so":
            w.model = MODEL_TF2_11P_SO
            w.sampler_seed = 9501
        if name == "tf2_3det_rb_walk":
            w.likelihood = LIKE_RB
            w.kernel = 1
            w.sampler_seed = 9001
        if name == "tf2_3det_rb_paper":
            w.likelihood = LIKE_RB
            w.n_live, w.n_delete, w.n_steps = 3000, 1500, 10 * 11
            w.periodic = np.array([0, 0, 0, 0, 0, 0, 1, 1, 0, 0, 1], dtype=np.int32)
            w.sampler_seed = 8001
        return w
    raise KeyError(name)


# Serving workload: events of uneven duration, network and size.
SERVING_EVENTS = 64
SERVING_DURATIONS = (4, 8, 16, 32)            # seconds of data: 4017 ... 32129 bins per detector
SERVING_NETWORKS = (("H1",), ("H1", "L1"), ("H1", "L1", "V1"))
SERVING_N_LIVE = (500, 1000, 2000)
# total mass (solar masses) whose innermost-stable-orbit frequency is 30 Hz;
# heavier draws are rejected because they leave almost no signal in band
SERVING_MAX_TOTAL_MASS = 146.6


def serving_event(i: int, distance: float | None = None) -> Workload:
    """Event ``i`` of the serving workload (parameters seeded by 5000+i,
    noise by 6000+i, sampler by 7000+i).  Duration T in {4, 8, 16, 32} s
    (grid 20-1024 Hz with df = 1/T), 1-3 detectors, network SNR U[8, 40],
    Mc U[5, 60], q U[0.125, 1], n_live in {500, 1000, 2000} with
    n_delete = n_live / 2; chirp-mass prior [0.7, 1.3] Mc clipped to
    [5, 60], the other priors as the 3-detector workload.  ``distance``
    overrides the stored SNR-scaled injection distance."""
    rng = np.random.Generator(np.random.PCG64(5000 + i))
    T = int(rng.choice(SERVING_DURATIONS))
    dets = SERVING_NETWORKS[int(rng.integers(0, 3))]
    snr = float(rng.uniform(8.0, 40.0))
    while True:
        mc = float(rng.uniform(5.0, 60.0))
        q = float(rng.uniform(0.125, 1.0))
        eta = q / (1.0 + q) ** 2
        if mc * eta ** -0.6 <= SERVING_MAX_TOTAL_MASS:
            break
    n_live = int(rng.choice(SERVING_N_LIVE))
    chi1, chi2 = (float(x) for x in rng.uniform(-0.5, 0.5, size=2))
    theta_jn = math.acos(float(rng.uniform(-1.0, 1.0)))
    psi = float(rng.uniform(0.0, math.pi))
    ra = float(rng.uniform(0.0, 2.0 * math.pi))
    dec = math.asin(float(rng.uniform(-1.0, 1.0)))
    phi_c = float(rng.uniform(0.0, 2.0 * math.pi))
    if distance is None:
        stored = _load_injections().get("serving", {}).get("distance_mpc", [])
        distance = stored[i] if i < len(stored) else 0.0
    d = float(distance)
    two_pi = 2.0 * math.pi
    return Workload(
        name=f"event/{i}", model=MODEL_TF2_11P, likelihood=LIKE_FULL, f_lo=20.0, df=1.0 / T,
        n_bins=1004 * T + 1, detectors=dets,
        prior_kind=_kinds(0, 0, 0, 0, 3, 1, 0, 0, 2, 0, 0),
        prior_lo=np.array([max(5.0, 0.7 * mc), 0.125, -0.8, -0.8, 0.25 * d, 0.0, 0.0, 0.0, -0.5 * math.pi, -0.1, 0.0]),
        prior_hi=np.array([min(60.0, 1.3 * mc), 1.0, 0.8, 0.8, 3.0 * d, math.pi, math.pi, two_pi, 0.5 * math.pi, 0.1,
                           two_pi]),
        theta_inj=np.array([mc, q, chi1, chi2, d, theta_jn, psi, ra, dec, 0.0, phi_c]),
        noise_seed=6000 + i, snr_target=snr,
        n_live=n_live, n_delete=n_live // 2, n_steps=55, sampler_seed=7000 + i,
    )


def serving_arrivals(n: int = SERVING_EVENTS, seed: int = 5999) -> np.ndarray:
    """Arrival times of a unit-rate Poisson process (first arrival at 0);
    scale by 1/rate for a given arrival rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0, size=n)
    gaps[0] = 0.0
    return np.cumsum(gaps)


def gauss_workload(d: int, sigma: float, mu=None, n_live: int = 500, n_delete: int = 250,
                   n_steps: int | None = None, seed: int = 11) -> Workload:
    """Gaussian likelihood N(u; mu, sigma^2 I) inside the unit cube (an evidence test problem)."""
    mu = np.full(d, 0.5) if mu is None else np.asarray(mu, dtype=np.float64)
    return Workload(
        name=f"gauss{d}", model=0, likelihood=LIKE_GAUSS, f_lo=0.0, df=1.0, n_bins=0, detectors=(),
        prior_kind=np.zeros(d, dtype=np.int32), prior_lo=np.zeros(d), prior_hi=np.ones(d),
        theta_inj=mu.copy(), noise_seed=0, n_live=n_live, n_delete=n_delete,
        n_steps=(5 * d if n_steps is None else n_steps), sampler_seed=seed,
        gauss_mu=mu, gauss_sigma=sigma,
    )


def proposal_batch(w: Workload, n: int, seed: int, frac_local: float = 0.5, scale: float = 0.02) -> np.ndarray:
    """[n, n_dim] unit-cube points: a fraction drawn from the prior, the rest
    clustered around the injection (posterior-region probes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random((n, w.n_dim))
    n_loc = int(round(frac_local * n))
    if n_loc:
        c = theta_to_cube_box(w, w.theta_inj)
        loc = c[None, :] + scale * rng.standard_normal((n_loc, w.n_dim))
        u[:n_loc] = np.clip(loc, 0.0, 1.0)
    return u


def theta_to_cube_box(w: Workload, theta) -> np.ndarray:
    """Place physical parameters into the unit cube of the prior box (inverse of
    the prior transforms; used only to aim synthetic probe batches)."""
    th = np.asarray(theta, dtype=np.float64)
    u = np.empty(w.n_dim)
    for i, (k, a, b) in enumerate(zip(w.prior_kind, w.prior_lo, w.prior_hi)):
        if k == PRIOR_UNIFORM:
            u[i] = (th[i] - a) / (b - a)
        elif k == PRIOR_COS:
            u[i] = (math.cos(a) - math.cos(th[i])) / (math.cos(a) - math.cos(b))
        elif k == PRIOR_SIN:
            u[i] = (math.sin(th[i]) - math.sin(a)) / (math.sin(b) - math.sin(a))
        else:
            u[i] = (th[i] ** 3 - a ** 3) / (b ** 3 - a ** 3)
    return np.clip(u, 0.0, 1.0)
