/*
 * ns.h -- C ABI of libns, nested slice sampling for gravitational-wave
 * parameter estimation on AMD Instinct MI355X (gfx950).
 *
 * The method (paper Section 2): classic nested sampling over a static
 * population of n_live points; each iteration deletes the n_delete
 * lowest-likelihood points, adds their prior-volume shells to the evidence,
 * and refills the deleted slots by running one constrained hit-and-run slice
 * sampling chain per deleted point, started from a surviving point, with
 * directions tuned by the particle covariance.  Each probe of a chain costs
 * one frequency-domain waveform plus a noise-weighted (Whittle) likelihood,
 * on the full frequency grid or on a coarse heterodyned grid (relative
 * binning; Sections 1 and 3).
 *
 * Conventions shared by every entry point:
 *   - Return value: NS_OK (0) on success, a negative ns_status on failure.
 *     Nothing aborts or throws across the ABI; ns_last_error() returns a
 *     thread-local message describing the most recent failure.  On failure
 *     no state is left half-built (an ns_run is either complete or NULL).
 *   - "host" pointers are ordinary CPU memory owned by the caller and only
 *     read (or written, for outputs) during the call.  "device" pointers are
 *     HIP device allocations owned by the caller.
 *   - Arrays are row-major and contiguous; all floating point is IEEE double
 *     unless stated.
 *   - stream: a hipStream_t passed as void* (NULL = the default stream);
 *     borrowed, never destroyed by the library.  Every kernel of a run is
 *     launched on the run's stream.
 *   - The unit cube: sampling happens in u in [0,1]^n_dim; prior transforms
 *     map u to physical parameters.
 *   - The likelihood is reported as the log-likelihood ratio against the
 *     noise-only model, lambda = sum_det [<d|h> - 1/2 <h|h>], with
 *     <a|b> = 4 df Re sum_k conj(a_k) b_k / S_k over the inclusive grid
 *     f_k = f_lo + k df; the waveform is zero above the innermost-stable-
 *     circular-orbit frequency f_ISCO = 1/(6^(3/2) pi M).  log Z is therefore
 *     the log Bayes factor of signal against noise.
 */
#ifndef NS_H
#define NS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define NS_API __attribute__((visibility("default")))
#else
#define NS_API
#endif

typedef enum {
    NS_OK = 0,
    NS_E_ARG = -1,      /* invalid argument (sizes, ranges, NULL pointers) */
    NS_E_OOM = -2,      /* device or host allocation failed */
    NS_E_HIP = -3,      /* a HIP runtime call failed */
    NS_E_CAPACITY = -4, /* caller buffer too small; the required size is reported */
    NS_E_STATE = -5     /* call not valid in the run's current state */
} ns_status;

/* Prior kinds for one unit-cube coordinate with interval [lo, hi]:
 *   UNIFORM  theta = lo + (hi - lo) u
 *   COS      uniform in cos(theta), 0 <= lo < hi <= pi   (isotropic inclination)
 *   SIN      uniform in sin(theta), -pi/2 <= lo < hi <= pi/2 (isotropic declination)
 *   VOLUME   density proportional to theta^2, 0 <= lo < hi (uniform in volume)
 * The waveform models accept UNIFORM for every coordinate, and in addition
 * VOLUME for d_L, COS for theta_jn and SIN for Dec (TF2_11P); the Gaussian
 * test likelihood ignores the kinds (it works on u directly). */
enum { NS_PRIOR_UNIFORM = 0, NS_PRIOR_COS = 1, NS_PRIOR_SIN = 2, NS_PRIOR_VOLUME = 3 };

/* Waveform models (stationary-phase TaylorF2, 3.5PN phase, Newtonian amplitude):
 *   TF2_4P   parameters (Mc [Msun], eta, t_c [s], phi_c [rad]); one detector,
 *            optimally oriented (antenna factor 1, no delay), at the fixed
 *            distance fixed_dist_mpc.
 *   TF2_11P  parameters (Mc [Msun], q = m2/m1 in (0,1], chi1, chi2 (aligned
 *            spins), d_L [Mpc], theta_jn [rad], psi [rad], RA [rad], Dec [rad],
 *            t_c [s], phi_c [rad]); a detector network.  Spin terms: spin-orbit
 *            at 1.5PN, spin-spin (chi1 chi2) at 2PN.
 *   TF2_11P_SO  TF2_11P with the spin-orbit phase terms above 1.5PN as
 *            well (2.5PN, the 3PN tail term and 3.5PN, linear in the spins),
 *            the richer aligned-spin waveform of paper Sections 2-3's family. */
enum { NS_MODEL_TF2_4P = 1, NS_MODEL_TF2_11P = 2, NS_MODEL_TF2_11P_SO = 3 };

/* Likelihood forms: full grid; relative binning (heterodyned coarse grid,
 * rb_n_bins geometric bins, fiducial waveform at rb_fiducial); and a
 * Gaussian test likelihood N(u; gauss_mu, gauss_sigma^2 I) on the unit cube
 * (for evidence checks against its closed form). */
enum { NS_LIKE_FULL = 0, NS_LIKE_RB = 1, NS_LIKE_GAUSS = 2 };

/* Arithmetic: all double, or the mixed form (float bulk, double phase and evidence). */
enum { NS_FP64 = 0, NS_MIXED = 1 };

/* Chain kernel that refills the deleted points (paper Section 2):
 *   SLICE  constrained hit-and-run slice sampling, n_steps steps per chain,
 *          directions tuned by the particle covariance (the paper's NSS);
 *   WALK   the random-walk alternative of bilby's sampler, read as
 *          differential-evolution moves: each proposal is x + g (u_a - u_b)
 *          for two distinct surviving live points a, b, with g = 1 or
 *          2.38 / sqrt(2 n_dim) with probability 1/2 each, times a factor
 *          uniform on [0.9, 1.1], accepted iff
 *          in the unit cube (periodic coordinates wrap) with lambda > L*
 *          (a pair of survivors at one point is a null move, not evaluated).
 *          Every chain of an iteration makes the same number of proposals,
 *          set for the next iteration to walk_accept / (the iteration's
 *          acceptance rate), rounded up, within [1, walk_max]; the first
 *          iteration makes walk_accept.  Needs n_live - n_delete >= 2.
 *          Not supported by the server. */
enum { NS_KERNEL_SLICE = 0, NS_KERNEL_WALK = 1 };

typedef struct {
    int model;                 /* NS_MODEL_*; ignored for NS_LIKE_GAUSS */
    int likelihood;            /* NS_LIKE_* */
    int n_dim;                 /* 1..12; must match the model (4 or 11) unless GAUSS */
    const int* prior_kind;     /* host [n_dim] */
    const double* prior_lo;    /* host [n_dim] */
    const double* prior_hi;    /* host [n_dim] */
    double f_lo, df;           /* grid f_k = f_lo + k df, Hz; f_lo > 0, df > 0 */
    int n_bins;                /* >= 2 */
    int n_det;                 /* 1..3 (exactly 1 for TF2_4P) */
    const double* data_re;     /* host [n_det][n_bins], strain/Hz */
    const double* data_im;     /* host [n_det][n_bins] */
    const double* psd;         /* host [n_det][n_bins], one-sided, 1/Hz, > 0 */
    const double* det_geom;    /* host [n_det][9]: vertex (m, Earth-fixed), x-arm, y-arm unit vectors */
    double gmst;               /* Greenwich sidereal angle, rad */
    double fixed_dist_mpc;     /* TF2_4P only: distance, Mpc, > 0 */
    int rb_n_bins;             /* NS_LIKE_RB: number of coarse bins (1..min(n_bins-1, 1024)) */
    const double* rb_fiducial; /* NS_LIKE_RB: host [n_dim] physical fiducial parameters */
    const double* gauss_mu;    /* NS_LIKE_GAUSS: host [n_dim] */
    double gauss_sigma;        /* NS_LIKE_GAUSS: > 0 */
    const int* periodic;       /* host [n_dim] or NULL: 1 = the coordinate is an angle whose UNIFORM prior
                                  covers one full period (coalescence phase, polarisation angle, right
                                  ascension); slice moves take it modulo 1 in the unit cube, so the slice
                                  extends across the seam of its interval (paper Section 2 names the
                                  wrapped phase and polarisation as a tuning problem); 0 = bounded */
} ns_problem;

typedef struct {
    int n_live;          /* live population n, 2..16384 */
    int n_delete;        /* deleted per iteration k, 1..n_live-1 (the paper uses n_live/2) */
    int n_steps;         /* slice steps per chain per iteration (a multiple of n_dim) */
    double slice_width;  /* initial bracket width w along the tuned direction (> 0) */
    int max_stepout;     /* step-out budget per step, split between the sides (>= 1) */
    int max_shrink;      /* shrink attempts per step before the state is kept (>= 1) */
    double term_frac;    /* stop when the live evidence fraction falls below it; <= 0 never */
    uint64_t seed;       /* Philox key word 0 */
    uint64_t run_id;     /* Philox key word 1 */
    int max_iter;        /* iteration capacity of the dead-point record (>= 1) */
    int precision;       /* NS_FP64 or NS_MIXED */
    int kernel;          /* NS_KERNEL_SLICE (the paper's), or NS_KERNEL_WALK */
    int walk_accept;     /* NS_KERNEL_WALK: target accepted proposals per chain (>= 1) */
    int walk_max;        /* NS_KERNEL_WALK: cap on proposals per chain (>= 1) */
    int count_moves;     /* NS_KERNEL_SLICE, 0 or 1: the chains count their moves for the
                            per-iteration metrics (ns_trace: bracket expansions, rejected
                            shrink candidates, moved steps, evaluations per step).  The
                            counting chain kernels run 64 threads per chain; without it the
                            other chain kernels carry no counting code and those fields read
                            -1 (the histogram 0).  The counting kernels sum the likelihood in
                            another order, so results agree to rounding (in double precision
                            both follow the sequential walk; in the mixed form a decision at
                            the threshold can differ).  Served runs (ns_server) do not count. */
} ns_opts;

typedef struct ns_run ns_run;

/* Create a run: validate, copy the problem to HBM, build the likelihood
 * tables (and relative-binning summary data), draw n_live prior points and
 * evaluate them.  The run's state then stays resident on the device.
 * out: receives the run (NULL on failure).  Host arrays may be freed on
 * return.  Errors: NS_E_ARG, NS_E_OOM, NS_E_HIP. */
NS_API int ns_init(ns_run** out, const ns_problem* problem, const ns_opts* opts, void* stream);

/* Run up to max_iters "replace the k lowest" iterations (Section 2): select
 * the k lowest (ties to the lower slot, NaN as -inf), update log X, log Z and
 * the information H, tune directions from the covariance of the live points,
 * run the k slice chains, refill the dead slots, test termination.  Once the
 * termination test passes the remaining enqueued iterations do nothing.
 * Synchronises the stream; done (may be NULL) receives 1 when the run has
 * terminated (criterion met or capacity reached). */
NS_API int ns_step(ns_run* run, int max_iters, int* done);

/* Enqueue n_iters iterations on the run's stream without synchronising. */
NS_API int ns_step_async(ns_run* run, int n_iters);

/* Final evidence: dead shells plus the live points, each taking X_end/n.
 * logZ: log Bayes factor; sigma_sim: spread of log Z over n_sim replicas with
 * redrawn prior-volume shrinkages (n_sim >= 2, else 0); sigma_h:
 * sqrt(H / n_live); ess: Kish effective sample size 1/sum p_i^2.  Any output
 * pointer may be NULL.  Synchronises. */
NS_API int ns_logZ(ns_run* run, int n_sim, double* logZ, double* sigma_sim, double* sigma_h, double* ess);

/* Weighted posterior samples: dead points in death order, then the live
 * points in slot order.  theta: host [cap][n_dim] physical parameters
 * (unit-cube coordinates for GAUSS); logl: host [cap]; logw: host [cap],
 * normalised so that sum exp(logw) = 1.  n_out receives the count; returns
 * NS_E_CAPACITY (with n_out set) if cap is too small.  Outputs may be NULL. */
NS_API int ns_samples(ns_run* run, long cap, double* theta, double* logl, double* logw, long* n_out);

/* Equal-weight posterior samples (the equal-weight sample count beside the
 * Kish ESS in the paper's results table, Section 3): systematic resampling of
 * the weighted samples of ns_samples (same order, weights normalised by the
 * final log Z) with one uniform u0 of the run's random stream: output m is the
 * first weighted sample whose running weight sum exceeds (m + u0) / n_out of
 * the total.  idx: host [n_out] receives indices into ns_samples' order;
 * theta: host [n_out][n_dim] physical parameters (unit-cube coordinates for
 * GAUSS); either may be NULL.  1 <= n_out <= 2^30.  Synchronises. */
NS_API int ns_resample(ns_run* run, long n_out, int* idx, double* theta);

/* Scalars of the run (any pointer may be NULL).  n_evals counts likelihood
 * evaluations (probes inside the unit cube, plus the initial population). */
NS_API int ns_state(ns_run* run, double* logX, double* logZ, double* H, int* iter, long* n_dead, long* n_evals,
             int* done);

/* Live population, host [n_live][n_dim] and [n_live] (either may be NULL). */
NS_API int ns_live(ns_run* run, double* u, double* logl);

/* Dead-point record, in death order: unit-cube point, lambda, log X after the
 * death, log w (unnormalised), iteration and slot.  Host arrays of length
 * cap (u: cap*n_dim); any may be NULL.  NS_E_CAPACITY if cap < count. */
NS_API int ns_dead(ns_run* run, long cap, double* u, double* logl, double* logx, double* logw, int* iter, int* slot,
            long* n_out);

/* Batched likelihood with the run's tables: out[i] = lambda(u[i]).
 * u_dev: device [n][n_dim] unit-cube points; out_dev: device [n];
 * terms_dev (may be NULL): device [n] receives the terms each probe costs
 * (full grid: its active bins k with f_k <= f_ISCO; relative binning: the
 * edges its active coarse bins need, one more than those bins, or 0 if none
 * is active; Gaussian: 0).  Launched on the run's stream, asynchronous.
 * This is the fused waveform-plus-likelihood kernel the slice chains call,
 * exposed for direct use. */
NS_API int ns_loglike(ns_run* run, const double* u_dev, long n, double* out_dev, int* terms_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ns_loglike
 * with the same kernels and results, whose probe-record scratch (used by the
 * full-grid form; the relative-binning and Gaussian forms need none) is a
 * fixed array of NS_LOGLIKE_NOALLOC_MAX records per device (about 3.3 MB,
 * held from the first ns_init on that device until the process ends) instead
 * of a buffer the run allocates.  It calls no allocator.  The size limit
 * applies to every likelihood form.  u_dev, out_dev,
 * terms_dev as for ns_loglike; the current device must be the run's.
 * Errors: NS_E_ARG if n > NS_LOGLIKE_NOALLOC_MAX or the arguments are bad,
 * NS_E_HIP.  All calls on one device share the one array: calls that
 * overlap in time on that device (other streams, other threads) race and
 * must be serialised by the caller. */
#define NS_LOGLIKE_NOALLOC_MAX 16384
NS_API int ns_loglike_noalloc(ns_run* run, const double* u_dev, long n, double* out_dev, int* terms_dev);

/* Detector strain h_det(f_k) of the problem's model at physical parameters
 * theta (host [n_dim]) on the problem's grid, computed on the device.
 * apply_cut = 1 zeroes bins above f_ISCO.  h_re, h_im: host [n_bins].
 * Only the model, grid, detector and fixed-distance fields of problem are
 * read.  Synchronises the stream. */
NS_API int ns_waveform(const ns_problem* problem, const double* theta, int det, int apply_cut, double* h_re,
                double* h_im, void* stream);

/* k lowest of n values (Section 2 deletion step) in the sampler's total order:
 * ascending lambda, NaN ordered as -inf, -0 equal to +0, ties to the lower
 * index.  logl_dev: device [n]; dead_dev: device [k] receives the indices in
 * ascending order; lstar_dev: device [1] receives the k-th lowest value.
 * 1 <= k <= n <= 16384.  Asynchronous on stream. */
NS_API int ns_select(const double* logl_dev, int n, int k, int* dead_dev, double* lstar_dev, void* stream);

/* Per-kernel timing of a run's iterations (hipEvents recorded on the run's
 * stream around every kernel of every iteration while enabled).  Enabling
 * clears the accumulated statistics. */
NS_API int ns_profile(ns_run* run, int enable);

typedef struct {
    long iterations;         /* iterations enqueued while profiling */
    double ms_select;        /* summed kernel durations, milliseconds */
    double ms_prep;
    double ms_slice;
    double ms_term;
    long long evals;         /* likelihood evaluations of the whole run so far */
    long long bin_terms;     /* sum over evaluations of the terms ns_loglike reports per probe */
    int slice_threads;       /* threads per chain workgroup */
    int lds_tables;          /* 1 if the likelihood tables are staged in LDS */
} ns_stats_t;

/* Statistics of the profiled iterations (synchronises the stream). */
NS_API int ns_stats(ns_run* run, ns_stats_t* out);

/* Metrics of one "replace the k lowest" iteration (Section 2), written by
 * the device at the end of the iteration.  Counts are those of the
 * sequential slice walk the chains carry out (the batched evaluation of
 * candidates does not change them): a probe outside the unit cube is no
 * evaluation, but its rejection still shrinks the bracket. */
#define NS_PROBE_HIST 32
typedef struct {
    int iter;                /* iteration index, from 0 */
    int probes_min;          /* fewest likelihood evaluations of one chain */
    int probes_max;          /* most evaluations of one chain */
    int pad;
    double lstar;            /* the threshold L*: the k-th lowest lambda of the iteration */
    double logX;             /* log prior volume after the iteration's k deaths */
    double logZ;             /* accumulated log evidence after them */
    double log_remaining;    /* log X + log mean exp(lambda) of the refilled live
                              * points, minus log Z: the log of the evidence still
                              * held by the live points relative to log Z, the
                              * quantity the termination test compares with
                              * ln(term_frac) */
    long long probes;        /* likelihood evaluations of all chains */
    long long steps;         /* slice steps (k * n_steps); random walk: proposals (k * chain length) */
    long long accepted;      /* slice steps that moved the chain (all but those whose
                              * shrink budget ran out); random walk: accepted proposals */
    long long stepouts;      /* slice: bracket expansions by w */
    long long shrinks;       /* slice: rejected shrink candidates */
    int hist[NS_PROBE_HIST]; /* slice: steps by the evaluations they made, hist[p]
                              * for p evaluations, the last bin for
                              * NS_PROBE_HIST - 1 or more; random walk: zeros.
                              * accepted (slice), stepouts, shrinks and hist need
                              * opts.count_moves; without it they read -1 and 0 */
} ns_iter_t;

/* Per-iteration metrics of the iterations run so far, in order, into out[cap]
 * (host).  n_out receives their count (at most opts.max_iter); NS_E_CAPACITY
 * (nothing written) if cap is smaller; out may be NULL to ask for the count.
 * Synchronises the run's stream.  Restored runs (ns_load) carry the records
 * of the iterations before the checkpoint. */
NS_API int ns_trace(ns_run* run, long cap, ns_iter_t* out, long* n_out);

/* Log-likelihood of the data under the noise-only model (Whittle: in every
 * bin the real and imaginary parts are Gaussian with variance S/(4 df)),
 * computed on the device at ns_init.  logZ from ns_logZ plus this value is
 * the absolute log evidence of the signal model.  NS_E_STATE for the
 * Gaussian test likelihood. */
NS_API int ns_noise_loglike(ns_run* run, double* out);

/* Checkpoint: serialise the run (problem, options, live points, evidence
 * state and dead-point record) into buf[cap].  n_out receives the size;
 * NS_E_CAPACITY (nothing written) if cap is too small, so a first call with
 * buf = NULL, cap = 0 asks for the size.  Synchronises the run's stream.
 * Random numbers are counter-based (iteration, chain, step), so a run
 * restored with ns_load continues bit-identically to the uninterrupted one. */
NS_API int ns_save(ns_run* run, void* buf, size_t cap, size_t* n_out);

/* Restore a checkpoint written by ns_save of this library version into a
 * new run on stream (tables are rebuilt from the stored problem).
 * NS_E_ARG if buf[size] is not a well-formed checkpoint. */
NS_API int ns_load(ns_run** out, const void* buf, size_t size, void* stream);

/* Release a run (NULL is allowed). */
NS_API void ns_free(ns_run* run);

/* ---- Serving -------------------------------------------------------------
 * A server keeps many runs resident on one device and advances them
 * together: every tick runs one iteration (Section 2) of each resident run,
 * with one packed launch per kernel over the chains of all resident runs
 * that share a likelihood form and precision.  Requests (one per event) wait
 * in a queue until a run slot and device memory are free; a request that
 * does not fit may be overtaken by later ones that do, at most 16 times.
 * Each run's arithmetic is the same alone and in any mix: its results are
 * bit-identical whatever else is resident (they may differ in the last bits
 * from ns_init's, which picks the chain-workgroup size per problem). */
typedef struct ns_server ns_server;

enum { NS_SERVER_GRAPH = 1 };   /* replay each tick's launches from a captured HIP graph */

typedef struct {
    long long ticket;
    int status;          /* NS_OK, or the error code of the run's construction */
    int done;            /* termination code: 1 criterion met, 2 capacity reached */
    int iterations;
    double t_submit;     /* seconds since the server was created */
    double t_admit;      /* construction started */
    double t_finish;     /* the tick that saw the run terminate returned */
    size_t bytes;        /* device bytes the run holds until it is taken */
} ns_ticket_info;

/* Create a server.  hbm_budget: device bytes the resident runs may hold
 * (0: 90% of the free memory now); max_runs: resident-run slots, 1..4096;
 * flags: 0 or NS_SERVER_GRAPH (needs a stream other than the null stream).
 * Resident runs are sorted into three lanes by the cost of one probe
 * (detectors times the most bins a probe can have active: below 1024, below
 * 4096, above), each advanced on a stream of its own; runs are built on a
 * further stream (all four created by the server at the default priority).
 * A run taken from the server is handed over on stream, which the caller
 * keeps alive while it uses such runs.  Errors: NS_E_ARG, NS_E_OOM, NS_E_HIP. */
NS_API int ns_server_create(ns_server** out, size_t hbm_budget, int max_runs, int flags, void* stream);

/* Queue a request.  problem and opts are validated now and copied (the
 * caller may free its arrays on return); likelihood must be NS_LIKE_FULL or
 * NS_LIKE_RB.  ticket receives the request's handle.  NS_E_OOM if the run
 * alone would exceed the budget. */
NS_API int ns_server_submit(ns_server* server, const ns_problem* problem, const ns_opts* opts, long long* ticket);

/* Admit what fits, start n_iters (1..1000) iterations of every resident run
 * on each lane without a tick in flight, wait until some lane's tick has
 * finished and retire its runs that terminated, admit again and start the
 * idle lanes' next ticks.  A lane's tick covers the runs resident when it
 * started; runs admitted meanwhile join its next one.  Outputs (may be
 * NULL): resident, queued, and finished-but-not-yet-polled counts. */
NS_API int ns_server_tick(ns_server* server, int n_iters, int* n_running, int* n_queued, int* n_finished);

/* Report finished requests not reported before, up to cap, in the order
 * they finished; n_out receives the count. */
NS_API int ns_server_poll(ns_server* server, ns_ticket_info* out, int cap, int* n_out);

/* Hand a finished run to the caller, who then owns it (ns_logZ, ns_samples,
 * ns_dead, ..., ns_free) and whose bytes leave the server's budget.
 * NS_E_STATE while the ticket is queued or running, or if its construction
 * failed (the ticket is then forgotten). */
NS_API int ns_server_take(ns_server* server, long long ticket, ns_run** out);

/* Budget, bytes held, resident and queued counts (any pointer may be NULL). */
NS_API int ns_server_info(ns_server* server, size_t* budget, size_t* used, int* n_running, int* n_queued);

/* Release the server with every run it still holds (NULL is allowed). */
NS_API void ns_server_free(ns_server* server);

/* Message for the calling thread's most recent failure ("" if none). */
NS_API const char* ns_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
