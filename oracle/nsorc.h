/*
 * Reference oracle for nested slice sampling on a gravitational-wave
 * frequency-domain likelihood.  TEST INFRASTRUCTURE ONLY: a plain, slow,
 * double-precision CPU implementation used to check the HIP library.  Only
 * the tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header or table with the HIP library.
 *
 * Every function computes its result by the plain definition (direct sums
 * over frequency bins, a full sort for the selection, sequential evidence
 * updates).  No blocking, fusion or prefix tables.
 */
#ifndef NSORC_H
#define NSORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_PRIOR_UNIFORM = 0, ORC_PRIOR_COS = 1, ORC_PRIOR_SIN = 2, ORC_PRIOR_VOLUME = 3 };
enum { ORC_MODEL_TF2_4P = 1, ORC_MODEL_TF2_11P = 2, ORC_MODEL_TF2_11P_SO = 3 };
enum { ORC_LIKE_FULL = 0, ORC_LIKE_RB = 1, ORC_LIKE_GAUSS = 2 };

typedef struct {
    int model, likelihood, n_dim;
    const int* prior_kind;      /* [n_dim] */
    const double* prior_lo;     /* [n_dim] */
    const double* prior_hi;     /* [n_dim] */
    double f_lo, df;
    int n_bins, n_det;
    const double* data_re;      /* [n_det * n_bins] strain / Hz */
    const double* data_im;
    const double* psd;          /* [n_det * n_bins] one-sided, 1/Hz */
    const double* det_geom;     /* [n_det * 9]: vertex (m), x arm, y arm */
    double gmst;                /* rad */
    double fixed_dist_mpc;      /* 4-parameter model only */
    int rb_n_bins;
    const double* rb_fiducial;  /* [n_dim] physical parameters */
    const double* gauss_mu;     /* [n_dim] */
    double gauss_sigma;
    const int* periodic;        /* [n_dim] or NULL: 1 = the unit-cube coordinate wraps around */
} orc_problem;

enum { ORC_KERNEL_SLICE = 0, ORC_KERNEL_WALK = 1 };

typedef struct {
    int n_live, n_delete, n_steps;
    double slice_width;
    int max_stepout, max_shrink;
    double term_frac;
    uint64_t seed, run_id;
    int max_iter;
    int n_threads;
    int kernel;                 /* ORC_KERNEL_SLICE, or ORC_KERNEL_WALK (random-walk chains) */
    int walk_accept, walk_max;  /* walk: target accepted proposals per chain, chain-length cap */
} orc_opts;

typedef struct orc_run orc_run;

/* Philox4x64-10 block for one counter and key. */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Unit cube -> physical parameters. */
void orc_prior_transform(const orc_problem* p, const double* u, double* theta);

/* Antenna pattern and geocentre-to-detector delay for one detector. */
void orc_antenna(const double* geom9, double ra, double dec, double psi, double gmst,
                 double* fplus, double* fcross, double* dt);

/* Detector strain h_det(f_k) on the grid for physical parameters theta.
 * apply_cut = 1 zeroes bins above f_ISCO. */
int orc_waveform(const orc_problem* p, const double* theta, int det, int apply_cut,
                 double* h_re, double* h_im);

/* TaylorF2 phase Psi(f) (radians) for the given masses/spins (test helper). */
double orc_tf2_phase(double f, double mc_msun, double eta, double beta, double sigma,
                     double tc, double phic);
/* The same with the higher-order spin-orbit terms: gamma5 (2.5PN), so6
 * (3PN) and so7 (3.5PN) (test helper). */
double orc_tf2_phase_so(double f, double mc_msun, double eta, double beta, double sigma, double gamma5,
                        double so6, double so7, double tc, double phic);

/* Symmetric mass ratio and the leading-order aligned-spin phase terms
 * (spin-orbit beta, spin-spin sigma) of a parameter point (test helper). */
int orc_pn_params(const orc_problem* p, const double* theta, double* eta, double* beta, double* sigma);
/* The higher-order spin-orbit phase terms (zero unless ORC_MODEL_TF2_11P_SO). */
int orc_pn_params_so(const orc_problem* p, const double* theta, double* gamma5, double* so6, double* so7);

/* Noise-weighted inner product 4 df Re sum conj(a) b / S over one detector. */
double orc_inner(const orc_problem* p, int det, const double* a_re, const double* a_im,
                 const double* b_re, const double* b_im);

/* Log-likelihood of the data under the noise-only model: every bin of every
 * detector holds a complex Gaussian whose real and imaginary parts each have
 * variance S_k / (4 df).  Adding it to the log Bayes factor gives the
 * absolute log evidence of the signal model. */
double orc_noise_loglike(const orc_problem* p);

/* Log-likelihood ratio lambda(theta) = sum_det <d|h> - 1/2 <h|h>, full grid. */
double orc_loglike_full(const orc_problem* p, const double* theta);

/* Relative binning: build summary data at the fiducial, then evaluate. */
typedef struct orc_rb orc_rb;
orc_rb* orc_rb_build(const orc_problem* p);
void orc_rb_free(orc_rb* rb);
int orc_rb_edges(const orc_rb* rb, int* edge_index);       /* [n_rb + 1] grid indices */
double orc_loglike_rb(const orc_rb* rb, const double* theta);

/* Gaussian test likelihood on the unit cube. */
double orc_loglike_gauss(const orc_problem* p, const double* u);

/* lambda(u) for the problem's likelihood form (u in the unit cube). */
double orc_loglike_u(const orc_problem* p, const orc_rb* rb, const double* u);
int orc_loglike_batch(const orc_problem* p, const double* u, long n, double* out, int n_threads);

/* k lowest of n values in the sampler's total order. */
int orc_select(int n, const double* logl, int k, int* dead_idx, double* lstar);

/* Metrics of one iteration (Section 2's replace-the-k-lowest step), for
 * checking the sampler's per-iteration record.  Counts are of the
 * sequential walk: a probe outside the unit cube is no evaluation but its
 * rejection still shrinks the bracket. */
#define ORC_PROBE_HIST 32
typedef struct {
    int iter;                 /* iteration index, from 0 */
    int probes_min, probes_max;   /* fewest and most evaluations of one chain */
    int pad;
    double lstar;             /* the threshold L*: the k-th lowest lambda */
    double logX, logZ;        /* after the iteration's k deaths */
    double log_remaining;     /* logX + log mean exp(lambda) of the refilled live set, minus logZ */
    long long probes;         /* likelihood evaluations of all chains */
    long long steps;          /* slice steps (k * n_steps); random walk: proposals (k * chain length) */
    long long accepted;       /* slice steps that moved the chain; random walk: accepted proposals */
    long long stepouts;       /* bracket expansions */
    long long shrinks;        /* rejected shrink candidates */
    int hist[ORC_PROBE_HIST]; /* slice steps by evaluations made (last bin: that many or more) */
} orc_iter;

/* Nested sampling run. */
int orc_init(orc_run** out, const orc_problem* p, const orc_opts* o);
int orc_step(orc_run* r, int max_iters, int* done);
int orc_state(const orc_run* r, double* logX, double* logZ, double* H, int* iter, long* n_dead, long* n_evals);
int orc_live(const orc_run* r, double* u, double* logl);
int orc_dead(const orc_run* r, long cap, double* u, double* logl, double* logx, double* logw,
             int* iter, int* slot, long* n_out);
int orc_logZ(const orc_run* r, int n_sim, double* logZ, double* sigma_sim, double* sigma_h, double* ess);
/* Information H (unclipped) and Kish ESS of the final weighted samples. */
int orc_information(const orc_run* r, double* H, double* ess);
/* Per-iteration metrics of the iterations run so far, in order; n_out
 * receives their count; -3 (nothing written) if cap is smaller. */
int orc_trace(const orc_run* r, long cap, orc_iter* out, long* n_out);
int orc_samples(const orc_run* r, long cap, double* theta, double* logl, double* logw, long* n_out);
/* Equal-weight samples by systematic resampling of the weighted samples. */
int orc_resample(const orc_run* r, long n_out, int* idx, double* theta);
void orc_free(orc_run* r);

/* One random-walk chain (ORC_KERNEL_WALK) of n_prop proposals from x over
 * the population pop [npop][n_dim] (every point a survivor), with the draws
 * of chain j in iteration t of the key (seed, run_id) (test hook); returns
 * the accepted count, or -1. */
int orc_walk_from(const orc_problem* p, const orc_opts* o, const double* pop, int npop, int n_prop, double* x,
                  double* lx, double lstar, uint64_t t, uint64_t j, long* evals);

/* One slice update with a caller-supplied direction and uniforms (test
 * hook); moves (may be NULL) receives the bracket expansions, the rejected
 * shrink candidates and 1 if the point moved. */
int orc_slice_update_fixed(const orc_problem* p, const orc_opts* o, double* x, double* lx, const double* dir,
                           double lstar, double uw, double uj, const double* ushr, int n_ushr, long* evals,
                           int* moves);

#ifdef __cplusplus
}
#endif
#endif
