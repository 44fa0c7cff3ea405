/*
 * A plain C11 caller of libns: a Gaussian test problem (N(u; mu, s^2 I) on
 * the unit cube, whose evidence has the closed form prod_i of the normal
 * mass inside [0, 1]) run to termination through the C ABI alone, with the
 * per-iteration metrics and the weighted samples read back.
 *
 * Build: cc -std=c11 -Wall -Wextra -Werror -I include tests/c/ns_abi_demo.c
 *        -L paper_2509_24949_amd -lns -lm -Wl,-rpath,<dir of libns.so>
 * Exit status 0 when log Z lies within 4 sigma + 0.05 of the closed form and
 * the records are consistent; 1 otherwise; 2 when a call fails.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "ns.h"

#define D 3

static int check(int rc, const char* what) {
    if (rc != NS_OK) {
        fprintf(stderr, "%s failed (%d): %s\n", what, rc, ns_last_error());
        exit(2);
    }
    return rc;
}

int main(void) {
    const double mu[D] = {0.4, 0.5, 0.6}, sigma = 0.05;
    int kind[D] = {NS_PRIOR_UNIFORM, NS_PRIOR_UNIFORM, NS_PRIOR_UNIFORM};
    double lo[D] = {0.0, 0.0, 0.0}, hi[D] = {1.0, 1.0, 1.0};

    ns_problem p = {0};
    p.likelihood = NS_LIKE_GAUSS;
    p.n_dim = D;
    p.prior_kind = kind;
    p.prior_lo = lo;
    p.prior_hi = hi;
    p.f_lo = 1.0;
    p.df = 1.0;
    p.gauss_mu = mu;
    p.gauss_sigma = sigma;

    ns_opts o = {0};
    o.n_live = 400;
    o.n_delete = 200;
    o.n_steps = 5 * D;
    o.slice_width = 1.0;
    o.max_stepout = 100;
    o.max_shrink = 100;
    o.term_frac = 1e-3;
    o.seed = 11;
    o.run_id = 0;
    o.max_iter = 1000;
    o.precision = NS_FP64;
    o.kernel = NS_KERNEL_SLICE;
    o.walk_accept = 1;
    o.walk_max = 1;
    o.count_moves = 1;

    ns_run* run = NULL;
    check(ns_init(&run, &p, &o, NULL), "ns_init");
    int done = 0, iters = 0;
    while (!done && iters < o.max_iter) {
        check(ns_step(run, 25, &done), "ns_step");
        iters += 25;
    }
    double logz = 0.0, sig = 0.0, sig_h = 0.0, ess = 0.0;
    check(ns_logZ(run, 200, &logz, &sig, &sig_h, &ess), "ns_logZ");

    double want = 0.0;
    for (int i = 0; i < D; ++i)
        want += log(0.5 * (erf((1.0 - mu[i]) / (sigma * sqrt(2.0))) + erf(mu[i] / (sigma * sqrt(2.0)))));

    long n_rec = 0;
    check(ns_trace(run, 0, NULL, &n_rec), "ns_trace (count)");
    ns_iter_t* rec = (ns_iter_t*)malloc(sizeof(ns_iter_t) * (size_t)(n_rec > 0 ? n_rec : 1));
    check(ns_trace(run, n_rec, rec, &n_rec), "ns_trace");
    int ok = done != 0 && n_rec > 0;
    long long probes = 0;
    for (long t = 0; t < n_rec; ++t) {
        long long steps = 0, first = 0;
        for (int b = 0; b < NS_PROBE_HIST; ++b) {
            steps += rec[t].hist[b];
            first += (long long)b * rec[t].hist[b];
        }
        /* every step is in the histogram; below its last bin the first moment is the evaluation count */
        ok = ok && rec[t].iter == t && steps == rec[t].steps && rec[t].stepouts >= 0 && rec[t].shrinks >= 0;
        ok = ok && (rec[t].hist[NS_PROBE_HIST - 1] != 0 || first == rec[t].probes);
        probes += rec[t].probes;
    }
    long n_samples = 0;
    int rc = ns_samples(run, 0, NULL, NULL, NULL, &n_samples);
    ok = ok && rc == NS_E_CAPACITY && n_samples == (long)n_rec * o.n_delete + o.n_live;
    long n_evals = 0;
    check(ns_state(run, NULL, NULL, NULL, NULL, NULL, &n_evals, NULL), "ns_state");
    ok = ok && n_evals == probes + o.n_live;
    ok = ok && fabs(logz - want) < 4.0 * sig + 0.05;
    printf("ns_abi_demo: %ld iterations, logZ %.4f +- %.4f (closed form %.4f), %lld evaluations, ESS %.0f: %s\n",
           n_rec, logz, sig, want, probes, ess, ok ? "ok" : "FAILED");
    free(rec);
    ns_free(run);
    return ok ? 0 : 1;
}
