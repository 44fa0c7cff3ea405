/*
 * Host sanitizer run of the oracle: built together with oracle/nsorc.c under
 * AddressSanitizer and UndefinedBehaviorSanitizer (gcc, CPU only), it drives
 * every entry point the tests use: complete Gaussian runs with the slice and
 * the random-walk kernels (evidence, metrics records, weighted and
 * equal-weight samples), and a small two-detector TaylorF2 problem on the
 * full grid and with relative binning (waveform, likelihoods, two sampler
 * iterations each).  Exit status 0 when every call succeeds and the
 * evidence is finite; the sanitizers abort on the first error they find.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "nsorc.h"

static int fails = 0;
#define CHECK(cond)                                                  \
    do {                                                             \
        if (!(cond)) {                                               \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++fails;                                                 \
        }                                                            \
    } while (0)

static void run_and_read(const orc_problem* p, const orc_opts* o, int iters) {
    orc_run* r = NULL;
    CHECK(orc_init(&r, p, o) == 0 && r != NULL);
    if (!r) return;
    int done = 0;
    orc_step(r, iters, &done);
    double logz = 0, sig = 0, sig_h = 0, ess = 0;
    CHECK(orc_logZ(r, 50, &logz, &sig, &sig_h, &ess) == 0);
    CHECK(isfinite(logz) && isfinite(ess));
    long n_rec = 0;
    orc_trace(r, 0, NULL, &n_rec);
    orc_iter* rec = (orc_iter*)calloc((size_t)(n_rec > 0 ? n_rec : 1), sizeof(orc_iter));
    CHECK(orc_trace(r, n_rec, rec, &n_rec) == 0);
    long n_s = 0;
    orc_samples(r, 0, NULL, NULL, NULL, &n_s);
    double* th = (double*)calloc((size_t)n_s * p->n_dim, sizeof(double));
    double* ll = (double*)calloc((size_t)n_s, sizeof(double));
    double* lw = (double*)calloc((size_t)n_s, sizeof(double));
    CHECK(orc_samples(r, n_s, th, ll, lw, &n_s) == 0);
    int idx[64];
    double eq[64 * 16];
    CHECK(orc_resample(r, 64, idx, eq) == 0);
    free(rec); free(th); free(ll); free(lw);
    orc_free(r);
}

int main(void) {
    /* Gaussian in the unit cube: slice and random-walk kernels */
    {
        const int d = 3;
        int kind[3] = {ORC_PRIOR_UNIFORM, ORC_PRIOR_UNIFORM, ORC_PRIOR_UNIFORM};
        double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, mu[3] = {0.4, 0.5, 0.6};
        orc_problem p;
        memset(&p, 0, sizeof p);
        p.likelihood = ORC_LIKE_GAUSS;
        p.n_dim = d;
        p.prior_kind = kind; p.prior_lo = lo; p.prior_hi = hi;
        p.gauss_mu = mu; p.gauss_sigma = 0.05;
        orc_opts o;
        memset(&o, 0, sizeof o);
        o.n_live = 100; o.n_delete = 50; o.n_steps = 15; o.slice_width = 1.0;
        o.max_stepout = 100; o.max_shrink = 100; o.term_frac = 1e-3; o.seed = 3; o.max_iter = 200;
        o.n_threads = 2; o.kernel = ORC_KERNEL_SLICE; o.walk_accept = 10; o.walk_max = 200;
        run_and_read(&p, &o, 200);
        o.kernel = ORC_KERNEL_WALK;
        run_and_read(&p, &o, 200);
    }
    /* two detectors, 11 parameters, zero data: full grid and relative binning */
    {
        enum { NB = 400, ND = 2, DIM = 11 };
        int kind[DIM] = {0, 0, 0, 0, ORC_PRIOR_VOLUME, ORC_PRIOR_COS, 0, 0, ORC_PRIOR_SIN, 0, 0};
        double lo[DIM] = {20, 0.5, -0.5, -0.5, 100, 0, 0, 0, -1.5707963267948966, -0.05, 0};
        double hi[DIM] = {40, 1.0, 0.5, 0.5, 1000, 3.141592653589793, 3.141592653589793, 6.283185307179586,
                          1.5707963267948966, 0.05, 6.283185307179586};
        double geom[ND * 9] = {4.0e6, 1.0e6, 4.6e6, 0.6, 0.8, 0.0, -0.8, 0.6, 0.0,
                               -2.0e6, 5.0e6, 3.0e6, 0.0, 0.6, -0.8, 1.0, 0.0, 0.0};
        static double dre[ND * NB], dim[ND * NB], psd[ND * NB];
        for (int i = 0; i < ND * NB; ++i) psd[i] = 1e-46;
        double fid[DIM] = {30, 0.8, 0.1, -0.1, 400, 1.0, 0.5, 2.0, 0.3, 0.0, 1.0};
        orc_problem p;
        memset(&p, 0, sizeof p);
        p.model = ORC_MODEL_TF2_11P; p.likelihood = ORC_LIKE_FULL; p.n_dim = DIM;
        p.prior_kind = kind; p.prior_lo = lo; p.prior_hi = hi;
        p.f_lo = 20.0; p.df = 0.25; p.n_bins = NB; p.n_det = ND;
        p.data_re = dre; p.data_im = dim; p.psd = psd; p.det_geom = geom; p.gmst = 0.7;
        p.rb_n_bins = 16; p.rb_fiducial = fid;
        double hr[NB], hi2[NB];
        CHECK(orc_waveform(&p, fid, 1, 1, hr, hi2) == 0);
        const double lf = orc_loglike_full(&p, fid);
        CHECK(isfinite(lf) && lf <= 0.0);
        double u[DIM], th[DIM];
        for (int i = 0; i < DIM; ++i) u[i] = 0.3 + 0.04 * i;
        orc_prior_transform(&p, u, th);
        CHECK(isfinite(orc_loglike_u(&p, NULL, u)));
        orc_opts o;
        memset(&o, 0, sizeof o);
        o.n_live = 40; o.n_delete = 20; o.n_steps = 11; o.slice_width = 1.0;
        o.max_stepout = 100; o.max_shrink = 100; o.term_frac = 0.0; o.seed = 5; o.max_iter = 4;
        o.n_threads = 2; o.kernel = ORC_KERNEL_SLICE; o.walk_accept = 1; o.walk_max = 1;
        run_and_read(&p, &o, 2);
        p.model = ORC_MODEL_TF2_11P_SO;
        p.likelihood = ORC_LIKE_RB;
        orc_rb* rb = orc_rb_build(&p);
        CHECK(rb != NULL);
        if (rb) {
            int edges[17];
            CHECK(orc_rb_edges(rb, edges) == 16 && edges[0] == 0 && edges[16] <= NB - 1);
            CHECK(isfinite(orc_loglike_rb(rb, th)));
            orc_rb_free(rb);
        }
        run_and_read(&p, &o, 2);
    }
    printf("orc_sanitize: %s\n", fails ? "FAILED" : "ok");
    return fails ? 1 : 0;
}
